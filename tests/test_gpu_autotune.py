"""GPU tests of the product-kernel variants and the autotuner.

Every variant of every engine computes the same products (checked through a
whole recursion against the oracle); the autotuner's choice is the one later
products use; options.autotune tunes every bucket size of a batched solve;
the tuning cache file makes a second context take the same choice.
"""
import os

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def dm():
    import paper_1503_07037_amd as m
    m.load()
    return m


def T(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=_dev())


@pytest.mark.parametrize("prec,extra,variants,tol", [
    ("fp64", {}, 3, 1e-12), ("fp32", {}, 3, 1e-6), ("bf16x3", {}, 2, 5e-5),
    ("bf16x6", {"acc64": 0}, 2, 2e-6), ("bf16x6", {"acc64": 1}, 1, 1e-6), ("int8x13", {}, 4, 1e-6),
    ("int8x6", {}, 4, 1e-5)])
def test_every_variant_matches_the_oracle(dm, prec, extra, variants, tol):
    """P0 at fixed mu through each pinned variant (N = 512: the 256-wide tiles apply)."""
    N, beta, n, mu = 512, 10.0, 20, 0.05
    h0 = workloads.chain_1d(N, 21)
    ref = oracle.density(h0, beta, n, mu)
    with dm.Context(N, dirs_max=0, prec=prec, **extra) as ctx:
        for v in range(variants):
            ctx.set_variant(N, v)
            got, tuned, name = ctx.get_variant(N)
            assert got == v and tuned
            P0, _ = ctx.fermi_recursion(T(h0), beta, mu, n)
            err = float(np.abs(P0.cpu().numpy() - ref).max())
            print(f"  {prec} {extra} variant {v} ({name}): {err:.2e}", flush=True)
            assert err < tol
        with pytest.raises(dm.DMPTError):
            ctx.set_variant(N, variants)


def test_autotune_choice_is_used_and_cached(dm, tmp_path):
    N = 1024
    path = str(tmp_path / "tune.txt")
    old = os.environ.get("DMPT_TUNE_CACHE")
    os.environ["DMPT_TUNE_CACHE"] = path
    try:
        with dm.Context(N, dirs_max=0, prec="fp32") as ctx:
            assert ctx.get_variant(N)[1] is False
            v = ctx.autotune(N)
            got, tuned, name = ctx.get_variant(N)
            print(f"  tuned fp32 N={N}: variant {v} ({name})", flush=True)
            assert got == v and tuned
        lines = open(path).read().split("\n")
        assert any(l.split()[2:3] == [str(N)] for l in lines if l.strip())
        with dm.Context(N, dirs_max=0, prec="fp32") as ctx2:
            assert ctx2.autotune(N) == v  # from the cache
    finally:
        if old is None:
            os.environ.pop("DMPT_TUNE_CACHE", None)
        else:
            os.environ["DMPT_TUNE_CACHE"] = old


def test_batched_solve_tunes_every_bucket(dm):
    """options.autotune on a batched FP32 solve: every bucket size gets a tuned variant, and the
    results still match the oracle."""
    systems = [((4, 4, 4), 7.0), ((6, 5, 4), 31.0), ((10, 8, 5), 5.5)]
    hs, h1s, refs = [], [], []
    for k, (dims, beta) in enumerate(systems):
        h0 = workloads.cubic_lattice(*dims, seed=300 + k)
        x = list(workloads.lattice_dipoles(*dims))[:1]
        hs.append(h0)
        h1s.append([np.diag(x[0])])
        refs.append(oracle.canonical_response(h0, x, None, beta, h0.shape[0] / 2.0, 25, order=1))
    nmax = max(h.shape[0] for h in hs)
    with dm.Context(nmax, dirs_max=1, prec="fp32", autotune=1) as ctx:
        P0, P1, _, mus, st = ctx.mu_newton_batched([T(h) for h in hs], [[T(h) for h in l] for l in h1s],
                                                   [b for _, b in systems], [h.shape[0] / 2.0 for h in hs],
                                                   n=25, order=1)
        for h in hs:
            v, tuned, name = ctx.get_variant(h.shape[0])
            print(f"  N={h.shape[0]}: variant {v} ({name}) tuned={tuned}", flush=True)
            assert tuned
    for k, r in enumerate(refs):
        assert np.abs(P0[k].cpu().numpy() - r["P0"]).max() < 1e-6
        assert np.abs(P1[k][0].cpu().numpy() - r["P1"][0]).max() < 1e-6 * np.abs(r["P1"][0]).max()
