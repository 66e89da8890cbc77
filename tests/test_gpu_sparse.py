"""GPU parity of the thresholded block-sparse path (dmpt_sparse_response, Sec. V.B).

Without truncation (tau = 0) the sparse path computes the canonical response
itself, so it must match the FP64 oracle like the dense FP64 path (<= 1e-10).
With truncation its error stays within a small multiple of tau, and the
numbers of elements above the counting threshold 1e-5 (the quantity of
Fig. Fig_Scaling) agree with the oracle's exact matrices; on gapped chains of
growing length those counts, the stored blocks and the block products grow
linearly with N.
"""
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


def _count(a, thr):
    return int(np.count_nonzero(np.abs(a) >= thr))


def _rel(p, r):
    return float(np.abs(p.cpu().numpy() - r).max() / np.abs(r).max())


def test_sparse_untruncated_matches_oracle(dm):
    """tau = 0, ragged N = 300 (the last 32-block row is partial), two directions, orders 0-2."""
    print("case sparse tau=0", flush=True)
    N, n, beta, Ne = 300, 20, 10.0, 151.0
    h0 = workloads.chain_1d(N, 4)
    x = np.arange(N) - N / 2.0
    h1 = [np.diag(x / N), np.diag(np.cos(0.2 * np.arange(N)))]
    ref = oracle.canonical_response(h0, h1, None, beta, Ne, n, order=2)
    with dm.Context(128, dirs_max=2, prec="fp64") as ctx:
        P0, P1, P2, mu, st = ctx.sparse_response(T(h0), [T(h) for h in h1], beta=beta, Ne=Ne, n=n, order=2,
                                                 tau=0.0, count_thr=1e-5)
    e0 = float(np.abs(P0.cpu().numpy() - ref["P0"]).max())
    e1 = max(_rel(p, r) for p, r in zip(P1, ref["P1"]))
    e2 = max(_rel(p, r) for p, r in zip(P2, ref["P2"]))
    print(f"  errs {e0:.2e} {e1:.2e} {e2:.2e} passes={st['newton_iters']} blocks_max={st['blocks_max']} "
          f"products={st['block_products']:.0f}")
    assert e0 < 1e-10 and e1 < 1e-10 and e2 < 1e-10
    assert abs(mu[0] - ref["mu0"]) < 1e-10
    for z in range(2):
        assert abs(mu[1 + z] - ref["mu1"][z]) < 1e-9 * max(1.0, abs(ref["mu1"][z]))
        assert abs(mu[3 + z] - ref["mu2"][z]) < 1e-9 * max(1.0, abs(ref["mu2"][z]))
        assert abs(st["tr_h1p1"][z] - ref["tr_h1p1"][z]) < 1e-10 * max(1.0, abs(ref["tr_h1p1"][z]))
        assert abs(st["tr_h1p2"][z] - ref["tr_h1p2"][z]) < 1e-10 * max(1.0, abs(ref["tr_h1p2"][z]))
    assert abs(st["nnz_p0"] - _count(ref["P0"], 1e-5)) <= 2
    for z in range(2):
        assert abs(st["nnz_p1"][z] - _count(ref["P1"][z], 1e-5)) <= 2
        assert abs(st["nnz_p2"][z] - _count(ref["P2"][z], 1e-5)) <= 2


@pytest.mark.parametrize("beta", [10.0, 40.0])
def test_sparse_truncated_gapped_chain(dm, beta):
    """Gapped chain N = 2048, tau = 1e-8: absolute errors far below the counting threshold and
    element counts above 1e-5 that agree with the oracle's exact matrices."""
    print(f"case sparse dimer chain beta={beta}", flush=True)
    N, n = 2048, 22
    h0 = workloads.dimer_chain(N, 7)
    x = (np.arange(N) - N / 2.0) / N
    ref = oracle.canonical_response(h0, [x], None, beta, N / 2.0, n, order=2)
    with dm.Context(128, dirs_max=1, prec="fp64") as ctx:
        P0, P1, P2, mu, st = ctx.sparse_response(T(h0), [T(np.diag(x))], beta=beta, Ne=N / 2.0, n=n,
                                                 order=2, tau=1e-8, count_thr=1e-5, blocks_per_row=64)
    # absolute errors: the counts resolve elements of 1e-5, so the errors must sit well below it
    e0 = float(np.abs(P0.cpu().numpy() - ref["P0"]).max())
    e1 = float(np.abs(P1[0].cpu().numpy() - ref["P1"][0]).max())
    e2 = float(np.abs(P2[0].cpu().numpy() - ref["P2"][0]).max())
    c0, c1, c2 = _count(ref["P0"], 1e-5), _count(ref["P1"][0], 1e-5), _count(ref["P2"][0], 1e-5)
    print(f"  abs errs {e0:.2e} {e1:.2e} {e2:.2e} (max |P1| {np.abs(ref['P1'][0]).max():.2e}, "
          f"max |P2| {np.abs(ref['P2'][0]).max():.2e}); counts gpu {st['nnz_p0']:.0f} {st['nnz_p1'][0]:.0f} "
          f"{st['nnz_p2'][0]:.0f} oracle {c0} {c1} {c2}; blocks {st['blocks_p0']:.0f} / {(N // 32) ** 2} "
          f"max {st['blocks_max']:.0f} products {st['block_products']:.0f} {st['seconds']:.2f} s")
    assert e0 < 1e-6 and e1 < 1e-6 and e2 < 1e-6
    assert abs(st["nnz_p0"] - c0) <= 0.01 * c0
    assert abs(st["nnz_p1"][0] - c1) <= 0.01 * c1
    assert abs(st["nnz_p2"][0] - c2) <= 0.01 * c2 + 2
    assert st["blocks_p0"] < 0.25 * (N // 32) ** 2


def test_sparse_linear_scaling(dm):
    """Element counts above 1e-5, stored blocks and block products per unit length are the same
    on gapped chains of 2048, 4096 and 8192 sites (statistics only, no dense outputs)."""
    print("case sparse scaling", flush=True)
    beta, n = 10.0, 22
    per = []
    with dm.Context(128, dirs_max=1, prec="fp64") as ctx:
        for N in (2048, 4096, 8192):
            h0 = workloads.dimer_chain(N, 7)
            x = (np.arange(N) - N / 2.0) / N
            _, _, _, _, st = ctx.sparse_response(T(h0), [T(np.diag(x))], beta=beta, Ne=N / 2.0, n=n,
                                                 order=2, tau=1e-8, count_thr=1e-5, blocks_per_row=64,
                                                 outputs=False)
            row = (st["nnz_p0"] / N, st["nnz_p1"][0] / N, st["nnz_p2"][0] / N, st["blocks_max"] / (N / 32),
                   st["block_products"] / (N / 32), st["seconds"])
            print(f"  N={N}: per site nnz P0 {row[0]:.2f} P1 {row[1]:.2f} P2 {row[2]:.2f}; per block row "
                  f"blocks {row[3]:.2f} products {row[4]:.1f}; {row[5]:.2f} s", flush=True)
            per.append(row)
    for q in range(5):
        vals = [r[q] for r in per]
        assert max(vals) <= 1.1 * min(vals), (q, vals)
