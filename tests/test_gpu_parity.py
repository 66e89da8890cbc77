"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Bars: FP64 path <= 1e-10 (P0 absolute; P1, P2 normalised by max |P^(k)|
of the oracle), FP32 / split-BF16 paths <= 1e-6 on the same measures.
Sizes span several 128-wide tiles and ragged tails (N not a multiple of 128).
"""
import math
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


def errs(P0, P1, P2, ref):
    e0 = float(np.abs(P0.cpu().numpy() - ref["P0"]).max())
    e1 = [float(np.abs(p.cpu().numpy() - r).max() / max(np.abs(r).max(), 1e-300))
          for p, r in zip(P1, ref["P1"])]
    e2 = [float(np.abs(p.cpu().numpy() - r).max() / max(np.abs(r).max(), 1e-300))
          for p, r in zip(P2, ref["P2"])]
    return e0, max(e1, default=0.0), max(e2, default=0.0)


def _sym(rng, n, s=1.0):
    a = rng.standard_normal((n, n)) * s
    return 0.5 * (a + a.T)


# ------------------------------------------------------------------ grand canonical

@pytest.mark.parametrize("N", [128, 200, 300])
def test_fermi_recursion_fp64(dm, N):
    print(f"case fermi_recursion fp64 N={N}", flush=True)
    h0 = workloads.chain_1d(N, 7)
    beta, n, mu = 10.0, 20, 0.05
    ref = oracle.density(h0, beta, n, mu)
    with dm.Context(N, dirs_max=0, prec="fp64") as ctx:
        P0, st = ctx.fermi_recursion(T(h0), beta, mu, n)
    assert float(np.abs(P0.cpu().numpy() - ref).max()) < 1e-12


@pytest.mark.parametrize("order", [1, 2])
def test_response_at_fixed_mu_fp64(dm, order):
    print(f"case response fp64 order={order}", flush=True)
    N, n, beta = 160, 18, 8.0
    rng = np.random.default_rng(3)
    h0 = workloads.chain_1d(N, 3)
    h1 = [np.diag(np.arange(N) - N / 2.0) / N, _sym(rng, N, 0.1)]
    h2 = [_sym(rng, N, 0.05), None]
    mu = [0.02, 0.3, -0.1, 0.05, 0.2][: 1 + order * 2]
    mu_o = (mu[0], mu[1:3], mu[3:5] if order >= 2 else [0.0, 0.0])
    ref = oracle.response(h0, h1, h2, beta, n, mu_o, order=order)
    with dm.Context(N, dirs_max=2, prec="fp64") as ctx:
        P0, P1, P2, st = ctx.response(T(h0), [T(h) for h in h1],
                                      [T(h2[0]), None] if order >= 2 else None,
                                      beta=beta, n=n, order=order, mu=mu)
    e0, e1, e2 = errs(P0, P1, P2, ref)
    assert e0 < 1e-12 and e1 < 1e-10 and e2 < 1e-10, (e0, e1, e2)


def _rel(gpu, ref):
    return max(float(np.abs(g.cpu().numpy() - r).max()) / float(np.abs(r).max()) for g, r in zip(gpu, ref))


def test_response_third_order_at_fixed_mu_fp64(dm):
    """Algorithm 1's fourth solve line at a fixed mu jet (H2, H3 partly zero) against the oracle."""
    print("case response fp64 order=3", flush=True)
    N, n, beta = 160, 18, 8.0
    rng = np.random.default_rng(31)
    h0 = workloads.chain_1d(N, 3)
    h1 = [np.diag(np.arange(N) - N / 2.0) / N, _sym(rng, N, 0.1)]
    h2 = [_sym(rng, N, 0.05), None]
    h3 = [None, _sym(rng, N, 0.04)]
    mu = [0.02, 0.3, -0.1, 0.05, 0.2, -0.15, 0.1]
    ref = oracle.response(h0, h1, h2, beta, n, (mu[0], mu[1:3], mu[3:5], mu[5:7]), order=3, h3s=h3)
    with dm.Context(N, dirs_max=2, prec="fp64") as ctx:
        r = ctx.response(T(h0), [T(h) for h in h1], [T(h2[0]), None], beta=beta, n=n, order=3, mu=mu,
                         H3=[None, T(h3[1])])
    P0, P1, P2, st = r
    e0, e1, e2 = errs(P0, P1, P2, ref)
    e3 = _rel(r.P3, ref["P3"])
    print(f"  errs {e0:.2e} {e1:.2e} {e2:.2e} {e3:.2e}")
    assert e0 < 1e-12 and e1 < 1e-10 and e2 < 1e-10 and e3 < 1e-10, (e0, e1, e2, e3)
    assert abs(st["trP"][5] - float(np.trace(ref["P3"][0]))) < 1e-9 * float(np.abs(ref["P3"][0]).max()) * N


@pytest.mark.parametrize("schedule", [1, 2, 0])
def test_third_order_canonical_fp64(dm, schedule):
    """Canonical orders 0..3 (mu1, mu2, mu3 from Tr P^(k) = 0), ragged N, two directions."""
    print(f"case canonical fp64 order=3 schedule={schedule}", flush=True)
    N, n, beta, Ne = 200, 20, 10.0, 97.0
    rng = np.random.default_rng(32)
    h0 = workloads.banded(N, 5, bandwidth=16, decay=6.0)
    h1 = [np.diag(np.arange(N) % 9 - 4.0), np.diag(np.cos(0.3 * np.arange(N)))]
    h2 = [_sym(rng, N, 0.03), None]
    h3 = [None, _sym(rng, N, 0.02)]
    ref = oracle.canonical_response(h0, h1, h2, beta, Ne, n, order=3, h3s=h3)
    with dm.Context(N, dirs_max=2, prec="fp64", schedule=schedule) as ctx:
        r = ctx.mu_newton(T(h0), [T(h) for h in h1], [T(h2[0]), None], beta=beta, Ne=Ne, n=n,
                          order=3, H3=[None, T(h3[1])])
    P0, P1, P2, mu, st = r
    e0, e1, e2 = errs(P0, P1, P2, ref)
    e3 = _rel(r.P3, ref["P3"])
    print(f"  errs {e0:.2e} {e1:.2e} {e2:.2e} {e3:.2e} newton={st['newton_iters']}")
    assert e0 < 1e-10 and e1 < 1e-10 and e2 < 1e-10 and e3 < 1e-10, (e0, e1, e2, e3)
    for z in range(2):
        assert abs(mu[5 + z] - ref["mu3"][z]) < 1e-9 * max(1.0, abs(ref["mu3"][z]))
        for key in ("tr_h1p3", "tr_h2p2", "tr_h3p1", "tr_h3p0", "omega3", "omega4"):
            assert abs(st[key][z] - ref[key][z]) < 1e-9 * max(1.0, abs(ref[key][z])), (key, z)


@pytest.mark.parametrize("prec", ["bf16x6", "int8x13"])
def test_third_order_canonical_low_precision(dm, prec):
    """Third order through the 6-product split with FP64 slice sums and through the 13-product int8
    slices: <= 1e-6 (normalised)."""
    print(f"case canonical {prec} order=3", flush=True)
    c = workloads.config("chain128")
    h3 = [_sym(np.random.default_rng(33), c["N"], 0.02)]
    ref = oracle.canonical_response(c["H0"], c["H1"], None, c["beta"], c["Ne"], c["n"], order=3, h3s=h3)
    with dm.Context(c["N"], dirs_max=1, prec=prec) as ctx:
        r = ctx.mu_newton(T(c["H0"]), [T(h) for h in c["H1"]], None, beta=c["beta"], Ne=c["Ne"],
                          n=c["n"], order=3, H3=[T(h3[0])])
    P0, P1, P2, mu, st = r
    e0, e1, e2 = errs(P0, P1, P2, ref)
    e3 = _rel(r.P3, ref["P3"])
    print(f"  errs {e0:.2e} {e1:.2e} {e2:.2e} {e3:.2e}")
    assert e0 < 1e-6 and e1 < 1e-6 and e2 < 1e-6 and e3 < 1e-6, (e0, e1, e2, e3)


# ------------------------------------------------------------------ canonical

@pytest.fixture(scope="module")
def chain128_ref():
    c = workloads.config("chain128")
    r = oracle.canonical_response(c["H0"], c["H1"], None, c["beta"], c["Ne"], c["n"], order=2)
    return c, r


@pytest.mark.parametrize("schedule,warm_traj", [(1, 1), (1, 0), (2, 1), (0, 1), (0, 0)])
def test_chain128_canonical_fp64(dm, chain128_ref, schedule, warm_traj):
    """Both canonical schedules: the linear one (mu0 loop, then one pass per
    order with the identity response) and Algorithm 1's joint Newton loop."""
    print(f"case chain128 canonical fp64 schedule={schedule} warm_traj={warm_traj}", flush=True)
    c, ref = chain128_ref
    with dm.Context(c["N"], dirs_max=1, prec="fp64", warm_traj=warm_traj, schedule=schedule) as ctx:
        P0, P1, P2, mu, st = ctx.mu_newton(T(c["H0"]), [T(h) for h in c["H1"]], None,
                                           beta=c["beta"], Ne=c["Ne"], n=c["n"], order=2)
    e0, e1, e2 = errs(P0, P1, P2, ref)
    print(f"  errs {e0:.2e} {e1:.2e} {e2:.2e} newton={st['newton_iters']} cg={st['cg_iters_total']}")
    assert e0 < 1e-10 and e1 < 1e-10 and e2 < 1e-10
    assert abs(mu[0] - ref["mu0"]) < 1e-10
    assert abs(mu[1] - ref["mu1"][0]) < 1e-9 * max(1, abs(ref["mu1"][0]))
    assert abs(mu[2] - ref["mu2"][0]) < 1e-9 * max(1, abs(ref["mu2"][0]))
    assert abs(st["tr_h1p1"][0] - ref["tr_h1p1"][0]) < 1e-10 * abs(ref["tr_h1p1"][0])
    assert abs(st["tr_h1p2"][0] - ref["tr_h1p2"][0]) < 1e-10 * abs(ref["tr_h1p2"][0])
    assert abs(st["trP"][0] - c["Ne"]) < 1e-9


def test_chain128_taylor_guess_fp64(dm, chain128_ref):
    """The Taylor initial guess 2D - 8D^3 for the order-0 solves (no trajectory) reaches the same result."""
    print("case chain128 taylor guess", flush=True)
    c, ref = chain128_ref
    cg = {}
    for guess in ("prev", "taylor"):
        with dm.Context(c["N"], dirs_max=1, prec="fp64", warm_traj=0, guess=guess) as ctx:
            P0, P1, P2, mu, st = ctx.mu_newton(T(c["H0"]), [T(h) for h in c["H1"]], None,
                                               beta=c["beta"], Ne=c["Ne"], n=c["n"], order=2)
        e0, e1, e2 = errs(P0, P1, P2, ref)
        cg[guess] = st["cg_iters_total"]
        print(f"  {guess}: errs {e0:.2e} {e1:.2e} {e2:.2e} cg={st['cg_iters_total']}")
        assert e0 < 1e-10 and e1 < 1e-10 and e2 < 1e-10


@pytest.mark.parametrize("prec,extra,tol", [
    ("fp32", {}, 1e-6),                # FP32 products, FP64 slice sums and iterates
    ("bf16x6", {}, 1e-6),              # 6-product split, FP64 iterates
    ("bf16x3", {}, 5e-5),              # 3-product split alone
    ("bf16x3", {"refine": 1}, 1e-6),   # 3-product passes, then the 6-product refinement
    ("int8x13", {}, 1e-6),             # int8 slices, exact int32 sums
    ("bf16x3", {"refine": 2}, 1e-6),   # 3-product passes, then int8 slices
    ("int8x6", {}, 1e-5),              # the first three int8 digits alone
    ("int8x6", {"refine": 2}, 1e-6),   # int8 6-product passes, then the 13-product order-1/2 passes
    ("int8x6", {"refine": 2, "schedule": 0}, 1e-6),  # the same with Algorithm 1's joint Newton
])
def test_chain128_canonical_low_precision(dm, chain128_ref, prec, extra, tol):
    print(f"case chain128 canonical {prec} {extra}", flush=True)
    c, ref = chain128_ref
    with dm.Context(c["N"], dirs_max=1, prec=prec, **extra) as ctx:
        P0, P1, P2, mu, st = ctx.mu_newton(T(c["H0"]), [T(h) for h in c["H1"]], None,
                                           beta=c["beta"], Ne=c["Ne"], n=c["n"], order=2)
    e0, e1, e2 = errs(P0, P1, P2, ref)
    print(f"  errs {e0:.2e} {e1:.2e} {e2:.2e} newton={st['newton_iters']} cg={st['cg_iters_total']}")
    assert e0 < tol and e1 < tol and e2 < tol


@pytest.mark.parametrize("N,d,schedule", [(250, 3, 1), (384, 2, 1), (250, 3, 2), (250, 3, 0)])
def test_ragged_multi_direction_fp64(dm, N, d, schedule):
    """N not a multiple of the tile, several directions, non-zero H2."""
    print(f"case ragged canonical fp64 N={N} d={d} schedule={schedule}", flush=True)
    rng = np.random.default_rng(N)
    h0 = workloads.banded(N, 9, bandwidth=24, decay=8.0)
    grid = [np.arange(N) % 7 - 3.0, (np.arange(N) // 7) % 5 - 2.0, np.sin(np.arange(N))]
    h1 = [np.diag(g) for g in grid][:d]
    h2 = [_sym(rng, N, 0.02) if i == 0 else None for i in range(d)]
    beta, n, Ne = 12.0, 22, N / 2.0 - 3.0
    ref = oracle.canonical_response(h0, h1, h2, beta, Ne, n, order=2)
    with dm.Context(N, dirs_max=d, prec="fp64", schedule=schedule) as ctx:
        P0, P1, P2, mu, st = ctx.mu_newton(T(h0), [T(h) for h in h1],
                                           [T(h) if h is not None else None for h in h2],
                                           beta=beta, Ne=Ne, n=n, order=2)
    e0, e1, e2 = errs(P0, P1, P2, ref)
    print(f"  errs {e0:.2e} {e1:.2e} {e2:.2e}")
    assert e0 < 1e-10 and e1 < 1e-10 and e2 < 1e-10
    for z in range(d):
        assert abs(st["tr_h2p0"][z] - ref["tr_h2p0"][z]) < 1e-10 * max(1, abs(ref["tr_h2p0"][z]))
        assert abs(mu[1 + z] - ref["mu1"][z]) < 1e-9 * max(1, abs(ref["mu1"][z]))
        assert abs(mu[1 + d + z] - ref["mu2"][z]) < 1e-9 * max(1, abs(ref["mu2"][z]))
        assert abs(st["tr_h1p2"][z] - ref["tr_h1p2"][z]) < 1e-10 * max(1, abs(ref["tr_h1p2"][z]))
        # Eq. Resp_0 observables: Tr(H2 P1), Omega^(1..3)
        for key in ("tr_h1p0", "tr_h2p1", "omega1", "omega2", "omega3"):
            assert abs(st[key][z] - ref[key][z]) < 1e-10 * max(1, abs(ref[key][z])), (key, z)


@pytest.mark.parametrize("N,d", [(250, 3), (1000, 2)])
def test_ragged_multi_direction_int8(dm, N, d):
    """Int8 slices with N not a multiple of the tile (ragged last tile and zero padding inside the
    slices), several directions, non-zero H2: every element against the oracle at 1e-6."""
    print(f"case ragged canonical int8x13 N={N} d={d}", flush=True)
    rng = np.random.default_rng(N)
    h0 = workloads.banded(N, 9, bandwidth=24, decay=8.0)
    grid = [np.arange(N) % 7 - 3.0, (np.arange(N) // 7) % 5 - 2.0, np.sin(np.arange(N))]
    h1 = [np.diag(g) for g in grid][:d]
    h2 = [_sym(rng, N, 0.02) if i == 0 else None for i in range(d)]
    beta, n, Ne = 12.0, 22, N / 2.0 - 3.0
    ref = oracle.canonical_response(h0, h1, h2, beta, Ne, n, order=2)
    with dm.Context(N, dirs_max=d, prec="int8x13") as ctx:
        P0, P1, P2, mu, st = ctx.mu_newton(T(h0), [T(h) for h in h1],
                                           [T(h) if h is not None else None for h in h2],
                                           beta=beta, Ne=Ne, n=n, order=2)
    e0, e1, e2 = errs(P0, P1, P2, ref)
    print(f"  errs {e0:.2e} {e1:.2e} {e2:.2e} newton={st['newton_iters']} flags={st['flags']}")
    assert e0 < 1e-6 and e1 < 1e-6 and e2 < 1e-6


def test_single_site(dm):
    """N = 1: P0 = Ne exactly, mu = H00 - (1/beta) log(1/Ne - 1) in the Fermi-Dirac limit."""
    print("case single site", flush=True)
    h0 = np.array([[0.3]])
    with dm.Context(1, dirs_max=1, prec="fp64") as ctx:
        P0, P1, P2, mu, st = ctx.mu_newton(T(h0), [T(np.array([[2.0]]))], None, beta=4.0, Ne=0.25,
                                           n=30, order=2)
    assert abs(P0.item() - 0.25) < 1e-12
    assert abs(P1[0].item()) < 1e-12 and abs(P2[0].item()) < 1e-12
    assert abs(mu[1] - 2.0) < 1e-10
    assert abs(mu[0] - (0.3 - math.log(3.0) / 4.0)) < 1e-9


# ------------------------------------------------------------------ failure paths

def test_range_guard(dm):
    print("case range guard", flush=True)
    h0 = workloads.chain_1d(64, 1)
    with dm.Context(64, dirs_max=0) as ctx:
        with pytest.raises(dm.DMPTError) as ei:
            ctx.fermi_recursion(T(h0), 1e6, 0.0, 4)
    assert ei.value.status == -5


def test_nonfinite_input(dm):
    print("case nonfinite", flush=True)
    h0 = workloads.chain_1d(64, 1)
    h0[3, 5] = np.nan
    with dm.Context(64, dirs_max=0) as ctx:
        with pytest.raises(dm.DMPTError) as ei:
            ctx.fermi_recursion(T(h0), 5.0, 0.0, 10)
    assert ei.value.status == -6


def test_newton_cap_reports_noconv(dm):
    """Too few Newton passes: status NOCONV with the last pass's statistics filled."""
    print("case noconv", flush=True)
    h0 = workloads.chain_1d(64, 2)
    with dm.Context(64, dirs_max=0, max_newton=1) as ctx:
        P0, _, _, mu, st = ctx.mu_newton(T(h0), beta=10.0, Ne=20.0, n=20, order=0,
                                         raise_on_error=False)
    assert st["status"] == -4
    assert st["newton_iters"] == 1 and math.isfinite(st["trP"][0])


# ------------------------------------------------------------------ non-orthogonal basis

def test_congruence_fp64(dm):
    """Z^T A Z and Z A Z^T on the FP64 engine against numpy (ragged N, general Z)."""
    print("case congruence", flush=True)
    N = 230
    rng = np.random.default_rng(41)
    A = _sym(rng, N)
    Z = workloads.inverse_factor(workloads.overlap(N, 5))
    with dm.Context(N, dirs_max=1, prec="fp64") as ctx:
        B0 = ctx.congruence(T(Z), T(A), 0).cpu().numpy()
        B1 = ctx.congruence(T(Z), T(A), 1).cpu().numpy()
    r0, r1 = Z.T @ A @ Z, Z @ A @ Z.T
    assert np.abs(B0 - r0).max() < 1e-13 * np.abs(r0).max()
    assert np.abs(B1 - r1).max() < 1e-13 * np.abs(r1).max()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("bf16x6", 1e-6)])
def test_nonorthogonal_canonical(dm, prec, tol):
    """D^(k) = Z P^(k)(Z^T F Z) Z^T with Tr P_perp = Ne against the oracle (orders 0-2)."""
    print(f"case non-orthogonal canonical {prec}", flush=True)
    N, n, beta, Ne = 200, 20, 9.0, 93.0
    rng = np.random.default_rng(42)
    f0 = workloads.chain_1d(N, 12)
    f1 = [np.diag(np.arange(N) - N / 2.0) / N]
    f2 = [_sym(rng, N, 0.02)]
    S = workloads.overlap(N, 6)
    Z = workloads.inverse_factor(S)
    ref = oracle.nonorthogonal_response(f0, f1, f2, Z, beta, Ne, n, order=2)
    with dm.Context(N, dirs_max=1, prec=prec) as ctx:
        D0, D1, D2, mu, st = ctx.mu_newton_nonorthogonal(T(f0), T(Z), [T(f1[0])], [T(f2[0])], beta=beta,
                                                         Ne=Ne, n=n, order=2)
    e0 = float(np.abs(D0.cpu().numpy() - ref["D0"]).max())
    e1 = float(np.abs(D1[0].cpu().numpy() - ref["D1"][0]).max() / np.abs(ref["D1"][0]).max())
    e2 = float(np.abs(D2[0].cpu().numpy() - ref["D2"][0]).max() / np.abs(ref["D2"][0]).max())
    print(f"  errs {e0:.2e} {e1:.2e} {e2:.2e}")
    assert e0 < tol and e1 < tol and e2 < tol
    assert abs(float(np.trace(D0.cpu().numpy() @ S)) - Ne) < max(tol, 1e-9) * N


# ------------------------------------------------------------------ Newton-Schulz shared inverse

@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("bf16x6", 1e-6), ("fp32", 1e-6), ("int8x13", 1e-6)])
def test_newton_schulz_solver_canonical(dm, chain128_ref, prec, tol):
    """The shared-inverse solver (one inverse of T' per step for all orders) reaches the oracle."""
    print(f"case newton-schulz {prec}", flush=True)
    c, ref = chain128_ref
    with dm.Context(c["N"], dirs_max=1, prec=prec, solver="ns") as ctx:
        P0, P1, P2, mu, st = ctx.mu_newton(T(c["H0"]), [T(h) for h in c["H1"]], None,
                                           beta=c["beta"], Ne=c["Ne"], n=c["n"], order=2)
    e0, e1, e2 = errs(P0, P1, P2, ref)
    print(f"  errs {e0:.2e} {e1:.2e} {e2:.2e} newton={st['newton_iters']} cg={st['cg_iters_total']}")
    assert e0 < tol and e1 < tol and e2 < tol
    assert st["cg_iters_total"] == 0


@pytest.mark.parametrize("prec,refine,tol,schedule", [
    ("fp64", 0, 1e-10, 1), ("fp64", 0, 1e-10, 0), ("fp64", 0, 1e-10, 2), ("int8x13", 0, 1e-6, 1),
    ("int8x6", 2, 1e-6, 1), ("bf16x3", 2, 1e-6, 1), ("bf16x6", 0, 1e-6, 1), ("fp32", 0, 1e-6, 1)])
def test_hybrid_solver_canonical(dm, chain128_ref, prec, refine, tol, schedule):
    """The shared inverse in the passes with FP64 or int8x13 products (schedule 1: the order-1 pass
    stores Z of every step and the order-2 pass reuses it; 2: the order-2 pass solves again;
    0: Algorithm 1's joint Newton), CG in the passes with BF16 and FP32 products: the oracle's
    result either way."""
    print(f"case hybrid {prec} refine={refine} schedule={schedule}", flush=True)
    c, ref = chain128_ref
    with dm.Context(c["N"], dirs_max=1, prec=prec, refine=refine, solver="hybrid", schedule=schedule) as ctx:
        P0, P1, P2, mu, st = ctx.mu_newton(T(c["H0"]), [T(h) for h in c["H1"]], None,
                                           beta=c["beta"], Ne=c["Ne"], n=c["n"], order=2)
    e0, e1, e2 = errs(P0, P1, P2, ref)
    print(f"  errs {e0:.2e} {e1:.2e} {e2:.2e} newton={st['newton_iters']} cg={st['cg_iters_total']}")
    assert e0 < tol and e1 < tol and e2 < tol
    assert abs(mu[0] - ref["mu0"]) < 10 * tol
    if prec in ("fp64", "int8x13") or (prec == "int8x6" and refine == 2):
        assert st["cg_iters_total"] == 0  # every pass solved with the shared inverse
    else:
        assert st["cg_iters_total"] > 0   # passes with FP32 or BF16 products ran CG


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-13), ("int8x13", 5e-8)])
def test_newton_schulz_short_start_matches_full_iterations(dm, chain128_ref, prec, tol, monkeypatch):
    """The step-dependent start (fewer Newton-Schulz iterations while ||D_s|| is small) gives the
    results of four iterations in every step (DMPT_NS_ITERS=4 forces them): to rounding in FP64;
    with int8x13 products, whose dropped digit products leave ~1e-8 on P2, within a few times
    that (the two forms round different products)."""
    print(f"case newton-schulz short start {prec}", flush=True)
    c, _ = chain128_ref
    out = []
    for force in (None, "4"):
        if force:
            monkeypatch.setenv("DMPT_NS_ITERS", force)
        else:
            monkeypatch.delenv("DMPT_NS_ITERS", raising=False)
        with dm.Context(c["N"], dirs_max=1, prec=prec, solver="ns") as ctx:
            P0, P1, P2, mu, st = ctx.mu_newton(T(c["H0"]), [T(h) for h in c["H1"]], None,
                                               beta=c["beta"], Ne=c["Ne"], n=c["n"], order=2)
        out.append((P0.cpu().numpy(), P1[0].cpu().numpy(), P2[0].cpu().numpy(), st["mfma_flops"]))
    monkeypatch.delenv("DMPT_NS_ITERS", raising=False)
    (a0, a1, a2, fa), (b0, b1, b2, fb) = out
    d0 = np.abs(a0 - b0).max()
    d1 = np.abs(a1 - b1).max() / np.abs(b1).max()
    d2 = np.abs(a2 - b2).max() / np.abs(b2).max()
    print(f"  differences {d0:.2e} {d1:.2e} {d2:.2e}; products {fa:.3e} vs {fb:.3e}")
    assert d0 < tol and d1 < tol and d2 < tol
    assert fa < fb  # the short start did fewer products


@pytest.mark.parametrize("prec,solver,tol", [("fp64", "hybrid", 1e-12), ("fp64", "cg", 1e-12),
                                              ("int8x13", "hybrid", 5e-8), ("bf16x3", "cg", 3e-5)])
def test_symmetric_products_match_full_tiles(dm, prec, solver, tol, monkeypatch):
    """Products with a symmetric result (D0 D0, the Newton-Schulz products, D1 D1, R Z at order 0)
    compute the tiles on and below the diagonal and mirror them; DMPT_FULL_TILES=1 computes every
    tile.  Ragged N = 1000 (Np = 1024: eight 128-wide tile rows, four 256-wide ones) and
    N = 640 (five 128-wide rows: odd, so every tile is computed), orders 0-2: the two agree to
    rounding (int8x13: within the engine's own error; bf16x3 without refinement: within its ~1e-5)."""
    rng = np.random.default_rng(5)
    for N in (1000, 640):
        print(f"case symmetric products {prec} {solver} N={N}", flush=True)
        h0 = workloads.banded(N, 11, bandwidth=24, decay=8.0)
        h1 = [np.diag(np.linspace(-1.0, 1.0, N)), _sym(rng, N, 0.05)]
        out = []
        for full in (False, True):
            if full:
                monkeypatch.setenv("DMPT_FULL_TILES", "1")
            else:
                monkeypatch.delenv("DMPT_FULL_TILES", raising=False)
            with dm.Context(N, dirs_max=2, prec=prec, solver=solver) as ctx:
                P0, P1, P2, mu, st = ctx.mu_newton(T(h0), [T(h) for h in h1], None, beta=12.0,
                                                   Ne=N / 2.0, n=22, order=2)
            out.append((P0.cpu().numpy(), [p.cpu().numpy() for p in P1], [p.cpu().numpy() for p in P2],
                        st["mfma_flops"]))
        monkeypatch.delenv("DMPT_FULL_TILES", raising=False)
        (a0, a1, a2, fa), (b0, b1, b2, fb) = out
        d0 = np.abs(a0 - b0).max()
        d1 = max(np.abs(x - y).max() / np.abs(y).max() for x, y in zip(a1, b1))
        d2 = max(np.abs(x - y).max() / np.abs(y).max() for x, y in zip(a2, b2))
        print(f"  differences {d0:.2e} {d1:.2e} {d2:.2e}; executed {fa:.3e} vs {fb:.3e}")
        assert d0 < tol and d1 < tol and d2 < tol
        assert np.abs(a0 - a0.T).max() == 0.0
        if N == 1000:
            assert fa < fb
        else:
            assert fa == fb


@pytest.mark.parametrize("prec,refine", [("int8x13", 0), ("int8x6", 2)])
def test_split_diagonal_tiles_match_whole_tiles(dm, prec, refine, monkeypatch):
    """Symmetric int8 products with at least eight 128-wide tile rows compute each diagonal tile as
    four blocks over quarters of the inner index plus a summing kernel (DMPT_DIAG_SPLIT=0: one
    block per diagonal tile).  The int32 sums of a quarter are exact, so only the FP64 addition of
    the four partial tiles rounds differently: N = 1000 (8 tile rows) and N = 2000 (16), orders 0-2,
    agree far below the engine's own error (int8x13: 1e-9; int8x6 with refine = 2: 5e-8, the
    13-product engine's error, since the loose first phase's different rounding moves the mu0 its
    Newton step hands on, and the final passes end anywhere within their tolerance), and against
    the oracle."""
    rng = np.random.default_rng(8)
    for N in (1000, 2000):
        print(f"case split diagonal {prec} N={N}", flush=True)
        h0 = workloads.banded(N, 13, bandwidth=24, decay=8.0)
        h1 = [np.diag(np.linspace(-1.0, 1.0, N)), _sym(rng, N, 0.05)]
        out = []
        for split in (True, False):
            if split:
                monkeypatch.delenv("DMPT_DIAG_SPLIT", raising=False)
            else:
                monkeypatch.setenv("DMPT_DIAG_SPLIT", "0")
            with dm.Context(N, dirs_max=2, prec=prec, refine=refine, solver="hybrid") as ctx:
                P0, P1, P2, mu, st = ctx.mu_newton(T(h0), [T(h) for h in h1], None, beta=12.0,
                                                   Ne=N / 2.0, n=22, order=2)
            out.append((P0.cpu().numpy(), [p.cpu().numpy() for p in P1], [p.cpu().numpy() for p in P2]))
        monkeypatch.delenv("DMPT_DIAG_SPLIT", raising=False)
        (a0, a1, a2), (b0, b1, b2) = out
        d0 = np.abs(a0 - b0).max()
        d1 = max(np.abs(x - y).max() / np.abs(y).max() for x, y in zip(a1, b1))
        d2 = max(np.abs(x - y).max() / np.abs(y).max() for x, y in zip(a2, b2))
        print(f"  split vs whole: {d0:.2e} {d1:.2e} {d2:.2e}", flush=True)
        tol = 1e-9 if refine == 0 else 5e-8
        assert d0 < tol and d1 < tol and d2 < tol
        assert np.abs(a0 - a0.T).max() == 0.0
        if N == 1000:
            ref = oracle.canonical_response(h0, h1, None, 12.0, N / 2.0, 22, order=2)
            e0 = np.abs(a0 - ref["P0"]).max()
            e1 = max(np.abs(x - y).max() / np.abs(y).max() for x, y in zip(a1, ref["P1"]))
            e2 = max(np.abs(x - y).max() / np.abs(y).max() for x, y in zip(a2, ref["P2"]))
            print(f"  against the oracle: {e0:.2e} {e1:.2e} {e2:.2e}", flush=True)
            assert e0 < 1e-6 and e1 < 1e-6 and e2 < 1e-6


def test_newton_schulz_third_order_ragged(dm):
    print("case newton-schulz order 3 ragged", flush=True)
    N, n, beta, Ne = 200, 20, 10.0, 97.0
    rng = np.random.default_rng(32)
    h0 = workloads.banded(N, 5, bandwidth=16, decay=6.0)
    h1 = [np.diag(np.arange(N) % 9 - 4.0), np.diag(np.cos(0.3 * np.arange(N)))]
    h2 = [_sym(rng, N, 0.03), None]
    h3 = [None, _sym(rng, N, 0.02)]
    ref = oracle.canonical_response(h0, h1, h2, beta, Ne, n, order=3, h3s=h3)
    with dm.Context(N, dirs_max=2, prec="fp64", solver="ns") as ctx:
        r = ctx.mu_newton(T(h0), [T(h) for h in h1], [T(h2[0]), None], beta=beta, Ne=Ne, n=n,
                          order=3, H3=[None, T(h3[1])])
    P0, P1, P2, mu, st = r
    e0, e1, e2 = errs(P0, P1, P2, ref)
    e3 = _rel(r.P3, ref["P3"])
    print(f"  errs {e0:.2e} {e1:.2e} {e2:.2e} {e3:.2e}")
    assert e0 < 1e-10 and e1 < 1e-10 and e2 < 1e-10 and e3 < 1e-10


# ------------------------------------------------------------------ N = 2048 cubic lattice

@pytest.fixture(scope="module")
def cubic2048_ref():
    c = workloads.config("cubic2048")
    x = [np.diag(h) for h in c["H1"]]
    r = oracle.canonical_response(c["H0"], x, None, c["beta"], c["Ne"], c["n"], order=2)
    return c, r


@pytest.mark.timeout(300)
@pytest.mark.parametrize("prec,refine,tol,solver", [
    ("fp64", 0, 1e-10, "cg"), ("fp32", 0, 1e-6, "cg"), ("bf16x6", 0, 1e-6, "cg"), ("bf16x3", 1, 1e-6, "cg"),
    ("int8x13", 0, 1e-6, "cg"), ("bf16x3", 2, 1e-6, "cg"), ("int8x6", 2, 1e-6, "cg"),
    ("fp64", 0, 1e-10, "hybrid"), ("int8x13", 0, 1e-6, "hybrid"), ("bf16x3", 2, 1e-6, "hybrid"),
    ("int8x6", 2, 1e-6, "hybrid")])
def test_cubic2048_all_forms(dm, cubic2048_ref, prec, refine, tol, solver):
    """16 x 16 x 8 simple-cubic lattice, beta 20, n 25, orders 0-2: every element of P0, P1 and P2
    against the oracle (P0 absolute, P1 and P2 relative to max |P^(k)|), every form, with CG in
    every pass or with the shared inverse in the passes that carry jets."""
    print(f"case cubic2048 {prec} refine={refine} solver={solver}", flush=True)
    c, ref = cubic2048_ref
    with dm.Context(c["N"], dirs_max=len(c["H1"]), prec=prec, refine=refine, solver=solver) as ctx:
        P0, P1, P2, mu, st = ctx.mu_newton(T(c["H0"]), [T(h) for h in c["H1"]], None, beta=c["beta"],
                                           Ne=c["Ne"], n=c["n"], order=2)
    e0, e1, e2 = errs(P0, P1, P2, ref)
    t1 = max(abs(a - b) / abs(b) for a, b in zip(st["tr_h1p1"], ref["tr_h1p1"]))
    t2 = max(abs(a - b) / abs(b) for a, b in zip(st["tr_h1p2"], ref["tr_h1p2"]))
    print(f"  errs {e0:.2e} {e1:.2e} {e2:.2e} Tr(H1P1) {t1:.2e} Tr(H1P2) {t2:.2e} "
          f"seconds={st['seconds']:.2f} flags={st['flags']}")
    assert e0 < tol and e1 < tol and e2 < tol and t1 < tol and t2 < tol


# ------------------------------------------------------------------ N = 8192 banded (the benchmark)

@pytest.mark.timeout(600)
@pytest.mark.parametrize("prec,refine,solver", [("int8x6", 2, "hybrid"), ("int8x13", 0, "hybrid"),
                                                ("bf16x3", 2, "hybrid"), ("int8x6", 2, "cg"), ("bf16x3", 2, "cg"),
                                                ("bf16x3", 1, "cg")])
def test_banded8192_benchmark_configuration(dm, prec, refine, solver):
    """The benchmark's workload and launch configuration (one int8 6-product order-0 pass, then int8
    13-product passes, every solve with the shared inverse), and the other forms: int8 13-product
    passes only, bf16x3 first passes, CG everywhere, the bf16x6 refinement with FP64 slice
    accumulation (1); orders 0-2, 3 directions; against the oracle's stored samples and whole row
    blocks."""
    print(f"case banded8192 {prec} refine={refine} solver={solver}", flush=True)
    c = workloads.config("banded8192")
    g = np.load(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "banded8192_samples.npz"))
    with dm.Context(c["N"], dirs_max=len(c["H1"]), prec=prec, refine=refine, acc64=1, solver=solver) as ctx:
        P0, P1, P2, mu, st = ctx.mu_newton(T(c["H0"]), [T(h) for h in c["H1"]], None, beta=c["beta"],
                                           Ne=c["Ne"], n=c["n"], order=2)
    ii = torch.as_tensor(g["i"], device=P0.device)
    jj = torch.as_tensor(g["j"], device=P0.device)
    e0 = float(np.abs(P0[ii, jj].cpu().numpy() - g["P0"]).max())
    e1 = max(float(np.abs(p[ii, jj].cpu().numpy() - g["P1"][z]).max() / g["max_P1"][z]) for z, p in enumerate(P1))
    e2 = max(float(np.abs(p[ii, jj].cpu().numpy() - g["P2"][z]).max() / g["max_P2"][z]) for z, p in enumerate(P2))
    t1 = max(abs(a - b) / abs(b) for a, b in zip(st["tr_h1p1"], g["tr_h1p1"]))
    t2 = max(abs(a - b) / abs(b) for a, b in zip(st["tr_h1p2"], g["tr_h1p2"]))
    print(f"  errs {e0:.2e} {e1:.2e} {e2:.2e} Tr(H1P1) {t1:.2e} Tr(H1P2) {t2:.2e} seconds={st['seconds']:.1f}")
    assert e0 < 1e-6 and e1 < 1e-6 and e2 < 1e-6 and t1 < 1e-6 and t2 < 1e-6
    assert abs(mu[0] - float(g["mu0"])) < 1e-6
    # the canonical conditions hold on the device results
    assert abs(float(torch.trace(P0)) - c["Ne"]) < 1e-6 * c["N"]
    for p in P1 + P2:
        assert abs(float(torch.trace(p))) < 1e-6 * float(p.abs().max()) * c["N"]
    # whole rows: the first and last 128-wide tiles and across the tile edge at 4096 (x direction)
    rb = np.load(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "banded8192_rows.npz"))
    rows = torch.as_tensor(rb["rows"], device=P0.device)
    q = float(rb["quantum"])
    r0 = float(np.abs(P0[rows].cpu().numpy() - rb["P0"] * q).max())
    r1 = float(np.abs(P1[0][rows].cpu().numpy() / float(rb["max_P1"]) - rb["P1"] * q).max())
    r2 = float(np.abs(P2[0][rows].cpu().numpy() / float(rb["max_P2"]) - rb["P2"] * q).max())
    print(f"  row blocks ({len(rb['rows'])} rows x {c['N']}): {r0:.2e} {r1:.2e} {r2:.2e}")
    assert r0 < 1e-6 and r1 < 1e-6 and r2 < 1e-6


# ------------------------------------------------------------------ checks (check = 1)

@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("bf16x6", 1e-6), ("int8x13", 1e-6)])
def test_final_checks_against_oracle(dm, chain128_ref, prec, tol):
    """check = 1: the commutator ||H0 P0 - P0 H0||_F, the idempotency Tr[P0 (I - P0)] and the output
    asymmetry of the returned P0, against the same quantities of the oracle's P0."""
    print(f"case final checks {prec}", flush=True)
    c, ref = chain128_ref
    with dm.Context(c["N"], dirs_max=1, prec=prec, check=1) as ctx:
        P0, P1, P2, mu, st = ctx.mu_newton(T(c["H0"]), [T(h) for h in c["H1"]], None,
                                           beta=c["beta"], Ne=c["Ne"], n=c["n"], order=2)
    h0, p0 = c["H0"], ref["P0"]
    comm_ref = float(np.linalg.norm(h0 @ p0 - p0 @ h0))
    idem_ref = float(np.trace(p0 - p0 @ p0))
    scale = float(np.linalg.norm(h0)) * float(np.linalg.norm(p0))
    print(f"  commutator {st['commutator']:.3e} (oracle {comm_ref:.3e}) idempotency {st['idempotency']:.6e} "
          f"(oracle {idem_ref:.6e}) asymmetry {st['asymmetry']:.1e}")
    assert st["commutator"] < max(tol, 1e-12) * scale
    assert abs(st["idempotency"] - idem_ref) < tol * c["N"]
    assert st["asymmetry"] == 0.0
    # the same commutator from the returned P0 on the host
    g = P0.cpu().numpy()
    assert abs(st["commutator"] - float(np.linalg.norm(h0 @ g - g @ h0))) < 1e-12 * scale


# ------------------------------------------------------------------ stream order

def test_inputs_written_on_the_callers_stream_are_read_in_order(dm):
    """An input written by a torch kernel queued behind long work on the caller's stream (the null
    stream, and a side stream) is complete before the library reads it."""
    print("case stream order", flush=True)
    N, beta, n, mu = 512, 10.0, 20, 0.05
    h0 = workloads.chain_1d(N, 5)
    ref = oracle.density(h0, beta, n, mu)
    src = T(h0)
    big = torch.randn(4096, 4096, device=src.device)
    torch.cuda.synchronize()
    for side in (False, True):
        stream = torch.cuda.Stream() if side else torch.cuda.current_stream()
        with torch.cuda.stream(stream):
            with dm.Context(N, dirs_max=0, prec="fp64") as ctx:
                H = torch.zeros((N, N), dtype=torch.float64, device=src.device)
                torch.cuda.synchronize()
                x = big
                for _ in range(6):
                    x = torch.tanh(x @ x * 1e-3)  # long kernels ahead of the copy
                H.copy_(src)                      # the input is written last
                P0, _ = ctx.fermi_recursion(H, beta, mu, n)
                err = float(np.abs(P0.cpu().numpy() - ref).max())
        print(f"  side stream {side}: err {err:.2e}")
        assert err < 1e-12


def test_int8_paths_without_int8_products_say_so(dm):
    """The batched solve and the adjoint have no int8 products: they return DMPT_ERR_UNSUPPORTED
    instead of computing with another engine."""
    print("case int8 unsupported paths", flush=True)
    from paper_1503_07037_amd import _lib as L
    N, beta, n = 128, 10.0, 20
    h0 = workloads.chain_1d(N, 3)
    with dm.Context(N, dirs_max=1, prec="int8x13") as ctx:
        with pytest.raises(dm.DMPTError) as e:
            ctx.mu_newton_batched([T(h0)], [[T(np.diag(np.arange(N) - N / 2.0))]], [beta], [N / 2.0], n=n, order=1)
        assert e.value.status == L.DMPT_ERR_UNSUPPORTED
        with pytest.raises(dm.DMPTError) as e:
            ctx.backward(T(h0), beta=beta, Ne=N / 2.0, n=n, Abar=T(np.eye(N)))
        assert e.value.status == L.DMPT_ERR_UNSUPPORTED


@pytest.mark.parametrize("prec,extra", [("fp64", {}), ("bf16x3", {"refine": 2}), ("int8x13", {})])
def test_debug_checks_leave_results_unchanged(dm, chain128_ref, prec, extra, monkeypatch):
    """DMPT_DEBUG_CHECKS (every product output scanned for non-finite values, every iterate checked
    for non-finite values and exact symmetry after every recursion step) passes on a canonical
    solve and changes no bit of the results."""
    print(f"case debug checks {prec} {extra}", flush=True)
    c, ref = chain128_ref
    out = {}
    for dbg in (0, 1):
        if dbg:
            monkeypatch.setenv("DMPT_DEBUG_CHECKS", "1")
        else:
            monkeypatch.delenv("DMPT_DEBUG_CHECKS", raising=False)
        with dm.Context(c["N"], dirs_max=1, prec=prec, **extra) as ctx:
            P0, P1, P2, mu, st = ctx.mu_newton(T(c["H0"]), [T(h) for h in c["H1"]], None,
                                               beta=c["beta"], Ne=c["Ne"], n=c["n"], order=2)
        out[dbg] = (P0.cpu().numpy(), P1[0].cpu().numpy(), P2[0].cpu().numpy(), list(mu))
    for a, b in zip(out[0][:3], out[1][:3]):
        assert np.array_equal(a, b)
    assert out[0][3] == out[1][3]
