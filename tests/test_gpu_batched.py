"""GPU parity of the batched canonical solve (dmpt_mu_newton_batched).

Systems of uneven size share graph-captured batched passes; each one must
match the FP64 oracle as if solved alone.  The full 64-system workload runs
with FP32 products at orders 0-2 and is compared on the oracle's stored
per-system samples and, for five systems, element by element.
"""
import os

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
HERE = os.path.dirname(os.path.abspath(__file__))


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


SMALL = [((4, 4, 4), 7.0), ((6, 5, 4), 31.0), ((7, 7, 5), 12.5), ((8, 6, 6), 22.0), ((10, 8, 5), 5.5)]


@pytest.fixture(scope="module")
def small_batch():
    systems = []
    for k, (dims, beta) in enumerate(SMALL):
        h0 = workloads.cubic_lattice(*dims, seed=100 + k)
        h1 = list(workloads.lattice_dipoles(*dims))
        N = h0.shape[0]
        ref = oracle.canonical_response(h0, h1, None, beta, N / 2.0, 25, order=2)
        systems.append(dict(h0=h0, h1=[np.diag(v) for v in h1], beta=beta, Ne=N / 2.0, ref=ref))
    return systems


@pytest.mark.parametrize("prec,order,tol", [("fp64", 2, 1e-10), ("fp32", 1, 1e-6), ("fp32", 2, 1e-6)])
def test_small_uneven_batch(dm, small_batch, prec, order, tol):
    print(f"case batched {prec} order {order}", flush=True)
    nmax = max(s["h0"].shape[0] for s in small_batch)
    with dm.Context(nmax, dirs_max=3, prec=prec) as ctx:
        P0, P1, P2, mus, st = ctx.mu_newton_batched(
            [T(s["h0"]) for s in small_batch], [[T(h) for h in s["h1"]] for s in small_batch],
            [s["beta"] for s in small_batch], [s["Ne"] for s in small_batch], n=25, order=order)
    print(f"  passes={st['newton_iters']} seconds={st['seconds']:.2f} mfma_flops={st['mfma_flops']:.3e}")
    # executed work is tallied on the device: positive, and at most every captured
    # product of every system on every replay
    assert 0.0 < st["mfma_flops"] and st["useful_flops"] <= st["mfma_flops"]
    for k, s in enumerate(small_batch):
        r = s["ref"]
        e0 = np.abs(P0[k].cpu().numpy() - r["P0"]).max()
        e1 = max(np.abs(P1[k][z].cpu().numpy() - r["P1"][z]).max() / np.abs(r["P1"][z]).max()
                 for z in range(3))
        e2 = 0.0
        if order >= 2:
            e2 = max(np.abs(P2[k][z].cpu().numpy() - r["P2"][z]).max() / np.abs(r["P2"][z]).max()
                     for z in range(3))
        print(f"  system {k} N={s['h0'].shape[0]}: {e0:.2e} {e1:.2e} {e2:.2e}")
        assert e0 < tol and e1 < tol and e2 < tol
        assert abs(mus[k][0] - r["mu0"]) < 10 * tol


def test_batch_matches_single_system_path(dm, small_batch):
    """The batched solve and the single-system solve agree (FP64)."""
    print("case batched vs single", flush=True)
    s = small_batch[2]
    N = s["h0"].shape[0]
    with dm.Context(N, dirs_max=3, prec="fp64") as ctx:
        P0b, P1b, _, _, _ = ctx.mu_newton_batched([T(s["h0"])], [[T(h) for h in s["h1"]]], [s["beta"]],
                                                  [s["Ne"]], n=25, order=1)
        P0, P1, _, _, _ = ctx.mu_newton(T(s["h0"]), [T(h) for h in s["h1"]], None, beta=s["beta"],
                                        Ne=s["Ne"], n=25, order=1)
    assert np.abs(P0b[0].cpu().numpy() - P0.cpu().numpy()).max() < 1e-11
    assert np.abs(P1b[0][0].cpu().numpy() - P1[0].cpu().numpy()).max() < 1e-10 * np.abs(
        P1[0].cpu().numpy()).max()


@pytest.mark.timeout(900)
def test_batch64_fp32_full_workload(dm):
    """64 cubic systems, N in [256, 3072] log-uniform, beta in U(5, 40), 3 directions, orders 0-2,
    FP32 products: every system on the oracle's stored samples of P0, P1 and P2, and five systems
    (the smallest, the largest and three between) element by element against the oracle."""
    print("case batch64 fp32", flush=True)
    path = os.path.join(HERE, "golden", "batch64_samples.npz")
    if not os.path.exists(path):
        pytest.skip("golden samples missing")
    g = np.load(path)
    c = workloads.CONFIGS["batch64"]
    systems = workloads.batched_systems(c["seed"], count=c["count"])
    H0s, H1s = [], []
    for sy in systems:
        lx, ly, lz = sy["dims"]
        H0s.append(T(workloads.cubic_lattice(lx, ly, lz, sy["seed"])))
        H1s.append([T(np.diag(v)) for v in workloads.lattice_dipoles(lx, ly, lz)])
    nmax = max(sy["N"] for sy in systems)
    with dm.Context(nmax, dirs_max=3, prec="fp32") as ctx:
        P0, P1, P2, mus, st = ctx.mu_newton_batched(H0s, H1s, [sy["beta"] for sy in systems],
                                                    [sy["Ne"] for sy in systems], n=c["n"], order=2)
    print(f"  passes={st['newton_iters']} seconds={st['seconds']:.1f} cg={st['cg_iters_total']} "
          f"unconverged={st['cg_unconverged']} flags={st['flags']} "
          f"useful TFLOP/s={st['useful_flops'] / st['seconds'] / 1e12:.1f}")
    worst = 0.0
    for k in range(len(systems)):
        ii = torch.as_tensor(g["i"][k], device=P0[k].device)
        jj = torch.as_tensor(g["j"][k], device=P0[k].device)
        e0 = float(np.abs(P0[k][ii, jj].cpu().numpy() - g["P0"][k]).max())
        e1 = max(float(np.abs(P1[k][z][ii, jj].cpu().numpy() - g["P1"][k][z]).max() / g["max_P1"][k][z])
                 for z in range(3))
        e2 = max(float(np.abs(P2[k][z][ii, jj].cpu().numpy() - g["P2"][k][z]).max() / g["max_P2"][k][z])
                 for z in range(3))
        worst = max(worst, e0, e1, e2)
    print(f"  worst sampled error {worst:.2e}")
    assert worst < 1e-6
    order = sorted(range(len(systems)), key=lambda k: systems[k]["N"])
    for k in [order[0], order[16], order[32], order[48], order[-1]]:
        sy = systems[k]
        lx, ly, lz = sy["dims"]
        r = oracle.canonical_response(workloads.cubic_lattice(lx, ly, lz, sy["seed"]),
                                      list(workloads.lattice_dipoles(lx, ly, lz)), None, sy["beta"],
                                      sy["Ne"], c["n"], order=2)
        e0 = float(np.abs(P0[k].cpu().numpy() - r["P0"]).max())
        e1 = max(float(np.abs(P1[k][z].cpu().numpy() - r["P1"][z]).max() / np.abs(r["P1"][z]).max())
                 for z in range(3))
        e2 = max(float(np.abs(P2[k][z].cpu().numpy() - r["P2"][z]).max() / np.abs(r["P2"][z]).max())
                 for z in range(3))
        print(f"  system {k} N={sy['N']} beta={sy['beta']:.1f}: full {e0:.2e} {e1:.2e} {e2:.2e}")
        assert e0 < 1e-6 and e1 < 1e-6 and e2 < 1e-6


@pytest.mark.parametrize("d,order", [(1, 1), (3, 1), (3, 2)])
def test_linear_and_joint_schedules_agree(dm, small_batch, d, order):
    """FP64: the device-side linear schedule (identity response as an extra direction, exact
    Tr P1 = 0 and Tr P2 = 0 corrections) and Algorithm 1's joint Newton reach the oracle's fixed
    point at orders 1 and 2."""
    print(f"case batched schedules d={d} order={order}", flush=True)
    nmax = max(s["h0"].shape[0] for s in small_batch)
    out = {}
    for sched in (0, 1):
        with dm.Context(nmax, dirs_max=d, prec="fp64", schedule=sched) as ctx:
            P0, P1, P2, mus, st = ctx.mu_newton_batched(
                [T(s["h0"]) for s in small_batch], [[T(h) for h in s["h1"][:d]] for s in small_batch],
                [s["beta"] for s in small_batch], [s["Ne"] for s in small_batch], n=25, order=order)
        out[sched] = (P0, P1, P2, mus)
        print(f"  schedule {sched}: passes={st['newton_iters']} seconds={st['seconds']:.2f} "
              f"flags={st['flags']}")
    for k, s in enumerate(small_batch):
        r = s["ref"]
        for sched in (0, 1):
            P0, P1, P2, mus = out[sched]
            e0 = np.abs(P0[k].cpu().numpy() - r["P0"]).max()
            e1 = max(np.abs(P1[k][z].cpu().numpy() - r["P1"][z]).max() / np.abs(r["P1"][z]).max()
                     for z in range(d))
            e2 = 0.0
            if order >= 2:
                e2 = max(np.abs(P2[k][z].cpu().numpy() - r["P2"][z]).max() / np.abs(r["P2"][z]).max()
                         for z in range(d))
            assert e0 < 1e-10 and e1 < 1e-10 and e2 < 1e-10, (k, sched, e0, e1, e2)
            for z in range(d):
                assert abs(mus[k][1 + z] - r["mu1"][z]) < 1e-9 * max(1.0, abs(r["mu1"][z]))
                if order >= 2:
                    assert abs(mus[k][1 + d + z] - r["mu2"][z]) < 1e-9 * max(1.0, abs(r["mu2"][z]))


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-9)])
def test_grouped_and_per_bucket_launches_agree(dm, small_batch, prec, tol):
    """The grouped launches (every product of a step as one launch over all size buckets) give the
    results of the bucket-by-bucket launches (orders 0-2, five buckets)."""
    print(f"case batched grouped vs per-bucket {prec}", flush=True)
    nmax = max(s["h0"].shape[0] for s in small_batch)
    out = {}
    for grouped in (1, 0):
        with dm.Context(nmax, dirs_max=3, prec=prec, grouped=grouped) as ctx:
            P0, P1, P2, mus, st = ctx.mu_newton_batched(
                [T(s["h0"]) for s in small_batch], [[T(h) for h in s["h1"]] for s in small_batch],
                [s["beta"] for s in small_batch], [s["Ne"] for s in small_batch], n=25, order=2)
        out[grouped] = (P0, P1, P2)
        print(f"  grouped={grouped}: passes={st['newton_iters']} seconds={st['seconds']:.2f}")
    for k in range(len(small_batch)):
        a, b = out[1], out[0]
        assert np.abs(a[0][k].cpu().numpy() - b[0][k].cpu().numpy()).max() < tol
        for z in range(3):
            for o in (1, 2):
                x, y = a[o][k][z].cpu().numpy(), b[o][k][z].cpu().numpy()
                assert np.abs(x - y).max() < tol * max(1.0, np.abs(y).max())
