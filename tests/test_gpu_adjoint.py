"""GPU parity of the adjoint dmpt_backward: G = d Tr(A P0)/d H0 (canonical).

Checked against the oracle's canonical first-order response to sym(A) (the
exact adjoint of the canonical map), the identity Tr(A P1[H1]) = <G, H1>,
Tr G = 0 (a shift of H0 by the identity only moves mu0), checkpoint-stride
independence, the torch.autograd wrapper, and the full-size workload
(16^3 cubic lattice, FP32 products) element by element.
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


def _sym(rng, n, s=1.0):
    a = rng.standard_normal((n, n)) * s
    return 0.5 * (a + a.T)


@pytest.mark.parametrize("N,dims", [(96, (6, 4, 4)), (250, (10, 5, 5))])
def test_adjoint_fp64_vs_oracle(dm, N, dims):
    print(f"case adjoint fp64 N={N}", flush=True)
    h0 = workloads.cubic_lattice(*dims, seed=N)
    x, _, _ = workloads.lattice_dipoles(*dims)
    A = np.diag(x)
    beta, n, Ne = 10.0, 20, N / 2.0
    ref = oracle.adjoint_grad(h0, beta, Ne, n, A)
    with dm.Context(N, dirs_max=1, prec="fp64", ckpt_every=5) as ctx:
        G, st = ctx.backward(T(h0), beta, Ne, n, T(A))
    g = G.cpu().numpy()
    err = np.abs(g - ref).max() / np.abs(ref).max()
    print(f"  rel err {err:.2e} newton={st['newton_iters']} cg={st['cg_iters_total']}")
    assert err < 1e-10
    assert np.abs(g - g.T).max() == 0.0
    assert abs(np.trace(g)) < 1e-10 * np.abs(g).sum()


def test_adjoint_identity_with_forward_response(dm):
    """Tr(A P1[H1]) = <G, H1> for a random symmetric H1 (both from the GPU)."""
    print("case adjoint identity", flush=True)
    N, beta, n, Ne = 160, 8.0, 18, 75.0
    rng = np.random.default_rng(7)
    h0 = workloads.chain_1d(N, 7)
    A = _sym(rng, N, 0.3)
    H1 = _sym(rng, N, 0.2)
    with dm.Context(N, dirs_max=1, prec="fp64") as ctx:
        G, _ = ctx.backward(T(h0), beta, Ne, n, T(A))
        _, P1, _, _, _ = ctx.mu_newton(T(h0), [T(H1)], None, beta=beta, Ne=Ne, n=n, order=1)
    lhs = float(np.sum(A * P1[0].cpu().numpy()))
    rhs = float(np.sum(G.cpu().numpy() * H1))
    assert abs(lhs - rhs) < 1e-10 * max(1.0, abs(lhs))


def test_checkpoint_stride_does_not_change_result(dm):
    print("case adjoint checkpoints", flush=True)
    N, beta, n, Ne = 128, 6.0, 17, 60.0
    h0 = workloads.chain_1d(N, 3)
    A = np.diag(np.arange(N) - N / 2.0)
    out = []
    for ck in (1, 5, 17):
        with dm.Context(N, dirs_max=1, prec="fp64", ckpt_every=ck) as ctx:
            G, _ = ctx.backward(T(h0), beta, Ne, n, T(A), mu0=0.05)
        out.append(G.cpu().numpy())
    assert np.array_equal(out[0], out[1]) and np.array_equal(out[1], out[2])


def test_autograd_function(dm):
    print("case autograd", flush=True)
    from paper_1503_07037_amd.autograd import fermi_canonical
    N, beta, n, Ne = 96, 9.0, 16, 40.0
    rng = np.random.default_rng(4)
    h0 = workloads.chain_1d(N, 4)
    A = _sym(rng, N)
    with dm.Context(N, dirs_max=1, prec="fp64") as ctx:
        H = T(h0).requires_grad_(True)
        P0 = fermi_canonical(H, beta, Ne, n, ctx)
        loss = (T(A) * P0).sum()
        (g,) = torch.autograd.grad(loss, H)
    ref = oracle.adjoint_grad(h0, beta, Ne, n, A)
    assert np.abs(g.cpu().numpy() - ref).max() < 1e-10 * np.abs(ref).max()


@pytest.mark.timeout(600)
def test_adjoint4096_fp32_full_size(dm):
    """The 16^3 cubic workload (beta 20, n 25, A = diag(x), checkpoints every 5), FP32 products:
    every element of G against the oracle's canonical first-order response to A (relative to
    max |G|), and Tr G = 0."""
    print("case adjoint4096 fp32", flush=True)
    c = workloads.config("adjoint4096")
    x = np.diag(c["H1"][0]).copy()
    ref = oracle.adjoint_grad(c["H0"], c["beta"], c["Ne"], c["n"], x)
    with dm.Context(c["N"], dirs_max=1, prec="fp32", ckpt_every=5) as ctx:
        G, st = ctx.backward(T(c["H0"]), c["beta"], c["Ne"], c["n"], T(np.diag(x)))
    g = G.cpu().numpy()
    err = float(np.abs(g - ref).max() / np.abs(ref).max())
    print(f"  rel err {err:.2e} seconds={st['seconds']:.1f} cg={st['cg_iters_total']}")
    assert err < 1e-6
    assert abs(np.trace(g)) < 1e-6 * np.abs(g).sum()
