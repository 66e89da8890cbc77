"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: the
closed forms of Appendix A evaluated independently, the scalar recursions of
Eq. (Rec_F_2), the Fermi-Dirac limit of Eq. (Rec_F_1), the matrix recursion
of Eq. (Rec_F_2) carried out on truncated power series in lambda (X form, no
eigenvalues), canonical finite differences in lambda,
special cases with known answers, brute-force sums and the free-energy
identities of Sec. III.
"""
import math

import numpy as np
import pytest

import oracle as o
import workloads as w
import series_recursion as sr

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _sym(rng, n, scale=1.0):
    a = rng.standard_normal((n, n)) * scale
    return 0.5 * (a + a.T)


# ---------------------------------------------------------------- scalar map

@pytest.mark.parametrize("M", [1, 2, 5, 10, 20, 30])
def test_phi_matches_scalar_recursions(M):
    """Closed form == M steps of the paper's map x -> x^2/(x^2+(1-x)^2) (Eq. Rec_F_2).

    The X-form is iterated in extended precision for small M; the shifted
    d-form d -> 2d/(1+4d^2) (x = 1/2 - d) in FP64 for every M.
    """
    beta = 10.0
    lim = min(3.0, 0.95 / math.ldexp(beta, -(M + 1)))   # stay inside the range |s e| < 1
    e = np.linspace(-lim, lim, 241)
    ref = o.phi(e, beta, M)
    # d-form in fp64
    d = math.ldexp(beta, -(M + 2)) * e
    for _ in range(M):
        d = 2.0 * d / (1.0 + 4.0 * d * d)
    assert np.max(np.abs((0.5 - d) - ref)) < 2e-15
    if M <= 10:
        x = np.longdouble(0.5) - np.longdouble(math.ldexp(beta, -(M + 2))) * e.astype(np.longdouble)
        for _ in range(M):
            x = x * x / (x * x + (1 - x) * (1 - x))
        assert np.max(np.abs(x.astype(np.float64) - ref)) < 1e-15 * 2 ** M


@pytest.mark.parametrize("M", [1, 3, 8, 16, 30])
def test_phi_matches_pade_power_form(M):
    """Appendix A: phi_M(e) = f_{2^M}(x), f_n(x) = x^n/(x^n+(1-x)^n), x = 1/2 - beta e/(4n)."""
    beta = 40.0
    lim = min(4.0, 0.95 / math.ldexp(beta, -(M + 1)))
    e = np.linspace(-lim, lim, 161)
    assert np.max(np.abs(o.phi_pade(e, beta, M) - o.phi(e, beta, M))) < 5e-15
    if M <= 4:
        n = 2 ** M
        x = 0.5 - beta * e / (4 * n)
        if np.all((x > 0) & (x < 1)):
            direct = x ** n / (x ** n + (1 - x) ** n)
            assert np.max(np.abs(direct - o.phi(e, beta, M))) < 1e-14


def test_pade_composition():
    """Appendix A: f_{m n} = f_m o f_n for the Pade polynomial."""
    x = np.linspace(0.01, 0.99, 99)

    def f(n, t):
        return t ** n / (t ** n + (1 - t) ** n)

    for m, n in ((2, 2), (2, 4), (4, 2), (2, 8)):
        assert np.max(np.abs(f(m, f(n, x)) - f(m * n, x))) < 1e-14


def test_phi_tends_to_fermi_dirac():
    """Eq. (Rec_F_1): the expansion approaches [exp(beta(e)) + 1]^-1 as M grows."""
    beta = 10.0
    e = np.linspace(-3.0, 3.0, 601)
    fd = o.fermi_dirac(e, beta)
    errs = [np.max(np.abs(o.phi(e, beta, M) - fd)) for M in (4, 8, 12, 16, 20, 25)]
    assert all(b < a for a, b in zip(errs, errs[1:]) if a > 1e-15)
    assert errs[0] > 1e-4           # a short expansion is visibly different
    assert errs[-1] < 1e-14


def test_phi_derivatives_vs_finite_differences():
    beta, M = 20.0, 12
    e = np.linspace(-1.0, 1.0, 41)
    p1, p2, p4 = o.phi_derivs(e, beta, M)
    h = 1e-4
    f = lambda x: o.phi(x, beta, M)
    d1 = (f(e - 2 * h) - 8 * f(e - h) + 8 * f(e + h) - f(e + 2 * h)) / (12 * h)
    d2 = (-f(e - 2 * h) + 16 * f(e - h) - 30 * f(e) + 16 * f(e + h) - f(e + 2 * h)) / (12 * h * h)
    assert np.max(np.abs(d1 - p1)) < 1e-8 * beta
    assert np.max(np.abs(d2 - p2)) < 1e-4 * beta ** 2
    # fourth derivative from the analytic second derivative, differenced twice
    h = 1e-3
    g = lambda x: o.phi_derivs(x, beta, M)[1]
    d4 = (g(e - h) - 2 * g(e) + g(e + h)) / (h * h)
    assert np.max(np.abs(d4 - p4)) < 2e-3 * beta ** 4


def test_divided_differences_vs_extended_precision():
    """dd1/dd2 against plain quotients of phi evaluated in 80-bit long double."""
    beta, M = 40.0, 30
    s = np.longdouble(math.ldexp(beta, -(M + 1)))
    K = np.longdouble(2.0) ** M

    def phil(e):
        e = np.asarray(e, dtype=np.longdouble)
        return np.longdouble(0.5) - np.tanh(K * np.arctanh(s * e)) / 2

    rng = np.random.default_rng(3)
    a = rng.uniform(-0.3, 0.3, 200)
    b = a + rng.uniform(1e-3, 0.2, 200) * rng.choice([-1, 1], 200)
    ref1 = (phil(a) - phil(b)) / (a.astype(np.longdouble) - b.astype(np.longdouble))
    assert np.max(np.abs(o.dd1(a, b, beta, M) - ref1.astype(np.float64))) < 1e-12
    c = b + rng.uniform(1e-3, 0.2, 200)
    ref2 = (ref1 - (phil(b) - phil(c)) / (b.astype(np.longdouble) - c.astype(np.longdouble))) / (
        a.astype(np.longdouble) - c.astype(np.longdouble))
    got2 = o.dd2(a, b, c, beta, M, 1e-5)
    assert np.max(np.abs(got2 - ref2.astype(np.float64))) < 1e-9
    # coincident points reduce to derivatives
    p1, p2, _ = o.phi_derivs(a, beta, M)
    assert np.max(np.abs(o.dd1(a, a, beta, M) - p1)) < 1e-12 * beta
    assert np.max(np.abs(o.dd2(a, a, a, beta, M, 1e-5) - 0.5 * p2)) < 1e-12 * beta ** 2
    # a nearly coincident pair next to a far point: continuity across delta
    near = o.dd2(a, a + 2e-5, c, beta, M, 1e-5)
    ref_near = (o.dd1(a, c, beta, M) - o.dd1(a + 2e-5, c, beta, M)) / (-2e-5)
    assert np.max(np.abs(near - ref_near)) < 1e-6 * beta ** 2


# ---------------------------------------------------------------- P0

@pytest.mark.parametrize("name", ["chain128"])
def test_p0_invariants(name):
    """Tr P0 = Ne, [H0, P0] = 0, symmetric, spectrum in (0, 1) (Sec. II)."""
    c = w.config(name)
    r = o.canonical_response(c["H0"], c["H1"], None, c["beta"], c["Ne"], c["n"], order=0)
    P0, H0 = r["P0"], c["H0"]
    assert abs(np.trace(P0) - c["Ne"]) < 1e-11
    assert np.max(np.abs(H0 @ P0 - P0 @ H0)) < 1e-12
    assert np.max(np.abs(P0 - P0.T)) < 1e-14
    ev = np.linalg.eigvalsh(P0)
    assert ev.min() > 0 and ev.max() < 1


def test_mu_root_is_unique_and_tight():
    c = w.config("chain128")
    ev = np.linalg.eigvalsh(c["H0"])
    mu = o.mu_canonical(ev, c["beta"], c["n"], c["Ne"])
    occ = np.sum(o.phi(ev - mu, c["beta"], c["n"]))
    assert abs(occ - c["Ne"]) < 1e-12
    # strictly increasing occupation
    assert np.sum(o.phi(ev - (mu - 1e-6), c["beta"], c["n"])) < occ < np.sum(o.phi(ev - (mu + 1e-6), c["beta"], c["n"]))


# ---------------------------------------------------------------- series evaluation of Eq. (Rec_F_2)

@pytest.mark.parametrize("M,beta", [(6, 4.0), (10, 8.0), (12, 3.0)])
def test_series_recursion_canonical_agrees(M, beta):
    """Eq. (Rec_F_2) on truncated series in lambda (X form, Newton on the mu jet) reaches the oracle's fixed point."""
    n = 14
    rng = np.random.default_rng(M)
    h0 = w.chain_1d(n, M)
    h1 = np.diag(np.arange(n) - n / 2.0)
    h2 = _sym(rng, n, 0.05)
    Ne = 6.0
    P, mu, _ = sr.canonical([h0, h1, h2], beta, Ne, M, 2)
    r = o.canonical_response(h0, [h1], [h2], beta, Ne, M, order=2)
    tol = 1e-15 * 2 ** M * 10
    assert np.max(np.abs(P[0] - r["P0"])) < tol
    assert np.max(np.abs(P[1] - r["P1"][0])) < tol * np.max(np.abs(r["P1"][0])) * 10
    assert np.max(np.abs(P[2] - r["P2"][0])) < tol * np.max(np.abs(r["P2"][0])) * 20
    assert abs(mu[0] - r["mu0"]) < tol
    assert abs(mu[1] - r["mu1"][0]) < tol * 10
    assert abs(mu[2] - r["mu2"][0]) < tol * 100


def test_grand_canonical_response_agrees_with_series_pass():
    """One pass at a fixed mu jet (no Newton) against the series recursion."""
    n, M, beta = 10, 8, 5.0
    rng = np.random.default_rng(11)
    h0 = _sym(rng, n)
    h1 = _sym(rng, n, 0.3)
    h2 = _sym(rng, n, 0.2)
    mu = [0.1, 0.25, -0.4]
    X = sr.recursion([h0, h1, h2], beta, M, mu, 2)
    r = o.response(h0, [h1], [h2], beta, M, (mu[0], [mu[1]], [mu[2]]), order=2)
    assert np.max(np.abs(X[0] - r["P0"])) < 1e-12
    assert np.max(np.abs(X[1] - r["P1"][0])) < 1e-12
    assert np.max(np.abs(X[2] - r["P2"][0])) < 1e-11


# ---------------------------------------------------------------- perturbations

def _p_of_lambda(h0, h1, h2, lam, beta, Ne, M):
    h = h0 + lam * h1 + (lam * lam) * h2
    wv = o.eig(h)
    mu = o.mu_canonical(wv[0], beta, M, Ne)
    return o.density(h, beta, M, mu, eigh=wv), mu


def test_canonical_finite_differences_in_lambda():
    """P1 = dP/dlambda and P2 = (1/2) d^2P/dlambda^2 with mu(lambda) re-solved (Eqs. P_resp, H_prt)."""
    n, M, beta, Ne = 24, 20, 10.0, 11.0
    rng = np.random.default_rng(5)
    h0 = w.chain_1d(n, 5)
    h1 = np.diag(np.arange(n) - n / 2.0) / n
    h2 = _sym(rng, n, 0.05)
    r = o.canonical_response(h0, [h1], [h2], beta, Ne, M, order=2)

    def d1(h):
        pp, mp = _p_of_lambda(h0, h1, h2, h, beta, Ne, M)
        pm, mm = _p_of_lambda(h0, h1, h2, -h, beta, Ne, M)
        return (pp - pm) / (2 * h), (mp - mm) / (2 * h)

    def d2(h):
        pp, mp = _p_of_lambda(h0, h1, h2, h, beta, Ne, M)
        pm, mm = _p_of_lambda(h0, h1, h2, -h, beta, Ne, M)
        p0, m0 = _p_of_lambda(h0, h1, h2, 0.0, beta, Ne, M)
        return (pp - 2 * p0 + pm) / (2 * h * h), (mp - 2 * m0 + mm) / (2 * h * h)

    h = 1e-3
    a1, b1 = d1(h)
    a2, b2 = d1(2 * h)
    P1_fd = (4 * a1 - a2) / 3
    mu1_fd = (4 * b1 - b2) / 3
    s1 = np.max(np.abs(r["P1"][0]))
    assert np.max(np.abs(P1_fd - r["P1"][0])) < 1e-9 * max(s1, 1)
    assert abs(mu1_fd - r["mu1"][0]) < 1e-9
    h = 4e-3
    a1, b1 = d2(h)
    a2, b2 = d2(2 * h)
    P2_fd = (4 * a1 - a2) / 3
    mu2_fd = (4 * b1 - b2) / 3
    s2 = np.max(np.abs(r["P2"][0]))
    assert np.max(np.abs(P2_fd - r["P2"][0])) < 2e-6 * max(s2, 1)
    assert abs(mu2_fd - r["mu2"][0]) < 2e-6 * max(abs(r["mu2"][0]), 1)
    assert abs(np.trace(r["P1"][0])) < 1e-12 and abs(np.trace(r["P2"][0])) < 1e-11


def test_identity_perturbation_only_shifts_mu():
    """H1 = I moves mu1 by exactly 1 and leaves P1 = 0; H2 = I (H1 = 0) gives mu2 = 1, P2 = 0."""
    c = w.config("chain128")
    n = c["N"]
    r = o.canonical_response(c["H0"], [np.eye(n)], None, c["beta"], c["Ne"], c["n"], order=2)
    assert abs(r["mu1"][0] - 1.0) < 1e-13
    assert np.max(np.abs(r["P1"][0])) < 1e-12
    assert np.max(np.abs(r["P2"][0])) < 1e-10
    r = o.canonical_response(c["H0"], [np.zeros((n, n))], [np.eye(n)], c["beta"], c["Ne"], c["n"], order=2)
    assert abs(r["mu2"][0] - 1.0) < 1e-13
    assert np.max(np.abs(r["P2"][0])) < 1e-12


def test_two_level_analytic():
    """2x2: H0 = diag(a, b), off-diagonal H1 = v: P1_12 = v (phi(a) - phi(b))/(a - b), mu1 = 0."""
    beta, M = 7.0, 15
    a, b, v = -0.3, 0.45, 0.2
    h0 = np.diag([a, b])
    h1 = np.array([[0.0, v], [v, 0.0]])
    mu = 0.1
    r = o.response(h0, [h1], None, beta, M, (mu, [0.0], [0.0]), order=1)
    expect = v * (o.phi(a - mu, beta, M) - o.phi(b - mu, beta, M)) / (a - b)
    assert abs(r["P1"][0][0, 1] - expect) < 1e-15
    assert abs(r["P1"][0][0, 0]) < 1e-16 and abs(r["P1"][0][1, 1]) < 1e-16
    # canonical: mu1 = 0 because the diagonal of H1 in the eigenbasis vanishes
    rc = o.canonical_response(h0, [h1], None, beta, 1.0, M, order=1)
    assert abs(rc["mu1"][0]) < 1e-15


def test_second_order_kernel_bruteforce():
    """Q_ij = sum_k phi[e_i,e_k,e_j] E_ik E_kj by a plain triple loop with a plain quotient rule."""
    n, M, beta = 9, 14, 6.0
    rng = np.random.default_rng(2)
    e = np.sort(rng.uniform(-1, 1, n))
    e[4] = e[3] + 3e-7            # a near-degenerate pair goes through the direct path
    E = _sym(rng, n)
    F1 = o.dd1(e[:, None], e[None, :], beta, M)
    got = o.dmpt_oracle._second_order_kernel(e, F1, E, beta, M, 1e-5)
    ref = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            acc = 0.0
            for k in range(n):
                pts = sorted([e[i], e[k], e[j]])
                if pts[2] - pts[0] > 1e-3:
                    lo, mid, hi = pts
                    f01 = (o.phi(lo, beta, M) - o.phi(mid, beta, M)) / (lo - mid) if mid - lo > 1e-3 else o.dd1(lo, mid, beta, M)
                    f12 = (o.phi(mid, beta, M) - o.phi(hi, beta, M)) / (mid - hi) if hi - mid > 1e-3 else o.dd1(mid, hi, beta, M)
                    dd = (f01 - f12) / (lo - hi)
                else:
                    dd = 0.5 * o.phi_derivs(np.mean(pts), beta, M)[1]
                acc += dd * E[i, k] * E[k, j]
            ref[i, j] = acc
    assert np.max(np.abs(got - ref)) < 1e-9 * np.max(np.abs(ref))


def test_reciprocity_of_first_order_response():
    """Tr(A P1[B]) = Tr(B P1[A]) for the canonical first-order kernel."""
    n, M, beta, Ne = 30, 18, 8.0, 13.0
    rng = np.random.default_rng(9)
    h0 = _sym(rng, n)
    A, B = _sym(rng, n), _sym(rng, n)
    pa = o.canonical_response(h0, [A], None, beta, Ne, M, order=1)["P1"][0]
    pb = o.canonical_response(h0, [B], None, beta, Ne, M, order=1)["P1"][0]
    assert abs(np.sum(A * pb) - np.sum(B * pa)) < 1e-12 * max(1.0, abs(np.sum(A * pb)))


def test_adjoint_matches_directional_derivatives():
    """G = d Tr(A P0)/dH0 (canonical) against central differences along symmetric directions."""
    n, M, beta, Ne = 20, 16, 9.0, 9.0
    rng = np.random.default_rng(21)
    h0 = w.chain_1d(n, 21)
    A = np.diag(np.arange(n) - n / 2.0)
    G = o.adjoint_grad(h0, beta, Ne, M, A)
    assert np.max(np.abs(G - G.T)) < 1e-13
    for t in range(4):
        E = _sym(rng, n)
        E /= np.linalg.norm(E)
        f = lambda h: float(np.sum(A * _p_of_lambda(h0, E, np.zeros_like(E), h, beta, Ne, M)[0]))
        hh = 1e-4
        fd1 = (f(hh) - f(-hh)) / (2 * hh)
        fd2 = (f(2 * hh) - f(-2 * hh)) / (4 * hh)
        fd = (4 * fd1 - fd2) / 3
        assert abs(fd - np.sum(G * E)) < 1e-8 * max(1.0, abs(fd))


# ---------------------------------------------------------------- free energy

def test_n_plus_one_rule_second_order():
    """Eq. (Resp_0): Omega^(2) = (1/2) Tr[H1 P1] + Tr[H2 P0] equals the lambda^2 coefficient of Omega."""
    n, beta, Ne, M = 24, 6.0, 10.0, 40  # M large: the expansion equals Fermi-Dirac to rounding
    rng = np.random.default_rng(4)
    h0 = w.chain_1d(n, 4)
    h1 = np.diag(np.arange(n) - n / 2.0) / n
    h2 = _sym(rng, n, 0.05)
    r = o.canonical_response(h0, [h1], [h2], beta, Ne, M, order=2)
    om2 = r["omega2"][0]
    om3 = r["omega3"][0]
    f = lambda lam: o.omega(h0 + lam * h1 + lam * lam * h2, beta, Ne, M)
    h = 2e-3
    f0, fp, fm, fp2, fm2 = f(0), f(h), f(-h), f(2 * h), f(-2 * h)
    c2 = (-fp2 + 16 * fp - 30 * f0 + 16 * fm - fm2) / (12 * h * h) / 2.0
    c3 = (fp2 - 2 * fp + 2 * fm - fm2) / (2 * h ** 3) / 6.0
    assert abs(c2 - om2) < 1e-6 * max(1.0, abs(om2))
    assert abs(c3 - om3) < 1e-3 * max(1.0, abs(om3))
    # first order: Omega^(1) = Tr[H1 P0]
    c1 = (fp - fm) / (2 * h)
    assert abs(c1 - float(np.sum(h1 * r["P0"]))) < 1e-5


def test_n_plus_one_rule_third_and_fourth_order():
    """Eq. (Resp_0) at m = 3 and 4 with H = H0 + l H1 + l^2 H2 + l^3 H3: the oracle's Omega^(3) and
    Omega^(4) from Tr[H^(k) P^(m-k)] equal the l^3 and l^4 coefficients of the canonical free energy
    (seven-point differences), while dropping the weights k of the sum misses them."""
    n, beta, Ne, M = 16, 5.0, 7.0, 40
    rng = np.random.default_rng(9)
    h0 = w.chain_1d(n, 2)
    h1 = np.diag(np.linspace(-1, 1, n))
    h2 = _sym(rng, n, 0.05)
    h3 = _sym(rng, n, 0.03)
    r = o.canonical_response(h0, [h1], [h2], beta, Ne, M, order=3, h3s=[h3])
    f = lambda lam: o.omega(h0 + lam * h1 + lam ** 2 * h2 + lam ** 3 * h3, beta, Ne, M)
    h = 0.02
    F = {k: f(k * h) for k in range(-3, 4)}
    c3 = (-F[3] + 8 * F[2] - 13 * F[1] + 13 * F[-1] - 8 * F[-2] + F[-3]) / (8 * h ** 3) / 6.0
    c4 = (-F[3] + 12 * F[2] - 39 * F[1] + 56 * F[0] - 39 * F[-1] + 12 * F[-2] - F[-3]) / (6 * h ** 4) / 24.0
    assert abs(c3 - r["omega3"][0]) < 1e-4 * abs(c3)
    assert abs(c4 - r["omega4"][0]) < 1e-2 * abs(c4)
    unweighted = (r["tr_h1p3"][0] + r["tr_h2p2"][0] + r["tr_h3p1"][0]) / 4.0
    assert abs(c4 - unweighted) > 0.1 * abs(c4)
    # the traces are those of the returned matrices
    assert abs(r["tr_h2p1"][0] - float(np.sum(h2 * r["P1"][0]))) < 1e-12 * max(1.0, abs(r["tr_h2p1"][0]))
    assert abs(r["tr_h3p0"][0] - float(np.sum(h3 * r["P0"]))) < 1e-12
    assert abs(r["omega1"][0] - float(np.sum(h1 * r["P0"]))) < 1e-12


def test_entropy_derivative_identity():
    """Eq. (EntDer): dS/dlambda = k_B beta Tr[H P^(1)] for a canonical perturbation (Fermi-Dirac limit)."""
    n, beta, Ne, M = 16, 5.0, 7.0, 40
    rng = np.random.default_rng(8)
    h0 = _sym(rng, n)
    h1 = _sym(rng, n, 0.2)
    r = o.canonical_response(h0, [h1], None, beta, Ne, M, order=1)

    def S(lam):
        wv = o.eig(h0 + lam * h1)
        mu = o.mu_canonical(wv[0], beta, M, Ne)
        return o.entropy(o.phi(wv[0] - mu, beta, M))

    h = 1e-4
    dS = (S(h) - S(-h)) / (2 * h)
    assert abs(dS - beta * float(np.sum(h0 * r["P1"][0]))) < 1e-6


# ---------------------------------------------------------------- planted mistakes

def test_planted_mistakes_are_caught(monkeypatch):
    """A wrong sign in the canonical mu1 shift, or a dropped second-order term, fails a pin."""
    n, M, beta, Ne = 12, 10, 5.0, 5.0
    h0 = w.chain_1d(n, 3)
    h1 = np.diag(np.arange(n) - n / 2.0) / n
    P, mu, _ = sr.canonical([h0, h1, np.zeros((n, n))], beta, Ne, M, 2)
    good = o.canonical_response(h0, [h1], None, beta, Ne, M, order=2)
    assert np.max(np.abs(good["P2"][0] - P[2])) < 1e-10
    orig = o.dmpt_oracle._second_order_kernel
    monkeypatch.setattr(o.dmpt_oracle, "_second_order_kernel", lambda *a: 0.0 * orig(*a))
    bad = o.canonical_response(h0, [h1], None, beta, Ne, M, order=2)
    assert np.max(np.abs(bad["P2"][0] - P[2])) > 1e-3
    monkeypatch.setattr(o.dmpt_oracle, "_second_order_kernel", orig)
    orig_dd1 = o.dmpt_oracle.dd1
    monkeypatch.setattr(o.dmpt_oracle, "dd1", lambda a, b, be, m: orig_dd1(b, a, be, m) * 1.01)
    bad = o.canonical_response(h0, [h1], None, beta, Ne, M, order=1)
    assert np.max(np.abs(bad["P1"][0] - P[1])) > 1e-4


# ---------------------------------------------------------------- third order

def test_third_and_fifth_derivatives_vs_finite_differences():
    """phi''' and phi^(5) of phi_derivs5 against differences of the analytic lower derivatives."""
    beta, M = 20.0, 12
    e = np.linspace(-1.0, 1.0, 41)
    p1, p2, p3, p4, p5 = o.phi_derivs5(e, beta, M)
    h = 1e-4
    g2 = lambda x: o.phi_derivs5(x, beta, M)[1]
    g4 = lambda x: o.phi_derivs5(x, beta, M)[3]
    d3 = (g2(e - 2 * h) - 8 * g2(e - h) + 8 * g2(e + h) - g2(e + 2 * h)) / (12 * h)
    d5 = (g4(e - 2 * h) - 8 * g4(e - h) + 8 * g4(e + h) - g4(e + 2 * h)) / (12 * h)
    assert np.max(np.abs(d3 - p3)) < 1e-6 * beta ** 3
    assert np.max(np.abs(d5 - p5)) < 1e-4 * beta ** 5
    # the two functions agree on what they share
    q1, q2, q4 = o.phi_derivs(e, beta, M)
    assert np.array_equal(q1, p1) and np.array_equal(q2, p2) and np.array_equal(q4, p4)


def _dd_mp(pts, beta, M):
    """Divided difference of phi by the plain recursive quotient rule at 150 digits.

    Repeated points are separated by multiples of 1e-35 (the confluent limit
    is reached to about 1e-35; each quotient level loses at most ~35 digits).
    """
    import mpmath as mp
    mp.mp.dps = 150
    s = mp.ldexp(mp.mpf(beta), -(M + 1))
    K = mp.mpf(2) ** M
    f = lambda x: mp.mpf(1) / 2 - mp.tanh(K * mp.atanh(s * x)) / 2
    xs = [mp.mpf(float(p)) + (j + 1) * mp.mpf(10) ** -35 for j, p in enumerate(pts)]

    def rec(lo, hi):
        if lo == hi:
            return f(xs[lo])
        return (rec(lo, hi - 1) - rec(lo + 1, hi)) / (xs[lo] - xs[hi])
    return float(rec(0, len(xs) - 1))


def test_third_divided_differences_vs_high_precision():
    """dd3 against the plain quotient rule in 150-digit arithmetic; coincident points give phi'''/6."""
    beta, M = 20.0, 16
    rng = np.random.default_rng(9)
    for _ in range(40):
        pts = rng.uniform(-0.4, 0.4, 4)
        if rng.random() < 0.3:
            pts[1] = pts[0] + 3e-6                      # a nearly coincident pair
        ref = _dd_mp(pts, beta, M)
        got = float(o.dd3(*pts, beta, M, 1e-5))
        assert abs(got - ref) < 1e-8 * max(1.0, abs(ref)), (pts, got, ref)
    a = np.linspace(-0.3, 0.3, 7)
    _, _, p3, _, _ = o.phi_derivs5(a, beta, M)
    assert np.max(np.abs(o.dd3(a, a, a, a, beta, M, 1e-5) - p3 / 6.0)) < 1e-12 * beta ** 3
    # a tight cluster (expansion path) agrees with the high-precision quotient rule
    for c in (-0.2, 0.05, 0.3):
        pts = np.array([c, c + 2e-6, c - 1e-6, c + 4e-6])
        ref = _dd_mp(pts, beta, M)
        assert abs(float(o.dd3(*pts, beta, M, 1e-5)) - ref) < 1e-9 * max(1.0, abs(ref))


def test_third_order_kernels_bruteforce():
    """T2(X, Y) and T3(X, X, X) against plain loops over 150-digit divided differences."""
    n, M, beta = 6, 12, 5.0
    rng = np.random.default_rng(21)
    e = np.sort(rng.uniform(-1, 1, n))
    e[3] = e[2] + 2e-7              # a near-degenerate pair takes the direct path
    X = _sym(rng, n)
    Y = _sym(rng, n)
    F1 = o.dd1(e[:, None], e[None, :], beta, M)
    T2 = o.dmpt_oracle._t2(e, F1, X, Y, beta, M, 1e-5, 1e-3)
    Q = o.dmpt_oracle._t2(e, F1, X, X, beta, M, 1e-5, 1e-3)
    T3 = o.dmpt_oracle._t3(e, F1, X, Q, beta, M, 1e-5, 1e-3)
    ref2 = np.zeros((n, n))
    ref3 = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            ref2[i, j] = sum(_dd_mp([e[i], e[k], e[j]], beta, M) * X[i, k] * Y[k, j] for k in range(n))
            ref3[i, j] = sum(_dd_mp([e[i], e[k], e[l], e[j]], beta, M) * X[i, k] * X[k, l] * X[l, j]
                             for k in range(n) for l in range(n))
    assert np.max(np.abs(T2 - ref2)) < 1e-9 * np.max(np.abs(ref2))
    assert np.max(np.abs(T3 - ref3)) < 1e-8 * np.max(np.abs(ref3))


def test_third_order_agrees_with_series_recursion():
    """Fixed-mu pass and canonical fixed point at third order against the series recursion."""
    n, M, beta = 10, 8, 5.0
    rng = np.random.default_rng(12)
    h0 = _sym(rng, n)
    h1 = _sym(rng, n, 0.3)
    h2 = _sym(rng, n, 0.2)
    h3 = _sym(rng, n, 0.1)
    mu = [0.1, 0.25, -0.4, 0.3]
    X = sr.recursion([h0, h1, h2, h3], beta, M, mu, 3)
    r = o.response(h0, [h1], [h2], beta, M, (mu[0], [mu[1]], [mu[2]], [mu[3]]), order=3, h3s=[h3])
    assert np.max(np.abs(X[3] - r["P3"][0])) < 1e-11 * max(1.0, np.max(np.abs(X[3])))
    # canonical
    n, M, beta, Ne = 14, 10, 8.0, 6.0
    h0 = w.chain_1d(n, M)
    h1 = np.diag(np.arange(n) - n / 2.0)
    h2 = _sym(rng, n, 0.05)
    h3 = _sym(rng, n, 0.03)
    # the third-order traces are O(100) here: their rounding floor is ~1e-11
    P, muj, _ = sr.canonical([h0, h1, h2, h3], beta, Ne, M, 3, tol=1e-10)
    rc = o.canonical_response(h0, [h1], [h2], beta, Ne, M, order=3, h3s=[h3])
    tol = 1e-15 * 2 ** M * 10
    assert np.max(np.abs(P[3] - rc["P3"][0])) < tol * np.max(np.abs(rc["P3"][0])) * 100
    assert abs(muj[3] - rc["mu3"][0]) < tol * 1000 * max(1.0, abs(rc["mu3"][0]))
    assert abs(np.trace(rc["P3"][0])) < 1e-10 * np.max(np.abs(rc["P3"][0]))


def test_canonical_third_order_finite_differences():
    """P3 = (1/6) d^3 P / dlambda^3 with mu(lambda) re-solved, H = H0 + l H1 + l^2 H2 + l^3 H3."""
    n, M, beta, Ne = 20, 16, 8.0, 9.0
    rng = np.random.default_rng(6)
    h0 = w.chain_1d(n, 6)
    h1 = np.diag(np.arange(n) - n / 2.0) / n
    h2 = _sym(rng, n, 0.05)
    h3 = _sym(rng, n, 0.05)
    r = o.canonical_response(h0, [h1], [h2], beta, Ne, M, order=3, h3s=[h3])

    def p_of(lam):
        h = h0 + lam * h1 + lam ** 2 * h2 + lam ** 3 * h3
        wv = o.eig(h)
        mu = o.mu_canonical(wv[0], beta, M, Ne)
        return o.density(h, beta, M, mu, eigh=wv), mu

    def d3(h):
        vals = [p_of(k * h) for k in (-2, -1, 1, 2)]
        P = (vals[3][0] - 2 * vals[2][0] + 2 * vals[1][0] - vals[0][0]) / (2 * h ** 3)
        m = (vals[3][1] - 2 * vals[2][1] + 2 * vals[1][1] - vals[0][1]) / (2 * h ** 3)
        return P / 6.0, m / 6.0

    h = 2e-2
    a1, b1 = d3(h)
    a2, b2 = d3(2 * h)
    P3_fd = (4 * a1 - a2) / 3
    mu3_fd = (4 * b1 - b2) / 3
    s3 = np.max(np.abs(r["P3"][0]))
    assert np.max(np.abs(P3_fd - r["P3"][0])) < 2e-5 * s3
    assert abs(mu3_fd - r["mu3"][0]) < 2e-5 * max(abs(r["mu3"][0]), s3)


def test_third_order_identity_perturbations():
    """H3 = I gives mu3 = 1 and P3 = 0; H1 = I gives P3 = 0 (a pure shift of mu)."""
    c = w.config("chain128")
    n = c["N"]
    z = np.zeros((n, n))
    r = o.canonical_response(c["H0"], [z], [z], c["beta"], c["Ne"], c["n"], order=3, h3s=[np.eye(n)])
    assert abs(r["mu3"][0] - 1.0) < 1e-13
    assert np.max(np.abs(r["P3"][0])) < 1e-12
    r = o.canonical_response(c["H0"][:48, :48], [np.eye(48)], None, c["beta"], 24.0, c["n"], order=3)
    assert np.max(np.abs(r["P3"][0])) < 1e-9 * max(1.0, np.max(np.abs(r["P2"][0])) + 1)
    assert abs(r["mu1"][0] - 1.0) < 1e-13


def test_planted_third_order_mistakes_are_caught(monkeypatch):
    """A dropped T3 term or a swapped T2 pair is caught by the series recursion pin."""
    n, M, beta = 10, 8, 5.0
    rng = np.random.default_rng(12)
    h0 = _sym(rng, n)
    h1 = _sym(rng, n, 0.3)
    h2 = _sym(rng, n, 0.2)
    h3 = _sym(rng, n, 0.1)
    mu = [0.1, 0.25, -0.4, 0.3]
    X = sr.recursion([h0, h1, h2, h3], beta, M, mu, 3)
    args = (h0, [h1], [h2], beta, M, (mu[0], [mu[1]], [mu[2]], [mu[3]]))
    orig3 = o.dmpt_oracle._t3
    monkeypatch.setattr(o.dmpt_oracle, "_t3", lambda *a: 0.0 * orig3(*a))
    bad = o.response(*args, order=3, h3s=[h3])
    assert np.max(np.abs(bad["P3"][0] - X[3])) > 1e-4 * np.max(np.abs(X[3]))
    monkeypatch.setattr(o.dmpt_oracle, "_t3", orig3)
    orig2 = o.dmpt_oracle._t2
    monkeypatch.setattr(o.dmpt_oracle, "_t2", lambda e, F1, Xm, Ym, *a: orig2(e, F1, Xm, Xm, *a))
    bad = o.response(*args, order=3, h3s=[h3])
    assert np.max(np.abs(bad["P3"][0] - X[3])) > 1e-4 * np.max(np.abs(X[3]))


# ---------------------------------------------------------------- non-orthogonal basis

def test_nonorthogonal_basis_matches_generalized_eigenproblem():
    """D = Z P(Z^T F Z) Z^T equals C phi(eps - mu) C^T from F C = S C eps (LAPACK sygvd),
    is the same for two different inverse factors (Cholesky and Loewdin), and 2 Tr(D S) / 2 = Ne."""
    import scipy.linalg as sl
    n, M, beta, Ne = 40, 18, 9.0, 17.0
    f0 = w.chain_1d(n, 8)
    S = w.overlap(n, 3)
    z1 = w.inverse_factor(S)
    ev, U = np.linalg.eigh(S)
    z2 = (U / np.sqrt(ev)) @ U.T                      # S^(-1/2), symmetric
    r1 = o.nonorthogonal_response(f0, [], None, z1, beta, Ne, M, order=0)
    r2 = o.nonorthogonal_response(f0, [], None, z2, beta, Ne, M, order=0)
    eps, C = sl.eigh(f0, S)
    mu = o.mu_canonical(eps, beta, M, Ne)
    D = (C * o.phi(eps - mu, beta, M)) @ C.T
    assert np.max(np.abs(r1["D0"] - D)) < 1e-12
    assert np.max(np.abs(r2["D0"] - D)) < 1e-12
    assert abs(np.trace(r1["D0"] @ S) - Ne) < 1e-11


def test_nonorthogonal_first_order_finite_difference():
    """D1 = dD/dlambda for F = F0 + lambda F1 in the non-orthogonal basis (generalized eigenproblem, FD)."""
    import scipy.linalg as sl
    n, M, beta, Ne = 30, 16, 7.0, 13.0
    f0 = w.chain_1d(n, 9)
    f1 = np.diag(np.arange(n) - n / 2.0) / n
    S = w.overlap(n, 4)
    z = w.inverse_factor(S)
    r = o.nonorthogonal_response(f0, [f1], None, z, beta, Ne, M, order=1)

    def d_of(lam):
        eps, C = sl.eigh(f0 + lam * f1, S)
        mu = o.mu_canonical(eps, beta, M, Ne)
        return (C * o.phi(eps - mu, beta, M)) @ C.T

    h = 1e-4
    fd = (d_of(h) - d_of(-h)) / (2 * h)
    assert np.max(np.abs(fd - r["D1"][0])) < 1e-7 * np.max(np.abs(r["D1"][0]))
    # the congruence with Z^T instead of Z (a plausible slip) is visibly wrong
    bad = o.nonorthogonal_response(f0, [f1], None, z.T, beta, Ne, M, order=1)
    assert np.max(np.abs(bad["D0"] - d_of(0.0))) > 1e-3


# ---------------------------------------------------------------- diagonal perturbations given as vectors

def test_diagonal_vector_perturbation_matches_full_matrix():
    """A diagonal H1 passed as its vector (the scaling branch of the basis rotation) gives the same
    P1, P2, mu jet and response traces as the same H1 passed as a full matrix, at every order, and the
    adjoint accepts a diagonal A as a vector; the full-matrix branch is pinned by every other test."""
    n, M, beta, Ne = 24, 14, 9.0, 11.0
    rng = np.random.default_rng(71)
    h0 = w.banded(n, 4, bandwidth=5, decay=3.0)
    x = np.linspace(-1.0, 1.0, n) + 0.1 * rng.standard_normal(n)
    h2 = _sym(rng, n, 0.05)
    h3 = _sym(rng, n, 0.03)
    rv = o.canonical_response(h0, [x], [h2], beta, Ne, M, order=3, h3s=[h3])
    rm = o.canonical_response(h0, [np.diag(x)], [h2], beta, Ne, M, order=3, h3s=[h3])
    for key in ("P1", "P2", "P3"):
        assert np.max(np.abs(rv[key][0] - rm[key][0])) < 1e-13 * np.max(np.abs(rm[key][0]))
    for key in ("mu1", "mu2", "mu3", "tr_h1p1", "tr_h1p2", "tr_h1p3"):
        assert abs(rv[key][0] - rm[key][0]) < 1e-12 * max(1.0, abs(rm[key][0])), key
    # second-order perturbation as a vector too
    rv2 = o.canonical_response(h0, [np.diag(x)], [x ** 2], beta, Ne, M, order=2)
    rm2 = o.canonical_response(h0, [np.diag(x)], [np.diag(x ** 2)], beta, Ne, M, order=2)
    assert np.max(np.abs(rv2["P2"][0] - rm2["P2"][0])) < 1e-13 * np.max(np.abs(rm2["P2"][0]))
    assert abs(rv2["tr_h2p0"][0] - rm2["tr_h2p0"][0]) < 1e-12 * abs(rm2["tr_h2p0"][0])
    # fixed mu jet (grand canonical pass)
    mu = (0.05, [0.2], [-0.1])
    pv = o.response(h0, [x], [x], beta, M, mu, order=2)
    pm = o.response(h0, [np.diag(x)], [np.diag(x)], beta, M, mu, order=2)
    assert np.max(np.abs(pv["P2"][0] - pm["P2"][0])) < 1e-13 * np.max(np.abs(pm["P2"][0]))
    # the adjoint with A = diag(x) as a vector
    gv = o.adjoint_grad(h0, beta, Ne, M, x)
    gm = o.adjoint_grad(h0, beta, Ne, M, np.diag(x))
    assert np.max(np.abs(gv - gm)) < 1e-13 * np.max(np.abs(gm))


def test_diagonal_vector_against_series_recursion():
    """The vector form of a diagonal H1 against the power-series recursion, which never sees vectors."""
    n, M, beta, Ne = 12, 10, 5.0, 5.0
    h0 = w.chain_1d(n, 5)
    x = (np.arange(n) - n / 2.0) / n
    P, mu, _ = sr.canonical([h0, np.diag(x), np.zeros((n, n))], beta, Ne, M, 2)
    r = o.canonical_response(h0, [x], None, beta, Ne, M, order=2)
    assert np.max(np.abs(r["P1"][0] - P[1])) < 1e-10 * np.max(np.abs(P[1]))
    assert np.max(np.abs(r["P2"][0] - P[2])) < 1e-10 * np.max(np.abs(P[2]))
    assert abs(r["tr_h1p1"][0] - float(np.sum(x * np.diag(P[1])))) < 1e-10 * abs(r["tr_h1p1"][0])


def test_planted_row_column_slip_in_diagonal_branch_is_caught(monkeypatch):
    """Scaling the columns of V by h (h[None, :] * V, which gives V^T V diag(h) = diag(h)) instead of
    its rows (diag(h) V, giving V^T diag(h) V) changes P1 and Tr(H1 P1) far beyond rounding."""
    n, M, beta, Ne = 16, 12, 6.0, 7.0
    h0 = w.chain_1d(n, 9)
    x = np.linspace(-2.0, 2.0, n)
    good = o.canonical_response(h0, [np.diag(x)], None, beta, Ne, M, order=2)
    orig = o.dmpt_oracle._rot

    def slipped(v, h):
        if h is not None and h.ndim == 1:
            return v.T @ (h[None, :] * v)
        return orig(v, h)

    monkeypatch.setattr(o.dmpt_oracle, "_rot", slipped)
    bad = o.canonical_response(h0, [x], None, beta, Ne, M, order=2)
    assert np.max(np.abs(bad["P1"][0] - good["P1"][0])) > 1e-3 * np.max(np.abs(good["P1"][0]))
    assert abs(bad["tr_h1p1"][0] - good["tr_h1p1"][0]) > 1e-3 * abs(good["tr_h1p1"][0])


# ---------------------------------------------------------------- range of the recursion (Appendix A)

@pytest.mark.parametrize("M,beta", [(4, 3.0), (10, 40.0), (20, 7.0), (30, 40.0)])
def test_range_ok_is_appendix_a_interval(M, beta):
    """range_ok(e) holds exactly when the start x = 1/2 - beta e / (4 n), n = 2^M, of Appendix A's
    Pade form lies in the open interval (0, 1).  At the edge x = 0 the recursion is stuck at 0 and
    beyond it the occupation computed by the scalar X-form recursion rises again with the energy:
    the monotone Fermi-like map is lost exactly where range_ok turns false."""
    n = 2.0 ** M
    edge = 2.0 * n / beta                      # x = 0 at e = +edge, x = 1 at e = -edge
    inside = [0.0, 0.5 * edge, edge * (1 - 1e-9), -edge * (1 - 1e-9)]
    outside = [edge * (1 + 1e-9), -edge * (1 + 1e-9), 3.0 * edge, -7.0 * edge]
    for e in inside:
        x = 0.5 - beta * e / (4.0 * n)
        assert 0.0 < x < 1.0
        assert o.range_ok(np.array([e]), beta, M)
    for e in outside:
        x = 0.5 - beta * e / (4.0 * n)
        assert not (0.0 < x < 1.0)
        assert not o.range_ok(np.array([e]), beta, M)
    # a spectrum is in range only when every eigenvalue is
    assert not o.range_ok(np.array(inside + outside[:1]), beta, M)
    assert o.range_ok(np.array(inside), beta, M)
    # the closed forms refuse exactly the out-of-range energies
    with pytest.raises(ValueError):
        o.phi(np.array([outside[0]]), beta, M)
    with pytest.raises(ValueError):
        o.phi_pade(np.array([outside[1]]), beta, M)


def test_range_edge_breaks_monotone_occupation():
    """Scalar X-form recursion of Eq. (Rec_F_2) across the range edge: decreasing in e inside,
    stuck at 0 on the edge, increasing in e beyond it."""
    M, beta = 3, 2.0
    n = 2.0 ** M
    edge = 2.0 * n / beta

    def occ(e):
        x = 0.5 - beta * e / (4.0 * n)
        for _ in range(M):
            x = x * x / (x * x + (1.0 - x) ** 2)
        return x

    es = np.linspace(0.9 * edge, 0.999 * edge, 20)
    vals = [occ(e) for e in es]
    assert all(a > b for a, b in zip(vals, vals[1:]))
    assert occ(edge) == 0.0
    beyond = [occ(e) for e in np.linspace(1.01 * edge, 1.5 * edge, 20)]
    assert all(b > a for a, b in zip(beyond, beyond[1:]))
    assert all(o.range_ok(np.array([e]), beta, M) for e in es)
    assert not any(o.range_ok(np.array([e]), beta, M) for e in np.linspace(1.01 * edge, 1.5 * edge, 20))
