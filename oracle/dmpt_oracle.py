"""Plain FP64 CPU oracle for canonical density-matrix perturbation theory.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import or call
this module: only the tests, the smoke check and the CPU-baseline leg of the
benchmark use it.  It shares no code with the GPU library.

What it computes (Niklasson, Rubensson, Rudberg, Cawkwell, "Canonical density
matrix perturbation theory"):

* Sec. II, Eq. (Rec_F_2): the recursive Fermi-operator expansion
  X0 = I/2 - 2^-(M+2) beta (H - mu I),  X_n = X^2 / (X^2 + (I - X)^2).
  Every step is a rational function of the previous iterate, so X_M is an
  exact matrix function of H: on an eigenvalue e = eps - mu it equals the
  Pade function f_{2^M}(x) = x^n / (x^n + (1-x)^n) at x = 1/2 - beta e / (4n),
  n = 2^M (Appendix A, recursive Fermi operator expansion).  Writing
  x = 1/2 - d, the one-step map d -> 2d / (1 + 4 d^2) is tanh doubling, so
  phi_M(e) = 1/2 - tanh(2^M artanh(s e)) / 2  with  s = 2^-(M+1) beta.
  ``phi`` evaluates this closed form; ``phi_pade`` evaluates the Pade power
  form of Appendix A in log space, an independent second closed form.
* Sec. II, Eqs. (P_resp), (H_prt) and the mu expansion: P(lambda) is the same
  matrix function of K(lambda) = H(lambda) - mu(lambda) I, so P^(1), P^(2)
  and P^(3) are the Taylor coefficients of that matrix function, written in
  the eigenbasis of H0 with divided differences of phi (Daleckii-Krein):
  with E_k = V^T H^(k) V - mu^(k) I,
    P^(1) = phi[1] o E_1,
    P^(2) = phi[1] o E_2 + T2(E_1, E_1),
    P^(3) = phi[1] o E_3 + T2(E_1, E_2) + T2(E_2, E_1) + T3(E_1, E_1, E_1),
  T2(X, Y)_ij = sum_k phi[e_i, e_k, e_j] X_ik Y_kj and
  T3(X, Y, Z)_ij = sum_kl phi[e_i, e_k, e_l, e_j] X_ik Y_kl Z_lj.  The
  canonical mu^(k) are fixed by Tr P^(k) = 0 (Tr P^(0) = Ne).  Algorithm 1
  (written there up to third order) converges to exactly this fixed point;
  the oracle computes the fixed point directly.
* Sec. III, Eq. (Resp_0): free-energy response traces Tr[H^(k) P^(m-k)].
* The adjoint d Tr(A P0)/d H0 of the canonical map, which by the symmetry of
  the first-order kernel equals the canonical first-order response to sym(A).

All arithmetic is FP64 (numpy / LAPACK).  Eigenvalue-space divided
differences are evaluated in forms that avoid cancellation (see ``dd1`` and
``dd2``); near-coincident eigenvalues use short Taylor expansions.
"""
import math
import numpy as np

__all__ = [
    "phi", "phi_pade", "phi_derivs", "phi_derivs5", "fermi_dirac", "dd1", "dd2", "dd3",
    "mu_canonical", "eig", "density", "response", "canonical_response",
    "adjoint_grad", "entropy", "omega", "range_ok", "nonorthogonal_response",
]


# ----------------------------------------------------------------------------
# scalar functions of an eigenvalue e = eps - mu
# ----------------------------------------------------------------------------

def _s(beta, M):
    """Scale s = 2^-(M+1) beta of the closed form; also returns K = 2^M."""
    return math.ldexp(beta, -(M + 1)), math.ldexp(1.0, M)


def range_ok(e, beta, M):
    """True when every |s e| < 1, i.e. x = 1/2 - beta e/2^(M+2) lies in (0, 1)."""
    s, _ = _s(beta, M)
    return bool(np.all(np.abs(s * np.asarray(e)) < 1.0))


def _u(e, beta, M):
    s, K = _s(beta, M)
    z = s * np.asarray(e, dtype=np.float64)
    if np.any(np.abs(z) >= 1.0):
        raise ValueError("spectrum outside the recursion's range: need 2^(M+1) > beta*|eps-mu|")
    return K * np.arctanh(z)


def phi(e, beta, M):
    """Occupation computed by M recursion steps: 1/2 - tanh(2^M artanh(s e))/2."""
    return 0.5 - 0.5 * np.tanh(_u(e, beta, M))


def phi_pade(e, beta, M):
    """Appendix A's Pade form f_n(x) = x^n/(x^n+(1-x)^n), n = 2^M, x = 1/2 - beta e/(4n).

    Evaluated as 1/(1 + exp(n (log(1-x) - log x))) so n = 2^30 does not
    overflow; valid for x in (0, 1).
    """
    n = math.ldexp(1.0, M)
    e = np.asarray(e, dtype=np.float64)
    x = 0.5 - beta * e / (4.0 * n)
    if np.any((x <= 0) | (x >= 1)):
        raise ValueError("x outside (0, 1)")
    # log(1-x) - log(x) = log1p(-2x + 1 ...) computed as log((1-x)/x) with the
    # small quantity y = beta e/(4n):  (1/2 + y)/(1/2 - y)
    y = beta * e / (4.0 * n)
    t = n * (np.log1p(2.0 * y) - np.log1p(-2.0 * y))
    return 0.5 * (1.0 - np.tanh(0.5 * t))


def fermi_dirac(e, beta):
    """Fermi-Dirac occupation 1/(1 + exp(beta e)), the M -> infinity limit (Eq. Rec_F_1)."""
    return 0.5 * (1.0 - np.tanh(0.5 * beta * np.asarray(e, dtype=np.float64)))


def phi_derivs5(e, beta, M):
    """Analytic derivatives phi', ..., phi^(5) of the closed form at e.

    phi = h(u(e)) with h(u) = 1/2 - tanh(u)/2 and u = 2^M artanh(s e);
    chain rule (Faa di Bruno, Bell polynomials) with t = tanh u, c = 1 - t^2:
      h1 = -c/2, h2 = t c, h3 = c (1 - 3t^2), h4 = -4 t c (2 - 3t^2),
      h5 = -4 c (2 - 15 t^2 + 15 t^4)   (hk the k-th derivative of h);
      w = artanh(z), z = s e, q = 1 - z^2:  w1 = 1/q, w2 = 2z/q^2,
      w3 = 2 (1 + 3z^2)/q^3, w4 = 24 z (1 + z^2)/q^4,
      w5 = 24 (1 + 10 z^2 + 5 z^4)/q^5, and the k-th derivative of u is
      2^M s^k wk.
    """
    s, K = _s(beta, M)
    e = np.asarray(e, dtype=np.float64)
    z = s * e
    q = 1.0 - z * z
    t = np.tanh(_u(e, beta, M))
    c = 1.0 - t * t
    t2 = t * t
    h1 = -0.5 * c
    h2 = t * c
    h3 = c * (1.0 - 3.0 * t2)
    h4 = -4.0 * t * c * (2.0 - 3.0 * t2)
    h5 = -4.0 * c * (2.0 - 15.0 * t2 + 15.0 * t2 * t2)
    u1 = K * s / q
    u2 = K * 2.0 * s * s * z / q**2
    u3 = K * 2.0 * s**3 * (1.0 + 3.0 * z * z) / q**3
    u4 = K * 24.0 * s**4 * z * (1.0 + z * z) / q**4
    u5 = K * 24.0 * s**5 * (1.0 + 10.0 * z * z + 5.0 * z**4) / q**5
    p1 = h1 * u1
    p2 = h2 * u1**2 + h1 * u2
    p3 = h3 * u1**3 + 3.0 * h2 * u1 * u2 + h1 * u3
    p4 = h4 * u1**4 + 6.0 * h3 * u1**2 * u2 + h2 * (3.0 * u2**2 + 4.0 * u1 * u3) + h1 * u4
    p5 = (h5 * u1**5 + 10.0 * h4 * u1**3 * u2 + h3 * (15.0 * u1 * u2**2 + 10.0 * u1**2 * u3)
          + h2 * (10.0 * u2 * u3 + 5.0 * u1 * u4) + h1 * u5)
    return p1, p2, p3, p4, p5


def phi_derivs(e, beta, M):
    """The first, second and fourth derivatives of phi at e (see ``phi_derivs5``)."""
    p1, p2, _, p4, _ = phi_derivs5(e, beta, M)
    return p1, p2, p4


def _sinhc(x):
    """sinh(x)/x, accurate near 0."""
    x = np.asarray(x, dtype=np.float64)
    out = np.ones_like(x)
    big = np.abs(x) > 1e-4
    out[big] = np.sinh(x[big]) / x[big]
    sm = ~big
    out[sm] = 1.0 + x[sm] ** 2 / 6.0
    return out


def _artanhc(z):
    """artanh(z)/z, accurate near 0."""
    z = np.asarray(z, dtype=np.float64)
    out = np.ones_like(z)
    big = np.abs(z) > 1e-4
    out[big] = np.arctanh(z[big]) / z[big]
    sm = ~big
    out[sm] = 1.0 + z[sm] ** 2 / 3.0
    return out


def dd1(a, b, beta, M):
    """First divided difference phi[a, b] (= phi'(a) when a == b), broadcasting.

    phi(a) - phi(b) = -(tanh u_a - tanh u_b)/2 with
    tanh u_a - tanh u_b = sinh(du)/(cosh u_a cosh u_b) and
    du = 2^M artanh(s(a-b)/(1 - s^2 ab)); the factor (a - b) is divided out
    analytically through sinh(du)/du and artanh(z)/z, so there is no
    cancellation for a close to b.  The cosh product is formed in log space.
    """
    s, K = _s(beta, M)
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    a, b = np.broadcast_arrays(a, b)
    ua = _u(a, beta, M)
    ub = _u(b, beta, M)
    den = 1.0 - s * s * a * b
    z = s * (a - b) / den
    du = K * np.arctanh(z)
    r = K * s / den * _artanhc(z)          # du / (a - b)
    # 1/(cosh ua cosh ub) = 4 exp(-|ua|-|ub|) / ((1+exp(-2|ua|))(1+exp(-2|ub|)))
    aa, ab = np.abs(ua), np.abs(ub)
    inv_cc = 4.0 / ((1.0 + np.exp(-2.0 * aa)) * (1.0 + np.exp(-2.0 * ab)))
    # sinh(du) exp(-|ua|-|ub|) without overflow: |du| <= |ua| + |ub|
    lg = -(aa + ab)
    small = np.abs(du) < 1.0
    sh = np.empty_like(du)
    # small |du|: sinh(du)/(a-b) = sinhc(du) * r, times exp(lg)
    sh[small] = (_sinhc(du[small]) * r[small]) * np.exp(lg[small])
    big = ~small
    if np.any(big):
        d = du[big]
        val = 0.5 * (np.exp(d + lg[big]) - np.exp(-d + lg[big]))
        sh[big] = val / (a[big] - b[big])
    return -0.5 * sh * inv_cc


def dd2(x, y, z, beta, M, delta):
    """Second divided difference phi[x, y, z] (symmetric in its arguments), broadcasting.

    If the largest pairwise gap |p - q| is at least ``delta`` the recurrence
    phi[p, r, q] = (phi[p, r] - phi[r, q]) / (p - q) is used with that pair,
    so the division is by the largest gap.  Otherwise all three points lie in
    a cluster of width < delta and the expansion about their mean m,
    phi''(m)/2 + phi''''(m) * sum((x_i - m)^2) / 48, is used (the linear term
    vanishes at the mean; the first neglected term is O(delta^3 phi^(5))).
    """
    x, y, z = np.broadcast_arrays(*(np.asarray(v, dtype=np.float64) for v in (x, y, z)))
    gxy, gyz, gxz = np.abs(x - y), np.abs(y - z), np.abs(x - z)
    # pick the pair with the largest gap: (p, q) and the third point r
    use_xz = (gxz >= gxy) & (gxz >= gyz)
    use_xy = ~use_xz & (gxy >= gyz)
    p = np.where(use_xz, x, np.where(use_xy, x, y))
    q = np.where(use_xz, z, np.where(use_xy, y, z))
    r = np.where(use_xz, y, np.where(use_xy, z, x))
    gap = np.abs(p - q)
    out = np.empty(x.shape)
    far = gap >= delta
    if np.any(far):
        pf, qf, rf = p[far], q[far], r[far]
        out[far] = (dd1(pf, rf, beta, M) - dd1(rf, qf, beta, M)) / (pf - qf)
    near = ~far
    if np.any(near):
        m = (x[near] + y[near] + z[near]) / 3.0
        ss = (x[near] - m) ** 2 + (y[near] - m) ** 2 + (z[near] - m) ** 2
        _, p2, p4 = phi_derivs(m, beta, M)
        out[near] = 0.5 * p2 + p4 * ss / 48.0
    return out


def dd3(a, b, c, d, beta, M, delta):
    """Third divided difference phi[a, b, c, d] (symmetric in its arguments), broadcasting.

    As in ``dd2``: the pair (p, q) with the largest gap gives
    phi[p, r1, r2, q] = (phi[p, r1, r2] - phi[r1, r2, q]) / (p - q) when the gap
    is at least ``delta``; otherwise the four points lie in a cluster of width
    < delta and the expansion about their mean m,
    p3(m)/6 + p5(m) * sum((x_i - m)^2) / 240 (pk the k-th derivative of phi),
    is used; the term in the fourth derivative vanishes at the mean.
    """
    pts = np.broadcast_arrays(*(np.asarray(v, dtype=np.float64) for v in (a, b, c, d)))
    X = np.stack(pts, axis=0)                      # (4, ...)
    pairs = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]
    gaps = np.stack([np.abs(X[i] - X[j]) for i, j in pairs], axis=0)
    best = np.argmax(gaps, axis=0)
    gap = np.max(gaps, axis=0)
    out = np.empty(X.shape[1:])
    far = gap >= delta
    if np.any(far):
        for idx, (i, j) in enumerate(pairs):
            sel = far & (best == idx)
            if not np.any(sel):
                continue
            rest = [k for k in range(4) if k not in (i, j)]
            p, q = X[i][sel], X[j][sel]
            r1, r2 = X[rest[0]][sel], X[rest[1]][sel]
            out[sel] = (dd2(p, r1, r2, beta, M, delta) - dd2(r1, r2, q, beta, M, delta)) / (p - q)
    near = ~far
    if np.any(near):
        Xn = X[:, near]
        m = Xn.mean(axis=0)
        ss = np.sum((Xn - m) ** 2, axis=0)
        _, _, p3, _, p5 = phi_derivs5(m, beta, M)
        out[near] = p3 / 6.0 + p5 * ss / 240.0
    return out


# ----------------------------------------------------------------------------
# chemical potential and matrices
# ----------------------------------------------------------------------------

def mu_canonical(eps, beta, M, Ne):
    """Unique mu with sum_i phi_M(eps_i - mu) = Ne (Sec. II, canonical ensemble).

    The occupation sum is strictly increasing in mu, so bracketed bisection
    converges; it is finished with safeguarded Newton steps using the exact
    slope -sum phi'(eps_i - mu).
    """
    eps = np.asarray(eps, dtype=np.float64)
    n = eps.size
    if not (0.0 < Ne < n):
        raise ValueError("Ne must lie strictly between 0 and N")
    s, _ = _s(beta, M)
    lim = 1.0 / s  # |eps - mu| must stay below this
    lo = max(eps.max() - lim * (1 - 1e-12), eps.min() - 50.0 / beta - 1.0)
    hi = min(eps.min() + lim * (1 - 1e-12), eps.max() + 50.0 / beta + 1.0)

    def occ(mu):
        return float(np.sum(phi(eps - mu, beta, M)))

    if not (lo < hi and occ(lo) <= Ne <= occ(hi)):
        raise ValueError("cannot bracket the chemical potential")
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if mid == lo or mid == hi:
            break
        if occ(mid) < Ne:
            lo = mid
        else:
            hi = mid
    mu = 0.5 * (lo + hi)
    # one Newton step with the exact slope, kept only if it lowers the residual
    f = occ(mu) - Ne
    d1, _, _ = phi_derivs(eps - mu, beta, M)
    slope = -float(np.sum(d1))
    if slope > 0:
        cand = mu - f / slope
        if abs(occ(cand) - Ne) < abs(f):
            mu = cand
    return mu


def eig(h0):
    """Eigen-decomposition of sym(H0) with LAPACK dsyevd."""
    h = 0.5 * (h0 + h0.T)
    w, v = np.linalg.eigh(h)
    return w, v


def density(h0, beta, M, mu, eigh=None):
    """Grand-canonical P0 = phi_M(H0 - mu I) (Eq. Rec_F_2 after M steps)."""
    w, v = eigh if eigh is not None else eig(h0)
    f = phi(w - mu, beta, M)
    return (v * f) @ v.T


def _rot(v, h):
    """V^T sym(H) V; a diagonal H (given as a vector) is applied by scaling."""
    if h is None:
        return np.zeros((v.shape[1], v.shape[1]))
    if h.ndim == 1:
        return v.T @ (h[:, None] * v)
    hs = 0.5 * (h + h.T)
    return v.T @ hs @ v


def _second_order_kernel(e, F1, E, beta, M, delta):
    """Q_ij = sum_k phi[e_i, e_k, e_j] E_ik E_kj (second-order Daleckii-Krein term).

    Pairs with |e_i - e_j| >= delta use the identity
    phi[e_i, e_k, e_j] = (phi[e_i, e_k] - phi[e_k, e_j]) / (e_i - e_j), i.e.
    Q = ((F1 o E) E - E (F1 o E)) / (e_i - e_j); the remaining (nearly
    coincident) pairs, including the diagonal, are summed directly over k.
    """
    n = e.size
    G = F1 * E
    num = G @ E - E @ G
    de = e[:, None] - e[None, :]
    close = np.abs(de) < delta
    with np.errstate(divide="ignore", invalid="ignore"):
        Q = np.where(close, 0.0, num / np.where(close, 1.0, de))
    ii, jj = np.nonzero(close)
    # only the upper triangle (Q is symmetric), in chunks of pairs
    keep = ii <= jj
    ii, jj = ii[keep], jj[keep]
    chunk = max(1, (1 << 22) // max(n, 1))
    for c0 in range(0, ii.size, chunk):
        i = ii[c0:c0 + chunk]
        j = jj[c0:c0 + chunk]
        w2 = dd2(e[i][:, None], e[None, :], e[j][:, None], beta, M, delta)
        val = np.sum(w2 * E[i, :] * E[:, j].T, axis=1)
        Q[i, j] = val
        Q[j, i] = val
    return Q


def _t2(e, F1, X, Y, beta, M, delta, pair_delta):
    """T2(X, Y)_ij = sum_k phi[e_i, e_k, e_j] X_ik Y_kj for general X, Y.

    Separated pairs (|e_i - e_j| >= pair_delta) use
    phi[e_i, e_k, e_j] = (phi[e_i, e_k] - phi[e_k, e_j]) / (e_i - e_j):
    T2 = ((F1 o X) Y - X (F1 o Y)) / (e_i - e_j); the other pairs, the
    diagonal included, are summed directly over k (``dd2`` with its own
    cluster threshold delta).
    """
    n = e.size
    num = (F1 * X) @ Y - X @ (F1 * Y)
    de = e[:, None] - e[None, :]
    close = np.abs(de) < pair_delta
    with np.errstate(divide="ignore", invalid="ignore"):
        T = np.where(close, 0.0, num / np.where(close, 1.0, de))
    ii, jj = np.nonzero(close)
    chunk = max(1, (1 << 22) // max(n, 1))
    for c0 in range(0, ii.size, chunk):
        i = ii[c0:c0 + chunk]
        j = jj[c0:c0 + chunk]
        w2 = dd2(e[i][:, None], e[None, :], e[j][:, None], beta, M, delta)
        T[i, j] = np.sum(w2 * X[i, :] * Y[:, j].T, axis=1)
    return T


def _t3(e, F1, X, Q, beta, M, delta, pair_delta):
    """T3(X, X, X)_ij = sum_kl phi[e_i, e_k, e_l, e_j] X_ik X_kl X_lj, Q = T2(X, X).

    Separated pairs (|e_i - e_j| >= pair_delta) use phi[e_i, e_k, e_l, e_j] =
    (phi[e_i, e_k, e_l] - phi[e_k, e_l, e_j]) / (e_i - e_j), i.e.
    T3 = (Q X - X Q) / (e_i - e_j); the other pairs are summed directly over
    (k, l) with ``dd3``.
    """
    num = Q @ X - X @ Q
    de = e[:, None] - e[None, :]
    close = np.abs(de) < pair_delta
    with np.errstate(divide="ignore", invalid="ignore"):
        T = np.where(close, 0.0, num / np.where(close, 1.0, de))
    for i, j in zip(*np.nonzero(close)):
        w3 = dd3(e[i], e[:, None], e[None, :], e[j], beta, M, delta)
        T[i, j] = float(np.sum(w3 * X[i, :][:, None] * X * X[:, j][None, :]))
    return T


def _delta(e):
    width = float(e.max() - e.min()) if e.size > 1 else 1.0
    return 1e-5 * max(width, 1e-3)


def _pair_delta(e):
    """Eigenvalue gap below which the third-order kernels sum a pair (i, j) directly.

    The separated-pair identities divide by e_i - e_j twice over (T3 is
    built from T2), so a pair just above the scalar threshold of ``_delta``
    would lose about eps * width / gap^2; 1e-3 of the spectral width keeps
    that below ~1e-12 at a few direct sums per eigenvalue.
    """
    width = float(e.max() - e.min()) if e.size > 1 else 1.0
    return 1e-3 * max(width, 1e-3)


def response(h0, h1s, h2s, beta, M, mu, order=2, eigh=None, h3s=None):
    """P0, P1[d], P2[d], P3[d] at a fixed mu jet (grand canonical; one pass of Algorithm 1).

    mu = (mu0, [mu1_d], [mu2_d]) or (mu0, [mu1_d], [mu2_d], [mu3_d]).  H1s,
    H2s, H3s are lists of N x N matrices or length-N vectors (diagonal); an
    entry of H2s / H3s may be None (zero), and H2s / H3s may be None.
    Returns a dict with P0, P1, P2, P3 (lists) in the original basis.
    """
    w, v = eigh if eigh is not None else eig(h0)
    mu0 = mu[0]
    e = w - mu0
    F = phi(e, beta, M)
    P0 = (v * F) @ v.T
    out = dict(P0=P0, P1=[], P2=[], P3=[], eigh=(w, v))
    if order == 0:
        return out
    F1 = dd1(e[:, None], e[None, :], beta, M)
    delta = _delta(e)
    eye = np.eye(e.size)
    for d, h1 in enumerate(h1s):
        E1 = _rot(v, h1) - mu[1][d] * eye
        out["P1"].append(v @ (F1 * E1) @ v.T)
        if order >= 2:
            h2 = h2s[d] if h2s is not None else None
            E2 = _rot(v, h2) - mu[2][d] * eye
            Q = _second_order_kernel(e, F1, E1, beta, M, delta)
            out["P2"].append(v @ (Q + F1 * E2) @ v.T)
        if order >= 3:
            h3 = h3s[d] if h3s is not None else None
            E3 = _rot(v, h3) - mu[3][d] * eye
            pd = _pair_delta(e)
            R = (F1 * E3 + _t2(e, F1, E1, E2, beta, M, delta, pd)
                 + _t2(e, F1, E2, E1, beta, M, delta, pd) + _t3(e, F1, E1, Q, beta, M, delta, pd))
            out["P3"].append(v @ R @ v.T)
    return out


def canonical_response(h0, h1s, h2s, beta, Ne, M, order=2, eigh=None, h3s=None):
    """Canonical P0, P1, P2, P3 and the mu jet (the fixed point of Algorithm 1).

    mu0 solves Tr P0 = Ne; mu1 = sum_i phi'(e_i) E_ii / sum_i phi'(e_i) makes
    Tr P1 = 0; mu2 = (Tr Q + sum_i phi'(e_i) (V^T H2 V)_ii) / sum_i phi'(e_i)
    makes Tr P2 = 0; mu3 likewise with the third-order terms (each P^(k) is
    affine in mu^(k) with slope -phi'(K)).  Returns a dict with P0, P1, P2,
    P3, mu0, mu1, mu2, mu3, the response traces tr_hkpj[d] = Tr(H^(k) P^(j))
    for k >= 1, j <= order, k + j <= order + 1 (tr_h1p0, tr_h1p1, tr_h1p2,
    tr_h1p3, tr_h2p0, tr_h2p1, tr_h2p2, tr_h3p0, tr_h3p1 as far as the order
    reaches; an absent H2 or H3 counts as zero) and the free-energy responses
    omega1 .. omega(order + 1) of Sec. III, Eq. (Resp_0):
    Omega^(m) = (1/m) sum_{k=1..m} k Tr[H^(k) P^(m-k)], H^(k) = 0 beyond the order.
    """
    w, v = eigh if eigh is not None else eig(h0)
    n = w.size
    mu0 = mu_canonical(w, beta, M, Ne)
    e = w - mu0
    F = phi(e, beta, M)
    P0 = (v * F) @ v.T
    res = dict(P0=P0, P1=[], P2=[], P3=[], mu0=mu0, mu1=[], mu2=[], mu3=[], tr_h1p1=[],
               tr_h1p2=[], tr_h2p0=[], tr_h1p3=[], eigh=(w, v), occ=F)
    if order == 0:
        return res
    F1 = dd1(e[:, None], e[None, :], beta, M)
    fd = np.diag(F1).copy()
    sfd = float(np.sum(fd))
    delta = _delta(e)
    eye = np.eye(n)
    for d, h1 in enumerate(h1s):
        H1t = _rot(v, h1)
        mu1 = float(np.sum(fd * np.diag(H1t)) / sfd)
        E1 = H1t - mu1 * eye
        Pt1 = F1 * E1
        P1 = v @ Pt1 @ v.T
        res["P1"].append(P1)
        res["mu1"].append(mu1)
        h1m = np.diag(h1) if h1.ndim == 1 else h1
        res["tr_h1p1"].append(float(np.sum(0.5 * (h1m + h1m.T) * P1)))
        if order >= 2:
            h2 = h2s[d] if h2s is not None else None
            H2t = _rot(v, h2)
            Q = _second_order_kernel(e, F1, E1, beta, M, delta)
            mu2 = float((np.trace(Q) + np.sum(fd * np.diag(H2t))) / sfd)
            P2 = v @ (Q + F1 * (H2t - mu2 * eye)) @ v.T
            res["P2"].append(P2)
            res["mu2"].append(mu2)
            res["tr_h1p2"].append(float(np.sum(0.5 * (h1m + h1m.T) * P2)))
            if h2 is None:
                res["tr_h2p0"].append(0.0)
            else:
                h2m = np.diag(h2) if h2.ndim == 1 else h2
                res["tr_h2p0"].append(float(np.sum(0.5 * (h2m + h2m.T) * P0)))
        if order >= 3:
            E2 = H2t - mu2 * eye
            h3 = h3s[d] if h3s is not None else None
            H3t = _rot(v, h3)
            pd = _pair_delta(e)
            R = (_t2(e, F1, E1, E2, beta, M, delta, pd) + _t2(e, F1, E2, E1, beta, M, delta, pd)
                 + _t3(e, F1, E1, Q, beta, M, delta, pd))
            mu3 = float((np.trace(R) + np.sum(fd * np.diag(H3t))) / sfd)
            P3 = v @ (R + F1 * (H3t - mu3 * eye)) @ v.T
            res["P3"].append(P3)
            res["mu3"].append(mu3)
            res["tr_h1p3"].append(float(np.sum(0.5 * (h1m + h1m.T) * P3)))
    _response_traces(res, h1s, h2s, h3s, order)
    return res


def _response_traces(res, h1s, h2s, h3s, order):
    """Tr[H^(k) P^(j)] for k >= 1, k + j <= order + 1, and Omega^(m), m <= order + 1 (Eq. Resp_0)."""
    def full(h):
        if h is None:
            return None
        h = np.diag(h) if np.ndim(h) == 1 else np.asarray(h)
        return 0.5 * (h + h.T)

    for d in range(len(h1s)):
        H = {1: full(h1s[d]),
             2: full(h2s[d]) if (order >= 2 and h2s is not None) else None,
             3: full(h3s[d]) if (order >= 3 and h3s is not None) else None}
        P = {0: res["P0"]}
        for j in range(1, order + 1):
            P[j] = res["P%d" % j][d]
        tr = {}
        for k in range(1, order + 1):
            for j in range(0, order + 2 - k):
                if j > order:
                    continue
                tr[(k, j)] = 0.0 if H[k] is None else float(np.sum(H[k] * P[j]))
                key = "tr_h%dp%d" % (k, j)
                if key in ("tr_h1p1", "tr_h1p2", "tr_h2p0", "tr_h1p3"):
                    continue  # already filled above
                res.setdefault(key, []).append(tr[(k, j)])
        for m in range(1, order + 2):
            om = sum(k * tr.get((k, m - k), 0.0) for k in range(1, m + 1) if k <= order) / m
            res.setdefault("omega%d" % m, []).append(om)


def adjoint_grad(h0, beta, Ne, M, A, eigh=None):
    """G = d Tr(A P0)/d H0 for the canonical map (mu0 follows H0 through Tr P0 = Ne).

    For symmetric dH, d Tr(A P0) = Tr(A P1[dH]) with P1 the canonical first
    response, and the Daleckii-Krein kernel with the mu-projection is
    self-adjoint, so G is the canonical first-order response to sym(A).
    """
    r = canonical_response(h0, [np.asarray(A)], None, beta, Ne, M, order=1, eigh=eigh)
    return r["P1"][0]


def nonorthogonal_response(f0, f1s, f2s, z, beta, Ne, M, order=2):
    """Canonical response in a non-orthogonal basis (Sec. II, self-consistent free energy response).

    With Z the inverse factor of the overlap (Z^T S Z = I) the operators are
    taken to the orthogonalised basis, F_perp = Z^T F Z, the canonical problem
    is solved there with Tr P_perp = Ne, and D^(k) = Z P^(k) Z^T.
    Returns a dict with D0, D1, D2 (lists) and the mu jet.
    """
    to = lambda f: None if f is None else z.T @ (0.5 * (f + f.T)) @ z
    r = canonical_response(to(f0), [to(f) for f in f1s],
                           None if f2s is None else [to(f) for f in f2s], beta, Ne, M, order=order)
    back = lambda p: z @ p @ z.T
    return dict(D0=back(r["P0"]), D1=[back(p) for p in r["P1"]], D2=[back(p) for p in r["P2"]],
                mu0=r["mu0"], mu1=r["mu1"], mu2=r["mu2"])


# ----------------------------------------------------------------------------
# free energy (Sec. III) -- used only by tests of the n+1 rule
# ----------------------------------------------------------------------------

def entropy(occ):
    """S/k_B = -sum_i [f ln f + (1-f) ln(1-f)] over occupations f (Eq. SED)."""
    f = np.clip(np.asarray(occ, dtype=np.float64), 1e-300, 1 - 1e-16)
    g = 1.0 - f
    return float(-np.sum(np.where(f > 0, f * np.log(f), 0.0) + np.where(g > 0, g * np.log(g), 0.0)))


def omega(h, beta, Ne, M):
    """Canonical free energy Tr[P H] - T_e S[P] with k_B T_e = 1/beta (Eq. FreeE)."""
    w, v = eig(h)
    mu = mu_canonical(w, beta, M, Ne)
    f = phi(w - mu, beta, M)
    return float(np.sum(f * w)) - entropy(f) / beta
