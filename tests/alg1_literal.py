"""Algorithm 1 of the paper, written out literally (X-form, dense solves), FP64.

A test pin for the oracle: an independent path (no eigenvalues, no closed
form) that follows the paper's steps in its own notation: the X_0 start of
Eq. (Rec_F_2), the per-step systems T X_n^(k) = C^(k) + sum B X of
Algorithm 1 (solved here with LAPACK instead of conjugate gradients), the
definitions of T, C and B given under "using", and the Newton updates of the
mu jet with P_mu = beta P0 (I - P0).  Orders 0..3 are supported.

Because it keeps the paper's X = I/2 - D form, rounding near x = 1/2 is
amplified by up to 2^M, so it is only used with small M (<= 12) where that
stays below 1e-12.
"""
import numpy as np


def _c(x, m):
    """C^(m) = sum_{i+j=m} X^(i) X^(j)."""
    return sum(x[i] @ x[m - i] for i in range(m + 1))


def recursion(h, beta, M, mu, order):
    """One pass: returns [X_M^(0..order)] for H = [H^(0..order)], mu = [mu^(0..order)]."""
    n = h[0].shape[0]
    eye = np.eye(n)
    c = 2.0 ** (-(M + 2)) * beta
    x = [0.5 * eye - c * (h[0] - mu[0] * eye)]
    for i in range(1, order + 1):
        x.append(-c * (h[i] - mu[i] * eye))
    for _ in range(M):
        T = 2.0 * x[0] @ (x[0] - eye) + eye
        C = [_c(x, m) for m in range(order + 1)]
        B = [None] + [2.0 * (x[m] - C[m]) for m in range(1, order + 1)]
        new = [np.linalg.solve(T, C[0])]
        for m in range(1, order + 1):
            rhs = C[m] + sum(B[m - k] @ new[k] for k in range(m))
            new.append(np.linalg.solve(T, rhs))
        x = new
    return x


def canonical(h, beta, Ne, M, order, mu0=None, tol=1e-12, max_iter=100):
    """Algorithm 1's while loop; returns (P[0..order], mu[0..order], iterations)."""
    n = h[0].shape[0]
    mu = [float(np.trace(h[0]) / n) if mu0 is None else mu0] + [0.0] * order
    for it in range(1, max_iter + 1):
        P = recursion(h, beta, M, mu, order)
        tr = [float(np.trace(p)) for p in P]
        tr_pmu = beta * float(np.trace(P[0] @ (np.eye(n) - P[0])))
        err = abs(tr[0] - Ne) + sum(abs(t) for t in tr[1:])
        if err <= tol:
            return P, mu, it
        mu[0] = mu[0] + (Ne - tr[0]) / tr_pmu
        for i in range(1, order + 1):
            mu[i] = mu[i] - tr[i] / tr_pmu
    raise RuntimeError("Algorithm 1 did not converge")
