"""Eq. (Rec_F_2) evaluated on a truncated power series in lambda, FP64.

A test pin for the oracle that uses neither eigenvalues nor the closed form
nor divided differences.  The perturbed Hamiltonian
H(lambda) = H0 + lambda H1 + lambda^2 H2 + ... (Sec. II, Eq. (H_prt)) and the
chemical-potential expansion mu(lambda) make the recursion's start
X_0(lambda) = I/2 - 2^-(M+2) beta (H(lambda) - mu(lambda) I) a matrix
polynomial in lambda.  Every step of Eq. (Rec_F_2) is a rational function of
the iterate, so it is carried out in the ring of matrix series truncated
after lambda^m: products are Cauchy products and the inverse of
X^2 + (I - X)^2 is the series inverse.  The coefficients of X_M(lambda) are
then P^(0), ..., P^(m) of Eq. (P_resp).  This is a different computation from
Algorithm 1's per-order linear systems and from the oracle's
eigenbasis formulas, and it reaches the same result.

The canonical values of mu^(k) are found by a separate Newton iteration on
the trace conditions Tr P^(0) = Ne, Tr P^(k) = 0 (k >= 1) with the slope
d Tr P^(0)/d mu0 approximated by beta Tr[P0 (I - P0)] (Eq. NewtRaphs).

The X form keeps every eigen-component near x = 1/2, where the map has slope
2, so rounding is amplified by up to 2^M: use M <= 12.
"""
import numpy as np


class Series:
    """Matrix power series c[0] + lambda c[1] + ... truncated after lambda^(len(c) - 1)."""

    def __init__(self, coeffs):
        self.c = [np.asarray(a, dtype=np.float64) for a in coeffs]

    @property
    def order(self):
        return len(self.c) - 1

    def __add__(self, other):
        return Series([a + b for a, b in zip(self.c, other.c)])

    def __sub__(self, other):
        return Series([a - b for a, b in zip(self.c, other.c)])

    def scale(self, s):
        return Series([s * a for a in self.c])

    def __matmul__(self, other):
        m = self.order
        return Series([sum(self.c[i] @ other.c[k - i] for i in range(k + 1)) for k in range(m + 1)])

    def inverse(self):
        """B with A B = I up to lambda^m: B0 = A0^-1, Bk = -A0^-1 sum_{i=1..k} Ai B(k-i)."""
        a0inv = np.linalg.inv(self.c[0])
        b = [a0inv]
        for k in range(1, self.order + 1):
            b.append(-a0inv @ sum(self.c[i] @ b[k - i] for i in range(1, k + 1)))
        return Series(b)


def identity(n, m):
    return Series([np.eye(n)] + [np.zeros((n, n))] * m)


def recursion(h, beta, M, mu, order):
    """Coefficients [P^(0), ..., P^(order)] of X_M(lambda) for H = sum_k lambda^k h[k], mu likewise."""
    n = h[0].shape[0]
    eye = identity(n, order)
    c = 2.0 ** (-(M + 2)) * beta
    K = Series([h[k] - mu[k] * np.eye(n) for k in range(order + 1)])
    x = eye.scale(0.5) - K.scale(c)
    for _ in range(M):
        x2 = x @ x
        den = x2 + (eye - x) @ (eye - x)
        x = x2 @ den.inverse()
    return x.c


def canonical(h, beta, Ne, M, order, mu0=None, tol=1e-12, max_iter=100):
    """mu jet with Tr P^(0) = Ne and Tr P^(k) = 0; returns (P[0..order], mu[0..order], iterations)."""
    n = h[0].shape[0]
    mu = [float(np.trace(h[0]) / n) if mu0 is None else mu0] + [0.0] * order
    for it in range(1, max_iter + 1):
        P = recursion(h, beta, M, mu, order)
        tr = [float(np.trace(p)) for p in P]
        err = abs(tr[0] - Ne) + sum(abs(t) for t in tr[1:])
        if err <= tol:
            return P, mu, it
        slope = beta * float(np.trace(P[0] - P[0] @ P[0]))
        mu = [mu[0] + (Ne - tr[0]) / slope] + [m - t / slope for m, t in zip(mu[1:], tr[1:])]
    raise RuntimeError("the mu jet did not converge")
