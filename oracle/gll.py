"""GLL nodes, weights and the 1D derivative matrix (Section 2.1, eq. (D); Section 2.4).

Test infrastructure: plain FP64 definitions.

* Points: the n+1 Gauss-Lobatto-Legendre points are -1, +1 and the roots of
  P_n'(t) (the paper takes them from Deville, Fischer and Mund).
* Weights: the GLL quadrature weights rho_i = 2 / (n (n+1) P_n(t_i)^2), exact
  for polynomials of degree 2n-1 (Section 2.4).
* Derivative matrix: the value at node t_i of the derivative of the j-th
  Lagrange interpolant through the GLL points.  The paper writes eq. (D) with
  the indices the other way round, but its derivative formulas in Section 2.4
  sum D_{im} u_m to get the derivative at t_i, which is only right for
  D[i, j] = phi_j'(t_i); that reading is used throughout.

Pinned by: closed-form points/weights for n = 1..4, sum of weights = 2,
quadrature exactness to degree 2n-1, exact differentiation of t^p for p <= n,
and the corner entries -n(n+1)/4, +n(n+1)/4.
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as npleg


def legendre(n: int, t):
    """P_n(t) via numpy's Legendre series (library primitive)."""
    c = np.zeros(n + 1)
    c[n] = 1.0
    return npleg.legval(t, c)


def gll_points(n: int) -> np.ndarray:
    """The n+1 GLL points on [-1, 1], ascending."""
    if n < 1:
        raise ValueError("order must be >= 1")
    c = np.zeros(n + 1)
    c[n] = 1.0
    inner = np.sort(np.real(npleg.legroots(npleg.legder(c)))) if n >= 2 else np.array([])
    # polish the interior roots of P_n' with Newton steps on the same series
    d1 = npleg.legder(c)
    d2 = npleg.legder(c, 2)
    for _ in range(3):
        if inner.size:
            inner = inner - npleg.legval(inner, d1) / npleg.legval(inner, d2)
    return np.concatenate([[-1.0], inner, [1.0]])


def gll_weights(n: int, t=None) -> np.ndarray:
    if t is None:
        t = gll_points(n)
    return 2.0 / (n * (n + 1) * legendre(n, t) ** 2)


def lagrange_derivative_matrix(t: np.ndarray) -> np.ndarray:
    """D[i, j] = phi_j'(t_i) for the Lagrange basis phi_j through the points t.

    Written out from the definition phi_j(x) = prod_{m != j} (x - t_m)/(t_j - t_m):
    its derivative is the sum over l != j of 1/(t_j - t_l) times the product over
    m not in {j, l} of (x - t_m)/(t_j - t_m).
    """
    n1 = len(t)
    D = np.zeros((n1, n1))
    for i in range(n1):
        for j in range(n1):
            s = 0.0
            for l in range(n1):
                if l == j:
                    continue
                prod = 1.0 / (t[j] - t[l])
                for m in range(n1):
                    if m == j or m == l:
                        continue
                    prod *= (t[i] - t[m]) / (t[j] - t[m])
                s += prod
            D[i, j] = s
    return D


def lagrange_values(t: np.ndarray, x) -> np.ndarray:
    """phi_j(x) for all j (columns), x a 1D array (rows)."""
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n1 = len(t)
    V = np.ones((x.size, n1))
    for j in range(n1):
        for m in range(n1):
            if m != j:
                V[:, j] *= (x - t[m]) / (t[j] - t[m])
    return V


class GLL:
    """Bundle of the 1D reference data for order n."""

    def __init__(self, n: int):
        self.n = n
        self.t = gll_points(n)
        self.rho = gll_weights(n, self.t)
        self.D = lagrange_derivative_matrix(self.t)
