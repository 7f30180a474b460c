"""Pins of the oracle's 1D reference data (Section 2.1, eq. (D); Section 2.4)."""
import math

import numpy as np
import pytest

from oracle.gll import GLL, gll_points, gll_weights, lagrange_derivative_matrix
from oracle.schwarz import stiffness_1d

CLOSED_FORM = {
    1: ([-1, 1], [1, 1]),
    2: ([-1, 0, 1], [1 / 3, 4 / 3, 1 / 3]),
    3: ([-1, -1 / math.sqrt(5), 1 / math.sqrt(5), 1], [1 / 6, 5 / 6, 5 / 6, 1 / 6]),
    4: ([-1, -math.sqrt(3 / 7), 0, math.sqrt(3 / 7), 1],
        [1 / 10, 49 / 90, 32 / 45, 49 / 90, 1 / 10]),
}


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_points_weights_closed_form(n):
    t, w = CLOSED_FORM[n]
    assert np.allclose(gll_points(n), t, atol=1e-15, rtol=0)
    assert np.allclose(gll_weights(n), w, atol=1e-15, rtol=0)


@pytest.mark.parametrize("n", range(1, 16))
def test_quadrature_exact_to_2n_minus_1(n):
    g = GLL(n)
    assert abs(g.rho.sum() - 2.0) < 1e-14
    for p in range(2 * n):
        exact = 0.0 if p % 2 else 2.0 / (p + 1)
        assert abs((g.rho * g.t ** p).sum() - exact) < 1e-13, p
    # degree 2n is not integrated exactly (the rule has n+1 points with both ends fixed)
    p = 2 * n
    assert abs((g.rho * g.t ** p).sum() - 2.0 / (p + 1)) > 1e-12


@pytest.mark.parametrize("n", range(1, 16))
def test_derivative_matrix(n):
    g = GLL(n)
    D = g.D
    # D[i, j] = phi_j'(t_i): differentiates t^p exactly for p <= n
    for p in range(n + 1):
        exact = p * g.t ** (p - 1) if p > 0 else np.zeros_like(g.t)
        assert np.allclose(D @ g.t ** p, exact, atol=1e-11 * max(1, n * n)), p
    assert np.allclose(D.sum(axis=1), 0.0, atol=1e-11)
    assert abs(D[0, 0] + n * (n + 1) / 4) < 1e-10
    assert abs(D[n, n] - n * (n + 1) / 4) < 1e-10
    # closed form off the diagonal: P_n(t_i) / (P_n(t_j) (t_i - t_j))
    from oracle.gll import legendre
    Pn = legendre(n, g.t)
    for i in range(n + 1):
        for j in range(n + 1):
            if i != j:
                assert abs(D[i, j] - Pn[i] / (Pn[j] * (g.t[i] - g.t[j]))) < 1e-10 * n * n


def test_derivative_orientation_distinguishes_transpose():
    # the transpose of D does not differentiate: guards the index reading of eq. (D)
    g = GLL(4)
    assert not np.allclose(g.D.T @ g.t ** 2, 2 * g.t, atol=1e-6)


@pytest.mark.parametrize("n", range(1, 10))
def test_second_derivative_matrix(n):
    g = GLL(n)
    d = stiffness_1d(g)
    assert np.allclose(d, d.T, atol=1e-12)
    assert np.allclose(d @ np.ones(n + 1), 0.0, atol=1e-11)
    # d integrates u'v' exactly for u, v of degree <= n  (2n-2 <= 2n-1)
    for p in range(1, n + 1):
        for q in range(1, n + 1):
            exact = p * q * (0.0 if (p + q) % 2 else 2.0 / (p + q - 1))
            assert abs(g.t ** p @ d @ g.t ** q - exact) < 1e-10 * n ** 3
    if n == 1:
        assert np.allclose(d, [[0.5, -0.5], [-0.5, 0.5]], atol=1e-15)


def test_lagrange_definition_small():
    # hand-computed: points -1, 0, 1 give D = [[-3/2, 2, -1/2], [-1/2, 0, 1/2], [1/2, -2, 3/2]]
    D = lagrange_derivative_matrix(np.array([-1.0, 0.0, 1.0]))
    assert np.allclose(D, [[-1.5, 2, -0.5], [-0.5, 0, 0.5], [0.5, -2, 1.5]], atol=1e-15)
