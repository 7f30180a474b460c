"""Pins of the oracle's aggregation AMG with K-cycle (Section 4.1, "Algebraic
multigrid"): structural facts of the hierarchy checked against dense
algebra, exactness on a one-level hierarchy, h-independent convergence (the
property the paper reports), and that the AMG-preconditioned solve reaches the
same discrete solution as the exact coarse solve.
"""
import numpy as np
import pytest

import meshgen
from oracle.amg import KCycle, hierarchy, pairwise
from oracle.coarse import coarse_matrix
from oracle.numbering import number_mesh
from oracle.problem import Problem


def _free_Ac(k, seed=3):
    m = meshgen.cube_mesh(k, perturb=0.15, seed=seed)
    num = number_mesh(m.hex, 1)
    A = coarse_matrix(m.vtx, m.hex, num.n_global).tocsr()
    free = np.nonzero(num.dirichlet == 0)[0]
    return A[free][:, free].tocsr()


def test_aggregates_partition_the_unknowns():
    A = _free_Ac(14)
    As, aggs = hierarchy(A)
    assert len(As) >= 3
    for l, agg in enumerate(aggs):
        n, nc = As[l].shape[0], As[l + 1].shape[0]
        assert agg.shape == (n,) and agg.min() == 0 and agg.max() == nc - 1
        sizes = np.bincount(agg)
        assert sizes.min() >= 1 and sizes.max() <= 4
    a1 = pairwise(A)
    assert np.bincount(a1).max() <= 2


def test_galerkin_matrices_equal_dense_products():
    A = _free_Ac(12)
    As, aggs = hierarchy(A)
    for l, agg in enumerate(aggs):
        P = np.zeros((As[l].shape[0], As[l + 1].shape[0]))
        P[np.arange(agg.size), agg] = 1.0
        ref = P.T @ As[l].toarray() @ P
        assert np.abs(As[l + 1].toarray() - ref).max() <= 1e-13 * np.abs(ref).max()


def test_one_level_hierarchy_is_the_exact_inverse():
    A = _free_Ac(6)  # 125 unknowns: coarsest at once
    K = KCycle(A)
    assert K.L == 0
    b = np.random.default_rng(1).uniform(-1, 1, A.shape[0])
    x = K(b)
    assert np.linalg.norm(A @ x - b) <= 1e-12 * np.linalg.norm(b)


def _pcg_iterations(A, K, rtol=1e-8):
    b = np.random.default_rng(0).uniform(-1, 1, A.shape[0])
    x = np.zeros_like(b)
    r = b.copy()
    z = K(r)
    p = z.copy()
    rz = r @ z
    it = 0
    while np.linalg.norm(r) > rtol * np.linalg.norm(b) and it < 300:
        w = A @ p
        a = rz / (p @ w)
        x += a * p
        r -= a * w
        z = K(r)
        rzn = r @ z
        p = z + (rzn / rz) * p
        rz = rzn
        it += 1
    return it


def test_kcycle_convergence_is_h_independent():
    its = [_pcg_iterations(A, KCycle(A)) for A in (_free_Ac(12), _free_Ac(20), _free_Ac(28))]
    assert max(its) <= 25 and max(its) - min(its) <= 5, its


def test_amg_preconditioned_solve_reaches_the_exact_solution():
    m = meshgen.cube_mesh(10, perturb=0.1, seed=6)  # 729 free vertices: a two-level hierarchy or more
    P_exact = Problem(m.vtx, m.hex, 2)
    P_amg = Problem(m.vtx, m.hex, 2, coarse_solver="amg")
    assert P_amg.coarse.kcycle.L >= 1
    b = P_exact.load(lambda x: meshgen.manufactured_s(x))
    ue, it_e, _, _ = P_exact.solve(b, rtol=1e-12)
    ua, it_a, _, _ = P_amg.solve(b, rtol=1e-12)
    assert np.linalg.norm(ua - ue) <= 1e-9 * np.linalg.norm(ue)
    assert it_a <= 2 * it_e + 10


# --- pins of the two pieces of the K-cycle against closed forms --------------
#
# Two flexible-CG steps with search directions v = B b and v2 = B r2 (B any
# preconditioner, here the next cycle) are a Galerkin method: the result is
# the A-orthogonal projection of A^{-1} b onto span{v, v2},
# x = V (V^T A V)^{-1} V^T b with V = [v, v2], and the first step leaves the
# residual r2 = b - A v (v^T b)/(v^T A v).  A two-grid cycle (damped Jacobi
# S = I - omega D^{-1} A before and after, exact coarse solve on the Galerkin
# matrix with the aggregate indicator P) is the linear operator B with error
# propagation I - B A = S (I - P A_c^{-1} P^T A) S, i.e. B = (I - E) A^{-1}.
# Both are textbook identities, checked here with dense algebra only.


def _multilevel():
    K = KCycle(_free_Ac(14))  # levels 2197, 559, 146
    assert K.L >= 2, K.L
    return K


class _Recorder:
    """Wraps KCycle.cycle at one level and keeps the (input, output) pairs."""

    def __init__(self, K, level):
        self.K, self.level, self.calls = K, level, []
        self.orig = K.cycle

    def __call__(self, l, b):
        x = self.orig(l, b)
        if l == self.level:
            self.calls.append((b.copy(), x.copy()))
        return x


def fcg2_pin_error(K, l, b):
    """Largest relative deviation of K.fcg2(l, b) from the Galerkin projection
    onto the two directions the cycle produced (and of the second direction's
    input from the residual after the first step)."""
    rec = _Recorder(K, l)
    K.cycle = rec
    try:
        x = K.fcg2(l, b)
    finally:
        del K.cycle  # back to the class method
    A = K.As[l].toarray()
    (b1, v), (r2, v2) = rec.calls[:2]
    assert len(rec.calls) == 2 and np.array_equal(b1, b)
    r2_ref = b - A @ v * ((v @ b) / (v @ A @ v))
    V = np.stack([v, v2], axis=1)
    x_ref = V @ np.linalg.solve(V.T @ A @ V, V.T @ b)
    return max(np.linalg.norm(r2 - r2_ref) / np.linalg.norm(b), np.linalg.norm(x - x_ref) / np.linalg.norm(x_ref))


def two_grid_pin_error(K, l, b):
    """Relative deviation of K.cycle(l, b) from the two-grid operator
    (I - S (I - P A_c^{-1} P^T A) S) A^{-1} b; needs l + 1 == K.L."""
    assert l + 1 == K.L
    A = K.As[l].toarray()
    Ac = K.As[l + 1].toarray()
    n = A.shape[0]
    P = np.zeros((n, Ac.shape[0]))
    P[np.arange(n), K.aggs[l]] = 1.0
    S = np.eye(n) - (2.0 / 3.0) * A / np.diag(A)[:, None]
    E = S @ (np.eye(n) - P @ np.linalg.solve(Ac, P.T @ A)) @ S
    x_ref = (np.eye(n) - E) @ np.linalg.solve(A, b)
    x = K.cycle(l, b)
    return np.linalg.norm(x - x_ref) / np.linalg.norm(x_ref)


def test_fcg2_is_the_galerkin_projection_on_its_two_directions():
    K = _multilevel()
    rng = np.random.default_rng(11)
    for l in range(1, K.L):
        b = rng.uniform(-1, 1, K.As[l].shape[0])
        assert fcg2_pin_error(K, l, b) <= 1e-11


def test_cycle_is_the_two_grid_operator_on_the_last_two_levels():
    K = _multilevel()
    rng = np.random.default_rng(12)
    for _ in range(3):
        b = rng.uniform(-1, 1, K.As[K.L - 1].shape[0])
        assert two_grid_pin_error(K, K.L - 1, b) <= 1e-11


class _WrongOrthogonalisation(KCycle):
    def fcg2(self, l, b):  # planted mistake: the second direction is not A-orthogonalised
        A = self.As[l]
        v = self.cycle(l, b)
        w = A @ v
        rho, a1 = float(v @ b), float(v @ w)
        r2 = b - (rho / a1) * w
        v2 = self.cycle(l, r2)
        return (rho / a1) * v + (float(v2 @ r2) / float(v2 @ (A @ v2))) * v2


class _WrongFirstStep(KCycle):
    def fcg2(self, l, b):  # planted mistake: the first step length uses r^T r instead of v^T b
        A = self.As[l]
        v = self.cycle(l, b)
        w = A @ v
        rho, a1 = float(b @ b), float(v @ w)
        r2 = b - (rho / a1) * w
        v2 = self.cycle(l, r2)
        w2 = A @ v2
        g, be, a2 = float(v2 @ w), float(v2 @ w2), float(v2 @ r2)
        den = be - g * g / a1
        return (rho / a1) * v + (a2 / den) * (v2 - (g / a1) * v)


class _NoPostSmoothing(KCycle):
    def cycle(self, l, b):  # planted mistake: the Jacobi sweep after the coarse correction is dropped
        if l == self.L:
            return self.coarsest(b)
        A, D = self.As[l], self.D[l]
        x = (2.0 / 3.0) * b / D
        rc = self.restrict(l, b - A @ x)
        xc = self.coarsest(rc) if l + 1 == self.L else self.fcg2(l + 1, rc)
        return x + xc[self.aggs[l]]


class _UndampedJacobi(KCycle):
    def cycle(self, l, b):  # planted mistake: omega = 1 in the pre-smoothing sweep
        if l == self.L:
            return self.coarsest(b)
        A, D = self.As[l], self.D[l]
        x = b / D
        rc = self.restrict(l, b - A @ x)
        xc = self.coarsest(rc) if l + 1 == self.L else self.fcg2(l + 1, rc)
        x = x + xc[self.aggs[l]]
        return x + (2.0 / 3.0) * (b - A @ x) / D


@pytest.mark.parametrize("cls", [_WrongOrthogonalisation, _WrongFirstStep])
def test_fcg2_pin_rejects_planted_mistakes(cls):
    K = cls(_free_Ac(14))
    b = np.random.default_rng(11).uniform(-1, 1, K.As[1].shape[0])
    assert fcg2_pin_error(K, 1, b) > 1e-4


@pytest.mark.parametrize("cls", [_NoPostSmoothing, _UndampedJacobi])
def test_two_grid_pin_rejects_planted_mistakes(cls):
    K = cls(_free_Ac(14))
    b = np.random.default_rng(12).uniform(-1, 1, K.As[K.L - 1].shape[0])
    assert two_grid_pin_error(K, K.L - 1, b) > 1e-4
