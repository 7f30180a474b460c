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
