"""Pins of the oracle's per-element kappa and c (Algorithm 2 takes them per
element) and of its Neumann boundary term (eq. (pde), eq. (pdeweak)).

Fixed by the dense brute-force assembly element by element, the dense inverse
of each patch's box operator, the exact area of planar boundary faces, and a
manufactured solution with Dirichlet and Neumann parts of the boundary.
"""
import numpy as np
import pytest

import meshgen
from oracle.brute import element_matrix
from oracle.coarse import coarse_matrix
from oracle.gll import GLL
from oracle.neumann import face_mass
from oracle.numbering import number_mesh
from oracle.problem import Problem
from oracle.schwarz import extended_pencil, fdm_basis, fdm_patch_solve


def _per_element(E, seed=0):
    rng = np.random.default_rng(seed)
    return rng.uniform(0.2, 3.0, E), rng.uniform(0.0, 5.0, E)


def _dense(vtx, hexes, l2g, n_global, gll, kappa, c):
    A = np.zeros((n_global, n_global))
    for e in range(len(hexes)):
        K = element_matrix(vtx[hexes[e]], gll, kappa[e], c[e])
        idx = l2g[e].reshape(-1)
        A[np.ix_(idx, idx)] += K
    return A


def test_operator_with_element_coefficients_equals_brute_force():
    m = meshgen.cube_mesh(2, perturb=0.12, seed=9)
    n = 3
    kap, c = _per_element(len(m.hex))
    ng = number_mesh(m.hex, n).n_global
    P = Problem(m.vtx, m.hex, n, fine=False, coarse=False, dirichlet=np.zeros(ng, np.uint8), kappa=kap, c=c)
    A = _dense(m.vtx, m.hex, P.num.l2g, ng, P.gll, kap, c)
    u = np.random.default_rng(1).uniform(-1, 1, ng)
    assert np.linalg.norm(P.A(u) - A @ u) <= 1e-12 * np.linalg.norm(A @ u)


def test_coarse_matrix_with_element_coefficients_equals_brute_force():
    m = meshgen.cube_mesh(3, perturb=0.12, seed=10)
    kap, c = _per_element(len(m.hex), seed=2)
    num1 = number_mesh(m.hex, 1)
    A = coarse_matrix(m.vtx, m.hex, num1.n_global, kappa=kap, c=c).toarray()
    B = _dense(m.vtx, m.hex, num1.l2g, num1.n_global, GLL(1), kap, c)
    assert np.abs(A - B).max() <= 1e-13 * np.abs(B).max()


@pytest.mark.parametrize("n", [2, 4])
def test_patch_solve_with_per_patch_coefficients(n):
    # each patch's FDM solve inverts its own box operator with its own kappa, c
    K, M = extended_pencil(GLL(n))
    S, lam = fdm_basis(GLL(n))
    h = np.array([[0.4, 0.55, 0.7], [0.9, 0.3, 0.5]])
    kap = np.array([0.3, 2.0])
    c = np.array([4.0, 0.5])
    r = np.random.default_rng(6).standard_normal((2, n + 3, n + 3, n + 3))
    z = fdm_patch_solve(S, lam, r, h, kap, c)
    kron = np.kron
    for s in range(2):
        hx, hy, hz = h[s]
        Abox = (hx * hy * hz / 8.0) * (
            4 * kap[s] * (kron(M, kron(M, K)) / hx ** 2 + kron(M, kron(K, M)) / hy ** 2
                          + kron(K, kron(M, M)) / hz ** 2) + c[s] * kron(M, kron(M, M)))
        zr = np.linalg.solve(Abox, r[s].reshape(-1))
        assert np.allclose(z[s].reshape(-1), zr, rtol=1e-11, atol=1e-11 * np.abs(zr).max())


def test_face_mass_sums_to_the_face_areas():
    m = meshgen.cube_mesh((3, 2, 4), lengths=(1.0, 2.0, 0.5), perturb=0.15, seed=4)
    for n in (2, 5):
        num = number_mesh(m.hex, n)
        ws = face_mass(num, m.vtx, m.hex, GLL(n), meshgen.top_faces(m))
        assert abs(ws.sum() - 1.0 * 2.0) <= 1e-13
        assert (ws >= 0).all()


def test_mixed_dirichlet_neumann_solution_converges():
    # u = sin(pi x) sin(pi y) (z + z^2): Dirichlet on every face but z = 1,
    # Neumann data 3 sin(pi x) sin(pi y) there (a dropped term errs by O(1))
    errs = []
    for n in (4, 6):
        m = meshgen.cube_mesh(2, perturb=0.1, seed=12)
        P0 = Problem(m.vtx, m.hex, n)
        x = P0.x
        top = np.abs(x[:, 2] - 1.0) <= 1e-12
        side = ((np.abs(x[:, 0]) <= 1e-12) | (np.abs(x[:, 0] - 1) <= 1e-12)
                | (np.abs(x[:, 1]) <= 1e-12) | (np.abs(x[:, 1] - 1) <= 1e-12))
        dirichlet = (P0.num.dirichlet.astype(bool) & ~(top & ~side)).astype(np.uint8)
        P = Problem(m.vtx, m.hex, n, dirichlet=dirichlet)
        ws = face_mass(P.num, m.vtx, m.hex, P.gll, meshgen.top_faces(m))
        b = P.m * meshgen.mixed_bc_s(x) + ws * meshgen.mixed_bc_g(x)
        b[dirichlet.astype(bool)] = 0.0
        u, _, _, _ = P.solve(b, rtol=1e-13)
        errs.append(np.abs(u - meshgen.mixed_bc_u(x)).max())
    assert errs[1] < errs[0] / 20 and errs[1] <= 1e-5, errs
