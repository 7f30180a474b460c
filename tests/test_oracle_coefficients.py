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
from oracle.schwarz import element_mean, extended_pencil, fdm_basis, fdm_patch_solve


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


# --- kappa and c per node (eq. (R) weights each quadrature point by its own kappa)

def _per_node(E, n, seed=0):
    rng = np.random.default_rng(seed)
    shape = (E, n + 1, n + 1, n + 1)
    return rng.uniform(0.2, 3.0, shape), rng.uniform(0.0, 5.0, shape)


def test_operator_with_node_coefficients_equals_brute_force():
    m = meshgen.cube_mesh(2, perturb=0.12, seed=14)
    n = 3
    kap, c = _per_node(len(m.hex), n, seed=3)
    ng = number_mesh(m.hex, n).n_global
    P = Problem(m.vtx, m.hex, n, fine=False, coarse=False, dirichlet=np.zeros(ng, np.uint8), kappa=kap, c=c)
    A = _dense(m.vtx, m.hex, P.num.l2g, ng, P.gll, kap, c)
    assert np.abs(A - A.T).max() <= 1e-13 * np.abs(A).max()
    u = np.random.default_rng(1).uniform(-1, 1, ng)
    assert np.linalg.norm(P.A(u) - A @ u) <= 1e-12 * np.linalg.norm(A @ u)


@pytest.mark.parametrize("n", [2, 5])
def test_coordinate_functions_under_node_kappa(n):
    # x and y lie in the trilinear SEM space, so their gradients are exact at
    # every quadrature point: y^T A x = sum_q w_q kappa_q (e_x . e_y) = 0 and
    # x^T A x = sum of kappa times the local mass (no derivative matrices)
    m = meshgen.cube_mesh((2, 3, 2), perturb=0.15, seed=15)
    kap, _ = _per_node(len(m.hex), n, seed=4)
    ng = number_mesh(m.hex, n).n_global
    P = Problem(m.vtx, m.hex, n, fine=False, coarse=False, dirichlet=np.zeros(ng, np.uint8), kappa=kap)
    ux, uy = P.x[:, 0].copy(), P.x[:, 1].copy()
    Ax = P.A(ux)
    energy = float(np.sum(kap * P.geo.mass))
    assert abs(ux @ Ax - energy) <= 1e-12 * energy
    assert abs(uy @ Ax) <= 1e-12 * energy


def test_node_coefficients_constant_in_each_element_match_element_mode():
    m = meshgen.cube_mesh(2, perturb=0.1, seed=16)
    n = 4
    E = len(m.hex)
    kap, c = _per_element(E, seed=5)
    full = (E, n + 1, n + 1, n + 1)
    Pe = Problem(m.vtx, m.hex, n, kappa=kap, c=c)
    Pn = Problem(m.vtx, m.hex, n, kappa=np.broadcast_to(kap[:, None, None, None], full).copy(),
                 c=np.broadcast_to(c[:, None, None, None], full).copy())
    u = np.random.default_rng(2).uniform(-1, 1, Pe.num.n_global)
    ye, yn = Pe.A(u), Pn.A(u)
    assert np.linalg.norm(ye - yn) <= 1e-13 * np.linalg.norm(ye)
    ze, zn = Pe.precond()(u), Pn.precond()(u)
    assert np.linalg.norm(ze - zn) <= 1e-13 * np.linalg.norm(ze)


@pytest.mark.parametrize("n", [3, 6])
def test_element_mean_is_exact_for_low_degree_polynomials(n):
    # the GLL rule is exact to degree 2n - 1: the mean of
    # 1 + xi^2 + eta^4 + zeta^3 over the reference cube is 1 + 1/3 + 1/5
    g = GLL(n)
    t = g.t
    v = (1 + t[None, None, :] ** 2 + t[None, :, None] ** 4 + t[:, None, None] ** 3)[None]
    v = np.concatenate([v, 2.5 * np.ones_like(v)])
    assert np.allclose(element_mean(g, v), [1 + 1 / 3 + 1 / 5, 2.5], rtol=0, atol=1e-14)


def test_variable_kappa_solution_converges():
    # -div((1 + x) grad u) = s with u = sin(pi x) sin(pi y) sin(pi z):
    # s = (1 + x) 3 pi^2 u - pi cos(pi x) sin(pi y) sin(pi z); kappa sampled at
    # the nodes (a kappa dropped or applied after the derivative transpose errs by O(1))
    errs = []
    for n in (4, 6):
        m = meshgen.cube_mesh(2, perturb=0.1, seed=17)
        P0 = Problem(m.vtx, m.hex, n, fine=False, coarse=False)
        xl = P0.x[P0.num.l2g]  # [E, k, j, i, 3]
        P = Problem(m.vtx, m.hex, n, kappa=1.0 + xl[..., 0])
        x = P.x
        sx, sy, sz = (np.sin(np.pi * x[:, d]) for d in range(3))
        u_ex = sx * sy * sz
        s = (1.0 + x[:, 0]) * 3 * np.pi ** 2 * u_ex - np.pi * np.cos(np.pi * x[:, 0]) * sy * sz
        b = P.m * s
        b[P.dirichlet.astype(bool)] = 0.0
        u, _, _, _ = P.solve(b, rtol=1e-13)
        errs.append(np.abs(u - u_ex).max())
    assert errs[1] < errs[0] / 20 and errs[1] <= 1e-4, errs
