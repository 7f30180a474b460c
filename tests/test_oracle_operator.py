"""Pins of the oracle's geometry and matrix-free operator (Sections 2.3-2.4, eq. (R))."""
import numpy as np
import pytest

import meshgen
from oracle.brute import assemble_dense
from oracle.geometry import Geometry, lumped_mass, node_coords_global
from oracle.gll import GLL
from oracle.numbering import number_mesh
from oracle.operator import apply_A, element_action
from oracle.problem import Problem


def sheared_mesh(k, n_seed=0):
    """Cube mesh under one global affine map (every element affine)."""
    m = meshgen.cube_mesh(k)
    M = np.array([[1.0, 0.3, -0.2], [0.1, 0.9, 0.25], [-0.15, 0.2, 1.1]])
    vtx = m.vtx @ M.T + np.array([0.2, -0.1, 0.05])
    return vtx, m.hex, M


@pytest.mark.parametrize("name,lengths,expect", [("unit", (1, 1, 1), 1.0),
                                                 ("stretched", (1, 1, 8), 8.0)])
@pytest.mark.parametrize("n", [2, 4, 7])
def test_lumped_mass_sums_to_volume(name, lengths, expect, n):
    m = meshgen.cube_mesh(3, lengths=lengths, perturb=0.1)
    num = number_mesh(m.hex, n)
    geo = Geometry(m.vtx, m.hex, GLL(n))
    assert abs(lumped_mass(num, geo).sum() - expect) < 1e-12 * expect


def test_affine_geometric_factors_closed_form():
    vtx, hexes, M = sheared_mesh(2)
    n = 3
    g = GLL(n)
    geo = Geometry(vtx, hexes, g)
    h = 0.5
    J = M * (h / 2)  # d x / d xi for an element of side h mapped by M
    detJ = np.linalg.det(J)
    Ginv = np.linalg.inv(J.T @ J)
    w = np.einsum("k,j,i->kji", g.rho, g.rho, g.rho)
    for e in range(len(hexes)):
        assert np.allclose(geo.mass[e], w * detJ, atol=1e-14)
        for a, (r, c) in enumerate([(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]):
            assert np.allclose(geo.G[a, e], w * detJ * Ginv[r, c], atol=1e-13)


@pytest.mark.parametrize("k,n,pert", [(1, 4, 0.0), (2, 2, 0.15), (2, 3, 0.15), (1, 5, 0.0)])
def test_matrix_free_equals_dense_brute_force(k, n, pert):
    m = meshgen.cube_mesh(k, perturb=pert, seed=3)
    if k == 1:  # perturb the single element's corners directly
        rng = np.random.default_rng(4)
        m.vtx = m.vtx + rng.uniform(-0.08, 0.08, m.vtx.shape)
    g = GLL(n)
    num = number_mesh(m.hex, n)
    geo = Geometry(m.vtx, m.hex, g)
    A = assemble_dense(m.vtx, m.hex, num.l2g, num.n_global, g)
    rng = np.random.default_rng(1)
    none = np.zeros(num.n_global, dtype=np.uint8)
    for _ in range(3):
        u = rng.uniform(-1, 1, num.n_global)
        y = apply_A(num, geo, g, u, dirichlet=none)
        assert np.linalg.norm(y - A @ u) <= 1e-13 * np.linalg.norm(A @ u)
    assert np.allclose(A, A.T, atol=1e-13 * np.abs(A).max())
    assert np.abs(A @ np.ones(num.n_global)).max() < 1e-12 * np.abs(A).max()
    free = num.dirichlet == 0
    if free.any():
        assert np.linalg.eigvalsh(A[np.ix_(free, free)]).min() > 0


def test_with_reaction_term_matches_dense():
    m = meshgen.cube_mesh(2, perturb=0.1, seed=9)
    n = 3
    g = GLL(n)
    num = number_mesh(m.hex, n)
    geo = Geometry(m.vtx, m.hex, g)
    A = assemble_dense(m.vtx, m.hex, num.l2g, num.n_global, g, kappa=0.7, c=2.5)
    u = np.random.default_rng(2).uniform(-1, 1, num.n_global)
    E = num.n_elem
    r = element_action(u[num.l2g], geo.G, g.D, kappa=np.full(E, 0.7), c=np.full(E, 2.5),
                       mass=geo.mass)
    y = np.zeros(num.n_global)
    np.add.at(y, num.l2g.reshape(-1), r.reshape(-1))
    assert np.linalg.norm(y - A @ u) <= 1e-13 * np.linalg.norm(A @ u)


def poly_and_laplacian(x, n):
    """A fixed polynomial of total degree n and its negative Laplacian."""
    X, Y, Z = x[:, 0], x[:, 1], x[:, 2]
    if n == 2:
        u = X * X + 2 * X * Y - Y * Z + 0.5 * Z * Z + X - 1
        lap = 2 + 1.0
    else:
        u = X ** n + Y ** (n - 1) * Z - 2 * X * Y ** (n - 1) + Z ** n
        lap = (n * (n - 1) * X ** (n - 2) + (n - 1) * (n - 2) * Y ** (n - 3) * Z
               - 2 * (n - 1) * (n - 2) * X * Y ** (n - 3) + n * (n - 1) * Z ** (n - 2))
    return u, -lap


@pytest.mark.parametrize("n", [2, 3, 4, 5])
def test_polynomial_exactness_on_affine_mesh(n):
    """On affine elements every GLL integrand has degree <= 2n-1 per variable,
    so (A u)_N = m_N (-Laplace u)(x_N) at interior nodes for deg(u) <= n."""
    vtx, hexes, _ = sheared_mesh(2)
    P = Problem(vtx, hexes, n, fine=False, coarse=False)
    u, mlap = poly_and_laplacian(P.x, n)
    none = np.zeros(P.num.n_global, dtype=np.uint8)
    y = apply_A(P.num, P.geo, P.gll, u, dirichlet=none)
    inner = P.num.dirichlet == 0
    expect = P.m * mlap
    assert np.abs(y[inner] - expect[inner]).max() < 1e-10 * np.abs(expect).max()


@pytest.mark.parametrize("n", [2, 3, 4])
def test_linear_patch_test_trilinear(n):
    """A linear field has zero residual at interior nodes of a perturbed mesh."""
    m = meshgen.cube_mesh(3, perturb=0.2, seed=11)
    P = Problem(m.vtx, m.hex, n, fine=False, coarse=False)
    u = 0.3 * P.x[:, 0] - 1.2 * P.x[:, 1] + 0.7 * P.x[:, 2] + 0.4
    none = np.zeros(P.num.n_global, dtype=np.uint8)
    y = apply_A(P.num, P.geo, P.gll, u, dirichlet=none)
    inner = P.num.dirichlet == 0
    assert np.abs(y[inner]).max() < 1e-12


def test_spectral_convergence_manufactured():
    """Nodal error of the discrete solution falls geometrically with n."""
    mesh = meshgen.cube_mesh(2, perturb=0.1)
    errs = []
    ns = [2, 3, 4, 5, 6, 7, 8]
    for n in ns:
        P = Problem(mesh.vtx, mesh.hex, n, fine=False, coarse=False)
        b = P.load(meshgen.manufactured_s)
        free = P.num.dirichlet == 0
        import scipy.linalg
        A = assemble_dense(mesh.vtx, mesh.hex, P.num.l2g, P.num.n_global, P.gll) if n <= 3 else None
        u, it, hist, _ = P.solve(b, rtol=1e-13, max_iter=5000, fine=False, coarse=False)
        ue = meshgen.manufactured_u(P.x)
        ue[~free] = 0
        errs.append(np.abs(u - ue).max())
        if A is not None:
            ud = np.zeros_like(u)
            ud[free] = scipy.linalg.solve(A[np.ix_(free, free)], b[free])
            assert np.abs(ud - u).max() < 1e-10
    errs = np.array(errs)
    slope = np.polyfit(ns, np.log(errs), 1)[0]
    assert slope < -1.0, errs
    assert (np.diff(np.log(errs)) < 0).all(), errs
    assert errs[-1] < 1e-6
