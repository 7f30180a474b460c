"""Pins of the oracle's constant-coefficient operator (kappa, c of eq. (pde)),
its order-1 coarse matrix, and the backward Euler heat steps of Section 6.2.

Each pin is fixed by something other than the oracle's own formulas: the dense
brute-force assembly, the exact volume of the domain, and the closed-form
backward Euler recursion for a Dirichlet eigenmode of the cube.
"""
import numpy as np

import meshgen
from oracle import heat
from oracle.brute import assemble_dense
from oracle.coarse import coarse_matrix
from oracle.gll import GLL
from oracle.numbering import number_mesh
from oracle.problem import Problem


def test_coarse_matrix_with_kappa_c_equals_brute_force():
    m = meshgen.cube_mesh(3, perturb=0.15, seed=5)
    num1 = number_mesh(m.hex, 1)
    for kappa, c in ((1.0, 0.0), (0.7, 2.5), (1e-2, 25.0)):
        A = coarse_matrix(m.vtx, m.hex, num1.n_global, kappa=kappa, c=c).toarray()
        B = assemble_dense(m.vtx, m.hex, num1.l2g, num1.n_global, GLL(1), kappa=kappa, c=c)
        assert np.abs(A - B).max() <= 1e-13 * np.abs(B).max()


def test_mass_term_integrates_the_volume():
    # No Dirichlet nodes: the stiffness part maps constants to zero and the
    # mass part gives c m_N; GLL with n >= 2 integrates |J| of a trilinear map
    # exactly, so the entries sum to c times the box volume (1 x 2 x 0.5).
    m = meshgen.cube_mesh((3, 2, 4), lengths=(1.0, 2.0, 0.5), perturb=0.15, seed=3)
    for n in (2, 4):
        ng = number_mesh(m.hex, n).n_global
        P = Problem(m.vtx, m.hex, n, fine=False, coarse=False, dirichlet=np.zeros(ng, np.uint8),
                    kappa=0.3, c=2.5)
        y = P.A(np.ones(ng))
        assert abs(y.sum() - 2.5) <= 1e-12
        # the order-1 coarse mass at the corners is exact only for affine elements
    mu = meshgen.cube_mesh((3, 2, 4), lengths=(1.0, 2.0, 0.5), perturb=0.0)
    A1 = coarse_matrix(mu.vtx, mu.hex, len(mu.vtx), kappa=1.0, c=2.5)
    assert abs(A1.sum() - 2.5) <= 1e-12


def test_kappa_scales_the_stiffness():
    m = meshgen.cube_mesh(2, perturb=0.1, seed=8)
    P1 = Problem(m.vtx, m.hex, 4, fine=False, coarse=False)
    Pk = Problem(m.vtx, m.hex, 4, fine=False, coarse=False, kappa=0.37)
    u = np.random.default_rng(0).uniform(-1, 1, P1.num.n_global)
    a, b = Pk.A(u), 0.37 * P1.A(u)
    assert np.linalg.norm(a - b) <= 1e-14 * np.linalg.norm(b)


def _mode_setup(n=6, k=3):
    m = meshgen.cube_mesh(k, perturb=0.0)
    kappa, dt = 0.5, 0.01
    P = heat.heat_problem(m.vtx, m.hex, n, kappa, dt)
    phi = meshgen.manufactured_u(P.x)
    phi[P.dirichlet.astype(bool)] = 0.0
    lam = 3.0 * np.pi ** 2  # -Laplace(phi) = lam phi on the unit cube
    return P, phi, kappa, dt, lam


def test_backward_euler_decays_an_eigenmode():
    # u^t = g^s u^0 with g = 1 / (1 + dt kappa lam) for u^0 = phi, q = 0, up to
    # the spatial error of order 6 on h = 1/3 (4e-9 measured; a dropped c or
    # kappa term gives errors of order 1)
    P, phi, kappa, dt, lam = _mode_setup()
    g = 1.0 / (1.0 + dt * kappa * lam)
    us, its = heat.backward_euler(P, phi, [np.zeros_like(phi)] * 4, dt, rtol=1e-13)
    for s, u in enumerate(us, 1):
        assert np.abs(u - g ** s * phi).max() <= 1e-7 * g ** s
    assert all(k > 0 for k in its)


def test_backward_euler_approaches_the_steady_state():
    # source q = a phi, u^0 = 0: u^t = (1 - g^s) a phi / (kappa lam)
    P, phi, kappa, dt, lam = _mode_setup()
    a = 3.0
    g = 1.0 / (1.0 + dt * kappa * lam)
    us, _ = heat.backward_euler(P, np.zeros_like(phi), [a * phi] * 3, dt, rtol=1e-13)
    for s, u in enumerate(us, 1):
        exact = (1.0 - g ** s) * a / (kappa * lam) * phi
        assert np.abs(u - exact).max() <= 1e-7 * np.abs(exact).max()
