"""Pins of the oracle's two-scale preconditioner and PCG (Sections 3-4)."""
import itertools
import os

import numpy as np
import pytest
import scipy.linalg

import meshgen
from oracle.brute import assemble_dense
from oracle.coarse import CoarseCorrection, coarse_matrix
from oracle.geometry import box_sizes
from oracle.gll import GLL
from oracle.problem import Problem
from oracle.schwarz import extended_pencil, fdm_basis, patch_table, stiffness_1d

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _pos(tok, n):
    return {"-1": 0, "0": 1, "N": n + 1, "N+1": n + 2}[tok]


@pytest.mark.parametrize("n", [2, 3, 5, 7])
def test_pencil_matches_displayed_pattern(n):
    """Entries of the displayed 1D system of Section 4.2 (golden file)."""
    g = GLL(n)
    K, M = extended_pencil(g)
    d = stiffness_1d(g)
    with open(os.path.join(GOLDEN, "pencil_pattern.txt")) as f:
        for line in f:
            if not line.strip() or line.startswith("#"):
                continue
            kind, r, c, fac, a, b = line.split()
            r, c = _pos(r, n), _pos(c, n)
            if kind == "K":
                assert abs(K[r, c] - float(fac) * d[int(a), int(b)]) < 1e-12 * n * n
            else:
                assert abs(M[r, c] - float(fac) * g.rho[int(a)]) < 1e-15
    # interior rows are the element's own d; rows -1 and n+1 couple to one node only
    assert np.allclose(K[2:n + 1, 1:n + 2], d[1:n, :], atol=1e-12)
    assert np.count_nonzero(K[0]) == 2 and np.count_nonzero(K[n + 2]) == 2
    assert np.allclose(M, np.diag(np.diag(M)))


def test_pencil_singular_at_order_one():
    """At n = 1 the neighbour's node n-1 is its far vertex, nothing is held at
    zero and the extended pencil is the singular free-free stiffness: the fine
    preconditioner needs n >= 2."""
    K, M = extended_pencil(GLL(1))
    assert abs(np.linalg.eigvalsh(K).min()) < 1e-14


@pytest.mark.parametrize("n", [2, 3, 4, 7, 10, 15])
def test_generalised_eigenbasis(n):
    g = GLL(n)
    K, M = extended_pencil(g)
    S, lam = fdm_basis(g)
    assert np.allclose(S.T @ M @ S, np.eye(n + 3), atol=1e-10)
    assert np.allclose(S.T @ K @ S, np.diag(lam), atol=1e-9 * lam.max())
    assert lam.min() > 0


def box_operator(n, h, kappa=1.0, c=0.0):
    K, M = extended_pencil(GLL(n))
    hx, hy, hz = h
    kron = np.kron
    return (hx * hy * hz / 8.0) * (
        4 * kappa * (kron(M, kron(M, K)) / hx ** 2 + kron(M, kron(K, M)) / hy ** 2
                     + kron(K, kron(M, M)) / hz ** 2) + c * kron(M, kron(M, M)))


@pytest.mark.parametrize("n", [2, 3, 4])
def test_fdm_equals_dense_box_inverse(n):
    mesh = meshgen.cube_mesh(2, perturb=0.1)
    P = Problem(mesh.vtx, mesh.hex, n, coarse=False)
    fine = P.fine
    rng = np.random.default_rng(5)
    h = np.array([[0.4, 0.55, 0.7]])
    r = rng.standard_normal((1, n + 3, n + 3, n + 3))
    z = fine.patch_solve(r, h)
    Abox = box_operator(n, h[0])
    z_ref = np.linalg.solve(Abox, r.reshape(-1))
    assert np.allclose(z.reshape(-1), z_ref, rtol=1e-11, atol=1e-11 * np.abs(z_ref).max())


def test_fdm_equals_true_patch_operator_on_uniform_mesh():
    """On an axis-aligned uniform mesh the box operator is the assembled
    operator restricted to the (n+3)^3 patch nodes of an interior element."""
    n = 3
    mesh = meshgen.cube_mesh(3)
    P = Problem(mesh.vtx, mesh.hex, n, coarse=False)
    A = assemble_dense(mesh.vtx, mesh.hex, P.num.l2g, P.num.n_global, P.gll)
    e = 13  # centre element of the 3^3 lattice
    Ip = P.fine.Ip[e].reshape(-1)
    assert (Ip >= 0).all()
    As = A[np.ix_(Ip, Ip)]
    Abox = box_operator(n, box_sizes(mesh.vtx, mesh.hex)[e])
    assert np.allclose(As, Abox, atol=1e-12 * np.abs(As).max())


@pytest.mark.parametrize("rotate", [False, True])
def test_patch_table_matches_coordinates(rotate):
    """I^p by unfolding across faces equals a coordinate lookup of the
    extended tensor grid on unperturbed meshes (any element orientation)."""
    n = 3
    mesh = meshgen.cube_mesh(3)
    if rotate:
        mesh, _ = meshgen.rotate_elements(mesh, seed=21)
        mesh, _ = meshgen.permute_elements(mesh, seed=22)
    P = Problem(mesh.vtx, mesh.hex, n, coarse=False)
    Ip = patch_table(P.num, mesh.hex)
    t = P.gll.t
    text = np.concatenate([[-2 + t[n - 1]], t, [2 + t[1]]])
    key = {tuple(np.round(x * 1e9).astype(np.int64)): g for g, x in enumerate(P.x)}
    Phi = np.stack([(1 - text) / 2, (1 + text) / 2], axis=1)
    for e in range(mesh.n_elem):
        X = mesh.vtx[mesh.hex[e]].reshape(2, 2, 2, 3)  # [c, b, a]
        xs = np.einsum("cbax,ia,jb,kc->kjix", X, Phi, Phi, Phi)
        for c, b, a in itertools.product(range(n + 3), repeat=3):
            g = key.get(tuple(np.round(xs[c, b, a] * 1e9).astype(np.int64)), -1)
            assert Ip[e, c, b, a] == g, (e, a, b, c)


def test_fine_preconditioner_symmetric_psd():
    mesh = meshgen.cube_mesh(2, perturb=0.1)
    P = Problem(mesh.vtx, mesh.hex, 3, coarse=False)
    ng = P.num.n_global
    Pm = np.stack([P.fine.apply(np.eye(ng)[i]) for i in range(ng)], axis=1)
    assert np.allclose(Pm, Pm.T, atol=1e-12 * np.abs(Pm).max())
    assert np.linalg.eigvalsh(0.5 * (Pm + Pm.T)).min() > -1e-10


def trilinear_interpolation(P):
    """I[N, v]: value at node N of the Q1 hat function of vertex v, built node
    by node from each node's first local copy."""
    n = P.n
    t = P.gll.t
    I = np.zeros((P.num.n_global, P.num.n_vertices))
    done = np.zeros(P.num.n_global, dtype=bool)
    for e in range(P.num.n_elem):
        for k, j, i in itertools.product(range(n + 1), repeat=3):
            g = P.num.l2g[e, k, j, i]
            if done[g]:
                continue
            done[g] = True
            for K, J, II in itertools.product((0, 1), repeat=3):
                v = P.num.l2g[e, K * n, J * n, II * n]
                w = ((1 + t[i]) / 2 if II else (1 - t[i]) / 2) * \
                    ((1 + t[j]) / 2 if J else (1 - t[j]) / 2) * \
                    ((1 + t[k]) / 2 if K else (1 - t[k]) / 2)
                I[g, v] += w
    return I


@pytest.mark.parametrize("n", [2, 4])
def test_coarse_transfer_is_trilinear_interpolation(n):
    mesh = meshgen.cube_mesh(3, perturb=0.15, seed=8)
    P = Problem(mesh.vtx, mesh.hex, n, fine=False)
    C = P.coarse
    I = trilinear_interpolation(P)
    rng = np.random.default_rng(3)
    r = rng.standard_normal(P.num.n_global)
    assert np.allclose(C.restrict(r), I.T @ r, atol=1e-13 * np.abs(r).sum())
    Z = rng.standard_normal(P.num.n_vertices)
    assert np.allclose(C.prolong(Z), I @ Z, atol=1e-13)


def test_coarse_matrix_is_order_one_operator():
    mesh = meshgen.cube_mesh(3, perturb=0.15, seed=8)
    P = Problem(mesh.vtx, mesh.hex, 4, fine=False)
    Ac = coarse_matrix(mesh.vtx, mesh.hex, P.num.n_vertices).toarray()
    from oracle.numbering import number_mesh
    num1 = number_mesh(mesh.hex, 1)
    Ad = assemble_dense(mesh.vtx, mesh.hex, num1.l2g, num1.n_global, GLL(1))
    assert np.allclose(Ac, Ad, atol=1e-13 * np.abs(Ad).max())
    free = P.coarse.free
    assert np.linalg.eigvalsh(Ac[np.ix_(free, free)]).min() > 0
    assert len(free) == 8  # (3-1)^3 interior vertices


def test_pcg_equals_direct_solve():
    mesh = meshgen.cube_mesh(2, perturb=0.1, seed=4)
    n = 3
    P = Problem(mesh.vtx, mesh.hex, n)
    A = assemble_dense(mesh.vtx, mesh.hex, P.num.l2g, P.num.n_global, P.gll)
    free = P.num.dirichlet == 0
    b = P.load(meshgen.manufactured_s)
    ud = np.zeros_like(b)
    ud[free] = scipy.linalg.solve(A[np.ix_(free, free)], b[free])
    for f, c in [(True, True), (True, False)]:
        u, it, hist, _ = P.solve(b, rtol=1e-14, fine=f, coarse=c)
        assert np.abs(u - ud).max() < 1e-12 * np.abs(ud).max()
        assert it < 60


def test_two_scale_preconditioner_symmetric_positive():
    mesh = meshgen.cube_mesh(2, perturb=0.1)
    P = Problem(mesh.vtx, mesh.hex, 2)
    prec = P.precond()
    free = np.nonzero(P.num.dirichlet == 0)[0]
    ng = P.num.n_global
    cols = []
    for i in free:
        e = np.zeros(ng)
        e[i] = 1.0
        cols.append(prec(e)[free])
    Pm = np.stack(cols, axis=1)
    assert np.allclose(Pm, Pm.T, atol=1e-12 * np.abs(Pm).max())
    assert np.linalg.eigvalsh(Pm).min() > 0


def test_b_zero_returns_zero():
    mesh = meshgen.cube_mesh(1)
    P = Problem(mesh.vtx, mesh.hex, 2)
    u, it, _, _ = P.solve(np.zeros(P.num.n_global))
    assert it == 0 and not u.any()


@pytest.mark.slow
def test_h_independence_trend():
    """Table 1's behaviour: two-scale counts stay nearly flat under refinement
    while fine-only counts grow (n = 3, constant source as in Section 6.1)."""
    counts = {}
    for k in (4, 8):
        mesh = meshgen.cube_mesh(k, perturb=0.1)
        P = Problem(mesh.vtx, mesh.hex, 3)
        b = P.load(lambda x: np.ones(len(x)))
        counts[k] = (P.solve(b, rtol=1e-8)[1], P.solve(b, rtol=1e-8, coarse=False)[1])
    two4, fine4 = counts[4]
    two8, fine8 = counts[8]
    assert two8 <= 1.25 * two4
    assert fine8 >= 1.3 * fine4
    assert two8 < fine8


# --- box sizes h_x, h_y, h_z on anisotropic and rotated meshes (Section 4.2) ---
ANISO = (1.0, 2.0, 3.0)  # domain lengths: h differs along each axis


def _box_sizes_eta_for_xi(vtx, hexes):
    """Planted mistake: h_x taken from the eta-edges."""
    h = box_sizes(vtx, hexes).copy()
    h[:, 0] = h[:, 1]
    return h


def _box_sizes_diagonal(vtx, hexes):
    """Planted mistake: mean face-diagonal length instead of the edge length."""
    X = vtx[np.asarray(hexes)].reshape(-1, 2, 2, 2, 3)
    hx = np.linalg.norm(X[:, :, 1, 1] - X[:, :, 0, 0], axis=-1).mean(axis=1)
    h = box_sizes(vtx, hexes).copy()
    h[:, 0] = hx
    return h


def box_size_pin_error(fn, k=3, rotate=False):
    """Largest deviation of fn's sizes from the extent of each element along the
    physical axis its reference axis points to (axis-aligned box, exact)."""
    mesh = meshgen.cube_mesh(k, lengths=ANISO)
    if rotate:
        mesh, _ = meshgen.rotate_elements(mesh, seed=31)
    h = fn(mesh.vtx, mesh.hex)
    X = mesh.vtx[mesh.hex]  # [E, 8, 3], corner a + 2b + 4c
    err = 0.0
    for d, corner in enumerate((1, 2, 4)):  # reference axes xi, eta, zeta
        edge = X[:, corner] - X[:, 0]
        axis = np.abs(edge).argmax(axis=1)
        ref = np.array(ANISO)[axis] / k
        err = max(err, float(np.abs(h[:, d] - ref).max()))
    return err


@pytest.mark.parametrize("rotate", [False, True])
def test_box_sizes_follow_each_reference_axis(rotate):
    assert box_size_pin_error(box_sizes, rotate=rotate) <= 1e-14


@pytest.mark.parametrize("fn", [_box_sizes_eta_for_xi, _box_sizes_diagonal])
def test_box_size_pin_rejects_planted_mistakes(fn):
    assert box_size_pin_error(fn, rotate=True) > 1e-2


def patch_identity_error(fn, rotate=False):
    """Deviation of the box operator built with fn's sizes from the assembled
    operator restricted to the centre element's (n+3)^3 patch, on an
    axis-aligned box with different h along each axis."""
    n = 3
    mesh = meshgen.cube_mesh(3, lengths=ANISO)
    if rotate:
        mesh, _ = meshgen.rotate_elements(mesh, seed=33)
    P = Problem(mesh.vtx, mesh.hex, n, coarse=False)
    A = assemble_dense(mesh.vtx, mesh.hex, P.num.l2g, P.num.n_global, P.gll)
    e = 13  # centre element of the 3^3 lattice
    Ip = P.fine.Ip[e].reshape(-1)
    assert (Ip >= 0).all()
    As = A[np.ix_(Ip, Ip)]
    Abox = box_operator(n, fn(mesh.vtx, mesh.hex)[e])
    return float(np.abs(As - Abox).max() / np.abs(As).max())


@pytest.mark.parametrize("rotate", [False, True])
def test_fdm_equals_true_patch_operator_on_anisotropic_mesh(rotate):
    assert patch_identity_error(box_sizes, rotate) <= 1e-12


def test_patch_identity_rejects_swapped_axes():
    assert patch_identity_error(_box_sizes_eta_for_xi) > 1e-2
