"""GPU parity with one kappa_e and c_e per element (Algorithm 2), with kappa
and c at every node (eq. (R)) and with a Neumann part of the boundary
(eq. (pdeweak)), against the FP64 oracle through the C ABI.

Tolerances as for the Poisson path: FP64 operator, preconditioner and coarse
solve 1e-12 relative L2; FP64 solutions 1e-10 (both sides solved to 1e-13).
"""
import numpy as np
import pytest

import meshgen
from oracle.neumann import face_mass
from oracle.problem import Problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


CASES = [
    ("cube3_N3", dict(k=3, perturb=0.10), 3),
    ("rot2_N7", dict(k=2, perturb=0.15), 7),
    ("one_N15", dict(k=(2, 1, 1), perturb=0.0), 15),
]


@pytest.mark.parametrize("name,kw,N", CASES, ids=[c[0] for c in CASES])
def test_element_coefficients(name, kw, N):
    from paper_1506_05996_amd import sem
    dev = _dev()
    print(f"[coef case] {name}", flush=True)
    m = meshgen.cube_mesh(**kw)
    m, _ = meshgen.rotate_elements(m, seed=46)
    m, _ = meshgen.permute_elements(m, seed=47)
    E = len(m.hex)
    rng = np.random.default_rng(30)
    kap, c = rng.uniform(0.2, 3.0, E), rng.uniform(0.0, 5.0, E)
    M = sem.Mesh(m.vtx, m.hex, N)
    P = Problem(m.vtx, m.hex, N, kappa=kap, c=c)
    M.set_element_coefficients(kap, c)
    u = rng.uniform(-1, 1, M.n_global)
    tiles = [None] + ([sem.TILE_GEO, sem.TILE_LINE_GEO, sem.TILE_LINE] if N <= 9 else []) + ([16] if N == 15 else [])
    for tile in tiles:
        if tile is not None:
            M.set_tile(tile)
        y = M.apply_A(torch.tensor(u, device=dev)).cpu().numpy()
        assert rel_l2(y, P.A(u)) <= 1e-12, tile
    for tile in [None] + ([16] if N == 15 else []):
        if tile is not None:
            M.set_tile(tile, dtype=sem.SEM_F32)
        y32 = M.apply_A(torch.tensor(u, device=dev, dtype=torch.float32)).double().cpu().numpy()
        assert rel_l2(y32, P.A(u)) <= 1e-5, tile
    r = rng.uniform(-1, 1, M.n_global)
    r[P.num.dirichlet.astype(bool)] = 0.0
    for pc in (1, 2, 3):
        z = M.precond(torch.tensor(r, device=dev), pc=pc).cpu().numpy()
        assert rel_l2(z, P.precond(fine=bool(pc & 1), coarse=bool(pc & 2))(r)) <= 1e-12, pc
    R = rng.uniform(-1, 1, M.n_vertices)
    Z = M.coarse_solve(torch.tensor(R, device=dev)).cpu().numpy()
    assert rel_l2(Z, P.coarse.solve(R)) <= 1e-12
    b = P.load(lambda x: meshgen.manufactured_s(x, m.lengths))
    ut, _, _, _ = P.solve(b, rtol=1e-13)
    x, info = M.solve(torch.tensor(b, device=dev), rtol=1e-13)
    assert rel_l2(x.cpu().numpy(), ut) <= 1e-10
    x, info = M.solve(torch.tensor(b, device=dev), mode=sem.SOLVE_FP32_REFINED, rtol=1e-12)
    assert rel_l2(x.cpu().numpy(), ut) <= 1e-9
    # back to constant coefficients: the Poisson operator again
    M.set_coefficients(1.0, 0.0)
    P0 = Problem(m.vtx, m.hex, N)
    y = M.apply_A(torch.tensor(u, device=dev)).cpu().numpy()
    assert rel_l2(y, P0.A(u)) <= 1e-12


@pytest.mark.parametrize("name,kw,N", CASES, ids=[c[0] for c in CASES])
def test_node_coefficients(name, kw, N):
    from paper_1506_05996_amd import sem
    dev = _dev()
    print(f"[node coef case] {name}", flush=True)
    m = meshgen.cube_mesh(**kw)
    m, _ = meshgen.rotate_elements(m, seed=49)
    m, _ = meshgen.permute_elements(m, seed=50)
    E = len(m.hex)
    rng = np.random.default_rng(31)
    shape = (E, N + 1, N + 1, N + 1)
    kap, c = rng.uniform(0.2, 3.0, shape), rng.uniform(0.0, 5.0, shape)
    c[: E // 2] = 0.0  # elements without a mass term beside elements with one
    M = sem.Mesh(m.vtx, m.hex, N)
    G0, _ = M.geometry()
    P = Problem(m.vtx, m.hex, N, kappa=kap, c=c)
    M.set_node_coefficients(kap, c)
    assert np.isnan(M.coefficients()).all()
    assert np.array_equal(M.geometry()[0], G0)  # the host keeps the plain factors
    u = rng.uniform(-1, 1, M.n_global)
    yo = P.A(u)
    tiles = [None] + ([sem.TILE_GEO, sem.TILE_LINE_GEO, sem.TILE_LINE] if N <= 9 else []) + ([16] if N == 15 else [])
    for tile in tiles:
        if tile is not None:
            M.set_tile(tile)
        y = M.apply_A(torch.tensor(u, device=dev)).cpu().numpy()
        assert rel_l2(y, yo) <= 1e-12, tile
    for tile in [None] + ([sem.TILE_GEO, sem.TILE_LINE_GEO, sem.TILE_LINE] if N <= 9 else []) + ([16] if N == 15 else []):
        if tile is not None:
            M.set_tile(tile, dtype=sem.SEM_F32)
        y32 = M.apply_A(torch.tensor(u, device=dev, dtype=torch.float32)).double().cpu().numpy()
        assert rel_l2(y32, yo) <= 1e-5, tile
    r = rng.uniform(-1, 1, M.n_global)
    r[P.num.dirichlet.astype(bool)] = 0.0
    for pc in (1, 2, 3):
        z = M.precond(torch.tensor(r, device=dev), pc=pc).cpu().numpy()
        assert rel_l2(z, P.precond(fine=bool(pc & 1), coarse=bool(pc & 2))(r)) <= 1e-12, pc
    b = P.load(lambda x: meshgen.manufactured_s(x, m.lengths))
    ut, _, _, _ = P.solve(b, rtol=1e-13)
    x, info = M.solve(torch.tensor(b, device=dev), rtol=1e-13)
    assert rel_l2(x.cpu().numpy(), ut) <= 1e-10
    x, info = M.solve(torch.tensor(b, device=dev), mode=sem.SOLVE_FP32_REFINED, rtol=1e-12)
    assert rel_l2(x.cpu().numpy(), ut) <= 1e-9
    # back to constant, then per-element coefficients: the plain factors are
    # on the device again (also for the kernel that rebuilds them)
    M.set_coefficients(1.0, 0.0)
    P0 = Problem(m.vtx, m.hex, N)
    for tile in tiles:
        if tile is not None:
            M.set_tile(tile)
        y = M.apply_A(torch.tensor(u, device=dev)).cpu().numpy()
        assert rel_l2(y, P0.A(u)) <= 1e-12, tile
    ke = rng.uniform(0.5, 2.0, E)
    M.set_node_coefficients(kap)
    M.set_element_coefficients(ke)
    y = M.apply_A(torch.tensor(u, device=dev)).cpu().numpy()
    assert rel_l2(y, Problem(m.vtx, m.hex, N, fine=False, coarse=False, kappa=ke).A(u)) <= 1e-12


def test_node_mass_term_only_with_a_changed_dirichlet_set():
    # c per node with kappa left at 1, then a Dirichlet set with a free face:
    # the coarse matrix is refactorised with the element means of c
    from paper_1506_05996_amd import sem
    dev = _dev()
    m = meshgen.cube_mesh(3, perturb=0.1, seed=21)
    m, _ = meshgen.rotate_elements(m, seed=51)
    N = 4
    E = len(m.hex)
    c = np.random.default_rng(32).uniform(0.0, 8.0, (E, N + 1, N + 1, N + 1))
    M = sem.Mesh(m.vtx, m.hex, N)
    M.set_node_coefficients(None, c)
    x = M.node_coords()
    dirichlet = (M.boundary_mask().astype(bool) & ~(np.abs(x[:, 2] - 1.0) <= 1e-12)).astype(np.uint8)
    M.set_dirichlet(dirichlet)
    P = Problem(m.vtx, m.hex, N, dirichlet=dirichlet, c=c)
    rng = np.random.default_rng(33)
    u = rng.uniform(-1, 1, M.n_global)
    assert rel_l2(M.apply_A(torch.tensor(u, device=dev)).cpu().numpy(), P.A(u)) <= 1e-12
    r = rng.uniform(-1, 1, M.n_global)
    r[dirichlet.astype(bool)] = 0.0
    z = M.precond(torch.tensor(r, device=dev)).cpu().numpy()
    assert rel_l2(z, P.precond()(r)) <= 1e-12
    b = P.m * np.cos(x[:, 0])
    b[dirichlet.astype(bool)] = 0.0
    ut, it_o, _, _ = P.solve(b, rtol=1e-13)
    xs, info = M.solve(torch.tensor(b, device=dev), rtol=1e-13)
    assert rel_l2(xs.cpu().numpy(), ut) <= 1e-10
    assert abs(info["iterations"] - it_o) <= 2


@pytest.mark.parametrize("N", [4, 6])
def test_mixed_dirichlet_neumann_solve(N):
    from paper_1506_05996_amd import sem
    dev = _dev()
    m = meshgen.cube_mesh(2, perturb=0.1, seed=12)
    m, _ = meshgen.rotate_elements(m, seed=48)
    M = sem.Mesh(m.vtx, m.hex, N)
    x = M.node_coords()
    top = np.abs(x[:, 2] - 1.0) <= 1e-12
    side = ((np.abs(x[:, 0]) <= 1e-12) | (np.abs(x[:, 0] - 1) <= 1e-12)
            | (np.abs(x[:, 1]) <= 1e-12) | (np.abs(x[:, 1] - 1) <= 1e-12))
    dirichlet = (M.boundary_mask().astype(bool) & ~(top & ~side)).astype(np.uint8)
    M.set_dirichlet(dirichlet)
    faces = meshgen.top_faces(m)
    ws = M.boundary_face_mass(faces)
    b = M.lumped_mass() * meshgen.mixed_bc_s(x) + ws * meshgen.mixed_bc_g(x)
    b[dirichlet.astype(bool)] = 0.0
    P = Problem(m.vtx, m.hex, N, dirichlet=dirichlet)
    assert np.abs(ws - face_mass(P.num, m.vtx, m.hex, P.gll, faces)).max() <= 1e-14 * ws.max()
    ut, _, _, _ = P.solve(b, rtol=1e-13)
    xs, info = M.solve(torch.tensor(b, device=dev), rtol=1e-13)
    xs = xs.cpu().numpy()
    assert rel_l2(xs, ut) <= 1e-10
    err = np.abs(xs - meshgen.mixed_bc_u(x)).max()
    print(f"N={N} mixed-BC error vs exact {err:.2e}")
    assert err <= (1e-4 if N == 4 else 1e-6)


def test_single_element_mesh():
    # one hexahedron: every vertex is on the Dirichlet boundary, so the coarse
    # space is empty and P = P^f; operator, preconditioner and solve still match
    from paper_1506_05996_amd import sem
    dev = _dev()
    m = meshgen.cube_mesh(1, lengths=(1.0, 2.0, 0.5))
    for N in (2, 7, 15):
        M = sem.Mesh(m.vtx, m.hex, N)
        P = Problem(m.vtx, m.hex, N)
        assert M.n_vertices == 8
        u = np.random.default_rng(60).uniform(-1, 1, M.n_global)
        assert rel_l2(M.apply_A(torch.tensor(u, device=dev)).cpu().numpy(), P.A(u)) <= 1e-12
        r = np.random.default_rng(61).uniform(-1, 1, M.n_global)
        r[P.num.dirichlet.astype(bool)] = 0.0
        z = M.precond(torch.tensor(r, device=dev)).cpu().numpy()
        assert rel_l2(z, P.precond()(r)) <= 1e-12
        b = P.load(lambda x: meshgen.manufactured_s(x, m.lengths))
        ut, _, _, _ = P.solve(b, rtol=1e-13)
        x, _ = M.solve(torch.tensor(b, device=dev), rtol=1e-13)
        assert rel_l2(x.cpu().numpy(), ut) <= 1e-10


def test_no_dirichlet_nodes_with_a_mass_term():
    # c > 0 makes the problem definite without any Dirichlet node: every
    # vertex is a coarse unknown and nothing is masked
    from paper_1506_05996_amd import sem
    dev = _dev()
    m = meshgen.cube_mesh(3, perturb=0.1, seed=14)
    N = 4
    M = sem.Mesh(m.vtx, m.hex, N)
    M.set_dirichlet(np.zeros(M.n_global, np.uint8))
    M.set_coefficients(0.5, 3.0)
    none = np.zeros(M.n_global, np.uint8)
    P = Problem(m.vtx, m.hex, N, dirichlet=none, kappa=0.5, c=3.0)
    u = np.random.default_rng(62).uniform(-1, 1, M.n_global)
    assert rel_l2(M.apply_A(torch.tensor(u, device=dev)).cpu().numpy(), P.A(u)) <= 1e-12
    z = M.precond(torch.tensor(u, device=dev)).cpu().numpy()
    assert rel_l2(z, P.precond()(u)) <= 1e-12
    b = M.lumped_mass() * np.cos(M.node_coords()[:, 0])
    ut, _, _, _ = P.solve(b, rtol=1e-13)
    x, _ = M.solve(torch.tensor(b, device=dev), rtol=1e-13)
    assert rel_l2(x.cpu().numpy(), ut) <= 1e-10
