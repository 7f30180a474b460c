"""GPU parity of the HIP path against the FP64 oracle (through the C ABI).

Tolerances: FP64 operator and preconditioner 1e-12 relative L2; FP64 solution
1e-10; integer tables bit-exact (covered on the host side).
"""
import numpy as np
import pytest

import meshgen
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
    # name, mesh kwargs, order, rotate/permute
    ("cube4_N4", dict(k=4, perturb=0.10), 4, False),
    ("rot3_N3", dict(k=3, perturb=0.10), 3, True),
    ("rot3_N2", dict(k=3, perturb=0.15), 2, True),
    ("box_N5", dict(k=(3, 2, 5), perturb=0.1, lengths=(1, 1, 8)), 5, True),
    ("rot2_N6", dict(k=2, perturb=0.1), 6, True),
    ("rot3_N7", dict(k=3, perturb=0.15), 7, True),
    ("rot2_N8", dict(k=(2, 3, 2), perturb=0.1), 8, True),
    ("rot2_N11", dict(k=2, perturb=0.1), 11, True),
    ("one_N15", dict(k=(2, 1, 1), perturb=0.0), 15, True),
    # extruded polygons: interior mesh edges of valence 3, 4 and 5 (NULL patch slots inside)
    ("star5_N4", dict(star=5, layers=3, perturb=0.05), 4, True),
    ("star3_N6", dict(star=3, layers=2, perturb=0.05), 6, True),
]


def make_mesh(kw):
    kw = dict(kw)
    if "star" in kw:
        return meshgen.star_mesh(kw.pop("star"), **kw)
    return meshgen.cube_mesh(**kw)


@pytest.fixture(scope="module", params=CASES, ids=[c[0] for c in CASES])
def case(request):
    from paper_1506_05996_amd import sem
    dev = _dev()
    name, kw, N, rot = request.param
    print(f"[case] {name}", flush=True)
    m = make_mesh(kw)
    if rot:
        m, _ = meshgen.rotate_elements(m, seed=41)
        m, _ = meshgen.permute_elements(m, seed=42)
    M = sem.Mesh(m.vtx, m.hex, N)
    P = Problem(m.vtx, m.hex, N)
    return dict(m=m, M=M, P=P, dev=dev, sem=sem)


def test_apply_A_fp64(case):
    M, P, dev = case["M"], case["P"], case["dev"]
    rng = np.random.default_rng(7)
    u = rng.uniform(-1, 1, M.n_global)
    y = M.apply_A(torch.tensor(u, device=dev)).cpu().numpy()
    assert rel_l2(y, P.A(u)) <= 1e-12
    # manufactured interpolant (smooth field)
    us = meshgen.manufactured_u(P.x, case["m"].lengths)
    ys = M.apply_A(torch.tensor(us, device=dev)).cpu().numpy()
    assert rel_l2(ys, P.A(us)) <= 1e-12


def test_apply_A_deterministic(case):
    M, dev = case["M"], case["dev"]
    u = torch.tensor(np.random.default_rng(8).uniform(-1, 1, M.n_global), device=dev)
    y1 = M.apply_A(u)
    y2 = M.apply_A(u)
    assert torch.equal(y1, y2)


def test_apply_A_fp32(case):
    M, P, dev = case["M"], case["P"], case["dev"]
    u = np.random.default_rng(9).uniform(-1, 1, M.n_global)
    y = M.apply_A(torch.tensor(u, device=dev, dtype=torch.float32)).double().cpu().numpy()
    err = rel_l2(y, P.A(u))
    print(f"fp32 Ax rel err {err:.2e}")
    assert err <= 5e-6


@pytest.mark.parametrize("pc", [3, 1, 2])
def test_precond_fp64(case, pc):
    M, P, dev = case["M"], case["P"], case["dev"]
    r = np.random.default_rng(10).uniform(-1, 1, M.n_global)
    r[P.num.dirichlet.astype(bool)] = 0.0
    z = M.precond(torch.tensor(r, device=dev), pc=pc).cpu().numpy()
    ref = P.precond(fine=bool(pc & 1), coarse=bool(pc & 2))(r)
    assert rel_l2(z, ref) <= 1e-12


def test_precond_fp32(case):
    M, P, dev = case["M"], case["P"], case["dev"]
    r = np.random.default_rng(11).uniform(-1, 1, M.n_global)
    r[P.num.dirichlet.astype(bool)] = 0.0
    z = M.precond(torch.tensor(r, device=dev, dtype=torch.float32)).double().cpu().numpy()
    err = rel_l2(z, P.precond()(r))
    print(f"fp32 precond rel err {err:.2e}")
    assert err <= 1e-5


@pytest.mark.parametrize("k", [24, 36])
def test_coarse_solve_large_fronts(k):
    # k^3 hexes: separators of up to (k-1)^2 vertices, so the sweeps take the
    # tile shapes of large fronts (24: 4 and 2 rows per wave; 36: also rows
    # longer than 1024 split across a workgroup's waves), forward and
    # backward; against the oracle's coarse matrix factorised directly on the
    # free vertices
    import scipy.sparse.linalg as spla
    from oracle.coarse import coarse_matrix
    from oracle.numbering import number_mesh
    from paper_1506_05996_amd import sem
    dev = _dev()
    print(f"[coarse large fronts] k={k}", flush=True)
    m = meshgen.cube_mesh(k, perturb=0.1, seed=7)
    m, _ = meshgen.rotate_elements(m, seed=8)
    M = sem.Mesh(m.vtx, m.hex, 2)
    num = number_mesh(m.hex, 2)
    nv = num.n_vertices
    free = np.nonzero(num.dirichlet[:nv] == 0)[0]
    Ac = coarse_matrix(m.vtx, m.hex, nv).tocsr()[free][:, free].tocsc()
    R = np.random.default_rng(1509).uniform(-1, 1, nv)
    Z = M.coarse_solve(torch.tensor(R, device=dev)).cpu().numpy()
    lu = spla.splu(Ac, permc_spec="MMD_AT_PLUS_A", diag_pivot_thresh=0.0, options=dict(SymmetricMode=True))
    ref = lu.solve(R[free])
    assert np.abs(Z[num.dirichlet[:nv].astype(bool)]).max() == 0.0
    assert rel_l2(Z[free], ref) <= 1e-11
    M.close()


def test_coarse_solve(case):
    M, P, dev = case["M"], case["P"], case["dev"]
    C = P.coarse
    R = np.random.default_rng(12).uniform(-1, 1, M.n_vertices)
    Z = M.coarse_solve(torch.tensor(R, device=dev)).cpu().numpy()
    assert rel_l2(Z, C.solve(R)) <= 1e-12


def test_pcg_fp64_matches_oracle(case):
    M, P, dev = case["M"], case["P"], case["dev"]
    b = P.load(lambda x: meshgen.manufactured_s(x, case["m"].lengths))
    ur, it_ref, hist, _ = P.solve(b, rtol=1e-8)
    x, info = M.solve(torch.tensor(b, device=dev), rtol=1e-8)
    # same preconditioner, same Krylov iteration: same count, same iterate
    assert abs(info["iterations"] - it_ref) <= 1
    x = x.cpu().numpy()
    assert rel_l2(x, ur) <= 1e-7
    # both solved tight: the unique discrete solution
    ut, _, _, _ = P.solve(b, rtol=1e-13)
    xt, info = M.solve(torch.tensor(b, device=dev), rtol=1e-13)
    assert rel_l2(xt.cpu().numpy(), ut) <= 1e-10


def test_pcg_refined(case):
    M, P, dev = case["M"], case["P"], case["dev"]
    sem = case["sem"]
    b = P.load(lambda x: meshgen.manufactured_s(x, case["m"].lengths))
    x, info = M.solve(torch.tensor(b, device=dev), mode=sem.SOLVE_FP32_REFINED, rtol=1e-10, inner_rtol=1e-3)
    x = x.cpu().numpy()
    true_res = np.linalg.norm(b - P.A(x)) / np.linalg.norm(b)
    print(f"refined: outer {info['outer']} inner {info['iterations']} true res {true_res:.2e}")
    assert true_res <= 1.5e-10
    ut, _, _, _ = P.solve(b, rtol=1e-13)
    assert rel_l2(x, ut) <= 1e-8


def test_solve_edge_cases():
    from paper_1506_05996_amd import sem
    dev = _dev()
    m = meshgen.cube_mesh(2, perturb=0.1)
    M = sem.Mesh(m.vtx, m.hex, 3)
    b0 = torch.zeros(M.n_global, dtype=torch.float64, device=dev)
    x, info = M.solve(b0)
    assert info["iterations"] == 0 and not x.any()
    P = Problem(m.vtx, m.hex, 3)
    b = torch.tensor(P.load(meshgen.manufactured_s), device=dev)
    x, info = M.solve(b, max_iter=1, raise_on_noconv=False)
    assert info["status"] == sem.SEM_ENOCONV and info["iterations"] == 1
    bn = b.clone()
    free = np.nonzero(P.num.dirichlet == 0)[0]
    bn[int(free[0])] = float("nan")
    xn = torch.zeros_like(b)
    with pytest.raises(sem.SemError) as e:
        M.solve(bn, x=xn)
    assert e.value.status == sem.SEM_EBREAKDOWN
    assert torch.isfinite(xn).all()


def test_solve_start_dirichlet_values_and_argument_checks():
    """A start that already meets the tolerance returns after 0 iterations with
    x unchanged; values of b on the Dirichlet set take no part in the solve;
    the binding rejects overlapping or mistyped vectors before any launch."""
    from paper_1506_05996_amd import sem
    dev = _dev()
    m = meshgen.cube_mesh(3, perturb=0.1, seed=5)
    M = sem.Mesh(m.vtx, m.hex, 4)
    P = Problem(m.vtx, m.hex, 4)
    b = torch.tensor(P.load(meshgen.manufactured_s), device=dev)
    x, _ = M.solve(b, rtol=1e-12)
    for mode in (sem.SOLVE_FP64, sem.SOLVE_FP32_REFINED):
        x0 = x.clone()
        x1, info = M.solve(b, x=x0, use_x0=True, rtol=1e-8, mode=mode)
        assert info["iterations"] == 0 and torch.equal(x1, x)
    dirty = b.clone()
    dirty[torch.tensor(P.num.dirichlet.astype(bool), device=dev)] = 3.0
    for mode in (sem.SOLVE_FP64, sem.SOLVE_FP32_REFINED):
        xa, ia = M.solve(b, rtol=1e-10, mode=mode)
        xb, ib = M.solve(dirty, rtol=1e-10, mode=mode)
        assert torch.equal(xa, xb) and ia["iterations"] == ib["iterations"]
    u = torch.rand(M.n_global, dtype=torch.float64, device=dev)
    with pytest.raises(ValueError):
        M.apply_A(u, u)
    with pytest.raises(ValueError):
        M.solve(b, x=b)
    with pytest.raises(TypeError):
        M.precond(u, torch.empty(M.n_global, dtype=torch.float32, device=dev))
    with pytest.raises(TypeError):
        M.solve(b, x=torch.zeros(M.n_global, dtype=torch.float32, device=dev))
    with pytest.raises(ValueError):
        M.solve(b, x=torch.zeros(M.n_global - 1, dtype=torch.float64, device=dev))


def test_custom_dirichlet_set():
    """Dirichlet on the two faces x = 0 and x = 1 only (natural Neumann
    elsewhere): operator, preconditioner and solve follow the new set."""
    from paper_1506_05996_amd import sem
    dev = _dev()
    m = meshgen.cube_mesh(3, perturb=0.1)
    m, _ = meshgen.rotate_elements(m, seed=51)
    N = 4
    M = sem.Mesh(m.vtx, m.hex, N)
    x = M.node_coords()
    mask = ((np.abs(x[:, 0]) < 1e-12) | (np.abs(x[:, 0] - 1) < 1e-12)).astype(np.uint8)
    # interior nodes of one element also constrained: exercises the masked-interior path
    l2g = M.numbering()
    mask[l2g[5, 2, 2, 2]] = 1
    M.set_dirichlet(mask)
    P = Problem(m.vtx, m.hex, N, dirichlet=mask)
    rng = np.random.default_rng(13)
    u = rng.uniform(-1, 1, M.n_global)
    assert rel_l2(M.apply_A(torch.tensor(u, device=dev)).cpu().numpy(), P.A(u)) <= 1e-12
    r = rng.uniform(-1, 1, M.n_global)
    r[mask.astype(bool)] = 0
    for pc in (1, 2, 3):
        z = M.precond(torch.tensor(r, device=dev), pc=pc).cpu().numpy()
        assert rel_l2(z, P.precond(fine=bool(pc & 1), coarse=bool(pc & 2))(r)) <= 1e-12
    b = P.load(lambda xx: np.sin(np.pi * xx[:, 0]) * (1 + xx[:, 1]))
    ut, _, _, _ = P.solve(b, rtol=1e-13)
    xg, info = M.solve(torch.tensor(b, device=dev), rtol=1e-13)
    assert rel_l2(xg.cpu().numpy(), ut) <= 1e-10


def test_autotuned_tile_gives_identical_results():
    """The tuned tile is one of the candidates.  A tile of the same kernel only
    regroups elements into workgroups: bitwise the default tile's results; a
    tile of another operator kernel sums in another order: equal to rounding."""
    from paper_1506_05996_amd import sem
    dev = _dev()
    m = meshgen.cube_mesh(4, perturb=0.1)
    m, _ = meshgen.permute_elements(m, seed=61)
    for N in (3, 4, 7):
        Ma = sem.Mesh(m.vtx, m.hex, N, autotune=False)
        Mb = sem.Mesh(m.vtx, m.hex, N, autotune=True)
        tiles = (1, 2, 4, 8, sem.TILE_GEO, sem.TILE_LINE_GEO, sem.TILE_LINE)
        assert Mb.tile(sem.SEM_F64) in tiles and Mb.tile(sem.SEM_F32) in tiles
        u = torch.tensor(np.random.default_rng(62).uniform(-1, 1, Ma.n_global), device=dev)
        for uu, dt, tol in ((u, sem.SEM_F64, 1e-14), (u.float(), sem.SEM_F32, 1e-6)):
            ya, yb = Ma.apply_A(uu), Mb.apply_A(uu)
            if Mb.tile(dt) in (1, 2, 4, 8):
                assert torch.equal(ya, yb)
            else:
                assert float(torch.linalg.norm((ya - yb).double()) / torch.linalg.norm(ya.double())) <= tol


@pytest.mark.parametrize("tile", ["TILE_GEO", "TILE_LINE_GEO", "TILE_LINE"])
@pytest.mark.parametrize("N", [2, 4, 7, 9, 10, 15])
def test_operator_kernel_variants(N, tile):
    """The operator kernels that rebuild G from the vertices (plane-staged and
    line-phase) and the line-phase kernel with stored factors match the oracle
    (FP64 to 1e-12, FP32 to the FP32 bound) on a rotated, permuted mesh.  N = 10
    takes the FP64 line contractions by output pairs with an odd line length
    (the middle output and column); N = 2 and 4 take it in FP32."""
    from paper_1506_05996_amd import sem
    dev = _dev()
    m = meshgen.cube_mesh((2, 3, 2), perturb=0.15, seed=81)
    m, _ = meshgen.rotate_elements(m, seed=82)
    m, _ = meshgen.permute_elements(m, seed=83)
    M = sem.Mesh(m.vtx, m.hex, N, autotune=False)
    M.set_tile(getattr(sem, tile))
    M.set_tile(getattr(sem, tile), sem.SEM_F32)
    P = Problem(m.vtx, m.hex, N, fine=False, coarse=False)
    u = np.random.default_rng(84).uniform(-1, 1, M.n_global)
    ref = P.A(u)
    y = M.apply_A(torch.tensor(u, device=dev)).cpu().numpy()
    assert rel_l2(y, ref) <= 1e-12
    y32 = M.apply_A(torch.tensor(u, device=dev, dtype=torch.float32)).double().cpu().numpy()
    assert rel_l2(y32, ref) <= 5e-6


@pytest.mark.parametrize("tile", [1, 16])
def test_order15_operator_variants(tile):
    """N = 15: the vector kernel and the matrix-core kernel both match the
    oracle in FP64 and FP32 (two elements, one face shared, ragged permuted
    numbering)."""
    from paper_1506_05996_amd import sem
    dev = _dev()
    m = meshgen.cube_mesh((2, 1, 2), perturb=0.1, seed=71)
    m, _ = meshgen.rotate_elements(m, seed=72)
    m, _ = meshgen.permute_elements(m, seed=73)
    M = sem.Mesh(m.vtx, m.hex, 15, autotune=False)
    M.set_tile(tile)
    P = Problem(m.vtx, m.hex, 15, fine=False, coarse=False)
    u = np.random.default_rng(74).uniform(-1, 1, M.n_global)
    y = M.apply_A(torch.tensor(u, device=dev)).cpu().numpy()
    ref = P.A(u)
    assert rel_l2(y, ref) <= 1e-12
    M.set_tile(tile, sem.SEM_F32)
    assert M.tile(sem.SEM_F32) == tile
    y32 = M.apply_A(torch.tensor(u, device=dev, dtype=torch.float32)).double().cpu().numpy()
    assert rel_l2(y32, ref) <= 5e-6
