"""GPU parity of the constant-coefficient operator (kappa, c of eq. (pde)) and of
the backward Euler heat steps (Section 6.2) against the FP64 oracle, through
the C ABI.

Tolerances as for the Poisson path: FP64 operator and preconditioner 1e-12
relative L2, FP64 solutions 1e-10 (both sides solved to 1e-13).
"""
import numpy as np
import pytest

import meshgen
from oracle import heat
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
    ("cube3_N4", dict(k=3, perturb=0.10), 4),
    ("box_N5", dict(k=(2, 2, 6), perturb=0.1, lengths=(1, 1, 3)), 5),
    ("rot2_N7", dict(k=2, perturb=0.15), 7),
    ("one_N15", dict(k=(2, 1, 1), perturb=0.0), 15),
]
COEFS = [(0.3, 2.5), (1e-2, 25.0)]


@pytest.fixture(scope="module", params=CASES, ids=[c[0] for c in CASES])
def case(request):
    from paper_1506_05996_amd import sem
    dev = _dev()
    name, kw, N = request.param
    print(f"[heat case] {name}", flush=True)
    m = meshgen.cube_mesh(**kw)
    m, _ = meshgen.rotate_elements(m, seed=43)
    m, _ = meshgen.permute_elements(m, seed=44)
    M = sem.Mesh(m.vtx, m.hex, N)
    return dict(m=m, M=M, N=N, dev=dev, sem=sem)


@pytest.mark.parametrize("kc", COEFS, ids=["k0.3_c2.5", "k0.01_c25"])
def test_operator_and_precond_with_coefficients(case, kc):
    M, m, N, dev, sem = case["M"], case["m"], case["N"], case["dev"], case["sem"]
    kappa, c = kc
    P = Problem(m.vtx, m.hex, N, kappa=kappa, c=c)
    M.set_coefficients(kappa, c)
    assert M.coefficients() == (kappa, c)
    u = np.random.default_rng(20).uniform(-1, 1, M.n_global)
    tiles = [None] + ([sem.TILE_GEO, sem.TILE_LINE_GEO, sem.TILE_LINE] if N <= 9 else []) + ([16] if N == 15 else [])
    for tile in tiles:
        if tile is not None:
            M.set_tile(tile)
        y = M.apply_A(torch.tensor(u, device=dev)).cpu().numpy()
        assert rel_l2(y, P.A(u)) <= 1e-12, tile
    y32 = M.apply_A(torch.tensor(u, device=dev, dtype=torch.float32)).double().cpu().numpy()
    assert rel_l2(y32, P.A(u)) <= 1e-5
    r = np.random.default_rng(21).uniform(-1, 1, M.n_global)
    r[P.num.dirichlet.astype(bool)] = 0.0
    for pc in (1, 2, 3):
        z = M.precond(torch.tensor(r, device=dev), pc=pc).cpu().numpy()
        assert rel_l2(z, P.precond(fine=bool(pc & 1), coarse=bool(pc & 2))(r)) <= 1e-12, pc
    R = np.random.default_rng(22).uniform(-1, 1, M.n_vertices)
    Z = M.coarse_solve(torch.tensor(R, device=dev)).cpu().numpy()
    assert rel_l2(Z, P.coarse.solve(R)) <= 1e-12
    M.set_coefficients(1.0, 0.0)


def test_default_coefficients_restore_the_poisson_operator(case):
    # setting kappa, c and going back to (1, 0) gives bit for bit the operator
    # of a fresh handle
    M, m, N, dev, sem = case["M"], case["m"], case["N"], case["dev"], case["sem"]
    u = torch.tensor(np.random.default_rng(23).uniform(-1, 1, M.n_global), device=dev)
    y0 = M.apply_A(u).cpu().numpy()
    M.set_coefficients(0.3, 2.5)
    M.set_coefficients(1.0, 0.0)
    y1 = M.apply_A(u).cpu().numpy()
    assert np.array_equal(y0, y1)


def test_heat_steps_match_the_oracle(case):
    M, m, N, dev, sem = case["M"], case["m"], case["N"], case["dev"], case["sem"]
    kappa, dt, steps = 0.05, 0.02, 3
    P = heat.heat_problem(m.vtx, m.hex, N, kappa, dt)
    src = [meshgen.heat_source(P.x, dt * (s + 1), m.lengths, sigma=0.3, t_end=dt * steps, z_start=0.3,
                               z_end=0.7) for s in range(steps)]
    u0 = np.zeros(M.n_global)
    ref, its = heat.backward_euler(P, u0, src, dt, rtol=1e-13)
    u = torch.tensor(u0, device=dev)
    for s in range(steps):
        q = torch.tensor(src[s], device=dev)
        u, info = M.heat_step(u, dt, kappa, q=q, rtol=1e-13)
        assert rel_l2(u.cpu().numpy(), ref[s]) <= 1e-10, s
        assert abs(info["iterations"] - its[s]) <= 2, (info, its[s])
    # the FP32-refined form of the same step reaches the same solution
    u_prev = torch.tensor(ref[-2], device=dev)
    ur, info = M.heat_step(u_prev, dt, kappa, q=torch.tensor(src[-1], device=dev),
                           mode=sem.SOLVE_FP32_REFINED, rtol=1e-12)
    assert rel_l2(ur.cpu().numpy(), ref[-1]) <= 1e-9
    # no source: pure decay from the last state, in place (u_next is u_prev)
    u_last = torch.tensor(ref[-1], device=dev)
    ref_decay, _ = heat.backward_euler(P, ref[-1], [np.zeros(M.n_global)], dt, rtol=1e-13)
    u_dec, _ = M.heat_step(u_last, dt, kappa, q=None, u_next=u_last, rtol=1e-13)
    assert u_dec.data_ptr() == u_last.data_ptr()
    assert rel_l2(u_dec.cpu().numpy(), ref_decay[0]) <= 1e-10
    M.set_coefficients(1.0, 0.0)
