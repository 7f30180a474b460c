"""sem_pcg_solve_noalloc (work in the library's static scratch array) against
sem_pcg_solve on the same handles: two no-allocation solves in a row, the
second on a smaller mesh, in FP64 and in the FP32-refined form.  The solves
run the same kernels in the same order, so the solutions and iteration counts
are equal (checked to the FP64 solution bar, 1e-10, and exactly for counts)."""
import numpy as np
import pytest

import meshgen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def rel_l2(a, b):
    return float(torch.linalg.norm(a - b) / max(float(torch.linalg.norm(b)), 1e-300))


@pytest.mark.parametrize("mode", ["SOLVE_FP64", "SOLVE_FP32_REFINED"])
def test_noalloc_solve_matches_pcg_solve(mode):
    from paper_1506_05996_amd import sem
    dev = _dev()
    mode = getattr(sem, mode)
    cases = []
    for k, N, seed in ((5, 6, 91), (3, 4, 92)):  # the second mesh is the smaller one
        m = meshgen.cube_mesh(k, perturb=0.1, seed=seed)
        m, _ = meshgen.permute_elements(m, seed=seed + 1)
        M = sem.Mesh(m.vtx, m.hex, N)
        rng = np.random.default_rng(seed + 2)
        b = torch.tensor(rng.uniform(-1, 1, M.n_global) * (1 - M.boundary_mask()), device=dev)
        print(f"[noalloc] k={k} N={N} n_global={M.n_global} mode={mode}", flush=True)
        cases.append((M, b))
    xs = []
    for M, b in cases:  # two no-allocation solves in a row, large then small
        x = torch.zeros_like(b)
        _, info = M.solve(b, x=x, mode=mode, rtol=1e-10, noalloc=True)
        torch.cuda.synchronize()
        xs.append((x.clone(), info))
    for (M, b), (x_na, info_na) in zip(cases, xs):
        x_ref, info = M.solve(b, mode=mode, rtol=1e-10)
        assert info_na["iterations"] == info["iterations"] and info_na["outer"] == info["outer"]
        assert rel_l2(x_na, x_ref) <= 1e-10
        assert info_na["rel_residual"] <= 1e-10
        # the handle's own buffers serve the next ordinary solve
        assert torch.equal(M.solve(b, mode=mode, rtol=1e-10)[0], x_ref)
