"""Batched solves: results equal per-instance solves (same iteration counts,
same solutions to 1e-10 of the tight oracle solution), FP64 and refined."""
import numpy as np
import pytest

import meshgen
from oracle.problem import Problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


SPECS = [  # (k, N, perturb, rotate): orders 3..8 as in the 64-instance workload, sizes 343..24,389
    (2, 3, 0.1, False), (3, 3, 0.1, True), (3, 5, 0.1, False), (2, 5, 0.15, True),
    (4, 4, 0.1, False), (2, 4, 0.1, True), (1, 6, 0.0, False), (3, 4, 0.1, True),
    (3, 7, 0.1, True), (2, 8, 0.1, False), (4, 7, 0.1, False), (2, 6, 0.1, True),
]
BIG = 10  # index of the 24,389-DOF instance (4^3 hexes at N = 7)


@pytest.fixture(scope="module")
def batch():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1506_05996_amd import sem
    dev = torch.device("cuda:0")
    meshes, probs, rhs = [], [], []
    for i, (k, N, p, rot) in enumerate(SPECS):
        m = meshgen.cube_mesh(k, perturb=p, seed=100 + i)
        if rot:
            m, _ = meshgen.rotate_elements(m, seed=200 + i)
            m, _ = meshgen.permute_elements(m, seed=300 + i)
        meshes.append((m.vtx, m.hex, N))
        P = Problem(m.vtx, m.hex, N)
        probs.append(P)
        b = np.random.default_rng(400 + i).uniform(-1, 1, P.num.n_global)
        b[P.num.dirichlet.astype(bool)] = 0.0
        if i == 6:
            b[:] = 0.0  # one instance with b = 0
        rhs.append(b)
    B = sem.Batch(meshes)
    assert B.n_global == [P.num.n_global for P in probs]
    assert B.n_global[BIG] > 20000 and {7, 8} <= {N for _, _, N in meshes}
    # the oracle's solutions, solved tight
    tight = [P.solve(b, rtol=1e-13)[0] if b.any() else None for P, b in zip(probs, rhs)]
    return dict(B=B, meshes=meshes, probs=probs, rhs=rhs, tight=tight, dev=dev, sem=sem)


def test_batch_fp64_matches_single_solves(batch):
    """At the workload's tolerance: each instance's true residual within 1e-10
    and the iteration count of the single solve (+-1)."""
    B, sem, dev = batch["B"], batch["sem"], batch["dev"]
    bs = [torch.tensor(b, device=dev) for b in batch["rhs"]]
    xs, infos, status = B.solve(bs, rtol=1e-10)
    assert status == sem.SEM_OK
    for i, ((vtx, hexes, N), P, b) in enumerate(zip(batch["meshes"], batch["probs"], batch["rhs"])):
        M = sem.Mesh(vtx, hexes, N)
        x1, info1 = M.solve(bs[i], rtol=1e-10)
        assert abs(infos[i]["iterations"] - info1["iterations"]) <= 1, (i, infos[i], info1)
        xb = xs[i].cpu().numpy()
        M.close()
        if not b.any():
            assert infos[i]["iterations"] == 0 and not xb.any()
            continue
        assert rel_l2(xb, x1.cpu().numpy()) <= 1e-9
        assert np.linalg.norm(b - P.A(xb)) <= 1.05e-10 * np.linalg.norm(b), (i, infos[i])


def test_batch_fp64_tight_matches_oracle(batch):
    """Both sides solved to 1e-13: the unique discrete solution, within 1e-10."""
    B, sem, dev = batch["B"], batch["sem"], batch["dev"]
    bs = [torch.tensor(b, device=dev) for b in batch["rhs"]]
    xs, infos, status = B.solve(bs, rtol=1e-13, max_iter=3000)
    assert status == sem.SEM_OK, infos
    for i, (ut, b) in enumerate(zip(batch["tight"], batch["rhs"])):
        xb = xs[i].cpu().numpy()
        if ut is None:
            assert not xb.any()
            continue
        assert rel_l2(xb, ut) <= 1e-10, (i, infos[i], rel_l2(xb, ut))


def test_batch_ignores_b_on_the_dirichlet_set(batch):
    """b is read as 0 on each instance's Dirichlet set."""
    B, sem, dev = batch["B"], batch["sem"], batch["dev"]
    bs = [torch.tensor(b, device=dev) for b in batch["rhs"]]
    dirty = []
    for P, b in zip(batch["probs"], batch["rhs"]):
        d = b.copy()
        d[P.num.dirichlet.astype(bool)] = 7.0
        dirty.append(torch.tensor(d, device=dev))
    x1, _, _ = B.solve(bs, rtol=1e-10)
    x2, _, _ = B.solve(dirty, rtol=1e-10)
    for a, c in zip(x1, x2):
        assert torch.equal(a, c)


def test_batch_refined(batch):
    B, sem, dev = batch["B"], batch["sem"], batch["dev"]
    bs = [torch.tensor(b, device=dev) for b in batch["rhs"]]
    xs, infos, status = B.solve(bs, mode=sem.SOLVE_FP32_REFINED, rtol=1e-10, inner_rtol=1e-3)
    assert status == sem.SEM_OK
    for i, (P, b) in enumerate(zip(batch["probs"], batch["rhs"])):
        xb = xs[i].cpu().numpy()
        if not b.any():
            assert not xb.any()
            continue
        assert np.linalg.norm(b - P.A(xb)) <= 1.5e-10 * np.linalg.norm(b), (i, infos[i])


def test_batch_repeatable(batch):
    B, dev = batch["B"], batch["dev"]
    bs = [torch.tensor(b, device=dev) for b in batch["rhs"]]
    x1, _, _ = B.solve(bs, rtol=1e-8)
    x2, _, _ = B.solve(bs, rtol=1e-8)
    for a, b in zip(x1, x2):
        assert torch.equal(a, b)
