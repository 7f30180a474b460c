"""Parity at the full workload sizes, in the launch configuration bench.py
times: 56^3 hexes at N = 7 (60.7 M DOFs) and 20^3 hexes stretched 8:1 at
N = 15 (27.3 M DOFs).

Integer tables are compared whole and bit for bit; the operator and the fine
preconditioner at sampled global nodes, each computed by the oracle from the
elements / patches that touch it; the coarse solve through its residual with
the oracle's own coarse matrix; the solves through properties that hold at any
size (true FP64 residual with the parity-checked operator, nodal error
against the exact solution).
"""
import numpy as np
import pytest

import meshgen
from oracle.coarse import coarse_matrix
from oracle.geometry import Geometry, box_sizes
from oracle.gll import GLL
from oracle.numbering import number_mesh
from oracle.operator import element_action
from oracle.schwarz import fdm_basis, fdm_patch_solve, patch_table

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

WORKLOADS = ["cube56_N7", "box20x8_N15"]


def log(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module", params=WORKLOADS)
def big(request):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1506_05996_amd import sem
    name = request.param
    log(f"[fullsize] {name}: set-up")
    mesh, N = meshgen.workload_mesh(name)
    M = sem.Mesh(mesh.vtx, mesh.hex, N)
    log(f"[fullsize] {name}: oracle numbering")
    num = number_mesh(mesh.hex, N)
    yield dict(name=name, mesh=mesh, N=N, M=M, num=num, dev=torch.device("cuda:0"), sem=sem)
    M.close()
    torch.cuda.empty_cache()


def test_numbering_and_mask_bit_exact(big):
    M, num = big["M"], big["num"]
    assert M.n_global == num.n_global
    assert (M.numbering().astype(np.int64) == num.l2g).all()
    assert (M.boundary_mask() == num.dirichlet).all()


def _incident(num, nodes):
    offs, idx = num.gather_csr()
    n1 = num.n + 1
    lists = [idx[offs[g]:offs[g + 1]] for g in nodes]
    elems = np.unique(np.concatenate(lists) // n1 ** 3)
    return lists, elems


def test_apply_A_sampled(big):
    M, num, mesh, N, dev = big["M"], big["num"], big["mesh"], big["N"], big["dev"]
    rng = np.random.default_rng(1506)
    u = rng.uniform(-1, 1, num.n_global)
    y = M.apply_A(torch.tensor(u, device=dev)).cpu().numpy()
    # shared nodes are where assembly happens: sample both kinds
    n_shared = num.n_vertices + num.n_edges * (N - 1) + num.n_faces * (N - 1) ** 2
    nodes = np.unique(np.concatenate([rng.integers(0, n_shared, 300), rng.integers(n_shared, num.n_global, 100)]))
    lists, elems = _incident(num, nodes)
    g = GLL(N)
    geo = Geometry(mesh.vtx, mesh.hex[elems], g)
    r = element_action(u[num.l2g[elems]], geo.G, g.D).reshape(len(elems), -1)
    pos = {int(e): p for p, e in enumerate(elems)}
    n3 = (N + 1) ** 3
    ref = np.zeros(len(nodes))
    for q, (gid, lst) in enumerate(zip(nodes, lists)):
        s = 0.0
        for loc in lst:  # ascending local index
            s += r[pos[int(loc // n3)], int(loc % n3)]
        ref[q] = 0.0 if num.dirichlet[gid] else s
    got = y[nodes]
    assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)


def test_fine_precond_sampled(big):
    M, num, mesh, N, dev = big["M"], big["num"], big["mesh"], big["N"], big["dev"]
    rng = np.random.default_rng(1507)
    r = rng.uniform(-1, 1, num.n_global)
    r[num.dirichlet.astype(bool)] = 0.0
    z = M.precond(torch.tensor(r, device=dev), pc=1).cpu().numpy()
    nodes = np.unique(rng.integers(0, num.n_global, 12))
    lists, elems = _incident(num, nodes)
    # every patch that can hold one of these nodes belongs to an element that
    # shares a vertex with an element holding it
    verts = np.unique(mesh.hex[elems])
    cand = np.nonzero(np.isin(mesh.hex, verts).any(axis=1))[0]
    log(f"[fullsize] {len(cand)} candidate patches")
    Ip = patch_table(num, mesh.hex, elements=cand)
    g = GLL(N)
    S, lam = fdm_basis(g)
    valid = Ip >= 0
    r_s = np.where(valid, r[np.where(valid, Ip, 0)], 0.0)
    z_s = fdm_patch_solve(S, lam, r_s, box_sizes(mesh.vtx, mesh.hex[cand]))
    ref = np.zeros(len(nodes))
    flatI = Ip.reshape(-1)
    flatz = z_s.reshape(-1)
    for q, gid in enumerate(nodes):
        hits = np.nonzero(flatI == gid)[0]  # ascending slot order
        s = 0.0
        for h in hits:
            s += flatz[h]
        ref[q] = 0.0 if num.dirichlet[gid] else s
    assert np.linalg.norm(z[nodes] - ref) <= 1e-12 * max(np.linalg.norm(ref), 1e-300)


def test_coarse_solve_residual(big):
    M, num, mesh, dev = big["M"], big["num"], big["mesh"], big["dev"]
    nv = num.n_vertices
    Ac = coarse_matrix(mesh.vtx, mesh.hex, nv)
    free = np.nonzero(num.dirichlet[:nv] == 0)[0]
    R = np.random.default_rng(1508).uniform(-1, 1, nv)
    Z = M.coarse_solve(torch.tensor(R, device=dev)).cpu().numpy()
    assert np.abs(Z[num.dirichlet[:nv].astype(bool)]).max() == 0.0
    res = Ac[free][:, free] @ Z[free] - R[free]
    assert np.linalg.norm(res) <= 1e-10 * np.linalg.norm(R[free])


@pytest.mark.parametrize("mode", [0, 1])
def test_pcg_to_1e10(big, mode):
    M, mesh, dev, sem = big["M"], big["mesh"], big["dev"], big["sem"]
    lengths = mesh.lengths
    x_n = M.node_coords()
    m_n = M.lumped_mass()
    mask = M.boundary_mask().astype(bool)
    b = m_n * meshgen.manufactured_s(x_n, lengths)
    b[mask] = 0.0
    ue = meshgen.manufactured_u(x_n, lengths)
    ue[mask] = 0.0
    del x_n
    bd = torch.tensor(b, device=dev)
    x, info = M.solve(bd, mode=mode, rtol=1e-10, max_iter=3000, inner_rtol=1e-2, max_outer=60)
    log(f"[fullsize] {big['name']} mode {mode}: {info}")
    res = float(torch.linalg.vector_norm(bd - M.apply_A(x)) / torch.linalg.vector_norm(bd))
    assert res <= 1.2e-10
    err = np.abs(x.cpu().numpy() - ue).max()
    # spectral accuracy at these orders and mesh sizes is far below this bound
    assert err <= 1e-8, err
