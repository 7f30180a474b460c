"""Pins of the oracle's canonical global numbering (Section 2.2)."""
import os

import numpy as np
import pytest

import meshgen
from oracle.geometry import node_coords_local
from oracle.gll import GLL
from oracle.numbering import gather, number_mesh, scatter

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def lattice_count(k, n):
    return (k * n + 1) ** 3


def test_paper_dof_counts():
    """Counts printed in Tables 1-2 follow from (kn+1)^3; the oracle's
    numbering reproduces (kn+1)^3 on the meshes it can afford."""
    rows = []
    with open(os.path.join(GOLDEN, "dof_counts.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                k, n, printed = line.split()[:3]
                rows.append((int(k), int(n), float(printed)))
    for k, n, printed in rows:
        exact = lattice_count(k, n)
        # the tables truncate to two significant digits (15625 is printed 1.5e4)
        e10 = 10 ** (len(str(exact)) - 2)
        assert (exact // e10) * e10 == round(printed), (k, n, exact, printed)
    for k in (1, 2, 3, 4):
        for n in (1, 2, 3, 5):
            num = number_mesh(meshgen.cube_mesh(k).hex, n)
            assert num.n_global == lattice_count(k, n)
            V, Ed, F, E = num.n_vertices, num.n_edges, num.n_faces, num.n_elem
            assert V == (k + 1) ** 3 and E == k ** 3
            assert Ed == 3 * k * (k + 1) ** 2 and F == 3 * k * k * (k + 1)
            assert num.n_global == V + Ed * (n - 1) + F * (n - 1) ** 2 + E * (n - 1) ** 3


@pytest.mark.parametrize("k,n", [(2, 3), (3, 4), (2, 5)])
def test_numbering_matches_coordinates(k, n):
    """Brute force: on an unperturbed mesh, two local nodes share a global id
    exactly when they sit at the same physical point."""
    mesh = meshgen.cube_mesh(k)
    mesh, _ = meshgen.rotate_elements(mesh)
    mesh, _ = meshgen.permute_elements(mesh)
    num = number_mesh(mesh.hex, n)
    x = node_coords_local(mesh.vtx, mesh.hex, GLL(n)).reshape(-1, 3)
    key = np.round(x * 1e9).astype(np.int64)
    _, cls = np.unique(key, axis=0, return_inverse=True)
    g = num.l2g.reshape(-1)
    # same partition of local nodes
    pairs = np.unique(np.stack([cls.ravel(), g], axis=1), axis=0)
    assert len(pairs) == cls.max() + 1 == g.max() + 1 == num.n_global


def test_numbering_classes_and_layout():
    n = 4
    mesh = meshgen.cube_mesh(3, perturb=0.1)
    num = number_mesh(mesh.hex, n)
    l2g = num.l2g
    V, Ed, F = num.n_vertices, num.n_edges, num.n_faces
    base_i = V + Ed * (n - 1) + F * (n - 1) ** 2
    # corner nodes are the vertex ids in ascending mesh-vertex order
    assert (l2g[:, ::n, ::n, ::n].reshape(-1, 8) == np.searchsorted(num.vertex_ids, mesh.hex)).all()
    # interiors: contiguous per element, i fastest
    inner = l2g[:, 1:n, 1:n, 1:n].reshape(num.n_elem, -1)
    m = (n - 1) ** 3
    assert (inner == base_i + np.arange(num.n_elem)[:, None] * m + np.arange(m)[None, :]).all()
    # each edge's n-1 ids count from its smaller vertex id
    e = 0
    i_edge = l2g[e, 0, 0, 1:n]  # xi-edge at eta = zeta = 0
    va, vb = mesh.hex[e, 0], mesh.hex[e, 1]
    if va < vb:
        assert (np.diff(i_edge) == 1).all()
    else:
        assert (np.diff(i_edge) == -1).all()


def test_numbering_invariant_under_permutation_and_rotation():
    """Vertex, edge and face ids depend only on vertex ids; interior ids move
    with their element.  Compared through node coordinates."""
    n = 3
    base = meshgen.cube_mesh(3, perturb=0.1)
    moved, _ = meshgen.rotate_elements(base, seed=5)
    moved, perm = meshgen.permute_elements(moved, seed=6)
    g = GLL(n)
    num0 = number_mesh(base.hex, n)
    num1 = number_mesh(moved.hex, n)
    x0 = node_coords_local(base.vtx, base.hex, g).reshape(-1, 3)
    x1 = node_coords_local(moved.vtx, moved.hex, g).reshape(-1, 3)
    k0 = {tuple(np.round(x * 1e9).astype(np.int64)): int(i) for x, i in zip(x0, num0.l2g.ravel())}
    base_i = num0.n_vertices + num0.n_edges * (n - 1) + num0.n_faces * (n - 1) ** 2
    for x, i in zip(x1, num1.l2g.ravel()):
        j = k0[tuple(np.round(x * 1e9).astype(np.int64))]
        if j < base_i:
            assert i == j
        else:
            assert i >= base_i
            # interior node: same element, block moved by the permutation
            e1 = (i - base_i) // (n - 1) ** 3
            e0 = (j - base_i) // (n - 1) ** 3
            assert perm[e1] == e0


def test_gather_csr_and_scatter_gather():
    n = 3
    mesh = meshgen.cube_mesh(2, perturb=0.1)
    num = number_mesh(mesh.hex, n)
    offs, idx = num.gather_csr()
    flat = num.l2g.reshape(-1)
    for gid in range(0, num.n_global, 7):
        lst = idx[offs[gid]:offs[gid + 1]]
        assert (flat[lst] == gid).all()
        assert (np.diff(lst) > 0).all()
    # multiplicities: vertex nodes at the cube centre are shared by 8 elements
    counts = np.diff(offs)
    assert counts.max() == 8 and counts.min() == 1
    rng = np.random.default_rng(0)
    u = rng.standard_normal(num.n_global)
    ones = np.ones_like(scatter(num, u))
    assert np.allclose(gather(num, ones), counts)
    # gather is the transpose of scatter: <Q u, v>_local == <u, Q^T v>
    v = rng.standard_normal(ones.shape)
    assert abs((scatter(num, u) * v).sum() - u @ gather(num, v)) < 1e-10


def test_dirichlet_set_is_topological_boundary():
    n = 3
    mesh = meshgen.cube_mesh(3, perturb=0.1)
    num = number_mesh(mesh.hex, n)
    x = node_coords_local(mesh.vtx, mesh.hex, GLL(n))
    xg = np.zeros((num.n_global, 3))
    xg[num.l2g.reshape(-1)] = x.reshape(-1, 3)
    on_box = (np.isclose(xg, 0.0, atol=1e-12) | np.isclose(xg, 1.0, atol=1e-12)).any(axis=1)
    assert (num.dirichlet.astype(bool) == on_box).all()
    assert num.dirichlet.sum() == (3 * n + 1) ** 3 - (3 * n - 1) ** 3


def test_rejects_nonmanifold_face():
    mesh = meshgen.cube_mesh(1)
    h = np.concatenate([mesh.hex, mesh.hex, mesh.hex])
    with pytest.raises(ValueError):
        number_mesh(h, 2)
