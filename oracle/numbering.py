"""Local and global GLL node tables (Section 2.2, eq. (scatter), eq. (gather)).

Test infrastructure.  The paper only requires that every GLL node of the mesh
get one unique global number (Section 2.2); a canonical rule is fixed here so
that two independent implementations can be compared bit for bit:

* local node (i, j, k) of element e has local index
  ``e (n+1)^3 + i + (n+1) j + (n+1)^2 k``;
* a local node is a vertex node if three of i, j, k are in {0, n}, an edge node
  if two are, a face node if one is, interior otherwise;
* global ids are handed out class by class: the referenced mesh vertices in
  ascending vertex id; then edges (key = sorted vertex pair, sorted
  lexicographically), n-1 ids per edge counted from the smaller vertex id;
  then faces (key = sorted 4 vertex ids, sorted lexicographically), (n-1)^2
  ids per face in the face frame whose origin w0 is the face's smallest
  vertex id, with p running towards the smaller-id of w0's two face-adjacent
  corners and q towards the other, id = (q-1)(n-1) + (p-1); finally the element
  interiors, (n-1)^3 ids per element in element order, i fastest.

The gather table I_{g->l} lists the local copies of each global node in
ascending local index (eq. (gather)); it fixes the summation order.  The
default Dirichlet set is every node on a face that belongs to one hexahedron
only (the topological boundary).

Pinned by: node counts against (kn+1)^3 for k^3 cubes and the closed-form
class count; brute-force node identification through physical coordinates on
unperturbed meshes; invariance under element permutation and local rotation.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

# local faces: (axis, side); corners of a face listed by in-face coordinates
FACES = [(0, 0), (0, 1), (1, 0), (1, 1), (2, 0), (2, 1)]
# local edges: (axis, bit of first other axis, bit of second other axis)
EDGES = [(d, b1, b2) for d in range(3) for b2 in (0, 1) for b1 in (0, 1)]


def corner_pos(a, b, c):
    return a + 2 * b + 4 * c


def other_axes(d):
    return [x for x in range(3) if x != d]


@dataclass
class Numbering:
    n: int
    n_elem: int
    l2g: np.ndarray  # [E, n+1, n+1, n+1] indexed [e, k, j, i], int64
    n_global: int
    n_vertices: int
    n_edges: int
    n_faces: int
    vertex_ids: np.ndarray  # referenced mesh vertex ids, ascending (global id = position)
    face_keys: np.ndarray  # [F, 4]
    face_count: np.ndarray  # [F] number of hexes sharing each face
    elem_face: np.ndarray  # [E, 6] face rank of each local face
    edge_keys: np.ndarray  # [Ed, 2]
    dirichlet: np.ndarray  # [n_global] uint8, 1 on the topological boundary

    @property
    def l2g_flat(self):
        return self.l2g.reshape(self.n_elem, -1)

    def gather_csr(self):
        """I_{g->l} as CSR: offsets [n_global+1] and ascending local indices."""
        flat = self.l2g.reshape(-1)
        order = np.argsort(flat, kind="stable")
        counts = np.bincount(flat, minlength=self.n_global)
        offsets = np.zeros(self.n_global + 1, dtype=np.int64)
        np.cumsum(counts, out=offsets[1:])
        return offsets, order.astype(np.int64)


def number_mesh(hexes: np.ndarray, n: int) -> Numbering:
    """Canonical global numbering of the order-n GLL nodes of a hex mesh."""
    hexes = np.asarray(hexes, dtype=np.int64)
    E = hexes.shape[0]
    n1 = n + 1
    l2g = np.full((E, n1, n1, n1), -1, dtype=np.int64)
    ar = np.arange(E)

    def put(e_idx, i, j, k, vals):
        l2g[e_idx, k, j, i] = vals

    # --- vertices
    vertex_ids = np.unique(hexes)
    vrank = {int(v): r for r, v in enumerate(vertex_ids)}
    n_vert = len(vertex_ids)
    vr = np.searchsorted(vertex_ids, hexes)  # [E, 8] global id of each corner
    for c in (0, 1):
        for b in (0, 1):
            for a in (0, 1):
                put(ar, a * n, b * n, c * n, vr[:, corner_pos(a, b, c)])
    del vrank

    # --- edges
    inner = np.arange(1, n)  # positions along an edge / face axis
    edge_va = np.empty((E, 12), dtype=np.int64)
    edge_vb = np.empty((E, 12), dtype=np.int64)
    for le, (d, b1, b2) in enumerate(EDGES):
        o1, o2 = other_axes(d)
        c0 = [0, 0, 0]
        c0[o1], c0[o2] = b1, b2
        c1 = list(c0)
        c1[d] = 1
        edge_va[:, le] = hexes[:, corner_pos(*c0)]
        edge_vb[:, le] = hexes[:, corner_pos(*c1)]
    emin = np.minimum(edge_va, edge_vb)
    emax = np.maximum(edge_va, edge_vb)
    ekeys = np.stack([emin.ravel(), emax.ravel()], axis=1)
    edge_keys, edge_rank = np.unique(ekeys, axis=0, return_inverse=True)
    edge_rank = edge_rank.reshape(E, 12)
    n_edges = edge_keys.shape[0]
    base_e = n_vert
    if n >= 2:
        for le, (d, b1, b2) in enumerate(EDGES):
            o1, o2 = other_axes(d)
            forward = edge_va[:, le] < edge_vb[:, le]  # local direction runs min -> max
            q = np.where(forward[:, None], inner[None, :], n - inner[None, :])  # [E, n-1]
            ids = base_e + edge_rank[:, le][:, None] * (n - 1) + (q - 1)
            idx = [None, None, None]
            idx[d] = inner[None, :]
            idx[o1] = b1 * n
            idx[o2] = b2 * n
            put(ar[:, None], idx[0], idx[1], idx[2], ids)

    # --- faces
    fverts = np.empty((E, 6, 2, 2), dtype=np.int64)  # [e, face, s2, s1] vertex ids
    for lf, (d, s) in enumerate(FACES):
        t1, t2 = other_axes(d)
        for s2 in (0, 1):
            for s1 in (0, 1):
                c = [0, 0, 0]
                c[d], c[t1], c[t2] = s, s1, s2
                fverts[:, lf, s2, s1] = hexes[:, corner_pos(*c)]
    fkeys = np.sort(fverts.reshape(E * 6, 4), axis=1)
    face_keys, face_rank, face_count = np.unique(fkeys, axis=0, return_inverse=True,
                                                 return_counts=True)
    face_rank = face_rank.reshape(E, 6)
    if face_count.max() > 2:
        raise ValueError("a face is shared by more than two hexahedra")
    n_faces = face_keys.shape[0]
    base_f = n_vert + n_edges * (n - 1)
    if n >= 2:
        x1 = inner[None, :, None]  # along t1
        x2 = inner[None, None, :]  # along t2
        for lf, (d, s) in enumerate(FACES):
            t1, t2 = other_axes(d)
            fv = fverts[:, lf]  # [E, 2(s2), 2(s1)]
            flat = fv.reshape(E, 4)  # index s1 + 2 s2
            w0pos = np.argmin(flat, axis=1)
            s1_0 = w0pos % 2
            s2_0 = w0pos // 2
            nb_t1 = flat[ar, (1 - s1_0) + 2 * s2_0]  # neighbour of w0 along t1
            nb_t2 = flat[ar, s1_0 + 2 * (1 - s2_0)]  # neighbour of w0 along t2
            p_along_t1 = (nb_t1 < nb_t2)[:, None, None]
            d1 = np.abs(x1 - (s1_0 * n)[:, None, None])  # [E, n-1, 1]
            d2 = np.abs(x2 - (s2_0 * n)[:, None, None])  # [E, 1, n-1]
            p = np.where(p_along_t1, d1, d2)
            q = np.where(p_along_t1, d2, d1)
            ids = base_f + face_rank[:, lf][:, None, None] * (n - 1) ** 2 + (q - 1) * (n - 1) + (p - 1)
            idx = [None, None, None]
            idx[d] = s * n
            idx[t1] = x1
            idx[t2] = x2
            put(ar[:, None, None], idx[0], idx[1], idx[2], ids)

    # --- interiors
    base_i = base_f + n_faces * (n - 1) ** 2
    if n >= 2:
        m = n - 1
        kk, jj, ii = np.meshgrid(inner, inner, inner, indexing="ij")
        loc = (ii - 1) + m * (jj - 1) + m * m * (kk - 1)
        l2g[:, 1:n, 1:n, 1:n] = base_i + ar[:, None, None, None] * m ** 3 + loc[None]
    n_global = base_i + E * (n - 1) ** 3
    assert (l2g >= 0).all()

    # --- default Dirichlet set: all nodes of faces owned by a single hexahedron
    dirichlet = np.zeros(n_global, dtype=np.uint8)
    for lf, (d, s) in enumerate(FACES):
        on_bnd = face_count[face_rank[:, lf]] == 1
        if not on_bnd.any():
            continue
        sl = [slice(None)] * 3
        sl[2 - d] = s * n  # array axes are (k, j, i)
        nodes = l2g[on_bnd][(slice(None),) + tuple(sl)]
        dirichlet[nodes.ravel()] = 1

    return Numbering(n=n, n_elem=E, l2g=l2g, n_global=int(n_global), n_vertices=n_vert,
                     n_edges=int(n_edges), n_faces=int(n_faces), vertex_ids=vertex_ids,
                     face_keys=face_keys, face_count=face_count, elem_face=face_rank,
                     edge_keys=edge_keys, dirichlet=dirichlet)


def scatter(num: Numbering, u_global: np.ndarray) -> np.ndarray:
    """eq. (scatter): local copy u_{ijk;e} = u_{I(ijk;e)}; shape [E, k, j, i]."""
    return u_global[num.l2g]


def gather(num: Numbering, r_local: np.ndarray) -> np.ndarray:
    """eq. (gather): r_N = sum over the local copies of N, taken in ascending
    local index order (explicit loop over the gather table)."""
    offsets, idx = num.gather_csr()
    flat = r_local.reshape(-1)
    vals = flat[idx]
    out = np.zeros(num.n_global)
    # sequential accumulation per global node in list order
    counts = np.diff(offsets)
    maxc = counts.max() if counts.size else 0
    for c in range(maxc):
        has = counts > c
        out[has] += vals[offsets[:-1][has] + c]
    return out
