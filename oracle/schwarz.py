"""Fine-scale overlapping Schwarz preconditioner (Section 4.2, eq. (subd), eq. (z)).

Test infrastructure.  Steps, in the paper's order:

1. Box approximation: every hexahedron is treated as an axis-aligned box of
   sides h_x, h_y, h_z (reading: the mean length of its four edges parallel to
   each reference axis; the neighbour layers use the element's own sizes).
2. 1D element matrices with d_ij = sum_m phi_i'(t_m) phi_j'(t_m) rho_m
   (eq. (subd)), assembled on the pencil extended by one GLL node on each
   side: the neighbouring element (same size) contributes only through its
   two nodes nearest the shared vertex, its further nodes being held at zero
   (the homogeneous Dirichlet points -2 and n+2).  This gives the (n+3)x(n+3)
   stiffness K and diagonal mass M displayed in Section 4.2.
3. The generalised eigenproblem K S = M S Lambda, normalised S^T M S = I
   (equivalent to the paper's L = M^{-1} K = V^{-1} Lambda V with V = S^{-1}).
4. Per subdomain s (an element plus one layer of nodes from its neighbours,
   (n+3)^3 nodes, table I^p):
      r_s = r[I^p]                          (NULL entries give 0)
      z_s = 8/(h_x h_y h_z) (S x S x S) diag(1/(4 kappa (l_a/h_x^2 + l_b/h_y^2
            + l_c/h_z^2) + c)) (S x S x S)^T r_s,
   which is eq. (z) written in symmetric form.
5. Additive accumulation P^f[I^p] += z_s over all subdomains.

I^p reading (the figure defining the stencil is not available): patch node
(i, j, k) with -1 <= i, j, k <= n+1 is the element's own node when all three
indices are in [0, n]; otherwise one steps across the face in the first
out-of-range direction (xi, then eta, then zeta) into the face neighbour,
re-expresses the indices in the neighbour's frame (the unfolding across the
shared face) and repeats.  A missing neighbour, or an edge (corner) node whose
mesh edge is not shared by exactly 4 hexahedra (vertex by 8), gives NULL.

Library primitive used: scipy.linalg.eigh for step 3, numpy.einsum for the 1D
contractions of step 4.

Pinned by: the displayed 1D pattern entry by entry, S^T M S = I and
S^T K S = diag(lambda > 0), the FDM inverse equal to the dense inverse of the
assembled box operator, I^p against coordinate lookup on structured meshes.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from .gll import GLL
from .numbering import FACES, EDGES, Numbering, corner_pos, other_axes

NULL = -1


def stiffness_1d(gll: GLL) -> np.ndarray:
    """d_ij = sum_m phi_i'(t_m) phi_j'(t_m) rho_m (eq. (subd), kappa = 1, h = 2)."""
    D = gll.D  # D[m, i] = phi_i'(t_m)
    return D.T @ np.diag(gll.rho) @ D


def extended_pencil(gll: GLL):
    """(n+3)x(n+3) matrices K and M of Section 4.2 on nodes -1, 0, ..., n+1."""
    n = gll.n
    d = stiffness_1d(gll)
    rho = gll.rho
    m = n + 3
    K = np.zeros((m, m))
    M = np.zeros((m, m))
    # the element itself: nodes 0..n sit at positions 1..n+1
    K[1:n + 2, 1:n + 2] += d
    M[1:n + 2, 1:n + 2] += np.diag(rho)
    # left neighbour: its nodes n-1, n are our nodes -1, 0 (positions 0, 1)
    keep = [n - 1, n]
    K[np.ix_([0, 1], [0, 1])] += d[np.ix_(keep, keep)]
    M[np.ix_([0, 1], [0, 1])] += np.diag(rho[keep])
    # right neighbour: its nodes 0, 1 are our nodes n, n+1 (positions n+1, n+2)
    keep = [0, 1]
    K[np.ix_([n + 1, n + 2], [n + 1, n + 2])] += d[np.ix_(keep, keep)]
    M[np.ix_([n + 1, n + 2], [n + 1, n + 2])] += np.diag(rho[keep])
    return K, M


def fdm_basis(gll: GLL):
    """S, lambda with K S = M S diag(lambda), S^T M S = I."""
    K, M = extended_pencil(gll)
    lam, S = scipy.linalg.eigh(K, M)
    return S, lam


# --- subdomain table I^p ----------------------------------------------------

def _corner_lattice(n):
    """lattice coordinates (i, j, k) of the 8 corners, by tensor position."""
    out = {}
    for c in (0, 1):
        for b in (0, 1):
            for a in (0, 1):
                out[corner_pos(a, b, c)] = np.array([a * n, b * n, c * n])
    return out


def face_neighbours(num: Numbering):
    """nbr[e, lf] = (element, local face) across local face lf, or (-1, -1)."""
    E = num.n_elem
    nbr = np.full((E, 6, 2), -1, dtype=np.int64)
    owners = {}
    for e in range(E):
        for lf in range(6):
            owners.setdefault(int(num.elem_face[e, lf]), []).append((e, lf))
    for lst in owners.values():
        if len(lst) == 2:
            (e0, f0), (e1, f1) = lst
            nbr[e0, f0] = (e1, f1)
            nbr[e1, f1] = (e0, f0)
    return nbr


def face_map(hexes, n, e, lf, e2, lf2):
    """Integer affine map from e's lattice coordinates to e2's, unfolding
    across the shared face: y[perm[d]] = sign[d] * x[d] + off[d]."""
    cl = _corner_lattice(n)
    d, s = FACES[lf]
    d2, s2 = FACES[lf2]
    pos2 = {int(hexes[e2][p]): p for p in range(8)}
    perm = np.zeros(3, dtype=np.int64)
    sign = np.zeros(3, dtype=np.int64)
    off = np.zeros(3, dtype=np.int64)
    # tangential axes: compare two corners of the face that differ along t
    base = [0, 0, 0]
    base[d] = s
    v0 = int(hexes[e][corner_pos(*base)])
    y0 = cl[pos2[v0]]
    for t in other_axes(d):
        c1 = list(base)
        c1[t] = 1
        v1 = int(hexes[e][corner_pos(*c1)])
        y1 = cl[pos2[v1]]
        diff = y1 - y0
        ax = int(np.nonzero(diff)[0][0])
        perm[t] = ax
        sign[t] = diff[ax] // n
        off[t] = y0[ax]
    perm[d] = d2
    sign[d] = -1 if s == s2 else 1
    off[d] = {(0, 0): 0, (0, 1): n, (1, 0): -n, (1, 1): 2 * n}[(s, s2)]
    return perm, sign, off


def _valences(hexes):
    ev = {}
    vv = {}
    for h in hexes:
        for p in range(8):
            vv[int(h[p])] = vv.get(int(h[p]), 0) + 1
        for (d, b1, b2) in EDGES:
            o1, o2 = other_axes(d)
            c0 = [0, 0, 0]
            c0[o1], c0[o2] = b1, b2
            c1 = list(c0)
            c1[d] = 1
            key = tuple(sorted((int(h[corner_pos(*c0)]), int(h[corner_pos(*c1)]))))
            ev[key] = ev.get(key, 0) + 1
    return ev, vv


def patch_table(num: Numbering, hexes, elements=None) -> np.ndarray:
    """I^p[s, c, b, a] for patch indices a, b, c in 0..n+2 (node index = a - 1 etc.)."""
    n = num.n
    hexes = np.asarray(hexes)
    nbr = face_neighbours(num)
    ev, vv = _valences(hexes)
    if elements is None:
        elements = range(num.n_elem)
    elements = list(elements)
    m = n + 3
    out = np.full((len(elements), m, m, m), NULL, dtype=np.int64)
    maps = {}

    def get_map(e, lf):
        key = (e, lf)
        if key not in maps:
            e2, lf2 = nbr[e, lf]
            maps[key] = (int(e2), face_map(hexes, n, e, lf, int(e2), int(lf2)))
        return maps[key]

    for si, s in enumerate(elements):
        for c in range(m):
            for b in range(m):
                for a in range(m):
                    x = np.array([a - 1, b - 1, c - 1])
                    out_axes = [dd for dd in range(3) if x[dd] < 0 or x[dd] > n]
                    if len(out_axes) >= 2:
                        # the mesh edge / vertex that the extension wraps around
                        corner = [0 if x[dd] < 0 else 1 for dd in range(3)]
                        if len(out_axes) == 2:
                            d_free = [dd for dd in range(3) if dd not in out_axes][0]
                            c0 = list(corner)
                            c1 = list(corner)
                            c0[d_free], c1[d_free] = 0, 1
                            key = tuple(sorted((int(hexes[s][corner_pos(*c0)]),
                                                int(hexes[s][corner_pos(*c1)]))))
                            if ev.get(key, 0) != 4:
                                continue
                        else:
                            v = int(hexes[s][corner_pos(*corner)])
                            if vv.get(v, 0) != 8:
                                continue
                            ok = True
                            for dd in range(3):
                                c1 = list(corner)
                                c1[dd] = 1 - c1[dd]
                                key = tuple(sorted((v, int(hexes[s][corner_pos(*c1)]))))
                                if ev.get(key, 0) != 4:
                                    ok = False
                            if not ok:
                                continue
                    e = s
                    valid = True
                    while True:
                        bad = [dd for dd in range(3) if x[dd] < 0 or x[dd] > n]
                        if not bad:
                            break
                        dd = bad[0]
                        lf = 2 * dd + (0 if x[dd] < 0 else 1)
                        if nbr[e, lf, 0] < 0:
                            valid = False
                            break
                        e2, (perm, sign, off) = get_map(e, lf)
                        y = np.zeros(3, dtype=np.int64)
                        for q in range(3):
                            y[perm[q]] = sign[q] * x[q] + off[q]
                        x, e = y, e2
                    if valid:
                        out[si, c, b, a] = num.l2g[e, x[2], x[1], x[0]]
    return out


def element_mean(gll: GLL, v: np.ndarray) -> np.ndarray:
    """One value per element of a coefficient given at the nodes v[e, k, j, i].

    Reading: a patch solve (eq. (z)) and an order-1 coarse element (eq. (coarse))
    use one kappa and one c; for a coefficient known per node they take its mean
    over the reference cube by the GLL rule, (1/8) sum rho_i rho_j rho_k v_{ijk;e}."""
    r = gll.rho
    return np.einsum("ekji,k,j,i->e", v, r, r, r) / 8.0


def fdm_patch_solve(S, lam, r_s, h, kappa=1.0, c=0.0):
    """eq. (z) for patches r_s[s, c, b, a] with box sizes h[s, 3] (step 4);
    kappa and c are constants or one value per patch."""
    t = np.einsum("xa,...cbx->...cba", S, r_s)
    t = np.einsum("xb,...cxa->...cba", S, t)
    t = np.einsum("xc,...xba->...cba", S, t)
    hx, hy, hz = h[..., 0], h[..., 1], h[..., 2]
    kappa = np.asarray(kappa, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    if kappa.ndim:
        kappa = kappa[:, None, None, None]
    if c.ndim:
        c = c[:, None, None, None]
    diag = (4.0 * kappa * (lam[None, None, None, :] / hx[:, None, None, None] ** 2
                           + lam[None, None, :, None] / hy[:, None, None, None] ** 2
                           + lam[None, :, None, None] / hz[:, None, None, None] ** 2)
            + c)
    t = t / diag
    t = np.einsum("ax,...cbx->...cba", S, t)
    t = np.einsum("bx,...cxa->...cba", S, t)
    t = np.einsum("cx,...xba->...cba", S, t)
    return t * (8.0 / (hx * hy * hz))[:, None, None, None]


class FinePreconditioner:
    def __init__(self, num: Numbering, hexes, vtx, gll: GLL, box, kappa=1.0, c=0.0):
        self.num = num
        self.n = gll.n
        self.S, self.lam = fdm_basis(gll)
        self.box = box  # [E, 3]
        self.kappa = kappa
        self.c = c
        self.Ip = patch_table(num, hexes)

    def patch_solve(self, r_s: np.ndarray, h) -> np.ndarray:
        """eq. (z) for one or more patches r_s[..., c, b, a] with sizes h[..., 3]."""
        return fdm_patch_solve(self.S, self.lam, r_s, h, self.kappa, self.c)

    def apply(self, r: np.ndarray) -> np.ndarray:
        Ip = self.Ip
        valid = Ip >= 0
        r_s = np.where(valid, r[np.where(valid, Ip, 0)], 0.0)
        z_s = self.patch_solve(r_s, self.box)
        z = np.zeros(self.num.n_global)
        np.add.at(z, Ip[valid], z_s[valid])
        return z
