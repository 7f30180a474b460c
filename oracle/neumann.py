"""Neumann boundary data (eq. (pde), eq. (pdeweak)) -- test infrastructure.

With du/dn = g on part of the boundary, the weak form gains the surface term
int_{Gamma_N} kappa g w dS on the right-hand side.  With the GLL rule on each
boundary face (the face's (n+1)^2 nodes, weights rho_a rho_b) it becomes
kappa_e g_N ws_N, where the lumped surface mass ws_N sums, over the listed
faces that hold node N, rho_a rho_b |dx/da x dx/db| (the surface Jacobian of
the trilinear map restricted to the face, a and b the face's two reference
axes in increasing order).

Library primitive used: numpy.cross.

Pinned by: the faces of a box (planar, their vertices unperturbed) sum to their
area exactly; a manufactured solution with Dirichlet and Neumann parts of the
boundary converges spectrally.
"""
from __future__ import annotations

import numpy as np

from .geometry import jacobian
from .gll import GLL
from .numbering import FACES, Numbering, other_axes


def face_mass(num: Numbering, vtx, hexes, gll: GLL, faces) -> np.ndarray:
    """ws[n_global] for faces = [(element, local face 0..5), ...] (local face
    2 axis + side: xi-, xi+, eta-, eta+, zeta-, zeta+)."""
    n = gll.n
    rho = gll.rho
    ws = np.zeros(num.n_global)
    faces = np.asarray(faces, dtype=np.int64).reshape(-1, 2)
    if faces.size == 0:
        return ws
    J = jacobian(vtx, np.asarray(hexes)[faces[:, 0]], gll)  # [F, k, j, i, 3, 3]
    for f, (e, lf) in enumerate(faces):
        d, side = FACES[lf]
        a, b = other_axes(d)
        sl = [slice(None)] * 3
        sl[2 - d] = side * n  # array axes are (k, j, i)
        Jf = J[f][tuple(sl)]  # [(n+1), (n+1), 3, 3] over the two remaining array axes
        gids = num.l2g[e][tuple(sl)]
        t1 = Jf[..., :, a]
        t2 = Jf[..., :, b]
        area = np.linalg.norm(np.cross(t1, t2), axis=-1)
        # remaining array axes are in decreasing reference-axis order: (b, a)
        w = area * rho[:, None] * rho[None, :]
        np.add.at(ws, gids.ravel(), w.ravel())
    return ws
