"""Element geometry at GLL nodes (Sections 2.3 and 2.4).

Test infrastructure.  Each hexahedron is the trilinear image of the reference
cube [-1,1]^3 through its 8 vertices (tensor order a + 2b + 4c, coarse shape
functions Phi_0 = (1-t)/2, Phi_1 = (1+t)/2).  At every GLL node:

* J is the 3x3 Jacobian d(x,y,z)/d(xi,eta,zeta), |J| its determinant;
* m_{ijk;e} = rho_i rho_j rho_k |J| (the integration weight of Section 2.4);
* the six stiffness factors G^1..G^6 of eq. (R) are the entries
  (xx, xy, xz, yy, yz, zz) of m_{ijk;e} (J^T J)^{-1}.  The paper names the
  metric tensor J^T J in Section 2.3, but the stiffness form of Section 2.4
  needs the weighted inverse metric, and its kernel-traffic count of seven
  geometric factors (six G plus the weighted mass) fits that reading.

Pinned by: sum of the lumped mass = domain volume, closed-form G on affine
elements, and (through the operator pins) polynomial exactness.  The box
sizes of the patch solves are pinned on an axis-aligned box with a different
h along each axis, with and without random element rotations: each size equals
the extent along the physical axis its reference axis points to, and the box
operator built from them equals the assembled operator on an interior patch
(sizes taken from the wrong edges fail both).
"""
from __future__ import annotations

import numpy as np

from .gll import GLL
from .numbering import Numbering


def corner_coords(vtx: np.ndarray, hexes: np.ndarray) -> np.ndarray:
    """[E, 2(c), 2(b), 2(a), 3] vertex coordinates of each hexahedron."""
    X = vtx[np.asarray(hexes)]  # [E, 8, 3], position a + 2b + 4c
    return X.reshape(-1, 2, 2, 2, 3)


def node_coords_local(vtx, hexes, gll: GLL) -> np.ndarray:
    """Physical coordinates of every local GLL node, [E, k, j, i, 3]."""
    X = corner_coords(vtx, hexes)
    t = gll.t
    P = np.stack([(1 - t) / 2, (1 + t) / 2], axis=1)  # [n+1, 2]
    return np.einsum("ecbax,ia,jb,kc->ekjix", X, P, P, P)


def jacobian(vtx, hexes, gll: GLL) -> np.ndarray:
    """J[e, k, j, i, row, col] with rows x,y,z and columns d/dxi, d/deta, d/dzeta."""
    X = corner_coords(vtx, hexes)
    t = gll.t
    n1 = len(t)
    P = np.stack([(1 - t) / 2, (1 + t) / 2], axis=1)
    dP = np.array([-0.5, 0.5])
    E = X.shape[0]
    J = np.empty((E, n1, n1, n1, 3, 3))
    dxi = np.einsum("ecbax,a,jb,kc->ekjx", X, dP, P, P)
    deta = np.einsum("ecbax,ia,b,kc->ekix", X, P, dP, P)
    dzeta = np.einsum("ecbax,ia,jb,c->ejix", X, P, P, dP)
    J[..., :, 0] = dxi[:, :, :, None, :]
    J[..., :, 1] = deta[:, :, None, :, :]
    J[..., :, 2] = dzeta[:, None, :, :, :]
    return J


class Geometry:
    """Per-node geometric data of an order-n mesh."""

    def __init__(self, vtx, hexes, gll: GLL):
        J = jacobian(vtx, hexes, gll)
        self.detJ = np.linalg.det(J)
        if (self.detJ <= 0).any():
            raise ValueError("inverted or degenerate hexahedron (|J| <= 0 at a GLL node)")
        rho = gll.rho
        w = rho[None, :, None, None] * rho[None, None, :, None] * rho[None, None, None, :]
        # array axes (k, j, i): weight rho_k rho_j rho_i
        self.mass = w * self.detJ  # m_{ijk;e}
        JtJ = np.einsum("...ri,...rj->...ij", J, J)
        Ginv = np.linalg.inv(JtJ)
        self.Gfull = self.mass[..., None, None] * Ginv  # [E,k,j,i,3,3]
        g = self.Gfull
        # G^1..G^6 = (xi xi, xi eta, xi zeta, eta eta, eta zeta, zeta zeta)
        self.G = np.stack([g[..., 0, 0], g[..., 0, 1], g[..., 0, 2],
                           g[..., 1, 1], g[..., 1, 2], g[..., 2, 2]], axis=0)  # [6,E,k,j,i]
        self.x_local = node_coords_local(vtx, hexes, gll)


def lumped_mass(num: Numbering, geo: Geometry) -> np.ndarray:
    """m_N: sum of m_{ijk;e} over the local copies of N (Section 4.1)."""
    out = np.zeros(num.n_global)
    np.add.at(out, num.l2g.reshape(-1), geo.mass.reshape(-1))
    return out


def node_coords_global(num: Numbering, geo: Geometry) -> np.ndarray:
    """x_N taken from the first local copy of each global node."""
    offsets, idx = num.gather_csr()
    first = idx[offsets[:-1]]
    return geo.x_local.reshape(-1, 3)[first]


def box_sizes(vtx, hexes) -> np.ndarray:
    """h_x, h_y, h_z of each hexahedron: the mean length of its four edges
    parallel to the reference axis xi, eta, zeta (the box approximation of
    Section 4.2)."""
    X = corner_coords(vtx, hexes)  # [E, c, b, a, 3]
    hx = np.linalg.norm(X[:, :, :, 1] - X[:, :, :, 0], axis=-1).mean(axis=(1, 2))
    hy = np.linalg.norm(X[:, :, 1, :] - X[:, :, 0, :], axis=-1).mean(axis=(1, 2))
    hz = np.linalg.norm(X[:, 1, :, :] - X[:, 0, :, :], axis=-1).mean(axis=(1, 2))
    return np.stack([hx, hy, hz], axis=1)
