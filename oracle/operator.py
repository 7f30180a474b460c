"""Matrix-free stiffness action (Section 2.4, eq. (R), eq. (ABC); Algorithm 2).

Test infrastructure.  For each element, in this order:

1. scatter: u_{ijk;e} = u_{I(ijk;e)}                           (eq. (scatter))
2. reference derivatives
   du/dxi|_{ijk}   = sum_m D_{im} u_{mjk},
   du/deta|_{ijk}  = sum_m D_{jm} u_{imk},
   du/dzeta|_{ijk} = sum_m D_{km} u_{ijm};
3. A, B, C = G . (du/dxi, du/deta, du/dzeta) with the symmetric packing
   G^1..G^6 (eq. (ABC)); with kappa given at every node (eq. (R) weights each
   quadrature point by its own kappa_{ijk;e}) A, B, C are multiplied by it;
4. r_{ijk;e} = kappa_e sum_m [D_{mi} A_{mjk} + D_{mj} B_{imk} + D_{mk} C_{ijm}]
   + c_e m_{ijk;e} u_{ijk;e}                                       (Algorithm 2),
   kappa_e = 1 when kappa is per node, and c_{ijk;e} in place of c_e when c is
   per node;
5. gather r_N = sum of the local copies (eq. (gather)), then zero the
   Dirichlet nodes (the homogeneous Dirichlet condition u_0 = 0 of Section 2).

Library primitive used: numpy.einsum for each 1D contraction (no fusion).

Pinned by: equality with the dense brute-force assembly (oracle.brute);
symmetry, A 1 = 0 without the mask, SPD with it; exact -Laplace(u) for
polynomials of degree <= n on affine meshes; the linear patch test on
trilinear meshes.
"""
from __future__ import annotations

import numpy as np

from .geometry import Geometry
from .gll import GLL
from .numbering import Numbering, gather


def element_action(U: np.ndarray, G: np.ndarray, D: np.ndarray, kappa=None, c=None,
                   mass=None) -> np.ndarray:
    """Local residual r_{ijk;e} for local values U[e, k, j, i] (steps 2-4).

    kappa and c: None, one value per element [E], or one per node [E, k, j, i]."""
    kap = None if kappa is None else np.asarray(kappa)
    ur = np.einsum("im,ekjm->ekji", D, U)
    us = np.einsum("jm,ekmi->ekji", D, U)
    ut = np.einsum("km,emji->ekji", D, U)
    G1, G2, G3, G4, G5, G6 = G
    A = G1 * ur + G2 * us + G3 * ut
    B = G2 * ur + G4 * us + G5 * ut
    C = G3 * ur + G5 * us + G6 * ut
    if kap is not None and kap.ndim == 4:
        A, B, C = kap * A, kap * B, kap * C
    r = (np.einsum("mi,ekjm->ekji", D, A)
         + np.einsum("mj,ekmi->ekji", D, B)
         + np.einsum("mk,emji->ekji", D, C))
    if kap is not None and kap.ndim == 1:
        r = r * kap[:, None, None, None]
    if c is not None:
        cc = np.asarray(c)
        r = r + (cc[:, None, None, None] if cc.ndim == 1 else cc) * mass * U
    return r


def apply_A(num: Numbering, geo: Geometry, gll: GLL, u: np.ndarray, dirichlet=None,
            kappa=None, c=None) -> np.ndarray:
    """y = mask(gather(r(scatter(u)))): the assembled operator of eq. (R).

    Only the output is masked; the input is used as given."""
    U = u[num.l2g]
    r = element_action(U, geo.G, gll.D, kappa, c, geo.mass)
    y = gather(num, r)
    if dirichlet is None:
        dirichlet = num.dirichlet
    y[dirichlet.astype(bool)] = 0.0
    return y


def load_vector(num: Numbering, m_global: np.ndarray, s_at_nodes: np.ndarray,
                dirichlet=None) -> np.ndarray:
    """b_N = m_N s(x_N) on free nodes, 0 on Dirichlet nodes: the right-hand side
    of eq. (pdeweak) integrated with the GLL rule of Section 2.4."""
    b = m_global * s_at_nodes
    if dirichlet is None:
        dirichlet = num.dirichlet
    b[dirichlet.astype(bool)] = 0.0
    return b
