"""Dense brute-force assembly of the SEM stiffness matrix (pin for the oracle).

Test infrastructure.  Independent of the sum-factorised path in
:mod:`oracle.operator`: each element matrix is built from full 3D basis
gradients at every GLL quadrature point (no tensor-product shortcuts),

    K_e[a, b] = sum_q w_q |J_q| kappa_q (J_q^{-T} grad psi_a(q)) . (J_q^{-T} grad psi_b(q))
              + sum_q w_q |J_q| c_q psi_a(q) psi_b(q),

with psi_a = phi_i phi_j phi_k the nodal tensor basis of eq. (interp), the
Jacobian rebuilt here corner by corner from the trilinear map, and then
assembled into a dense global matrix through the local-to-global table.
Only for tiny meshes (a few thousand nodes).
"""
from __future__ import annotations

import itertools

import numpy as np

from .gll import GLL, lagrange_derivative_matrix, lagrange_values


def _jacobian_pointwise(Xc: np.ndarray, xi, eta, zeta) -> np.ndarray:
    """J at one reference point, summing over the 8 trilinear corner functions."""
    J = np.zeros((3, 3))
    for c, b, a in itertools.product((0, 1), (0, 1), (0, 1)):
        fa = (1 - xi) / 2 if a == 0 else (1 + xi) / 2
        fb = (1 - eta) / 2 if b == 0 else (1 + eta) / 2
        fc = (1 - zeta) / 2 if c == 0 else (1 + zeta) / 2
        da = -0.5 if a == 0 else 0.5
        db = -0.5 if b == 0 else 0.5
        dc = -0.5 if c == 0 else 0.5
        x = Xc[a + 2 * b + 4 * c]
        J[:, 0] += x * da * fb * fc
        J[:, 1] += x * fa * db * fc
        J[:, 2] += x * fa * fb * dc
    return J


def element_matrix(Xc: np.ndarray, gll: GLL, kappa=1.0, c=0.0) -> np.ndarray:
    """Dense (n+1)^3 x (n+1)^3 element matrix; local index i + (n+1)j + (n+1)^2 k.

    kappa and c: constants, or their values at the quadrature points [k, j, i]."""
    kq = np.broadcast_to(np.asarray(kappa, dtype=np.float64), (len(gll.t),) * 3)
    cq = np.broadcast_to(np.asarray(c, dtype=np.float64), (len(gll.t),) * 3)
    t, rho = gll.t, gll.rho
    n1 = len(t)
    Dq = lagrange_derivative_matrix(t)  # Dq[l, i] = phi_i'(t_l)
    Vq = lagrange_values(t, t)  # Vq[l, i] = phi_i(t_l) (identity up to rounding)
    nloc = n1 ** 3
    K = np.zeros((nloc, nloc))
    for qn, qm, ql in itertools.product(range(n1), range(n1), range(n1)):
        J = _jacobian_pointwise(Xc, t[ql], t[qm], t[qn])
        detJ = np.linalg.det(J)
        JinvT = np.linalg.inv(J).T
        w = rho[ql] * rho[qm] * rho[qn] * detJ
        grad = np.zeros((nloc, 3))
        vals = np.zeros(nloc)
        for k, j, i in itertools.product(range(n1), range(n1), range(n1)):
            a = i + n1 * j + n1 * n1 * k
            grad[a, 0] = Dq[ql, i] * Vq[qm, j] * Vq[qn, k]
            grad[a, 1] = Vq[ql, i] * Dq[qm, j] * Vq[qn, k]
            grad[a, 2] = Vq[ql, i] * Vq[qm, j] * Dq[qn, k]
            vals[a] = Vq[ql, i] * Vq[qm, j] * Vq[qn, k]
        gp = grad @ JinvT.T  # rows: J^{-T} grad psi_a
        K += w * kq[qn, qm, ql] * (gp @ gp.T) + w * cq[qn, qm, ql] * np.outer(vals, vals)
    return K


def assemble_dense(vtx, hexes, l2g: np.ndarray, n_global: int, gll: GLL, kappa=1.0,
                   c=0.0) -> np.ndarray:
    A = np.zeros((n_global, n_global))
    for e in range(len(hexes)):
        Xc = vtx[hexes[e]]
        K = element_matrix(Xc, gll, kappa, c)
        idx = l2g[e].reshape(-1)
        A[np.ix_(idx, idx)] += K
    return A
