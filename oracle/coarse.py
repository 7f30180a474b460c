"""Coarse-scale correction of the two-scale preconditioner (Section 4.1, eq. (coarse)).

Test infrastructure.  Steps, in the paper's order and notation:

1. Coarse space: order n = 1 elements on the mesh vertices; the coarse matrix
   A_c is the same spectral-element operator at n = 1 (two-point GLL rule,
   i.e. quadrature at the 8 corners), assembled on the vertices, with the
   problem's kappa and c (the c term then lumps to c |J| at each corner).
   Vertices on the Dirichlet boundary are removed.
2. Vandermonde B_{IJK,ijk} = Phi_I(t_i) Phi_J(t_j) Phi_K(t_k), 8 x (n+1)^3,
   with Phi_0 = (1 - t)/2, Phi_1 = (1 + t)/2.
3. Restriction: y_N = r_N / m_N, scattered to y_{ijk;e};
   R_{IJK;e} = sum_ijk B_{IJK,ijk} y_{ijk;e} m_{ijk;e}; gathered (summed) to
   the vertices.
4. Z = P_0 R.  Reading: P_0 is the exact inverse of A_c (a dense Cholesky
   factorisation, FP64), so that the preconditioner is a fixed symmetric
   linear operator; the paper's algebraic multigrid approximates it
   (solver="amg": one K-cycle of :mod:`oracle.amg`).
5. Prolongation: Z scattered to Z_{IJK;e}; z_{ijk;e} = sum_IJK B_{IJK,ijk}
   Z_{IJK;e} m_{ijk;e}; gathered (summed) to z_N; and the coarse correction is
   z_N / m_N.  (The paper says "scatter" and "y_N" in this last step; the
   assembly it describes is a sum over the local copies of z, divided by m_N.)

Library primitives: numpy.einsum, scipy.linalg.cho_factor / cho_solve.

Pinned by: restriction == I^T r and prolongation == I Z for the trilinear
interpolation matrix I assembled independently node by node; A_c symmetric
positive definite; A_c equal to the dense order-1 brute-force assembly, with
and without kappa and c.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg
import scipy.sparse

from .geometry import Geometry
from .gll import GLL
from .numbering import Numbering, number_mesh
from .operator import element_action


def vandermonde(gll: GLL) -> np.ndarray:
    """B[K, J, I, k, j, i] = Phi_I(t_i) Phi_J(t_j) Phi_K(t_k)."""
    t = gll.t
    P = np.stack([(1 - t) / 2, (1 + t) / 2], axis=0)  # [I, i]
    return np.einsum("Ii,Jj,Kk->KJIkji", P, P, P)


def coarse_vertex_ids(num: Numbering) -> np.ndarray:
    """Global id of the vertex node at corner (I, J, K) of each element: [E, K, J, I]."""
    n = num.n
    return num.l2g[:, ::n, ::n, ::n]


def coarse_matrix(vtx, hexes, n_vertices: int, kappa=1.0, c=0.0) -> scipy.sparse.csr_matrix:
    """A_c: the order-1 operator kappa K + c M on the mesh vertices (sparse, all
    vertices); kappa and c are constants or one value per element."""
    g1 = GLL(1)
    num1 = number_mesh(hexes, 1)
    geo1 = Geometry(vtx, hexes, g1)
    E = num1.n_elem
    kap = np.broadcast_to(np.asarray(kappa, dtype=np.float64), (E,))
    cc = np.broadcast_to(np.asarray(c, dtype=np.float64), (E,))
    # element matrices: action on the 8 unit vectors of each element
    K = np.empty((E, 8, 8))
    for col in range(8):
        U = np.zeros((E, 2, 2, 2))
        U.reshape(E, 8)[:, col] = 1.0
        K[:, :, col] = element_action(U, geo1.G, g1.D, kap, cc, geo1.mass).reshape(E, 8)
    idx = num1.l2g.reshape(E, 8)
    rows = np.repeat(idx, 8, axis=1).ravel()
    cols = np.tile(idx, (1, 8)).ravel()
    A = scipy.sparse.coo_matrix((K.ravel(), (rows, cols)), shape=(n_vertices, n_vertices))
    return A.tocsr()


class CoarseCorrection:
    def __init__(self, num: Numbering, geo: Geometry, gll: GLL, vtx, hexes, m_global,
                 dirichlet=None, kappa=1.0, c=0.0, solver="exact"):
        self.num = num
        self.geo = geo
        self.B = vandermonde(gll)
        self.m_global = m_global
        self.cv = coarse_vertex_ids(num)  # [E, 2, 2, 2]
        nv = num.n_vertices
        if dirichlet is None:
            dirichlet = num.dirichlet
        self.free = np.nonzero(dirichlet[:nv] == 0)[0]
        A = coarse_matrix(vtx, hexes, nv, kappa, c)
        self.A_full = A
        self.solver = solver
        if solver == "amg":
            from .amg import KCycle
            self.Ac = A[self.free][:, self.free].tocsr()
            self.kcycle = KCycle(self.Ac) if self.free.size else None
            self.chol = None
        else:
            self.Ac = A[self.free][:, self.free].toarray()
            self.chol = scipy.linalg.cho_factor(self.Ac, lower=True) if self.free.size else None

    def restrict(self, r: np.ndarray) -> np.ndarray:
        """Global coarse residual R on all vertices (step 3)."""
        y = r / self.m_global
        y_loc = y[self.num.l2g]
        R_e = np.einsum("KJIkji,ekji->eKJI", self.B, y_loc * self.geo.mass)
        R = np.zeros(self.num.n_vertices)
        np.add.at(R, self.cv.ravel(), R_e.ravel())
        return R

    def solve(self, R: np.ndarray) -> np.ndarray:
        """Z = A_c^{-1} R on free vertices, 0 on Dirichlet vertices (step 4)."""
        Z = np.zeros_like(R)
        if self.solver == "amg":
            if self.kcycle is not None:
                Z[self.free] = self.kcycle(R[self.free])
        elif self.chol is not None:
            Z[self.free] = scipy.linalg.cho_solve(self.chol, R[self.free])
        return Z

    def prolong(self, Z: np.ndarray) -> np.ndarray:
        """Coarse correction z_N / m_N from vertex values Z (step 5)."""
        Z_e = Z[self.cv]  # [E, K, J, I]
        z_loc = np.einsum("KJIkji,eKJI->ekji", self.B, Z_e) * self.geo.mass
        z = np.zeros(self.num.n_global)
        np.add.at(z, self.num.l2g.ravel(), z_loc.ravel())
        return z / self.m_global

    def apply(self, r: np.ndarray) -> np.ndarray:
        return self.prolong(self.solve(self.restrict(r)))
