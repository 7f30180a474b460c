"""Aggregation-based algebraic multigrid for the coarse system (Section 4.1,
"Algebraic multigrid") -- test infrastructure.

The paper names the ingredients only: a hierarchy built by unsmoothed
aggregation on the order-1 matrix, and a recursive K-cycle with damped Jacobi
smoothing at every level (its references hold the details).  The readings
taken here (and by the library):

* unknowns in ascending vertex id;
* strong couplings of row i: j != i with a_ij < 0 and -a_ij >= 0.25 max_k(-a_ik);
* one coarsening step = two pairwise passes (aggregates of at most 4): visit
  rows in order; an unmatched row i takes, among its unmatched strong
  neighbours, the one with the most negative a_ij (ties: smallest index), or
  stays alone; aggregates are numbered in order of creation; the second pass
  runs on the Galerkin matrix of the first;
* Galerkin coarse matrices A_{l+1} = P^T A_l P with P the 0/1 aggregate
  indicator; coarsening stops at 400 unknowns or less (or when a step removes
  less than a third of them), and the coarsest system is solved exactly;
* damped Jacobi with omega = 2/3, one sweep before and one after the coarse
  correction, starting from zero;
* the K-cycle: on every level but the coarsest two, the coarse correction is
  two flexible-CG iterations preconditioned by the next cycle (no early exit);
  P_0 R is one cycle on the finest level.

Library primitives used: scipy.sparse products, scipy.linalg.cho_factor /
cho_solve for the coarsest level.

Pinned by: the aggregates partition the unknowns with sizes 1..4; the
Galerkin matrices equal the dense products P^T A P; a one-level hierarchy
returns A^{-1} b; on the last two levels the cycle equals the two-grid
operator (I - S (I - P A_c^{-1} P^T A) S) A^{-1} with S = I - omega D^{-1} A
(dense algebra); the two flexible-CG steps return the Galerkin projection
V (V^T A V)^{-1} V^T b onto the two directions V = [v, v2] the cycle produced,
with the second direction taken at the residual left by the first; planted
mistakes (post-smoothing dropped, undamped sweep, no A-orthogonalisation, a
wrong first step length) fail those pins; the K-cycle as a preconditioner for
CG on the coarse matrix converges in a number of iterations that stays flat
as the mesh is refined.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg
import scipy.sparse

OMEGA = 2.0 / 3.0
BETA = 0.25
COARSEST = 400


def pairwise(A: scipy.sparse.csr_matrix) -> np.ndarray:
    """One pairwise pass: aggregate id of every row."""
    n = A.shape[0]
    agg = np.full(n, -1, dtype=np.int64)
    nagg = 0
    ip, ix, av = A.indptr, A.indices, A.data
    for i in range(n):
        if agg[i] >= 0:
            continue
        cols = ix[ip[i]:ip[i + 1]]
        vals = av[ip[i]:ip[i + 1]]
        off = (cols != i) & (vals < 0)
        best, bj = 0.0, -1
        if off.any():
            thr = BETA * float((-vals[off]).max())
            for j, a in zip(cols[off], vals[off]):
                if -a >= thr and agg[j] < 0 and (bj < 0 or a < best or (a == best and j < bj)):
                    best, bj = a, j
        agg[i] = nagg
        if bj >= 0:
            agg[bj] = nagg
        nagg += 1
    return agg


def indicator(agg: np.ndarray) -> scipy.sparse.csr_matrix:
    n = agg.size
    return scipy.sparse.csr_matrix((np.ones(n), (np.arange(n), agg)), shape=(n, int(agg.max()) + 1))


def hierarchy(A: scipy.sparse.csr_matrix):
    """Lists (matrices A_0..A_L, aggregate maps agg_0..agg_{L-1}); agg_l maps
    rows of A_l to rows of A_{l+1}."""
    As = [scipy.sparse.csr_matrix(A)]
    aggs = []
    while As[-1].shape[0] > COARSEST:
        Al = As[-1]
        a1 = pairwise(Al)
        P1 = indicator(a1)
        A1 = (P1.T @ Al @ P1).tocsr()
        a2 = pairwise(A1)
        agg = a2[a1]
        if agg.max() + 1 > (2 * Al.shape[0]) // 3:
            break
        P = indicator(agg)
        As.append((P.T @ Al @ P).tocsr())
        aggs.append(agg)
    for M in As:
        M.sort_indices()
    return As, aggs


class KCycle:
    """P_0 R: one K-cycle on the hierarchy of A (Section 4.1)."""

    def __init__(self, A: scipy.sparse.csr_matrix):
        self.As, self.aggs = hierarchy(A)
        self.D = [M.diagonal() for M in self.As]
        self.L = len(self.As) - 1
        Ac = self.As[-1].toarray()
        self.chol = scipy.linalg.cho_factor(Ac, lower=True) if Ac.size else None

    def coarsest(self, b):
        return scipy.linalg.cho_solve(self.chol, b) if self.chol is not None else b * 0.0

    def restrict(self, l, r):
        out = np.zeros(self.As[l + 1].shape[0])
        np.add.at(out, self.aggs[l], r)
        return out

    def cycle(self, l, b):
        if l == self.L:
            return self.coarsest(b)
        A, D = self.As[l], self.D[l]
        x = OMEGA * b / D
        r = b - A @ x
        rc = self.restrict(l, r)
        xc = self.coarsest(rc) if l + 1 == self.L else self.fcg2(l + 1, rc)
        x = x + xc[self.aggs[l]]
        x = x + OMEGA * (b - A @ x) / D
        return x

    def fcg2(self, l, b):
        A = self.As[l]
        v = self.cycle(l, b)
        w = A @ v
        rho, a1 = float(v @ b), float(v @ w)
        r2 = b - (rho / a1) * w
        v2 = self.cycle(l, r2)
        w2 = A @ v2
        g, be, a2 = float(v2 @ w), float(v2 @ w2), float(v2 @ r2)
        den = be - g * g / a1
        return (rho / a1) * v + (a2 / den) * (v2 - (g / a1) * v)

    def __call__(self, b):
        return self.cycle(0, np.asarray(b, dtype=np.float64))
