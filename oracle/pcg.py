"""Preconditioned conjugate gradients (Section 3, Algorithm 1) and the two-scale
preconditioner P = P^c + P^f (Section 4).

Test infrastructure.  Readings:

* in Algorithm 1, r(.) stands for the operator action; r_0 = b - A u_0 with
  u_0 = 0, so r_0 = b;
* the stopping rule (not stated in the paper) is ||r_k||_2 <= rtol ||b||_2 on
  the recursively updated residual; b = 0 returns u = 0 with 0 iterations;
* Dirichlet nodes are held at zero by masking the operator output and the
  preconditioner output.

Pinned by: equality with a dense direct solve on tiny meshes.
"""
from __future__ import annotations

import numpy as np


class TwoScale:
    """P r = mask(P^f r + P^c r); either part may be switched off."""

    def __init__(self, fine=None, coarse=None, dirichlet=None):
        self.fine = fine
        self.coarse = coarse
        self.dirichlet = None if dirichlet is None else dirichlet.astype(bool)

    def __call__(self, r):
        z = np.zeros_like(r)
        if self.fine is not None:
            z = z + self.fine.apply(r)
        if self.coarse is not None:
            z = z + self.coarse.apply(r)
        if self.fine is None and self.coarse is None:
            z = r.copy()
        if self.dirichlet is not None:
            z[self.dirichlet] = 0.0
        return z


def pcg(apply_A, b, precond, rtol=1e-8, max_iter=1000, x0=None):
    """Algorithm 1.  Returns (u, iterations, residual history, (alphas, betas))."""
    bnorm = np.linalg.norm(b)
    u = np.zeros_like(b) if x0 is None else x0.copy()
    if bnorm == 0.0:
        return u, 0, [0.0], ([], [])
    r = b - apply_A(u) if x0 is not None else b.copy()
    z = precond(r)
    p = z.copy()
    rz = float(z @ r)
    hist = [np.linalg.norm(r) / bnorm]
    alphas, betas = [], []
    k = 0
    while hist[-1] > rtol and k < max_iter:
        f = apply_A(p)
        pf = float(p @ f)
        if not np.isfinite(pf) or pf <= 0.0:
            raise FloatingPointError("PCG breakdown: p^T A p <= 0")
        alpha = rz / pf
        u = u + alpha * p
        r = r - alpha * f
        z = precond(r)
        rz_new = float(z @ r)
        beta = rz_new / rz
        p = z + beta * p
        rz = rz_new
        alphas.append(alpha)
        betas.append(beta)
        k += 1
        hist.append(np.linalg.norm(r) / bnorm)
    return u, k, hist, (alphas, betas)
