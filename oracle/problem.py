"""One-stop set-up of the oracle for a mesh (test infrastructure).

Bundles the steps of Sections 2-4 for a given mesh and order: numbering,
geometry, lumped mass, node coordinates, operator, two-scale preconditioner
and PCG, for the model problem c u - div(kappa grad u) = s with kappa > 0 and
c >= 0 constant, one value per element (Algorithm 2) or one value per node
of every element (eq. (R)); kappa = 1, c = 0 is the Poisson problem.  With
per-node values the patch solves and the coarse matrix take each element's
mean (:func:`oracle.schwarz.element_mean`).
Nothing here adds arithmetic of its own.
"""
from __future__ import annotations

import numpy as np

from .coarse import CoarseCorrection
from .geometry import Geometry, box_sizes, lumped_mass, node_coords_global
from .gll import GLL
from .numbering import number_mesh
from .operator import apply_A, load_vector
from .pcg import TwoScale, pcg
from .schwarz import FinePreconditioner, element_mean


class Problem:
    def __init__(self, vtx, hexes, n, fine=True, coarse=True, dirichlet=None, kappa=1.0, c=0.0,
                 coarse_solver="exact"):
        self.vtx = np.asarray(vtx, dtype=np.float64)
        self.hexes = np.asarray(hexes, dtype=np.int64)
        self.n = n
        self.gll = GLL(n)
        self.num = number_mesh(self.hexes, n)
        self.geo = Geometry(self.vtx, self.hexes, self.gll)
        self.m = lumped_mass(self.num, self.geo)
        self.x = node_coords_global(self.num, self.geo)
        self.dirichlet = self.num.dirichlet if dirichlet is None else dirichlet
        E = len(self.hexes)
        n1 = n + 1

        def coefficient(v):
            if np.ndim(v) == 0:
                return float(v)
            a = np.asarray(v, dtype=np.float64)
            return a.reshape(E) if a.size == E else a.reshape(E, n1, n1, n1)

        self.kappa = coefficient(kappa)
        self.c = coefficient(c)
        self.kappa_pc = element_mean(self.gll, self.kappa) if np.ndim(self.kappa) == 4 else self.kappa
        self.c_pc = element_mean(self.gll, self.c) if np.ndim(self.c) == 4 else self.c
        self._fine_on = fine
        self._coarse_on = coarse
        self.coarse_solver = coarse_solver
        self._fine = None
        self._coarse = None

    @property
    def fine(self):
        if self._fine is None and self._fine_on:
            self._fine = FinePreconditioner(self.num, self.hexes, self.vtx, self.gll,
                                            box_sizes(self.vtx, self.hexes), self.kappa_pc, self.c_pc)
        return self._fine

    @property
    def coarse(self):
        if self._coarse is None and self._coarse_on:
            self._coarse = CoarseCorrection(self.num, self.geo, self.gll, self.vtx, self.hexes,
                                            self.m, self.dirichlet, self.kappa_pc, self.c_pc, self.coarse_solver)
        return self._coarse

    def A(self, u):
        if np.all(np.asarray(self.kappa) == 1.0) and np.all(np.asarray(self.c) == 0.0):
            return apply_A(self.num, self.geo, self.gll, u, self.dirichlet)
        E = self.num.n_elem

        def per_element_or_node(v):
            return v if np.ndim(v) == 4 else np.broadcast_to(v, (E,))

        return apply_A(self.num, self.geo, self.gll, u, self.dirichlet,
                       per_element_or_node(self.kappa), per_element_or_node(self.c))

    def precond(self, fine=True, coarse=True):
        return TwoScale(self.fine if fine else None, self.coarse if coarse else None,
                        self.dirichlet)

    def load(self, s_fn):
        return load_vector(self.num, self.m, s_fn(self.x), self.dirichlet)

    def solve(self, b, rtol=1e-8, max_iter=2000, fine=True, coarse=True, x0=None):
        return pcg(self.A, b, self.precond(fine, coarse), rtol=rtol, max_iter=max_iter, x0=x0)
