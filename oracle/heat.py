"""Heat equation by backward Euler (Section 6.2) -- test infrastructure.

Model problem eq. (pde) turned into a heat equation: with time step dt, each
step solves

    c u^{t} - div(kappa grad u^{t}) = u^{t-dt} / dt + q^{t},   c = 1 / dt,

for u^{t} with u = 0 on the Dirichlet boundary.  Discretised as in Section 2:
the operator kappa A + c M (eq. (R) with constant kappa and c), and the
right-hand side integrated with the GLL rule, b_N = m_N (u_N^{t-dt} / dt +
q_N^{t}) on free nodes (the load vector of eq. (pdeweak)), 0 on Dirichlet
nodes.  Each step is one PCG solve (Algorithm 1, two-scale preconditioner
built for the same kappa and c) started from the previous solution.

Readings: the source values q_N^{t} (the paper's Q / (rho c_p) spread over the
moving heat source) are inputs, one nodal array per step; the paper does not
state the PCG tolerance of a step, it is an argument here.

Pinned by: the decay of a single Dirichlet eigenmode of the cube,
u^{t} = (1 + dt kappa 3 pi^2)^{-t/dt} u^0 for u^0 = sin(pi x) sin(pi y)
sin(pi z) and q = 0, up to the spatial error of the discretisation.
"""
from __future__ import annotations

import numpy as np

from .operator import load_vector
from .problem import Problem


def heat_problem(vtx, hexes, n, kappa, dt, dirichlet=None) -> Problem:
    """The oracle set up for kappa A + (1/dt) M."""
    return Problem(vtx, hexes, n, dirichlet=dirichlet, kappa=kappa, c=1.0 / dt)


def rhs(P: Problem, u_prev: np.ndarray, q: np.ndarray, dt: float) -> np.ndarray:
    """b_N = m_N (u^{t-dt}_N / dt + q^{t}_N), 0 on Dirichlet nodes."""
    return load_vector(P.num, P.m, u_prev / dt + q, P.dirichlet)


def backward_euler(P: Problem, u0: np.ndarray, sources, dt: float, rtol=1e-10, max_iter=2000):
    """Advance u0 by len(sources) steps.  Returns (u after each step, PCG
    iterations of each step)."""
    u = np.array(u0, dtype=np.float64)
    us, its = [], []
    for q in sources:
        b = rhs(P, u, q, dt)
        u, k, _, _ = P.solve(b, rtol=rtol, max_iter=max_iter, x0=u)
        us.append(u.copy())
        its.append(k)
    return us, its
