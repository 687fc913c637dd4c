"""Implicit Euler steps of the time-dependent Stokes problem.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Section 1 introduces the generalized Stokes problem as what one implicit
time step of the time-dependent Stokes problem leaves to solve, with beta
proportional to the inverse time step.  For the implicit (backward) Euler
step of length dt = 1 / beta the discrete problem of Section 2 reads

    (K + beta M) u^{n+1} + B^T p^{n+1} = M_full f + beta M u^n,
    B u^{n+1}                          = M_P g,

with int p^{n+1} = 0: the saddle system calA(beta) with a right-hand side
that carries the previous velocity.  It is solved here directly (the plain
definition).
"""
from __future__ import annotations

import numpy as np

from .multigrid import Level


def step(lv: Level, u_prev: np.ndarray, f_nodal: np.ndarray | None = None,
         g_nodal: np.ndarray | None = None) -> np.ndarray:
    """x^{n+1} = (u^{n+1}, p^{n+1}) from the interior velocity u^n (length nu2)."""
    d = lv.disc
    fn = np.zeros((2, d.n2)) if f_nodal is None else f_nodal
    gn = np.zeros(d.n1) if g_nodal is None else g_nodal
    fu, gp = d.load(fn, gn)
    rhs_u = fu + lv.beta * (d.mass_u() @ u_prev)
    return lv.project_mean(lv.direct_solve(np.concatenate([rhs_u, gp])))


def march(lv: Level, u0: np.ndarray, nsteps: int, f_nodal=None, g_nodal=None):
    """The velocities and pressures of nsteps steps from u^0 (constant data)."""
    u = u0.copy()
    out = []
    for _ in range(nsteps):
        x = step(lv, u, f_nodal, g_nodal)
        u = x[: lv.nu2]
        out.append(x)
    return out
