"""Implicit Euler time stepping of the time-dependent Stokes problem.

Section 1 motivates the generalized problem as what one implicit time step
leaves to solve: with dt = 1 / beta, a backward Euler step is the saddle
system calA(beta) with right-hand side (M_full f + beta M u^n, M_P g).  The
library forms that right-hand side and solves the step warm-started from the
previous state (smg_implicit_step); a hierarchy is set up once per dt and
reused for every step.  Several dt (or several trajectories) march together
as one batch.  mixed=True solves each step with FP32 cycles inside FP64
iterative refinement (smg_implicit_step_mixed).
"""
from __future__ import annotations

from .solver import Batch, Hierarchy


class ImplicitEuler:
    """One trajectory: state (u, p) on an h = 1/N grid, time step dt."""

    def __init__(self, N: int, dt: float, u0=None, mixed: bool = False, **kw):
        if not dt > 0:
            raise ValueError("dt must be positive")
        self.dt = float(dt)
        self.mixed = bool(mixed)
        self.h = Hierarchy(N, 1.0 / self.dt, **kw)
        self.u, self.p = self.h.zeros()
        if u0 is not None:
            self.u.copy_(u0)
        self.t = 0.0

    def step(self, f_nodal=None, g_nodal=None, rtol=1e-10, maxit=200):
        info = self.h.implicit_step(self.u, self.p, f_nodal, g_nodal, rtol=rtol, maxit=maxit, mixed=self.mixed)
        if info.status != "ok":
            raise RuntimeError(f"implicit step at t={self.t}: {info}")
        self.t += self.dt
        return info

    def run(self, nsteps: int, forcing=None, rtol=1e-10, maxit=200):
        """nsteps steps; forcing(t) -> f_nodal at the new time (or None)."""
        infos = []
        for _ in range(nsteps):
            f = forcing(self.t + self.dt) if forcing is not None else None
            infos.append(self.step(f, rtol=rtol, maxit=maxit))
        return infos


class BatchImplicitEuler:
    """Several trajectories (sizes Ns, time steps dts) stepped together."""

    def __init__(self, Ns, dts, u0s=None, mixed: bool = False, **kw):
        if any(not dt > 0 for dt in dts):
            raise ValueError("dt must be positive")
        self.dts = [float(dt) for dt in dts]
        self.mixed = bool(mixed)
        self.B = Batch(list(Ns), [1.0 / dt for dt in self.dts], **kw)
        outs = [h.zeros() for h in self.B.instances]
        self.us = [u for u, _ in outs]
        self.ps = [p for _, p in outs]
        if u0s is not None:
            for u, u0 in zip(self.us, u0s):
                u.copy_(u0)
        self.steps = 0

    def step(self, f_nodals=None, g_nodals=None, rtol=1e-10, maxit=200):
        infos = self.B.implicit_step(self.us, self.ps, f_nodals, g_nodals, rtol=rtol, maxit=maxit,
                                     mixed=self.mixed)
        bad = [i for i in infos if i.status != "ok"]
        if bad:
            raise RuntimeError(f"batched implicit step {self.steps}: {bad[:3]}")
        self.steps += 1
        return infos
