"""Differentiable solves of the generalized Stokes system (adjoint method).

Forward (per instance, data as nodal interpolants in the lattice layout):
    g  <- g - (m^T g / m^T 1)             (compatible data: int g = 0)
    F  = (M_full f, M_P g)                (load vectors, Section 2)
    x  = (u, p): calA(beta) x = F, int p = 0, by the multigrid of Section 3.
The saddle matrix is symmetric, so the backward pass solves with the same
multigrid:
    calA lambda = (dL/du, Pi^T dL/dp),    Pi^T v = v - m (1^T v) / (m^T 1)
    dL/df = M_full[interior, :]^T lambda_u      (all lattice points)
    dL/dg = Pi^T M_P lambda_p
    dL/dbeta = -lambda_u^T M u                  (d calA / d beta = diag(M, M, 0)).
With mixed=True both solves are FP32 cycles inside FP64 iterative refinement
(the FP64 residual and projection decide convergence), else FP64 cycles.
Every step runs in the HIP library (loads, masses, projections, solves, dots);
this module only wires them into torch.autograd.
"""
from __future__ import annotations

import torch

from .solver import Batch, Hierarchy

_CACHE: dict = {}


def hierarchy(N: int, beta: float, **kw) -> Hierarchy:
    """A cached hierarchy for (N, beta, solver options)."""
    key = (int(N), float(beta), tuple(sorted(kw.items())))
    h = _CACHE.get(key)
    if h is None:
        h = Hierarchy(N, float(beta), **kw)
        _CACHE[key] = h
    return h


def _beta_value(beta) -> float:
    return float(beta.detach().cpu()) if torch.is_tensor(beta) else float(beta)


class StokesSolve(torch.autograd.Function):
    """(f_nodal (2,M,M), g_nodal (N+1,N+1), beta (0-d)) -> (u, p)."""

    @staticmethod
    def forward(ctx, f_nodal, g_nodal, beta, rtol, maxit, mixed, opts):
        N = f_nodal.shape[-1] // 2
        h = hierarchy(N, _beta_value(beta), **opts)
        g = g_nodal.detach().clone().contiguous()
        h.project_mean(g)
        fu, gp = h.load(f_nodal.detach().contiguous(), g)
        u, p, info = (h.solve_mixed if mixed else h.solve)(fu, gp, rtol=rtol, maxit=maxit)
        if info.status != "ok":
            raise RuntimeError(f"forward solve: {info}")
        ctx.h, ctx.rtol, ctx.maxit, ctx.mixed = h, rtol, maxit, mixed
        ctx.beta_is_tensor = torch.is_tensor(beta)
        ctx.save_for_backward(u, p)
        return u, p

    @staticmethod
    def backward(ctx, gu, gp):
        h = ctx.h
        u, p = ctx.saved_tensors
        ru = torch.zeros_like(u) if gu is None else gu.contiguous().clone()
        rp = torch.zeros_like(p) if gp is None else gp.contiguous().clone()
        h.project_dual(rp)
        lu, lp, info = (h.solve_mixed if ctx.mixed else h.solve)(ru, rp, rtol=ctx.rtol, maxit=ctx.maxit)
        if info.status != "ok":
            raise RuntimeError(f"adjoint solve: {info}")
        df = h.mass(lu, all_nodes=True)
        dg = h.pressure_mass(lp)
        h.project_dual(dg)
        dbeta = None
        if ctx.beta_is_tensor and ctx.needs_input_grad[2]:
            dbeta = -h.dot(lu, h.mass(u), 0).reshape(())
        return df, dg, dbeta, None, None, None, None


def stokes_solve(f_nodal, g_nodal, beta, rtol: float = 1e-10, maxit: int = 500, mixed: bool = False, **opts):
    """Differentiable solve; gradients flow to f_nodal, g_nodal and beta (a tensor).
    mixed: FP32 cycles inside FP64 iterative refinement for both solves."""
    return StokesSolve.apply(f_nodal, g_nodal, beta, rtol, maxit, bool(mixed), opts)


class MassProduct(torch.autograd.Function):
    """y = M u on the interior velocity nodes (M symmetric: the backward is M again)."""

    @staticmethod
    def forward(ctx, u, N, beta):
        h = hierarchy(N, beta)
        ctx.h = h
        return h.mass(u.contiguous())

    @staticmethod
    def backward(ctx, gy):
        return ctx.h.mass(gy.contiguous()), None, None


def mass_product(u, N: int):
    """Differentiable M u (the velocity mass matrix; independent of beta)."""
    return MassProduct.apply(u, int(N), 0.0)


# ---------------------------------------------------------------------------
# batched
# ---------------------------------------------------------------------------

_BCACHE: dict = {}


def batch(Ns, betas, **kw) -> Batch:
    key = (tuple(int(n) for n in Ns), tuple(float(b) for b in betas), tuple(sorted(kw.items())))
    b = _BCACHE.get(key)
    if b is None:
        b = Batch(list(Ns), list(betas), **kw)
        _BCACHE[key] = b
    return b


class BatchStokesSolve(torch.autograd.Function):
    """Stacked instances of one size: f (B,2,M,M), g (B,N+1,N+1), beta (B,) -> (u, p) stacked."""

    @staticmethod
    def forward(ctx, f, g, beta, rtol, maxit, mixed, opts):
        nb, N = f.shape[0], f.shape[-1] // 2
        betas = beta.detach().cpu().tolist() if torch.is_tensor(beta) else [float(v) for v in beta]
        B = batch([N] * nb, betas, **opts)
        fus, gps = [], []
        for k, h in enumerate(B.instances):
            gk = g[k].detach().clone().contiguous()
            h.project_mean(gk)
            fu, gp = h.load(f[k].detach().contiguous(), gk)
            fus.append(fu)
            gps.append(gp)
        us, ps, infos = (B.solve_mixed if mixed else B.solve)(fus, gps, rtol=rtol, maxit=maxit)
        if any(i.status != "ok" for i in infos):
            raise RuntimeError(f"batched forward solve: {infos}")
        u = torch.stack(us)
        p = torch.stack(ps)
        ctx.B, ctx.rtol, ctx.maxit, ctx.mixed = B, rtol, maxit, mixed
        ctx.beta_is_tensor = torch.is_tensor(beta)
        ctx.save_for_backward(u, p)
        return u, p

    @staticmethod
    def backward(ctx, gu, gp):
        B = ctx.B
        u, p = ctx.saved_tensors
        rus, rps = [], []
        for k, h in enumerate(B.instances):
            ru = torch.zeros_like(u[k]) if gu is None else gu[k].contiguous().clone()
            rp = torch.zeros_like(p[k]) if gp is None else gp[k].contiguous().clone()
            h.project_dual(rp)
            rus.append(ru)
            rps.append(rp)
        lus, lps, infos = (B.solve_mixed if ctx.mixed else B.solve)(rus, rps, rtol=ctx.rtol, maxit=ctx.maxit)
        if any(i.status != "ok" for i in infos):
            raise RuntimeError(f"batched adjoint solve: {infos}")
        dfs, dgs, dbs = [], [], []
        for k, h in enumerate(B.instances):
            dfs.append(h.mass(lus[k], all_nodes=True))
            dg = h.pressure_mass(lps[k])
            h.project_dual(dg)
            dgs.append(dg)
            if ctx.beta_is_tensor:
                dbs.append(-h.dot(lus[k], h.mass(u[k].contiguous()), 0).reshape(()))
        dbeta = torch.stack(dbs) if ctx.beta_is_tensor and ctx.needs_input_grad[2] else None
        return torch.stack(dfs), torch.stack(dgs), dbeta, None, None, None, None


def batch_stokes_solve(f, g, beta, rtol: float = 1e-10, maxit: int = 500, mixed: bool = False, **opts):
    """Differentiable batched solve of B instances of one size.
    mixed: FP32 cycles inside FP64 iterative refinement for both solves."""
    return BatchStokesSolve.apply(f, g, beta, rtol, maxit, bool(mixed), opts)
