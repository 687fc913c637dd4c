"""Loss gradients of the discrete generalized Stokes solution by the adjoint method.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Forward map (Section 2, discrete problem; data as nodal interpolants):
    g  <- g - (m^T g / m^T 1)                 (data made compatible: int g = 0)
    F  = (M_full f, M_P g)                    (load vectors of the P2 / P1 interpolants)
    x  = (u, p) solves  calA(beta) x = F,  with int p_h = 0.
The saddle matrix is symmetric, so the adjoint system uses the same matrix:
    calA lambda = (dL/du, Pi^T dL/dp),   Pi = I - 1 m^T / (m^T 1),
and with it
    dL/df_nodal = M_full[interior, :]^T lambda_u      (per component)
    dL/dg_nodal = Pi^T M_P lambda_p
    dL/dbeta    = -lambda_u^T M u                      (d calA / d beta = diag(M, M, 0)).
The solves are sparse direct solves (the plain definition) by default; for
grids where a direct factorization is out of reach, `mg_solver` gives the
same linear solves by the multigrid iterate of Section 3 run to a tight
relative residual (exact up to that tolerance).
"""
from __future__ import annotations

import numpy as np

from . import multigrid as mg
from .multigrid import Level


def project(lv: Level, g: np.ndarray) -> np.ndarray:
    return g - (lv.m @ g) / lv.m.sum()


def mg_solver(h: mg.Hierarchy, tol: float = 1e-12, maxit: int = 400):
    """A linear solve x = calA^{-1} F (F compatible) by NE V(2,2) iterates."""
    def solve(F: np.ndarray) -> np.ndarray:
        res = mg.solve(h, F, mg.Params(), tol=tol, maxit=maxit)
        if res.status != "ok":
            raise RuntimeError(f"oracle multigrid solve: {res.status} at {res.relres}")
        return res.x
    return solve


def forward(lv: Level, f_nodal: np.ndarray, g_nodal: np.ndarray, solve=None) -> np.ndarray:
    d = lv.disc
    fu, gp = d.load(f_nodal, project(lv, g_nodal))
    F = np.concatenate([fu, gp])
    return lv.project_mean(solve(F) if solve is not None else lv.direct_solve(F))


def mass_loss(lv: Level, x: np.ndarray, u_target: np.ndarray) -> float:
    """L = 1/2 (u - u_t)^T M (u - u_t) over the interior velocity unknowns."""
    e = x[: lv.nu2] - u_target
    return 0.5 * float(e @ (lv.disc.mass_u() @ e))


def gradients(lv: Level, x: np.ndarray, dL_du: np.ndarray, dL_dp: np.ndarray, solve=None):
    """(dL/df_nodal (2, n2), dL/dg_nodal (n1,), dL/dbeta) for cotangents of (u, p)."""
    d = lv.disc
    rhs_p = dL_dp - lv.m * (dL_dp.sum() / lv.m.sum())          # Pi^T dL/dp
    R = np.concatenate([dL_du, rhs_p])
    lam = solve(R) if solve is not None else lv.direct_solve(R)
    lu, lp = lam[: lv.nu2], lam[lv.nu2:]
    Mi = d.M_full[d.interior]                                   # (nu, n2)
    df = np.stack([Mi.T @ lu[: d.nu], Mi.T @ lu[d.nu:]])
    MPl = d.MP @ lp
    dg = MPl - lv.m * (lv.m @ lp) / lv.m.sum()                  # Pi^T M_P lambda_p
    dbeta = -float(lu @ (d.mass_u() @ x[: lv.nu2]))
    return df, dg, dbeta
