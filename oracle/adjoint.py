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
All solves here are sparse direct solves (the plain definition).
"""
from __future__ import annotations

import numpy as np

from .multigrid import Level


def project(lv: Level, g: np.ndarray) -> np.ndarray:
    return g - (lv.m @ g) / lv.m.sum()


def forward(lv: Level, f_nodal: np.ndarray, g_nodal: np.ndarray) -> np.ndarray:
    d = lv.disc
    fu, gp = d.load(f_nodal, project(lv, g_nodal))
    return lv.project_mean(lv.direct_solve(np.concatenate([fu, gp])))


def mass_loss(lv: Level, x: np.ndarray, u_target: np.ndarray) -> float:
    """L = 1/2 (u - u_t)^T M (u - u_t) over the interior velocity unknowns."""
    e = x[: lv.nu2] - u_target
    return 0.5 * float(e @ (lv.disc.mass_u() @ e))


def gradients(lv: Level, x: np.ndarray, dL_du: np.ndarray, dL_dp: np.ndarray):
    """(dL/df_nodal (2, n2), dL/dg_nodal (n1,), dL/dbeta) for cotangents of (u, p)."""
    d = lv.disc
    rhs_p = dL_dp - lv.m * (dL_dp.sum() / lv.m.sum())          # Pi^T dL/dp
    lam = lv.direct_solve(np.concatenate([dL_du, rhs_p]))
    lu, lp = lam[: lv.nu2], lam[lv.nu2:]
    Mi = d.M_full[d.interior]                                   # (nu, n2)
    df = np.stack([Mi.T @ lu[: d.nu], Mi.T @ lu[d.nu:]])
    MPl = d.MP @ lp
    dg = MPl - lv.m * (lv.m @ lp) / lv.m.sum()                  # Pi^T M_P lambda_p
    dbeta = -float(lu @ (d.mass_u() @ x[: lv.nu2]))
    return df, dg, dbeta
