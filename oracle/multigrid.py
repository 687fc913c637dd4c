"""The coupled multigrid method for the discretized generalized Stokes system.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Follows the paper step by step:
  * Section 3: one iterate = nu_pre smoothing steps, coarse-grid correction
    (defect, restriction with the transposed embedding, approximate coarse
    solve by gamma = 1 (V) or 2 (W) recursive iterates, prolongation and add),
    then nu_post smoothing steps; level 0 is solved exactly.
  * Section 4: the normal-equation smoother
        x <- x + tau L^{-1} A L^{-1} (f - A x)
    and the Uzawa-type smoother (three half-steps, velocity / pressure /
    velocity).
  * Section 6, equation (numintroduc): the practical preconditioner
        L = diag(Ahat, Shat),  Ahat = diag A,  Shat = diag(B Ahat^{-1} B^T),
    with tau = 0.35 (normal equation) and tau = sigma = 0.8 (Uzawa).

Readings where the paper is silent:
  * the pressure space P_k = P1 with mean zero is represented by the full P1
    nodal basis; iterates are projected to mean zero (weights m_i = int phi_i)
    after every top-level cycle, and the coarsest grid is solved with the
    constraint m^T p = 0 as a bordered system;
  * the initial guess is zero and the stopping rule of the solver is the
    relative Euclidean residual ||f - A x|| / ||f||.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import mesh as meshmod
from .fem import Discretization
from .transfer import saddle_prolongation


@dataclass
class Params:
    smoother: str = "ne"       # "ne" (normal equation) or "uzawa"
    tau: float = 0.35
    sigma: float = 0.8
    nu_pre: int = 2
    nu_post: int = 2
    gamma: int = 1             # 1 = V-cycle, 2 = W-cycle
    level_tau: tuple | None = None     # damping per level k (index k), replacing tau
    level_sigma: tuple | None = None   # the same for sigma

    def tau_at(self, k: int) -> float:
        return self.tau if self.level_tau is None else self.level_tau[k]

    def sigma_at(self, k: int) -> float:
        return self.sigma if self.level_sigma is None else self.level_sigma[k]

    @staticmethod
    def uzawa(nu_pre=3, nu_post=3, gamma=1):
        return Params("uzawa", 0.8, 0.8, nu_pre, nu_post, gamma)


class Level:
    """Matrices and smoother data of one grid level at a given beta."""

    def __init__(self, disc: Discretization, beta: float):
        self.disc = disc
        self.beta = float(beta)
        self.A = disc.A(beta)
        self.B = disc.B()
        self.Bt = self.B.T.tocsr()
        self.calA = disc.saddle(beta)
        self.nu2 = 2 * disc.nu
        self.n1 = disc.n1
        self.n = self.nu2 + self.n1
        # equation (numintroduc): Ahat = diag A, Shat = diag(B Ahat^{-1} B^T)
        self.Ahat = self.A.diagonal().copy()
        self.Shat = np.asarray(self.B.multiply(self.B) @ (1.0 / self.Ahat)).ravel()
        self.Ldiag = np.concatenate([self.Ahat, self.Shat])
        self.m = disc.m
        self.P = None          # prolongation from the next coarser level
        self._lu = None

    # -- pressure normalisation ----------------------------------------------
    def project_mean(self, x: np.ndarray) -> np.ndarray:
        """p <- p - (sum_i m_i p_i / sum_i m_i): the representative with int p = 0."""
        x = x.copy()
        p = x[self.nu2:]
        x[self.nu2:] = p - (self.m @ p) / self.m.sum()
        return x

    # -- exact solve (used on level 0, and as the discrete solution) ----------
    def bordered(self) -> sp.csc_matrix:
        """[[A, B^T, 0], [B, 0, m], [0, m^T, 0]]: the saddle system with the
        mean-zero constraint on the pressure and a multiplier."""
        e = np.zeros(self.n)
        e[self.nu2:] = self.m
        col = sp.csr_matrix(e[:, None])
        return sp.bmat([[self.calA, col], [col.T, None]], format="csc")

    def direct_solve(self, f: np.ndarray) -> np.ndarray:
        if self._lu is None:
            self._lu = spla.splu(self.bordered())
        z = self._lu.solve(np.concatenate([f, [0.0]]))
        return z[:-1]


class Hierarchy:
    """Levels 0..L of a uniformly refined mesh, re-discretized on every level."""

    def __init__(self, kind: str, levels: int, beta: float, n0: int = 2):
        meshes = meshmod.hierarchy(kind, levels, n0)
        self.discs = [Discretization(m) for m in meshes]
        self.levels = [Level(d, beta) for d in self.discs]
        for k in range(1, len(self.levels)):
            self.levels[k].P = saddle_prolongation(self.discs[k - 1], self.discs[k])
        self.beta = float(beta)

    @property
    def top(self) -> Level:
        return self.levels[-1]

    @property
    def L(self) -> int:
        return len(self.levels) - 1


# ---------------------------------------------------------------------------
# smoothers (Section 4)
# ---------------------------------------------------------------------------

def ne_step(lv: Level, x: np.ndarray, f: np.ndarray, tau: float) -> np.ndarray:
    """Normal-equation smoother: x + tau L^{-1} A L^{-1} (f - A x)."""
    r = f - lv.calA @ x
    y = r / lv.Ldiag
    return x + x.dtype.type(tau) * (lv.calA @ y) / lv.Ldiag


def uzawa_step(lv: Level, x: np.ndarray, f: np.ndarray, tau: float, sigma: float) -> np.ndarray:
    """Uzawa-type smoother, the three half-steps as stated in Section 4:
        u' = u + tau Ahat^{-1} (f - A u - B^T p)
        p+ = p - sigma Shat^{-1} (g - B u')
        u+ = u + tau Ahat^{-1} (f - A u - B^T p+)
    """
    nu2 = lv.nu2
    u, p = x[:nu2], x[nu2:]
    fu, g = f[:nu2], f[nu2:]
    tau, sigma = x.dtype.type(tau), x.dtype.type(sigma)
    Au = lv.A @ u
    u_half = u + tau * (fu - Au - lv.Bt @ p) / lv.Ahat
    p_new = p - sigma * (g - lv.B @ u_half) / lv.Shat
    u_new = u + tau * (fu - Au - lv.Bt @ p_new) / lv.Ahat
    return np.concatenate([u_new, p_new])


def smooth(lv: Level, x: np.ndarray, f: np.ndarray, prm: Params, k: int | None = None) -> np.ndarray:
    """One smoothing step on level k (the damping of level k when per-level
    values are given; Section 6 remarks that they may depend on the level)."""
    tau = prm.tau if k is None else prm.tau_at(k)
    sigma = prm.sigma if k is None else prm.sigma_at(k)
    if prm.smoother == "ne":
        return ne_step(lv, x, f, tau)
    if prm.smoother == "uzawa":
        return uzawa_step(lv, x, f, tau, sigma)
    raise ValueError(prm.smoother)


# ---------------------------------------------------------------------------
# multigrid cycle (Section 3)
# ---------------------------------------------------------------------------

def restrict_residual(h: Hierarchy, k: int, x: np.ndarray, f: np.ndarray) -> np.ndarray:
    """r_{k-1} = I_k^{k-1} (f - A_k x), with I_k^{k-1} = (I_{k-1}^k)^T."""
    lv = h.levels[k]
    return lv.P.T @ (f - lv.calA @ x)


def cycle(h: Hierarchy, k: int, x: np.ndarray, f: np.ndarray, prm: Params) -> np.ndarray:
    """One multigrid iterate on level k."""
    if k == 0:
        return h.levels[0].direct_solve(f)
    lv = h.levels[k]
    for _ in range(prm.nu_pre):
        x = smooth(lv, x, f, prm, k)
    rc = restrict_residual(h, k, x, f)
    # the coarse correction starts from zero in the arithmetic of the cycle
    # (float32 when the cycle runs in single precision)
    z = np.zeros(h.levels[k - 1].n, dtype=rc.dtype)
    for _ in range(prm.gamma):
        z = cycle(h, k - 1, z, rc, prm)
    x = x + lv.P @ z
    for _ in range(prm.nu_post):
        x = smooth(lv, x, f, prm, k)
    return x


def top_cycle(h: Hierarchy, x: np.ndarray, f: np.ndarray, prm: Params) -> np.ndarray:
    """One iterate of the solver on the finest level, followed by the mean projection."""
    return h.top.project_mean(cycle(h, h.L, x, f, prm))


def residual(lv: Level, x: np.ndarray, f: np.ndarray) -> np.ndarray:
    return f - lv.calA @ x


@dataclass
class SolveResult:
    x: np.ndarray
    iters: int
    relres: float
    history: list
    status: str            # "ok", "noconv", "diverged", "nonfinite"


def solve(h: Hierarchy, f: np.ndarray, prm: Params, tol: float = 1e-8, maxit: int = 100,
          x0: np.ndarray | None = None) -> SolveResult:
    """Repeat top-level iterates until ||f - A x|| <= tol ||f||."""
    lv = h.top
    x = np.zeros(lv.n) if x0 is None else lv.project_mean(np.asarray(x0, float))
    nf = np.linalg.norm(f)
    if nf == 0.0:
        return SolveResult(np.zeros(lv.n), 0, 0.0, [], "ok")
    rel = np.linalg.norm(residual(lv, x, f)) / nf
    hist = []
    it = 0
    status = "ok" if rel <= tol else "noconv"
    while rel > tol and it < maxit:
        x = top_cycle(h, x, f, prm)
        it += 1
        rel = np.linalg.norm(residual(lv, x, f)) / nf
        hist.append(rel)
        if not np.isfinite(rel):
            status = "nonfinite"
            break
        if rel > 1e6:
            status = "diverged"
            break
        status = "ok" if rel <= tol else "noconv"
    return SolveResult(x, it, rel, hist, status)


# ---------------------------------------------------------------------------
# the error norm of the experiments (Section 6)
# ---------------------------------------------------------------------------

def l_norm(lv: Level, e: np.ndarray) -> float:
    """||e||_L = (L e, e)^{1/2} with L = diag(Ahat, Shat); the pressure part of
    e is taken mean-free first (the constant is not part of P_k)."""
    e = lv.project_mean(e)
    return float(np.sqrt(e @ (lv.Ldiag * e)))


def error_reduction_run(h: Hierarchy, xstar: np.ndarray, prm: Params, eps: float = 1e-9,
                        maxit: int = 200, x0: np.ndarray | None = None):
    """The measurement protocol of Section 6: iterate from x0 (zero by default)
    on f = A x*, until the L-norm of the error has dropped by eps.  Returns the
    number of iterates n and the mean rate q = (|e_n| / |e_0|)^(1/n); n is None
    when the error grows by 1e6 (divergence) or maxit is hit."""
    lv = h.top
    f = lv.calA @ xstar
    x = np.zeros(lv.n) if x0 is None else x0.copy()
    e0 = l_norm(lv, x - xstar)
    e = e0
    for n in range(1, maxit + 1):
        x = top_cycle(h, x, f, prm)
        e = l_norm(lv, x - xstar)
        if not np.isfinite(e) or e > 1e6 * e0:
            return None, float("inf")
        if e <= eps * e0:
            return n, (e / e0) ** (1.0 / n)
    return None, (e / e0) ** (1.0 / maxit)
