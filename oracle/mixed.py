"""FP32 multigrid cycles as the inner solver of FP64 iterative refinement.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The iterate of Section 3 is applied, in single precision, to the correction
equation calA d = r of classical iterative refinement:
    r = F - calA x            (FP64)
    d = one FP32 cycle on calA d = r from d = 0 (coarsest grid solved in FP64)
    x <- x + d, pressure mean removed (FP64)
until ||r|| <= tol ||F||.
"""
from __future__ import annotations

import numpy as np

from . import multigrid as mg


class _Level32:
    def __init__(self, lv: mg.Level):
        self.base = lv
        self.calA = lv.calA.astype(np.float32)
        self.A = lv.A.astype(np.float32)
        self.B = lv.B.astype(np.float32)
        self.Bt = lv.Bt.astype(np.float32)
        self.Ahat = lv.Ahat.astype(np.float32)
        self.Shat = lv.Shat.astype(np.float32)
        self.Ldiag = lv.Ldiag.astype(np.float32)
        self.P = None if lv.P is None else lv.P.astype(np.float32)
        self.nu2, self.n1, self.n = lv.nu2, lv.n1, lv.n

    def direct_solve(self, f):
        return self.base.direct_solve(f.astype(np.float64)).astype(np.float32)


class _Hierarchy32:
    def __init__(self, h: mg.Hierarchy):
        self.levels = [_Level32(lv) for lv in h.levels]
        self.L = h.L


def ir_solve(h: mg.Hierarchy, F: np.ndarray, prm: mg.Params, tol: float = 1e-10, maxit: int = 400):
    """Returns (x, outer iterations, relative residual history)."""
    h32 = _Hierarchy32(h)
    lv = h.top
    x = np.zeros(lv.n)
    nF = np.linalg.norm(F)
    hist = []
    if nF == 0:
        return x, 0, hist
    it = 0
    while it < maxit:
        r = F - lv.calA @ x
        rel = np.linalg.norm(r) / nF
        hist.append(rel)
        if rel <= tol:
            break
        d = mg.cycle(h32, h.L, np.zeros(lv.n, np.float32), r.astype(np.float32), prm)
        x = lv.project_mean(x + d.astype(np.float64))
        it += 1
    return x, it, hist
