"""Pins of the oracle's FP32-cycle / FP64-refinement solver: it reaches an FP64
residual far below FP32 rounding, its solution matches the FP64 sparse direct
solve, and one FP32 correction cycle equals one FP64 cycle to FP32 rounding
(a linear stationary iterate x + C (F - calA x) is the same either way)."""
import numpy as np

from oracle import mixed
from oracle import multigrid as mg


def test_ir_reaches_fp64_accuracy():
    for beta in [1.0, 1e4]:
        h = mg.Hierarchy("same_diag", 3, beta, n0=2)
        rng = np.random.default_rng(1)
        F = rng.uniform(-1, 1, h.top.n)
        F[h.top.nu2:] -= F[h.top.nu2:].mean()
        x, it, hist = mixed.ir_solve(h, F, mg.Params(), tol=1e-11)
        assert hist[-1] <= 1e-11
        xd = h.top.project_mean(h.top.direct_solve(F))
        assert np.linalg.norm(x - xd) <= 1e-8 * np.linalg.norm(xd)


def test_fp32_correction_equals_fp64_cycle_to_fp32_rounding():
    h = mg.Hierarchy("same_diag", 3, 10.0, n0=2)
    rng = np.random.default_rng(2)
    F = rng.uniform(-1, 1, h.top.n)
    F[h.top.nu2:] -= F[h.top.nu2:].mean()
    x0 = h.top.project_mean(rng.standard_normal(h.top.n))
    x64 = mg.top_cycle(h, x0, F, mg.Params())
    r = F - h.top.calA @ x0
    d = mg.cycle(mixed._Hierarchy32(h), h.L, np.zeros(h.top.n, np.float32), r.astype(np.float32), mg.Params())
    x32 = h.top.project_mean(x0 + d.astype(np.float64))
    assert np.linalg.norm(x32 - x64) <= 1e-5 * np.linalg.norm(x64 - x0)
