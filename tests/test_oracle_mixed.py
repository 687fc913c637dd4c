"""Pins of the oracle's FP32-cycle / FP64-refinement solver.

* Refinement reaches an FP64 residual far below FP32 rounding, and its
  solution matches the FP64 sparse direct solve.
* The FP32 cycle really runs in single precision at every level: every
  smoothing step (including the post-smoothing steps, which see the iterate
  with the prolongated coarse correction added) and every restricted defect
  is float32, and only the coarsest-level solve (FP64 by design)
  sees float64 operands.  An FP64 cycle stays float64 throughout.
* One FP32 correction cycle differs from the FP64 cycle by FP32 rounding:
  more than FP64 rounding could explain (so the single-precision arithmetic is
  present), less than the error of a wrong step (a linear stationary iterate
  x + C (F - calA x) is the same either way in exact arithmetic).
"""
import numpy as np
import pytest

from oracle import mixed
from oracle import multigrid as mg


def _problem(beta, levels=3, seed=2):
    h = mg.Hierarchy("same_diag", levels, beta, n0=2)
    rng = np.random.default_rng(seed)
    F = rng.uniform(-1, 1, h.top.n)
    F[h.top.nu2:] -= F[h.top.nu2:].mean()
    x0 = h.top.project_mean(rng.standard_normal(h.top.n))
    return h, F, x0


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


def _record_dtypes(monkeypatch):
    """Wrap the cycle's building blocks and record the dtype of every operand."""
    seen = {"smooth": [], "restrict": [], "coarse_in": [], "coarse_out": []}
    smooth, restrict = mg.smooth, mg.restrict_residual

    def smooth_rec(lv, x, f, prm, k=None):
        out = smooth(lv, x, f, prm, k)
        seen["smooth"].append((k, x.dtype, f.dtype, out.dtype))
        return out

    def restrict_rec(h, k, x, f):
        out = restrict(h, k, x, f)
        seen["restrict"].append((k, out.dtype))
        return out

    monkeypatch.setattr(mg, "smooth", smooth_rec)
    monkeypatch.setattr(mg, "restrict_residual", restrict_rec)
    base_solve = mg.Level.direct_solve

    def direct_rec(self, f):
        seen["coarse_in"].append(f.dtype)
        return base_solve(self, f)

    monkeypatch.setattr(mg.Level, "direct_solve", direct_rec)
    base32 = mixed._Level32.direct_solve

    def direct32_rec(self, f):
        out = base32(self, f)
        seen["coarse_out"].append(out.dtype)
        return out

    monkeypatch.setattr(mixed._Level32, "direct_solve", direct32_rec)
    return seen


@pytest.mark.parametrize("prm", [mg.Params(), mg.Params.uzawa(gamma=2)], ids=["ne_V22", "uzawa_W33"])
def test_fp32_cycle_is_single_precision_at_every_level(monkeypatch, prm):
    h, F, _ = _problem(10.0)
    seen = _record_dtypes(monkeypatch)
    d = mg.cycle(mixed._Hierarchy32(h), h.L, np.zeros(h.top.n, np.float32), F.astype(np.float32), prm)
    assert d.dtype == np.float32
    steps = (prm.nu_pre + prm.nu_post)
    # every smoothing step of every level (levels 1..L), gamma^(L-k) visits of level k
    assert len(seen["smooth"]) == steps * sum(prm.gamma ** (h.L - k) for k in range(1, h.L + 1))
    assert {k for k, *_ in seen["smooth"]} == set(range(1, h.L + 1))
    assert all(dx == df == do == np.float32 for _, dx, df, do in seen["smooth"]), seen["smooth"]
    assert all(dt == np.float32 for _, dt in seen["restrict"])
    # the coarsest level is solved in FP64 (its operand is upcast) and handed back in FP32
    assert seen["coarse_in"] and all(dt == np.float64 for dt in seen["coarse_in"])
    assert seen["coarse_out"] and all(dt == np.float32 for dt in seen["coarse_out"])


def test_fp64_cycle_stays_double(monkeypatch):
    h, F, x0 = _problem(10.0)
    seen = _record_dtypes(monkeypatch)
    x = mg.cycle(h, h.L, x0, F, mg.Params())
    assert x.dtype == np.float64
    assert all(dx == df == do == np.float64 for _, dx, df, do in seen["smooth"])
    assert all(dt == np.float64 for _, dt in seen["restrict"])


@pytest.mark.parametrize("beta", [0.0, 10.0, 1e4])
@pytest.mark.parametrize("prm", [mg.Params(), mg.Params.uzawa()], ids=["ne", "uzawa"])
def test_fp32_correction_differs_from_fp64_cycle_by_fp32_rounding(beta, prm):
    """x + cycle32(F - calA x) against the FP64 cycle from x: the relative
    difference (to the update) lies between 1e-9 (above FP64 rounding, about
    1e-15, so FP32 arithmetic is present) and 1e-5 (a few hundred FP32 units,
    far below the effect of a wrong term)."""
    h, F, x0 = _problem(beta)
    x64 = mg.top_cycle(h, x0, F, prm)
    r = F - h.top.calA @ x0
    d = mg.cycle(mixed._Hierarchy32(h), h.L, np.zeros(h.top.n, np.float32), r.astype(np.float32), prm)
    x32 = h.top.project_mean(x0 + d.astype(np.float64))
    rel = np.linalg.norm(x32 - x64) / np.linalg.norm(x64 - x0)
    assert 1e-9 <= rel <= 1e-5, rel


def test_fp32_cycle_from_a_nonzero_iterate():
    """The same bracket for a cycle started from an FP32 iterate (the form the
    library's FP32 cycle entry point takes)."""
    h, F, x0 = _problem(1.0, seed=7)
    x64 = mg.top_cycle(h, x0.astype(np.float32).astype(np.float64), F.astype(np.float32).astype(np.float64),
                       mg.Params())
    x32 = mg.cycle(mixed._Hierarchy32(h), h.L, x0.astype(np.float32), F.astype(np.float32), mg.Params())
    assert x32.dtype == np.float32
    x32 = h.top.project_mean(x32.astype(np.float64))
    upd = np.linalg.norm(x64 - h.top.project_mean(x0.astype(np.float32).astype(np.float64)))
    rel = np.linalg.norm(x32 - x64) / upd
    assert 1e-9 <= rel <= 1e-5, rel
