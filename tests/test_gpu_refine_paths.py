"""GPU tests of the solve-loop variants:

* FP32 cycles in FP64 refinement take two forms: where the cycle's last
  smoothing step on the finest level is a single fused NE launch, that launch
  adds its result to the FP64 iterate; otherwise (two steps per launch, the
  Uzawa smoother) a separate pass does.  The two schedules used here differ
  also in how the FP32 cycle groups its steps into launches, which changes
  the FP32 rounding (about 1e-7 of each update) but not the FP64 solution:
  both forms take the same number of steps to the same solution, single and
  batched.
* rtol = 0 runs exactly maxit iterates (the loop launches them without
  host checks), ends with status noconv and reports the same history as a
  tolerance no solve reaches (1e-11: tolerances below it switch the coarse
  levels from their dense map to the level-by-level kernel).
* The last smoothing step with the residual pass fused into it gives the
  same iterates and residual history as the separate pass.
"""
import numpy as np
import pytest

from paper_1502_04070_amd import Batch, Hierarchy, inputs
from tests.test_gpu_ops import dev

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float((a - b).abs().max()) / max(float(b.abs().max()), 1e-300)


def _load(h, seed):
    F, G = inputs.normal_fg(h.level_N(), seed)
    Gd = dev(G)
    h.project_mean(Gd)
    return h.load(dev(F), Gd)


@pytest.mark.parametrize("beta", [1.0, 1e4])
def test_fp32_refinement_same_with_and_without_the_fused_update(beta):
    N = 64
    print(f"refine paths N={N} beta={beta}", flush=True)
    # 8 x 8 tiles: the last two steps share a launch (separate update pass);
    # 16 x 8 tiles, one step per launch: the last launch adds to x
    ha = Hierarchy(N, beta, schedule={"tile_x": 8, "fuse_depth": 2})
    hb = Hierarchy(N, beta, schedule={"tile_x": 16, "fuse_depth": 1})
    fu, gp = _load(ha, 3)
    Ua, Pa, ia = ha.solve_mixed(fu, gp, rtol=1e-11, maxit=300)
    Ub, Pb, ib = hb.solve_mixed(fu, gp, rtol=1e-11, maxit=300)
    assert ia.status == ib.status == "ok"
    assert abs(ia.iters - ib.iters) <= 1, (ia.iters, ib.iters)
    # FP32 rounding of the cycle: about 1e-7 of the residual in early steps
    assert np.allclose(ia.history[:20], ib.history[:20], rtol=1e-5, atol=0)
    assert _rel(Ub, Ua) <= 1e-9 and _rel(Pb, Pa) <= 1e-9, (_rel(Ub, Ua), _rel(Pb, Pa))
    # and both reach the FP64 solve's solution
    U64, P64, _ = ha.solve(fu, gp, rtol=1e-11, maxit=300)
    assert _rel(Ub, U64) <= 1e-9 and _rel(Pb, P64) <= 1e-9


def test_batched_fp32_refinement_same_with_and_without_the_fused_update():
    Ns, betas = [32, 64, 128], [1.0, 1e3, 0.5]
    print(f"batched refine paths Ns={Ns}", flush=True)
    Ba = Batch(Ns, betas, schedule={"tile_x": 8, "fuse_depth": 2})
    Bb = Batch(Ns, betas, schedule={"tile_x": 16, "fuse_depth": 1})
    loads = [_load(h, sd) for h, sd in zip(Ba.instances, range(3))]
    fus = [a for a, _ in loads]
    gps = [b for _, b in loads]
    ua, pa, ia = Ba.solve_mixed(fus, gps, rtol=1e-10, maxit=300)
    ub, pb, ib = Bb.solve_mixed(fus, gps, rtol=1e-10, maxit=300)
    for k in range(3):
        assert ia[k].status == ib[k].status == "ok"
        assert abs(ia[k].iters - ib[k].iters) <= 1, (k, ia[k].iters, ib[k].iters)
        assert _rel(ub[k], ua[k]) <= 1e-8 and _rel(pb[k], pa[k]) <= 1e-8, k


def test_rtol_zero_runs_maxit_iterates():
    N, beta = 32, 1.0
    print(f"rtol 0 N={N}", flush=True)
    h = Hierarchy(N, beta)
    fu, gp = _load(h, 5)
    U0, P0, i0 = h.solve(fu, gp, rtol=0.0, maxit=9)
    # a tolerance no solve reaches in 9 iterates, at or above 1e-11 so that
    # both runs apply the same (dense) coarse map
    U1, P1, i1 = h.solve(fu, gp, rtol=1e-11, maxit=9)
    assert i0.iters == i1.iters == 9 and len(i0.history) == 9
    assert i0.status == i1.status == "noconv"
    assert np.array_equal(i0.history, i1.history)
    assert _rel(U0, U1) == 0.0 and _rel(P0, P1) == 0.0
    B = Batch([32, 64], [1.0, 1e2])
    loads = [_load(hh, sd) for hh, sd in zip(B.instances, (5, 6))]
    us, ps, infos = B.solve([a for a, _ in loads], [b for _, b in loads], rtol=0.0, maxit=7)
    assert [i.iters for i in infos] == [7, 7] and all(i.status == "noconv" for i in infos)


@pytest.mark.parametrize("domain", ["square", "l_shape"])
def test_fused_last_step_residual_matches_separate_pass(domain):
    """16 x 8 tiles: the last smoothing step also forms the residual pieces
    (k_ne_res); 8 x 8 tiles with one step per launch: a separate residual
    pass does.  Same iterates, same residual history to rounding."""
    N, beta = 128, 10.0
    print(f"fused residual N={N} domain={domain}", flush=True)
    ha = Hierarchy(N, beta, domain=domain, schedule={"tile_x": 16, "fuse_depth": 1})
    hb = Hierarchy(N, beta, domain=domain, schedule={"tile_x": 8, "fuse_depth": 1})
    fu, gp = _load(ha, 11)
    Ua, Pa, ia = ha.solve(fu, gp, rtol=1e-10, maxit=300)
    Ub, Pb, ib = hb.solve(fu, gp, rtol=1e-10, maxit=300)
    assert ia.status == ib.status == "ok"
    assert ia.iters == ib.iters, (ia.iters, ib.iters)
    # equal to rounding of the residual itself (about 1e-15 of ||F||), which
    # dominates the last, smallest entries
    assert np.allclose(ia.history, ib.history, rtol=1e-9, atol=1e-14)
    assert _rel(Ua, Ub) <= 1e-12 and _rel(Pa, Pb) <= 1e-12, (_rel(Ua, Ub), _rel(Pa, Pb))
