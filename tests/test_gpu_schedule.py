"""GPU tests of the launch schedule: every schedule the autotuner may pick
runs the same iterate (same iterate count, iterates equal to rounding), and
the autotuner returns the fastest of the candidates it timed."""
import numpy as np
import pytest
import torch

from paper_1502_04070_amd import Batch, Hierarchy, inputs
from paper_1502_04070_amd import tune
from tests.test_gpu_ops import dev

pytestmark = pytest.mark.gpu

SCHEDULES = [{"fuse_depth": 1}, {"fuse_depth": 2, "tile_x": 16}, {"tile_x": 8},
             {"coarse_max_n": 2}, {"coarse_max_n": 4, "fuse_depth": 1}, {"coarse_max_n": 16},
             {"coarse_max_n": 16, "tile_x": 8, "fuse_depth": 2}]


def _rel(a, b):
    return float((a - b).abs().max()) / max(float(b.abs().max()), 1e-300)


@pytest.mark.parametrize("smoother,nu", [("ne", 2), ("ne", 3), ("uzawa", 3)])
def test_every_schedule_runs_the_same_iterate(smoother, nu):
    N, beta = 128, 30.0
    print(f"schedules {smoother} nu={nu}", flush=True)
    F, G = inputs.normal_fg(N, seed=7)
    ref = Hierarchy(N, beta, smoother=smoother, nu_pre=nu, nu_post=nu)
    Gd = dev(G)
    ref.project_mean(Gd)
    fu, gp = ref.load(dev(F), Gd)
    U0, P0, i0 = ref.solve(fu, gp, rtol=1e-9, maxit=300)
    assert i0.status == "ok"
    for sch in SCHEDULES:
        h = Hierarchy(N, beta, smoother=smoother, nu_pre=nu, nu_post=nu, schedule=sch)
        U, P, info = h.solve(fu, gp, rtol=1e-9, maxit=300)
        assert info.iters == i0.iters, (sch, info.iters, i0.iters)
        assert _rel(U, U0) <= 1e-12 and _rel(P, P0) <= 1e-12, (sch, _rel(U, U0), _rel(P, P0))


def test_batched_schedules_match_default():
    Ns, betas = [32, 64, 128], [1.0, 1e3, 0.5]
    ref = Batch(Ns, betas)
    loads = []
    for h, sd in zip(ref.instances, range(3)):
        F, G = inputs.normal_fg(h.level_N(), sd)
        Gd = dev(G)
        h.project_mean(Gd)
        loads.append(h.load(dev(F), Gd))
    fus = [a for a, _ in loads]
    gps = [b for _, b in loads]
    us0, ps0, infos0 = ref.solve(fus, gps, rtol=1e-9, maxit=300)
    for sch in SCHEDULES[:4]:
        B = Batch(Ns, betas, schedule=sch)
        us, ps, infos = B.solve(fus, gps, rtol=1e-9, maxit=300)
        for k in range(3):
            assert infos[k].iters == infos0[k].iters, (sch, k)
            assert _rel(us[k], us0[k]) <= 1e-12 and _rel(ps[k], ps0[k]) <= 1e-12, (sch, k)


def test_autotune_returns_the_fastest_candidate(tmp_path, monkeypatch):
    monkeypatch.setenv("SMG_TUNE_CACHE", str(tmp_path / "schedules.json"))
    Ns, betas = [64, 64], [1.0, 100.0]
    sched, rec = tune.schedule_for(Ns, betas, iters=5)
    cands = rec["candidates"]
    assert len(cands) >= 10
    assert all(c["ms_per_iterate"] > 0 for c in cands)
    best = min(cands, key=lambda c: c["ms_per_iterate"])
    assert rec["ms_per_iterate"] == pytest.approx(best["ms_per_iterate"])
    assert sched == {k: best[k] for k in ("fuse_depth", "coarse_max_n", "tile_x")}
    # the second request is served from the cache file
    sched2, rec2 = tune.schedule_for(Ns, betas, iters=5)
    assert sched2 == sched and rec2["candidates"] == cands
    # the schedule is usable as is
    B = Batch(Ns, betas, schedule=sched)
    assert len(B) == 2


def test_bad_schedules_are_rejected():
    with pytest.raises(Exception, match="tile_x"):
        Hierarchy(32, 1.0, schedule={"tile_x": 4})
    with pytest.raises(ValueError, match="unknown schedule field"):
        Hierarchy(32, 1.0, schedule={"tiles": 8})
