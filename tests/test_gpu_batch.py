"""GPU tests of batched solves: every instance of a batch must reach the same
iterates as when it is solved alone (same kernels and arithmetic per node;
only the tile decomposition and hence the order of the reductions differ),
for equal and uneven sizes, both smoothers, V and W cycles, and the
mixed-precision refinement; and the batched result must solve the oracle's
discrete system."""
import numpy as np
import pytest
import torch

from oracle import multigrid as mg
from paper_1502_04070_amd import Batch, inputs
from tests import lattice as lat
from tests.test_gpu_ops import dev, gpu_hier, host, oracle_level

pytestmark = pytest.mark.gpu


def _loads(hs, seeds, kind="normal"):
    out = []
    for h, sd in zip(hs, seeds):
        N = h.level_N()
        F, G = inputs.normal_fg(N, sd) if kind == "normal" else inputs.uniform_f(N, sd)
        # compatible data: remove the P1-weighted mean of g before loading
        Gd = dev(G)
        h.project_mean(Gd)
        fu, gp = h.load(dev(F), Gd)
        out.append((fu, gp))
    return out


def _check_batch_vs_single(Ns, betas, rtol=1e-9, mixed=False, **kw):
    print(f"batch Ns={Ns} betas={betas} kw={kw} mixed={mixed}", flush=True)
    B = Batch(Ns, betas, **kw)
    loads = _loads(B.instances, range(len(Ns)))
    fus = [a for a, _ in loads]
    gps = [b for _, b in loads]
    solve = B.solve_mixed if mixed else B.solve
    us, ps, infos = solve(fus, gps, rtol=rtol, maxit=400)
    assert all(i.status == "ok" for i in infos), infos
    for k, (N, beta) in enumerate(zip(Ns, betas)):
        h = gpu_hier(N, beta, **kw)
        fu, gp = fus[k], gps[k]
        single = h.solve_mixed if mixed else h.solve
        U, P, info = single(fu, gp, rtol=rtol, maxit=400)
        assert abs(info.iters - infos[k].iters) <= 1, (k, info.iters, infos[k].iters)
        if info.iters == infos[k].iters:
            du = float((U - us[k]).abs().max()) / max(float(U.abs().max()), 1e-300)
            dp = float((P - ps[k]).abs().max()) / max(float(P.abs().max()), 1e-300)
            assert du <= 1e-12 and dp <= 1e-12, (k, du, dp)
    return B, us, ps, infos, fus, gps


def test_equal_size_beta_sweep_batch():
    """The five beta values of the h = 1/128 sweep in one batch."""
    betas = [0.0, 1.0, 1e2, 1e4, 1e6]
    _check_batch_vs_single([128] * 5, betas, rtol=1e-8)


def test_uneven_sizes_batch_matches_single_and_oracle():
    Ns = [16, 32, 64, 128, 32, 64]
    betas = [10.0 ** e for e in [-2, 0.5, 2, 4, 6, 1]]
    B, us, ps, infos, fus, gps = _check_batch_vs_single(Ns, betas, rtol=1e-10)
    # instance 2 against the oracle's direct solution of the same load vector
    k = 2
    oh = oracle_level(Ns[k], betas[k], 2)
    d = oh.discs[-1]
    f = lat.from_lattice(d, host(fus[k]), host(gps[k]))
    xd = oh.top.project_mean(oh.top.direct_solve(f))
    got = lat.from_lattice(d, host(us[k]), host(ps[k]))
    assert np.linalg.norm(got - xd) <= 1e-7 * np.linalg.norm(xd)


def test_uzawa_batch():
    _check_batch_vs_single([32, 64, 64], [1.0, 1e3, 0.0], smoother="uzawa", nu_pre=3, nu_post=3)


def test_w_cycle_uneven_batch():
    _check_batch_vs_single([32, 64, 128], [1.0, 1e2, 1e5], gamma=2)


def test_mixed_precision_batch():
    _check_batch_vs_single([64, 128], [1.0, 1e4], rtol=1e-10, mixed=True)


def test_batch_with_tiny_instances():
    """Instances whose whole hierarchy fits the single-workgroup kernel."""
    _check_batch_vs_single([4, 8, 16, 32], [1.0, 2.0, 3.0, 4.0])


def test_batch_rejects_bad_sizes():
    from paper_1502_04070_amd import _lib
    with pytest.raises(_lib.SmgError):
        Batch([32, 48], [1.0, 1.0])
