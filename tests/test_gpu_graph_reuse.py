"""GPU tests of captured iterates reused across solves.

* A solve whose maxit outgrows the history buffer drops the captured
  iterates (they write the old buffer) and captures them again: the returned
  residual history equals the oracle's, before and after the growth, for the
  FP64 and the FP32-refined solver.
* A batch solved twice with different right-hand sides reuses the iterate
  graphs it captured for subsets of still-running instances: both runs equal
  single solves.
* Damping changed on one instance through its batch handle reaches the
  batch's next solve (its plans and graphs are made again).
"""
import numpy as np
import pytest

from oracle import multigrid as mg
from paper_1502_04070_amd import Batch, inputs
from tests import lattice as lat
from tests.test_gpu_batch import _loads
from tests.test_gpu_cycle import _rhs
from tests.test_gpu_ops import gpu_hier, host, oracle_level

pytestmark = pytest.mark.gpu


def test_history_buffer_growth_recaptures_iterates():
    N, beta = 32, 1.0
    print(f"history growth N={N}", flush=True)
    oh = oracle_level(N, beta, 2)
    gh = gpu_hier(N, beta)
    F, G = inputs.uniform_f(N, seed=3)
    f, FU, GP = _rhs(gh, oh, F, G)
    res8 = mg.solve(oh, f, mg.Params(), tol=1e-8, maxit=300)
    res11 = mg.solve(oh, f, mg.Params(), tol=1e-11, maxit=300)
    # 1: captured with the initial buffer (maxit within it)
    _, _, i1 = gh.solve(FU, GP, rtol=1e-8, maxit=200)
    # 2: maxit beyond the buffer: new buffer, iterates captured again
    U, P, i2 = gh.solve(FU, GP, rtol=1e-11, maxit=1500)
    # 3: the same buffer again (graph reused)
    _, _, i3 = gh.solve(FU, GP, rtol=1e-8, maxit=1500)
    for info, res in ((i1, res8), (i2, res11), (i3, res8)):
        assert info.status == "ok"
        assert info.iters == res.iters, (info.iters, res.iters)
        # relative residuals agree to 1e-7 of their size, down to FP64
        # rounding of the residual itself (about 1e-15 of ||F||) at the end
        assert np.allclose(info.history, res.history, rtol=1e-7, atol=1e-14)
    got = lat.from_lattice(oh.discs[-1], host(U), host(P))
    assert np.linalg.norm(got - res11.x) <= 1e-10 * np.linalg.norm(res11.x)
    # the FP32-refined solver after a further growth of the buffer
    _, _, m1 = gh.solve_mixed(FU, GP, rtol=1e-10, maxit=300)
    _, _, m2 = gh.solve_mixed(FU, GP, rtol=1e-10, maxit=2500)
    assert m1.status == m2.status == "ok"
    assert m1.iters == m2.iters and len(m2.history) == m2.iters
    assert np.allclose(m1.history, m2.history, rtol=1e-6, atol=0)
    assert m2.history[-1] <= 1e-10


def _single(N, beta, fu, gp, rtol, tau=None):
    h = gpu_hier(N, beta)
    if tau is not None:
        h.set_damping(-1, tau)
    return h.solve(fu, gp, rtol=rtol, maxit=400)


def _compare(us, ps, infos, singles):
    for k, (U, P, info) in enumerate(singles):
        assert infos[k].status == "ok"
        assert abs(info.iters - infos[k].iters) <= 1, (k, info.iters, infos[k].iters)
        if info.iters == infos[k].iters:
            du = float((U - us[k]).abs().max()) / max(float(U.abs().max()), 1e-300)
            dp = float((P - ps[k]).abs().max()) / max(float(P.abs().max()), 1e-300)
            assert du <= 1e-12 and dp <= 1e-12, (k, du, dp)


def test_batch_reuses_subset_graphs_and_sees_damping_changes():
    Ns = [16, 32, 64, 32, 16, 64]
    betas = [1e6, 1.0, 1e2, 1e5, 0.0, 1e4]
    rtol = 1e-9
    print(f"batch reuse Ns={Ns}", flush=True)
    B = Batch(Ns, betas)
    for run, seeds in enumerate((range(0, 6), range(10, 16))):
        loads = _loads(B.instances, seeds)
        fus = [a for a, _ in loads]
        gps = [b for _, b in loads]
        us, ps, infos = B.solve(fus, gps, rtol=rtol, maxit=400)
        its = [i.iters for i in infos]
        print(f"  run {run}: iterates {its}", flush=True)
        assert len(set(its)) > 1          # uneven: subsets of instances were captured
        _compare(us, ps, infos, [_single(N, b, fu, gp, rtol) for N, b, fu, gp in zip(Ns, betas, fus, gps)])
    # damping of instance 1 changed through its handle: the batch plans again
    B.instances[1].set_damping(-1, 0.3)
    us, ps, infos = B.solve(fus, gps, rtol=rtol, maxit=400)
    singles = [_single(N, b, fu, gp, rtol, tau=0.3 if k == 1 else None)
               for k, (N, b, fu, gp) in enumerate(zip(Ns, betas, fus, gps))]
    _compare(us, ps, infos, singles)
    default = _single(Ns[1], betas[1], fus[1], gps[1], rtol)[2]
    print(f"  instance 1: tau 0.3 -> {infos[1].iters} iterates, default {default.iters}", flush=True)
    assert default.iters != singles[1][2].iters      # the change is visible in the result
