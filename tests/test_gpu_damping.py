"""GPU tests of per-level damping (Section 6: tau and sigma may depend on the
level and beta): iterates with per-level values against the oracle with the
same values (fused, unfused, batched), and the damping search."""
import numpy as np
import pytest

from oracle import multigrid as mg
from paper_1502_04070_amd import Batch, Hierarchy, inputs
from paper_1502_04070_amd import tune
from tests import lattice as lat
from tests.test_gpu_cycle import _rhs
from tests.test_gpu_ops import dev, host, oracle_level

pytestmark = pytest.mark.gpu

TAUS = {"ne": (0.35, 0.30, 0.33, 0.36, 0.31, 0.38), "uzawa": (0.8, 0.7, 0.75, 0.85, 0.9, 0.8)}
SIGMAS = (0.8, 0.9, 0.7, 0.85, 0.75, 0.8)


@pytest.mark.parametrize("fused", [True, False], ids=["fused", "unfused"])
@pytest.mark.parametrize("smoother", ["ne", "uzawa"])
def test_level_damping_iterates_match_oracle(smoother, fused):
    N, beta = 64, 20.0                      # levels N = 2 ... 64
    print(f"level damping {smoother} fused={fused}", flush=True)
    nu = 2 if smoother == "ne" else 3
    taus, sigmas = TAUS[smoother], SIGMAS
    oh = oracle_level(N, beta, 2)
    prm = mg.Params(smoother, taus[0], sigmas[0], nu, nu, 1, level_tau=taus, level_sigma=sigmas)
    gh = Hierarchy(N, beta, smoother=smoother, nu_pre=nu, nu_post=nu, fused=fused,
                   damping={"tau": list(taus), "sigma": list(sigmas)})
    assert gh.damping(3) == pytest.approx((taus[3], sigmas[3]))
    F, G = inputs.normal_fg(N, seed=70)
    f, FU, GP = _rhs(gh, oh, F, G)
    d = oh.discs[-1]
    x = np.zeros(oh.top.n)
    U, P = gh.zeros()
    for it in range(3):
        x = mg.top_cycle(oh, x, f, prm)
        gh.cycle(FU, GP, U, P)
        got = lat.from_lattice(d, host(U), host(P))
        assert np.linalg.norm(got - x) <= 1e-10 * np.linalg.norm(x), it


def test_batched_level_damping_matches_single():
    Ns, betas = [32, 64], [5.0, 500.0]
    damping = {"tau": [0.35, 0.3, 0.34, 0.37, 0.32, 0.36], "sigma": [0.8] * 6}
    B = Batch(Ns, betas, damping=damping)
    loads = []
    for h, sd in zip(B.instances, range(2)):
        F, G = inputs.normal_fg(h.level_N(), sd)
        Gd = dev(G)
        h.project_mean(Gd)
        loads.append(h.load(dev(F), Gd))
    us, ps, infos = B.solve([a for a, _ in loads], [b for _, b in loads], rtol=1e-9, maxit=300)
    for k, (N, beta) in enumerate(zip(Ns, betas)):
        h = Hierarchy(N, beta, damping={"tau": damping["tau"][: h_levels(N)], "sigma": damping["sigma"][: h_levels(N)]})
        U, P, info = h.solve(loads[k][0], loads[k][1], rtol=1e-9, maxit=300)
        assert info.iters == infos[k].iters
        assert float((U - us[k]).abs().max()) <= 1e-12 * float(U.abs().max())
    # changing one level's damping afterwards changes the batch's iterate
    B.set_damping(1, 3, 0.2, 0.8)
    us2, _, infos2 = B.solve([a for a, _ in loads], [b for _, b in loads], rtol=1e-9, maxit=300)
    assert infos2[1].iters != infos[1].iters or float((us2[1] - us[1]).abs().max()) > 0


def h_levels(N, n0=2):
    return int(round(np.log2(N // n0))) + 1


def test_damping_search_does_not_lose(tmp_path, monkeypatch):
    monkeypatch.setenv("SMG_TUNE_CACHE", str(tmp_path / "t.json"))
    d, rec = tune.damping_for(32, 1e4, factors=(0.9, 1.0, 1.1))
    assert rec["rate"] <= rec["rate_default"] and rec["iterations"] <= rec["iterations_default"] + 1
    assert len(d["tau"]) == h_levels(32)
    d2, rec2 = tune.damping_for(32, 1e4, factors=(0.9, 1.0, 1.1))
    assert d2 == d
