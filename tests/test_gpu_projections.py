"""GPU tests of the pressure projections on every grid: the mean projection
Pi p = p - 1 (m^T p) / (m^T 1) and its transpose Pi^T v = v - m (1^T v) /
(m^T 1) (used by the adjoint) against the oracle's P1 weights m, and the
pairing (Pi p) . v = p . (Pi^T v); plus the kernel timer's contract."""
import numpy as np
import pytest

from oracle import multigrid as mg
from tests import lattice as lat
from tests.test_gpu_ops import dev, gpu_hier, host

pytestmark = pytest.mark.gpu

GRIDS = {"square": "same_diag", "l_shape": "l_shape", "union_jack": "union_jack"}


@pytest.mark.parametrize("N", [16, 64])
@pytest.mark.parametrize("domain", list(GRIDS))
def test_projections_match_oracle_weights(domain, N):
    oh = mg.Hierarchy(GRIDS[domain], int(round(np.log2(N // 2))), 1.0, n0=2)
    lv, d = oh.top, oh.discs[-1]
    gh = gpu_hier(N, 1.0, domain=domain)
    rng = np.random.default_rng(40 + N)
    x = rng.standard_normal(lv.n) + 2.0
    _, p = lat.to_lattice(d, x)
    _, v = lat.to_lattice(d, rng.standard_normal(lv.n) - 1.0)
    zu = np.zeros((2, 2 * N + 1, 2 * N + 1))
    pv = lat.from_lattice(d, zu, p)[lv.nu2:]
    vv = lat.from_lattice(d, zu, v)[lv.nu2:]
    P, V = dev(p), dev(v)
    gh.project_mean(P)
    gh.project_dual(V)
    ref_p = pv - (lv.m @ pv) / lv.m.sum()
    ref_v = vv - lv.m * vv.sum() / lv.m.sum()
    got_p = lat.from_lattice(d, zu, host(P))[lv.nu2:]
    got_v = lat.from_lattice(d, zu, host(V))[lv.nu2:]
    assert np.abs(got_p - ref_p).max() <= 1e-13 * np.abs(ref_p).max()
    assert np.abs(got_v - ref_v).max() <= 1e-13 * np.abs(ref_v).max()
    # the two are transposes of each other
    assert abs(got_p @ vv - pv @ got_v) <= 1e-12 * np.abs(pv).sum() * np.abs(vv).max()
    # both are projections: applying them again changes nothing
    gh.project_mean(P)
    gh.project_dual(V)
    assert np.abs(lat.from_lattice(d, zu, host(P))[lv.nu2:] - got_p).max() <= 1e-13 * np.abs(ref_p).max()
    assert np.abs(lat.from_lattice(d, zu, host(V))[lv.nu2:] - got_v).max() <= 1e-13 * np.abs(ref_v).max()


def test_kernel_timer_reports_a_positive_duration():
    gh = gpu_hier(64, 1.0)
    for which in range(4):
        ms = gh.time_kernel(which, reps=5)
        assert 0.0 < ms < 100.0, (which, ms)
