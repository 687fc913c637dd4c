"""GPU tests of implicit Euler stepping (Section 1: the generalized problem with
beta = 1/dt is one implicit time step): every step against the oracle's step
(a sparse direct solve of the same system), batched against single."""
import numpy as np
import pytest
import torch

from oracle import timestep as ots
from paper_1502_04070_amd import inputs
from paper_1502_04070_amd.timestep import BatchImplicitEuler, ImplicitEuler
from tests import lattice as lat
from tests.test_gpu_ops import dev, host, oracle_level

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("mixed", [False, True], ids=["fp64", "fp32_refine"])
@pytest.mark.parametrize("dt", [1e-3, 0.1])
def test_steps_match_oracle(dt, mixed):
    N = 32
    print(f"implicit steps N={N} dt={dt} mixed={mixed}", flush=True)
    oh = oracle_level(N, 1.0 / dt, 2)
    lv, d = oh.top, oh.discs[-1]
    F, _ = inputs.normal_fg(N, seed=80, with_g=False)
    u0, _ = inputs.random_state(N, seed=81)
    G = np.zeros((N + 1, N + 1))
    fn, _ = lat.lattice_to_nodal(d, F, G)
    xs = ots.march(lv, lat.from_lattice(d, u0, G)[: lv.nu2], 4, fn)
    ts = ImplicitEuler(N, dt, u0=dev(u0), mixed=mixed)
    Fd = dev(F)
    for k in range(4):
        info = ts.step(Fd, rtol=1e-12 if mixed else 1e-13, maxit=300)
        got = lat.from_lattice(d, host(ts.u), host(ts.p))
        err = np.linalg.norm(got - xs[k]) / np.linalg.norm(xs[k])
        assert err <= 1e-9, (k, err, info)
    assert ts.t == pytest.approx(4 * dt)


def test_step_with_divergence_data_and_warm_start():
    """g != 0 (compatible): B u^{n+1} = M_P g; a second step from the new state
    with the same data converges in fewer iterates than the first."""
    N, dt = 32, 0.05
    oh = oracle_level(N, 1.0 / dt, 2)
    lv, d = oh.top, oh.discs[-1]
    F, G = inputs.normal_fg(N, seed=82)
    gn = lat.lattice_to_nodal(d, F, G)[1]
    gn = gn - (lv.m @ gn) / lv.m.sum()
    _, Gc = lat.nodal_to_lattice(d, np.zeros((2, d.n2)), gn)
    fn, _ = lat.lattice_to_nodal(d, F, G)
    x1 = ots.step(lv, np.zeros(lv.nu2), fn, gn)
    ts = ImplicitEuler(N, dt)
    i1 = ts.step(dev(F), dev(Gc), rtol=1e-13, maxit=300)
    got = lat.from_lattice(d, host(ts.u), host(ts.p))
    assert np.linalg.norm(got - x1) <= 1e-9 * np.linalg.norm(x1)
    i2 = ts.step(dev(F), dev(Gc), rtol=1e-13, maxit=300)
    assert i2.iters < i1.iters


@pytest.mark.parametrize("mixed", [False, True], ids=["fp64", "fp32_refine"])
@pytest.mark.parametrize("domain", ["square", "l_shape", "union_jack"])
def test_batched_steps_match_single(domain, mixed):
    Ns, dts = [32, 64, 32], [1e-2, 1e-3, 1.0]
    u0s = [dev(inputs.random_state(N, seed=90 + k)[0]) for k, N in enumerate(Ns)]
    Fs = [dev(inputs.normal_fg(N, seed=95 + k, with_g=False)[0]) for k, N in enumerate(Ns)]
    bt = BatchImplicitEuler(Ns, dts, u0s=u0s, domain=domain, mixed=mixed)
    singles = [ImplicitEuler(N, dt, u0=u0, domain=domain, mixed=mixed) for N, dt, u0 in zip(Ns, dts, u0s)]
    for _ in range(3):
        binfo = bt.step(Fs, rtol=1e-12, maxit=300)
        for k, ts in enumerate(singles):
            info = ts.step(Fs[k], rtol=1e-12, maxit=300)
            assert abs(info.iters - binfo[k].iters) <= 1
            du = float((ts.u - bt.us[k]).abs().max()) / float(ts.u.abs().max())
            assert du <= 1e-10, (k, du)
