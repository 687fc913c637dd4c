"""Pins of the oracle's implicit Euler step (Section 1: the generalized problem
is what an implicit time step leaves to solve), by properties of the time
discretization that do not restate its formula:

* a stationary Stokes solution (beta = 0) is a fixed point of every step
  with the same data;
* without data the kinetic energy u^T M u never grows (the discrete
  divergence of each new velocity is zero, so the pressure does no work);
* from a divergence-free velocity, as dt -> 0 the difference quotient
  (u^{n+1} - u^n) / dt tends to the rate of the semi-discrete problem, with
  an error proportional to dt (first order);
* as dt -> infinity the step tends to the stationary solution.
"""
import numpy as np

from oracle import timestep
from oracle.multigrid import Hierarchy, Level


def _level(beta, lev=2):
    return Hierarchy("same_diag", lev, beta, n0=2).top


def _data(lv, seed):
    rng = np.random.default_rng(seed)
    d = lv.disc
    return rng.standard_normal((2, d.n2)), rng.standard_normal(lv.nu2)


def test_stationary_solution_is_a_fixed_point():
    lv0 = _level(0.0)
    f, _ = _data(lv0, 1)
    xs = lv0.project_mean(lv0.direct_solve(np.concatenate(lv0.disc.load(f, np.zeros(lv0.disc.n1)))))
    for beta in (1.0, 40.0, 1e4):
        lv = Level(lv0.disc, beta)
        x = timestep.step(lv, xs[: lv.nu2], f)
        assert np.linalg.norm(x - xs) <= 1e-11 * np.linalg.norm(xs), beta


def test_energy_never_grows_without_data():
    lv = _level(20.0)
    _, u = _data(lv, 2)
    M = lv.disc.mass_u()
    e = [u @ (M @ u)]
    for x in timestep.march(lv, u, 6):
        un = x[: lv.nu2]
        e.append(un @ (M @ un))
        assert np.linalg.norm(lv.B @ un) <= 1e-12 * np.linalg.norm(un)
    assert all(b <= a * (1 + 1e-12) for a, b in zip(e, e[1:])), e
    assert e[-1] < 0.9 * e[0]


def test_small_steps_are_first_order():
    lv0 = _level(0.0)
    f, u = _data(lv0, 3)
    # start from a discretely divergence-free velocity (a random one is
    # projected within the first step, so its difference quotient grows like 1/dt)
    u = timestep.step(Level(lv0.disc, 1.0), u, f)[: lv0.nu2]
    # steps far below the stiffest time scale of the h = 1/8 grid
    rates = []
    for dt in (4e-6, 2e-6, 1e-6):
        lv = Level(lv0.disc, 1.0 / dt)
        rates.append((timestep.step(lv, u, f)[: lv.nu2] - u) / dt)
    r0, r1, r2 = rates
    d1, d2 = np.linalg.norm(r1 - r0), np.linalg.norm(r2 - r1)
    assert d1 <= 0.02 * np.linalg.norm(r1)
    # halving dt halves the change of the difference quotient (first order)
    assert 0.45 < d2 / d1 < 0.55, (d1, d2)


def test_long_steps_tend_to_the_stationary_solution():
    lv0 = _level(0.0)
    f, u = _data(lv0, 4)
    xs = lv0.project_mean(lv0.direct_solve(np.concatenate(lv0.disc.load(f, np.zeros(lv0.disc.n1)))))
    errs = []
    for beta in (1e-2, 1e-4):
        x = timestep.step(Level(lv0.disc, beta), u, f)
        errs.append(np.linalg.norm(x - xs) / np.linalg.norm(xs))
    assert errs[1] < 0.02 * errs[0] and errs[1] < 1e-3, errs
