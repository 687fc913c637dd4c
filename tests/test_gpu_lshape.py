"""GPU parity on the L-shaped domain (0,1)^2 minus [1/2,1]^2 (Section 1: the
method is defined for it, the analysis needs convexity), against the oracle's
L-shaped hierarchy.

The library keeps the square's lattice layouts; lattice points and vertices of
the removed quarter carry no unknowns.  Every input gets junk there (and on
the re-entrant edges, which are Dirichlet boundary), which must be ignored:
operators agree with the oracle's assembly to 1e-13, iterates to 1e-10, and
outputs at removed points are zero.  Sizes: n0 = 2 and 6 (24 = 6 * 4 squares
per side: 25 vertices, a ragged tail for every tile edge), up to h = 1/256.
"""
import numpy as np
import pytest
import torch

from oracle import multigrid as mg
from oracle import timestep as ots
from paper_1502_04070_amd import Batch, inputs
from tests import lattice as lat
from tests.test_gpu_cycle import PARITY, _params
from tests.test_gpu_ops import TOL, dev, gpu_hier, host, relmax

pytestmark = pytest.mark.gpu
_ORACLE = {}


def oracle_l(N, beta, n0=2):
    key = (N, beta, n0)
    if key not in _ORACLE:
        _ORACLE[key] = mg.Hierarchy("l_shape", int(round(np.log2(N // n0))), beta, n0=n0)
    return _ORACLE[key]


def gpu_l(N, beta, n0=2, **kw):
    return gpu_hier(N, beta, n0=n0, domain="l_shape", **kw)


def removed_u(N):
    """Velocity lattice points that are not unknowns on the L-shape (boundary included)."""
    a = np.arange(2 * N + 1)
    A, B = np.meshgrid(a, a)
    inner = (A > 0) & (A < 2 * N) & (B > 0) & (B < 2 * N) & ~((A >= N) & (B >= N))
    return ~inner                            # indexed [b, a]


def removed_p(N):
    i = np.arange(N + 1)
    I, J = np.meshgrid(i, i)
    return (2 * I > N) & (2 * J > N)         # indexed [j, i]


def junk(N, u, p, value=7.0):
    """Copies of (u, p) with junk at every non-unknown lattice entry."""
    u, p = u.copy(), p.copy()
    ru = removed_u(N)
    u[:, ru] = value
    p[removed_p(N)] = -value
    return u, p


def assert_clean(N, u=None, p=None):
    if u is not None:
        assert np.all(u[:, removed_u(N)] == 0)
    if p is not None:
        assert np.all(p[removed_p(N)] == 0)


def _rhs(oh, F, G):
    d = oh.discs[-1]
    fn, gn = lat.lattice_to_nodal(d, F, G)
    gn = gn - (oh.top.m @ gn) / oh.top.m.sum()
    fu, gp = d.load(fn, gn)
    f = np.concatenate([fu, gp])
    FU, GP = lat.to_lattice(d, f)
    return f, FU, GP


SIZES = [(2, 2, 1.0), (8, 2, 0.0), (24, 6, 3.0), (64, 2, 1e4), (256, 2, 1e2)]


@pytest.mark.parametrize("N,n0,beta", SIZES)
def test_apply_and_residual_on_l_shape(N, n0, beta):
    print(f"l-shape apply N={N} n0={n0} beta={beta}", flush=True)
    oh = oracle_l(N, beta, n0)
    gh = gpu_l(N, beta, n0)
    d = oh.discs[-1]
    u, p = inputs.random_state(N, seed=N + 1)
    uj, pj = junk(N, u, p)
    yu, yp = gh.apply(dev(uj), dev(pj))
    ref = oh.top.calA @ lat.from_lattice(d, u, p)
    assert relmax(lat.from_lattice(d, host(yu), host(yp)), ref) <= TOL
    assert_clean(N, host(yu), host(yp))
    fu, gp = inputs.random_state(N, seed=N + 2)
    fj, gj = junk(N, fu, gp, -3.0)
    ru, rp, n2 = gh.residual(dev(fj), dev(gj), dev(uj), dev(pj), norm=True)
    r = lat.from_lattice(d, fu, gp) - ref
    assert relmax(lat.from_lattice(d, host(ru), host(rp)), r) <= TOL
    assert abs(host(n2)[0] - r @ r) <= 1e-13 * (r @ r)
    assert_clean(N, host(ru), host(rp))


@pytest.mark.parametrize("smoother", ["ne", "uzawa"])
@pytest.mark.parametrize("N,n0,beta", [(8, 2, 1.0), (24, 6, 1e4), (64, 2, 0.0)])
def test_smoothing_steps_on_l_shape(smoother, N, n0, beta):
    oh = oracle_l(N, beta, n0)
    gh = gpu_l(N, beta, n0, smoother=smoother)
    prm = mg.Params() if smoother == "ne" else mg.Params.uzawa()
    d = oh.discs[-1]
    u, p = inputs.random_state(N, seed=3)
    fu, gp = inputs.random_state(N, seed=4)
    x, f = lat.from_lattice(d, u, p), lat.from_lattice(d, fu, gp)
    uj, pj = junk(N, u, p)
    fj, gj = junk(N, fu, gp, 5.0)
    U, P, FU, GP = dev(uj), dev(pj), dev(fj), dev(gj)
    for step in range(3):
        gh.smooth(FU, GP, U, P, nsteps=1)
        x = mg.smooth(oh.top, x, f, prm)
        assert relmax(lat.from_lattice(d, host(U), host(P)), x) <= 1e-12, step
    assert_clean(N, u=host(U))


@pytest.mark.parametrize("Nc,n0", [(2, 2), (6, 6), (32, 2), (128, 2)])
def test_transfers_on_l_shape(Nc, n0):
    Nf = 2 * Nc
    oh = oracle_l(Nf, 1.0, n0)
    gh = gpu_l(Nf, 1.0, n0)
    P = oh.levels[-1].P
    dc, df = oh.discs[-2], oh.discs[-1]
    rf_u, rf_p = inputs.random_state(Nf, seed=5)
    cu, cp = gh.restrict(*map(dev, junk(Nf, rf_u, rf_p)))
    ref = P.T @ lat.from_lattice(df, rf_u, rf_p)
    assert relmax(lat.from_lattice(dc, host(cu), host(cp)), ref) <= TOL
    assert_clean(Nc, host(cu), host(cp))
    zu, zp = inputs.random_state(Nc, seed=6)
    xu, xp = inputs.random_state(Nf, seed=7)
    xu[:, removed_u(Nf)] = 0.0
    xp[removed_p(Nf)] = 0.0
    U, Pp = dev(xu), dev(xp)
    gh.prolong_add(*map(dev, junk(Nc, zu, zp)), U, Pp)
    ref = lat.from_lattice(df, xu, xp) + P @ lat.from_lattice(dc, zu, zp)
    assert relmax(lat.from_lattice(df, host(U), host(Pp)), ref) <= TOL
    assert_clean(Nf, host(U), host(Pp))


@pytest.mark.parametrize("n0,beta", [(2, 0.0), (2, 1.0), (4, 1e4), (6, 10.0)])
def test_coarse_solve_on_l_shape(n0, beta):
    oh = oracle_l(n0, beta, n0)
    gh = gpu_l(n0, beta, n0)
    d, lv = oh.discs[0], oh.levels[0]
    ru, rp = inputs.random_state(n0, seed=8)
    r = lat.from_lattice(d, ru, rp)
    r[lv.nu2:] -= r[lv.nu2:].mean()          # compatible: orthogonal to the constants
    ru, rp = junk(n0, *lat.to_lattice(d, r))
    zu, zp = gh.coarse_solve(dev(ru), dev(rp))
    got = lat.from_lattice(d, host(zu), host(zp))
    ref = lv.project_mean(lv.direct_solve(r))
    Bd = lv.bordered().toarray()
    assert relmax(got, ref) <= max(1e-12, 1e-15 * np.linalg.cond(Bd))
    assert abs(lv.m @ got[lv.nu2:]) <= 1e-13 * np.abs(got).max()
    assert_clean(n0, host(zu), host(zp))


@pytest.mark.parametrize("N", [8, 24, 256])
def test_mean_load_mass_dot_on_l_shape(N):
    n0 = 6 if N == 24 else 2
    oh = oracle_l(N, 1.0, n0)
    gh = gpu_l(N, 1.0, n0)
    d, lv = oh.discs[-1], oh.top
    zero_u = np.zeros((2, 2 * N + 1, 2 * N + 1))
    # mean projection with the L-shape's P1 weights; removed vertices untouched
    _, p = inputs.random_state(N, seed=9)
    p += 3.0
    P = dev(p)
    gh.project_mean(P)
    pref = lat.from_lattice(d, zero_u, p)[lv.nu2:]
    pref = pref - (lv.m @ pref) / lv.m.sum()
    got = host(P)
    assert np.abs(lat.from_lattice(d, zero_u, got)[lv.nu2:] - pref).max() <= 1e-13 * np.abs(pref).max()
    assert np.array_equal(got[removed_p(N)], p[removed_p(N)])
    # load vectors from nodal data on the closed domain (values outside it are junk)
    F, G = inputs.normal_fg(N, seed=10)
    fu, gp = gh.load(dev(F), dev(G))
    fn, gn = lat.lattice_to_nodal(d, F, G)
    rfu, rgp = d.load(fn, gn)
    assert relmax(lat.from_lattice(d, host(fu), host(gp)), np.concatenate([rfu, rgp])) <= TOL
    assert_clean(N, host(fu), host(gp))
    gpm = host(gh.pressure_mass(dev(G)))
    assert relmax(lat.lattice_to_nodal(d, F, gpm)[1], d.MP @ gn) <= TOL
    # velocity mass, and its transpose to all nodes of the closed domain
    u, pp = inputs.random_state(N, seed=11)
    uj, _ = junk(N, u, pp)
    ref = d.mass_u() @ lat.from_lattice(d, u, pp)[: 2 * d.nu]
    assert relmax(lat.from_lattice(d, host(gh.mass(dev(uj))), pp)[: 2 * d.nu], ref) <= TOL
    yall = host(gh.mass(dev(uj), all_nodes=True))
    lam = lat.from_lattice(d, u, pp)[: 2 * d.nu]
    Mi = d.M_full[d.interior]
    got_all, _ = lat.lattice_to_nodal(d, yall, pp)
    assert relmax(got_all, np.stack([Mi.T @ lam[: d.nu], Mi.T @ lam[d.nu:]])) <= TOL
    # dots skip every non-unknown entry
    a_u, a_p = junk(N, *inputs.random_state(N, seed=12))
    b_u, b_p = junk(N, *inputs.random_state(N, seed=13))
    va, vb = lat.from_lattice(d, a_u, a_p), lat.from_lattice(d, b_u, b_p)
    du = host(gh.dot(dev(a_u), dev(b_u), 0))[0]
    dp = host(gh.dot(dev(a_p), dev(b_p), 1))[0]
    nu2 = 2 * d.nu
    assert abs(du - va[:nu2] @ vb[:nu2]) <= 1e-13 * np.abs(va[:nu2] * vb[:nu2]).sum()
    assert abs(dp - va[nu2:] @ vb[nu2:]) <= 1e-13 * np.abs(va[nu2:] * vb[nu2:]).sum()


@pytest.mark.parametrize("fused", [True, False], ids=["fused", "unfused"])
@pytest.mark.parametrize("kind", ["ne", "uzawa", "ne_w"])
@pytest.mark.parametrize("N,n0,beta", [(8, 2, 1.0), (24, 6, 1e4), (64, 2, 0.0), (128, 2, 1e6)])
def test_iterates_on_l_shape(kind, N, n0, beta, fused):
    print(f"l-shape cycle {kind} N={N} n0={n0} beta={beta} fused={fused}", flush=True)
    gkw, prm = _params(kind)
    oh = oracle_l(N, beta, n0)
    gh = gpu_l(N, beta, n0, fused=fused, **gkw)
    F, G = inputs.normal_fg(N, seed=21)
    f, FU, GP = _rhs(oh, F, G)
    FU, GP = junk(N, FU, GP, 2.0)
    d = oh.discs[-1]
    x = np.zeros(oh.top.n)
    U, P = gh.zeros()
    FU, GP = dev(FU), dev(GP)
    for it in range(4):
        gh.cycle(FU, GP, U, P)
        x = mg.top_cycle(oh, x, f, prm)
        got = lat.from_lattice(d, host(U), host(P))
        err = np.linalg.norm(got - x) / np.linalg.norm(x)
        assert err <= PARITY, (it, err)
    assert_clean(N, host(U), host(P))


@pytest.mark.parametrize("beta", [1.0, 1e4])
def test_solve_on_l_shape(beta):
    """h = 1/256 on the L-shape, f iid U[-1,1] (seed 0), g = 0, NE V(2,2) to
    1e-8: the oracle's iterate count and solution; the FP32-inside-FP64 solve
    reaches 1e-10 in the oracle's residual."""
    N = 256
    print(f"l-shape solve N={N} beta={beta}", flush=True)
    oh = oracle_l(N, beta)
    gh = gpu_l(N, beta)
    F, G = inputs.uniform_f(N, seed=0)
    f, FU, GP = _rhs(oh, F, G)
    FU, GP = dev(FU), dev(GP)
    res = mg.solve(oh, f, mg.Params(), tol=1e-8, maxit=300)
    U, P, info = gh.solve(FU, GP, rtol=1e-8, maxit=300)
    assert info.status == "ok"
    near = abs(res.relres - 1e-8) < 1e-3 * 1e-8
    assert info.iters == res.iters or (near and abs(info.iters - res.iters) == 1), (info.iters, res.iters)
    d = oh.discs[-1]
    got = lat.from_lattice(d, host(U), host(P))
    assert np.linalg.norm(got - res.x) <= PARITY * np.linalg.norm(res.x)
    assert np.allclose(info.history, res.history, rtol=1e-8, atol=0)
    Um, Pm, im = gh.solve_mixed(FU, GP, rtol=1e-10, maxit=400)
    assert im.status == "ok"
    xm = lat.from_lattice(d, host(Um), host(Pm))
    assert np.linalg.norm(f - oh.top.calA @ xm) <= 1.01e-10 * np.linalg.norm(f)
    assert_clean(N, host(Um), host(Pm))


def test_batch_on_l_shape():
    """Uneven L-shaped instances (h = 1/16 ... 1/128) in one batch, FP64 and
    mixed: each equals its own single-instance solve (same count, same
    solution to 1e-10), and the h = 1/64 one equals the oracle's solve."""
    Ns, betas = [16, 64, 128, 32, 64], [1.0, 1e3, 0.5, 1e4, 20.0]
    B = Batch(Ns, betas, domain="l_shape")
    fus, gps, fs = [], [], []
    for k, N in enumerate(Ns):
        oh = oracle_l(N, betas[k])
        F, G = inputs.normal_fg(N, seed=50 + k)
        f, FU, GP = _rhs(oh, F, G)
        FU, GP = junk(N, FU, GP, 1.5)
        fus.append(dev(FU))
        gps.append(dev(GP))
        fs.append(f)
    us, ps, infos = B.solve(fus, gps, rtol=1e-9, maxit=300)
    for k, N in enumerate(Ns):
        assert infos[k].status == "ok", (k, infos[k])
        gh = gpu_l(N, betas[k])
        U, P, info = gh.solve(fus[k], gps[k], rtol=1e-9, maxit=300)
        assert abs(info.iters - infos[k].iters) <= 1, (k, info.iters, infos[k].iters)
        if info.iters == infos[k].iters:
            d = oracle_l(N, betas[k]).discs[-1]
            a = lat.from_lattice(d, host(us[k]), host(ps[k]))
            b = lat.from_lattice(d, host(U), host(P))
            assert np.linalg.norm(a - b) <= PARITY * np.linalg.norm(b)
        assert_clean(N, host(us[k]), host(ps[k]))
    k = 1
    oh = oracle_l(Ns[k], betas[k])
    res = mg.solve(oh, fs[k], mg.Params(), tol=1e-9, maxit=300)
    got = lat.from_lattice(oh.discs[-1], host(us[k]), host(ps[k]))
    assert abs(res.iters - infos[k].iters) <= 1
    if res.iters == infos[k].iters:
        assert np.linalg.norm(got - res.x) <= PARITY * np.linalg.norm(res.x)
    um, pm, im = B.solve_mixed(fus, gps, rtol=1e-10, maxit=400)
    for k, N in enumerate(Ns):
        oh = oracle_l(N, betas[k])
        x = lat.from_lattice(oh.discs[-1], host(um[k]), host(pm[k]))
        assert im[k].status == "ok"
        assert np.linalg.norm(fs[k] - oh.top.calA @ x) <= 1.01e-10 * np.linalg.norm(fs[k])


def test_divergence_on_l_shape_matches_oracle():
    """Without convexity the iterate need not contract: NE V(2,2) at h = 1/32,
    beta = 1e5 on the L-shape grows by about 8% per iterate (on the square it
    contracts by about 0.89).  The GPU reports the same divergence at the same
    iterate as the oracle, with the same residual history."""
    N, beta = 32, 1e5
    oh = oracle_l(N, beta)
    gh = gpu_l(N, beta)
    F, G = inputs.normal_fg(N, seed=53)
    f, FU, GP = _rhs(oh, F, G)
    res = mg.solve(oh, f, mg.Params(), tol=1e-9, maxit=300)
    assert res.status == "diverged"
    U, P, info = gh.solve(dev(FU), dev(GP), rtol=1e-9, maxit=300)
    assert info.status == "diverged" and info.iters == res.iters, (info, res.iters)
    assert np.allclose(info.history, res.history, rtol=1e-7, atol=0)


def test_implicit_step_on_l_shape():
    """Two implicit Euler steps (dt = 1e-2, h = 1/32) from a random
    divergence-carrying start: each equals the oracle's direct step."""
    N, dt = 32, 1e-2
    oh = oracle_l(N, 1.0 / dt)
    gh = gpu_l(N, 1.0 / dt)
    d, lv = oh.discs[-1], oh.top
    F, G = inputs.normal_fg(N, seed=60)
    fn, _ = lat.lattice_to_nodal(d, F, G)
    u0, _ = inputs.random_state(N, seed=61)
    u0[:, removed_u(N)] = 0.0
    x = lat.from_lattice(d, u0, np.zeros((N + 1, N + 1)))
    U, P = dev(u0), torch.zeros((N + 1, N + 1), dtype=torch.float64, device="cuda")
    u = x[: lv.nu2]
    for s in range(2):
        info = gh.implicit_step(U, P, f_nodal=dev(F), rtol=1e-13, maxit=300)
        assert info.status == "ok", info
        xr = ots.step(lv, u, fn)
        got = lat.from_lattice(d, host(U), host(P))
        assert np.linalg.norm(got - xr) <= 1e-9 * np.linalg.norm(xr), s
        u = xr[: lv.nu2]
