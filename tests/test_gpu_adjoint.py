"""GPU tests of the differentiable solve (adjoint method): gradients against
the oracle's adjoint (sparse direct solves), against central finite
differences of the GPU forward solve, and batched against single."""
import numpy as np
import pytest
import torch

from oracle import adjoint as oadj
from paper_1502_04070_amd import autograd as ag
from paper_1502_04070_amd import inputs
from tests import lattice as lat
from tests.test_gpu_ops import dev, host, oracle_level

pytestmark = pytest.mark.gpu


def _loss(u, p, ut, wp, N):
    e = u - ut
    return 0.5 * (e * ag.mass_product(e, N)).sum() + (wp * p).sum()


@pytest.mark.parametrize("mixed", [False, True], ids=["fp64", "fp32_refine"])
@pytest.mark.parametrize("beta", [1.0, 300.0])
def test_gradients_match_oracle_adjoint(beta, mixed):
    N = 16
    F, G = inputs.normal_fg(N, seed=50)
    ut, _ = inputs.random_state(N, seed=51)
    wp = np.random.default_rng(52).standard_normal((N + 1, N + 1))
    f = dev(F).requires_grad_(True)
    g = dev(G).requires_grad_(True)
    b = torch.tensor(beta, dtype=torch.float64, device="cuda", requires_grad=True)
    u, p = ag.stokes_solve(f, g, b, rtol=1e-13, mixed=mixed)
    loss = _loss(u, p, dev(ut), dev(wp), N)
    loss.backward()
    # oracle
    oh = oracle_level(N, beta, 2)
    lv = oh.top
    d = oh.discs[-1]
    fn, gn = lat.lattice_to_nodal(d, F, G)
    x = oadj.forward(lv, fn, gn)
    got_x = lat.from_lattice(d, host(u), host(p))
    assert np.linalg.norm(got_x - x) <= 1e-10 * np.linalg.norm(x)
    ut_v = lat.from_lattice(d, ut, np.zeros((N + 1, N + 1)))[: lv.nu2]
    wp_v = lat.from_lattice(d, np.zeros_like(ut), wp)[lv.nu2:]
    dLdu = d.mass_u() @ (x[: lv.nu2] - ut_v)
    df, dg, dbeta = oadj.gradients(lv, x, dLdu, wp_v)
    gdf, gdg = lat.lattice_to_nodal(d, host(f.grad), host(g.grad))
    assert np.abs(gdf - df).max() <= 1e-8 * np.abs(df).max()
    assert np.abs(gdg - dg).max() <= 1e-8 * np.abs(dg).max()
    assert abs(float(b.grad) - dbeta) <= 1e-8 * abs(dbeta)


def test_gradients_match_central_differences():
    N, beta = 32, 50.0
    F, G = inputs.normal_fg(N, seed=60)
    ut, _ = inputs.random_state(N, seed=61)
    wp = np.random.default_rng(62).standard_normal((N + 1, N + 1))
    utd, wpd = dev(ut), dev(wp)

    def L(Fa, Ga, be):
        with torch.no_grad():
            u, p = ag.stokes_solve(dev(Fa), dev(Ga), torch.tensor(be, dtype=torch.float64, device="cuda"),
                                   rtol=1e-13)
            return float(_loss(u, p, utd, wpd, N))

    f = dev(F).requires_grad_(True)
    g = dev(G).requires_grad_(True)
    b = torch.tensor(beta, dtype=torch.float64, device="cuda", requires_grad=True)
    u, p = ag.stokes_solve(f, g, b, rtol=1e-13)
    _loss(u, p, utd, wpd, N).backward()
    rng = np.random.default_rng(63)
    vf = rng.standard_normal(F.shape)
    vf /= np.abs(vf).max()
    vg = rng.standard_normal(G.shape)
    vg /= np.abs(vg).max()
    eps = 1e-5
    fd = (L(F + eps * vf, G + eps * vg, beta) - L(F - eps * vf, G - eps * vg, beta)) / (2 * eps)
    ad = float((f.grad * dev(vf)).sum() + (g.grad * dev(vg)).sum())
    assert abs(fd - ad) <= 1e-6 * max(1.0, abs(ad)), (fd, ad)
    eb = 1e-6 * beta
    fdb = (L(F, G, beta + eb) - L(F, G, beta - eb)) / (2 * eb)
    assert abs(fdb - float(b.grad)) <= 1e-5 * abs(float(b.grad)), (fdb, float(b.grad))


@pytest.mark.parametrize("domain", ["square", "union_jack"])
def test_batched_gradients_match_single(domain):
    N, nb = 32, 3
    betas = [1.0, 1e3, 1e5]
    fs, gs, uts = [], [], []
    for k in range(nb):
        F, G = inputs.normal_fg(N, seed=70 + k)
        ut, _ = inputs.random_state(N, seed=80 + k)
        fs.append(F); gs.append(G); uts.append(ut)
    f = torch.stack([dev(a) for a in fs]).requires_grad_(True)
    g = torch.stack([dev(a) for a in gs]).requires_grad_(True)
    b = torch.tensor(betas, dtype=torch.float64, device="cuda", requires_grad=True)
    ut = torch.stack([dev(a) for a in uts])
    u, p = ag.batch_stokes_solve(f, g, b, rtol=1e-12, domain=domain)
    e = u - ut
    loss = sum(0.5 * (e[k] * ag.mass_product(e[k], N)).sum() for k in range(nb))
    loss.backward()
    for k in range(nb):
        fk = dev(fs[k]).requires_grad_(True)
        gk = dev(gs[k]).requires_grad_(True)
        bk = torch.tensor(betas[k], dtype=torch.float64, device="cuda", requires_grad=True)
        uk, pk = ag.stokes_solve(fk, gk, bk, rtol=1e-12, domain=domain)
        ek = uk - dev(uts[k])
        (0.5 * (ek * ag.mass_product(ek, N)).sum()).backward()
        for a, r in ((f.grad[k], fk.grad), (g.grad[k], gk.grad)):
            assert float((a - r).abs().max()) <= 1e-9 * float(r.abs().max())
        assert abs(float(b.grad[k]) - float(bk.grad)) <= 1e-9 * abs(float(bk.grad))


@pytest.mark.parametrize("domain", ["l_shape", "union_jack"])
def test_gradients_on_other_grids_match_oracle_adjoint(domain):
    """The differentiable solve on the L-shape and on the union-jack grid
    (h = 1/16, beta = 30): solution, dL/df, dL/dg and dL/dbeta equal the
    oracle's adjoint on that grid (sparse direct solves) to 1e-8, for
    L = 1/2 |u - u_t|^2 + w_p . p over the lattice (targets and weights zero
    off the domain's unknowns)."""
    from oracle import multigrid as mg
    N, beta = 16, 30.0
    oh = mg.Hierarchy(domain, int(round(np.log2(N // 2))), beta, n0=2)
    lv, d = oh.top, oh.discs[-1]
    rng = np.random.default_rng(70)
    ut, wp = lat.to_lattice(d, rng.standard_normal(lv.n))
    F, G = inputs.normal_fg(N, seed=71)
    f = dev(F).requires_grad_(True)
    g = dev(G).requires_grad_(True)
    b = torch.tensor(beta, dtype=torch.float64, device="cuda", requires_grad=True)
    u, p = ag.stokes_solve(f, g, b, rtol=1e-13, domain=domain)
    loss = 0.5 * ((u - dev(ut)) ** 2).sum() + (dev(wp) * p).sum()
    loss.backward()
    fn, gn = lat.lattice_to_nodal(d, F, G)
    x = oadj.forward(lv, fn, gn)
    got_x = lat.from_lattice(d, host(u), host(p))
    assert np.linalg.norm(got_x - x) <= 1e-10 * np.linalg.norm(x)
    tv = lat.from_lattice(d, ut, wp)
    df, dg, dbeta = oadj.gradients(lv, x, x[: lv.nu2] - tv[: lv.nu2], tv[lv.nu2:])
    gdf, gdg = lat.lattice_to_nodal(d, host(f.grad), host(g.grad))
    assert np.abs(gdf - df).max() <= 1e-8 * np.abs(df).max()
    assert np.abs(gdg - dg).max() <= 1e-8 * np.abs(dg).max()
    assert abs(float(b.grad) - dbeta) <= 1e-8 * abs(dbeta)


def test_batched_mixed_precision_gradients_match_fp64():
    """FP32 cycles in FP64 refinement for the batched forward and adjoint
    solves (h = 1/64, three beta): u and the gradients of the mass loss equal
    those of the FP64 solves to 1e-8, both solved to a relative residual of
    1e-11 (the refinement with FP32 cycles levels off near 1e-12 at
    beta = 1e5)."""
    N, betas = 64, [1.0, 1e3, 1e5]
    fs = [dev(inputs.normal_fg(N, seed=90 + k)[0]) for k in range(3)]
    gs = [dev(inputs.normal_fg(N, seed=90 + k)[1]) for k in range(3)]
    ut = torch.stack([dev(inputs.random_state(N, seed=95 + k)[0]) for k in range(3)])
    res = {}
    for mixed in (False, True):
        f = torch.stack(fs).requires_grad_(True)
        g = torch.stack(gs).requires_grad_(True)
        b = torch.tensor(betas, dtype=torch.float64, device="cuda", requires_grad=True)
        u, p = ag.batch_stokes_solve(f, g, b, rtol=1e-11, maxit=600, mixed=mixed)
        e = u - ut
        sum(0.5 * (e[k] * ag.mass_product(e[k], N)).sum() for k in range(3)).backward()
        res[mixed] = (u.detach(), f.grad, g.grad, b.grad)
    for a, r in zip(res[True], res[False]):
        assert float((a - r).abs().max()) <= 1e-8 * float(r.abs().max())
