"""Pins of the oracle's multigrid iterate (Sections 3, 4 and 6).

  * the iterate converges to the sparse direct solution and has it as a fixed point;
  * the Uzawa half-steps equal one solve with the compact preconditioner
    [[tau^-1 Ahat, B^T], [B, tau B Ahat^-1 B^T - sigma^-1 Shat]] (Section 4);
  * with exact coarse solve and no smoothing, the coarse-grid correction is a
    projection (Galerkin identity), so a second application changes nothing;
  * the smoother conditions of Section 4 (tau rho < 2) hold for tau = 0.35;
  * the printed Tables 1-3 of Section 6 are reproduced within a band under the
    paper's own protocol (union-jack mesh, W-cycle, 1e-9 error reduction).
"""
import json
import os

import numpy as np
import pytest
import scipy.linalg as sl

from oracle import multigrid as mg
from oracle import problem as pb

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")))


def _rhs(lv, seed):
    rng = np.random.default_rng(seed)
    f = rng.uniform(-1, 1, lv.n)
    f[lv.nu2:] -= f[lv.nu2:].mean()         # compatible: sum of pressure loads is zero
    return f


@pytest.mark.parametrize("kind", ["same_diag", "union_jack"])
@pytest.mark.parametrize("prm", [mg.Params(), mg.Params.uzawa(), mg.Params("ne", 0.35, 0.8, 3, 3, 2)],
                         ids=["NE-V22", "UZ-V33", "NE-W33"])
@pytest.mark.parametrize("beta", [0.0, 1.0, 1e4])
def test_converges_to_direct_solution(kind, prm, beta):
    h = mg.Hierarchy(kind, 3, beta, n0=2)
    f = _rhs(h.top, 3)
    res = mg.solve(h, f, prm, tol=1e-11, maxit=600)
    assert res.status == "ok"
    xd = h.top.project_mean(h.top.direct_solve(f))
    assert np.linalg.norm(res.x - xd) <= 1e-9 * np.linalg.norm(xd)


def test_exact_solution_is_fixed_point():
    h = mg.Hierarchy("same_diag", 3, 10.0, n0=2)
    f = _rhs(h.top, 4)
    xs = h.top.project_mean(h.top.direct_solve(f))
    for prm in [mg.Params(), mg.Params.uzawa()]:
        x1 = mg.top_cycle(h, xs, f, prm)
        assert np.linalg.norm(x1 - xs) <= 1e-11 * np.linalg.norm(xs)


def test_uzawa_half_steps_equal_compact_form():
    h = mg.Hierarchy("same_diag", 1, 3.0, n0=2)
    lv = h.top
    rng = np.random.default_rng(1)
    x = rng.standard_normal(lv.n)
    f = rng.standard_normal(lv.n)
    tau, sigma = 0.8, 0.8
    A, B = lv.A.toarray(), lv.B.toarray()
    Ah, Sh = np.diag(lv.Ahat), np.diag(lv.Shat)
    hatA = np.block([[Ah / tau, B.T], [B, tau * B @ np.linalg.solve(Ah, B.T) - Sh / sigma]])
    calA = lv.calA.toarray()
    expect = x + np.linalg.solve(hatA, f - calA @ x)
    got = mg.uzawa_step(lv, x, f, tau, sigma)
    assert np.allclose(got, expect, rtol=1e-12, atol=1e-12 * np.abs(expect).max())


def test_coarse_correction_is_a_projection():
    h = mg.Hierarchy("same_diag", 2, 2.0, n0=2)
    prm = mg.Params("ne", 0.35, 0.8, 0, 0, 1)
    f = _rhs(h.top, 2)
    x0 = np.random.default_rng(9).standard_normal(h.top.n)
    # two-grid on levels (1, 2): drop level 0 so level 1 is solved exactly
    h2 = mg.Hierarchy("same_diag", 1, 2.0, n0=4)
    x1 = mg.cycle(h2, 1, x0, _rhs(h2.top, 2), prm)
    x2 = mg.cycle(h2, 1, x1, _rhs(h2.top, 2), prm)
    assert np.linalg.norm(h2.top.project_mean(x2 - x1)) <= 1e-11 * np.linalg.norm(x1)


@pytest.mark.parametrize("kind", ["same_diag", "union_jack"])
def test_normal_equation_damping_condition(kind):
    """Section 4: tau must keep rho(tau Lhat^{-1} A L^{-1} A) below 2 for all levels and beta."""
    for k in [1, 2]:
        for beta in [0.0, 1.0, 1e2, 1e4, 1e6, 1e8, 1e10]:
            lv = mg.Hierarchy(kind, k, beta, n0=2).top
            C = lv.calA.toarray()
            s = np.sqrt(lv.Ldiag)
            Ks = C / s[:, None] / s[None, :]
            ev = sl.eigvalsh(Ks)
            assert 0.35 * np.max(ev ** 2) < 2.0


def test_uzawa_conditions_are_level_independent():
    """Section 4 asks tau^-1 Ahat >= A and sigma^-1 Shat >= tau B Ahat^-1 B^T with
    tau, sigma independent of the level.  With Ahat = diag A the two largest
    generalized eigenvalues stay bounded under refinement (they approach about
    2.2 and 2.0 with shrinking increments), so the literal condition with
    tau = sigma = 0.8 (bounds 1.25 and 1.5625) is only met up to the constant the
    theory allows; the measured values are pinned here."""
    l1s, l2s = [], []
    for k in [1, 2, 3]:
        lv = mg.Hierarchy("same_diag", k, 1.0, n0=2).top
        A, B = lv.A.toarray(), lv.B.toarray()
        l1s.append(sl.eigh(A, np.diag(lv.Ahat), eigvals_only=True)[-1])
        S = B @ (B.T / lv.Ahat[:, None])
        l2s.append(sl.eigh(S, np.diag(lv.Shat), eigvals_only=True)[-1])
    for ls, hi in ((l1s, 2.3), (l2s, 2.1)):
        d = np.diff(ls)
        assert max(ls) < hi and np.all(d > 0) and d[1] < 0.5 * d[0], ls
    assert l1s[-1] > 1 / 0.8 and l2s[-1] > 1 / (0.8 * 0.8)


def test_h_independent_rates_same_diag():
    """Robustness in h (Section 6 tables): the asymptotic per-iterate residual
    reduction of NE V(2,2) and Uzawa V(3,3) stays bounded and saturates as the
    level grows.  (The
    Euclidean residual first rises by a factor that grows like 1/h, because the
    velocity and pressure rows are scaled differently, so counts to a fixed
    tolerance grow by about one iterate per level; the rate does not.)"""
    for prm, qmax in ((mg.Params(), 0.8), (mg.Params.uzawa(), 0.5)):
        qs = []
        for k in [3, 4, 5]:
            h = mg.Hierarchy("same_diag", k, 1.0, n0=2)
            f = _rhs(h.top, 0)
            hist = mg.solve(h, f, prm, tol=1e-10, maxit=300).history
            qs.append((hist[-1] / hist[-6]) ** 0.2)
        d = np.diff(qs)
        assert max(qs) < qmax and d[1] < 0.5 * max(d[0], 0.01), qs   # saturates


def _band(n, n_paper):
    return abs(n - n_paper) <= max(5, 0.25 * n_paper)


def test_table1_normal_equation_band_and_uzawa_divergence():
    k, beta = GOLD["table1_level"], GOLD["table1_beta"]
    nus = GOLD["table1_nu"][:4]
    h = mg.Hierarchy("union_jack", k, beta, n0=2)
    xs = pb.paper_exact_discrete(h)
    ne = []
    for nu, (n_p, q_p) in zip(nus, GOLD["table1_ne"]):
        n, q = mg.error_reduction_run(h, xs, mg.Params("ne", 0.35, 0.8, nu, nu, 2))
        ne.append(n)
        assert n is not None and _band(n, n_p), (nu, n, n_p)
        assert abs(q - q_p) < 0.08, (nu, q, q_p)
    assert ne == sorted(ne, reverse=True)           # more smoothing, fewer iterates
    for nu, gold in zip([1, 2, 3], GOLD["table1_uzawa"]):
        n, q = mg.error_reduction_run(h, xs, mg.Params("uzawa", 0.8, 0.8, nu, nu, 2), maxit=80)
        if gold is None:
            assert n is None, (nu, n)                # printed "divergent"
        else:
            assert n is not None and _band(n, gold[0]), (nu, n, gold)


@pytest.mark.parametrize("ib", range(6))
def test_tables_2_3_level4_band(ib):
    beta = GOLD["table23_beta"][ib]
    h = mg.Hierarchy("union_jack", 4, beta, n0=2)
    xs = pb.paper_exact_discrete(h)
    n_ne, q_ne = mg.error_reduction_run(h, xs, mg.Params("ne", 0.35, 0.8, 3, 3, 2))
    n_uz, q_uz = mg.error_reduction_run(h, xs, mg.Params("uzawa", 0.8, 0.8, 3, 3, 2))
    gne = GOLD["table2_ne_3p3"][0][ib]
    guz = GOLD["table3_uzawa_3p3"][0][ib]
    assert _band(n_ne, gne[0]), (beta, n_ne, gne)
    assert _band(n_uz, guz[0]), (beta, n_uz, guz)
    assert n_uz < n_ne                                 # Uzawa converges faster (Section 6)


def test_level_damping_acts_on_its_own_level():
    """Per-level damping (Section 6 remarks that the rates improve when tau depends
    on the level).  With x = L^{-1/2} v, v an eigenvector of the symmetric
    L^{-1/2} calA L^{-1/2} with eigenvalue lambda, one normal-equation step with
    f = 0 multiplies x by 1 - tau lambda^2.  A two-level iterate with nu_pre = 1,
    nu_post = 0 therefore maps x to (1 - tau_top lambda^2) C x (C the coarse-grid
    correction), whatever the coarsest level's value (it is solved exactly)."""
    h = mg.Hierarchy("same_diag", 1, 10.0, n0=2)
    lv = h.top
    s = np.sqrt(lv.Ldiag)
    Ks = lv.calA.toarray() / s[:, None] / s[None, :]
    w, V = sl.eigh(Ks)
    k = int(np.argmax(np.abs(w)))
    lam, x = w[k], V[:, k] / s
    out = {}
    for t_top, t_coarse in ((0.2, 0.9), (0.35, 0.1)):
        prm = mg.Params("ne", 0.5, 0.8, 1, 0, 1, level_tau=(t_coarse, t_top))
        out[t_top] = mg.cycle(h, 1, x, np.zeros(lv.n), prm) / (1 - t_top * lam ** 2)
    a, b = out[0.2], out[0.35]
    assert np.linalg.norm(a - b) <= 1e-10 * np.linalg.norm(a)
    # the same values on every level reproduce the scalar damping exactly
    h3 = mg.Hierarchy("same_diag", 2, 10.0, n0=2)
    f = _rhs(h3.top, 5)
    x0 = np.zeros(h3.top.n)
    y1 = mg.cycle(h3, 2, x0, f, mg.Params())
    y2 = mg.cycle(h3, 2, x0, f, mg.Params(level_tau=(0.35, 0.35, 0.35)))
    assert np.array_equal(y1, y2)
    # a middle level's value enters the iterate
    y3 = mg.cycle(h3, 2, x0, f, mg.Params(level_tau=(0.35, 0.2, 0.35)))
    assert np.linalg.norm(y3 - y1) > 1e-6 * np.linalg.norm(y1)


def test_level_only_exact_solution_equals_hierarchy_one():
    """x* of Section 6 built on the finest level alone equals the one built
    through a whole hierarchy (same mesh, same projection)."""
    from oracle import problem as pb
    h = mg.Hierarchy("union_jack", 3, 1.0)
    disc, xs = pb.paper_exact_on_level("union_jack", 3)
    assert disc.mesh.nt == h.discs[-1].mesh.nt
    assert np.array_equal(xs, pb.paper_exact_discrete(h))
