"""Pins of the oracle's adjoint gradients: central finite differences of the
forward solve (which never touches the adjoint formulas) and reciprocity of
the symmetric saddle system (Section 2: calA is symmetric)."""
import numpy as np
import pytest

from oracle import adjoint
from oracle.multigrid import Hierarchy


def _setup(beta, N0=2, lev=2, seed=0):
    lv = Hierarchy("same_diag", lev, beta, n0=N0).top
    rng = np.random.default_rng(seed)
    d = lv.disc
    f = rng.standard_normal((2, d.n2))
    g = rng.standard_normal(d.n1)
    ut = rng.standard_normal(lv.nu2)
    return lv, f, g, ut


def _loss(lv, f, g, ut, wp):
    x = adjoint.forward(lv, f, g)
    return adjoint.mass_loss(lv, x, ut) + wp @ x[lv.nu2:]


@pytest.mark.parametrize("beta", [1.0, 300.0])
def test_adjoint_matches_central_differences(beta):
    lv, f, g, ut = _setup(beta)
    wp = np.random.default_rng(7).standard_normal(lv.n1)     # a pressure term in the loss too
    x = adjoint.forward(lv, f, g)
    dLdu = lv.disc.mass_u() @ (x[: lv.nu2] - ut)
    df, dg, db = adjoint.gradients(lv, x, dLdu, wp)
    rng = np.random.default_rng(11)
    # directional derivatives in f and g, and the beta derivative
    for _ in range(2):
        vf = rng.standard_normal(f.shape)
        vg = rng.standard_normal(g.shape)
        eps = 1e-6
        fd = (_loss(lv, f + eps * vf, g + eps * vg, ut, wp) - _loss(lv, f - eps * vf, g - eps * vg, ut, wp)) / (2 * eps)
        ad = np.sum(df * vf) + dg @ vg
        assert abs(fd - ad) <= 1e-6 * max(1.0, abs(ad)), (fd, ad)
    eb = 1e-6 * beta
    lp = Hierarchy("same_diag", 2, beta + eb, n0=2).top
    lm = Hierarchy("same_diag", 2, beta - eb, n0=2).top
    fdb = (_loss(lp, f, g, ut, wp) - _loss(lm, f, g, ut, wp)) / (2 * eb)
    assert abs(fdb - db) <= 1e-5 * max(abs(db), 1e-12), (fdb, db)


def test_reciprocity():
    """For the symmetric saddle matrix, c^T x = lambda^T F when calA x = F and calA lambda = c
    (both compatible, pressures mean-free)."""
    lv, f, g, ut = _setup(5.0, seed=3)
    rng = np.random.default_rng(4)
    F = rng.standard_normal(lv.n)
    F[lv.nu2:] -= F[lv.nu2:].mean()
    c = rng.standard_normal(lv.n)
    c[lv.nu2:] -= c[lv.nu2:].mean()
    x = lv.project_mean(lv.direct_solve(F))
    lam = lv.project_mean(lv.direct_solve(c))
    assert np.isclose(c @ x, lam @ F, rtol=1e-10)


def test_gradient_of_g_is_blind_to_constants():
    """Adding a constant to g does not change the mean-projected data, so the
    solution is unchanged and the gradient in g is orthogonal to constants."""
    lv, f, g, ut = _setup(2.0, seed=5)
    x = adjoint.forward(lv, f, g)
    x2 = adjoint.forward(lv, f, g + 3.0)
    assert np.allclose(x, x2, atol=1e-12)
    dLdu = lv.disc.mass_u() @ (x[: lv.nu2] - ut)
    _, dg, _ = adjoint.gradients(lv, x, dLdu, np.zeros(lv.n1))
    assert abs(dg.sum()) < 1e-12 * np.abs(dg).sum()


def test_multigrid_solves_give_the_direct_gradients():
    """The multigrid variant (used where a direct factorization is too large)
    reproduces the direct-solve gradients to the solve tolerance."""
    h = Hierarchy("same_diag", 3, 40.0, n0=2)
    lv = h.top
    rng = np.random.default_rng(5)
    d = lv.disc
    f = rng.standard_normal((2, d.n2))
    g = rng.standard_normal(d.n1)
    ut = rng.standard_normal(lv.nu2)
    wp = rng.standard_normal(lv.n1)
    out = []
    for solve in (None, adjoint.mg_solver(h, tol=1e-13)):
        x = adjoint.forward(lv, f, g, solve=solve)
        dLdu = d.mass_u() @ (x[: lv.nu2] - ut)
        out.append((x,) + adjoint.gradients(lv, x, dLdu, wp, solve=solve))
    (x0, df0, dg0, db0), (x1, df1, dg1, db1) = out
    assert np.linalg.norm(x1 - x0) <= 1e-11 * np.linalg.norm(x0)
    assert np.abs(df1 - df0).max() <= 1e-9 * np.abs(df0).max()
    assert np.abs(dg1 - dg0).max() <= 1e-9 * np.abs(dg0).max()
    assert abs(db1 - db0) <= 1e-9 * abs(db0)
