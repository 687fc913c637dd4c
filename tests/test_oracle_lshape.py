"""Pins of the oracle on the L-shaped domain (0,1)^2 minus [1/2,1]^2 (Section 1:
the method applies to non-convex domains; the analysis does not), by facts
that hold independently of the oracle's assembly:

* refining the coarse L-shaped grid gives the finer one (nested spaces);
* closed forms: area 3/4 (1^T M_P 1 and sum of the P1 weights), K 1 = 0,
  B^T 1 = 0, and the boundary nodes include the two re-entrant edges;
* the Galerkin identity P^T calA_f P = calA_c on the L-shape hierarchy;
* Taylor-Hood orders (h^3, h^2, h^2) for a smooth solution that vanishes
  on the whole boundary, re-entrant edges included;
* the multigrid iterate converges to the sparse direct solution.
"""
import numpy as np
import pytest
import sympy as sy

from oracle import mesh, quadrature
from oracle import multigrid as mg
from oracle.fem import Discretization
from oracle.multigrid import Level


def _tri_set(m):
    return {tuple(sorted(map(tuple, np.round(m.pts[t], 12)))) for t in m.tris}


@pytest.mark.parametrize("n0", [2, 4])
def test_refined_l_shape_is_the_finer_l_shape(n0):
    assert _tri_set(mesh.refine(mesh.l_shape(n0))) == _tri_set(mesh.l_shape(2 * n0))


def test_closed_forms():
    d = Discretization(mesh.l_shape(8))
    one1 = np.ones(d.n1)
    assert abs(one1 @ (d.MP @ one1) - 0.75) < 1e-13
    lv = Level(d, 1.0)
    assert abs(lv.m.sum() - 0.75) < 1e-13
    assert np.abs(d.K_full @ np.ones(d.n2)).max() < 1e-12
    assert np.abs(lv.B.T @ one1).max() < 1e-12
    # P2 nodes on the re-entrant edges x = 1/2 (y >= 1/2) and y = 1/2 (x >= 1/2) are boundary nodes
    c = d.coords2
    on_reentrant = ((np.abs(c[:, 0] - 0.5) < 1e-12) & (c[:, 1] >= 0.5 - 1e-12)) | \
                   ((np.abs(c[:, 1] - 0.5) < 1e-12) & (c[:, 0] >= 0.5 - 1e-12))
    interior = np.zeros(d.n2, dtype=bool)
    interior[d.interior] = True
    assert on_reentrant.sum() == 2 * 9 - 1 and not (interior & on_reentrant).any()
    # every other node with 0 < x, y < 1 and not both >= 1/2 is interior
    inside = (c[:, 0] > 1e-12) & (c[:, 0] < 1 - 1e-12) & (c[:, 1] > 1e-12) & (c[:, 1] < 1 - 1e-12) & ~on_reentrant
    assert np.array_equal(inside, interior)


def test_galerkin_identity_on_l_shape():
    h = mg.Hierarchy("l_shape", 2, 3.0, n0=2)
    for k in (1, 2):
        f, c = h.levels[k], h.levels[k - 1]
        G = (f.P.T @ f.calA @ f.P).toarray()
        assert np.abs(G - c.calA.toarray()).max() <= 1e-12 * np.abs(G).max()


X, Y = sy.symbols("x y")
_Q = X * (1 - X) * Y * (1 - Y) * (X - sy.Rational(1, 2)) * (Y - sy.Rational(1, 2))
PSI = _Q ** 2
U_EX = (sy.diff(PSI, Y) * 64, -sy.diff(PSI, X) * 64)
P_EX = sy.cos(sy.pi * X) * sy.sin(sy.pi * Y)


def _fields(beta):
    lap = [sy.diff(c, X, 2) + sy.diff(c, Y, 2) for c in U_EX]
    f = [-lap[0] + beta * U_EX[0] - sy.diff(P_EX, X), -lap[1] + beta * U_EX[1] - sy.diff(P_EX, Y)]
    L = lambda e: sy.lambdify((X, Y), e, "numpy")
    fx, fy = L(sy.expand(f[0])), L(sy.expand(f[1]))
    ux, uy, pp = L(U_EX[0]), L(U_EX[1]), L(P_EX)
    gu = [[L(sy.diff(c, v)) for v in (X, Y)] for c in U_EX]

    def vec(fun):
        return lambda P: np.broadcast_to(fun(P[..., 0], P[..., 1]), P.shape[:-1]).astype(float)

    u_exact = lambda P: np.stack([vec(ux)(P), vec(uy)(P)], -1)
    grad_u = lambda P: np.stack([np.stack([vec(gu[c][d])(P) for d in range(2)], -1) for c in range(2)], -2)
    return vec(fx), vec(fy), u_exact, vec(pp), grad_u


def test_taylor_hood_orders_on_l_shape():
    beta = 10.0
    fx, fy, u_exact, p_exact, grad_u = _fields(beta)
    errs = []
    for N in [4, 8, 16, 32]:
        d = Discretization(mesh.l_shape(N))
        lv = Level(d, beta)
        fu = np.concatenate([quadrature.load_p2(d.mesh, fx)[d.interior],
                             quadrature.load_p2(d.mesh, fy)[d.interior]])
        x = lv.direct_solve(np.concatenate([fu, np.zeros(d.n1)]))
        uh = np.zeros((2, d.n2))
        uh[0, d.interior] = x[: d.nu]
        uh[1, d.interior] = x[d.nu: 2 * d.nu]
        errs.append(quadrature.l2_errors(d, uh, x[2 * d.nu:], u_exact, p_exact, grad_u))
    errs = np.array(errs)
    rates = np.log2(errs[:-1] / errs[1:])
    assert rates[-1, 0] > 2.8, rates
    assert rates[-1, 1] > 1.9, rates
    assert rates[-1, 2] > 1.8, rates


@pytest.mark.parametrize("smoother", ["ne", "uzawa"])
def test_multigrid_converges_to_direct_solution_on_l_shape(smoother):
    h = mg.Hierarchy("l_shape", 3, 50.0, n0=2)
    rng = np.random.default_rng(4)
    lv = h.top
    f = rng.standard_normal(lv.n)
    f[lv.nu2:] -= lv.m * (f[lv.nu2:].sum() / lv.m.sum())        # compatible pressure data
    prm = mg.Params() if smoother == "ne" else mg.Params.uzawa()
    res = mg.solve(h, f, prm, tol=1e-11, maxit=300)
    assert res.status == "ok"
    xd = lv.project_mean(lv.direct_solve(f))
    assert np.linalg.norm(res.x - xd) <= 1e-8 * np.linalg.norm(xd)
