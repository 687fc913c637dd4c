"""Pins of the discrete problem: textbook Taylor-Hood convergence orders.

For a smooth exact solution the P2-P1 Galerkin solution of Section 2 converges
with ||u - u_h||_L2 ~ h^3, |u - u_h|_H1 ~ h^2 and ||p - p_h||_L2 ~ h^2.  A wrong
sign of the coupling, a transposed block, a dropped term of A = K + beta M or a
wrong load would all destroy these orders.  The sign convention is that of the
variational form: (grad u, grad v) + beta (u, v) + (p, div v) = (f, v), i.e. the
strong form -Lap u + beta u - grad p = f, div u = g.
"""
import numpy as np
import pytest
import sympy as sy

from oracle import mesh, quadrature
from oracle.multigrid import Level
from oracle.fem import Discretization

X, Y = sy.symbols("x y")
U_EX = (sy.sin(sy.pi * X) * sy.sin(sy.pi * Y), X * (1 - X) * Y * (1 - Y) * (1 + X))
P_EX = sy.cos(sy.pi * X) * sy.cos(2 * sy.pi * Y) + X * Y


def _fields(beta):
    lap = [sy.diff(c, X, 2) + sy.diff(c, Y, 2) for c in U_EX]
    f = [-lap[0] + beta * U_EX[0] - sy.diff(P_EX, X), -lap[1] + beta * U_EX[1] - sy.diff(P_EX, Y)]
    g = sy.diff(U_EX[0], X) + sy.diff(U_EX[1], Y)
    L = lambda e: sy.lambdify((X, Y), e, "numpy")
    fx, fy, gg = L(f[0]), L(f[1]), L(g)
    ux, uy, pp = L(U_EX[0]), L(U_EX[1]), L(P_EX)
    gu = [[L(sy.diff(c, v)) for v in (X, Y)] for c in U_EX]

    def vec(fun):
        return lambda P: np.broadcast_to(fun(P[..., 0], P[..., 1]), P.shape[:-1]).astype(float)

    u_exact = lambda P: np.stack([vec(ux)(P), vec(uy)(P)], -1)
    grad_u = lambda P: np.stack([np.stack([vec(gu[c][d])(P) for d in range(2)], -1) for c in range(2)], -2)
    return vec(fx), vec(fy), vec(gg), u_exact, vec(pp), grad_u


@pytest.mark.parametrize("beta", [0.0, 1.0, 1e4])
def test_taylor_hood_orders(beta):
    fx, fy, gg, u_exact, p_exact, grad_u = _fields(beta)
    errs = []
    for N in [4, 8, 16, 32]:
        d = Discretization(mesh.same_diag(N))
        lv = Level(d, beta)
        fu = np.concatenate([quadrature.load_p2(d.mesh, fx)[d.interior],
                             quadrature.load_p2(d.mesh, fy)[d.interior]])
        gp = quadrature.load_p1(d.mesh, gg)
        x = lv.direct_solve(np.concatenate([fu, gp]))
        uh = np.zeros((2, d.n2))
        uh[0, d.interior] = x[: d.nu]
        uh[1, d.interior] = x[d.nu: 2 * d.nu]
        errs.append(quadrature.l2_errors(d, uh, x[2 * d.nu:], u_exact, p_exact, grad_u))
    errs = np.array(errs)
    rates = np.log2(errs[:-1] / errs[1:])
    # last refinement step: asymptotic orders 3, 2, 2
    assert rates[-1, 0] > 2.8, rates
    assert rates[-1, 1] > 1.9, rates
    assert rates[-1, 2] > 1.8, rates


def test_discrete_inf_sup_bounded_below_same_diag():
    """Discrete inf-sup constant min eig(B K^{-1} B^T, M_P) on mean-free pressures
    stays bounded away from zero under refinement for the same-diagonal mesh
    (diagnostic of well-posedness; the union-jack mesh is covered by theory)."""
    vals = []
    for N in [2, 4, 8, 16]:
        d = Discretization(mesh.same_diag(N))
        K = d.K.toarray()
        Kb = np.kron(np.eye(2), K)
        B = d.B().toarray()
        S = B @ np.linalg.solve(Kb, B.T)
        MP = d.MP.toarray()
        # restrict to mean-free pressures (M_P-orthogonal to constants)
        one = np.ones(d.n1)
        Q, _ = np.linalg.qr(np.column_stack([one, np.eye(d.n1)[:, :-1]]))
        Z = Q[:, 1:]
        import scipy.linalg as sl
        ev = sl.eigh(Z.T @ S @ Z, Z.T @ MP @ Z, eigvals_only=True)
        vals.append(ev[0])
    vals = np.array(vals)
    assert np.all(vals > 1e-2), vals
    assert vals[-1] > 0.5 * vals[-2], vals
