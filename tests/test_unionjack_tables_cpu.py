"""CPU pins of the square-local tables behind the union-jack kernels.

gen_stencils.square_matrices() gives, for both diagonal directions, the exact
square-local stiffness, mass and divergence matrices and the local
prolongation weights.  Here they are scattered square by square with plain
numpy loops (the grid's diagonal direction from the quarter a square lies in)
and compared with the oracle's independent unstructured assembly on its
union-jack hierarchy (Section 6 grid): the saddle operator, the P1 mass, the
velocity mass and the prolongation.  The main-diagonal tables must also
reproduce the same-diagonal lattice stencils.
"""
import importlib.util
import os

import numpy as np
import pytest

from oracle import multigrid as mg
from tests import lattice as lat

_GEN = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                    "paper_1502_04070_amd", "csrc", "gen_stencils.py")
_spec = importlib.util.spec_from_file_location("gen_stencils_uj", _GEN)
gen = importlib.util.module_from_spec(_spec)
_spec.loader.exec_module(gen)
SQ = {k: tuple(np.array(m, dtype=float) for m in v) for k, v in gen.square_matrices().items()}


def orient(N, si, sj):
    return 1 if ((2 * si < N) != (2 * sj < N)) else 0


def interior_mask(N):
    a = np.arange(2 * N + 1)
    A, B = np.meshgrid(a, a)
    return (A > 0) & (A < 2 * N) & (B > 0) & (B < 2 * N)


def apply_uj(N, beta, u, p):
    """calA (u, p) on the union-jack grid by scattering square-local products."""
    h = 1.0 / N
    yu = np.zeros_like(u)
    yp = np.zeros_like(p)
    for sj in range(N):
        for si in range(N):
            o = orient(N, si, sj)
            A = SQ["K"][o] + beta * h * h * SQ["M"][o]
            la = [(2 * si + m % 3, 2 * sj + m // 3) for m in range(9)]
            lp = [(si + q % 2, sj + q // 2) for q in range(4)]
            ul = np.array([[u[c, b, a] for (a, b) in la] for c in range(2)])
            pl = np.array([p[j, i] for (i, j) in lp])
            yl = [A @ ul[0] + h * SQ["BX"][o].T @ pl, A @ ul[1] + h * SQ["BY"][o].T @ pl]
            ypl = h * (SQ["BX"][o] @ ul[0] + SQ["BY"][o] @ ul[1])
            for m, (a, b) in enumerate(la):
                yu[0, b, a] += yl[0][m]
                yu[1, b, a] += yl[1][m]
            for q, (i, j) in enumerate(lp):
                yp[j, i] += ypl[q]
    yu[:, ~interior_mask(N)] = 0.0
    return yu, yp


def prolong_uj(Nc, zu, zp):
    """P z on the union-jack grid: every coarse square interpolates at the
    fine points it owns (right and top boundary owned by squares I = Nc, J = Nc)."""
    Nf = 2 * Nc
    u = np.zeros((2, 2 * Nf + 1, 2 * Nf + 1))
    p = np.zeros((Nf + 1, Nf + 1))
    for J in range(Nc + 1):
        for I in range(Nc + 1):
            o = orient(Nc, min(I, Nc - 1), min(J, Nc - 1))
            z = np.zeros((2, 9))
            for k in range(9):
                A, B = 2 * I + k % 3, 2 * J + k // 3
                if A <= 2 * Nc and B <= 2 * Nc:
                    z[:, k] = zu[:, B, A]
            for f in range(16):
                a, b = 4 * I + f % 4, 4 * J + f // 4
                if a <= 2 * Nf and b <= 2 * Nf:
                    u[:, b, a] += SQ["PRO"][o][f] @ z.T
            zc = np.array([zp[J + q // 2, I + q % 2] if (I + q % 2 <= Nc and J + q // 2 <= Nc) else 0.0
                           for q in range(4)])
            for v in range(4):
                fi, fj = 2 * I + v % 2, 2 * J + v // 2
                if fi <= Nf and fj <= Nf:
                    p[fj, fi] += SQ["PP"][o][v] @ zc
    u[:, ~interior_mask(Nf)] = 0.0
    return u, p


@pytest.fixture(scope="module")
def uj():
    return mg.Hierarchy("union_jack", 2, 7.0)          # N = 2, 4, 8


def _rand_state(N, seed):
    rng = np.random.default_rng(seed)
    u = rng.standard_normal((2, 2 * N + 1, 2 * N + 1))
    u[:, ~interior_mask(N)] = 0.0
    return u, rng.standard_normal((N + 1, N + 1))


@pytest.mark.parametrize("k", [0, 1, 2])
def test_saddle_operator_matches_oracle_assembly(uj, k):
    d, lv = uj.discs[k], uj.levels[k]
    N = lat.level_N(d)
    u, p = _rand_state(N, 10 + k)
    yu, yp = apply_uj(N, 7.0, u, p)
    ref = lv.calA @ lat.from_lattice(d, u, p)
    got = lat.from_lattice(d, yu, yp)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_masses_match_oracle_assembly(uj):
    d = uj.discs[2]
    N = lat.level_N(d)
    rng = np.random.default_rng(3)
    g = rng.standard_normal((N + 1, N + 1))
    h = 1.0 / N
    yp = np.zeros_like(g)
    yu = np.zeros((2 * N + 1, 2 * N + 1))
    f = rng.standard_normal((2 * N + 1, 2 * N + 1))
    for sj in range(N):
        for si in range(N):
            o = orient(N, si, sj)
            lp = [(si + q % 2, sj + q // 2) for q in range(4)]
            la = [(2 * si + m % 3, 2 * sj + m // 3) for m in range(9)]
            yl = h * h * SQ["MP"][o] @ np.array([g[j, i] for (i, j) in lp])
            for q, (i, j) in enumerate(lp):
                yp[j, i] += yl[q]
            ym = h * h * SQ["M"][o] @ np.array([f[b, a] for (a, b) in la])
            for m, (a, b) in enumerate(la):
                yu[b, a] += ym[m]
    _, gn = lat.lattice_to_nodal(d, np.zeros((2, 2 * N + 1, 2 * N + 1)), g)
    got_p = lat.lattice_to_nodal(d, np.zeros((2, 2 * N + 1, 2 * N + 1)), yp)[1]
    assert np.abs(got_p - d.MP @ gn).max() <= 1e-14
    fn = lat.lattice_to_nodal(d, np.stack([f, f]), g)[0][0]
    got_u = lat.lattice_to_nodal(d, np.stack([yu, yu]), g)[0][0]
    assert np.abs(got_u - d.M_full @ fn).max() <= 1e-14


@pytest.mark.parametrize("k", [1, 2])
def test_prolongation_matches_oracle(uj, k):
    dc, df = uj.discs[k - 1], uj.discs[k]
    Nc = lat.level_N(dc)
    zu, zp = _rand_state(Nc, 20 + k)
    u, p = prolong_uj(Nc, zu, zp)
    ref = uj.levels[k].P @ lat.from_lattice(dc, zu, zp)
    assert np.abs(lat.from_lattice(df, u, p) - ref).max() <= 1e-14 * np.abs(ref).max()


def test_main_diagonal_tables_give_the_lattice_stencils():
    """Orientation 0 scattered over the 2 x 2 squares around a node equals the
    same-diagonal row stencils (A, B^T, B) of the lattice kernels."""
    A_TAPS, BT_TAPS, B_TAPS, PRO, _ = gen.build()
    for cls, (DA, DB) in enumerate(gen.CLASS_POS):
        K, M = {}, {}
        for dj in ([-1, 0] if DB == 0 else [0]):
            for di in ([-1, 0] if DA == 0 else [0]):
                ln = 3 * (DB - 2 * dj) + (DA - 2 * di)
                for m in range(9):
                    off = (2 * di + m % 3 - DA, 2 * dj + m // 3 - DB)
                    K[off] = K.get(off, 0.0) + SQ["K"][0][ln][m]
                    M[off] = M.get(off, 0.0) + SQ["M"][0][ln][m]
        ref = {(da, db): (float(k), float(m)) for (da, db, k, m) in A_TAPS[cls]}
        got = {o: (K[o], M[o]) for o in K if abs(K[o]) > 0 or abs(M[o]) > 0}
        assert set(got) == set(ref)
        for o in ref:
            assert abs(got[o][0] - ref[o][0]) < 1e-15 and abs(got[o][1] - ref[o][1]) < 1e-15
    bx = {}
    for dj in (-1, 0):
        for di in (-1, 0):
            q = 2 * (-dj) + (-di)
            for m in range(9):
                off = (2 * di + m % 3, 2 * dj + m // 3)
                bx[off] = bx.get(off, np.zeros(2)) + np.array([SQ["BX"][0][q][m], SQ["BY"][0][q][m]])
    for (da, db, x, y) in B_TAPS:
        assert np.allclose(bx[(da, db)], [float(x), float(y)], atol=1e-15)
    for (ra, rb), taps in PRO.items():
        row = SQ["PRO"][0][rb * 4 + ra]
        for (dA, dB, w) in taps:
            assert abs(row[dB * 3 + dA] - float(w)) < 1e-15
