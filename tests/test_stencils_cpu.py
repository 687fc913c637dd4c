"""CPU check of the lattice stencil tables that the HIP kernels are generated from.

The tables (gen_stencils.build(), exact rationals) are applied here with plain
numpy loops on the lattice layout and compared against the oracle's
unstructured CSR assembly on small grids.  This pins the constant-coefficient
stencils (A, B, B^T, the P2 mass, Shat and both transfers) before any kernel
runs; the GPU parity tests then pin the kernels themselves.
"""
import importlib.util
import os

import numpy as np
import pytest

from oracle import multigrid as mg
from tests import lattice as lat

_GEN = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                    "paper_1502_04070_amd", "csrc", "gen_stencils.py")
_spec = importlib.util.spec_from_file_location("gen_stencils", _GEN)
gen = importlib.util.module_from_spec(_spec)
_spec.loader.exec_module(gen)
A_TAPS, BT_TAPS, B_TAPS, PRO, RES = gen.build()
PAD = 4


def _cls(a, b):
    return (a % 2) + 2 * (b % 2)


def _pad(x):
    return np.pad(x, [(0, 0)] * (x.ndim - 2) + [(PAD, PAD), (PAD, PAD)])


def apply_lattice(N, beta, u, p):
    h = 1.0 / N
    M = 2 * N + 1
    U = _pad(u)
    P = _pad(p)
    yu = np.zeros_like(u)
    yp = np.zeros_like(p)
    for b in range(1, 2 * N):
        for a in range(1, 2 * N):
            c = _cls(a, b)
            for (da, db, K, Mm) in A_TAPS[c]:
                coef = float(K) + beta * h * h * float(Mm)
                yu[:, b, a] += coef * U[:, PAD + b + db, PAD + a + da]
            for (di, dj, bx, by) in BT_TAPS[c]:
                i, j = a // 2 + di, b // 2 + dj
                yu[0, b, a] += h * float(bx) * P[PAD + j, PAD + i]
                yu[1, b, a] += h * float(by) * P[PAD + j, PAD + i]
    for j in range(N + 1):
        for i in range(N + 1):
            for (da, db, bx, by) in B_TAPS:
                yp[j, i] += h * (float(bx) * U[0, PAD + 2 * j + db, PAD + 2 * i + da]
                                 + float(by) * U[1, PAD + 2 * j + db, PAD + 2 * i + da])
    return yu, yp


@pytest.mark.parametrize("N,beta", [(2, 1.0), (4, 0.0), (6, 37.0), (8, 1e4)])
def test_saddle_stencils_match_assembly(N, beta):
    lv = mg.Level(mg.Discretization(mg.meshmod.same_diag(N)), beta)
    rng = np.random.default_rng(N)
    x = rng.standard_normal(lv.n)
    u, p = lat.to_lattice(lv.disc, x)
    yu, yp = apply_lattice(N, beta, u, p)
    y = lat.from_lattice(lv.disc, yu, yp)
    ref = lv.calA @ x
    assert np.abs(y - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("N,beta", [(4, 2.5), (8, 1e3)])
def test_smoother_diagonals_match(N, beta):
    lv = mg.Level(mg.Discretization(mg.meshmod.same_diag(N)), beta)
    h = 1.0 / N
    # Ahat per class
    ahat = [float(gen.Fr(0)) for _ in range(4)]
    for c in range(4):
        d = [t for t in A_TAPS[c] if t[0] == 0 and t[1] == 0][0]
        ahat[c] = float(d[2]) + beta * h * h * float(d[3])
    A_l = np.zeros((2, 2 * N + 1, 2 * N + 1))
    for b in range(2 * N + 1):
        for a in range(2 * N + 1):
            A_l[:, b, a] = ahat[_cls(a, b)]
    S_l = np.zeros((N + 1, N + 1))
    for j in range(N + 1):
        for i in range(N + 1):
            for (da, db, bx, by) in B_TAPS:
                a, b = 2 * i + da, 2 * j + db
                if 0 < a < 2 * N and 0 < b < 2 * N:
                    S_l[j, i] += h * h * (float(bx) ** 2 + float(by) ** 2) / ahat[_cls(a, b)]
    got = lat.from_lattice(lv.disc, A_l, S_l)
    assert np.allclose(got, lv.Ldiag, rtol=1e-14)


@pytest.mark.parametrize("Nc", [2, 3, 4])
def test_transfer_stencils_match_prolongation(Nc):
    h = mg.Hierarchy("same_diag", 1, 1.0, n0=Nc)
    dc, df = h.discs
    P = h.levels[1].P
    rng = np.random.default_rng(Nc)
    zc = rng.standard_normal(h.levels[0].n)
    uc, pc = lat.to_lattice(dc, zc)
    Nf = 2 * Nc
    uf = np.zeros((2, 2 * Nf + 1, 2 * Nf + 1))
    pf = np.zeros((Nf + 1, Nf + 1))
    UC = _pad(uc)
    for b in range(1, 2 * Nf):
        for a in range(1, 2 * Nf):
            I, J, ra, rb = a // 4, b // 4, a % 4, b % 4
            for (dA, dB, w) in PRO[(ra, rb)]:
                uf[:, b, a] += float(w) * UC[:, PAD + 2 * J + dB, PAD + 2 * I + dA]
    PC = _pad(pc)
    for j in range(Nf + 1):
        for i in range(Nf + 1):
            I, J = i // 2, j // 2
            if i % 2 == 0 and j % 2 == 0:
                pf[j, i] = PC[PAD + J, PAD + I]
            elif j % 2 == 0:
                pf[j, i] = 0.5 * (PC[PAD + J, PAD + I] + PC[PAD + J, PAD + I + 1])
            elif i % 2 == 0:
                pf[j, i] = 0.5 * (PC[PAD + J, PAD + I] + PC[PAD + J + 1, PAD + I])
            else:
                pf[j, i] = 0.5 * (PC[PAD + J, PAD + I] + PC[PAD + J + 1, PAD + I + 1])
    assert np.allclose(lat.from_lattice(df, uf, pf), P @ zc, atol=1e-14)
    # restriction = transpose, as a gather per coarse class
    rf = rng.standard_normal(h.levels[1].n)
    ru, rp = lat.to_lattice(df, rf)
    RU = _pad(ru)
    rcu = np.zeros_like(uc)
    for b in range(1, 2 * Nc):
        for a in range(1, 2 * Nc):
            for (fa, fb, w) in RES[_cls(a, b)]:
                rcu[:, b, a] += float(w) * RU[:, PAD + 2 * b + fb, PAD + 2 * a + fa]
    ref_u, _ = lat.to_lattice(dc, P.T @ rf)
    assert np.allclose(rcu, ref_u, atol=1e-13)


def test_mass_row_gives_load_vector():
    N = 6
    d = mg.Discretization(mg.meshmod.same_diag(N))
    rng = np.random.default_rng(0)
    fn = rng.standard_normal((2, d.n2))
    F, _ = lat.nodal_to_lattice(d, fn, np.zeros(d.n1))
    FP = _pad(F)
    h = 1.0 / N
    fu = np.zeros_like(F)
    for b in range(1, 2 * N):
        for a in range(1, 2 * N):
            for (da, db, K, Mm) in A_TAPS[_cls(a, b)]:
                fu[:, b, a] += h * h * float(Mm) * FP[:, PAD + b + db, PAD + a + da]
    ref, _ = d.load(fn, np.zeros(d.n1))
    got = lat.from_lattice(d, fu, np.zeros((N + 1, N + 1)))[: 2 * d.nu]
    assert np.allclose(got, ref, atol=1e-15)
