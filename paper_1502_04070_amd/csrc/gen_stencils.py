#!/usr/bin/env python3
"""Derive the constant-coefficient lattice stencils of the Taylor-Hood P2-P1
discretization on the uniformly refined same-diagonal grid and emit them as a
C++ header (stencils.inc) for the HIP kernels.

The grid: N x N squares of side h, each cut by the diagonal from its lower-left
to its upper-right corner.  P2 nodes form a lattice of spacing h/2 ("half
units"); lattice point (a, b) is a vertex if a and b are even, a horizontal
edge midpoint if only a is odd, a vertical edge midpoint if only b is odd and
a diagonal midpoint if both are odd.  Square (i, j) "owns" the four lattice
points (2i, 2j), (2i+1, 2j), (2i, 2j+1), (2i+1, 2j+1) and the pressure vertex
(i, j).

Every local integral is computed exactly over the rationals: the P2 basis is
obtained by inverting the 6 x 6 monomial Vandermonde matrix of each triangle
and monomials are integrated in closed form.  Scaling with h: the stiffness
part is h-independent, the mass part scales with h^2 and the divergence
coupling with h (two space dimensions).

Outputs (all in half-unit offsets):
  A_TAPS[class]  : (da, db, K, M)   row of K and M for a velocity node of a class
  BT_TAPS[class] : (di, dj, Bx, By) row of B^T: pressure vertices (offsets in
                   vertex units from the owning square) coupled to the node
  B_TAPS         : (da, db, Bx, By) row of B for the pressure vertex (0, 0)
  PRO_TAPS[ra][rb]: P2 prolongation weights: fine lattice point (4I+ra, 4J+rb)
                   from coarse lattice points (2I+dA, 2J+dB)
  RES_TAPS[class]: the transposed (restriction) gather per coarse class:
                   (fa, fb, w) fine offsets relative to the fine point (2A, 2B)
                   of the coarse lattice point (A, B)
"""
from __future__ import annotations

import os
import sys
from fractions import Fraction as Fr
from itertools import product

MONO = [(0, 0), (1, 0), (0, 1), (2, 0), (1, 1), (0, 2)]   # 1, x, y, x^2, xy, y^2


def _solve(Amat, rhs_cols):
    """Exact Gauss-Jordan inverse applied to columns."""
    n = len(Amat)
    M = [list(r) + list(c) for r, c in zip(Amat, rhs_cols)]
    for col in range(n):
        piv = next(r for r in range(col, n) if M[r][col] != 0)
        M[col], M[piv] = M[piv], M[col]
        pv = M[col][col]
        M[col] = [v / pv for v in M[col]]
        for r in range(n):
            if r != col and M[r][col] != 0:
                f = M[r][col]
                M[r] = [a - f * b for a, b in zip(M[r], M[col])]
    return [row[n:] for row in M]


class Tri:
    """A triangle of the unit-leg lattice, given by its three vertices in half
    units; nodes = 3 vertices + 3 edge midpoints (all in half units)."""

    def __init__(self, verts, kind):
        self.kind = kind                 # "L": below the diagonal, "U": above
        self.verts = verts
        v = verts
        mids = [((v[0][0] + v[1][0]) // 2, (v[0][1] + v[1][1]) // 2),
                ((v[1][0] + v[2][0]) // 2, (v[1][1] + v[2][1]) // 2),
                ((v[2][0] + v[0][0]) // 2, (v[2][1] + v[0][1]) // 2)]
        self.nodes = list(v) + mids
        # P2 basis: coefficient vectors over MONO; node coordinates in unit legs
        V = [[Fr(x, 2) ** e[0] * Fr(y, 2) ** e[1] for e in MONO] for (x, y) in self.nodes]
        # solve V c_j = e_j  (column j of V^{-1})
        ident = [[Fr(int(i == j)) for j in range(6)] for i in range(6)]
        inv = _solve(V, ident)                       # inv = V^{-1}
        self.p2 = [[inv[r][j] for r in range(6)] for j in range(6)]
        # P1 basis on the vertices
        V1 = [[Fr(1), Fr(x, 2), Fr(y, 2)] for (x, y) in v]
        inv1 = _solve(V1, [[Fr(int(i == j)) for j in range(3)] for i in range(3)])
        self.p1 = [[inv1[r][j] for r in range(3)] for j in range(3)]   # over (1, x, y)
        # integration: translate so that the lower-left corner of the square is 0
        self.x0 = min(x for x, _ in v) // 2
        self.y0 = min(y for _, y in v) // 2

    def int_mono(self, a, b):
        """Exact integral of x^a y^b over the triangle (unit legs)."""
        # expand (x0 + s)^a (y0 + t)^b over the reference triangle in (s, t)
        from math import comb
        tot = Fr(0)
        for i in range(a + 1):
            for j in range(b + 1):
                c = comb(a, i) * comb(b, j) * Fr(self.x0) ** (a - i) * Fr(self.y0) ** (b - j)
                if self.kind == "L":          # 0 <= t <= s <= 1
                    tot += c * Fr(1, (j + 1) * (i + j + 2))
                else:                          # 0 <= s <= t <= 1
                    tot += c * Fr(1, (i + 1) * (i + j + 2))
        return tot


def _poly_mul(p, q):
    out = {}
    for (a, b), c in p.items():
        for (d, e), f in q.items():
            out[(a + d, b + e)] = out.get((a + d, b + e), 0) + c * f
    return out


def _poly(coeffs, mono):
    return {m: c for m, c in zip(mono, coeffs) if c != 0}


def _dx(p):
    return {(a - 1, b): c * a for (a, b), c in p.items() if a > 0}


def _dy(p):
    return {(a, b - 1): c * b for (a, b), c in p.items() if b > 0}


def _integrate(tri, p):
    return sum((c * tri.int_mono(a, b) for (a, b), c in p.items()), Fr(0))


def local_matrices(tri):
    P = [_poly(c, MONO) for c in tri.p2]
    L = [_poly(c, [(0, 0), (1, 0), (0, 1)]) for c in tri.p1]
    K = [[_integrate(tri, _poly_mul(_dx(P[i]), _dx(P[j]))) + _integrate(tri, _poly_mul(_dy(P[i]), _dy(P[j])))
          for j in range(6)] for i in range(6)]
    M = [[_integrate(tri, _poly_mul(P[i], P[j])) for j in range(6)] for i in range(6)]
    Bx = [[_integrate(tri, _poly_mul(L[k], _dx(P[j]))) for j in range(6)] for k in range(3)]
    By = [[_integrate(tri, _poly_mul(L[k], _dy(P[j]))) for j in range(6)] for k in range(3)]
    return P, K, M, Bx, By


def lattice_triangles(r=3):
    tris = []
    for i, j in product(range(-r, r), range(-r, r)):
        a, b, c, d = (2 * i, 2 * j), (2 * i + 2, 2 * j), (2 * i + 2, 2 * j + 2), (2 * i, 2 * j + 2)
        tris.append(Tri([a, b, c], "L"))
        tris.append(Tri([a, c, d], "U"))
    return tris


CLASS_POS = [(0, 0), (1, 0), (0, 1), (1, 1)]          # V, H, E, D
CLASS_NAME = ["V", "H", "E", "D"]


def build():
    tris = lattice_triangles()
    loc = {}
    # local matrices only depend on the triangle kind (translation invariance);
    # compute once per kind at the origin and reuse.
    ref = {"L": Tri([(0, 0), (2, 0), (2, 2)], "L"), "U": Tri([(0, 0), (2, 2), (0, 2)], "U")}
    for k, t in ref.items():
        loc[k] = local_matrices(t)
    A_TAPS, BT_TAPS = [], []
    for pos in CLASS_POS:
        acc = {}
        bt = {}
        for t in tris:
            if pos not in t.nodes:
                continue
            _, K, M, Bx, By = loc[t.kind]
            a = t.nodes.index(pos)
            for b, nb in enumerate(t.nodes):
                off = (nb[0] - pos[0], nb[1] - pos[1])
                k0, m0 = acc.get(off, (Fr(0), Fr(0)))
                acc[off] = (k0 + K[a][b], m0 + M[a][b])
            for kv, vv in enumerate(t.verts):
                offp = (vv[0] // 2, vv[1] // 2)          # owning square of pos is (0, 0)
                x0, y0 = bt.get(offp, (Fr(0), Fr(0)))
                bt[offp] = (x0 + Bx[kv][a], y0 + By[kv][a])
        A_TAPS.append(sorted((d[0], d[1], k, m) for d, (k, m) in acc.items() if k != 0 or m != 0))
        BT_TAPS.append(sorted((d[0], d[1], x, y) for d, (x, y) in bt.items() if x != 0 or y != 0))
    # B row of the pressure vertex (0, 0)
    brow = {}
    for t in tris:
        if (0, 0) not in t.verts:
            continue
        _, K, M, Bx, By = loc[t.kind]
        kv = t.verts.index((0, 0))
        for b, nb in enumerate(t.nodes):
            x0, y0 = brow.get(nb, (Fr(0), Fr(0)))
            brow[nb] = (x0 + Bx[kv][b], y0 + By[kv][b])
    B_TAPS = sorted((d[0], d[1], x, y) for d, (x, y) in brow.items() if x != 0 or y != 0)
    # consistency: B^T taps are the transpose of the B taps
    for ci, pos in enumerate(CLASS_POS):
        for (di, dj, x, y) in BT_TAPS[ci]:
            # pressure vertex (di, dj) sees pos at offset pos - (2di, 2dj)
            off = (pos[0] - 2 * di, pos[1] - 2 * dj)
            match = [tp for tp in B_TAPS if (tp[0], tp[1]) == off]
            assert match and match[0][2] == x and match[0][3] == y, (ci, di, dj)
    # P2 prolongation from the coarse cell (I, J) to the 16 fine points it owns
    coarse = {"L": Tri([(0, 0), (2, 0), (2, 2)], "L"), "U": Tri([(0, 0), (2, 2), (0, 2)], "U")}
    PRO = {}
    for ra, rb in product(range(4), range(4)):
        x, y = Fr(ra, 4), Fr(rb, 4)                      # in coarse unit legs
        t = coarse["L"] if rb <= ra else coarse["U"]
        w = []
        for j, node in enumerate(t.nodes):
            c = t.p2[j]
            val = sum((cc * x ** e[0] * y ** e[1] for cc, e in zip(c, MONO)), Fr(0))
            if val != 0:
                w.append((node[0], node[1], val))
        PRO[(ra, rb)] = sorted(w)
    RES = []
    for cpos in CLASS_POS:
        acc = {}
        for I, J in product(range(-2, 2), range(-2, 2)):
            for (ra, rb), taps in PRO.items():
                for (dA, dB, w) in taps:
                    if (2 * I + dA, 2 * J + dB) == cpos:
                        f = (4 * I + ra - 2 * cpos[0], 4 * J + rb - 2 * cpos[1])
                        acc[f] = acc.get(f, Fr(0)) + w
        RES.append(sorted((a, b, w) for (a, b), w in acc.items() if w != 0))
    return A_TAPS, BT_TAPS, B_TAPS, PRO, RES


def square_matrices():
    """Square-local matrices of one grid square and both diagonal directions
    (union-jack grid), over the 9 P2 lattice nodes of the square (index
    3 lb + la, half units (la, lb) in 0..2) and its 4 corners (index 2 pb + pa):
    K, M (9 x 9), Bx, By (4 x 9), MP (4 x 4, P1 mass), PRO (16 x 9: owned fine
    point 4 rb + ra of the refined square from the square's nodes), PP (4 x 4:
    owned fine vertex 2 pb + pa from the corners).  Orientation 0: diagonal
    from the lower-left to the upper-right corner; 1: the other diagonal, the
    mirror image x -> 1 - x of orientation 0 (stiffness and mass invariant,
    the x-derivative changes sign)."""
    ref = {"L": Tri([(0, 0), (2, 0), (2, 2)], "L"), "U": Tri([(0, 0), (2, 2), (0, 2)], "U")}
    z9 = lambda: [[Fr(0)] * 9 for _ in range(9)]
    K0, M0 = z9(), z9()
    BX0 = [[Fr(0)] * 9 for _ in range(4)]
    BY0 = [[Fr(0)] * 9 for _ in range(4)]
    MP0 = [[Fr(0)] * 4 for _ in range(4)]
    for t in ref.values():
        _, K, M, Bx, By = local_matrices(t)
        idx = [n[1] * 3 + n[0] for n in t.nodes]
        cidx = [(v[1] // 2) * 2 + v[0] // 2 for v in t.verts]
        for a in range(6):
            for b in range(6):
                K0[idx[a]][idx[b]] += K[a][b]
                M0[idx[a]][idx[b]] += M[a][b]
        for k in range(3):
            for b in range(6):
                BX0[cidx[k]][idx[b]] += Bx[k][b]
                BY0[cidx[k]][idx[b]] += By[k][b]
        # P1 mass of the triangle: area/12 (1 + delta_kl), area 1/2 in unit legs
        for k in range(3):
            for l in range(3):
                MP0[cidx[k]][cidx[l]] += Fr(1, 24) * (2 if k == l else 1)
    mir9 = lambda n: (n // 3) * 3 + (2 - n % 3)
    mir4 = lambda q: (q // 2) * 2 + (1 - q % 2)
    K1 = [[K0[mir9(a)][mir9(b)] for b in range(9)] for a in range(9)]
    M1 = [[M0[mir9(a)][mir9(b)] for b in range(9)] for a in range(9)]
    BX1 = [[-BX0[mir4(q)][mir9(b)] for b in range(9)] for q in range(4)]
    BY1 = [[BY0[mir4(q)][mir9(b)] for b in range(9)] for q in range(4)]
    MP1 = [[MP0[mir4(q)][mir4(r)] for r in range(4)] for q in range(4)]
    _, _, _, PRO, _ = build()
    PRO0 = [[Fr(0)] * 9 for _ in range(16)]
    for (ra, rb), taps in PRO.items():
        for (dA, dB, w) in taps:
            PRO0[rb * 4 + ra][dB * 3 + dA] = w
    PRO1 = [[Fr(0)] * 9 for _ in range(16)]
    for ra, rb in product(range(4), range(4)):
        for c in range(9):
            if ra == 0:                       # the square's left edge: the same 1-D rule
                PRO1[rb * 4 + ra][c] = PRO0[rb * 4 + ra][c]
            else:
                PRO1[rb * 4 + ra][c] = PRO0[rb * 4 + (4 - ra)][mir9(c)]
    h = Fr(1, 2)
    PP0 = [[Fr(1), 0, 0, 0], [h, h, 0, 0], [h, 0, h, 0], [h, 0, 0, h]]
    PP1 = [[Fr(1), 0, 0, 0], [h, h, 0, 0], [h, 0, h, 0], [0, h, h, 0]]
    return {"K": (K0, K1), "M": (M0, M1), "BX": (BX0, BX1), "BY": (BY0, BY1), "MP": (MP0, MP1),
            "PRO": (PRO0, PRO1), "PP": (PP0, PP1)}


def _lit(fr):
    """C++ literal of an exact rational, converted to the arithmetic type T of
    the code that expands the macro (T must be a type name in scope)."""
    if fr.denominator == 1:
        return f"T({fr.numerator}.0)"
    return f"T({fr.numerator}.0/{fr.denominator}.0)"


def _dlit(fr):
    """Plain double literal (for constexpr tables)."""
    if fr.denominator == 1:
        return f"{fr.numerator}.0"
    return f"({fr.numerator}.0/{fr.denominator}.0)"


def emit(path):
    A_TAPS, BT_TAPS, B_TAPS, PRO, RES = build()
    L = []
    w = L.append
    w("// Generated by gen_stencils.py -- do not edit.")
    w("// Constant lattice stencils of the Taylor-Hood P2-P1 discretization on the")
    w("// same-diagonal grid (offsets in half cells; see gen_stencils.py).")
    w("#pragma once")
    w("namespace smg_stencil {")
    # A: group taps by identical (K, M) pairs -> coefficient index per class
    w("// ---- velocity block A = K + (beta h^2) M, one table per node class ----")
    w("// A_NGROUP[c] groups; group g has stiffness A_K[c][g] and mass A_M[c][g];")
    w("// the row is sum_g (A_K + beta h^2 A_M)[c][g] * sum_{taps in g} u(da, db).")
    groups_all = []
    for ci, taps in enumerate(A_TAPS):
        groups = {}
        for (da, db, k, m) in taps:
            groups.setdefault((k, m), []).append((da, db))
        groups_all.append(groups)
    maxg = max(len(g) for g in groups_all)
    w(f"constexpr int A_MAXG = {maxg};")
    w("constexpr int A_NGROUP[4] = {" + ", ".join(str(len(g)) for g in groups_all) + "};")
    w("constexpr double A_K[4][A_MAXG] = {")
    for g in groups_all:
        vals = [_dlit(k) for (k, m) in g.keys()] + ["0.0"] * (maxg - len(g))
        w("  {" + ", ".join(vals) + "},")
    w("};")
    w("constexpr double A_M[4][A_MAXG] = {")
    for g in groups_all:
        vals = [_dlit(m) for (k, m) in g.keys()] + ["0.0"] * (maxg - len(g))
        w("  {" + ", ".join(vals) + "},")
    w("};")
    w("// Row of A for class c at the lattice point P: U(da, db) reads u at P + (da, db),")
    w("// C(g) is the combined coefficient of group g of class c.")
    for ci, g in enumerate(groups_all):
        w(f"#define SMG_A_ROW_{CLASS_NAME[ci]}(U, C) ( \\")
        terms = []
        for gi, (key, offs) in enumerate(g.items()):
            s = " + ".join(f"U({da},{db})" for (da, db) in offs)
            terms.append(f"    C({gi}) * ({s})")
        w(" + \\\n".join(terms) + " )")
    # B^T rows (velocity node, pressure columns): x and y component, h-scaled
    w("// ---- B^T: velocity row of class c, pressure vertices at (i+di, j+dj), times h ----")
    for ci, taps in enumerate(BT_TAPS):
        for comp, idx in (("X", 2), ("Y", 3)):
            terms = [f"{_lit(tp[idx])} * P({tp[0]},{tp[1]})" for tp in taps if tp[idx] != 0] or ["0.0"]
            w(f"#define SMG_BT{comp}_ROW_{CLASS_NAME[ci]}(P) ( " + " + ".join(terms) + " )")
    # B row (pressure vertex): sum over velocity lattice offsets, times h
    w("// ---- B: row of the pressure vertex at lattice point (2i, 2j), times h ----")
    for comp, idx in (("X", 2), ("Y", 3)):
        terms = [f"{_lit(tp[idx])} * U({tp[0]},{tp[1]})" for tp in B_TAPS if tp[idx] != 0]
        w(f"#define SMG_B{comp}_ROW(U) ( " + " + \\\n    ".join(terms) + " )")
    # tap lists for S-hat (needs per-tap B values and classes)
    w("// ---- B taps as a table (for diag(B Ahat^-1 B^T)) ----")
    w(f"constexpr int B_NTAP = {len(B_TAPS)};")
    w("constexpr int B_TAP_OFF[B_NTAP][2] = {" + ", ".join(f"{{{a},{b}}}" for a, b, _, _ in B_TAPS) + "};")
    w("constexpr double B_TAP_X[B_NTAP] = {" + ", ".join(_dlit(x) for _, _, x, _ in B_TAPS) + "};")
    w("constexpr double B_TAP_Y[B_NTAP] = {" + ", ".join(_dlit(y) for _, _, _, y in B_TAPS) + "};")
    # diag(B Ahat^-1 B^T) row: sum over taps of (Bx^2 + By^2) / Ahat(class of the tap),
    # skipping taps that are not interior velocity nodes; IN(da, db) is that test,
    # AD(c) is 1 / Ahat of class c.  Times h^2.
    terms = []
    for (da, db, x, y) in B_TAPS:
        c = (da % 2) + 2 * (db % 2)
        terms.append(f"(IN({da},{db}) ? {_lit(x * x + y * y)} * AD({c}) : T(0))")
    w("#define SMG_SHAT_ROW(IN, AD) ( " + " + \\\n    ".join(terms) + " )")
    # diagonal of A per class
    w("// ---- diagonal of K and M per class (V, H, E, D) ----")
    dk = []
    dm = []
    for taps in A_TAPS:
        d = [tp for tp in taps if tp[0] == 0 and tp[1] == 0][0]
        dk.append(_dlit(d[2]))
        dm.append(_dlit(d[3]))
    w("constexpr double DIAG_K[4] = {" + ", ".join(dk) + "};")
    w("constexpr double DIAG_M[4] = {" + ", ".join(dm) + "};")
    # mass-only rows for the load vector M_full f (all lattice points)
    w("// ---- P2 mass row per class (load vectors; taps over all lattice points), times h^2 ----")
    for ci, taps in enumerate(A_TAPS):
        terms = [f"{_lit(tp[3])} * U({tp[0]},{tp[1]})" for tp in taps if tp[3] != 0]
        w(f"#define SMG_M_ROW_{CLASS_NAME[ci]}(U) ( " + " + \\\n    ".join(terms) + " )")
    # prolongation
    w("// ---- P2 prolongation: fine point (4I+ra, 4J+rb) from coarse points (2I+dA, 2J+dB) ----")
    for (ra, rb), taps in sorted(PRO.items()):
        terms = [f"{_lit(wt)} * Z({dA},{dB})" for (dA, dB, wt) in taps]
        w(f"#define SMG_PRO_{ra}{rb}(Z) ( " + " + ".join(terms) + " )")
    w("// ---- P2 restriction (transpose): coarse point (A, B) of class c gathers fine (2A+fa, 2B+fb) ----")
    for ci, taps in enumerate(RES):
        terms = [f"{_lit(wt)} * R({fa},{fb})" for (fa, fb, wt) in taps]
        w(f"#define SMG_RES_ROW_{CLASS_NAME[ci]}(R) ( " + " + \\\n    ".join(terms) + " )")
    # square-local matrices of both diagonal directions (union-jack grid)
    SQ = square_matrices()
    w("// ---- square-local matrices, orientation 0 (diagonal /) and 1 (diagonal \\) ----")
    w("// nodes 3 lb + la (half units in the square), corners 2 pb + pa; K, M and")
    w("// MP in unit legs (M, MP times h^2 and B times h at use); PRO: owned fine")
    w("// point 4 rb + ra of the refined square from the square's nodes; PP: owned")
    w("// fine vertex 2 pb + pa from the corners")
    shapes = {"K": (9, 9), "M": (9, 9), "BX": (4, 9), "BY": (4, 9), "MP": (4, 4), "PRO": (16, 9), "PP": (4, 4)}
    for name, (r, c) in shapes.items():
        w(f"constexpr double UJ_{name}[2][{r}][{c}] = {{")
        for o in range(2):
            rows = ["{" + ", ".join(_dlit(Fr(v)) for v in row) + "}" for row in SQ[name][o]]
            w("  {" + ",\n   ".join(rows) + "},")
        w("};")
    w("}  // namespace smg_stencil")
    with open(path, "w") as fh:
        fh.write("\n".join(L) + "\n")
    return A_TAPS, BT_TAPS, B_TAPS, PRO, RES


if __name__ == "__main__":
    out = sys.argv[1] if len(sys.argv) > 1 else os.path.join(os.path.dirname(os.path.abspath(__file__)), "stencils.inc")
    A, BT, B, PRO, RES = emit(out)
    for ci in range(4):
        print(CLASS_NAME[ci], "A taps", len(A[ci]), "BT taps", len(BT[ci]), "RES taps", len(RES[ci]))
    print("B taps", len(B))
