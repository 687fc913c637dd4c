"""Taylor-Hood P2-P1 element matrices and global assembly, by exact integration.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Paper, Section 2 (discretization): Galerkin method on X_k = U_k x P_k with
continuous piecewise quadratic velocities (zero on the boundary, two
components) and continuous piecewise linear pressures (Taylor-Hood).  In a
nodal basis the discrete problem is the saddle-point system

        [ A_k  B_k^T ] [u]   [f]
        [ B_k    0   ] [p] = [g],

where A_k represents (grad u, grad v) + beta (u, v) and B_k represents
(div u, q) (the matrix form of the variational problem of Section 2).

Every integral below is a polynomial in the barycentric coordinates and is
computed exactly with

        int_T l1^a l2^b l3^c dx = 2 |T| a! b! c! / (a + b + c + 2)!.

Nothing is specialised to the structured meshes: any triangulation works.
"""
from __future__ import annotations

from functools import lru_cache
from itertools import product
from math import factorial

import numpy as np
import scipy.sparse as sp

from .mesh import Mesh

# ---------------------------------------------------------------------------
# polynomials in barycentric coordinates: dict {(a, b, c): coefficient}
# ---------------------------------------------------------------------------


def _pmul(p, q):
    out = {}
    for ea, ca in p.items():
        for eb, cb in q.items():
            e = (ea[0] + eb[0], ea[1] + eb[1], ea[2] + eb[2])
            out[e] = out.get(e, 0.0) + ca * cb
    return out


def _pderiv(p, k):
    out = {}
    for e, c in p.items():
        if e[k] > 0:
            f = list(e)
            f[k] -= 1
            f = tuple(f)
            out[f] = out.get(f, 0.0) + c * e[k]
    return out


def _pint(p):
    """Integral over a triangle of unit area."""
    s = 0.0
    for (a, b, c), coef in p.items():
        s += coef * 2.0 * factorial(a) * factorial(b) * factorial(c) / factorial(a + b + c + 2)
    return s


def _lam(k):
    e = [0, 0, 0]
    e[k] = 1
    return {tuple(e): 1.0}


def p2_basis():
    """Local P2 basis: vertex i -> l_i (2 l_i - 1); edge (i, j) -> 4 l_i l_j.
    Local order: v0, v1, v2, m01, m12, m20."""
    basis = []
    for i in range(3):
        li = _lam(i)
        two_li_minus_one = {(0, 0, 0): -1.0, tuple(1 if q == i else 0 for q in range(3)): 2.0}
        basis.append(_pmul(li, two_li_minus_one))
    for (i, j) in [(0, 1), (1, 2), (2, 0)]:
        basis.append(_pmul({(0, 0, 0): 4.0}, _pmul(_lam(i), _lam(j))))
    return basis


def p1_basis():
    return [_lam(i) for i in range(3)]


@lru_cache(maxsize=None)
def _reference_integrals():
    """Area-normalised integrals that do not depend on the triangle's shape."""
    b2 = p2_basis()
    b1 = p1_basis()
    d2 = [[_pderiv(f, k) for k in range(3)] for f in b2]
    IM = np.array([[_pint(_pmul(f, g)) for g in b2] for f in b2])                   # (6,6)
    IK = np.zeros((6, 6, 3, 3))
    for i, j, k, l in product(range(6), range(6), range(3), range(3)):
        IK[i, j, k, l] = _pint(_pmul(d2[i][k], d2[j][l]))
    IB = np.zeros((3, 6, 3))
    for i, j, k in product(range(3), range(6), range(3)):
        IB[i, j, k] = _pint(_pmul(b1[i], d2[j][k]))
    IM1 = np.array([[_pint(_pmul(f, g)) for g in b1] for f in b1])                  # (3,3)
    I2 = np.array([_pint(f) for f in b2])                                            # (6,)
    I1 = np.array([_pint(f) for f in b1])                                            # (3,)
    return IM, IK, IB, IM1, I2, I1


def _bary_gradients(mesh: Mesh):
    """grad l_k on every triangle: (nt, 3, 2), and areas (nt,)."""
    p = mesh.pts[mesh.tris]                       # (nt, 3, 2)
    x, y = p[..., 0], p[..., 1]
    area2 = (x[:, 1] - x[:, 0]) * (y[:, 2] - y[:, 0]) - (x[:, 2] - x[:, 0]) * (y[:, 1] - y[:, 0])
    g = np.empty((mesh.nt, 3, 2))
    for k in range(3):
        k1, k2 = (k + 1) % 3, (k + 2) % 3
        g[:, k, 0] = (y[:, k1] - y[:, k2]) / area2
        g[:, k, 1] = (x[:, k2] - x[:, k1]) / area2
    return g, 0.5 * area2


def element_matrices(mesh: Mesh):
    """Per-triangle P2 stiffness K_T, P2 mass M_T (6x6), the coupling blocks
    Bx_T[i, j] = int_T l_i d/dx psi_j and By_T (3x6), and the P1 mass (3x3)."""
    IM, IK, IB, IM1, _, _ = _reference_integrals()
    g, area = _bary_gradients(mesh)
    G = np.einsum("tkd,tld->tkl", g, g)                       # grad l_k . grad l_l
    K = area[:, None, None] * np.einsum("ijkl,tkl->tij", IK, G)
    M = area[:, None, None] * IM[None]
    Bx = area[:, None, None] * np.einsum("ijk,tk->tij", IB, g[:, :, 0])
    By = area[:, None, None] * np.einsum("ijk,tk->tij", IB, g[:, :, 1])
    M1 = area[:, None, None] * IM1[None]
    return K, M, Bx, By, M1


def _assemble(rows, cols, vals, shape):
    r = np.broadcast_to(rows[:, :, None], vals.shape).ravel()
    c = np.broadcast_to(cols[:, None, :], vals.shape).ravel()
    return sp.coo_matrix((vals.ravel(), (r, c)), shape=shape).tocsr()


class Discretization:
    """All matrices of one grid level.

    Velocity unknowns: both components at the interior P2 nodes, ordered
    [x-component interior nodes, y-component interior nodes].
    Pressure unknowns: all P1 nodes (= all vertices).  The constant pressure
    is the kernel of B^T; the mean-zero condition of P_k is imposed by
    projection (see multigrid.project_mean) and, on the coarsest grid, by a
    bordered direct solve.
    """

    def __init__(self, mesh: Mesh):
        self.mesh = mesh
        K, M, Bx, By, M1 = element_matrices(mesh)
        d2 = mesh.p2_tri_dofs()
        n2 = mesh.nv + mesh.ne
        n1 = mesh.nv
        self.n2, self.n1 = n2, n1
        self.K_full = _assemble(d2, d2, K, (n2, n2))
        self.M_full = _assemble(d2, d2, M, (n2, n2))
        self.Bx_full = _assemble(mesh.tris, d2, Bx, (n1, n2))
        self.By_full = _assemble(mesh.tris, d2, By, (n1, n2))
        self.MP = _assemble(mesh.tris, mesh.tris, M1, (n1, n1))
        self.coords2 = mesh.p2_coords()
        self.coords1 = mesh.pts.copy()
        self.interior = np.flatnonzero(~mesh.boundary_mask(self.coords2))
        ii = self.interior
        self.nu = len(ii)              # interior nodes per component
        self.K = self.K_full[ii][:, ii].tocsr()
        self.M = self.M_full[ii][:, ii].tocsr()
        self.Bx = self.Bx_full[:, ii].tocsr()
        self.By = self.By_full[:, ii].tocsr()
        # m_i = int phi_i  (P1 basis integrals; sum = |Omega| = 1)
        _, _, _, _, _, I1 = _reference_integrals()
        area = mesh.areas()
        self.m = np.zeros(n1)
        np.add.at(self.m, mesh.tris.ravel(), (area[:, None] * I1[None]).ravel())

    # -- operators at a given beta ------------------------------------------
    def A(self, beta: float) -> sp.csr_matrix:
        """Velocity block A = K + beta M for both components (block diagonal)."""
        A1 = (self.K + beta * self.M).tocsr()
        return sp.block_diag([A1, A1], format="csr")

    def B(self) -> sp.csr_matrix:
        """B = [B_x, B_y] with B_ij = (div psi_j, phi_i)."""
        return sp.hstack([self.Bx, self.By], format="csr")

    def saddle(self, beta: float) -> sp.csr_matrix:
        """The saddle-point matrix [[A, B^T], [B, 0]]."""
        A = self.A(beta)
        B = self.B()
        return sp.bmat([[A, B.T], [B, None]], format="csr")

    def mass_u(self) -> sp.csr_matrix:
        return sp.block_diag([self.M, self.M], format="csr")

    # -- load vectors ---------------------------------------------------------
    def load(self, f_nodal: np.ndarray, g_nodal: np.ndarray):
        """Load vector ((f, psi_j), (g, phi_i)) for P2-interpolated f (values at
        ALL P2 nodes, shape (2, n2)) and P1-interpolated g (shape (n1,))."""
        fu = np.concatenate([self.M_full[self.interior] @ f_nodal[0],
                             self.M_full[self.interior] @ f_nodal[1]])
        gp = self.MP @ g_nodal
        return fu, gp

    @property
    def n(self) -> int:
        return 2 * self.nu + self.n1
