"""Quadrature on triangles and L2 projections onto the Taylor-Hood spaces.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

A collapsed (Duffy) tensor Gauss-Legendre rule with ``n`` points per
direction, optionally applied on every triangle after ``split`` rounds of
red refinement of that triangle.  With n points the rule integrates
polynomials of degree 2n - 2 exactly (the Jacobian of the collapse adds one
degree).  Used to build loads for manufactured solutions (Section 2) and the
L2 projection of the non-smooth solution of the experiments (Section 6).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def reference_rule(n: int, split: int = 0):
    """Barycentric points (q, 3) and weights (q,) on a triangle of unit area."""
    g, w = np.polynomial.legendre.leggauss(n)
    a = 0.5 * (g + 1.0)
    wa = 0.5 * w
    A, Bq = np.meshgrid(a, a, indexing="ij")
    WA, WB = np.meshgrid(wa, wa, indexing="ij")
    s = (A * (1.0 - Bq)).ravel()
    t = Bq.ravel()
    wt = (WA * WB * (1.0 - Bq)).ravel() * 2.0     # reference triangle area 1/2 -> unit area
    lam = np.stack([1.0 - s - t, s, t], axis=1)
    # sub-split the reference triangle (in barycentric coordinates)
    tris = [np.eye(3)]
    for _ in range(split):
        new = []
        for T in tris:
            a_, b_, c_ = T
            mab, mbc, mca = 0.5 * (a_ + b_), 0.5 * (b_ + c_), 0.5 * (c_ + a_)
            new += [np.array([a_, mab, mca]), np.array([mab, b_, mbc]),
                    np.array([mca, mbc, c_]), np.array([mab, mbc, mca])]
        tris = new
    pts = np.vstack([lam @ T for T in tris])
    wts = np.concatenate([wt / len(tris) for _ in tris])
    return pts, wts


def physical_points(mesh, lam):
    """Physical coordinates (nt, q, 2) of barycentric points lam (q, 3)."""
    P = mesh.pts[mesh.tris]                  # (nt, 3, 2)
    return np.einsum("qk,tkd->tqd", lam, P)


def _p2_vals(lam):
    l0, l1, l2 = lam[:, 0], lam[:, 1], lam[:, 2]
    return np.stack([l0 * (2 * l0 - 1), l1 * (2 * l1 - 1), l2 * (2 * l2 - 1),
                     4 * l0 * l1, 4 * l1 * l2, 4 * l2 * l0], axis=1)


def load_p2(mesh, func, n=8, split=0):
    """(func, psi_j) for every P2 node j; func maps (..., 2) points to (...) values."""
    lam, w = reference_rule(n, split)
    X = physical_points(mesh, lam)
    F = func(X)                                       # (nt, q)
    phi = _p2_vals(lam)                               # (q, 6)
    area = mesh.areas()
    loc = np.einsum("tq,q,qi->ti", F, w, phi) * area[:, None]
    out = np.zeros(mesh.nv + mesh.ne)
    np.add.at(out, mesh.p2_tri_dofs().ravel(), loc.ravel())
    return out


def load_p1(mesh, func, n=8, split=0):
    """(func, phi_i) for every P1 node i."""
    lam, w = reference_rule(n, split)
    X = physical_points(mesh, lam)
    F = func(X)
    area = mesh.areas()
    loc = np.einsum("tq,q,qi->ti", F, w, lam) * area[:, None]
    out = np.zeros(mesh.nv)
    np.add.at(out, mesh.tris.ravel(), loc.ravel())
    return out


def l2_errors(disc, uh, ph, u_exact, p_exact, grad_u_exact, n=8):
    """||u - u_h||_L2, |u - u_h|_H1 and ||p - p_h||_L2 (pressure means removed).

    uh: (2, n2) nodal values at all P2 nodes; ph: (n1,) nodal P1 values.
    u_exact(X) -> (..., 2); grad_u_exact(X) -> (..., 2, 2) with [c, d] = d u_c / d x_d.
    """
    mesh = disc.mesh
    lam, w = reference_rule(n)
    X = physical_points(mesh, lam)
    area = mesh.areas()
    d2 = mesh.p2_tri_dofs()
    phi = _p2_vals(lam)                                           # (q,6)
    # gradients of the P2 basis on each triangle
    p = mesh.pts[mesh.tris]
    x, y = p[..., 0], p[..., 1]
    a2 = 2 * area
    gl = np.empty((mesh.nt, 3, 2))
    for k in range(3):
        k1, k2 = (k + 1) % 3, (k + 2) % 3
        gl[:, k, 0] = (y[:, k1] - y[:, k2]) / a2
        gl[:, k, 1] = (x[:, k2] - x[:, k1]) / a2
    l0, l1, l2 = lam[:, 0], lam[:, 1], lam[:, 2]
    L = [l0, l1, l2]
    # d phi_i / d lambda_k at quadrature points: (q, 6, 3)
    dphi = np.zeros((len(w), 6, 3))
    for i in range(3):
        dphi[:, i, i] = 4 * L[i] - 1
    for e, (i, j) in enumerate([(0, 1), (1, 2), (2, 0)]):
        dphi[:, 3 + e, i] = 4 * L[j]
        dphi[:, 3 + e, j] = 4 * L[i]
    gphi = np.einsum("qik,tkd->tqid", dphi, gl)                  # (nt,q,6,2)
    U = u_exact(X)                                                # (nt,q,2)
    GU = grad_u_exact(X)                                          # (nt,q,2,2)
    Pex = p_exact(X)
    eu2 = 0.0
    eh1 = 0.0
    for c in range(2):
        loc = uh[c][d2]                                           # (nt,6)
        uhq = loc @ phi.T                                         # (nt,q)
        guq = np.einsum("ti,tqid->tqd", loc, gphi)
        eu2 += np.sum(area[:, None] * w[None] * (U[..., c] - uhq) ** 2)
        eh1 += np.sum(area[:, None] * w[None] * np.sum((GU[:, :, c, :] - guq) ** 2, axis=-1))
    phq = np.einsum("ti,qi->tq", ph[mesh.tris], lam)
    wq = area[:, None] * w[None]
    vol = np.sum(wq)                       # |Omega| (1 on the unit square, 3/4 on the L-shape)
    mean_ex = np.sum(wq * Pex) / vol
    mean_h = np.sum(wq * phq) / vol
    ep2 = np.sum(wq * ((Pex - mean_ex) - (phq - mean_h)) ** 2)
    return np.sqrt(eu2), np.sqrt(eh1), np.sqrt(ep2)


def l2_project(disc, u_func, p_func, n=8, split=1):
    """L2 projection of (u, p) into X_k = U_k x P_k, as unknown vector
    [u_x interior; u_y interior; p]; the pressure projection is onto P1 with
    mean zero (projection onto P1, then the mean removed: constants are in P1)."""
    mesh = disc.mesh
    ii = disc.interior
    Mi = disc.M_full[ii][:, ii].tocsc()
    lu = spla.splu(Mi)
    ux = lu.solve(load_p2(mesh, lambda X: u_func(X)[..., 0], n, split)[ii])
    uy = lu.solve(load_p2(mesh, lambda X: u_func(X)[..., 1], n, split)[ii])
    ph = spla.spsolve(disc.MP.tocsc(), load_p1(mesh, p_func, n, split))
    ph = ph - (disc.m @ ph) / disc.m.sum()
    return np.concatenate([ux, uy, ph])
