"""Canonical intergrid transfers between nested Taylor-Hood spaces.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Paper, Section 3: the spaces are nested, so the prolongation I_{k-1}^k is the
canonical embedding (a coarse P2 / P1 function is re-expressed in the fine
nodal basis, i.e. evaluated at the fine nodes) and the restriction is its
transpose, I_k^{k-1} = (I_{k-1}^k)^T.

The matrices are built by evaluating, for every fine node, the basis of the
coarse triangle that contains it (each fine triangle knows its parent).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .mesh import Mesh


def _barycentric(tri_pts: np.ndarray, q: np.ndarray) -> np.ndarray:
    """Barycentric coordinates of points q (n, 2) in triangles tri_pts (n, 3, 2)."""
    a, b, c = tri_pts[:, 0], tri_pts[:, 1], tri_pts[:, 2]
    v0, v1, v2 = b - a, c - a, q - a
    det = v0[:, 0] * v1[:, 1] - v1[:, 0] * v0[:, 1]
    l1 = (v2[:, 0] * v1[:, 1] - v1[:, 0] * v2[:, 1]) / det
    l2 = (v0[:, 0] * v2[:, 1] - v2[:, 0] * v0[:, 1]) / det
    return np.stack([1.0 - l1 - l2, l1, l2], axis=1)


def _p2_values(lam: np.ndarray) -> np.ndarray:
    """The six local P2 basis functions (v0, v1, v2, m01, m12, m20) at barycentric points."""
    l0, l1, l2 = lam[:, 0], lam[:, 1], lam[:, 2]
    return np.stack([l0 * (2 * l0 - 1), l1 * (2 * l1 - 1), l2 * (2 * l2 - 1),
                     4 * l0 * l1, 4 * l1 * l2, 4 * l2 * l0], axis=1)


def prolongation(coarse: Mesh, fine: Mesh):
    """Full prolongation matrices (all nodes, boundary included):
    P2: (n2_fine, n2_coarse), P1: (nv_fine, nv_coarse)."""
    cd = coarse.p2_tri_dofs()
    fd = fine.p2_tri_dofs()
    fc = fine.p2_coords()
    par = fine.parent
    n2f, n2c = fine.nv + fine.ne, coarse.nv + coarse.ne
    # every fine triangle contributes its 6 nodes, evaluated in the parent
    nodes = fd.ravel()                                          # (6 ntf,)
    ptri = np.repeat(par, 6)
    lam = _barycentric(coarse.pts[coarse.tris[ptri]], fc[nodes])
    vals2 = _p2_values(lam)                                     # (6 ntf, 6)
    # keep one evaluation per fine node (continuity makes them all equal)
    _, first = np.unique(nodes, return_index=True)
    rows = np.repeat(nodes[first], 6)
    cols = cd[ptri[first]].ravel()
    v = vals2[first].ravel()
    keep = np.abs(v) > 1e-15
    P2 = sp.csr_matrix((v[keep], (rows[keep], cols[keep])), shape=(n2f, n2c))
    # P1: fine vertices only (indices < nv_fine), linear interpolation
    vmask = nodes[first] < fine.nv
    vn = nodes[first][vmask]
    lam1 = lam[first][vmask]
    rows1 = np.repeat(vn, 3)
    cols1 = coarse.tris[ptri[first][vmask]].ravel()
    v1 = lam1.ravel()
    keep1 = np.abs(v1) > 1e-15
    P1 = sp.csr_matrix((v1[keep1], (rows1[keep1], cols1[keep1])), shape=(fine.nv, coarse.nv))
    return P2, P1


def saddle_prolongation(coarse_disc, fine_disc) -> sp.csr_matrix:
    """I_{k-1}^k on the unknown vectors [u_x; u_y; p] (interior velocity nodes,
    all pressure nodes)."""
    P2, P1 = prolongation(coarse_disc.mesh, fine_disc.mesh)
    Pu = P2[fine_disc.interior][:, coarse_disc.interior]
    return sp.block_diag([Pu, Pu, P1], format="csr")
