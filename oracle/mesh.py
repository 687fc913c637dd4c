"""Triangulations of the unit square and their uniform refinement.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow FP64 reference
("oracle") that the GPU solver is checked against.  Only tests, the smoke
check and the CPU-baseline leg of the benchmark may import it; the product
path never does.

Paper: Section 6 takes Omega = (0,1)^2 and builds the grid levels k = 1, 2, ...
from a coarsest grid of 8 triangles by uniform refinement (each triangle is
cut into four).  Section 2 uses that the resulting discrete spaces are nested.

Three coarse meshes are provided:
  * ``same_diag(n0)``: n0 x n0 squares, every square cut by the diagonal from
    its lower-left to its upper-right corner.  Refining it once gives
    ``same_diag(2 n0)`` (checked in the tests).
  * ``union_jack()``: the 8-triangle mesh in which every triangle has the
    centre (1/2, 1/2) as a vertex, i.e. a 2 x 2 grid of squares whose
    diagonals all meet in the centre.  This is the reading of the paper's
    (missing) coarse-grid figure that satisfies its requirement that every
    element has a vertex inside the domain (Section 2, Taylor-Hood stability).
  * ``l_shape(n0)``: the same-diagonal grid on the L-shaped domain
    (0,1)^2 minus [1/2,1]^2 (n0 even), a non-convex domain (Section 1: the
    method applies there, the analysis does not).  Refining it gives
    ``l_shape(2 n0)``.
"""
from __future__ import annotations

import numpy as np


class Mesh:
    """A conforming triangulation with counter-clockwise triangles.

    Attributes
    ----------
    pts   : (nv, 2) float64 vertex coordinates
    tris  : (nt, 3) int64 vertex indices, counter-clockwise
    edges : (ne, 2) int64 unique edges, each stored as (low, high)
    tri_edges : (nt, 3) int64 edge index of local edges (v0v1, v1v2, v2v0)
    parent : (nt,) int64 index of the coarse triangle this one was cut from
             (-1 on the coarsest mesh)
    """

    def __init__(self, pts, tris, parent=None):
        self.pts = np.asarray(pts, dtype=np.float64)
        tris = np.asarray(tris, dtype=np.int64)
        # orient every triangle counter-clockwise
        p = self.pts
        d = ((p[tris[:, 1], 0] - p[tris[:, 0], 0]) * (p[tris[:, 2], 1] - p[tris[:, 0], 1])
             - (p[tris[:, 2], 0] - p[tris[:, 0], 0]) * (p[tris[:, 1], 1] - p[tris[:, 0], 1]))
        flip = d < 0
        tris[flip] = tris[flip][:, [0, 2, 1]]
        self.tris = tris
        self.parent = (np.full(len(tris), -1, dtype=np.int64) if parent is None
                       else np.asarray(parent, dtype=np.int64))
        loc = np.stack([tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [2, 0]]], axis=1)  # (nt,3,2)
        flat = np.sort(loc.reshape(-1, 2), axis=1)
        self.edges, inv = np.unique(flat, axis=0, return_inverse=True)
        self.tri_edges = inv.reshape(-1, 3)

    # -- sizes ---------------------------------------------------------------
    @property
    def nv(self) -> int:
        return len(self.pts)

    @property
    def ne(self) -> int:
        return len(self.edges)

    @property
    def nt(self) -> int:
        return len(self.tris)

    # -- P2 / P1 node sets ---------------------------------------------------
    def p2_coords(self) -> np.ndarray:
        """Coordinates of the P2 nodes: all vertices, then all edge midpoints."""
        mid = 0.5 * (self.pts[self.edges[:, 0]] + self.pts[self.edges[:, 1]])
        return np.vstack([self.pts, mid])

    def p2_tri_dofs(self) -> np.ndarray:
        """(nt, 6) P2 node indices per triangle: v0, v1, v2, m01, m12, m20."""
        return np.hstack([self.tris, self.nv + self.tri_edges])

    def boundary_edges(self) -> np.ndarray:
        """True for the edges that belong to exactly one triangle."""
        return np.bincount(self.tri_edges.ravel(), minlength=self.ne) == 1

    def boundary_mask(self, coords: np.ndarray) -> np.ndarray:
        """True for the boundary nodes among the vertices (coords = pts) or the
        P2 nodes (coords = p2_coords()): vertices of boundary edges and
        midpoints of boundary edges."""
        be = self.boundary_edges()
        bv = np.zeros(self.nv, dtype=bool)
        bv[self.edges[be].ravel()] = True
        if len(coords) == self.nv:
            return bv
        if len(coords) == self.nv + self.ne:
            return np.concatenate([bv, be])
        raise ValueError("coords must be the mesh vertices or its P2 nodes")

    def areas(self) -> np.ndarray:
        p, t = self.pts, self.tris
        return 0.5 * ((p[t[:, 1], 0] - p[t[:, 0], 0]) * (p[t[:, 2], 1] - p[t[:, 0], 1])
                      - (p[t[:, 2], 0] - p[t[:, 0], 0]) * (p[t[:, 1], 1] - p[t[:, 0], 1]))


def same_diag(n0: int) -> Mesh:
    """n0 x n0 squares, each cut by its diagonal from (x_i, y_j) to (x_{i+1}, y_{j+1})."""
    if n0 < 1:
        raise ValueError("n0 must be >= 1")
    xs = np.arange(n0 + 1) / n0
    X, Y = np.meshgrid(xs, xs)                  # row j = y index, column i = x index
    pts = np.stack([X.ravel(), Y.ravel()], axis=1)
    vid = lambda i, j: j * (n0 + 1) + i
    tris = []
    for j in range(n0):
        for i in range(n0):
            a, b, c, d = vid(i, j), vid(i + 1, j), vid(i + 1, j + 1), vid(i, j + 1)
            tris.append((a, b, c))
            tris.append((a, c, d))
    return Mesh(pts, tris)


def l_shape(n0: int) -> Mesh:
    """The same-diagonal n0 x n0 grid without the squares in [1/2, 1]^2 (n0 even)."""
    if n0 < 2 or n0 % 2:
        raise ValueError("n0 must be even and >= 2")
    xs = np.arange(n0 + 1) / n0
    vid = lambda i, j: j * (n0 + 1) + i
    tris = []
    for j in range(n0):
        for i in range(n0):
            if 2 * i >= n0 and 2 * j >= n0:
                continue
            a, b, c, d = vid(i, j), vid(i + 1, j), vid(i + 1, j + 1), vid(i, j + 1)
            tris.append((a, b, c))
            tris.append((a, c, d))
    tris = np.array(tris)
    used = np.unique(tris)
    new_id = np.full((n0 + 1) ** 2, -1)
    new_id[used] = np.arange(len(used))
    X, Y = np.meshgrid(xs, xs)
    pts = np.stack([X.ravel(), Y.ravel()], axis=1)[used]
    return Mesh(pts, new_id[tris])


def union_jack() -> Mesh:
    """The 8-triangle coarse grid: 2 x 2 squares whose diagonals meet at (1/2, 1/2)."""
    xs = np.array([0.0, 0.5, 1.0])
    X, Y = np.meshgrid(xs, xs)
    pts = np.stack([X.ravel(), Y.ravel()], axis=1)
    vid = lambda i, j: j * 3 + i
    c = vid(1, 1)
    tris = []
    for (i, j) in [(0, 0), (1, 0), (0, 1), (1, 1)]:
        corners = [vid(i, j), vid(i + 1, j), vid(i + 1, j + 1), vid(i, j + 1)]
        # the corner of this square opposite to the centre
        far = [q for q in corners if q != c and not (q in (vid(1, 0), vid(0, 1), vid(2, 1), vid(1, 2)))][0]
        others = [q for q in corners if q not in (c, far)]
        for q in others:
            tris.append((far, q, c))
    return Mesh(pts, tris)


def refine(mesh: Mesh) -> Mesh:
    """Uniform (red) refinement: every triangle (a, b, c) becomes
    (a, m_ab, m_ca), (m_ab, b, m_bc), (m_ca, m_bc, c), (m_ab, m_bc, m_ca)."""
    nv = mesh.nv
    mid = 0.5 * (mesh.pts[mesh.edges[:, 0]] + mesh.pts[mesh.edges[:, 1]])
    pts = np.vstack([mesh.pts, mid])
    t = mesh.tris
    e = mesh.tri_edges + nv
    a, b, c = t[:, 0], t[:, 1], t[:, 2]
    mab, mbc, mca = e[:, 0], e[:, 1], e[:, 2]
    children = np.stack([
        np.stack([a, mab, mca], 1),
        np.stack([mab, b, mbc], 1),
        np.stack([mca, mbc, c], 1),
        np.stack([mab, mbc, mca], 1),
    ], axis=1).reshape(-1, 3)
    parent = np.repeat(np.arange(mesh.nt), 4)
    return Mesh(pts, children, parent)


def hierarchy(kind: str, levels: int, n0: int = 2) -> list[Mesh]:
    """Meshes of levels 0..levels (coarse to fine) by repeated refinement."""
    if kind == "same_diag":
        meshes = [same_diag(n0)]
    elif kind == "union_jack":
        meshes = [union_jack()]
    elif kind == "l_shape":
        meshes = [l_shape(n0)]
    else:
        raise ValueError(kind)
    for _ in range(levels):
        meshes.append(refine(meshes[-1]))
    return meshes
