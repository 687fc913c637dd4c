"""Conversion between the oracle's unknown vectors and the lattice layout of the
HIP library (test helper; holds none of the method's arithmetic).

Lattice layout of a level with N x N squares:
  velocity u[2][2N+1][2N+1]  (component, y index b, x index a), P2 node (a, b)
  at (a/(2N), b/(2N)); boundary entries are zero;
  pressure p[N+1][N+1]       (y index j, x index i), vertex (i/N, j/N).
"""
import numpy as np


def _p2_lattice(disc, N):
    c = disc.coords2
    a = np.rint(c[:, 0] * 2 * N).astype(int)
    b = np.rint(c[:, 1] * 2 * N).astype(int)
    return a, b


def _p1_lattice(disc, N):
    c = disc.coords1
    return np.rint(c[:, 0] * N).astype(int), np.rint(c[:, 1] * N).astype(int)


def level_N(disc):
    """Squares per side: the inverse of the smallest positive vertex coordinate."""
    x = disc.mesh.pts[:, 0]
    return int(round(1.0 / x[x > 1e-14].min()))


def to_lattice(disc, x):
    """Oracle vector [u_x int; u_y int; p] -> (u (2, M, M), p (N+1, N+1))."""
    N = level_N(disc)
    M = 2 * N + 1
    a, b = _p2_lattice(disc, N)
    ii = disc.interior
    u = np.zeros((2, M, M))
    nu = disc.nu
    u[0, b[ii], a[ii]] = x[:nu]
    u[1, b[ii], a[ii]] = x[nu:2 * nu]
    pi, pj = _p1_lattice(disc, N)
    p = np.zeros((N + 1, N + 1))
    p[pj, pi] = x[2 * nu:]
    return u, p


def from_lattice(disc, u, p):
    N = level_N(disc)
    a, b = _p2_lattice(disc, N)
    ii = disc.interior
    pi, pj = _p1_lattice(disc, N)
    return np.concatenate([u[0, b[ii], a[ii]], u[1, b[ii], a[ii]], p[pj, pi]])


def nodal_to_lattice(disc, f_nodal, g_nodal):
    """Nodal values at all P2 nodes (2, n2) and all P1 nodes -> lattice arrays."""
    N = level_N(disc)
    M = 2 * N + 1
    a, b = _p2_lattice(disc, N)
    F = np.zeros((2, M, M))
    F[0, b, a] = f_nodal[0]
    F[1, b, a] = f_nodal[1]
    pi, pj = _p1_lattice(disc, N)
    G = np.zeros((N + 1, N + 1))
    G[pj, pi] = g_nodal
    return F, G


def lattice_to_nodal(disc, F, G):
    N = level_N(disc)
    a, b = _p2_lattice(disc, N)
    pi, pj = _p1_lattice(disc, N)
    return np.stack([F[0, b, a], F[1, b, a]]), G[pj, pi]
