"""Seeded synthetic inputs in the lattice layout (no solver arithmetic here).

Lattice layout of a level with N squares per side (M = 2N + 1):
    nodal velocity data  (2, M, M)   values at ALL P2 lattice points
    nodal pressure data  (N+1, N+1)  values at all P1 vertices
Both the oracle-side tests and the GPU side draw their inputs from here.
"""
from __future__ import annotations

import numpy as np


def lattice_shapes(N: int):
    return (2, 2 * N + 1, 2 * N + 1), (N + 1, N + 1)


def uniform_f(N: int, seed: int = 0):
    """f = P2 nodal values iid uniform[-1, 1] (both components), g = 0."""
    su, sp = lattice_shapes(N)
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, su), np.zeros(sp)


def normal_fg(N: int, seed, with_g: bool = True):
    """f ~ N(0,1) at all P2 lattice points; g ~ N(0,1) at all vertices (raw:
    the consumer removes its mean)."""
    su, sp = lattice_shapes(N)
    rng = np.random.default_rng(seed)
    f = rng.standard_normal(su)
    g = rng.standard_normal(sp) if with_g else np.zeros(sp)
    return f, g


def smooth_plus_noise(N: int, seed: int = 0, noise: float = 1e-3):
    """Both components sin(pi x) sin(pi y) + noise * N(0,1) at the P2 lattice points; g = 0."""
    su, sp = lattice_shapes(N)
    x = np.arange(2 * N + 1) / (2 * N)
    X, Y = np.meshgrid(x, x)          # [b, a]
    base = np.sin(np.pi * X) * np.sin(np.pi * Y)
    rng = np.random.default_rng(seed)
    f = np.stack([base, base]) + noise * rng.standard_normal(su)
    return f, np.zeros(sp)


def random_state(N: int, seed: int):
    """A random iterate (u, p) with zero velocity boundary (for operator tests)."""
    su, sp = lattice_shapes(N)
    rng = np.random.default_rng(seed)
    u = rng.standard_normal(su)
    u[:, 0, :] = u[:, -1, :] = u[:, :, 0] = u[:, :, -1] = 0.0
    return u, rng.standard_normal(sp)


def batched_instances(n_inst: int = 64, n_rhs: int = 4, seed: int = 0):
    """Uneven batch: N_i = 32 * 2^(i mod 4), beta_i = 10^U(-2, 6); RHS j of
    instance i from default_rng([i, j]): f ~ N(0,1), g ~ N(0,1) (raw)."""
    rng = np.random.default_rng(seed)
    betas = 10.0 ** rng.uniform(-2.0, 6.0, n_inst)
    out = []
    for i in range(n_inst):
        N = 32 * 2 ** (i % 4)
        rhs = [normal_fg(N, [i, j]) for j in range(n_rhs)]
        out.append((N, float(betas[i]), rhs))
    return out


def adjoint_instances(n_inst: int = 16, N: int = 256, seed: int = 0):
    """beta_i = 10^U(0, 5); f ~ N(0,1) (seed i); u_target ~ N(0,1) at interior
    nodes (seed 10000 + i), zero on the boundary."""
    rng = np.random.default_rng(seed)
    betas = 10.0 ** rng.uniform(0.0, 5.0, n_inst)
    out = []
    for i in range(n_inst):
        f, _ = normal_fg(N, i, with_g=False)
        ut, _ = random_state(N, 10000 + i)
        out.append((float(betas[i]), f, ut))
    return out


def section6_fields(N: int):
    """The fields of the experiment of Section 6 at the lattice points:
    u = phi (y - 1/2, 1/2 - x), p = phi, phi = max(0, min(1, 2 - 4 |x - (1/2, 1/2)|))
    (nodal values; the paper projects them in L2, which needs quadrature)."""
    su, sp = lattice_shapes(N)
    a = np.arange(2 * N + 1) / (2 * N)
    X, Y = np.meshgrid(a, a)                       # [b, a]
    phi = np.clip(2.0 - 4.0 * np.hypot(X - 0.5, Y - 0.5), 0.0, 1.0)
    u = np.stack([phi * (Y - 0.5), phi * (0.5 - X)])
    u[:, 0, :] = u[:, -1, :] = u[:, :, 0] = u[:, :, -1] = 0.0
    return u, np.ascontiguousarray(phi[::2, ::2])
