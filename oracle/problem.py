"""Model-problem data: the experiment of Section 6 and smooth manufactured solutions.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).
"""
from __future__ import annotations

import numpy as np

from . import multigrid as mg
from .quadrature import l2_project


def phi(X):
    """Section 6: phi = max{0, min{1, 2 - 4 |x - (1/2, 1/2)|}}."""
    r = np.sqrt((X[..., 0] - 0.5) ** 2 + (X[..., 1] - 0.5) ** 2)
    return np.maximum(0.0, np.minimum(1.0, 2.0 - 4.0 * r))


def paper_u(X):
    """Section 6: u = phi (y - 1/2, 1/2 - x)."""
    f = phi(X)
    return np.stack([f * (X[..., 1] - 0.5), f * (0.5 - X[..., 0])], axis=-1)


def paper_p(X):
    return phi(X)


def paper_exact_discrete(h: mg.Hierarchy, n=8, split=2):
    """x* on the finest level: the L2 projection of the exact (u, p) into X_k."""
    return l2_project(h.discs[-1], paper_u, paper_p, n=n, split=split)


def paper_exact_on_level(kind: str, k: int, n=8, split=2):
    """The same x* on level k alone (the finest discretization, no hierarchy):
    (discretization, x*).  The projection does not depend on beta."""
    from . import mesh as meshmod
    from .fem import Discretization
    disc = Discretization(meshmod.hierarchy(kind, k)[-1])
    return disc, l2_project(disc, paper_u, paper_p, n=n, split=split)


def paper_rate(kind: str, k: int, beta: float, prm: mg.Params, eps: float = 1e-9, maxit: int = 200):
    """(n, q) of the protocol of Section 6 on grid level k."""
    h = mg.Hierarchy(kind, k, beta, n0=2)
    xs = paper_exact_discrete(h)
    return mg.error_reduction_run(h, xs, prm, eps=eps, maxit=maxit)
