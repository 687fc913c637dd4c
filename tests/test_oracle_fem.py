"""Pins of the oracle's mesh, assembly and transfers against closed forms.

Each check is fixed by the mathematics of the Taylor-Hood discretization
(Section 2) or the nestedness of the refined grids (Sections 2 and 3), not by
re-running the oracle's own formulas.
"""
import numpy as np
import pytest
import sympy as sy

from oracle import fem, mesh, transfer
from oracle.multigrid import Hierarchy

X, Y = sy.symbols("x y")


def _tri_set(m):
    return {tuple(sorted(map(tuple, np.round(m.pts[t], 12)))) for t in m.tris}


@pytest.mark.parametrize("n0", [1, 2, 3])
def test_refined_same_diag_is_same_diag(n0):
    assert _tri_set(mesh.refine(mesh.same_diag(n0))) == _tri_set(mesh.same_diag(2 * n0))


def test_union_jack_every_triangle_has_interior_vertex():
    m = mesh.union_jack()
    assert m.nt == 8
    assert np.isclose(m.areas().sum(), 1.0)
    for lev in [m, mesh.refine(m), mesh.refine(mesh.refine(m))]:
        inner = ~lev.boundary_mask(lev.pts)
        assert inner[lev.tris].any(axis=1).all()


@pytest.mark.parametrize("kind", ["same_diag", "union_jack"])
def test_mass_and_stiffness_invariants(kind):
    m = mesh.hierarchy(kind, 2, 2)[-1]
    d = fem.Discretization(m)
    one2 = np.ones(d.n2)
    one1 = np.ones(d.n1)
    # constants are in the kernel of the Laplacian on the full node set
    assert np.abs(d.K_full @ one2).max() < 1e-12
    # total area
    assert np.isclose(one2 @ d.M_full @ one2, 1.0, atol=1e-14)
    assert np.isclose(one1 @ d.MP @ one1, 1.0, atol=1e-14)
    assert np.isclose(d.m.sum(), 1.0, atol=1e-14)
    # P2 basis integrals: vertex functions integrate to 0, edge functions to |T|/3 per triangle
    ip2 = d.M_full @ one2
    assert np.abs(ip2[: m.nv]).max() < 1e-15
    area = m.areas()
    expect = np.zeros(m.ne)
    np.add.at(expect, m.tri_edges.ravel(), np.repeat(area / 3.0, 3))
    assert np.allclose(ip2[m.nv:], expect, atol=1e-15)
    # symmetry
    for A in (d.K_full, d.M_full, d.MP):
        assert abs(A - A.T).max() < 1e-14


def test_p1_weights_same_diag_closed_form():
    """m_i = int phi_i: h^2 inside, h^2/2 on edges, h^2/3 at (0,0) and (1,1),
    h^2/6 at (1,0) and (0,1) (one triangle of area h^2/2 each third)."""
    N = 8
    d = fem.Discretization(mesh.same_diag(N))
    h = 1.0 / N
    m = d.m.reshape(N + 1, N + 1)   # [j, i]
    assert np.allclose(m[1:-1, 1:-1], h * h)
    assert np.allclose(m[0, 1:-1], h * h / 2) and np.allclose(m[-1, 1:-1], h * h / 2)
    assert np.allclose(m[1:-1, 0], h * h / 2) and np.allclose(m[1:-1, -1], h * h / 2)
    assert np.isclose(m[0, 0], h * h / 3) and np.isclose(m[-1, -1], h * h / 3)
    assert np.isclose(m[0, -1], h * h / 6) and np.isclose(m[-1, 0], h * h / 6)


def _nodal(expr, coords):
    f = sy.lambdify((X, Y), expr, "numpy")
    return np.broadcast_to(np.asarray(f(coords[:, 0], coords[:, 1]), dtype=float), (len(coords),)).copy()


def _square_integral(expr):
    return float(sy.integrate(sy.integrate(expr, (X, 0, 1)), (Y, 0, 1)))


@pytest.mark.parametrize("kind", ["same_diag", "union_jack"])
def test_energy_mass_and_divergence_of_quadratics_are_exact(kind):
    """P2 contains all quadratics and P1 all linears, so the discrete forms
    reproduce the exact integrals over the square."""
    m = mesh.hierarchy(kind, 1, 2)[-1]
    d = fem.Discretization(m)
    rng = np.random.default_rng(5)
    c = rng.uniform(-1, 1, 6)
    u = c[0] + c[1] * X + c[2] * Y + c[3] * X * X + c[4] * X * Y + c[5] * Y * Y
    e = rng.uniform(-1, 1, 3)
    p = e[0] + e[1] * X + e[2] * Y
    un = _nodal(u, d.coords2)
    pn = _nodal(p, d.coords1)
    grad2 = sy.diff(u, X) ** 2 + sy.diff(u, Y) ** 2
    assert np.isclose(un @ d.K_full @ un, _square_integral(grad2), rtol=1e-12)
    assert np.isclose(un @ d.M_full @ un, _square_integral(u * u), rtol=1e-12)
    assert np.isclose(pn @ d.Bx_full @ un, _square_integral(p * sy.diff(u, X)), rtol=1e-12, atol=1e-14)
    assert np.isclose(pn @ d.By_full @ un, _square_integral(p * sy.diff(u, Y)), rtol=1e-12, atol=1e-14)
    assert np.isclose(pn @ d.MP @ pn, _square_integral(p * p), rtol=1e-12)


def test_divergence_of_linear_field_gives_p1_weights():
    """For u = (x, 0): div u = 1, so (B u)_i = int phi_i = m_i."""
    d = fem.Discretization(mesh.same_diag(4))
    ux = d.coords2[:, 0]
    assert np.allclose(d.Bx_full @ ux, d.m, atol=1e-15)


def test_constant_pressure_is_the_kernel_of_BT():
    for kind in ["same_diag", "union_jack"]:
        d = fem.Discretization(mesh.hierarchy(kind, 2, 2)[-1])
        B = d.B()
        assert np.abs(B.T @ np.ones(d.n1)).max() < 1e-15
        # and it is the only one: B^T has a one-dimensional kernel
        s = np.linalg.svd(B.toarray(), compute_uv=False)
        assert s[-1] < 1e-12 and s[-2] > 1e-6


def test_load_of_constant_lives_on_edge_nodes():
    """Vertex rows of the P2 mass have zero row sum, so a constant f loads only edge dofs."""
    d = fem.Discretization(mesh.same_diag(4))
    fu, gp = d.load(np.ones((2, d.n2)), np.ones(d.n1))
    ii = d.interior
    is_vertex = ii < d.mesh.nv
    assert np.abs(fu[: d.nu][is_vertex]).max() < 1e-15
    assert np.all(fu[: d.nu][~is_vertex] > 0)
    assert np.allclose(gp, d.m)


@pytest.mark.parametrize("kind", ["same_diag", "union_jack"])
def test_galerkin_identity(kind):
    """Nested spaces + canonical transfers: P^T A_k P = A_{k-1} exactly
    (the oracle re-discretizes every level, so this pins the transfers)."""
    h = Hierarchy(kind, 3, 7.5, n0=2)
    for k in range(1, 4):
        P = h.levels[k].P
        G = (P.T @ h.levels[k].calA @ P).toarray()
        C = h.levels[k - 1].calA.toarray()
        assert np.abs(G - C).max() < 1e-12 * np.abs(C).max()
        # P1 pressure mass is also preserved
        n1f, n1c = h.levels[k].n1, h.levels[k - 1].n1
        Pp = P[-n1f:, -n1c:]
        assert np.abs((Pp.T @ h.discs[k].MP @ Pp - h.discs[k - 1].MP).toarray()).max() < 1e-15


def test_prolongation_reproduces_quadratics():
    cm, fm = mesh.same_diag(2), mesh.same_diag(4)
    fm = mesh.refine(cm)
    P2, P1 = transfer.prolongation(cm, fm)
    q = 1 + X - 2 * Y + 3 * X * X - X * Y + 0.5 * Y * Y
    assert np.allclose(P2 @ _nodal(q, cm.p2_coords()), _nodal(q, fm.p2_coords()), atol=1e-13)
    lin = 2 - X + 4 * Y
    assert np.allclose(P1 @ _nodal(lin, cm.pts), _nodal(lin, fm.pts), atol=1e-13)
