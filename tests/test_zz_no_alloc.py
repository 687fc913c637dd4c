"""The entry point that allocates nothing (smg_residual_noalloc) against the
existing residual entry point (smg_residual on a hierarchy's finest level):
the same kernels on the same tiles, so the residual and its squared norm must
agree to rounding (they are in fact produced by the same summation order).
Two calls in a row on each grid, the second on a smaller grid, so that the
second reads partials the first left behind only if it failed to rewrite
them; then a larger grid with more tiles."""
import pytest
import torch

from paper_1502_04070_amd import Hierarchy
from paper_1502_04070_amd.solver import residual_noalloc

pytestmark = pytest.mark.gpu


def _vectors(N, seed):
    g = torch.Generator(device="cuda").manual_seed(seed)
    M = 2 * N + 1
    dev = dict(device="cuda", dtype=torch.float64, generator=g)
    return (torch.randn((2, M, M), **dev), torch.randn((N + 1, N + 1), **dev),
            torch.randn((2, M, M), **dev), torch.randn((N + 1, N + 1), **dev))


def _check(N, beta, domain, seed):
    print(f"noalloc N={N} beta={beta} domain={domain}", flush=True)
    fu, gp, u, p = _vectors(N, seed)
    ru, rp, n2 = residual_noalloc(N, beta, fu, gp, u, p, domain=domain, norm=True)
    h = Hierarchy(N, beta, domain=domain)
    ru0, rp0, n20 = h.residual(fu, gp, u, p, norm=True)
    torch.cuda.synchronize()
    scale = max(float(ru0.abs().max()), float(rp0.abs().max()))
    assert float((ru - ru0).abs().max()) <= 1e-15 * scale
    assert float((rp - rp0).abs().max()) <= 1e-15 * scale
    assert abs(float(n2) - float(n20)) <= 1e-14 * float(n20)
    return float(n2)


@pytest.mark.parametrize("domain", ["square", "l_shape", "union_jack"])
def test_noalloc_residual_matches_residual_entry_point(domain):
    big = _check(64, 3.0, domain, seed=1)
    small = _check(32, 3.0, domain, seed=2)
    assert small < big           # the second, smaller call saw its own partials only
    _check(512, 1e4, domain, seed=3)


def test_noalloc_residual_largest_grids():
    _check(1024, 1.0, "square", seed=4)
    _check(8, 1.0, "square", seed=5)
