"""CPU-side checks of the C ABI: the library loads, exports every function the
public header declares, and rejects bad arguments before touching a device."""
import ctypes as C
import os
import re

import pytest

from paper_1502_04070_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "stokesmg.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(smg_\w+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libstokesmg.so not built (run `python -m paper_1502_04070_amd.build`)")
    return _lib.load()


def test_header_declares_the_expected_entry_points():
    names = _declared()
    for must in ["smg_setup", "smg_destroy", "smg_apply", "smg_residual", "smg_smooth",
                 "smg_restrict", "smg_prolong_add", "smg_coarse_solve", "smg_project_mean",
                 "smg_cycle", "smg_solve", "smg_solve_mixed", "smg_load", "smg_last_error"]:
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    for name in _declared():
        assert hasattr(lib, name), name
        assert name in _lib.SIGNATURES or name == "smg_last_error", f"{name} has no binding"


def test_default_params(lib):
    p = _lib.SmgParams()
    assert lib.smg_default_params(C.byref(p)) == 0
    assert (p.smoother, p.tau, p.sigma, p.nu_pre, p.nu_post, p.gamma, p.n0, p.unfused) == (0, 0.35, 0.8, 2, 2, 1, 2, 0)
    assert (p.fuse_depth, p.coarse_max_n, p.tile_x, p.domain) == (0, 0, 0, 0)


@pytest.mark.parametrize("N,beta,mod,needle", [
    (6, 1.0, {}, "not n0 * 2^L"),
    (1, 1.0, {}, "below n0"),
    (8, -1.0, {}, "beta"),
    (8, float("nan"), {}, "beta"),
    (8, 1.0, {"gamma": 3}, "gamma"),
    (8, 1.0, {"n0": 1}, "n0"),
    (8, 1.0, {"smoother": 7}, "smoother"),
    (8, 1.0, {"tau": 0.0}, "tau"),
    (8, 1.0, {"nu_pre": -1}, "smoothing steps"),
    (8, 1.0, {"fuse_depth": 3}, "fuse_depth"),
    (8, 1.0, {"tile_x": 12}, "tile_x"),
    (8, 1.0, {"coarse_max_n": -2}, "coarse_max_n"),
    (8, 1.0, {"domain": 5}, "domain"),
    (12, 1.0, {"domain": 1, "n0": 3}, "even n0"),
])
def test_setup_rejects_bad_arguments(lib, N, beta, mod, needle):
    p = _lib.SmgParams()
    lib.smg_default_params(C.byref(p))
    for k, v in mod.items():
        setattr(p, k, v)
    h = C.c_void_p()
    rc = lib.smg_setup(N, beta, C.byref(p), C.byref(h))
    assert rc == -1
    assert needle in lib.smg_last_error().decode()
    assert not h.value


def test_null_handle_is_rejected(lib):
    assert lib.smg_apply(None, 0, None, None, None, None, None) == -1
    assert lib.smg_solve(None, None, None, 1e-8, 10, None, None, None, None, None, None) == -1


def test_every_entry_point_rejects_a_null_handle(lib):
    """Each entry point that takes a hierarchy or a batch returns SMG_EINVAL
    with a message for a null handle (and null vectors), before touching the
    device; destroying NULL is a no-op."""
    import ctypes as C
    skip = {"smg_setup", "smg_batch_setup", "smg_default_params", "smg_tune"}
    for name, args in _lib.SIGNATURES.items():
        if name in skip:
            continue
        vals = [1 if a is C.c_int else 1e-8 if a is C.c_double else None for a in args]
        rc = getattr(lib, name)(*vals)
        if name in ("smg_destroy", "smg_batch_destroy"):
            assert rc == 0, name
        else:
            assert rc == -1, (name, rc)
            assert lib.smg_last_error().decode(), name


@pytest.mark.parametrize("N,beta,domain,needle", [
    (8192, 1.0, 0, "outside 2..4096"),
    (1, 1.0, 0, "outside 2..4096"),
    (7, 1.0, 1, "even N"),
    (7, 1.0, 2, "even N"),
    (8, -1.0, 0, "beta"),
    (8, float("inf"), 0, "beta"),
    (8, 1.0, 4, "domain"),
])
def test_residual_noalloc_rejects_bad_arguments(lib, N, beta, domain, needle):
    """The entry point that allocates nothing checks its sizes before any
    device call (the pointers are never dereferenced on this path)."""
    buf = (C.c_double * 4)()
    ptr = C.cast(buf, C.c_void_p)
    rc = lib.smg_residual_noalloc(N, beta, domain, ptr, ptr, ptr, ptr, ptr, ptr, ptr, None)
    assert rc == -1
    assert needle in lib.smg_last_error().decode()
