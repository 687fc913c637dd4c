"""The host-only runtime (paper_1502_04070_amd/csrc/smg_host.cpp) built for the
CPU with the address and undefined-behaviour sanitizers, and checked:

* its self-test (parameter checks, launch offsets and block maps, symmetry of
  the host operator) runs clean under the sanitizers;
* the bordered coarsest-grid matrix it assembles from the lattice stencils
  equals the oracle's bordered matrix (exact integration, generic assembly),
  permuted to the compact order, on all three grids;
* its inverse (equilibrated LU with partial pivoting) solves that system:
  against numpy.linalg.solve of the oracle's matrix (row and column scaled, a
  transformation that leaves the solution unchanged) for n0 = 2, 3, 4 and
  beta = 0, 1, 1e6, 1e10, and by its residual in the unscaled system.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import multigrid as mg
from tests import lattice as lat

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1502_04070_amd", "csrc")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
DOMS = {"same_diag": 0, "l_shape": 1, "union_jack": 2}
SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=1:halt_on_error=1:abort_on_error=0",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


@pytest.fixture(scope="module")
def host_check(tmp_path_factory):
    cxx = shutil.which("g++")
    if cxx is None or not os.path.isdir(os.path.join(ROCM, "include", "hip")):
        pytest.skip("needs g++ and the HIP headers")
    out = str(tmp_path_factory.mktemp("hostcheck") / "host_check")
    # the gen_stencils.py output is committed with the sources it serves
    cmd = [cxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROCM, "include"), "-I", CSRC,
           "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "host_check.cpp"), os.path.join(CSRC, "smg_host.cpp"), "-o", out]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return out


def _run(exe, *args):
    env = dict(os.environ, **SAN_ENV)
    return subprocess.run([exe, *map(str, args)], env=env, capture_output=True, text=True, timeout=120)


def test_selftest_clean_under_sanitizers(host_check):
    r = _run(host_check, "selftest")
    assert r.returncode == 0 and "selftest ok" in r.stdout, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr


def _coarse(exe, tmp_path, n0, beta, dom):
    path = tmp_path / f"c_{n0}_{beta:g}_{dom}.bin"
    r = _run(exe, "coarse", n0, repr(float(beta)), DOMS[dom], path)
    assert r.returncode == 0, r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
    raw = path.read_bytes()
    nc, status = np.frombuffer(raw[:8], dtype=np.int32)
    vals = np.frombuffer(raw[8:], dtype=np.float64)
    a = vals[: nc * nc].reshape(nc, nc)
    inv = vals[nc * nc:].reshape(nc, nc).T          # stored column-major
    return int(status), a, inv


def _compact_index(disc, n0):
    """For every unknown of the oracle's level (its order), the position in the
    compact order of the coarse-solve kernel."""
    ni, NP = 2 * n0 - 1, n0 + 1
    u, p = lat.to_lattice(disc, np.arange(1, disc.nu * 2 + disc.n1 + 1, dtype=float))
    pos = np.full(2 * disc.nu + disc.n1, -1)
    inner = [u[c, 1:2 * n0, 1:2 * n0].ravel() for c in range(2)]
    for c in range(2):
        for q, v in enumerate(inner[c]):
            if v > 0:
                pos[int(v) - 1] = c * ni * ni + q
    for k, v in enumerate(p.ravel()):
        if v > 0:
            pos[int(v) - 1] = 2 * ni * ni + k
    assert (pos >= 0).all() and len(set(pos)) == len(pos)
    nc = 2 * ni * ni + NP * NP + 1
    return pos, nc


@pytest.mark.parametrize("dom,n0", [("same_diag", 2), ("same_diag", 3), ("same_diag", 4),
                                    ("l_shape", 2), ("l_shape", 4), ("union_jack", 2), ("union_jack", 4)])
@pytest.mark.parametrize("beta", [0.0, 1.0, 1e6, 1e10])
def test_bordered_matrix_and_inverse_match_oracle(host_check, tmp_path, dom, n0, beta):
    if dom == "union_jack":
        # the oracle builds the 2 x 2 union jack and refines it (n0 = 4: once)
        h = mg.Hierarchy(dom, int(np.log2(n0 // 2)), beta)
    else:
        h = mg.Hierarchy(dom, 0, beta, n0=n0)
    lv = h.top
    ob = lv.bordered().toarray()                       # oracle order, multiplier last
    pos, nc = _compact_index(h.discs[-1], n0)
    status, a, inv = _coarse(host_check, tmp_path, n0, beta, dom)
    assert status == 0
    assert a.shape == (nc, nc)
    idx = np.concatenate([pos, [nc - 1]])
    # the oracle's matrix, moved to the compact order; removed unknowns
    # (L-shape) are identity rows and columns
    ref = np.zeros((nc, nc))
    ref[np.ix_(idx, idx)] = ob
    removed = np.setdiff1d(np.arange(nc), idx)
    ref[removed, removed] = 1.0
    scale = np.abs(ob).max()
    assert np.abs(a - ref).max() <= 1e-14 * scale
    # the inverse solves the system: a compatible right-hand side (zero
    # multiplier row) against LAPACK on the row/column-scaled oracle matrix
    rng = np.random.default_rng(n0 * 100 + int(np.log10(beta + 1)))
    b = np.zeros(nc)
    b[idx[:-1]] = rng.standard_normal(len(pos))
    s = 1.0 / np.sqrt(np.abs(ref).max(axis=1))
    x_ref = s * np.linalg.solve(ref * s[:, None] * s[None, :], s * b)
    x = inv @ b
    assert np.abs(x - x_ref).max() <= 1e-9 * np.abs(x_ref).max(), np.abs(x - x_ref).max() / np.abs(x_ref).max()
    # backward error in the unscaled system, row by row against the row's size
    r = ref @ x - b
    row = np.abs(ref) @ np.abs(x) + np.abs(b)
    assert (np.abs(r) <= 1e-11 * row).all(), (np.abs(r) / row).max()
