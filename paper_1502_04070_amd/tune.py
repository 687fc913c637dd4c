"""Launch-schedule and damping autotuning with a JSON cache.

The schedule of the fused kernels (normal-equation steps per launch, the
levels of the single-workgroup coarse kernel, the tile width) changes no
result beyond rounding order, so `smg_tune` in the library picks it by timing
one iterate per candidate on the device.  This module keys the outcome by
device, instance sizes and solver parameters, and stores it in a JSON file
($SMG_TUNE_CACHE, else ~/.cache/paper_1502_04070_amd/schedules.json).
"""
from __future__ import annotations

import ctypes as C
import json
import os

import numpy as np
import torch

from . import _lib, inputs
from .solver import SCHEDULE_FIELDS, Hierarchy, _stream

MAX_CANDIDATES = 32


def cache_path() -> str:
    return os.environ.get("SMG_TUNE_CACHE") or os.path.join(
        os.path.expanduser("~"), ".cache", "paper_1502_04070_amd", "schedules.json")


def _key(Ns, smoother, nu_pre, nu_post, gamma, n0):
    props = torch.cuda.get_device_properties(torch.cuda.current_device())
    arch = getattr(props, "gcnArchName", "") or props.name
    sizes = ",".join(str(int(n)) for n in sorted(Ns))
    return f"{arch}|{props.multi_processor_count}cu|N={sizes}|{smoother}|{nu_pre},{nu_post},{gamma}|n0={n0}"


def _load():
    try:
        with open(cache_path()) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _store(db):
    path = cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(db, fh, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass   # a read-only home: the schedule is still returned


def autotune(Ns, betas, smoother="ne", tau=None, sigma=0.8, nu_pre=2, nu_post=2, gamma=1, n0=2,
             iters=20):
    """Time every candidate schedule for these instances; returns
    {"schedule": {...}, "ms_per_iterate": t, "candidates": [...]}."""
    lib = _lib.load()
    if tau is None:
        tau = 0.35 if smoother == "ne" else 0.8
    base = _lib.SmgParams(_lib.SMOOTHERS[smoother], float(tau), float(sigma), int(nu_pre), int(nu_post),
                          int(gamma), int(n0), 0)
    n = len(Ns)
    Na = (C.c_int * n)(*[int(v) for v in Ns])
    Ba = (C.c_double * n)(*[float(v) for v in betas])
    best = _lib.SmgParams()
    best_ms = C.c_double()
    tried = (_lib.SmgParams * MAX_CANDIDATES)()
    tried_ms = (C.c_double * MAX_CANDIDATES)()
    nt = C.c_int()
    _lib.check(lib.smg_tune(n, Na, Ba, C.byref(base), int(iters), C.byref(best), C.byref(best_ms), tried,
                            tried_ms, MAX_CANDIDATES, C.byref(nt), _stream()), "smg_tune")
    cands = [{**{f: getattr(tried[k], f) for f in SCHEDULE_FIELDS}, "ms_per_iterate": tried_ms[k]}
             for k in range(min(nt.value, MAX_CANDIDATES))]
    return {"schedule": {f: getattr(best, f) for f in SCHEDULE_FIELDS}, "ms_per_iterate": best_ms.value,
            "candidates": cands}


def schedule_for(Ns, betas, smoother="ne", nu_pre=2, nu_post=2, gamma=1, n0=2, retune=False, **kw):
    """The cached schedule for these instances, tuning (and caching) it first
    when it is missing.  Returns (schedule dict, record)."""
    key = _key(Ns, smoother, nu_pre, nu_post, gamma, n0)
    db = _load()
    if retune or key not in db:
        rec = autotune(Ns, betas, smoother=smoother, nu_pre=nu_pre, nu_post=nu_post, gamma=gamma, n0=n0, **kw)
        db[key] = rec
        _store(db)
    rec = db[key]
    return dict(rec["schedule"]), rec


# ---------------------------------------------------------------------------
# damping per level (Section 6 remarks that the rates improve slightly when
# tau and sigma depend on the level and on beta)
# ---------------------------------------------------------------------------

def _rate(h, fu, gp, rtol, maxit):
    _, _, info = h.solve(fu, gp, rtol=rtol, maxit=maxit)
    if info.status != "ok" or info.iters == 0:
        return float("inf"), info.iters
    return float(info.relres) ** (1.0 / info.iters), info.iters


def tune_damping(N, beta, smoother="ne", nu_pre=2, nu_post=2, gamma=1, n0=2, rtol=1e-8, maxit=400,
                 factors=(0.8, 0.9, 1.0, 1.1, 1.2), sweeps=1, seed=0):
    """Coordinate search over the damping of every level above the coarsest
    (finest first): tau for the normal-equation smoother, tau and sigma for
    the Uzawa smoother, each scaled by the given factors around its current
    value.  The objective is the mean residual reduction per iterate of a
    solve from zero with synthetic data (f, g iid N(0, 1), seed).  Returns
    {"tau": [...], "sigma": [...], "rate": q, "iterations": n,
    "rate_default": q0, "iterations_default": n0}, level 0 first."""
    h = Hierarchy(N, beta, smoother=smoother, nu_pre=nu_pre, nu_post=nu_post, gamma=gamma, n0=n0)
    F, G = inputs.normal_fg(N, seed)
    Gd = torch.from_numpy(G).cuda()
    h.project_mean(Gd)
    fu, gp = h.load(torch.from_numpy(F).cuda(), Gd)
    taus = [h.damping(l)[0] for l in range(h.nlevels)]
    sigmas = [h.damping(l)[1] for l in range(h.nlevels)]
    q0, it0 = _rate(h, fu, gp, rtol, maxit)
    best_q, best_it = q0, it0
    for _ in range(sweeps):
        for level in range(h.L, 0, -1):
            t0, s0 = taus[level], sigmas[level]
            pairs = [(t0 * a, s0) for a in factors] if smoother == "ne" else \
                [(t0 * a, s0 * b) for a in factors for b in factors]
            for t, sg in pairs:
                if t == t0 and sg == s0:
                    continue
                h.set_damping(level, t, sg)
                q, it = _rate(h, fu, gp, rtol, maxit)
                if q < best_q:
                    best_q, best_it = q, it
                    taus[level], sigmas[level] = t, sg
            h.set_damping(level, taus[level], sigmas[level])
    return {"tau": taus, "sigma": sigmas, "rate": best_q, "iterations": best_it,
            "rate_default": q0, "iterations_default": it0}


def damping_for(N, beta, smoother="ne", nu_pre=2, nu_post=2, gamma=1, n0=2, retune=False, **kw):
    """The cached damping table for (N, beta, smoother, cycle), tuned first when missing."""
    key = "damping|" + _key([N], smoother, nu_pre, nu_post, gamma, n0) + f"|beta={float(beta)!r}"
    db = _load()
    if retune or key not in db:
        db[key] = tune_damping(N, beta, smoother=smoother, nu_pre=nu_pre, nu_post=nu_post, gamma=gamma,
                               n0=n0, **kw)
        _store(db)
    rec = db[key]
    return {"tau": rec["tau"], "sigma": rec["sigma"]}, rec
