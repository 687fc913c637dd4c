"""Launch-schedule autotuning with a JSON cache.

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

import torch

from . import _lib
from .solver import SCHEDULE_FIELDS, _stream

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
