#!/usr/bin/env python3
"""Benchmark: coupled multigrid solves of the generalized Stokes system on one MI355X.

Workload (one "step"): the unit square, same-diagonal grid refined to h = 1/128
(66049 P2 nodes per velocity component, 16641 P1 pressure nodes; 146691
unknowns), Taylor-Hood P2-P1, f = P2 nodal values iid uniform[-1, 1] (seed 0),
g = 0, solved to 1e-8 relative residual with the FP64 normal-equation V(2,2)
cycle (7 levels, coarsest h = 1/2) for each beta in {0, 1, 1e2, 1e4, 1e6}.
Inputs are synthetic and resident in HBM before the timed region.

Metric: velocity + pressure unknowns x multigrid cycles per second, summed
over the five solves; time to 1e-8 per beta is reported beside it, for the
FP64 solver and for FP32 cycles inside FP64 iterative refinement.

Prints one JSON line.  `--gpus N` with N > 1 is not supported (one GPU).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

N_GRID = 128
BETAS = [0.0, 1.0, 1e2, 1e4, 1e6]
TOL = 1e-8
HBM_PEAK_GBS = 8000.0

# HBM bytes per launch of the timed normal-equation kernel come from two
# rocprofv3 counter runs (FETCH_SIZE, WRITE_SIZE) summarised in this file,
# together with a hash of the sources the kernel is built from; the figure is
# reported only while those sources are unchanged.
COUNTER_SUMMARY = os.path.join(ROOT, "profiles", "ne_step_h128x5_counters.txt")
COUNTER_SUMMARY_H512 = os.path.join(ROOT, "profiles", "ne_step_h512_counters.txt")
COUNTER_SUMMARY_BATCH = os.path.join(ROOT, "profiles", "ne_step_batch64x4_counters.txt")
NE_KERNEL_SOURCES = ["smg_fused.hip", "smg_fused.h", "smg_cell.h", "smg_stage.h", "smg_internal.h", "gen_stencils.py"]


def dofs(N):
    return 2 * (2 * N - 1) ** 2 + (N + 1) ** 2


# Algorithmic bytes of one normal-equation smoothing step, per FP64 unknown:
# the step as stated (residual, scaled residual, operator, update) streams six
# vectors of the unknowns once each -- read x and F, write y = L^-1 (F - A x),
# read y and x, write x -- so 6 words = 48 B per unknown.  This is the figure
# the roofline fraction is quoted against.
MODEL_NE_STEP_BYTES_PER_DOF = 48


def ne_step_model_bytes(N):
    return MODEL_NE_STEP_BYTES_PER_DOF * dofs(N)


def ne_step_bytes(N):
    """The fused kernel's own minimum HBM bytes for one normal-equation step on
    one instance: read x and F (all unknowns), read Shat^-1 (one per pressure
    node), write the new x; 8-byte words, each once (the intermediate y stays
    on chip)."""
    n, npres = dofs(N), (N + 1) ** 2
    return 8 * (3 * n + npres)


def roofline_block(kernel, Ns, avg_ms, traffic=None):
    """The roofline object of one timed launch over instances of sizes Ns."""
    model = sum(ne_step_model_bytes(N) for N in Ns)
    own = sum(ne_step_bytes(N) for N in Ns)
    achieved = model / (avg_ms * 1e-3) / 1e9
    return {"bound": "hbm", "kernel": kernel, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "bytes_per_launch": model, "bytes_per_dof": MODEL_NE_STEP_BYTES_PER_DOF,
            "unknowns_per_launch": sum(dofs(N) for N in Ns), "avg_launch_us": avg_ms * 1e3,
            "kernel_min_bytes_per_launch": own,
            "kernel_min_GBps": own / (avg_ms * 1e-3) / 1e9,
            "kernel_min_frac": own / (avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS}


def _code_only(text, name):
    """The source without its comments and with whitespace collapsed, so that
    an edit of a comment keeps the hash of the code the counters measured."""
    import re
    if name.endswith(".py"):
        return text
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def ne_kernel_source_hash():
    """SHA-256 over the code (comments removed) of the NE kernel's sources."""
    import hashlib
    hsh = hashlib.sha256()
    for name in NE_KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1502_04070_amd", "csrc", name), encoding="utf-8") as fh:
            hsh.update(_code_only(fh.read(), name).encode())
    return hsh.hexdigest()


def counter_traffic(path=COUNTER_SUMMARY):
    """HBM bytes per launch from a committed counter summary, or None when
    it is missing or was taken from other kernel sources."""
    try:
        with open(path) as fh:
            kv = dict(line.split(":", 1) for line in fh if ":" in line and not line.startswith("#"))
    except OSError:
        return None
    if kv.get("source_sha256", "").strip() != ne_kernel_source_hash():
        return None
    try:
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(n_cycles=120):
    """The oracle (SciPy CSR, FP64) on a bounded sample of the same workload:
    `n_cycles` V(2,2) iterates plus residual norms for each beta at h = 1/128."""
    try:
        from threadpoolctl import threadpool_limits
    except ImportError:  # pragma: no cover
        threadpool_limits = None
    import numpy as np
    from oracle import multigrid as mg
    from paper_1502_04070_amd import inputs
    from tests import lattice as lat

    ctx = threadpool_limits(1) if threadpool_limits else None
    try:
        total_dof_cycles = 0
        t_total = 0.0
        for beta in BETAS:
            h = mg.Hierarchy("same_diag", 6, beta, n0=2)
            d = h.discs[-1]
            F, G = inputs.uniform_f(N_GRID, seed=0)
            fn, gn = lat.lattice_to_nodal(d, F, G)
            f = np.concatenate(d.load(fn, gn))
            x = np.zeros(h.top.n)
            t0 = time.perf_counter()
            for _ in range(n_cycles):
                x = mg.top_cycle(h, x, f, mg.Params())
                np.linalg.norm(mg.residual(h.top, x, f))
            t_total += time.perf_counter() - t0
            total_dof_cycles += dofs(N_GRID) * n_cycles
    finally:
        if ctx is not None:
            ctx.__exit__(None, None, None)
    return {"value": total_dof_cycles / t_total, "unit": "DOF*cycles/s", "cores": 1, "kind": "oracle",
            "sample": f"{n_cycles} NE V(2,2) iterates + residual norm per beta in {BETAS} at h=1/128 "
                      f"({len(BETAS) * n_cycles} cycles, {t_total:.1f} s, 1 thread, setup excluded)"}


def _oracle_rhs(h, F, G):
    import numpy as np
    from tests import lattice as lat
    d = h.discs[-1]
    fn, gn = lat.lattice_to_nodal(d, F, G)
    gn = gn - (h.top.m @ gn) / h.top.m.sum()
    return np.concatenate(d.load(fn, gn))


def _pool_worker(spec, barrier, queue):
    """One instance of a pooled oracle sample: setup, wait for every worker,
    then `cycles` V(2,2) iterates with residual norms, timed (wall clock)."""
    import numpy as np
    from oracle import multigrid as mg
    from paper_1502_04070_amd import inputs
    os.environ["OMP_NUM_THREADS"] = "1"
    kind, N, beta, seed, cycles = spec
    h = mg.Hierarchy("same_diag", int(round(np.log2(N // 2))), beta, n0=2)
    if kind == "normal_fg":
        F, G = inputs.normal_fg(N, seed)
    else:
        F, G = inputs.normal_fg(N, seed, with_g=False)
    f = _oracle_rhs(h, F, G)
    x = np.zeros(h.top.n)
    barrier.wait()
    t0 = time.time()
    for _ in range(cycles):
        x = mg.top_cycle(h, x, f, mg.Params())
        np.linalg.norm(mg.residual(h.top, x, f))
    queue.put((dofs(N) * cycles, t0, time.time()))


def _pooled(specs):
    import multiprocessing as mp
    ctx = mp.get_context("spawn")
    barrier = ctx.Barrier(len(specs))
    queue = ctx.Queue()
    procs = [ctx.Process(target=_pool_worker, args=(sp, barrier, queue)) for sp in specs]
    for pr in procs:
        pr.start()
    res = [queue.get() for _ in procs]
    for pr in procs:
        pr.join()
    work = sum(r[0] for r in res)
    wall = max(r[2] for r in res) - min(r[1] for r in res)
    return {"dof_cycles_per_s": work / wall, "processes": len(specs), "wall_s": wall}


def cpu_extras():
    """The oracle (SciPy CSR, FP64) timed on the host for the other workloads:
    one thread for the two-grid case, the h = 1/128 betas and h = 1/512 (to
    tolerance), and a process pool (one process per sampled instance, at most
    16) for the uneven batch and the adjoint instances (10 iterates each)."""
    from threadpoolctl import threadpool_limits
    import numpy as np
    from oracle import multigrid as mg
    from paper_1502_04070_amd import inputs

    out = {"host_cores": os.cpu_count()}
    try:
        out["host_cpu"] = next(l.split(":", 1)[1].strip() for l in open("/proc/cpuinfo") if l.startswith("model name"))
    except (OSError, StopIteration):
        out["host_cpu"] = None

    def solve_timed(h, f, tol):
        t0 = time.perf_counter()
        res = mg.solve(h, f, mg.Params(), tol=tol, maxit=500)
        dt = time.perf_counter() - t0
        return {"iterations": res.iters, "time_to_tol_s": dt, "s_per_cycle": dt / max(res.iters, 1),
                "status": res.status}

    with threadpool_limits(1):
        h = mg.Hierarchy("same_diag", 1, 1.0, n0=4)
        out["two_grid_h8"] = solve_timed(h, _oracle_rhs(h, *inputs.uniform_f(8, seed=0)), 1e-8)
        rec = {}
        for beta in BETAS:
            h = mg.Hierarchy("same_diag", 6, beta, n0=2)
            rec[str(beta)] = solve_timed(h, _oracle_rhs(h, *inputs.uniform_f(N_GRID, seed=0)), TOL)
        out["h128_betas"] = rec
        rec = {}
        for beta in (1.0, 1e4):
            h = mg.Hierarchy("same_diag", 8, beta, n0=2)
            rec[str(beta)] = solve_timed(h, _oracle_rhs(h, *inputs.smooth_plus_noise(512, seed=0)), 1e-10)
        out["h512_fp64_to_1e-10"] = rec
    nproc = max(1, min(16, os.cpu_count() or 1))
    insts = inputs.batched_instances()
    specs = [("normal_fg", N, beta, [i, 0], 10) for i, (N, beta, _) in enumerate(insts[:nproc])]
    out["batch_64x4_sample"] = dict(_pooled(specs), sample=f"instances 0..{nproc - 1} (rhs 0), 10 iterates each")
    ad = inputs.adjoint_instances()
    specs = [("forward", 256, beta, i, 10) for i, (beta, _, _) in enumerate(ad[:nproc])]
    out["adjoint_16x_h256_forward_sample"] = dict(_pooled(specs),
                                                  sample=f"instances 0..{nproc - 1}, forward iterates, 10 each")
    return out


def trace_gaps(path):
    """Per-iterate figures of the last solve in a kernel trace of
    --probe-iterate: each iterate ends with the projection/check kernel;
    `busy` is the summed duration of the iterate's kernels, `span` the time
    from the end of the previous iterate to the end of this one, and the
    difference the time the GPU spends between the kernels of the graph."""
    import csv
    rows = sorted(csv.DictReader(open(path)), key=lambda r: int(r["Start_Timestamp"]))
    ends = [k for k, r in enumerate(rows) if "k_pc_b" in r["Kernel_Name"]]
    last = ends[-20:]
    per = []
    for a, b in zip(last[:-1], last[1:]):
        ks = rows[a + 1:b + 1]
        busy = sum(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in ks)
        span = int(rows[b]["End_Timestamp"]) - int(rows[a]["End_Timestamp"])
        per.append((len(ks), busy, span))
    per.sort(key=lambda t: t[2])
    n, busy, span = per[len(per) // 2]
    return {"iterates_used": len(per), "kernels_per_iterate": n, "median_span_us": span / 1e3,
            "busy_us_of_that_iterate": busy / 1e3, "between_kernels_us": (span - busy) / 1e3,
            "between_kernels_per_launch_us": (span - busy) / 1e3 / n}


def copy_calibration(mib=512, reps=5):
    """A plain device-to-device copy of `mib` MiB, `reps` times: the reference
    kernel against which the HBM byte counters are scaled (it reads and writes
    exactly `mib` MiB per launch)."""
    import torch
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration": {"bytes_read_per_launch": n * 8, "bytes_written_per_launch": n * 8,
                                           "launches": reps}}), flush=True)


# HBM model of one FP64 V(2,2) iterate of the method as stated, per unknown of
# the finest level: every stage reads each input vector once and writes each
# output once (normal-equation step 6 words, defect + restriction and
# prolongation + add 2.25 words each, so 28.5 words per level), summed over the
# levels (factor 4/3): 304 bytes.  The fused kernels move less than this, so
# the fraction below can exceed what the kernels' own traffic would give.
MODEL_BYTES_PER_DOF_V22 = 8 * 28.5 * 4 / 3


def _timed(fn):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = fn()
    torch.cuda.synchronize()
    return out, time.perf_counter() - t0


EXTRA_SECTIONS = ("batch64x4", "shares8", "mixed512", "adjoint", "implicit", "damping", "lshape",
                  "smoothers", "protocol")


def extras(sections=EXTRA_SECTIONS):
    """The other workloads, each timed once after a warm-up run on resident
    inputs; `sections` selects some of them (names in EXTRA_SECTIONS)."""
    import numpy as np
    import torch
    from paper_1502_04070_amd import Batch, Hierarchy, inputs
    from paper_1502_04070_amd import autograd as ag
    from paper_1502_04070_amd import tune

    out = {}
    # 64 instances x 4 right-hand sides, h = 1/32 ... 1/256, one batch
    insts = inputs.batched_instances()
    Ns, betas, fg = [], [], []
    for N, beta, rhs in insts:
        for F, G in rhs:
            Ns.append(N)
            betas.append(beta)
            fg.append((F, G))
    if "batch64x4" in sections or "shares8" in sections:
        sched, _ = tune.schedule_for(Ns, betas, iters=5)
    if "batch64x4" in sections:
        out.update(_batch64x4(Ns, betas, fg, sched))
    if "shares8" in sections:
        out.update(_shares8(Ns, betas, fg, sched, out))
    for name in ("mixed512", "adjoint", "implicit", "damping", "lshape", "smoothers", "protocol"):
        if name in sections:
            out.update(globals()["_x_" + name]())
            torch.cuda.empty_cache()
    return out


def _batch64x4(Ns, betas, fg, sched):
    import numpy as np
    import torch
    from paper_1502_04070_amd import Batch
    out = {}
    B = Batch(Ns, betas, schedule=sched)
    fus, gps = [], []
    for h, (F, G) in zip(B.instances, fg):
        Gd = torch.from_numpy(G).cuda()
        h.project_mean(Gd)
        fu, gp = h.load(torch.from_numpy(F).cuda(), Gd)
        fus.append(fu)
        gps.append(gp)
    outs = [h.zeros() for h in B.instances]
    us = [u for u, _ in outs]
    ps = [p for _, p in outs]
    dof = np.array([dofs(n) for n in Ns], dtype=np.float64)
    rec = {"solves": len(Ns), "unknowns": int(dof.sum()), "tol": 1e-8, "schedule": sched}
    for name, fn in (("fp64", B.solve), ("fp32_refine", B.solve_mixed)):
        def run():
            for u, p in zip(us, ps):
                u.zero_()
                p.zero_()
            return fn(fus, gps, rtol=1e-8, maxit=400, us=us, ps=ps)[2]
        run()
        infos, dt = _timed(run)
        assert all(i.status == "ok" for i in infos), [i for i in infos if i.status != "ok"][:3]
        its = np.array([i.iters for i in infos], dtype=np.float64)
        r = {"time_to_tol_ms": 1e3 * dt, "iterations_max": int(its.max()), "iterations_mean": float(its.mean()),
             "dof_cycles_per_s": float((dof * its).sum() / dt)}
        if name == "fp64":
            gbs = MODEL_BYTES_PER_DOF_V22 * float((dof * its).sum()) / dt / 1e9
            r["per_cycle_model_GBps"] = gbs
            r["per_cycle_model_frac"] = gbs / HBM_PEAK_GBS
        rec[name] = r
    # the dominant kernel of this workload: the batched finest-level
    # normal-equation step of all 256 instances, timed with HIP events
    rec["roofline"] = roofline_block("finest-level fused normal-equation step, all 256 instances (k_ne_b)",
                                     Ns, B.time_kernel(0, reps=50), counter_traffic(COUNTER_SUMMARY_BATCH))
    out["batch_64x4_h32_to_h256"] = rec
    del B, fus, gps, us, ps
    torch.cuda.empty_cache()
    return out


def _shares8(Ns, betas, fg, sched, prev):
    import torch
    from paper_1502_04070_amd import Batch
    out = {}

    # The same 256 solves as the shares of an 8-GPU run: independent instances
    # need no communication, so each GPU gets a batch of its own, placed
    # longest first by unknowns; every share is timed here as its own batch
    # (the slowest share is the run's time, without gathering the results).
    n_gpu = 8
    order = sorted(range(len(Ns)), key=lambda k: (-dofs(Ns[k]), k))
    load, shares = [0] * n_gpu, [[] for _ in range(n_gpu)]
    for k in order:
        g = min(range(n_gpu), key=lambda q: (load[q], q))
        shares[g].append(k)
        load[g] += dofs(Ns[k])
    share_ms, share_its = [], []
    for sh in shares:
        Bs = Batch([Ns[k] for k in sh], [betas[k] for k in sh], schedule=sched)
        fus, gps = [], []
        for h, k in zip(Bs.instances, sh):
            F, G = fg[k]
            Gd = torch.from_numpy(G).cuda()
            h.project_mean(Gd)
            fu, gp = h.load(torch.from_numpy(F).cuda(), Gd)
            fus.append(fu)
            gps.append(gp)
        outs = [h.zeros() for h in Bs.instances]

        def run_share():
            for u, p in outs:
                u.zero_()
                p.zero_()
            return Bs.solve(fus, gps, rtol=1e-8, maxit=400, us=[u for u, _ in outs], ps=[p for _, p in outs])[2]
        run_share()
        infos, dt = _timed(run_share)
        assert all(i.status == "ok" for i in infos)
        share_ms.append(1e3 * dt)
        share_its.append(int(sum(i.iters for i in infos)))
        del Bs, fus, gps, outs
    torch.cuda.empty_cache()
    out["batch_64x4_shares_of_8_gpus"] = {
        "rule": "longest first by unknowns", "solves_per_share": [len(sh) for sh in shares],
        "unknowns_per_share": [int(v) for v in load], "iterates_per_share": share_its,
        "fp64_time_to_tol_ms_per_share": share_ms, "slowest_share_ms": max(share_ms),
        "one_gpu_whole_batch_ms": prev.get("batch_64x4_h32_to_h256", {}).get("fp64", {}).get("time_to_tol_ms")}
    return out


def _x_mixed512():
    """h = 1/512, FP64 against FP32 cycles in FP64 refinement, to 1e-10."""
    import torch
    from paper_1502_04070_amd import Hierarchy, inputs, tune
    out = {}
    N = 512
    F, G = inputs.smooth_plus_noise(N, seed=0)
    sched, _ = tune.schedule_for([N], [1.0], iters=10)
    rec = {"unknowns": dofs(N), "tol": 1e-10, "schedule": sched}
    for beta in (1.0, 1e4):
        h = Hierarchy(N, beta, schedule=sched)
        fu, gp = h.load(torch.from_numpy(F).cuda(), torch.from_numpy(G).cuda())
        r = {}
        sols = {}
        for name, fn in (("fp64", h.solve), ("fp32_refine", h.solve_mixed)):
            fn(fu, gp, rtol=1e-10, maxit=400)
            (u, p, info), dt = _timed(lambda: fn(fu, gp, rtol=1e-10, maxit=400))
            assert info.status == "ok", info
            r[name] = {"time_to_tol_ms": 1e3 * dt, "iterations": info.iters, "relres": info.relres}
            sols[name] = (u, p)
        (u64, p64), (u32, p32) = sols["fp64"], sols["fp32_refine"]
        # both pressures are projected to the same (weighted) zero mean
        num = torch.sqrt(((u32 - u64) ** 2).sum() + ((p32 - p64) ** 2).sum())
        den = torch.sqrt((u64 ** 2).sum() + (p64 ** 2).sum())
        r["rel_diff_fp32_refine_vs_fp64"] = float(num / den)
        rec[f"beta={beta:g}"] = r
        if beta == 1.0:
            # the dominant kernel of the FP64 solve: the finest-level fused
            # normal-equation step, timed with HIP events
            from paper_1502_04070_amd import Batch
            B1 = Batch([N], [beta], schedule=sched)
            rec["roofline"] = roofline_block("finest-level fused normal-equation step, h=1/512 (k_ne_b)",
                                             [N], B1.time_kernel(0, reps=100), counter_traffic(COUNTER_SUMMARY_H512))
            del B1
        del h
    out["mixed_h512"] = rec
    return out


def _x_adjoint():
    """16 instances at h = 1/256: forward solve against forward + adjoint gradients."""
    import torch
    from paper_1502_04070_amd import inputs
    from paper_1502_04070_amd import autograd as ag
    out = {}
    N = 256
    ai = inputs.adjoint_instances()
    nb = len(ai)
    fb = torch.stack([torch.from_numpy(Fa).cuda() for _, Fa, _ in ai])
    ut = torch.stack([torch.from_numpy(Ua).cuda() for _, _, Ua in ai])
    bt = torch.tensor([b for b, _, _ in ai], dtype=torch.float64, device="cuda")
    gz = torch.zeros((nb, N + 1, N + 1), dtype=torch.float64, device="cuda")

    def forward_only():
        with torch.no_grad():
            return ag.batch_stokes_solve(fb, gz, bt, rtol=1e-10, maxit=500)

    def forward_backward(mixed=False):
        f = fb.clone().requires_grad_(True)
        b = bt.clone().requires_grad_(True)
        u, _ = ag.batch_stokes_solve(f, gz, b, rtol=1e-10, maxit=500, mixed=mixed)
        e = u - ut
        loss = 0.5 * sum((e[k] * ag.mass_product(e[k], N)).sum() for k in range(nb))
        loss.backward()
        return f.grad, b.grad

    forward_only()
    forward_backward()
    forward_backward(True)
    _, t_fwd = _timed(forward_only)
    (gf64, gb64), t_all = _timed(forward_backward)
    (gf32, gb32), t_mix = _timed(lambda: forward_backward(True))
    out["adjoint_16x_h256"] = {"instances": nb, "unknowns_each": dofs(N), "tol": 1e-10,
                               "forward_ms": 1e3 * t_fwd, "forward_and_gradients_ms": 1e3 * t_all,
                               "ratio": t_all / t_fwd,
                               "fp32_refine_forward_and_gradients_ms": 1e3 * t_mix,
                               "fp32_refine_rel_diff_df": float((gf32 - gf64).abs().max() / gf64.abs().max()),
                               "fp32_refine_rel_diff_dbeta": float(((gb32 - gb64).abs() / gb64.abs()).max())}
    return out


def _x_implicit():
    """Implicit Euler: four time steps dt marching together at h = 1/256, f = sin(pi x) sin(pi y)."""
    import torch
    from paper_1502_04070_amd import inputs
    from paper_1502_04070_amd.timestep import BatchImplicitEuler
    out = {}
    N = 256
    dts = [1e-1, 1e-2, 1e-3, 1e-4]
    Fs, _ = inputs.smooth_plus_noise(N, seed=0, noise=0.0)
    Fd = torch.from_numpy(Fs).cuda()
    nsteps = 10
    rec, finals = {"dts": dts, "steps": nsteps, "tol": 1e-10}, {}
    for mixed in (False, True):
        te = BatchImplicitEuler([N] * len(dts), dts, mixed=mixed)
        te.step([Fd] * len(dts))
        infos, t_steps = _timed(lambda: [te.step([Fd] * len(dts)) for _ in range(nsteps)])
        key = "fp32_refine_" if mixed else ""
        rec[key + "ms_per_step"] = 1e3 * t_steps / nsteps
        rec[key + "iterations_last_step"] = [i.iters for i in infos[-1]]
        finals[mixed] = [u.clone() for u in te.us]
        del te
    # the same eleven steps in both precisions: largest velocity difference, relative to the FP64 state
    rec["fp32_refine_rel_diff_u"] = max(float((a - b).abs().max() / b.abs().max())
                                        for a, b in zip(finals[True], finals[False]))
    out["implicit_euler_4dt_h256"] = rec
    return out


def _x_damping():
    """Damping per level, searched for each beta of the main workload (h = 1/128)."""
    import torch
    from paper_1502_04070_amd import Hierarchy, inputs
    from paper_1502_04070_amd import tune as _tune
    out = {}
    rec = {}
    F128, G128 = inputs.uniform_f(N_GRID, seed=0)
    for beta in BETAS:
        damp, info = _tune.damping_for(N_GRID, beta, factors=(0.8, 0.9, 1.0, 1.1, 1.2))
        h0 = Hierarchy(N_GRID, beta)
        h1 = Hierarchy(N_GRID, beta, damping=damp)
        fu, gp = h0.load(torch.from_numpy(F128).cuda(), torch.from_numpy(G128).cuda())
        r = {"tau": [round(t, 4) for t in damp["tau"]]}
        for name, hh in (("default", h0), ("tuned", h1)):
            hh.solve(fu, gp, rtol=TOL, maxit=500)
            (_, _, inf), dt_s = _timed(lambda: hh.solve(fu, gp, rtol=TOL, maxit=500))
            r[name] = {"iterations": inf.iters, "time_to_tol_ms": 1e3 * dt_s}
        rec[str(beta)] = r
    out["level_damping_h128"] = rec
    return out


def _x_lshape():
    """The L-shaped domain at h = 1/256 (three quarters of the square's
    unknowns), f iid U[-1, 1], g = 0, NE V(2,2) to 1e-8, next to the unit square."""
    import torch
    from paper_1502_04070_amd import Hierarchy, inputs
    out = {}
    N = 256
    F, G = inputs.uniform_f(N, seed=0)
    rec = {"tol": TOL}
    for beta in (1.0, 1e4):
        r = {}
        for dom in ("l_shape", "square"):
            hh = Hierarchy(N, beta, domain=dom)
            fu, gp = hh.load(torch.from_numpy(F).cuda(), torch.from_numpy(G).cuda())
            hh.solve(fu, gp, rtol=TOL, maxit=500)
            (_, _, inf), t_s = _timed(lambda: hh.solve(fu, gp, rtol=TOL, maxit=500))
            assert inf.status == "ok", inf
            r[dom] = {"iterations": inf.iters, "time_to_tol_ms": 1e3 * t_s}
            del hh
        rec[f"beta={beta:g}"] = r
    out["l_shape_h256"] = rec
    return out


def _x_smoothers():
    """h = 1/128, the five betas: iterates to 1e-8 of NE and Uzawa V(3,3) and W(3,3)."""
    import torch
    from paper_1502_04070_amd import Hierarchy, inputs
    out = {}
    F128, G128 = inputs.uniform_f(N_GRID, seed=0)
    rec = {"tol": TOL}
    for name, kw in (("ne_V33", dict(smoother="ne", nu_pre=3, nu_post=3)),
                     ("uzawa_V33", dict(smoother="uzawa", nu_pre=3, nu_post=3)),
                     ("ne_W33", dict(smoother="ne", nu_pre=3, nu_post=3, gamma=2)),
                     ("uzawa_W33", dict(smoother="uzawa", nu_pre=3, nu_post=3, gamma=2))):
        r = {}
        for beta in BETAS:
            hh = Hierarchy(N_GRID, beta, **kw)
            fu, gp = hh.load(torch.from_numpy(F128).cuda(), torch.from_numpy(G128).cuda())
            hh.solve(fu, gp, rtol=TOL, maxit=500)
            (_, _, inf), t_s = _timed(lambda: hh.solve(fu, gp, rtol=TOL, maxit=500))
            r[str(beta)] = {"iterations": inf.iters if inf.status == "ok" else None,
                            "status": inf.status, "time_to_tol_ms": 1e3 * t_s}
            del hh
        rec[name] = r
    out["h128_smoothers_cycles"] = rec
    return out


def _x_protocol():
    """The measurement protocol of Section 6 on the union-jack grid."""
    import torch
    from paper_1502_04070_amd import Hierarchy, inputs
    out = {}
    # the measurement protocol of Section 6 on the union-jack grid (Tables 2
    # and 3): NE and Uzawa W(3,3), levels k = 4..8 (h = 1/32 .. 1/512), six
    # beta, x* = nodal values of the Section 6 fields (the paper projects
    # them in L2), f = calA x*, stop when the L-norm error dropped by 1e-9
    betas6 = [0.0, 1e2, 1e4, 1e6, 1e8, 1e10]
    rec = {"x_star": "nodal interpolant of u = phi (y - 1/2, 1/2 - x), p = phi (a variant of the paper's "
                     "setup, which projects the fields in L2; the GPU tests run level 7 with the L2 projection)",
           "eps": 1e-9,
           "cycle": "W(3,3)", "betas": betas6}
    for k in range(4, 9):
        N = 2 ** (k + 1)
        us, ps = inputs.section6_fields(N)
        Us, Ps = torch.from_numpy(us).cuda(), torch.from_numpy(ps).cuda()
        lev = {}
        for name, sm in (("ne", "ne"), ("uzawa", "uzawa")):
            runs, t_all = [], 0.0
            for beta in betas6:
                hh = Hierarchy(N, beta, smoother=sm, nu_pre=3, nu_post=3, gamma=2, domain="union_jack")
                FU, GP = hh.apply(Us, Ps)
                (_, _, n, q, st), t_s = _timed(lambda: hh.solve_error(FU, GP, Us, Ps, eps=1e-9, maxit=200))
                runs.append([n if st == "ok" else None, round(q, 3)])
                t_all += t_s
                del hh
            lev[name] = {"iterations_rate": runs, "ms_per_iterate": 1e3 * t_all / max(1, sum(r[0] or 0 for r in runs))}
        rec[f"k={k}"] = lev
    out["paper_protocol_union_jack_nodal_xstar"] = rec
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel-reps", type=int, default=200)
    ap.add_argument("--no-extras", action="store_true", help="skip the batched / h=1/512 / adjoint workloads")
    ap.add_argument("--extras-only", nargs="?", const=",".join(EXTRA_SECTIONS), default=None,
                    metavar="SECTIONS",
                    help="only the other workloads (comma list of: " + ", ".join(EXTRA_SECTIONS) + ")")
    ap.add_argument("--probe", type=int, default=0, metavar="N",
                    help="only time the batched fused normal-equation step at h=1/N (no graphs)")
    ap.add_argument("--probe-count", type=int, default=1,
                    help="instances of the probe batch (5: the betas of the main workload)")
    ap.add_argument("--probe-batch64x4", action="store_true",
                    help="only time the finest-level normal-equation step of the 64 x 4 batch (no graphs)")
    ap.add_argument("--probe-iterate", choices=["h128x5", "batch64x4"], default=None,
                    help="only run 20 batched iterates with every instance active (tolerance 0), for a kernel trace")
    ap.add_argument("--trace-gaps", metavar="CSV", default=None,
                    help="only summarise a rocprofv3 kernel trace of --probe-iterate: per-iterate kernel time and span")
    ap.add_argument("--probe-cycle", type=int, default=0, metavar="N",
                    help="only run single-instance V(2,2) iterates at h=1/N, launched directly (no graphs)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run the plain copy used to scale the HBM byte counters")
    ap.add_argument("--cpu-extras", action="store_true",
                    help="only time the oracle on the host for the other workloads (no GPU)")
    args = ap.parse_args()
    if args.cpu_extras:
        print(json.dumps({"cpu_extras": cpu_extras()}), flush=True)
        return
    if args.trace_gaps:
        print(json.dumps({"trace_gaps": trace_gaps(args.trace_gaps)}), flush=True)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the solver has no multi-GPU path "
              "(independent instances would be spread over GPUs, a single large one split into strips "
              "with halo exchanges)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1502_04070_amd import Batch, Hierarchy, inputs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.probe_iterate:
        from paper_1502_04070_amd import tune
        if args.probe_iterate == "h128x5":
            Ns, betas = [N_GRID] * len(BETAS), BETAS
            fg = [inputs.uniform_f(N_GRID, seed=0)] * len(BETAS)
        else:
            insts = inputs.batched_instances()
            Ns = [N for N, _, rhs in insts for _ in rhs]
            betas = [b for _, b, rhs in insts for _ in rhs]
            fg = [(F, G) for _, _, rhs in insts for F, G in rhs]
        sched, _ = tune.schedule_for(Ns, betas, iters=5)
        B = Batch(Ns, betas, schedule=sched)
        fus, gps = [], []
        for h, (F, G) in zip(B.instances, fg):
            Gd = torch.from_numpy(G).cuda()
            h.project_mean(Gd)
            fu, gp = h.load(torch.from_numpy(F).cuda(), Gd)
            fus.append(fu)
            gps.append(gp)
        # rtol = 0: every instance stays active, and the iterates run in
        # long chunks between host checks; the marginal time of 20 more
        # iterates excludes the solve's set-up
        wall = {}
        for its in (20, 40, 20):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            B.solve(fus, gps, rtol=0.0, maxit=its)
            torch.cuda.synchronize()
            wall[its] = time.perf_counter() - t0
        print(json.dumps({"probe_iterate": {"workload": args.probe_iterate, "schedule": sched,
                                            "ms_per_iterate": 1e3 * (wall[40] - wall[20]) / 20,
                                            "ms_solve_20": 1e3 * wall[20]}}), flush=True)
        return
    if args.probe_cycle:
        N = args.probe_cycle
        h = Hierarchy(N, 1.0)
        F, G = inputs.uniform_f(N, seed=0)
        fu, gp = h.load(torch.from_numpy(F).cuda(), torch.from_numpy(G).cuda())
        u, p = h.zeros()
        h.cycle(fu, gp, u, p)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.kernel_reps):
            h.cycle(fu, gp, u, p)
        torch.cuda.synchronize()
        print(json.dumps({"probe_cycle": {"N": N, "iterates": args.kernel_reps,
                                          "ms_per_iterate": 1e3 * (time.perf_counter() - t0) / args.kernel_reps}}),
              flush=True)
        return
    if args.probe or args.probe_batch64x4:
        if args.probe_batch64x4:
            Ns = [N for N, _, rhs in inputs.batched_instances() for _ in rhs]
            betas = [b for _, b, rhs in inputs.batched_instances() for _ in rhs]
            name = "64 x 4 batch"
        else:
            Ns = [args.probe] * args.probe_count
            betas = BETAS if args.probe_count == len(BETAS) else [1.0] * args.probe_count
            name = f"h=1/{args.probe} x {args.probe_count}"
        B = Batch(Ns, betas)
        ms = B.time_kernel(0, reps=args.kernel_reps)
        print(json.dumps({"probe": dict(roofline_block("fused normal-equation step (default tile), " + name,
                                                       Ns, ms), reps=args.kernel_reps)}), flush=True)
        return
    if args.extras_only is not None:
        secs = [x for x in args.extras_only.split(",") if x]
        bad = [x for x in secs if x not in EXTRA_SECTIONS]
        if bad:
            ap.error(f"unknown sections {bad}")
        print(json.dumps({"extras": extras(secs)}), flush=True)
        return
    F, G = inputs.uniform_f(N_GRID, seed=0)
    Fd = torch.from_numpy(F).cuda()
    Gd = torch.from_numpy(G).cuda()
    # launch schedules picked by the autotuner (setup, outside the timed region)
    from paper_1502_04070_amd import tune
    t_tune = time.perf_counter()
    sched_batch, rec_batch = tune.schedule_for([N_GRID] * len(BETAS), BETAS, iters=10)
    sched_single, rec_single = tune.schedule_for([N_GRID], [1.0], iters=10)
    t_tune = time.perf_counter() - t_tune
    torch.cuda.synchronize()
    t_setup = time.perf_counter()
    batch = Batch([N_GRID] * len(BETAS), BETAS, schedule=sched_batch)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t_setup
    loads = [h.load(Fd, Gd) for h in batch.instances]       # resident load vectors
    fus = [a for a, _ in loads]
    gps = [b for _, b in loads]
    outs = [h.zeros() for h in batch.instances]
    us = [u for u, _ in outs]
    ps = [p for _, p in outs]
    torch.cuda.synchronize()

    def step(mixed=False):
        for u, p in zip(us, ps):
            u.zero_()
            p.zero_()
        fn = batch.solve_mixed if mixed else batch.solve
        _, _, infos = fn(fus, gps, rtol=TOL, maxit=500, us=us, ps=ps)
        assert all(i.status == "ok" for i in infos), infos
        return [i.iters for i in infos]

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    all_its = []
    for _ in range(args.steps):
        all_its.append(step())
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    cycles = sum(sum(x) for x in all_its)
    value = dofs(N_GRID) * cycles / elapsed
    iters = all_its[-1]

    # FP32 cycles inside FP64 refinement on the same batch
    step(mixed=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    mixed_its = step(mixed=True)
    torch.cuda.synchronize()
    mixed_elapsed = time.perf_counter() - t1

    # time to tolerance of each beta solved alone (FP64 and FP32+refinement)
    tt64, tt32 = {}, {}
    for b, (fu, gp) in zip(BETAS, loads):
        h = Hierarchy(N_GRID, b, schedule=sched_single)
        for mixed, dst in ((False, tt64), (True, tt32)):
            fn = h.solve_mixed if mixed else h.solve
            fn(fu, gp, rtol=TOL, maxit=500)
            torch.cuda.synchronize()
            ta = time.perf_counter()
            _, _, info = fn(fu, gp, rtol=TOL, maxit=500)
            torch.cuda.synchronize()
            dst[str(b)] = 1e3 * (time.perf_counter() - ta)
        del h

    # dominant kernel: the batched finest-level fused normal-equation step,
    # timed with HIP events on the stream it runs on
    kern_ms = batch.time_kernel(0, reps=args.kernel_reps)
    roof = roofline_block("finest-level fused normal-equation step, all 5 instances (k_ne_b<double,16,8>)",
                          [N_GRID] * len(BETAS), kern_ms, counter_traffic())
    # the whole iterate against the model bytes of the cycle (304 B per
    # unknown for an FP64 V(2,2) iterate)
    roof["per_cycle_model_GBps"] = MODEL_BYTES_PER_DOF_V22 * dofs(N_GRID) * cycles / elapsed / 1e9
    roof["per_cycle_model_frac"] = roof["per_cycle_model_GBps"] / HBM_PEAK_GBS

    out = {
        "metric": "velocity+pressure DOF*cycles/s (FP64 NE V(2,2) to 1e-8, h=1/128, 5 betas)",
        "value": value,
        "unit": "DOF*cycles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "generalized Stokes, unit square, h=1/128 same-diagonal grid, Taylor-Hood "
                               "P2-P1, f iid U[-1,1] (seed 0), g=0, FP64 NE V(2,2) to 1e-8, beta in "
                               "{0,1,1e2,1e4,1e6} solved as one batch",
                   "N": N_GRID, "dof": dofs(N_GRID), "betas": BETAS, "levels": batch[0].nlevels},
        "iterations": dict(zip([str(b) for b in BETAS], iters)),
        "schedule": {"batch": sched_batch, "batch_ms_per_iterate": rec_batch["ms_per_iterate"],
                     "single": sched_single, "single_ms_per_iterate": rec_single["ms_per_iterate"],
                     "tuning_s": t_tune},
        "time_to_tol_ms_batch": 1e3 * elapsed / args.steps,
        "setup_ms_batch": 1e3 * t_setup,
        "time_to_tol_ms_single": tt64,
        "fp32_refine": {
            "value": dofs(N_GRID) * sum(mixed_its) / mixed_elapsed,
            "iterations": dict(zip([str(b) for b in BETAS], mixed_its)),
            "time_to_tol_ms_batch": 1e3 * mixed_elapsed,
            "time_to_tol_ms_single": tt32,
        },
        "roofline": roof,
    }
    if not args.no_extras:
        del batch, loads, fus, gps, outs, us, ps
        torch.cuda.empty_cache()
        out["extras"] = extras()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
