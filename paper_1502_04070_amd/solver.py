"""Python front end of the MI355X coupled Stokes multigrid (thin: it checks
shapes and marshals torch device pointers and the current stream into the C
ABI of libstokesmg.so; all arithmetic runs in the HIP kernels).

Layouts (level with N squares per side, M = 2N + 1), torch float64 on the GPU:
    velocity   (2, M, M)      [component, y index, x index]
    pressure   (N + 1, N + 1) [y index, x index]
Pressure sign: the paper's variational form, i.e. minus the strong-form
pressure of Section 1 (see include/stokesmg.h).
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import torch

from . import _lib


@dataclass
class SolveInfo:
    status: str
    iters: int
    relres: float
    history: list


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


SCHEDULE_FIELDS = ("fuse_depth", "coarse_max_n", "tile_x")


def _apply_damping(set_level, damping):
    """damping = {"tau": [per level], "sigma": [per level]} (level 0 first)."""
    taus, sigmas = damping.get("tau"), damping.get("sigma")
    n = len(taus) if taus is not None else len(sigmas)
    for level in range(n):
        set_level(level, taus[level] if taus is not None else None,
                  sigmas[level] if sigmas is not None else None)


def _set_domain(params, domain):
    """"square": the unit square; "l_shape": the unit square without
    [1/2, 1]^2 (needs an even n0); "union_jack": the unit square on the grid
    of the paper's experiments, the diagonals of the coarsest 2 x 2 grid
    meeting at the centre (even n0; fused and unfused kernels, batches).  The
    lattice layouts are those of the square; entries at points outside the
    domain are ignored and written zero or left as they were."""
    if domain not in _lib.DOMAINS:
        raise ValueError(f"domain must be one of {list(_lib.DOMAINS)}")
    params.domain = _lib.DOMAINS[domain]


def _set_schedule(params, schedule):
    """Launch schedule of the fused kernels (see smg_params); None: defaults."""
    for k, v in (schedule or {}).items():
        if k not in SCHEDULE_FIELDS:
            raise ValueError(f"unknown schedule field {k!r}")
        setattr(params, k, int(v))


def residual_noalloc(N, beta, fu, gp, u, p, domain="square", ru=None, rp=None, norm=False):
    """r = F - calA x on a grid of N x N squares with coefficient beta, without
    a hierarchy and without device allocation inside the library (the norm's
    partial sums use its fixed device scratch array; the caller passes every
    vector, ru / rp are allocated here only if not given).  Returns (ru, rp)
    or (ru, rp, norm2) with norm2 a one-element device tensor."""
    lib = _lib.load()
    if domain not in _lib.DOMAINS:
        raise ValueError(f"domain must be one of {list(_lib.DOMAINS)}")
    M = 2 * int(N) + 1
    for t, shape in ((fu, (2, M, M)), (gp, (N + 1, N + 1)), (u, (2, M, M)), (p, (N + 1, N + 1))):
        if tuple(t.shape) != shape or t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
            raise ValueError(f"expected a contiguous float64 CUDA tensor of shape {shape}")
    ru = torch.empty_like(u) if ru is None else ru
    rp = torch.empty_like(p) if rp is None else rp
    n2 = torch.zeros(1, dtype=torch.float64, device=u.device) if norm else None
    _lib.check(lib.smg_residual_noalloc(int(N), float(beta), _lib.DOMAINS[domain], _ptr(fu), _ptr(gp), _ptr(u),
                                        _ptr(p), _ptr(ru), _ptr(rp), _ptr(n2), _stream()), "smg_residual_noalloc")
    return (ru, rp, n2) if norm else (ru, rp)


class Hierarchy:
    """A multigrid hierarchy of the generalized Stokes system (Taylor-Hood
    P2-P1, uniformly refined grid): the unit square on the same-diagonal grid,
    the L-shaped domain on the same grid, or the unit square on the union-jack
    grid of the paper's experiments (the `domain` argument)."""

    def __init__(self, N: int, beta: float, smoother: str = "ne", tau: float | None = None,
                 sigma: float = 0.8, nu_pre: int = 2, nu_post: int = 2, gamma: int = 1,
                 n0: int = 2, fused: bool = True, device=None, schedule: dict | None = None,
                 damping: dict | None = None, domain: str = "square"):
        self.lib = _lib.load()
        if not torch.cuda.is_available():
            raise RuntimeError("the HIP solver needs a GPU")
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else
                                   torch.device(device).index or 0)
        if smoother not in _lib.SMOOTHERS:
            raise ValueError(f"smoother must be one of {list(_lib.SMOOTHERS)}")
        if tau is None:
            tau = 0.35 if smoother == "ne" else 0.8
        self.params = _lib.SmgParams(_lib.SMOOTHERS[smoother], float(tau), float(sigma),
                                     int(nu_pre), int(nu_post), int(gamma), int(n0), 0 if fused else 1)
        _set_schedule(self.params, schedule)
        _set_domain(self.params, domain)
        self.N, self.beta, self.smoother, self.domain = int(N), float(beta), smoother, domain
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            _lib.check(self.lib.smg_setup(self.N, self.beta, C.byref(self.params), C.byref(h)),
                       "smg_setup")
        self.h = h
        self._owned = True
        self.nlevels = self.lib.smg_num_levels(h)
        self.L = self.nlevels - 1
        if damping:
            _apply_damping(self.set_damping, damping)

    @classmethod
    def _view(cls, lib, handle, params, N, beta, smoother, device):
        """A non-owning front end for a hierarchy that belongs to a batch."""
        self = cls.__new__(cls)
        self.lib, self.h, self.params = lib, C.c_void_p(handle), params
        self.N, self.beta, self.smoother, self.device = N, beta, smoother, device
        self.domain = next(k for k, v in _lib.DOMAINS.items() if v == params.domain)
        self._owned = False
        self.nlevels = lib.smg_num_levels(self.h)
        self.L = self.nlevels - 1
        return self

    def __del__(self):
        h = getattr(self, "h", None)
        if getattr(self, "_owned", True) and h is not None and h.value:
            self.lib.smg_destroy(h)
            self.h = None

    # -- sizes / allocation ----------------------------------------------------
    def level_N(self, level: int | None = None) -> int:
        level = self.L if level is None else level
        n = C.c_int()
        _lib.check(self.lib.smg_level_size(self.h, level, C.byref(n), None, None), "smg_level_size")
        return n.value

    def shapes(self, level: int | None = None):
        N = self.level_N(level)
        return (2, 2 * N + 1, 2 * N + 1), (N + 1, N + 1)

    def zeros(self, level: int | None = None, dtype=torch.float64):
        su, sp = self.shapes(level)
        return (torch.zeros(su, dtype=dtype, device=self.device),
                torch.zeros(sp, dtype=dtype, device=self.device))

    def dofs(self, level: int | None = None) -> int:
        """Velocity (interior, both components) plus pressure (all nodes) unknowns."""
        N = self.level_N(level)
        return 2 * (2 * N - 1) ** 2 + (N + 1) ** 2

    def _chk(self, level, *pairs, dtype=torch.float64):
        su, sp = self.shapes(level)
        for t, kind in pairs:
            if t is None:
                continue
            shape = su if kind == "u" else sp
            if t.dtype != dtype or t.device != self.device or tuple(t.shape) != shape or not t.is_contiguous():
                raise ValueError(f"expected contiguous {dtype} tensor of shape {shape} on {self.device}, "
                                 f"got {t.dtype} {tuple(t.shape)} on {t.device}")

    # -- operators ---------------------------------------------------------------
    def load(self, f_nodal, g_nodal, level=None):
        level = self.L if level is None else level
        self._chk(level, (f_nodal, "u"), (g_nodal, "p"))
        fu, gp = self.zeros(level)
        _lib.check(self.lib.smg_load(self.h, level, _ptr(f_nodal), _ptr(g_nodal), _ptr(fu), _ptr(gp),
                                     _stream()), "smg_load")
        return fu, gp

    def mass(self, u, all_nodes=False, level=None):
        level = self.L if level is None else level
        self._chk(level, (u, "u"))
        y = torch.empty_like(u)
        _lib.check(self.lib.smg_mass(self.h, level, int(all_nodes), _ptr(u), _ptr(y), _stream()), "smg_mass")
        return y

    def pressure_mass(self, g, level=None):
        level = self.L if level is None else level
        self._chk(level, (g, "p"))
        y = torch.empty_like(g)
        _lib.check(self.lib.smg_pressure_mass(self.h, level, _ptr(g), _ptr(y), _stream()),
                   "smg_pressure_mass")
        return y

    def apply(self, u, p, level=None):
        level = self.L if level is None else level
        self._chk(level, (u, "u"), (p, "p"))
        yu, yp = torch.empty_like(u), torch.empty_like(p)
        _lib.check(self.lib.smg_apply(self.h, level, _ptr(u), _ptr(p), _ptr(yu), _ptr(yp), _stream()),
                   "smg_apply")
        return yu, yp

    def residual(self, fu, gp, u, p, level=None, norm=False):
        level = self.L if level is None else level
        self._chk(level, (fu, "u"), (gp, "p"), (u, "u"), (p, "p"))
        ru, rp = torch.empty_like(u), torch.empty_like(p)
        n2 = torch.zeros(1, dtype=torch.float64, device=self.device) if norm else None
        _lib.check(self.lib.smg_residual(self.h, level, _ptr(fu), _ptr(gp), _ptr(u), _ptr(p), _ptr(ru),
                                         _ptr(rp), _ptr(n2), _stream()), "smg_residual")
        return (ru, rp, n2) if norm else (ru, rp)

    def smooth(self, fu, gp, u, p, nsteps=1, level=None):
        """In place on (u, p)."""
        level = self.L if level is None else level
        self._chk(level, (fu, "u"), (gp, "p"), (u, "u"), (p, "p"))
        _lib.check(self.lib.smg_smooth(self.h, level, int(nsteps), _ptr(fu), _ptr(gp), _ptr(u), _ptr(p),
                                       _stream()), "smg_smooth")
        return u, p

    def restrict(self, ru, rp, fine_level=None):
        fine_level = self.L if fine_level is None else fine_level
        self._chk(fine_level, (ru, "u"), (rp, "p"))
        cu, cp = self.zeros(fine_level - 1)
        _lib.check(self.lib.smg_restrict(self.h, fine_level, _ptr(ru), _ptr(rp), _ptr(cu), _ptr(cp),
                                         _stream()), "smg_restrict")
        return cu, cp

    def prolong_add(self, zu, zp, u, p, fine_level=None):
        """In place on (u, p)."""
        fine_level = self.L if fine_level is None else fine_level
        self._chk(fine_level - 1, (zu, "u"), (zp, "p"))
        self._chk(fine_level, (u, "u"), (p, "p"))
        _lib.check(self.lib.smg_prolong_add(self.h, fine_level, _ptr(zu), _ptr(zp), _ptr(u), _ptr(p),
                                            _stream()), "smg_prolong_add")
        return u, p

    def coarse_solve(self, ru, rp):
        self._chk(0, (ru, "u"), (rp, "p"))
        zu, zp = self.zeros(0)
        _lib.check(self.lib.smg_coarse_solve(self.h, _ptr(ru), _ptr(rp), _ptr(zu), _ptr(zp), _stream()),
                   "smg_coarse_solve")
        return zu, zp

    def project_mean(self, p, level=None):
        """In place on p."""
        level = self.L if level is None else level
        self._chk(level, (p, "p"))
        _lib.check(self.lib.smg_project_mean(self.h, level, _ptr(p), _stream()), "smg_project_mean")
        return p

    def project_dual(self, v, level=None):
        """In place: v <- v - m (sum v) / (sum m), the transpose of project_mean."""
        level = self.L if level is None else level
        self._chk(level, (v, "p"))
        _lib.check(self.lib.smg_project_dual(self.h, level, _ptr(v), _stream()), "smg_project_dual")
        return v

    def dot(self, a, b, which, level=None):
        level = self.L if level is None else level
        self._chk(level, (a, "u" if which == 0 else "p"), (b, "u" if which == 0 else "p"))
        out = torch.zeros(1, dtype=torch.float64, device=self.device)
        _lib.check(self.lib.smg_dot(self.h, level, int(which), _ptr(a), _ptr(b), _ptr(out), _stream()),
                   "smg_dot")
        return out

    def time_kernel(self, which: int, reps: int = 50) -> float:
        """Mean duration (ms) of one finest-level stencil kernel (see smg_time_kernel)."""
        ms = C.c_double()
        _lib.check(self.lib.smg_time_kernel(self.h, int(which), int(reps), C.byref(ms), _stream()),
                   "smg_time_kernel")
        return ms.value

    # -- iterates ----------------------------------------------------------------
    def cycle(self, fu, gp, u, p):
        """One iterate on the finest level, in place on (u, p)."""
        self._chk(self.L, (fu, "u"), (gp, "p"), (u, "u"), (p, "p"))
        _lib.check(self.lib.smg_cycle(self.h, _ptr(fu), _ptr(gp), _ptr(u), _ptr(p), _stream()), "smg_cycle")
        return u, p

    def cycle_f32(self, fu, gp, u, p):
        self._chk(self.L, (fu, "u"), (gp, "p"), (u, "u"), (p, "p"), dtype=torch.float32)
        _lib.check(self.lib.smg_cycle_f32(self.h, _ptr(fu), _ptr(gp), _ptr(u), _ptr(p), _stream()),
                   "smg_cycle_f32")
        return u, p

    def _solve(self, fn, name, fu, gp, rtol, maxit, u, p):
        self._chk(self.L, (fu, "u"), (gp, "p"))
        if u is None:
            u, p = self.zeros()
        self._chk(self.L, (u, "u"), (p, "p"))
        it = C.c_int()
        rel = C.c_double()
        hist = (C.c_double * max(int(maxit), 1))()
        code = fn(self.h, _ptr(fu), _ptr(gp), float(rtol), int(maxit), _ptr(u), _ptr(p), C.byref(it),
                  C.byref(rel), hist, _stream())
        _lib.check(code, name, soft_ok=True)
        return u, p, SolveInfo(_lib.STATUS[code], it.value, rel.value, list(hist[: it.value]))

    def solve(self, fu, gp, rtol=1e-8, maxit=200, u=None, p=None):
        """Iterate to ||F - calA x|| <= rtol ||F||; returns (u, p, SolveInfo)."""
        return self._solve(self.lib.smg_solve, "smg_solve", fu, gp, rtol, maxit, u, p)

    def set_damping(self, level: int, tau: float | None, sigma: float | None = None):
        """Smoother damping of one level (-1: all levels); None keeps a value."""
        if tau is None or sigma is None:
            t0, s0 = self.damping(max(level, 0))
            tau = t0 if tau is None else tau
            sigma = s0 if sigma is None else sigma
        _lib.check(self.lib.smg_set_damping(self.h, int(level), float(tau), float(sigma)), "smg_set_damping")

    def damping(self, level: int):
        t, sg = C.c_double(), C.c_double()
        _lib.check(self.lib.smg_get_damping(self.h, int(level), C.byref(t), C.byref(sg)), "smg_get_damping")
        return t.value, sg.value

    def implicit_step(self, u, p, f_nodal=None, g_nodal=None, rtol=1e-10, maxit=200, mixed=False):
        """One implicit Euler step with dt = 1 / beta of this hierarchy, in place:
        (u, p) = (u^n, guess) -> (u^{n+1}, p^{n+1}).  f_nodal: nodal values at all
        P2 lattice points, g_nodal: P1 nodal values with zero integral.  mixed:
        FP32 cycles inside FP64 iterative refinement."""
        L = self.L
        self._chk(L, (u, "u"), (p, "p"))
        if f_nodal is not None:
            self._chk(L, (f_nodal, "u"))
        if g_nodal is not None:
            self._chk(L, (g_nodal, "p"))
        it, rel = C.c_int(), C.c_double()
        name = "smg_implicit_step_mixed" if mixed else "smg_implicit_step"
        code = getattr(self.lib, name)(self.h, _ptr(f_nodal), _ptr(g_nodal), float(rtol), int(maxit),
                                       _ptr(u), _ptr(p), C.byref(it), C.byref(rel), _stream())
        _lib.check(code, name, soft_ok=True)
        return SolveInfo(_lib.STATUS[code], it.value, rel.value, [])

    def error_norm(self, u, p, us, ps) -> float:
        """||(u, p) - (us, ps)||_L of Section 6 (pressure difference made mean-free)."""
        L = self.L
        self._chk(L, (u, "u"), (p, "p"), (us, "u"), (ps, "p"))
        out = C.c_double()
        _lib.check(self.lib.smg_error_norm(self.h, _ptr(u), _ptr(p), _ptr(us), _ptr(ps), C.byref(out), _stream()),
                   "smg_error_norm")
        return out.value

    def solve_error(self, fu, gp, us, ps, eps=1e-9, maxit=200, u=None, p=None):
        """The protocol of Section 6: iterate from (u, p) (zero by default) on
        (fu, gp) until the L-norm error to x* = (us, ps) has dropped by eps.
        Returns (u, p, iters, rate, status)."""
        L = self.L
        if u is None:
            u, p = self.zeros()
        self._chk(L, (fu, "u"), (gp, "p"), (us, "u"), (ps, "p"), (u, "u"), (p, "p"))
        it, rate = C.c_int(), C.c_double()
        code = self.lib.smg_solve_error(self.h, _ptr(fu), _ptr(gp), _ptr(us), _ptr(ps), float(eps), int(maxit),
                                        _ptr(u), _ptr(p), C.byref(it), C.byref(rate), _stream())
        _lib.check(code, "smg_solve_error", soft_ok=True)
        return u, p, it.value, rate.value, _lib.STATUS[code]

    def solve_mixed(self, fu, gp, rtol=1e-10, maxit=400, u=None, p=None):
        """FP32 cycles inside FP64 iterative refinement."""
        return self._solve(self.lib.smg_solve_mixed, "smg_solve_mixed", fu, gp, rtol, maxit, u, p)


def _fill(h, level, tau, sigma):
    t0, s0 = h.damping(level)
    return (t0 if tau is None else tau), (s0 if sigma is None else sigma)


class Batch:
    """Many independent instances (sizes N_k = n0 2^L_k, coefficients beta_k)
    solved together: one launch per stage for all of them, replayed from
    captured graphs of one and of four iterates.  Several right-hand sides of one problem are several
    instances with equal (N, beta)."""

    def __init__(self, Ns, betas, smoother: str = "ne", tau: float | None = None, sigma: float = 0.8,
                 nu_pre: int = 2, nu_post: int = 2, gamma: int = 1, n0: int = 2,
                 schedule: dict | None = None, damping: dict | None = None, domain: str = "square"):
        self.lib = _lib.load()
        if not torch.cuda.is_available():
            raise RuntimeError("the HIP solver needs a GPU")
        if len(Ns) != len(betas):
            raise ValueError("Ns and betas differ in length")
        if tau is None:
            tau = 0.35 if smoother == "ne" else 0.8
        self.params = _lib.SmgParams(_lib.SMOOTHERS[smoother], float(tau), float(sigma), int(nu_pre),
                                     int(nu_post), int(gamma), int(n0), 0)
        _set_schedule(self.params, schedule)
        _set_domain(self.params, domain)
        n = len(Ns)
        Na = (C.c_int * n)(*[int(v) for v in Ns])
        Ba = (C.c_double * n)(*[float(v) for v in betas])
        b = C.c_void_p()
        _lib.check(self.lib.smg_batch_setup(n, Na, Ba, C.byref(self.params), C.byref(b)), "smg_batch_setup")
        self.b = b
        self.n = n
        dev = torch.device("cuda", torch.cuda.current_device())
        self.instances = [Hierarchy._view(self.lib, self.lib.smg_batch_handle(b, k), self.params, int(Ns[k]),
                                          float(betas[k]), smoother, dev) for k in range(n)]
        if damping:
            # one damping table for every instance (levels beyond an instance's depth are skipped)
            for k, h in enumerate(self.instances):
                _apply_damping(lambda lv, t, sg, k=k, h=h: self.set_damping(k, lv, *_fill(h, lv, t, sg))
                               if lv <= h.L else None, damping)

    def __len__(self):
        return self.n

    def __getitem__(self, k) -> Hierarchy:
        return self.instances[k]

    def __del__(self):
        b = getattr(self, "b", None)
        if b is not None and b.value:
            self.lib.smg_batch_destroy(b)
            self.b = None

    def _solve(self, fn, name, fus, gps, rtol, maxit, us, ps):
        n = self.n
        if us is None:
            us, ps = zip(*[h.zeros() for h in self.instances])
        for k, h in enumerate(self.instances):
            h._chk(h.L, (fus[k], "u"), (gps[k], "p"), (us[k], "u"), (ps[k], "p"))
        arr = lambda ts: (C.c_void_p * n)(*[t.data_ptr() for t in ts])
        it = (C.c_int * n)()
        rel = (C.c_double * n)()
        st = (C.c_int * n)()
        code = fn(self.b, arr(fus), arr(gps), float(rtol), int(maxit), arr(us), arr(ps), it, rel, st, _stream())
        _lib.check(code, name, soft_ok=True)
        infos = [SolveInfo(_lib.STATUS[st[k]], it[k], rel[k], []) for k in range(n)]
        return list(us), list(ps), infos

    def time_kernel(self, which: int = 0, reps: int = 50) -> float:
        """Mean duration (ms) of one batched finest-level fused NE step launch."""
        ms = C.c_double()
        _lib.check(self.lib.smg_batch_time_kernel(self.b, int(which), int(reps), C.byref(ms), _stream()),
                   "smg_batch_time_kernel")
        return ms.value

    def solve(self, fus, gps, rtol=1e-8, maxit=200, us=None, ps=None):
        return self._solve(self.lib.smg_batch_solve, "smg_batch_solve", fus, gps, rtol, maxit, us, ps)

    def set_damping(self, instance: int, level: int, tau: float, sigma: float):
        """Smoother damping of one level (-1: all) of one instance (-1: all)."""
        _lib.check(self.lib.smg_batch_set_damping(self.b, int(instance), int(level), float(tau), float(sigma)),
                   "smg_batch_set_damping")

    def implicit_step(self, us, ps, f_nodals=None, g_nodals=None, rtol=1e-10, maxit=200, mixed=False):
        """Hierarchy.implicit_step for every instance (dt_k = 1 / beta_k), in place."""
        n = self.n
        for k, h in enumerate(self.instances):
            h._chk(h.L, (us[k], "u"), (ps[k], "p"))
            if f_nodals is not None and f_nodals[k] is not None:
                h._chk(h.L, (f_nodals[k], "u"))
            if g_nodals is not None and g_nodals[k] is not None:
                h._chk(h.L, (g_nodals[k], "p"))
        arr = lambda ts: (C.c_void_p * n)(*[(t.data_ptr() if t is not None else None) for t in ts])
        it = (C.c_int * n)()
        rel = (C.c_double * n)()
        st = (C.c_int * n)()
        name = "smg_batch_implicit_step_mixed" if mixed else "smg_batch_implicit_step"
        code = getattr(self.lib, name)(self.b, arr(f_nodals) if f_nodals is not None else None,
                                       arr(g_nodals) if g_nodals is not None else None, float(rtol),
                                       int(maxit), arr(us), arr(ps), it, rel, st, _stream())
        _lib.check(code, name, soft_ok=True)
        return [SolveInfo(_lib.STATUS[st[k]], it[k], rel[k], []) for k in range(n)]

    def solve_mixed(self, fus, gps, rtol=1e-10, maxit=400, us=None, ps=None):
        return self._solve(self.lib.smg_batch_solve_mixed, "smg_batch_solve_mixed", fus, gps, rtol, maxit, us, ps)
