// Host runtime and C ABI of the coupled Stokes multigrid (see include/stokesmg.h).
//
// A handle owns one hierarchy: per-level stencil coefficients and Shat^-1
// arrays (Section 6 preconditioner), work vectors in FP64 and FP32, the
// inverse of the bordered coarsest-grid matrix (Section 3: level 0 is solved
// exactly) and the device-side convergence state of the solve loop.
//
// The solve loop runs one iterate per replay of a captured HIP graph; every
// kernel of an iterate first reads a device flag and returns at once when
// the loop has already converged, so the host enqueues several iterates
// between synchronizations without changing the result.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <initializer_list>
#include <type_traits>
#include <vector>

#include "smg_fused.h"
#include "smg_host.h"
#include "smg_internal.h"
#include "stokesmg.h"

namespace smg {
#include "stencils.inc"
#include "smg_uj.h"
}

using namespace smg;
using smg::smg_stencil::A_K;
using smg::smg_stencil::A_M;
using smg::smg_stencil::DIAG_K;
using smg::smg_stencil::DIAG_M;

namespace {

using host::fail;

#define HIPCHK(x)                                                                      \
  do {                                                                                 \
    hipError_t e_ = (x);                                                               \
    if (e_ != hipSuccess) return fail(SMG_EHIP, "%s: %s", #x, hipGetErrorString(e_));  \
  } while (0)

// iterates per repeated-iterate graph of a solve (the iterate graph launched
// alone covers the rest of a chunk)
constexpr int ITER_GRAPH_REPS = 4;

template <class T>
struct Vec {
  T* u = nullptr;  // [2][M][M]
  T* p = nullptr;  // [N+1][N+1], directly after u
};

struct Level {
  int N = 0;
  int64_t n_u = 0, n_p = 0;  // lattice sizes: 2 M^2 and (N+1)^2
  LevelCoef<double> c64{};
  LevelCoef<float> c32{};
  Vec<double> x, f, t;
  Vec<float> x32, f32, t32;
  double* partial = nullptr;  // one double per stencil tile
  int ntiles = 0;
  double tau = 0.0, sigma = 0.0;  // smoother damping on this level (smg_set_damping)
};

template <class T> struct Sel;
template <> struct Sel<double> {
  static LevelCoef<double>& c(Level& L) { return L.c64; }
  static Vec<double>& x(Level& L) { return L.x; }
  static Vec<double>& f(Level& L) { return L.f; }
  static Vec<double>& t(Level& L) { return L.t; }
};
template <> struct Sel<float> {
  static LevelCoef<float>& c(Level& L) { return L.c32; }
  static Vec<float>& x(Level& L) { return L.x32; }
  static Vec<float>& f(Level& L) { return L.f32; }
  static Vec<float>& t(Level& L) { return L.t32; }
};

}  // namespace

struct smg_hier {
  int device = 0;
  smg_params prm{};
  double beta = 0;
  int L = 0;
  std::vector<Level> lv;
  double* cinv = nullptr;  // column-major inverse of the bordered coarse matrix
  int nc = 0;
  SolveState* st = nullptr;        // device
  SolveState* st_host = nullptr;   // pinned host mirror
  double* hist = nullptr;          // device, hist_cap doubles
  int hist_cap = 0;
  double* red = nullptr;           // reduction scratch
  int red_cap = 0;
  double* fdots = nullptr;         // 2 doubles
  double* enorm = nullptr;         // 4 doubles (error-measure pieces)
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t g64 = nullptr, g32 = nullptr;     // one iterate
  hipGraphExec_t g64r = nullptr, g32r = nullptr;   // ITER_GRAPH_REPS iterates
  hipGraphExec_t gerr = nullptr;   // protocol iterate (cycle, projection, error measure)
  const void* gerr_key[6] = {};    // the vectors it was captured with
  // bumped whenever a value that captured launches carry changes (damping,
  // history buffer): batches holding this instance re-plan when it moved
  unsigned gen = 0;
  // single-workgroup iterate of levels 0..Lc (Lc = -1: not used)
  int Lc = -1;
  int* cc_ops = nullptr;
  int cc_nops = 0;
  // dense map of levels 0..Lc from a zero iterate (kn = 0: not formed)
  double* kd = nullptr;
  float* kf = nullptr;
  int kn = 0, knu = 0;
  bool dense_on = true;            // used by the iterates (off for solves near its rounding floor)
  double* mpart = nullptr;         // pressure-mean partials of the finest level
  bool fused = true;
  bool ne2 = true;                 // pairs of normal-equation steps in one launch (8 x 8 levels)
  int tile_x = 0;                  // normal-equation tile width (0: by level size)
  int dom = SMG_DOM_SQUARE;        // domain of the grid (SMG_DOM_*)
  int ne_tx(int N) const { return tile_x ? tile_x : ne_tile_shape(N).tx; }
  std::vector<void*> allocs;

  template <class T>
  T* alloc(int64_t n) {
    void* p = nullptr;
    if (hipMalloc(&p, sizeof(T) * std::max<int64_t>(n, 1)) != hipSuccess) return nullptr;
    allocs.push_back(p);
    return static_cast<T*>(p);
  }
  ~smg_hier() {
    // teardown: errors cannot be reported from a destructor
    for (hipGraphExec_t g : {g64, g32, g64r, g32r, gerr})
      if (g) (void)hipGraphExecDestroy(g);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    for (void* p : allocs) (void)hipFree(p);
    if (st_host) (void)hipHostFree(st_host);
  }
};

namespace {

// ---------------------------------------------------------------------------
// enqueue helpers
// ---------------------------------------------------------------------------

template <class T>
StencilJob<T> job_of(Level& L) {
  StencilJob<T> J{};
  J.L = Sel<T>::c(L);
  J.w_u = J.w_p = T(1);
  return J;
}

// One smoothing step (Section 4) on (x, f) with scratch t.  zg: x is zero on
// entry (its reads are skipped; the arithmetic is that of x = 0).
template <class T>
void smooth_step(const smg_params& prm, Level& L, Vec<T> x, Vec<T> f, Vec<T> t, bool zg,
                 const int* done, hipStream_t s) {
  if (prm.smoother == SMG_SMOOTHER_NE) {
    // t = L^-1 (f - calA x);  x = x + tau L^-1 calA t
    StencilJob<T> A = job_of<T>(L);
    A.in_u = zg ? nullptr : x.u;
    A.in_p = zg ? nullptr : x.p;
    A.rhs_u = f.u; A.rhs_p = f.p;
    A.diag_u = A.diag_p = 1;
    A.out_u = t.u; A.out_p = t.p;
    A.done = done;
    launch_stencil<T>(A, ROWS_UP, s);
    StencilJob<T> B = job_of<T>(L);
    B.in_u = t.u; B.in_p = t.p;
    B.base_u = zg ? nullptr : x.u;
    B.base_p = zg ? nullptr : x.p;
    B.w_u = B.w_p = T(-L.tau);
    B.diag_u = B.diag_p = 1;
    B.out_u = x.u; B.out_p = x.p;
    B.done = done;
    launch_stencil<T>(B, ROWS_UP, s);
  } else {
    // t.u = u + tau Ahat^-1 (f - A u - B^T p)
    StencilJob<T> A = job_of<T>(L);
    A.in_u = zg ? nullptr : x.u;
    A.in_p = zg ? nullptr : x.p;
    A.rhs_u = f.u;
    A.base_u = zg ? nullptr : x.u;
    A.w_u = T(L.tau);
    A.diag_u = 1;
    A.out_u = t.u;
    A.done = done;
    launch_stencil<T>(A, ROWS_U, s);
    // t.p = dp = -sigma Shat^-1 (g - B t.u)
    StencilJob<T> B = job_of<T>(L);
    B.in_u = t.u;
    B.rhs_p = f.p;
    B.w_p = T(-L.sigma);
    B.diag_p = 1;
    B.out_p = t.p;
    B.done = done;
    launch_stencil<T>(B, ROWS_P, s);
    // x.u = t.u - tau Ahat^-1 B^T dp;  x.p = p + dp
    StencilJob<T> C = job_of<T>(L);
    C.in_p = t.p;
    C.base_u = t.u;
    C.w_u = T(L.tau);
    C.diag_u = 1;
    C.rhs_p = t.p;
    C.base_p = zg ? nullptr : x.p;
    C.w_p = T(1);
    C.out_u = x.u; C.out_p = x.p;
    C.done = done;
    launch_stencil<T>(C, ROWS_UP, s);
  }
}

template <class T>
void fill_vec(Level& L, Vec<T> v, hipStream_t s) {
  if constexpr (sizeof(T) == 8) launch_fill((double*)v.u, L.n_u + L.n_p, 0.0, s);
  else launch_fill_f32((float*)v.u, L.n_u + L.n_p, 0.0f, s);
}

// Multigrid iterate of Section 3 on level l for (x, f); zg: x = 0 on entry.
template <class T>
void coarse_cycle(smg_hier* H, Vec<T> x, Vec<T> f, bool zg, const int* done, hipStream_t s);

template <class T>
void cycle_rec(smg_hier* H, int l, Vec<T> x, Vec<T> f, bool zg, const int* done, hipStream_t s) {
  Level& L = H->lv[l];
  if (l == 0) {
    launch_coarse_solve<T>(L.N, H->dom, H->nc, H->cinv, f.u, f.p, x.u, x.p, done, s);
    return;
  }
  // the union-jack grid (always on this path) does its coarse levels in the
  // single-workgroup kernel: a W-cycle visits them thousands of times
  if (H->dom == SMG_DOM_UNIONJACK && l <= H->Lc) {
    coarse_cycle<T>(H, x, f, zg, done, s);
    return;
  }
  const smg_params& prm = H->prm;
  Vec<T> t = Sel<T>::t(L);
  bool z = zg;
  if (z && prm.nu_pre == 0) {
    fill_vec<T>(L, x, s);
    z = false;
  }
  for (int k = 0; k < prm.nu_pre; ++k) {
    smooth_step<T>(prm, L, x, f, t, z, done, s);
    z = false;
  }
  // defect, restricted with the transposed embedding
  StencilJob<T> R = job_of<T>(L);
  R.in_u = x.u; R.in_p = x.p;
  R.rhs_u = f.u; R.rhs_p = f.p;
  R.out_u = t.u; R.out_p = t.p;
  R.done = done;
  launch_stencil<T>(R, ROWS_UP, s);
  Level& C = H->lv[l - 1];
  Vec<T> xc = Sel<T>::x(C), fc = Sel<T>::f(C);
  launch_restrict<T>(C.N, H->dom, t.u, t.p, fc.u, fc.p, nullptr, nullptr, done, s);
  for (int g = 0; g < prm.gamma; ++g) cycle_rec<T>(H, l - 1, xc, fc, g == 0, done, s);
  launch_prolong_add<T>(C.N, H->dom, xc.u, xc.p, x.u, x.p, done, s);
  for (int k = 0; k < prm.nu_post; ++k) smooth_step<T>(prm, L, x, f, t, false, done, s);
}

// ---------------------------------------------------------------------------
// fused iterate: k_ne steps alternating between the level's x and t buffers,
// k_resid_restrict, and one k_coarse_cycle launch for levels 0..Lc
// ---------------------------------------------------------------------------

// op list of the single-workgroup kernel, the recursion of Section 3 on
// levels l..0 written out (zg: the iterate of level l is zero on entry)
void cc_emit(const smg_params& prm, int l, bool zg, std::vector<int>& ops) {
  if (l == 0) {
    ops.push_back(cc_op(CC_COARSE, 0, 0));
    return;
  }
  const int sm = prm.smoother == SMG_SMOOTHER_NE ? CC_NE : CC_UZAWA;
  bool z = zg;
  for (int k = 0; k < prm.nu_pre; ++k) {
    ops.push_back(cc_op(sm, l, z ? 1 : 0));
    z = false;
  }
  ops.push_back(cc_op(CC_RESTRICT, l, 0));     // also zeroes the coarse iterate
  for (int g = 0; g < prm.gamma; ++g) cc_emit(prm, l - 1, g == 0, ops);
  ops.push_back(cc_op(CC_PROLONG, l, 0));
  for (int k = 0; k < prm.nu_post; ++k) ops.push_back(cc_op(sm, l, 0));
}

template <class T>
void coarse_cycle(smg_hier* H, Vec<T> x, Vec<T> f, bool zg, const int* done, hipStream_t s) {
  CoarseJob<T> J{};
  for (int l = 0; l <= H->Lc; ++l) J.L[l] = Sel<T>::c(H->lv[l]);
  J.n0 = H->prm.n0;
  J.Lc = H->Lc;
  J.nc = H->nc;
  J.nops = H->cc_nops;
  J.ops = H->cc_ops;
  J.cinv = H->cinv;
  J.fu = f.u; J.fp = f.p;
  J.xu = x.u; J.xp = x.p;
  J.zero_guess = zg ? 1 : 0;
  for (int l = 0; l <= H->Lc; ++l) {
    J.tau[l] = T(H->lv[l].tau);
    J.sigma[l] = T(H->lv[l].sigma);
  }
  J.done = done;
  launch_coarse_cycle<T>(J, s);
}

template <class T>
const T* kmap(const smg_hier* H);
template <>
const double* kmap<double>(const smg_hier* H) { return H->kd; }
template <>
const float* kmap<float>(const smg_hier* H) { return H->kf; }

// x = K f on level Lc (the coarse part of an iterate from a zero iterate)
template <class T>
DenseJob<T> dense_job(const smg_hier* H, Vec<T> x, Vec<T> f, const int* done) {
  DenseJob<T> J{};
  J.K = kmap<T>(H);
  J.n = H->kn;
  J.nu = H->knu;
  J.fu = f.u; J.fp = f.p;
  J.xu = x.u; J.xp = x.p;
  J.done = done;
  return J;
}

// Column j of K is the coarse-level kernel's result for the j-th unit vector
// of the lattice of level Lc (from a zero iterate): one batched launch with
// a job per column, in the precision of the cycle that will use it; K is then
// stored by rows.
template <class T>
int form_dense_map(smg_hier* H, T* K, hipStream_t s) {
  const int n = H->kn, nu = H->knu;
  std::vector<T> eye((size_t)n * n, T(0));
  for (int j = 0; j < n; ++j) eye[(size_t)j * n + j] = T(1);
  T* E = nullptr;
  CoarseJob<T>* jd = nullptr;
  int rc = SMG_OK;
  if (hipMalloc(&E, sizeof(T) * eye.size()) != hipSuccess ||
      hipMalloc(&jd, sizeof(CoarseJob<T>) * n) != hipSuccess) {
    rc = fail(SMG_ENOMEM, "dense coarse map");
  } else {
    CoarseJob<T> J{};
    for (int l = 0; l <= H->Lc; ++l) J.L[l] = Sel<T>::c(H->lv[l]);
    J.n0 = H->prm.n0;
    J.Lc = H->Lc;
    J.nc = H->nc;
    J.nops = H->cc_nops;
    J.ops = H->cc_ops;
    J.cinv = H->cinv;
    J.zero_guess = 1;
    for (int l = 0; l <= H->Lc; ++l) {
      J.tau[l] = T(H->lv[l].tau);
      J.sigma[l] = T(H->lv[l].sigma);
    }
    J.done = nullptr;
    std::vector<CoarseJob<T>> jobs(n, J);
    for (int j = 0; j < n; ++j) {
      jobs[j].fu = E + (size_t)j * n;
      jobs[j].fp = jobs[j].fu + nu;
      jobs[j].xu = K + (size_t)j * n;
      jobs[j].xp = jobs[j].xu + nu;
    }
    if (hipMemcpyAsync(E, eye.data(), sizeof(T) * eye.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(jd, jobs.data(), sizeof(CoarseJob<T>) * n, hipMemcpyHostToDevice, s) != hipSuccess) {
      rc = fail(SMG_EHIP, "dense coarse map upload");
    } else {
      launch_cc_b<T>(jd, n, coarse_cycle_lds(H->prm.n0, H->Lc, sizeof(T)), H->dom, s);
      if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) {
        rc = fail(SMG_EHIP, "dense coarse map launch");
      } else {
        // the launch wrote K column by column; k_ccd reads it by rows
        std::vector<T> col((size_t)n * n);
        if (hipMemcpy(col.data(), K, sizeof(T) * col.size(), hipMemcpyDeviceToHost) != hipSuccess) {
          rc = fail(SMG_EHIP, "dense coarse map read-back");
        } else {
          for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) eye[(size_t)i * n + j] = col[(size_t)j * n + i];
          if (hipMemcpy(K, eye.data(), sizeof(T) * eye.size(), hipMemcpyHostToDevice) != hipSuccess)
            rc = fail(SMG_EHIP, "dense coarse map upload");
        }
      }
    }
  }
  (void)hipStreamSynchronize(s);
  if (E) (void)hipFree(E);
  if (jd) (void)hipFree(jd);
  return rc;
}

// (Re)form the dense coarse maps of a fused hierarchy whose levels 0..Lc
// have at most KD_MAX lattice entries at Lc (N <= 8 with n0 = 2); otherwise,
// or when forming fails, the coarse-level kernel runs in every iterate.
void form_dense_maps(smg_hier* H, hipStream_t s) {
  H->kn = 0;
  // (with Lc = L the kernel runs only from the caller's iterate: not a zero one)
  if (!H->fused || H->Lc < 1 || H->Lc >= H->L) return;
  const int N = H->prm.n0 << H->Lc, M = 2 * N + 1;
  const int nu = 2 * M * M, n = nu + (N + 1) * (N + 1);
  if (n > KD_MAX) return;
  if (!H->kd) H->kd = H->alloc<double>((int64_t)n * n);
  if (!H->kf) H->kf = H->alloc<float>((int64_t)n * n);
  if (!H->kd || !H->kf) return;
  H->kn = n;
  H->knu = nu;
  if (form_dense_map<double>(H, H->kd, s) != SMG_OK || form_dense_map<float>(H, H->kf, s) != SMG_OK) {
    (void)hipGetLastError();
    H->kn = 0;
  }
}

template <class T>
void copy_vec(Level& L, Vec<T> dst, Vec<T> src, const int* done, hipStream_t s) {
  StencilJob<T> C = job_of<T>(L);
  C.rhs_u = src.u; C.rhs_p = src.p;
  C.out_u = dst.u; C.out_p = dst.p;
  C.done = done;
  launch_stencil<T>(C, ROWS_UP, s);   // dst = 0 + 1 * (src - 0), boundary written 0
}

// Fused iterate on level l for (x, f).  Returns the buffer holding the
// result: x itself, or the level's t buffer (its ping-pong partner).
// one fused Uzawa step from cur into its ping-pong partner alt
template <class T>
void uzawa_fused(Level& L, Vec<T> cur, Vec<T> f, Vec<T> alt, bool zg, const int* done, hipStream_t s) {
  UZJob<T> J{};
  J.L = Sel<T>::c(L);
  J.xu = cur.u; J.xp = cur.p;
  J.fu = f.u; J.fp = f.p;
  J.ou = alt.u; J.op = alt.p;
  J.tau = T(L.tau);
  J.sigma = T(L.sigma);
  J.done = done;
  launch_uz<T>(J, zg, s);
}

// With acc_u / acc_p (FP32 cycles on the finest level), a last smoothing
// step that is a single fused NE launch adds its result to those FP64
// vectors instead of writing it; the return value then has null pointers.
// With rpart / mpart (FP64 cycles on the finest level), a last smoothing step
// that is a single NE launch on 16 x 8 tiles also forms the residual of its
// result: ||r||^2 per tile into rpart and the pressure mean pieces into
// mpart (k_ne_res); *resd is set then.
template <class T>
Vec<T> cycle_fused(smg_hier* H, int l, Vec<T> x, Vec<T> f, bool zg, const int* done, hipStream_t s,
                   double* acc_u = nullptr, double* acc_p = nullptr, double* rpart = nullptr,
                   double* mpart = nullptr, bool* resd = nullptr) {
  if (l <= H->Lc) {
    if (zg && H->kn && H->dense_on) launch_ccd<T>(dense_job<T>(H, x, f, done), s);
    else coarse_cycle<T>(H, x, f, zg, done, s);
    return x;
  }
  Level& L = H->lv[l];
  const smg_params& prm = H->prm;
  const bool ne = prm.smoother == SMG_SMOOTHER_NE;
  // ping-pong partner: whichever of the level's two buffers does not hold x
  Vec<T> cur = x, alt = (x.u == Sel<T>::t(L).u) ? Sel<T>::x(L) : Sel<T>::t(L);
  bool z = zg;
  if (z && prm.nu_pre == 0) {
    fill_vec<T>(L, cur, s);
    z = false;
  }
  // two steps per launch where the level uses 8 x 8 tiles
  const int tx = H->ne_tx(L.N);
  const bool pair = ne && H->ne2 && tx == 8;
  Level& C = H->lv[l - 1];
  Vec<T> xc = Sel<T>::x(C), fc = Sel<T>::f(C);
  // from a zero iterate with two pre-smoothing steps: the steps, the defect
  // and its restriction in one launch
  const bool fuse_rr = pair && z && prm.nu_pre == 2;
  if (fuse_rr) {
    NERRJob<T> J{};
    J.L = Sel<T>::c(L);
    J.fu = f.u; J.fp = f.p;
    J.ou = alt.u; J.op = alt.p;
    J.cu = fc.u; J.cp = fc.p;
    J.tau = T(L.tau);
    J.done = done;
    launch_ne2rr<T>(J, s);
    std::swap(cur, alt);
    z = false;
  }
  for (int k = 0; k < prm.nu_pre && !fuse_rr;) {
    if (ne) {
      NEJob<T> J{};
      J.L = Sel<T>::c(L);
      J.xu = cur.u; J.xp = cur.p;
      J.fu = f.u; J.fp = f.p;
      J.ou = alt.u; J.op = alt.p;
      J.tau = T(L.tau);
      J.done = done;
      const bool two = pair && k + 1 < prm.nu_pre;
      if (two) launch_ne2<T>(J, z, false, s);
      else launch_ne<T>(J, z, false, tx, s);
      std::swap(cur, alt);
      k += two ? 2 : 1;
    } else {
      uzawa_fused<T>(L, cur, f, alt, z, done, s);
      std::swap(cur, alt);
      ++k;
    }
    z = false;
  }
  if (!fuse_rr) {
    RRJob<T> R{};
    R.L = Sel<T>::c(L);
    R.xu = cur.u; R.xp = cur.p;
    R.fu = f.u; R.fp = f.p;
    R.cu = fc.u; R.cp = fc.p;
    R.done = done;
    launch_resid_restrict<T>(R, s);
  }
  Vec<T> zc = xc;
  for (int g = 0; g < prm.gamma; ++g) {
    zc = cycle_fused<T>(H, l - 1, zc, fc, g == 0, done, s);
  }
  int post = prm.nu_post;
  bool accd = false;
  if (ne && post > 0) {
    NEJob<T> J{};
    J.L = Sel<T>::c(L);
    J.xu = cur.u; J.xp = cur.p;
    J.fu = f.u; J.fp = f.p;
    J.ou = alt.u; J.op = alt.p;
    J.zu = zc.u; J.zp = zc.p;
    J.tau = T(L.tau);
    J.done = done;
    const bool two = pair && post >= 2;
    if (acc_u && !two && post == 1) {
      J.acc_u = acc_u; J.acc_p = acc_p;
      accd = true;
    }
    if (two) launch_ne2<T>(J, false, true, s);
    else launch_ne<T>(J, false, true, tx, s);
    std::swap(cur, alt);
    post -= two ? 2 : 1;
  } else {
    launch_prolong_add<T>(C.N, H->dom, zc.u, zc.p, cur.u, cur.p, done, s);
  }
  for (int k = 0; k < post;) {
    if (ne) {
      NEJob<T> J{};
      J.L = Sel<T>::c(L);
      J.xu = cur.u; J.xp = cur.p;
      J.fu = f.u; J.fp = f.p;
      J.ou = alt.u; J.op = alt.p;
      J.tau = T(L.tau);
      J.done = done;
      const bool two = pair && k + 1 < post;
      if (acc_u && !two && k + 1 == post) {
        J.acc_u = acc_u; J.acc_p = acc_p;
        accd = true;
      }
      bool fused_res = false;
      if constexpr (std::is_same<T, double>::value) {
        if (rpart && !two && k + 1 == post && tx == 16 && ne_res_tiles(L.N) <= NE_RES_MAX_TILES) {
          J.partial = rpart;
          J.mean_partial = mpart;
          launch_ne_res(J, s);
          fused_res = true;
          if (resd) *resd = true;
        }
      }
      if (fused_res) {
      } else if (two) launch_ne2<T>(J, false, false, s);
      else launch_ne<T>(J, false, false, tx, s);
      std::swap(cur, alt);
      k += two ? 2 : 1;
    } else {
      uzawa_fused<T>(L, cur, f, alt, false, done, s);
      std::swap(cur, alt);
      ++k;
    }
  }
  if (accd) return Vec<T>{nullptr, nullptr};
  return cur;
}

// iterate on the finest level with the result in x.  Returns TOP_ACC when
// the result was added to acc_u / acc_p instead, TOP_RES when the last
// launch also wrote the residual partials to rpart / mpart.
enum { TOP_ACC = 1, TOP_RES = 2 };
template <class T>
int top_cycle(smg_hier* H, Vec<T> x, Vec<T> f, bool zg, const int* done, hipStream_t s,
              double* acc_u = nullptr, double* acc_p = nullptr, double* rpart = nullptr,
              double* mpart = nullptr) {
  if (!H->fused) {
    if (zg) fill_vec<T>(H->lv[H->L], x, s);
    cycle_rec<T>(H, H->L, x, f, false, done, s);
    return 0;
  }
  bool resd = false;
  Vec<T> r = cycle_fused<T>(H, H->L, x, f, zg, done, s, acc_u, acc_p, rpart, mpart, &resd);
  if (!r.u) return TOP_ACC;
  if (r.u != x.u) {
    // the partials were formed for the other buffer's values, which are the
    // same numbers: the copy does not change them
    copy_vec<T>(H->lv[H->L], x, r, done, s);
  }
  return resd ? TOP_RES : 0;
}

void project_mean(smg_hier* H, int l, double* p, const int* done, hipStream_t s) {
  launch_project_mean(H->lv[l].N, H->dom, p, H->red, done, s);
}

// residual of the finest level: optional write (FP64, or rounded to FP32
// with r32u / r32p), partial sums in L.partial
void top_residual(Level& L, const double* xu, const double* xp, const double* fu, const double* fp,
                  double* ru, double* rp, const int* done, hipStream_t s, float* r32u = nullptr,
                  float* r32p = nullptr) {
  StencilJob<double> R = job_of<double>(L);
  R.in_u = xu; R.in_p = xp;
  R.rhs_u = fu; R.rhs_p = fp;
  R.out_u = ru; R.out_p = rp;
  R.out32_u = r32u; R.out32_p = r32p;
  R.partial = L.partial;
  R.done = done;
  launch_stencil<double>(R, ROWS_UP, s);
}

// end of an iterate: residual norm and pressure-mean pieces of x in one pass,
// mean projection, convergence test (the residual is blind to the mean)
void finish_iter(smg_hier* H, float* r32u, float* r32p, const int* done, hipStream_t s) {
  Level& T = H->lv[H->L];
  StencilJob<double> R = job_of<double>(T);
  R.in_u = T.x.u; R.in_p = T.x.p;
  R.rhs_u = T.f.u; R.rhs_p = T.f.p;
  R.out32_u = r32u; R.out32_p = r32p;
  R.partial = T.partial;
  R.mean_partial = H->mpart;
  R.done = done;
  launch_stencil<double>(R, ROWS_UP, s);
  launch_project_check(H->mpart, T.partial, T.ntiles, T.N, H->dom, T.x.p, H->st, H->hist, s);
}

// one FP64 iterate of the solve loop on the internal finest-level vectors
void enqueue_iter64(smg_hier* H, hipStream_t s) {
  Level& T = H->lv[H->L];
  const int* done = &H->st->done;
  // the last smoothing step forms the residual pieces where it can (k_ne_res)
  if (top_cycle<double>(H, T.x, T.f, false, done, s, nullptr, nullptr, T.partial, H->mpart) & TOP_RES)
    launch_project_check(H->mpart, T.partial, ne_res_tiles(T.N), T.N, H->dom, T.x.p, H->st, H->hist, s);
  else
    finish_iter(H, nullptr, nullptr, done, s);
}

// one refinement step: d = cycle_fp32(r), x += d, r = F - calA x, project, test
// (the FP32 right-hand side, the FP64 residual rounded, is written by the
// residual pass of the solve's set-up or of the previous step; the cycle's
// last smoothing step adds its result to x where it is a single NE launch)
void enqueue_iter_mixed(smg_hier* H, hipStream_t s) {
  Level& T = H->lv[H->L];
  const int* done = &H->st->done;
  if (!(top_cycle<float>(H, T.x32, T.f32, true, done, s, T.x.u, T.x.p) & TOP_ACC))
    launch_axpy_f32(T.x.u, T.x32.u, T.n_u + T.n_p, done, s);
  finish_iter(H, T.f32.u, T.f32.p, done, s);
}

// forget the captured iterates of one hierarchy (their launches carry values
// that changed)
void drop_solve_graphs(smg_hier* H) {
  for (hipGraphExec_t* g : {&H->g64, &H->g32, &H->g64r, &H->g32r, &H->gerr}) {
    if (*g) (void)hipGraphExecDestroy(*g);
    *g = nullptr;
  }
  ++H->gen;
}

// The dense coarse map applies the coarse levels' linear map as one matrix,
// whose FP64 rounding leaves a relative residual floor of about 1e-12 in the
// worst case measured (union-jack grid, large beta), against a few 1e-13 for
// the level-by-level kernel.  Solves asking for less than ten times that
// floor use the kernel; a change of mode drops the captured iterates.
constexpr double KD_RTOL_MIN = 1e-11;
void dense_mode(smg_hier* H, double rtol) {
  const bool on = !(rtol > 0 && rtol < KD_RTOL_MIN);
  if (on == H->dense_on) return;
  H->dense_on = on;
  drop_solve_graphs(H);
}

// grow the history buffer to hold maxit iterates; the captured iterates
// write the old buffer, so they are dropped
int reserve_history(smg_hier* H, int maxit) {
  if (maxit <= H->hist_cap) return SMG_OK;
  double* nh = H->alloc<double>(maxit);
  if (!nh) return fail(SMG_ENOMEM, "history buffer");
  drop_solve_graphs(H);
  H->hist = nh;
  H->hist_cap = maxit;
  return SMG_OK;
}

// `reps` iterates enqueued by fn, captured as one graph
int capture(smg_hier* H, void (*fn)(smg_hier*, hipStream_t), hipGraphExec_t* out, int reps = 1) {
  hipGraph_t g = nullptr;
  HIPCHK(hipStreamBeginCapture(H->cap_stream, hipStreamCaptureModeThreadLocal));
  for (int r = 0; r < reps; ++r) fn(H, H->cap_stream);
  HIPCHK(hipStreamEndCapture(H->cap_stream, &g));
  hipError_t e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return fail(SMG_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
  return SMG_OK;
}

int check_level(smg_hier* H, int level) {
  if (!H) return fail(SMG_EINVAL, "null handle");
  if (level < 0 || level > H->L) return fail(SMG_EINVAL, "level %d outside 0..%d", level, H->L);
  HIPCHK(hipSetDevice(H->device));
  return SMG_OK;
}

int launch_status(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(SMG_EHIP, "%s: kernel launch failed: %s", what, hipGetErrorString(e));
  return SMG_OK;
}

// c iterates: graphs of ITER_GRAPH_REPS iterates while they fit, then graphs
// of one (rep may be null).  Kernels within a graph follow each other without
// a gap; each graph launch starts after a bubble of several microseconds.
hipError_t launch_iters(hipGraphExec_t one, hipGraphExec_t rep, int c, hipStream_t s) {
  int q = 0;
  if (rep)
    for (; q + ITER_GRAPH_REPS <= c; q += ITER_GRAPH_REPS) {
      const hipError_t e = hipGraphLaunch(rep, s);
      if (e != hipSuccess) return e;
    }
  for (; q < c; ++q) {
    const hipError_t e = hipGraphLaunch(one, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// the solve loop shared by the FP64 and the mixed-precision variants
int run_solve(smg_hier* H, bool mixed, const double* fu, const double* gp, double rtol, int maxit,
              double* u, double* p, int* iters, double* relres, double* history, hipStream_t s) {
  if (!fu || !gp || !u || !p) return fail(SMG_EINVAL, "null vector");
  if (!(rtol >= 0) || maxit < 0) return fail(SMG_EINVAL, "bad rtol / maxit");
  HIPCHK(hipSetDevice(H->device));
  Level& T = H->lv[H->L];
  dense_mode(H, rtol);
  {
    int rc = reserve_history(H, maxit);
    if (rc) return rc;
  }
  hipGraphExec_t* gexec = mixed ? &H->g32 : &H->g64;
  hipGraphExec_t* grep = mixed ? &H->g32r : &H->g64r;
  if (!*gexec) {
    int rc = capture(H, mixed ? enqueue_iter_mixed : enqueue_iter64, gexec);
    if (rc) return rc;
  }
  if (!*grep) {
    int rc = capture(H, mixed ? enqueue_iter_mixed : enqueue_iter64, grep, ITER_GRAPH_REPS);
    if (rc) return rc;
  }
  const size_t bu = sizeof(double) * T.n_u, bp = sizeof(double) * T.n_p;
  HIPCHK(hipMemcpyAsync(T.f.u, fu, bu, hipMemcpyDeviceToDevice, s));
  HIPCHK(hipMemcpyAsync(T.f.p, gp, bp, hipMemcpyDeviceToDevice, s));
  HIPCHK(hipMemcpyAsync(T.x.u, u, bu, hipMemcpyDeviceToDevice, s));
  HIPCHK(hipMemcpyAsync(T.x.p, p, bp, hipMemcpyDeviceToDevice, s));
  {
    // boundary entries of the caller's guess are ignored: x.u <- 0 + 1 * (x.u - 0)
    // on interior rows and 0 on boundary rows (reads only the own entry)
    StencilJob<double> Z = job_of<double>(T);
    Z.rhs_u = T.x.u;
    Z.out_u = T.x.u;
    launch_stencil<double>(Z, ROWS_U, s);
  }
  project_mean(H, H->L, T.x.p, nullptr, s);
  SolveState init{};
  init.maxit = maxit;
  init.tol2 = rtol * rtol;
  *H->st_host = init;
  HIPCHK(hipMemcpyAsync(H->st, H->st_host, sizeof(SolveState), hipMemcpyHostToDevice, s));
  launch_dot(T.N, H->dom, 0, T.f.u, T.f.u, H->red, H->fdots, s);
  launch_dot(T.N, H->dom, 1, T.f.p, T.f.p, H->red, H->fdots + 1, s);
  top_residual(T, T.x.u, T.x.p, T.f.u, T.f.p, nullptr, nullptr, nullptr, s, mixed ? T.f32.u : nullptr,
               mixed ? T.f32.p : nullptr);
  launch_init_state(T.partial, T.ntiles, H->fdots, H->st, s);
  launch_psum(T.N, H->dom, T.f.p, H->red, H->enorm, s);
  int rc = launch_status("solve init");
  if (rc) return rc;
  double psum[2];
  HIPCHK(hipMemcpyAsync(H->st_host, H->st, sizeof(SolveState), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(psum, H->enorm, sizeof(psum), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  const bool incompatible = std::fabs(psum[0]) > SMG_COMPAT_TOL * psum[1];
  double rel_prev = H->st_host->relres;
  int launched = 0, chunk = 2;
  while (!H->st_host->done && launched < maxit) {
    const int k = std::min(chunk, maxit - launched);
    HIPCHK(launch_iters(*gexec, *grep, k, s));
    launched += k;
    HIPCHK(hipMemcpyAsync(H->st_host, H->st, sizeof(SolveState), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const double rel = H->st_host->relres;
    // predict the remaining iterates from the observed rate
    double q = (rel > 0 && rel_prev > 0 && rel < rel_prev) ? std::pow(rel / rel_prev, 1.0 / k) : 0.9;
    q = std::min(std::max(q, 1e-3), 0.99);
    // rtol = 0 asks for maxit iterates: launch the rest without host checks
    const double need = rtol > 0 ? (rel > rtol ? std::log(rtol / rel) / std::log(q) : 1.0)
                                 : (double)(maxit - launched);
    chunk = (int)std::min(64.0, std::max(1.0, std::ceil(need)));
    rel_prev = rel;
  }
  // a solve with maxit = 0 never runs the loop: report the initial state
  if (!H->st_host->done && maxit == 0) H->st_host->done = (H->st_host->relres <= rtol) ? 1 : 4;
  HIPCHK(hipMemcpyAsync(u, T.x.u, bu, hipMemcpyDeviceToDevice, s));
  HIPCHK(hipMemcpyAsync(p, T.x.p, bp, hipMemcpyDeviceToDevice, s));
  const int it = H->st_host->iters;
  if (history && it > 0)
    HIPCHK(hipMemcpyAsync(history, H->hist, sizeof(double) * it, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (iters) *iters = it;
  if (relres) *relres = H->st_host->relres;
  if (H->st_host->done != 1 && incompatible)
    return fail(SMG_EINCOMPAT, "no convergence: the pressure data are not compatible (1^T g_p = %g, sum |g_p| = %g)",
                psum[0], psum[1]);
  switch (H->st_host->done) {
    case 1: return SMG_OK;
    case 2: return fail(SMG_DIVERGED, "diverged after %d iterates (relres %g)", it, H->st_host->relres);
    case 3: return fail(SMG_ENONFINITE, "non-finite residual after %d iterates", it);
    default: return fail(SMG_NOCONV, "no convergence in %d iterates (relres %g)", it, H->st_host->relres);
  }
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================

extern "C" {

int smg_default_params(smg_params* prm) {
  if (!prm) return fail(SMG_EINVAL, "null params");
  prm->smoother = SMG_SMOOTHER_NE;
  prm->tau = 0.35;
  prm->sigma = 0.8;
  prm->nu_pre = 2;
  prm->nu_post = 2;
  prm->gamma = 1;
  prm->n0 = 2;
  prm->unfused = 0;
  prm->fuse_depth = 0;
  prm->coarse_max_n = 0;
  prm->tile_x = 0;
  prm->domain = SMG_DOM_SQUARE;
  return SMG_OK;
}

const char* smg_last_error(void) { return host::last_error(); }

int smg_setup(int N, double beta, const smg_params* prm_in, smg_t* out) {
  if (!out) return fail(SMG_EINVAL, "null output handle");
  *out = nullptr;
  smg_params prm;
  if (prm_in) prm = *prm_in; else smg_default_params(&prm);
  int L = 0;
  {
    int rc = host::check_params(N, beta, prm, &L);
    if (rc) return rc;
  }
  smg_hier* H = new smg_hier();
  H->prm = prm;
  H->beta = beta;
  H->fused = prm.unfused == 0;
  H->ne2 = prm.fuse_depth != 1;
  H->dom = prm.domain;
  H->tile_x = prm.tile_x;
  H->L = L;
  if (hipGetDevice(&H->device) != hipSuccess) { delete H; return fail(SMG_EHIP, "hipGetDevice"); }
  H->lv.resize(L + 1);
  int red_need = 8;
  for (int l = 0; l <= L; ++l) {
    Level& Lv = H->lv[l];
    Lv.N = prm.n0 << l;
    Lv.tau = prm.tau;
    Lv.sigma = prm.sigma;
    const int64_t M = 2 * Lv.N + 1;
    Lv.n_u = 2 * M * M;
    Lv.n_p = (int64_t)(Lv.N + 1) * (Lv.N + 1);
    host::make_coef(Lv.N, H->dom, beta, Lv.c64, Lv.c32);
    const int64_t nv = Lv.n_u + Lv.n_p;
    double* b64 = H->alloc<double>(3 * nv);
    float* b32 = H->alloc<float>(3 * nv);
    double* s64 = H->alloc<double>(Lv.n_p);
    float* s32 = H->alloc<float>(Lv.n_p);
    Lv.ntiles = stencil_tiles(Lv.N);
    // sized for the smallest tile shape, so that batched launches with any
    // tile shape fit
    Lv.partial = H->alloc<double>(std::max(Lv.ntiles, stencil_tiles_shape(Lv.N, 8, 8)));
    if (!b64 || !b32 || !s64 || !s32 || !Lv.partial) { delete H; return fail(SMG_ENOMEM, "level %d buffers", l); }
    Vec<double>* v64[3] = {&Lv.x, &Lv.f, &Lv.t};
    Vec<float>* v32[3] = {&Lv.x32, &Lv.f32, &Lv.t32};
    for (int k = 0; k < 3; ++k) {
      v64[k]->u = b64 + k * nv;
      v64[k]->p = v64[k]->u + Lv.n_u;
      v32[k]->u = b32 + k * nv;
      v32[k]->p = v32[k]->u + Lv.n_u;
    }
    Lv.c64.sinv = s64;
    Lv.c32.sinv = s32;
    red_need = std::max(red_need, 2 * mean_blocks(Lv.N));
    red_need = std::max(red_need, dot_blocks(Lv.N, 0));
    red_need = std::max(red_need, dot_blocks(Lv.N, 1));
    red_need = std::max(red_need, enorm_scratch(Lv.N));
  }
  H->red = H->alloc<double>(red_need);
  H->red_cap = red_need;
  H->fdots = H->alloc<double>(2);
  H->enorm = H->alloc<double>(4);
  H->st = H->alloc<SolveState>(1);
  H->hist_cap = 1000;
  H->hist = H->alloc<double>(H->hist_cap);
  if (!H->red || !H->fdots || !H->enorm || !H->st || !H->hist) { delete H; return fail(SMG_ENOMEM, "scratch"); }
  if (hipHostMalloc((void**)&H->st_host, sizeof(SolveState), hipHostMallocDefault) != hipSuccess) {
    H->st_host = nullptr;
    delete H;
    return fail(SMG_ENOMEM, "pinned state");
  }
  if (hipStreamCreateWithFlags(&H->cap_stream, hipStreamNonBlocking) != hipSuccess) {
    delete H;
    return fail(SMG_EHIP, "stream");
  }
  hipStream_t s = H->cap_stream;
  for (int l = 0; l <= L; ++l) {
    Level& Lv = H->lv[l];
    launch_shat_inv<double>(Lv.N, H->dom, Lv.c64.bh2, Lv.c64.adinv, const_cast<double*>(Lv.c64.sinv), s);
    launch_shat_inv<float>(Lv.N, H->dom, Lv.c64.bh2, Lv.c32.adinv, const_cast<float*>(Lv.c32.sinv), s);
    for (int k = 0; k < 1; ++k) {
      launch_fill(Lv.x.u, 3 * (Lv.n_u + Lv.n_p), 0.0, s);
      launch_fill_f32(Lv.x32.u, 3 * (Lv.n_u + Lv.n_p), 0.0f, s);
    }
  }
  std::vector<double> inv;
  int rc = host::coarse_inverse(prm.n0, H->lv[0].c64, inv);
  if (rc) { delete H; return rc; }
  H->nc = (int)std::sqrt((double)inv.size());
  H->cinv = H->alloc<double>((int64_t)inv.size());
  if (!H->cinv) { delete H; return fail(SMG_ENOMEM, "coarse inverse"); }
  if (hipMemcpyAsync(H->cinv, inv.data(), inv.size() * sizeof(double), hipMemcpyHostToDevice, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess || hipGetLastError() != hipSuccess) {
    delete H;
    return fail(SMG_EHIP, "setup upload / kernels failed");
  }
  // levels handled by the single-workgroup kernel: N <= cmax and all three
  // vectors of every such level in FP64 within the LDS of one workgroup
  {
    int lds_max = 0, lds_optin = 0;
    (void)hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, H->device);
    (void)hipDeviceGetAttribute(&lds_optin, hipDeviceAttributeSharedMemPerBlockOptin, H->device);
    const size_t limit = (size_t)std::max(lds_max, lds_optin);
    H->Lc = -1;
    // largest grid done by the single-workgroup kernel (default 8 squares per
    // side: from N = 16 on, the grid kernels with two smoothing steps per
    // launch finish a level sooner than one workgroup does)
    const int cmax = prm.coarse_max_n > 0 ? prm.coarse_max_n : 8;
    for (int l = 0; l <= L && l <= CC_MAX_LEVELS; ++l) {
      if ((prm.n0 << l) > cmax) break;
      const size_t need = coarse_cycle_lds(prm.n0, l, sizeof(double));
      // the job, the op list and level 0's inverse staged in static LDS come
      // on top of the dynamic part
      if (need + sizeof(CoarseJob<double>) + CC_STATIC_LDS > limit) break;
      if (need > 65536 && (coarse_cycle_allow_lds<double>(need) != 0 ||
                           coarse_cycle_allow_lds<float>(coarse_cycle_lds(prm.n0, l, sizeof(float))) != 0)) {
        (void)hipGetLastError();
        break;
      }
      H->Lc = l;
    }
    if (H->Lc < 0) H->Lc = 0;   // level 0 alone always fits: its exact solve
    {
      std::vector<int> ops;
      cc_emit(prm, H->Lc, true, ops);
      H->cc_nops = (int)ops.size();
      H->cc_ops = H->alloc<int>(H->cc_nops);
      if (!H->cc_ops) { delete H; return fail(SMG_ENOMEM, "op list"); }
      if (hipMemcpy(H->cc_ops, ops.data(), ops.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess) {
        delete H;
        return fail(SMG_EHIP, "op list upload");
      }
    }
    H->mpart = H->alloc<double>(2 * std::max(H->lv[L].ntiles, stencil_tiles_shape(H->lv[L].N, 8, 8)));
    if (!H->mpart) { delete H; return fail(SMG_ENOMEM, "mean partials"); }
    form_dense_maps(H, s);
  }
  *out = H;
  return SMG_OK;
}

int smg_destroy(smg_t h) {
  if (!h) return SMG_OK;
  HIPCHK(hipSetDevice(h->device));
  HIPCHK(hipDeviceSynchronize());
  delete h;
  return SMG_OK;
}

int smg_num_levels(smg_t h) { return h ? h->L + 1 : fail(SMG_EINVAL, "null handle"); }

int smg_level_size(smg_t h, int level, int* N, int64_t* nvel, int64_t* npres) {
  if (!h) return fail(SMG_EINVAL, "null handle");
  if (level < 0 || level > h->L) return fail(SMG_EINVAL, "level %d outside 0..%d", level, h->L);
  const Level& L = h->lv[level];
  if (N) *N = L.N;
  if (nvel) *nvel = L.n_u;
  if (npres) *npres = L.n_p;
  return SMG_OK;
}

int smg_load(smg_t h, int level, const double* f_nodal, const double* g_nodal, double* fu,
             double* gp, smg_stream_t sv) {
  int rc = check_level(h, level);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)sv;
  const int N = h->lv[level].N;
  if (fu) {
    if (!f_nodal) return fail(SMG_EINVAL, "null f_nodal");
    launch_mass_u(N, h->dom, 2, f_nodal, fu, s);
  }
  if (gp) {
    if (!g_nodal) return fail(SMG_EINVAL, "null g_nodal");
    launch_mass_p(N, h->dom, g_nodal, gp, s);
  }
  return launch_status("smg_load");
}

int smg_mass(smg_t h, int level, int all_nodes, const double* u, double* y, smg_stream_t sv) {
  int rc = check_level(h, level);
  if (rc) return rc;
  if (!u || !y) return fail(SMG_EINVAL, "null vector");
  launch_mass_u(h->lv[level].N, h->dom, all_nodes ? 1 : 0, u, y, (hipStream_t)sv);
  return launch_status("smg_mass");
}

int smg_pressure_mass(smg_t h, int level, const double* g, double* gp, smg_stream_t sv) {
  int rc = check_level(h, level);
  if (rc) return rc;
  if (!g || !gp) return fail(SMG_EINVAL, "null vector");
  launch_mass_p(h->lv[level].N, h->dom, g, gp, (hipStream_t)sv);
  return launch_status("smg_pressure_mass");
}

int smg_apply(smg_t h, int level, const double* u, const double* p, double* yu, double* yp,
              smg_stream_t sv) {
  int rc = check_level(h, level);
  if (rc) return rc;
  if (!u || !p || !yu || !yp) return fail(SMG_EINVAL, "null vector");
  StencilJob<double> J = job_of<double>(h->lv[level]);
  J.in_u = u; J.in_p = p;
  J.w_u = J.w_p = -1.0;
  J.out_u = yu; J.out_p = yp;
  launch_stencil<double>(J, ROWS_UP, (hipStream_t)sv);
  return launch_status("smg_apply");
}

int smg_residual(smg_t h, int level, const double* fu, const double* gp, const double* u,
                 const double* p, double* ru, double* rp, double* norm2, smg_stream_t sv) {
  int rc = check_level(h, level);
  if (rc) return rc;
  if (!fu || !gp || !u || !p || !ru || !rp) return fail(SMG_EINVAL, "null vector");
  hipStream_t s = (hipStream_t)sv;
  Level& L = h->lv[level];
  top_residual(L, u, p, fu, gp, ru, rp, nullptr, s);
  if (norm2) launch_reduce(L.partial, L.ntiles, norm2, s);
  return launch_status("smg_residual");
}

int smg_smooth(smg_t h, int level, int nsteps, const double* fu, const double* gp, double* u,
               double* p, smg_stream_t sv) {
  int rc = check_level(h, level);
  if (rc) return rc;
  if (!fu || !gp || !u || !p) return fail(SMG_EINVAL, "null vector");
  if (nsteps < 0) return fail(SMG_EINVAL, "nsteps < 0");
  Level& L = h->lv[level];
  Vec<double> x{u, p}, f{const_cast<double*>(fu), const_cast<double*>(gp)};
  for (int k = 0; k < nsteps; ++k) smooth_step<double>(h->prm, L, x, f, L.t, false, nullptr, (hipStream_t)sv);
  return launch_status("smg_smooth");
}

int smg_restrict(smg_t h, int fine_level, const double* ru, const double* rp, double* rcu,
                 double* rcp, smg_stream_t sv) {
  int rc = check_level(h, fine_level);
  if (rc) return rc;
  if (fine_level < 1) return fail(SMG_EINVAL, "restriction needs fine_level >= 1");
  if (!ru || !rp || !rcu || !rcp) return fail(SMG_EINVAL, "null vector");
  launch_restrict<double>(h->lv[fine_level - 1].N, h->dom, ru, rp, rcu, rcp, nullptr, nullptr, nullptr,
                          (hipStream_t)sv);
  return launch_status("smg_restrict");
}

int smg_prolong_add(smg_t h, int fine_level, const double* zcu, const double* zcp, double* u,
                    double* p, smg_stream_t sv) {
  int rc = check_level(h, fine_level);
  if (rc) return rc;
  if (fine_level < 1) return fail(SMG_EINVAL, "prolongation needs fine_level >= 1");
  if (!zcu || !zcp || !u || !p) return fail(SMG_EINVAL, "null vector");
  launch_prolong_add<double>(h->lv[fine_level - 1].N, h->dom, zcu, zcp, u, p, nullptr, (hipStream_t)sv);
  return launch_status("smg_prolong_add");
}

int smg_coarse_solve(smg_t h, const double* ru, const double* rp, double* zu, double* zp,
                     smg_stream_t sv) {
  int rc = check_level(h, 0);
  if (rc) return rc;
  if (!ru || !rp || !zu || !zp) return fail(SMG_EINVAL, "null vector");
  launch_coarse_solve<double>(h->lv[0].N, h->dom, h->nc, h->cinv, ru, rp, zu, zp, nullptr, (hipStream_t)sv);
  return launch_status("smg_coarse_solve");
}

int smg_project_mean(smg_t h, int level, double* p, smg_stream_t sv) {
  int rc = check_level(h, level);
  if (rc) return rc;
  if (!p) return fail(SMG_EINVAL, "null vector");
  project_mean(h, level, p, nullptr, (hipStream_t)sv);
  return launch_status("smg_project_mean");
}

int smg_project_dual(smg_t h, int level, double* v, smg_stream_t sv) {
  int rc = check_level(h, level);
  if (rc) return rc;
  if (!v) return fail(SMG_EINVAL, "null vector");
  launch_project_dual(h->lv[level].N, h->dom, v, h->red, (hipStream_t)sv);
  return launch_status("smg_project_dual");
}

int smg_cycle(smg_t h, const double* fu, const double* gp, double* u, double* p, smg_stream_t sv) {
  int rc = check_level(h, 0);
  if (rc) return rc;
  if (!fu || !gp || !u || !p) return fail(SMG_EINVAL, "null vector");
  hipStream_t s = (hipStream_t)sv;
  Vec<double> x{u, p}, f{const_cast<double*>(fu), const_cast<double*>(gp)};
  top_cycle<double>(h, x, f, false, nullptr, s);
  project_mean(h, h->L, p, nullptr, s);
  return launch_status("smg_cycle");
}

int smg_cycle_f32(smg_t h, const float* fu, const float* gp, float* u, float* p, smg_stream_t sv) {
  int rc = check_level(h, 0);
  if (rc) return rc;
  if (!fu || !gp || !u || !p) return fail(SMG_EINVAL, "null vector");
  Vec<float> x{u, p}, f{const_cast<float*>(fu), const_cast<float*>(gp)};
  top_cycle<float>(h, x, f, false, nullptr, (hipStream_t)sv);
  return launch_status("smg_cycle_f32");
}

static void enqueue_error_norm(smg_hier* h, const double* u, const double* p, const double* us, const double* ps,
                               hipStream_t s) {
  Level& T = h->lv[h->L];
  double ah[4];
  for (int k = 0; k < 4; ++k) ah[k] = 1.0 / T.c64.adinv[k];
  launch_error_norm(T.N, h->dom, T.c64.bh2, ah, T.c64.sinv, u, p, us, ps, h->red, h->enorm, s);
}

// One iterate of the protocol, its projection and the error measure, as one
// graph (a W-cycle on the unfused path is thousands of launches); captured
// once per set of vectors.
static int protocol_graph(smg_hier* H, const double* fu, const double* gp, const double* us, const double* ps,
                          double* u, double* p) {
  const void* key[6] = {fu, gp, us, ps, u, p};
  if (H->gerr && std::equal(key, key + 6, H->gerr_key)) return SMG_OK;
  if (H->gerr) (void)hipGraphExecDestroy(H->gerr);
  H->gerr = nullptr;
  hipGraph_t g = nullptr;
  hipStream_t cs = H->cap_stream;
  HIPCHK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
  Vec<double> x{u, p}, f{const_cast<double*>(fu), const_cast<double*>(gp)};
  top_cycle<double>(H, x, f, false, nullptr, cs);
  project_mean(H, H->L, p, nullptr, cs);
  enqueue_error_norm(H, u, p, us, ps, cs);
  HIPCHK(hipStreamEndCapture(cs, &g));
  hipError_t e = hipGraphInstantiate(&H->gerr, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    H->gerr = nullptr;
    return fail(SMG_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
  }
  std::copy(key, key + 6, H->gerr_key);
  return SMG_OK;
}

int smg_error_norm(smg_t h, const double* u, const double* p, const double* us, const double* ps, double* out,
                   smg_stream_t sv) {
  if (!h) return fail(SMG_EINVAL, "null handle");
  if (!u || !p || !us || !ps || !out) return fail(SMG_EINVAL, "null vector");
  hipStream_t s = (hipStream_t)sv;
  enqueue_error_norm(h, u, p, us, ps, s);
  double v[4];
  HIPCHK(hipMemcpyAsync(v, h->enorm, sizeof(v), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  *out = std::sqrt(std::max(v[2] + v[3], 0.0));
  return SMG_OK;
}

int smg_solve_error(smg_t h, const double* fu, const double* gp, const double* us, const double* ps, double eps,
                    int maxit, double* u, double* p, int* iters, double* rate, smg_stream_t sv) {
  if (!h) return fail(SMG_EINVAL, "null handle");
  if (!fu || !gp || !us || !ps || !u || !p) return fail(SMG_EINVAL, "null vector");
  if (!(eps > 0) || maxit < 1) return fail(SMG_EINVAL, "eps must be > 0 and maxit >= 1");
  double e0 = 0.0, e = 0.0;
  int rc = smg_error_norm(h, u, p, us, ps, &e0, sv);
  if (rc) return rc;
  if (iters) *iters = 0;
  if (rate) *rate = 0.0;
  if (e0 == 0.0) return SMG_OK;
  if ((rc = protocol_graph(h, fu, gp, us, ps, u, p)) != SMG_OK) return rc;
  hipStream_t s = (hipStream_t)sv;
  double v[4];
  for (int n = 1; n <= maxit; ++n) {
    HIPCHK(hipGraphLaunch(h->gerr, s));
    HIPCHK(hipMemcpyAsync(v, h->enorm, sizeof(v), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    e = std::sqrt(std::max(v[2] + v[3], 0.0));
    if (iters) *iters = n;
    if (!std::isfinite(e)) {
      if (rate) *rate = INFINITY;
      return SMG_ENONFINITE;
    }
    if (rate) *rate = std::pow(e / e0, 1.0 / n);
    if (e > 1e6 * e0) return SMG_DIVERGED;
    if (e <= eps * e0) return SMG_OK;
  }
  return SMG_NOCONV;
}

int smg_solve(smg_t h, const double* fu, const double* gp, double rtol, int maxit, double* u,
              double* p, int* iters, double* relres, double* history, smg_stream_t sv) {
  if (!h) return fail(SMG_EINVAL, "null handle");
  return run_solve(h, false, fu, gp, rtol, maxit, u, p, iters, relres, history, (hipStream_t)sv);
}

int smg_set_damping(smg_t h, int level, double tau, double sigma) {
  if (!h) return fail(SMG_EINVAL, "null handle");
  if (!(tau > 0) || !(sigma > 0) || !std::isfinite(tau) || !std::isfinite(sigma))
    return fail(SMG_EINVAL, "tau and sigma must be finite and > 0");
  if (level < -1 || level > h->L) return fail(SMG_EINVAL, "level %d not in -1..%d", level, h->L);
  for (int l = 0; l <= h->L; ++l)
    if (level < 0 || l == level) {
      h->lv[l].tau = tau;
      h->lv[l].sigma = sigma;
    }
  // the dense coarse maps carry the damping of levels 0..Lc
  if (h->kn && (level < 0 || level <= h->Lc)) {
    HIPCHK(hipSetDevice(h->device));
    form_dense_maps(h, h->cap_stream);
  }
  // captured iterates carry the old values in their launch arguments (and
  // so do the plans of a batch that holds this hierarchy: the generation
  // tells it)
  drop_solve_graphs(h);
  return SMG_OK;
}

int smg_get_damping(smg_t h, int level, double* tau, double* sigma) {
  int rc = check_level(h, level);
  if (rc) return rc;
  if (!tau || !sigma) return fail(SMG_EINVAL, "null output");
  *tau = h->lv[level].tau;
  *sigma = h->lv[level].sigma;
  return SMG_OK;
}

// Right-hand side of one implicit Euler step in the finest level's t buffer:
// (M_full f + beta M u, M_P g); the solve copies it to f before t is used.
static void implicit_rhs(smg_hier* H, const double* f_nodal, const double* g_nodal, const double* u,
                         hipStream_t s) {
  Level& T = H->lv[H->L];
  if (f_nodal) launch_mass_u(T.N, H->dom, 2, f_nodal, T.t.u, s);
  else launch_fill(T.t.u, T.n_u, 0.0, s);
  launch_mass_u_acc(T.N, H->dom, 0, u, H->beta, T.t.u, s);
  if (g_nodal) launch_mass_p(T.N, H->dom, g_nodal, T.t.p, s);
  else launch_fill(T.t.p, T.n_p, 0.0, s);
}

// The right-hand side is built in the finest level's scratch vector t; both
// solves copy it into f before the mixed one reuses t for its FP64 residual.
static int implicit_step(smg_t h, bool mixed, const double* f_nodal, const double* g_nodal, double rtol,
                         int maxit, double* u, double* p, int* iters, double* relres, smg_stream_t sv) {
  if (!h) return fail(SMG_EINVAL, "null handle");
  if (!u || !p) return fail(SMG_EINVAL, "null vector");
  HIPCHK(hipSetDevice(h->device));
  hipStream_t s = (hipStream_t)sv;
  implicit_rhs(h, f_nodal, g_nodal, u, s);
  Level& T = h->lv[h->L];
  return run_solve(h, mixed, T.t.u, T.t.p, rtol, maxit, u, p, iters, relres, nullptr, s);
}

int smg_implicit_step(smg_t h, const double* f_nodal, const double* g_nodal, double rtol, int maxit,
                      double* u, double* p, int* iters, double* relres, smg_stream_t sv) {
  return implicit_step(h, false, f_nodal, g_nodal, rtol, maxit, u, p, iters, relres, sv);
}

int smg_implicit_step_mixed(smg_t h, const double* f_nodal, const double* g_nodal, double rtol, int maxit,
                            double* u, double* p, int* iters, double* relres, smg_stream_t sv) {
  return implicit_step(h, true, f_nodal, g_nodal, rtol, maxit, u, p, iters, relres, sv);
}

int smg_solve_mixed(smg_t h, const double* fu, const double* gp, double rtol, int maxit,
                    double* u, double* p, int* iters, double* relres, double* history,
                    smg_stream_t sv) {
  if (!h) return fail(SMG_EINVAL, "null handle");
  return run_solve(h, true, fu, gp, rtol, maxit, u, p, iters, relres, history, (hipStream_t)sv);
}

int smg_dot(smg_t h, int level, int which, const double* a, const double* b, double* out,
            smg_stream_t sv) {
  int rc = check_level(h, level);
  if (rc) return rc;
  if (!a || !b || !out) return fail(SMG_EINVAL, "null vector");
  if (which != 0 && which != 1) return fail(SMG_EINVAL, "which must be 0 or 1");
  launch_dot(h->lv[level].N, h->dom, which, a, b, h->red, out, (hipStream_t)sv);
  return launch_status("smg_dot");
}

int smg_time_kernel(smg_t h, int which, int reps, double* avg_ms, smg_stream_t sv) {
  int rc = check_level(h, 0);
  if (rc) return rc;
  if (!avg_ms || reps < 1 || which < 0 || which > 3) return fail(SMG_EINVAL, "bad arguments");
  hipStream_t s = (hipStream_t)sv;
  Level& T = h->lv[h->L];
  StencilJob<double> J = job_of<double>(T);
  J.in_u = T.x.u; J.in_p = T.x.p;
  J.out_u = T.t.u; J.out_p = T.t.p;
  if (which == 0 || which == 2) { J.rhs_u = T.f.u; J.rhs_p = T.f.p; }
  if (which == 0) J.diag_u = J.diag_p = 1;
  if (which == 1) {
    J.in_u = T.t.u; J.in_p = T.t.p;
    J.base_u = T.x.u; J.base_p = T.x.p;
    J.out_u = T.x.u; J.out_p = T.x.p;
    J.w_u = J.w_p = -T.tau;
    J.diag_u = J.diag_p = 1;
  }
  if (which == 3) J.w_u = J.w_p = -1.0;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  launch_stencil<double>(J, ROWS_UP, s);  // warm-up
  HIPCHK(hipEventRecord(e0, s));
  for (int k = 0; k < reps; ++k) launch_stencil<double>(J, ROWS_UP, s);
  HIPCHK(hipEventRecord(e1, s));
  HIPCHK(hipEventSynchronize(e1));
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *avg_ms = (double)ms / reps;
  return launch_status("smg_time_kernel");
}

}  // extern "C"

// ===========================================================================
// The entry point that allocates nothing
// ===========================================================================
// Callers that cannot allocate device memory (code under HIP graph capture,
// tight serving loops) compute a residual and its norm with the per-tile
// partial sums in `scratch`, a file-scope device array of fixed size: every
// GPU the library runs on holds its own copy until the process ends.  Its
// address on a device is looked up once, with that device current, and only
// that address is ever passed to kernels.  Each call overwrites every partial
// it reads (one per tile), so nothing has to start at zero; calls that
// overlap on one device race on the array.

namespace {

constexpr int NOALLOC_SCRATCH_DOUBLES = 1 << 17;   // 1 MiB
__device__ __align__(256) double scratch[NOALLOC_SCRATCH_DOUBLES];

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

// device address of `scratch` on the current device
int noalloc_scratch(double** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return fail(SMG_EINVAL, "device %d beyond %d", dev, NOALLOC_MAX_DEVICES);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return fail(SMG_EHIP, "no address for the scratch array on device %d", dev);
    g_scratch_ptr[dev] = static_cast<double*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return SMG_OK;
}

}  // namespace

extern "C" int smg_residual_noalloc(int N, double beta, int domain, const double* fu, const double* gp,
                                    const double* u, const double* p, double* ru, double* rp, double* norm2,
                                    smg_stream_t sv) {
  if (!fu || !gp || !u || !p || !ru || !rp) return fail(SMG_EINVAL, "null vector");
  if (N < 2 || N > 4096) return fail(SMG_EINVAL, "N=%d outside 2..4096", N);
  if (domain != SMG_DOM_SQUARE && domain != SMG_DOM_LSHAPE && domain != SMG_DOM_UNIONJACK)
    return fail(SMG_EINVAL, "unknown domain %d", domain);
  if (domain != SMG_DOM_SQUARE && N % 2) return fail(SMG_EINVAL, "this domain needs an even N");
  if (!(beta >= 0) || !std::isfinite(beta)) return fail(SMG_EINVAL, "beta must be finite and >= 0");
  const int tiles = stencil_tiles(N);
  if (norm2 && tiles > NOALLOC_SCRATCH_DOUBLES)
    return fail(SMG_EINVAL, "N=%d needs %d partial sums, the scratch array holds %d", N, tiles,
                NOALLOC_SCRATCH_DOUBLES);
  double* part = nullptr;
  if (norm2) {
    int rc = noalloc_scratch(&part);
    if (rc) return rc;
  }
  hipStream_t s = (hipStream_t)sv;
  LevelCoef<double> c64;
  LevelCoef<float> c32;
  host::make_coef(N, domain, beta, c64, c32);
  StencilJob<double> R{};
  R.L = c64;
  R.w_u = R.w_p = 1.0;
  R.in_u = u; R.in_p = p;
  R.rhs_u = fu; R.rhs_p = gp;
  R.out_u = ru; R.out_p = rp;
  R.partial = part;
  launch_stencil<double>(R, ROWS_UP, s);
  if (norm2) launch_reduce(part, tiles, norm2, s);
  return launch_status("smg_residual_noalloc");
}

#include "smg_batch.inc"
