// HIP kernels (gfx950) of the coupled Stokes multigrid: matrix-free
// application of the Taylor-Hood saddle operator on the uniformly refined
// same-diagonal grid, the smoother passes of Section 4, the canonical
// transfers of Section 3, the exact coarsest-grid solve, the pressure-mean
// projection and deterministic reductions.
//
// Lattice layout of a level with N x N squares (M = 2N + 1):
//   u[c][b][a], c = component, P2 node (a, b) at (a / 2N, b / 2N);
//   p[j][i], P1 vertex (i / N, j / N).
// Work decomposition: square (i, j) owns the lattice points (2i, 2j) (V),
// (2i+1, 2j) (H), (2i, 2j+1) (E), (2i+1, 2j+1) (D) and the vertex (i, j); one
// thread per square, TX x TY squares per workgroup, the input window with a
// halo of one square staged in LDS.  All operators are HBM-bound (about 2-4
// flop per byte); no matrix core work is involved.
#include <algorithm>

#include "smg_internal.h"
#include "smg_stage.h"

namespace smg {
#include "stencils.inc"
#include "smg_uj.h"
using namespace smg_stencil;

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------

// Workgroups are dealt round-robin to the 8 XCDs; remap so that each XCD gets
// a contiguous range of tiles (neighbouring tiles share halo lines in that
// XCD's L2).
__device__ __forceinline__ int xcd_swizzle(int bid, int nb) {
  const int xcd = bid & 7, idx = bid >> 3;
  const int per = nb >> 3, rem = nb & 7;
  return xcd * per + (xcd < rem ? xcd : rem) + idx;
}

// Sum over the workgroup (NT a multiple of 64); result valid in thread 0.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NT / 64; ++k) s += red[k];
  }
  return s;
}

template <int CLS, class T, class FU, class FC>
__device__ __forceinline__ T a_row(FU U, FC C) {
  if constexpr (CLS == 0) return SMG_A_ROW_V(U, C);
  else if constexpr (CLS == 1) return SMG_A_ROW_H(U, C);
  else if constexpr (CLS == 2) return SMG_A_ROW_E(U, C);
  else return SMG_A_ROW_D(U, C);
}
template <int CLS, class T, class FP>
__device__ __forceinline__ T btx_row(FP P) {
  if constexpr (CLS == 0) return SMG_BTX_ROW_V(P);
  else if constexpr (CLS == 1) return SMG_BTX_ROW_H(P);
  else if constexpr (CLS == 2) return SMG_BTX_ROW_E(P);
  else return SMG_BTX_ROW_D(P);
}
template <int CLS, class T, class FP>
__device__ __forceinline__ T bty_row(FP P) {
  if constexpr (CLS == 0) return SMG_BTY_ROW_V(P);
  else if constexpr (CLS == 1) return SMG_BTY_ROW_H(P);
  else if constexpr (CLS == 2) return SMG_BTY_ROW_E(P);
  else return SMG_BTY_ROW_D(P);
}
template <int CLS, class T, class FU>
__device__ __forceinline__ T m_row(FU U) {
  if constexpr (CLS == 0) return SMG_M_ROW_V(U);
  else if constexpr (CLS == 1) return SMG_M_ROW_H(U);
  else if constexpr (CLS == 2) return SMG_M_ROW_E(U);
  else return SMG_M_ROW_D(U);
}
template <int CLS, class T, class FR>
__device__ __forceinline__ T res_row(FR R) {
  if constexpr (CLS == 0) return SMG_RES_ROW_V(R);
  else if constexpr (CLS == 1) return SMG_RES_ROW_H(R);
  else if constexpr (CLS == 2) return SMG_RES_ROW_E(R);
  else return SMG_RES_ROW_D(R);
}

// ---------------------------------------------------------------------------
// generic fused stencil: out = base + w D (rhs - calA in)
// ---------------------------------------------------------------------------

// Operation flags of the fused stencil.  F = 0 selects the generic kernel,
// which tests every pointer at run time; any other value is a compile-time
// specialization in which absent operands are known to be absent.
enum : unsigned {
  F_ROWS_U = 1u, F_ROWS_P = 2u, F_IN_U = 4u, F_IN_P = 8u, F_RHS_U = 16u, F_RHS_P = 32u,
  F_BASE_U = 64u, F_BASE_P = 128u, F_DIAG_U = 256u, F_DIAG_P = 512u, F_OUT_U = 1024u,
  F_OUT_P = 2048u, F_PARTIAL = 4096u, F_PSUB = 8192u, F_MEAN = 16384u, F_OUT32 = 32768u
};

template <unsigned F>
struct Flags {
  template <class P>
  static __device__ __forceinline__ bool on(unsigned flag, P ptr) {
    if constexpr (F == 0) return ptr != nullptr;
    else return (F & flag) != 0;
  }
  static __device__ __forceinline__ bool on_int(unsigned flag, int v) {
    if constexpr (F == 0) return v != 0;
    else return (F & flag) != 0;
  }
};

template <int CLS, unsigned F, int DOM, class T, int WX, int WY, int PX, int PY>
__device__ __forceinline__ void velocity_node(const StencilJob<T>& J, T (*su)[WY][WX],
                                              T (*sp)[PX], int tx, int ty, int i, int j,
                                              double& nrm, const T* rpre) {
  using FL = Flags<F>;
  constexpr int DA = CLS & 1, DB = CLS >> 1;
  const int N = J.L.N, M = 2 * N + 1;
  const int a = 2 * i + DA, b = 2 * j + DB;
  if (a > 2 * N || b > 2 * N) return;
  const bool interior = dom_u(N, DOM >= 0 ? DOM : J.L.dom, a, b);
  const int la = 2 * tx + 2 + DA, lb = 2 * ty + 2 + DB;
  const bool hu = FL::on(F_IN_U, J.in_u);
  const bool hp = FL::on(F_IN_P, J.in_p);
  auto C = [&](int g) -> T { return J.L.acoef[CLS][g]; };
  auto P = [&](int di, int dj) -> T { return sp[ty + 1 + dj][tx + 1 + di]; };
  T dscale = FL::on_int(F_DIAG_U, J.diag_u) ? J.L.adinv[CLS] : T(1);
  // union-jack grid: the rows summed over the squares at the node, and the
  // diagonal of A with them
  T yuj[2] = {T(0), T(0)};
  if constexpr (DOM == SMG_DOM_UNIONJACK) {
    auto Us = [&](int c, int da, int db) -> T { return su[c][2 * ty + 2 + db][2 * tx + 2 + da]; };
    auto Ps = [&](int di, int dj) -> T { return sp[ty + 1 + dj][tx + 1 + di]; };
    auto OR = [&](int di, int dj) { return uj_orient(N, i + di, j + dj); };
    T dg;
    uj_vel_rows<CLS, T>(J.L.bh2, J.L.h, hu, hp, Us, Ps, OR, yuj[0], yuj[1], dg);
    if (FL::on_int(F_DIAG_U, J.diag_u)) dscale = T(1) / dg;
  }
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    auto U = [&](int da, int db) -> T { return su[c][lb + db][la + da]; };
    T y = T(0);
    if constexpr (DOM == SMG_DOM_UNIONJACK) {
      y = yuj[c];
    } else {
      if (hu) y += a_row<CLS, T>(U, C);
      if (hp) y += J.L.h * (c == 0 ? btx_row<CLS, T>(P) : bty_row<CLS, T>(P));
    }
    const size_t g = (size_t)c * M * M + (size_t)b * M + a;
    const T r = (rpre ? rpre[c] : FL::on(F_RHS_U, J.rhs_u) ? J.rhs_u[g] : T(0)) - y;
    if (FL::on(F_PARTIAL, J.partial) && interior) nrm += (double)r * (double)r;
    if (FL::on(F_OUT32, J.out32_u)) {
      const T v = (FL::on(F_BASE_U, J.base_u) ? J.base_u[g] : T(0)) + J.w_u * dscale * r;
      J.out32_u[g] = interior ? (float)v : 0.0f;
    } else if (FL::on(F_OUT_U, J.out_u)) {
      const T v = (FL::on(F_BASE_U, J.base_u) ? J.base_u[g] : T(0)) + J.w_u * dscale * r;
      J.out_u[g] = interior ? v : T(0);
    }
  }
}

// DOM: the domain, or -1 to read it from the job (the stencil kernels take
// the run-time test; the fused kernels are instantiated per domain)
template <class T, int TX, int TY, unsigned F, int DOM>
__device__ __forceinline__ void stencil_tile(const StencilJob<T>& J, int tile) {
  using FL = Flags<F>;
  constexpr int NT = TX * TY;
  constexpr int WX = 2 * TX + 4, WY = 2 * TY + 4;
  constexpr int PX = TX + 2, PY = TY + 2;
  __shared__ T su[2][WY][WX];
  __shared__ T sp[PY][PX];
  __shared__ double red[NT / 64];
  const int N = J.L.N, M = 2 * N + 1, NP = N + 1;
  const int dom = DOM >= 0 ? DOM : J.L.dom;
  const int ntx = (N + TX) / TX;
  const int i0 = (tile % ntx) * TX, j0 = (tile / ntx) * TY;
  const int tid = threadIdx.x;
  const bool rows_u = (F == 0) ? (J.out_u || J.out32_u || J.partial) : (F & F_ROWS_U) != 0;
  const bool rows_p = (F == 0) ? (J.out_p || J.out32_p || J.partial) : (F & F_ROWS_P) != 0;
  const bool hu = FL::on(F_IN_U, J.in_u);
  const bool hp = rows_u && FL::on(F_IN_P, J.in_p);
  const int tx = tid % TX, ty = tid / TX;
  const int i = i0 + tx, j = j0 + ty;
  // the done flag, the input windows and (in the compile-time modes) this
  // thread's right-hand side: every load in flight at once; the flag is
  // tested once the windows have arrived
  const int dn = J.done ? *J.done : 0;
  constexpr bool PRE_U = F != 0 && (F & F_RHS_U) && (F & F_ROWS_U);
  constexpr bool PRE_P = F != 0 && (F & F_RHS_P) && (F & F_ROWS_P);
  T ru[4][2] = {}, rp = T(0);
  if (i <= N && j <= N) {
    if constexpr (PRE_U) {
#pragma unroll
      for (int cls = 0; cls < 4; ++cls) {
        const int a = 2 * i + (cls & 1), b = 2 * j + (cls >> 1);
        if (a <= 2 * N && b <= 2 * N) {
          ru[cls][0] = J.rhs_u[(size_t)b * M + a];
          ru[cls][1] = J.rhs_u[(size_t)M * M + (size_t)b * M + a];
        }
      }
    }
    if constexpr (PRE_P) rp = J.rhs_p[(size_t)j * NP + i];
  }
  Staged<WX * WY, NT, 2, T> uw;
  Staged<PX * PY, NT, 2, T> pw;
  if (hu)
    uw.fetch(tid, [&](int e, T* v) {
      const int a = 2 * i0 - 2 + e % WX, b = 2 * j0 - 2 + e / WX;
      const bool in = dom_u(N, dom, a, b);
      const size_t g = (size_t)b * M + a;
      v[0] = in ? J.in_u[g] : T(0);
      v[1] = in ? J.in_u[(size_t)M * M + g] : T(0);
    });
  if (hp)
    pw.fetch(tid, [&](int e, T* v) {
      const int i = i0 - 1 + e % PX, j = j0 - 1 + e / PX;
      const bool in = dom_p(N, dom, i, j);
      const bool sub = in && FL::on(F_PSUB, J.in_p_sub);
      v[0] = in ? J.in_p[(size_t)j * NP + i] : T(0);
      v[1] = sub ? J.in_p_sub[(size_t)j * NP + i] : T(0);
    });
  if (hu)
    uw.put(tid, [&](int e, const T* v) {
      su[0][e / WX][e % WX] = v[0];
      su[1][e / WX][e % WX] = v[1];
    });
  if (hp)
    pw.put(tid, [&](int e, const T* v) {
      T x = v[0];
      if (FL::on(F_PSUB, J.in_p_sub)) x -= v[1];
      sp[e / PX][e % PX] = x;
    });
  if (dn) return;   // the same value in every thread of the block
  if (hu || hp) __syncthreads();
  double nrm = 0.0;
  if (i <= N && j <= N) {
    if (rows_u) {
      velocity_node<0, F, DOM, T, WX, WY, PX, PY>(J, su, sp, tx, ty, i, j, nrm, PRE_U ? ru[0] : nullptr);
      velocity_node<1, F, DOM, T, WX, WY, PX, PY>(J, su, sp, tx, ty, i, j, nrm, PRE_U ? ru[1] : nullptr);
      velocity_node<2, F, DOM, T, WX, WY, PX, PY>(J, su, sp, tx, ty, i, j, nrm, PRE_U ? ru[2] : nullptr);
      velocity_node<3, F, DOM, T, WX, WY, PX, PY>(J, su, sp, tx, ty, i, j, nrm, PRE_U ? ru[3] : nullptr);
    }
    if (rows_p) {
      const int la = 2 * tx + 2, lb = 2 * ty + 2;
      auto U0 = [&](int da, int db) -> T { return su[0][lb + db][la + da]; };
      auto U1 = [&](int da, int db) -> T { return su[1][lb + db][la + da]; };
      T y;
      if constexpr (DOM == SMG_DOM_UNIONJACK) {
        auto Us = [&](int c, int da, int db) -> T { return su[c][lb + db][la + da]; };
        auto OR = [&](int di, int dj) { return uj_orient(N, i + di, j + dj); };
        y = hu ? uj_p_row<T>(J.L.h, Us, OR) : T(0);
      } else {
        y = hu ? J.L.h * (SMG_BX_ROW(U0) + SMG_BY_ROW(U1)) : T(0);
      }
      const size_t g = (size_t)j * NP + i;
      // vertices outside the domain carry no pressure unknown: zero row
      const bool pin = dom_p(N, dom, i, j);
      const T r = pin ? (PRE_P ? rp : FL::on(F_RHS_P, J.rhs_p) ? J.rhs_p[g] : T(0)) - y : T(0);
      if (FL::on(F_PARTIAL, J.partial)) nrm += (double)r * (double)r;
      if (FL::on(F_OUT32, J.out32_p)) {
        const T d = FL::on_int(F_DIAG_P, J.diag_p) ? J.L.sinv[g] : T(1);
        J.out32_p[g] = pin ? (float)((FL::on(F_BASE_P, J.base_p) ? J.base_p[g] : T(0)) + J.w_p * d * r) : 0.0f;
      } else if (FL::on(F_OUT_P, J.out_p)) {
        const T d = FL::on_int(F_DIAG_P, J.diag_p) ? J.L.sinv[g] : T(1);
        J.out_p[g] = pin ? (FL::on(F_BASE_P, J.base_p) ? J.base_p[g] : T(0)) + J.w_p * d * r : T(0);
      }
    }
  }
  if (FL::on(F_PARTIAL, J.partial)) {
    const double s = block_sum<NT>(nrm, red);
    if (tid == 0) J.partial[tile] = s;
  }
  if (FL::on(F_MEAN, J.mean_partial)) {
    // pressure mean pieces of in_p over the owned vertices
    double w = 0.0, wp = 0.0;
    if (i <= N && j <= N) {
      w = p1_count_w(N, dom, i, j);
      wp = w * (double)sp[ty + 1][tx + 1];
    }
    __syncthreads();
    const double s1 = block_sum<NT>(wp, red);
    __syncthreads();
    const double s2 = block_sum<NT>(w, red);
    if (tid == 0) {
      J.mean_partial[2 * tile] = s1;
      J.mean_partial[2 * tile + 1] = s2;
    }
  }
}

template <class T, int TX, int TY, unsigned F>
__global__ __launch_bounds__(TX* TY) void k_stencil(StencilJob<T> J) {
  stencil_tile<T, TX, TY, F, -1>(J, xcd_swizzle(blockIdx.x, gridDim.x));
}

TileShape stencil_tile(int N) {
  if (N >= 512) return {16, 16};
  if (N >= 128) return {16, 8};
  return {8, 8};
}

int stencil_tiles(int N) {
  const TileShape t = stencil_tile(N);
  return ((N + t.tx) / t.tx) * ((N + t.ty) / t.ty);
}

// operation modes used by the library (anything else runs the generic kernel)
constexpr unsigned RW_UP = F_ROWS_U | F_ROWS_P;
constexpr unsigned OUT_UP = F_OUT_U | F_OUT_P;
constexpr unsigned M_APPLY = RW_UP | F_IN_U | F_IN_P | OUT_UP;
constexpr unsigned M_RESID = RW_UP | F_IN_U | F_IN_P | F_RHS_U | F_RHS_P | OUT_UP;
constexpr unsigned M_RESID_NORM = RW_UP | F_IN_U | F_IN_P | F_RHS_U | F_RHS_P | F_PARTIAL;
constexpr unsigned M_RESID_NORM_MEAN = M_RESID_NORM | F_MEAN;
constexpr unsigned M_RESID_BOTH_MEAN = M_RESID_NORM_MEAN | OUT_UP;
constexpr unsigned M_RESID_BOTH32 = M_RESID_NORM | OUT_UP | F_OUT32;
constexpr unsigned M_RESID_BOTH_MEAN32 = M_RESID_BOTH_MEAN | F_OUT32;
constexpr unsigned M_RESID_BOTH = M_RESID | F_PARTIAL;
constexpr unsigned M_NE1 = M_RESID | F_DIAG_U | F_DIAG_P;
constexpr unsigned M_NE1Z = RW_UP | F_RHS_U | F_RHS_P | F_DIAG_U | F_DIAG_P | OUT_UP;
constexpr unsigned M_NE2 = M_APPLY | F_BASE_U | F_BASE_P | F_DIAG_U | F_DIAG_P;
constexpr unsigned M_NE2Z = M_APPLY | F_DIAG_U | F_DIAG_P;
constexpr unsigned M_UZ1 = F_ROWS_U | F_IN_U | F_IN_P | F_RHS_U | F_BASE_U | F_DIAG_U | F_OUT_U;
constexpr unsigned M_UZ1Z = F_ROWS_U | F_RHS_U | F_DIAG_U | F_OUT_U;
constexpr unsigned M_UZ2 = F_ROWS_P | F_IN_U | F_RHS_P | F_DIAG_P | F_OUT_P;
constexpr unsigned M_UZ3 = RW_UP | F_IN_P | F_RHS_P | F_BASE_U | F_BASE_P | F_DIAG_U | OUT_UP;
constexpr unsigned M_UZ3Z = RW_UP | F_IN_P | F_RHS_P | F_BASE_U | F_DIAG_U | OUT_UP;
constexpr unsigned M_MASK_U = F_ROWS_U | F_RHS_U | F_OUT_U;
constexpr unsigned M_COPY = RW_UP | F_RHS_U | F_RHS_P | OUT_UP;
constexpr unsigned M_ZERO = RW_UP | OUT_UP;

template <class T>
unsigned stencil_flags(const StencilJob<T>& J, int rows);
template <class T>
unsigned job_flags(const StencilJob<T>& J, int rows) {
  return stencil_flags<T>(J, rows);
}
template <class T>
unsigned stencil_flags(const StencilJob<T>& J, int rows) {
  unsigned f = 0;
  if (rows & ROWS_U) f |= F_ROWS_U;
  if (rows & ROWS_P) f |= F_ROWS_P;
  if (J.in_u) f |= F_IN_U;
  if (J.in_p && (rows & ROWS_U)) f |= F_IN_P;
  if (J.in_p_sub && (rows & ROWS_U)) f |= F_PSUB;
  if (J.rhs_u && (rows & ROWS_U)) f |= F_RHS_U;
  if (J.rhs_p && (rows & ROWS_P)) f |= F_RHS_P;
  if (J.base_u && (rows & ROWS_U)) f |= F_BASE_U;
  if (J.base_p && (rows & ROWS_P)) f |= F_BASE_P;
  if (J.diag_u && (rows & ROWS_U)) f |= F_DIAG_U;
  if (J.diag_p && (rows & ROWS_P)) f |= F_DIAG_P;
  if (J.out_u && (rows & ROWS_U)) f |= F_OUT_U;
  if (J.out_p && (rows & ROWS_P)) f |= F_OUT_P;
  // FP32 outputs: a specialization only when both row kinds go to FP32
  if (J.out32_u && J.out32_p && !J.out_u && !J.out_p && rows == ROWS_UP) f |= F_OUT_U | F_OUT_P | F_OUT32;
  else if (J.out32_u || J.out32_p) f |= 1u << 30;   // generic kernel
  if (J.partial) f |= F_PARTIAL;
  if (J.mean_partial && J.in_p && (rows & ROWS_U)) f |= F_MEAN;
  return f;
}

// union-jack grid: the generic kernel (flags read from the job) with the rows
// summed square by square
template <class T, int TX, int TY>
__global__ __launch_bounds__(TX* TY) void k_stencil_uj(StencilJob<T> J) {
  stencil_tile<T, TX, TY, 0u, SMG_DOM_UNIONJACK>(J, xcd_swizzle(blockIdx.x, gridDim.x));
}

template <class T, int TX, int TY>
static void launch_stencil_shape(const StencilJob<T>& J, int rows, hipStream_t s) {
  const int nb = ((J.L.N + TX) / TX) * ((J.L.N + TY) / TY);
  if (J.L.dom == SMG_DOM_UNIONJACK) {
    StencilJob<T> G = J;
    if (!(rows & ROWS_U)) { G.out_u = nullptr; G.out32_u = nullptr; }
    if (!(rows & ROWS_P)) { G.out_p = nullptr; G.out32_p = nullptr; }
    k_stencil_uj<T, TX, TY><<<nb, TX * TY, 0, s>>>(G);
    return;
  }
  const unsigned f = job_flags(J, rows);
#define SMG_CASE(MODE) \
  case MODE: k_stencil<T, TX, TY, MODE><<<nb, TX * TY, 0, s>>>(J); return;
  switch (f) {
    SMG_CASE(M_APPLY) SMG_CASE(M_RESID) SMG_CASE(M_RESID_NORM) SMG_CASE(M_RESID_BOTH)
    SMG_CASE(M_RESID_NORM_MEAN) SMG_CASE(M_RESID_BOTH_MEAN) SMG_CASE(M_RESID_BOTH32) SMG_CASE(M_RESID_BOTH_MEAN32)
    SMG_CASE(M_NE1) SMG_CASE(M_NE1Z) SMG_CASE(M_NE2) SMG_CASE(M_NE2Z)
    SMG_CASE(M_UZ1) SMG_CASE(M_UZ1Z) SMG_CASE(M_UZ2) SMG_CASE(M_UZ3) SMG_CASE(M_UZ3Z)
    SMG_CASE(M_MASK_U) SMG_CASE(M_COPY) SMG_CASE(M_ZERO)
    default: break;
  }
#undef SMG_CASE
  // generic kernel: rows are selected by the output / partial pointers, so
  // clear the pointers of the rows that were not asked for
  StencilJob<T> G = J;
  if (!(rows & ROWS_U)) { G.out_u = nullptr; G.out32_u = nullptr; }
  if (!(rows & ROWS_P)) { G.out_p = nullptr; G.out32_p = nullptr; }
  k_stencil<T, TX, TY, 0u><<<nb, TX * TY, 0, s>>>(G);
}

template <class T>
void launch_stencil(const StencilJob<T>& J, int rows, hipStream_t s) {
  const TileShape t = stencil_tile(J.L.N);
  if (t.tx == 16 && t.ty == 16)
    launch_stencil_shape<T, 16, 16>(J, rows, s);
  else if (t.tx == 16 && t.ty == 8)
    launch_stencil_shape<T, 16, 8>(J, rows, s);
  else
    launch_stencil_shape<T, 8, 8>(J, rows, s);
}
template void launch_stencil<double>(const StencilJob<double>&, int, hipStream_t);
template void launch_stencil<float>(const StencilJob<float>&, int, hipStream_t);
template unsigned stencil_flags<double>(const StencilJob<double>&, int);
template unsigned stencil_flags<float>(const StencilJob<float>&, int);

int stencil_tiles_shape(int N, int tx, int ty) { return ((N + tx) / tx) * ((N + ty) / ty); }

template <class T, int TX, int TY, unsigned F, bool PACK>
__global__ __launch_bounds__(TX* TY) void k_stencil_b(const JobArg<StencilJob<T>> A) {
  int tile;
  const StencilJob<T> J = block_job<PACK>(A, xcd_swizzle(blockIdx.x, gridDim.x), tile);
  stencil_tile<T, TX, TY, F, -1>(J, tile);
}

// union-jack grid, batched: the generic kernel with the rows summed square by square
template <class T, int TX, int TY, bool PACK>
__global__ __launch_bounds__(TX* TY) void k_stencil_uj_b(const JobArg<StencilJob<T>> A) {
  int tile;
  const StencilJob<T> J = block_job<PACK>(A, xcd_swizzle(blockIdx.x, gridDim.x), tile);
  stencil_tile<T, TX, TY, 0u, SMG_DOM_UNIONJACK>(J, tile);
}

template <class T, int TX, int TY>
static void launch_stencil_b_shape(const JobArg<StencilJob<T>>& A, int nb, unsigned f, int dom, hipStream_t s) {
  if (dom == SMG_DOM_UNIONJACK) {
    if (A.n > 0) k_stencil_uj_b<T, TX, TY, true><<<nb, TX * TY, 0, s>>>(A);
    else k_stencil_uj_b<T, TX, TY, false><<<nb, TX * TY, 0, s>>>(A);
    return;
  }
#define SMG_CASE(MODE)                                                          \
  case MODE:                                                                    \
    if (A.n > 0) k_stencil_b<T, TX, TY, MODE, true><<<nb, TX * TY, 0, s>>>(A);  \
    else k_stencil_b<T, TX, TY, MODE, false><<<nb, TX * TY, 0, s>>>(A);         \
    return;
  switch (f) {
    SMG_CASE(M_APPLY) SMG_CASE(M_RESID) SMG_CASE(M_RESID_NORM) SMG_CASE(M_RESID_BOTH)
    SMG_CASE(M_RESID_NORM_MEAN) SMG_CASE(M_RESID_BOTH_MEAN) SMG_CASE(M_RESID_BOTH32) SMG_CASE(M_RESID_BOTH_MEAN32)
    SMG_CASE(M_NE1) SMG_CASE(M_NE1Z) SMG_CASE(M_NE2) SMG_CASE(M_NE2Z)
    SMG_CASE(M_UZ1) SMG_CASE(M_UZ1Z) SMG_CASE(M_UZ2) SMG_CASE(M_UZ3) SMG_CASE(M_UZ3Z)
    SMG_CASE(M_MASK_U) SMG_CASE(M_COPY) SMG_CASE(M_ZERO)
    default:
      if (A.n > 0) k_stencil_b<T, TX, TY, 0u, true><<<nb, TX * TY, 0, s>>>(A);
      else k_stencil_b<T, TX, TY, 0u, false><<<nb, TX * TY, 0, s>>>(A);
      return;
  }
#undef SMG_CASE
}

template <class T>
void launch_stencil_b(const JobArg<StencilJob<T>>& A, int nb, int tx, int ty, unsigned flags, int dom,
                      hipStream_t s) {
  if (tx == 16 && ty == 16) launch_stencil_b_shape<T, 16, 16>(A, nb, flags, dom, s);
  else if (tx == 16 && ty == 8) launch_stencil_b_shape<T, 16, 8>(A, nb, flags, dom, s);
  else launch_stencil_b_shape<T, 8, 8>(A, nb, flags, dom, s);
}
template void launch_stencil_b<double>(const JobArg<StencilJob<double>>&, int, int, int, unsigned, int,
                                       hipStream_t);
template void launch_stencil_b<float>(const JobArg<StencilJob<float>>&, int, int, int, unsigned, int,
                                      hipStream_t);

// ---------------------------------------------------------------------------
// transfers (Section 3): one thread per coarse square
// ---------------------------------------------------------------------------

template <int CLS, class T>
__device__ __forceinline__ void restrict_node(int Nc, int dom, int I, int J, const T* rfu, T* rcu, T* xcu) {
  constexpr int CA = CLS & 1, CB = CLS >> 1;
  const int A = 2 * I + CA, B = 2 * J + CB;
  if (A > 2 * Nc || B > 2 * Nc) return;
  const int Mc = 2 * Nc + 1, Mf = 4 * Nc + 1;
  const bool interior = dom_u(Nc, dom, A, B);
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const T* rf = rfu + (size_t)c * Mf * Mf;
    auto R = [&](int fa, int fb) -> T {
      const int a = 2 * A + fa, b = 2 * B + fb;
      return dom_u(2 * Nc, dom, a, b) ? rf[(size_t)b * Mf + a] : T(0);
    };
    const T v = interior ? res_row<CLS, T>(R) : T(0);
    const size_t g = (size_t)c * Mc * Mc + (size_t)B * Mc + A;
    rcu[g] = v;
    if (xcu) xcu[g] = T(0);
  }
}

template <class T>
__global__ __launch_bounds__(256) void k_restrict(int Nc, int dom, const T* __restrict__ rfu,
                                                  const T* __restrict__ rfp, T* rcu, T* rcp,
                                                  T* xcu, T* xcp, const int* done) {
  if (done && *done) return;
  const int I = blockIdx.x * 16 + (threadIdx.x & 15);
  const int J = blockIdx.y * 16 + (threadIdx.x >> 4);
  if (I > Nc || J > Nc) return;
  restrict_node<0, T>(Nc, dom, I, J, rfu, rcu, xcu);
  restrict_node<1, T>(Nc, dom, I, J, rfu, rcu, xcu);
  restrict_node<2, T>(Nc, dom, I, J, rfu, rcu, xcu);
  restrict_node<3, T>(Nc, dom, I, J, rfu, rcu, xcu);
  const int Nf = 2 * Nc, NPf = Nf + 1;
  auto Rp = [&](int i, int j) -> T {
    return dom_p(Nf, dom, i, j) ? rfp[(size_t)j * NPf + i] : T(0);
  };
  const int fi = 2 * I, fj = 2 * J;
  const T v = Rp(fi, fj) + T(0.5) * (Rp(fi + 1, fj) + Rp(fi - 1, fj) + Rp(fi, fj + 1) +
                                     Rp(fi, fj - 1) + Rp(fi + 1, fj + 1) + Rp(fi - 1, fj - 1));
  rcp[(size_t)J * (Nc + 1) + I] = dom_p(Nc, dom, I, J) ? v : T(0);
  if (xcp) xcp[(size_t)J * (Nc + 1) + I] = T(0);
}

// Union-jack grid: the transpose of the prolongation gathered square by
// square.  Every fine point is owned by one coarse square (the lower-left
// closed, upper-right open part of it; squares I = Nc or J = Nc own the right
// and top boundary), and its prolongation weights involve only that square's
// coarse nodes, so the coarse node (A, B) collects from the squares that
// contain it the owned fine points weighted by its column of the square's
// prolongation table.
template <class T>
__global__ __launch_bounds__(256) void k_restrict_uj(int Nc, const T* __restrict__ rfu,
                                                     const T* __restrict__ rfp, T* rcu, T* rcp,
                                                     T* xcu, T* xcp, const int* done) {
  using namespace smg_stencil;
  if (done && *done) return;
  const int I = blockIdx.x * 16 + (threadIdx.x & 15);
  const int J = blockIdx.y * 16 + (threadIdx.x >> 4);
  if (I > Nc || J > Nc) return;
  const int Nf = 2 * Nc, Mc = 2 * Nc + 1, Mf = 2 * Nf + 1, NPf = Nf + 1;
  for (int cls = 0; cls < 4; ++cls) {
    const int CA = cls & 1, CB = cls >> 1, A = 2 * I + CA, B = 2 * J + CB;
    if (A > 2 * Nc || B > 2 * Nc) continue;
    const bool interior = dom_u(Nc, SMG_DOM_UNIONJACK, A, B);
    T v[2] = {T(0), T(0)};
    for (int dj = (CB ? 0 : -1); dj <= 0; ++dj)
      for (int di = (CA ? 0 : -1); di <= 0; ++di) {
        const int SI = I + di, SJ = J + dj;
        if (SI < 0 || SJ < 0) continue;
        const int o = uj_orient_c(Nc, SI, SJ), cl = 3 * (CB - 2 * dj) + (CA - 2 * di);
        for (int f = 0; f < 16; ++f) {
          const double w = UJ_PRO[o][f][cl];
          const int a = 4 * SI + (f & 3), b = 4 * SJ + (f >> 2);
          if (w == 0.0 || !dom_u(Nf, SMG_DOM_UNIONJACK, a, b)) continue;
          v[0] += T(w) * rfu[(size_t)b * Mf + a];
          v[1] += T(w) * rfu[(size_t)Mf * Mf + (size_t)b * Mf + a];
        }
      }
    for (int c = 0; c < 2; ++c) {
      const size_t g = (size_t)c * Mc * Mc + (size_t)B * Mc + A;
      rcu[g] = interior ? v[c] : T(0);
      if (xcu) xcu[g] = T(0);
    }
  }
  T vp = T(0);
  for (int dj = -1; dj <= 0; ++dj)
    for (int di = -1; di <= 0; ++di) {
      const int SI = I + di, SJ = J + dj;
      if (SI < 0 || SJ < 0) continue;
      const int o = uj_orient_c(Nc, SI, SJ), q = 2 * (-dj) + (-di);
      for (int v = 0; v < 4; ++v) {
        const double w = UJ_PP[o][v][q];
        const int fi = 2 * SI + (v & 1), fj = 2 * SJ + (v >> 1);
        if (w == 0.0 || fi > Nf || fj > Nf) continue;
        vp += T(w) * rfp[(size_t)fj * NPf + fi];
      }
    }
  rcp[(size_t)J * (Nc + 1) + I] = vp;
  if (xcp) xcp[(size_t)J * (Nc + 1) + I] = T(0);
}

template <class T>
void launch_restrict(int Nc, int dom, const T* rfu, const T* rfp, T* rcu, T* rcp, T* xcu, T* xcp,
                     const int* done, hipStream_t s) {
  dim3 grid((Nc + 16) / 16, (Nc + 16) / 16);
  if (dom == SMG_DOM_UNIONJACK) k_restrict_uj<T><<<grid, 256, 0, s>>>(Nc, rfu, rfp, rcu, rcp, xcu, xcp, done);
  else k_restrict<T><<<grid, 256, 0, s>>>(Nc, dom, rfu, rfp, rcu, rcp, xcu, xcp, done);
}
template void launch_restrict<double>(int, int, const double*, const double*, double*, double*,
                                      double*, double*, const int*, hipStream_t);
template void launch_restrict<float>(int, int, const float*, const float*, float*, float*, float*,
                                     float*, const int*, hipStream_t);

template <int RA, int RB, class T, class FZ>
__device__ __forceinline__ T pro_weights(FZ Z) {
  if constexpr (RA == 0 && RB == 0) return SMG_PRO_00(Z);
  else if constexpr (RA == 0 && RB == 1) return SMG_PRO_01(Z);
  else if constexpr (RA == 0 && RB == 2) return SMG_PRO_02(Z);
  else if constexpr (RA == 0 && RB == 3) return SMG_PRO_03(Z);
  else if constexpr (RA == 1 && RB == 0) return SMG_PRO_10(Z);
  else if constexpr (RA == 1 && RB == 1) return SMG_PRO_11(Z);
  else if constexpr (RA == 1 && RB == 2) return SMG_PRO_12(Z);
  else if constexpr (RA == 1 && RB == 3) return SMG_PRO_13(Z);
  else if constexpr (RA == 2 && RB == 0) return SMG_PRO_20(Z);
  else if constexpr (RA == 2 && RB == 1) return SMG_PRO_21(Z);
  else if constexpr (RA == 2 && RB == 2) return SMG_PRO_22(Z);
  else if constexpr (RA == 2 && RB == 3) return SMG_PRO_23(Z);
  else if constexpr (RA == 3 && RB == 0) return SMG_PRO_30(Z);
  else if constexpr (RA == 3 && RB == 1) return SMG_PRO_31(Z);
  else if constexpr (RA == 3 && RB == 2) return SMG_PRO_32(Z);
  else return SMG_PRO_33(Z);
}

template <int RA, int RB, class T, class FZ>
__device__ __forceinline__ void pro_point(int Nf, int dom, int I, int J, FZ Z, T* uf) {
  const int a = 4 * I + RA, b = 4 * J + RB;
  if (!dom_u(Nf, dom, a, b)) return;
  uf[(size_t)b * (2 * Nf + 1) + a] += pro_weights<RA, RB, T>(Z);
}

template <class T>
__device__ __forceinline__ void prolong_body(int Nc, int dom, const T* __restrict__ zu,
                                             const T* __restrict__ zp, T* u, T* p, int bx, int by) {
  const int I = bx * 16 + (threadIdx.x & 15);
  const int J = by * 16 + (threadIdx.x >> 4);
  if (I > Nc || J > Nc) return;
  const int Nf = 2 * Nc, Mc = 2 * Nc + 1, Mf = 2 * Nf + 1;
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const T* z = zu + (size_t)c * Mc * Mc;
    T* uf = u + (size_t)c * Mf * Mf;
    auto Z = [&](int dA, int dB) -> T {
      const int A = 2 * I + dA, B = 2 * J + dB;
      return dom_u(Nc, dom, A, B) ? z[(size_t)B * Mc + A] : T(0);
    };
    pro_point<0, 0, T>(Nf, dom, I, J, Z, uf); pro_point<1, 0, T>(Nf, dom, I, J, Z, uf);
    pro_point<2, 0, T>(Nf, dom, I, J, Z, uf); pro_point<3, 0, T>(Nf, dom, I, J, Z, uf);
    pro_point<0, 1, T>(Nf, dom, I, J, Z, uf); pro_point<1, 1, T>(Nf, dom, I, J, Z, uf);
    pro_point<2, 1, T>(Nf, dom, I, J, Z, uf); pro_point<3, 1, T>(Nf, dom, I, J, Z, uf);
    pro_point<0, 2, T>(Nf, dom, I, J, Z, uf); pro_point<1, 2, T>(Nf, dom, I, J, Z, uf);
    pro_point<2, 2, T>(Nf, dom, I, J, Z, uf); pro_point<3, 2, T>(Nf, dom, I, J, Z, uf);
    pro_point<0, 3, T>(Nf, dom, I, J, Z, uf); pro_point<1, 3, T>(Nf, dom, I, J, Z, uf);
    pro_point<2, 3, T>(Nf, dom, I, J, Z, uf); pro_point<3, 3, T>(Nf, dom, I, J, Z, uf);
  }
  // P1: copy at coarse vertices, mean of the two ends at edge midpoints
  const int NPc = Nc + 1, NPf = Nf + 1;
  auto Zp = [&](int i, int j) -> T { return zp[(size_t)j * NPc + i]; };
  const int fi = 2 * I, fj = 2 * J;
  // fine vertices of the domain only (their coarse parents belong to it too)
  if (dom_p(Nf, dom, fi, fj)) p[(size_t)fj * NPf + fi] += Zp(I, J);
  if (I < Nc && dom_p(Nf, dom, fi + 1, fj)) p[(size_t)fj * NPf + fi + 1] += T(0.5) * (Zp(I, J) + Zp(I + 1, J));
  if (J < Nc && dom_p(Nf, dom, fi, fj + 1)) p[(size_t)(fj + 1) * NPf + fi] += T(0.5) * (Zp(I, J) + Zp(I, J + 1));
  if (I < Nc && J < Nc && dom_p(Nf, dom, fi + 1, fj + 1))
    p[(size_t)(fj + 1) * NPf + fi + 1] += T(0.5) * (Zp(I, J) + Zp(I + 1, J + 1));
}

template <class T>
__global__ __launch_bounds__(256) void k_prolong_add(int Nc, int dom, const T* __restrict__ zu,
                                                     const T* __restrict__ zp, T* u, T* p,
                                                     const int* done) {
  if (done && *done) return;
  prolong_body<T>(Nc, dom, zu, zp, u, p, blockIdx.x, blockIdx.y);
}

int prolong_tiles(int Nc) { return ((Nc + 16) / 16) * ((Nc + 16) / 16); }

template <class T>
__device__ __forceinline__ void prolong_uj_body(int Nc, const T* __restrict__ zu, const T* __restrict__ zp,
                                                T* u, T* p, int bx, int by);

template <class T, bool PACK>
__global__ __launch_bounds__(256) void k_prolong_b(const JobArg<ProJob<T>> A) {
  int tile;
  const ProJob<T> J = block_job<PACK>(A, (int)blockIdx.x, tile);
  if (J.done && *J.done) return;
  const int ntx = (J.Nc + 16) / 16;
  if (J.dom == SMG_DOM_UNIONJACK) prolong_uj_body<T>(J.Nc, J.zu, J.zp, J.u, J.p, tile % ntx, tile / ntx);
  else prolong_body<T>(J.Nc, J.dom, J.zu, J.zp, J.u, J.p, tile % ntx, tile / ntx);
}

template <class T>
void launch_prolong_b(const JobArg<ProJob<T>>& A, int nb, hipStream_t s) {
  if (A.n > 0) k_prolong_b<T, true><<<nb, 256, 0, s>>>(A);
  else k_prolong_b<T, false><<<nb, 256, 0, s>>>(A);
}
template void launch_prolong_b<double>(const JobArg<ProJob<double>>&, int, hipStream_t);
template void launch_prolong_b<float>(const JobArg<ProJob<float>>&, int, hipStream_t);

// Union-jack grid: every coarse square adds the interpolant of its coarse
// nodes at the fine points it owns, with the table of its diagonal direction.
template <class T>
__device__ __forceinline__ void prolong_uj_body(int Nc, const T* __restrict__ zu, const T* __restrict__ zp,
                                                T* u, T* p, int bx, int by) {
  using namespace smg_stencil;
  const int I = bx * 16 + (threadIdx.x & 15);
  const int J = by * 16 + (threadIdx.x >> 4);
  if (I > Nc || J > Nc) return;
  const int Nf = 2 * Nc, Mc = 2 * Nc + 1, Mf = 2 * Nf + 1, NPc = Nc + 1, NPf = Nf + 1;
  const int o = uj_orient_c(Nc, I, J);
  for (int c = 0; c < 2; ++c) {
    T z[9];
    for (int k = 0; k < 9; ++k) {
      const int A = 2 * I + k % 3, B = 2 * J + k / 3;
      z[k] = dom_u(Nc, SMG_DOM_UNIONJACK, A, B) ? zu[(size_t)c * Mc * Mc + (size_t)B * Mc + A] : T(0);
    }
    for (int f = 0; f < 16; ++f) {
      const int a = 4 * I + (f & 3), b = 4 * J + (f >> 2);
      if (!dom_u(Nf, SMG_DOM_UNIONJACK, a, b)) continue;
      T v = T(0);
      for (int k = 0; k < 9; ++k) v += T(UJ_PRO[o][f][k]) * z[k];
      u[(size_t)c * Mf * Mf + (size_t)b * Mf + a] += v;
    }
  }
  T zc[4];
  for (int q = 0; q < 4; ++q) {
    const int ci = I + (q & 1), cj = J + (q >> 1);
    zc[q] = (ci <= Nc && cj <= Nc) ? zp[(size_t)cj * NPc + ci] : T(0);
  }
  for (int v = 0; v < 4; ++v) {
    const int fi = 2 * I + (v & 1), fj = 2 * J + (v >> 1);
    if (fi > Nf || fj > Nf) continue;
    T w = T(0);
    for (int q = 0; q < 4; ++q) w += T(UJ_PP[o][v][q]) * zc[q];
    p[(size_t)fj * NPf + fi] += w;
  }
}

template <class T>
__global__ __launch_bounds__(256) void k_prolong_uj(int Nc, const T* __restrict__ zu,
                                                    const T* __restrict__ zp, T* u, T* p,
                                                    const int* done) {
  if (done && *done) return;
  prolong_uj_body<T>(Nc, zu, zp, u, p, blockIdx.x, blockIdx.y);
}

template <class T>
void launch_prolong_add(int Nc, int dom, const T* zu, const T* zp, T* u, T* p, const int* done,
                        hipStream_t s) {
  dim3 grid((Nc + 16) / 16, (Nc + 16) / 16);
  if (dom == SMG_DOM_UNIONJACK) k_prolong_uj<T><<<grid, 256, 0, s>>>(Nc, zu, zp, u, p, done);
  else k_prolong_add<T><<<grid, 256, 0, s>>>(Nc, dom, zu, zp, u, p, done);
}
template void launch_prolong_add<double>(int, int, const double*, const double*, double*, double*,
                                         const int*, hipStream_t);
template void launch_prolong_add<float>(int, int, const float*, const float*, float*, float*,
                                        const int*, hipStream_t);

// ---------------------------------------------------------------------------
// coarsest grid: z = Cinv [r; 0] (Section 3, exact solve on level 0)
// Compact order: velocity x then y at interior lattice points (b-major, then
// a), then all pressure vertices, then the multiplier of m^T p = 0.
// ---------------------------------------------------------------------------

template <class T>
__global__ __launch_bounds__(256) void k_coarse_solve(int N0, int dom, int nc, const double* __restrict__ cinv,
                                                      const T* ru, const T* rp, T* zu, T* zp,
                                                      const int* done) {
  if (done && *done) return;
  extern __shared__ double sh[];
  double* sr = sh;
  double* sz = sh + nc;
  const int M0 = 2 * N0 + 1, ni = 2 * N0 - 1, nu = ni * ni, NP = N0 + 1;
  for (int k = threadIdx.x; k < nc; k += blockDim.x) {
    double v = 0.0;
    if (k < 2 * nu) {
      const int c = k / nu, q = k % nu;
      const int a = 1 + q % ni, b = 1 + q / ni;
      v = (double)ru[(size_t)c * M0 * M0 + (size_t)b * M0 + a];
    } else if (k < 2 * nu + NP * NP) {
      v = (double)rp[k - 2 * nu];
    }
    sr[k] = v;
  }
  __syncthreads();
  for (int row = threadIdx.x; row < nc; row += blockDim.x) {
    double z = 0.0;
    // eight columns' loads in flight at a time, added in column order
    for (int j0 = 0; j0 < nc; j0 += 8) {
      double cv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) cv[u] = j0 + u < nc ? cinv[(size_t)(j0 + u) * nc + row] : 0.0;
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (j0 + u < nc) z += cv[u] * sr[j0 + u];
    }
    sz[row] = z;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < 2 * M0 * M0; k += blockDim.x) {
    const int c = k / (M0 * M0), q = k % (M0 * M0);
    const int a = q % M0, b = q / M0;
    T v = T(0);
    if (dom_u(N0, dom, a, b)) v = (T)sz[c * nu + (b - 1) * ni + (a - 1)];
    zu[k] = v;
  }
  for (int k = threadIdx.x; k < NP * NP; k += blockDim.x)
    zp[k] = dom_p(N0, dom, k % NP, k / NP) ? (T)sz[2 * nu + k] : T(0);
}

template <class T>
void launch_coarse_solve(int N0, int dom, int nc, const double* cinv, const T* ru, const T* rp, T* zu,
                         T* zp, const int* done, hipStream_t s) {
  k_coarse_solve<T><<<1, 256, 2 * nc * sizeof(double), s>>>(N0, dom, nc, cinv, ru, rp, zu, zp, done);
}
template void launch_coarse_solve<double>(int, int, int, const double*, const double*, const double*,
                                          double*, double*, const int*, hipStream_t);
template void launch_coarse_solve<float>(int, int, int, const double*, const float*, const float*,
                                         float*, float*, const int*, hipStream_t);

// ---------------------------------------------------------------------------
// pressure mean: p <- p - (m . p) / sum m, m_i = int phi_i (relative weights
// from the triangles of the domain around each vertex: on the unit square 1
// inside, 1/2 on edges, 1/3 at (0,0) and (1,1), 1/6 at (1,0) and (0,1)).
// Vertices outside the domain keep their (zero) value.
// ---------------------------------------------------------------------------

constexpr int MEAN_PER_THREAD = 4;
int mean_blocks(int N) {
  const int n = (N + 1) * (N + 1);
  return (n + 256 * MEAN_PER_THREAD - 1) / (256 * MEAN_PER_THREAD);
}

// mode 0: p <- p - (sum w p / sum w)          (mean projection)
// mode 1: p <- p - w (sum p / sum w)          (its transpose, Pi^T)
__global__ __launch_bounds__(256) void k_mean_partial(int N, int dom, const double* __restrict__ p,
                                                      double* partials, const int* done, int mode) {
  if (done && *done) return;
  __shared__ double red[4];
  const int n = (N + 1) * (N + 1);
  double s1 = 0.0, s2 = 0.0;
  for (int k = 0; k < MEAN_PER_THREAD; ++k) {
    const int e = blockIdx.x * 256 * MEAN_PER_THREAD + k * 256 + threadIdx.x;
    if (e < n) {
      const double w = p1_count_w(N, dom, e % (N + 1), e / (N + 1));
      s1 += (mode == 0 ? w : (w > 0 ? 1.0 : 0.0)) * p[e];
      s2 += w;
    }
  }
  const double t1 = block_sum<256>(s1, red);
  __syncthreads();
  const double t2 = block_sum<256>(s2, red);
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = t1;
    partials[2 * blockIdx.x + 1] = t2;
  }
}

__global__ __launch_bounds__(256) void k_mean_apply(int N, int dom, double* p,
                                                    const double* __restrict__ partials, int nparts,
                                                    const int* done, int mode) {
  if (done && *done) return;
  __shared__ double red[4];
  __shared__ double mean;
  double s1 = 0.0, s2 = 0.0;
  for (int k = threadIdx.x; k < nparts; k += 256) {
    s1 += partials[2 * k];
    s2 += partials[2 * k + 1];
  }
  const double t1 = block_sum<256>(s1, red);
  __syncthreads();
  const double t2 = block_sum<256>(s2, red);
  if (threadIdx.x == 0) mean = t1 / t2;
  __syncthreads();
  const int n = (N + 1) * (N + 1);
  for (int k = 0; k < MEAN_PER_THREAD; ++k) {
    const int e = blockIdx.x * 256 * MEAN_PER_THREAD + k * 256 + threadIdx.x;
    if (e < n) {
      const double w = p1_count_w(N, dom, e % (N + 1), e / (N + 1));
      if (w > 0) p[e] -= (mode == 0 ? 1.0 : w) * mean;
    }
  }
}

void launch_project_mean(int N, int dom, double* p, double* partials, const int* done, hipStream_t s) {
  const int nb = mean_blocks(N);
  k_mean_partial<<<nb, 256, 0, s>>>(N, dom, p, partials, done, 0);
  k_mean_apply<<<nb, 256, 0, s>>>(N, dom, p, partials, nb, done, 0);
}

void launch_project_dual(int N, int dom, double* p, double* partials, hipStream_t s) {
  const int nb = mean_blocks(N);
  k_mean_partial<<<nb, 256, 0, s>>>(N, dom, p, partials, nullptr, 1);
  k_mean_apply<<<nb, 256, 0, s>>>(N, dom, p, partials, nb, nullptr, 1);
}

// ---------------------------------------------------------------------------
// setup: Shat^-1 at every pressure vertex (Section 6: Shat = diag(B Ahat^-1 B^T),
// the sum running over interior velocity nodes only)
// ---------------------------------------------------------------------------

template <class T>
__global__ __launch_bounds__(256) void k_shat_inv(int N, int dom, T ad0, T ad1, T ad2, T ad3, T* sinv) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= (N + 1) * (N + 1)) return;
  const int i = e % (N + 1), j = e / (N + 1);
  const T h = T(1) / T(N);
  auto IN = [&](int da, int db) -> bool { return dom_u(N, dom, 2 * i + da, 2 * j + db); };
  auto AD = [&](int c) -> T { return c == 0 ? ad0 : c == 1 ? ad1 : c == 2 ? ad2 : ad3; };
  const T S = h * h * SMG_SHAT_ROW(IN, AD);
  // a vertex outside the domain couples to no unknown: no pressure update there
  sinv[e] = dom_p(N, dom, i, j) ? T(1) / S : T(0);
}

// Union-jack grid: the B row of vertex (i, j) assembled from the four squares
// around it on the 5 x 5 lattice window centred at the vertex, then
// Shat = h^2 sum over interior nodes of (Bx^2 + By^2) / Ahat (Ahat per node).
template <class T>
__global__ __launch_bounds__(256) void k_shat_inv_uj(int N, double bh2, T* sinv) {
  using namespace smg_stencil;
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= (N + 1) * (N + 1)) return;
  const int i = e % (N + 1), j = e / (N + 1);
  double bx[25], by[25];
  for (int k = 0; k < 25; ++k) bx[k] = by[k] = 0.0;
  for (int dj = -1; dj <= 0; ++dj)
    for (int di = -1; di <= 0; ++di) {
      if (!dom_sq(N, SMG_DOM_UNIONJACK, i + di, j + dj)) continue;
      const int o = uj_orient(N, i + di, j + dj), q = 2 * (-dj) + (-di);
      for (int m = 0; m < 9; ++m) {
        const int w = (2 * dj + m / 3 + 2) * 5 + (2 * di + m % 3 + 2);
        bx[w] += UJ_BX[o][q][m];
        by[w] += UJ_BY[o][q][m];
      }
    }
  double S = 0.0;
  for (int w = 0; w < 25; ++w) {
    const int a = 2 * i + w % 5 - 2, b = 2 * j + w / 5 - 2;
    if (!dom_u(N, SMG_DOM_UNIONJACK, a, b) || (bx[w] == 0.0 && by[w] == 0.0)) continue;
    S += (bx[w] * bx[w] + by[w] * by[w]) / uj_adiag(N, a, b, bh2);
  }
  sinv[e] = T(1.0 / (S / ((double)N * (double)N)));
}

template <class T>
void launch_shat_inv(int N, int dom, double bh2, const T* ad, T* sinv, hipStream_t s) {
  const int n = (N + 1) * (N + 1);
  if (dom == SMG_DOM_UNIONJACK) k_shat_inv_uj<T><<<(n + 255) / 256, 256, 0, s>>>(N, bh2, sinv);
  else k_shat_inv<T><<<(n + 255) / 256, 256, 0, s>>>(N, dom, ad[0], ad[1], ad[2], ad[3], sinv);
}
template void launch_shat_inv<double>(int, int, double, const double*, double*, hipStream_t);
template void launch_shat_inv<float>(int, int, double, const float*, float*, hipStream_t);

// ---------------------------------------------------------------------------
// masses (load vectors and the adjoint): one thread per square, direct loads
// ---------------------------------------------------------------------------

template <int CLS>
__device__ __forceinline__ void mass_node(int N, int dom, int i, int j, int rows_all, int read_all,
                                          const double* u, double* y, double scale, int acc) {
  using T = double;
  constexpr int DA = CLS & 1, DB = CLS >> 1;
  const int M = 2 * N + 1;
  const int a = 2 * i + DA, b = 2 * j + DB;
  if (a > 2 * N || b > 2 * N) return;
  const bool interior = dom_u(N, dom, a, b);
  const double h2 = 1.0 / ((double)N * (double)N);
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const double* uc = u + (size_t)c * M * M;
    auto U = [&](int da, int db) -> T {
      const int aa = a + da, bb = b + db;
      const bool ok = read_all ? (aa >= 0 && aa <= 2 * N && bb >= 0 && bb <= 2 * N)
                               : dom_u(N, dom, aa, bb);
      return ok ? uc[(size_t)bb * M + aa] : 0.0;
    };
    const double v = (interior || rows_all) ? h2 * m_row<CLS, T>(U) : 0.0;
    const size_t g = (size_t)c * M * M + (size_t)b * M + a;
    y[g] = acc ? y[g] + scale * v : v;
  }
}

__global__ __launch_bounds__(256) void k_mass_u(int N, int dom, int rows_all, int read_all,
                                                const double* __restrict__ u, double* y, double scale,
                                                int acc) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= (N + 1) * (N + 1)) return;
  const int i = e % (N + 1), j = e / (N + 1);
  mass_node<0>(N, dom, i, j, rows_all, read_all, u, y, scale, acc);
  mass_node<1>(N, dom, i, j, rows_all, read_all, u, y, scale, acc);
  mass_node<2>(N, dom, i, j, rows_all, read_all, u, y, scale, acc);
  mass_node<3>(N, dom, i, j, rows_all, read_all, u, y, scale, acc);
}

// union-jack grid: P2 mass rows summed square by square (squares of the grid only)
__global__ __launch_bounds__(256) void k_mass_u_uj(int N, int rows_all, int read_all,
                                                   const double* __restrict__ u, double* y, double scale,
                                                   int acc) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= (N + 1) * (N + 1)) return;
  const int i = e % (N + 1), j = e / (N + 1), M = 2 * N + 1;
  const double h2 = 1.0 / ((double)N * (double)N);
  for (int cls = 0; cls < 4; ++cls) {
    const int a = 2 * i + (cls & 1), b = 2 * j + (cls >> 1);
    if (a > 2 * N || b > 2 * N) continue;
    const bool interior = dom_u(N, SMG_DOM_UNIONJACK, a, b);
    for (int c = 0; c < 2; ++c) {
      const double* uc = u + (size_t)c * M * M;
      auto U = [&](int la, int lb) -> double {
        const int aa = 2 * i + la, bb = 2 * j + lb;
        const bool ok = read_all ? (aa >= 0 && aa <= 2 * N && bb >= 0 && bb <= 2 * N)
                                 : dom_u(N, SMG_DOM_UNIONJACK, aa, bb);
        return ok ? uc[(size_t)bb * M + aa] : 0.0;
      };
      const double v = (interior || rows_all) ? h2 * uj_m_row<double>(N, a, b, U) : 0.0;
      const size_t g = (size_t)c * M * M + (size_t)b * M + a;
      y[g] = acc ? y[g] + scale * v : v;
    }
  }
}

void launch_mass_u(int N, int dom, int mode, const double* u, double* y, hipStream_t s) {
  // mode 0: rows interior, read interior; 1: rows all, read interior; 2: rows interior, read all
  const int n = (N + 1) * (N + 1);
  if (dom == SMG_DOM_UNIONJACK) k_mass_u_uj<<<(n + 255) / 256, 256, 0, s>>>(N, mode == 1, mode == 2, u, y, 1.0, 0);
  else k_mass_u<<<(n + 255) / 256, 256, 0, s>>>(N, dom, mode == 1, mode == 2, u, y, 1.0, 0);
}

void launch_mass_u_acc(int N, int dom, int mode, const double* u, double scale, double* y, hipStream_t s) {
  const int n = (N + 1) * (N + 1);
  if (dom == SMG_DOM_UNIONJACK) k_mass_u_uj<<<(n + 255) / 256, 256, 0, s>>>(N, mode == 1, mode == 2, u, y, scale, 1);
  else k_mass_u<<<(n + 255) / 256, 256, 0, s>>>(N, dom, mode == 1, mode == 2, u, y, scale, 1);
}

// P1 mass: the six triangles around vertex (i, j) of the same-diagonal grid,
// each of area h^2/2, contribute h^2/24 (2 g_i + g_a + g_b) when inside.
__global__ __launch_bounds__(256) void k_mass_p(int N, int dom, const double* __restrict__ g, double* gp) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= (N + 1) * (N + 1)) return;
  const int i = e % (N + 1), j = e / (N + 1), NP = N + 1;
  auto G = [&](int ii, int jj) { return g[(size_t)jj * NP + ii]; };
  auto sq = [&](int si, int sj) { return dom_sq(N, dom, si, sj); };
  const double gi = G(i, j);
  double s = 0.0;
  if (sq(i - 1, j - 1)) {
    s += 2 * gi + G(i - 1, j - 1) + G(i, j - 1);   // lower triangle of square (i-1, j-1)
    s += 2 * gi + G(i - 1, j - 1) + G(i - 1, j);   // upper triangle
  }
  if (sq(i, j - 1)) s += 2 * gi + G(i, j - 1) + G(i + 1, j);      // upper triangle of (i, j-1)
  if (sq(i - 1, j)) s += 2 * gi + G(i - 1, j) + G(i, j + 1);      // lower triangle of (i-1, j)
  if (sq(i, j)) {
    s += 2 * gi + G(i + 1, j) + G(i + 1, j + 1);   // lower triangle of (i, j)
    s += 2 * gi + G(i + 1, j + 1) + G(i, j + 1);   // upper triangle
  }
  gp[e] = s / (24.0 * (double)N * (double)N);
}

__global__ __launch_bounds__(256) void k_mass_p_uj(int N, const double* __restrict__ g, double* gp) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= (N + 1) * (N + 1)) return;
  const int i = e % (N + 1), j = e / (N + 1), NP = N + 1;
  auto G = [&](int di, int dj) -> double {
    const int ii = i + di, jj = j + dj;
    return (ii >= 0 && ii <= N && jj >= 0 && jj <= N) ? g[(size_t)jj * NP + ii] : 0.0;
  };
  gp[e] = uj_mp_row<double>(N, i, j, G) / ((double)N * (double)N);
}

void launch_mass_p(int N, int dom, const double* g, double* gp, hipStream_t s) {
  const int n = (N + 1) * (N + 1);
  if (dom == SMG_DOM_UNIONJACK) k_mass_p_uj<<<(n + 255) / 256, 256, 0, s>>>(N, g, gp);
  else k_mass_p<<<(n + 255) / 256, 256, 0, s>>>(N, dom, g, gp);
}

// ---------------------------------------------------------------------------
// deterministic dots and the solve-loop bookkeeping
// ---------------------------------------------------------------------------

constexpr int DOT_PER_THREAD = 4;
int dot_blocks(int N, int which) {
  const int64_t n = which == 0 ? 2LL * (2 * N + 1) * (2 * N + 1) : (int64_t)(N + 1) * (N + 1);
  return (int)((n + 256 * DOT_PER_THREAD - 1) / (256 * DOT_PER_THREAD));
}

__global__ __launch_bounds__(256) void k_dot_partial(int N, int dom, int which, const double* __restrict__ a,
                                                     const double* __restrict__ b, double* partials) {
  __shared__ double red[4];
  const int M = 2 * N + 1;
  const int64_t n = which == 0 ? 2LL * M * M : (int64_t)(N + 1) * (N + 1);
  double s = 0.0;
  for (int k = 0; k < DOT_PER_THREAD; ++k) {
    const int64_t e = (int64_t)blockIdx.x * 256 * DOT_PER_THREAD + k * 256 + threadIdx.x;
    if (e < n) {
      bool ok;
      if (which == 0) {
        const int q = (int)(e % ((int64_t)M * M));
        ok = dom_u(N, dom, q % M, q / M);
      } else {
        ok = dom_p(N, dom, (int)(e % (N + 1)), (int)(e / (N + 1)));
      }
      if (ok) s += a[e] * b[e];
    }
  }
  const double t = block_sum<256>(s, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

__global__ __launch_bounds__(256) void k_reduce_final(const double* __restrict__ partials, int np,
                                                      double* out) {
  __shared__ double red[4];
  double s = 0.0;
  for (int k = threadIdx.x; k < np; k += 256) s += partials[k];
  const double t = block_sum<256>(s, red);
  if (threadIdx.x == 0) out[0] = t;
}

void launch_reduce(const double* partials, int np, double* out, hipStream_t s) {
  k_reduce_final<<<1, 256, 0, s>>>(partials, np, out);
}

// ---------------------------------------------------------------------------
// error measure of the experiments (Section 6): ||(u, p) - (us, ps)||_L with
// L = diag(Ahat, Shat), the pressure difference made mean-free first
// ---------------------------------------------------------------------------

__device__ __forceinline__ double enorm_ahat(int N, int dom, double bh2, const double* ad, int a, int b) {
  if (dom == SMG_DOM_UNIONJACK) return uj_adiag(N, a, b, bh2);
  return ad[(a & 1) + 2 * (b & 1)];
}

// mode 0: partials of sum w d and sum w (d = p - ps, w = P1 weights), in two
// arrays of nb entries; mode 1: partials of sum Shat (d - mean)^2, the mean
// read from sums[0] / sums[1]
__global__ __launch_bounds__(256) void k_enorm_p(int N, int dom, int mode, const double* __restrict__ p,
                                                 const double* __restrict__ ps, const double* __restrict__ sinv,
                                                 const double* __restrict__ sums, double* partials, int nb) {
  __shared__ double red[4];
  const int n = (N + 1) * (N + 1);
  const double mean = mode == 1 ? sums[0] / sums[1] : 0.0;
  double s1 = 0.0, s2 = 0.0;
  for (int k = 0; k < 4; ++k) {
    const int e = blockIdx.x * 1024 + k * 256 + threadIdx.x;
    if (e >= n || !dom_p(N, dom, e % (N + 1), e / (N + 1))) continue;
    const double d = p[e] - ps[e];
    if (mode == 0) {
      const double w = p1_count_w(N, dom, e % (N + 1), e / (N + 1));
      s1 += w * d;
      s2 += w;
    } else if (sinv[e] != 0.0) {
      s1 += (d - mean) * (d - mean) / sinv[e];
    }
  }
  const double t1 = block_sum<256>(s1, red);
  __syncthreads();
  const double t2 = block_sum<256>(s2, red);
  if (threadIdx.x == 0) {
    partials[blockIdx.x] = t1;
    if (mode == 0) partials[nb + blockIdx.x] = t2;
  }
}

__global__ __launch_bounds__(256) void k_enorm_u(int N, int dom, double bh2, double a0, double a1, double a2,
                                                 double a3, const double* __restrict__ u,
                                                 const double* __restrict__ us, double* partials) {
  __shared__ double red[4];
  const int M = 2 * N + 1;
  const int64_t n = 2LL * M * M;
  const double ad[4] = {a0, a1, a2, a3};
  double s = 0.0;
  for (int k = 0; k < DOT_PER_THREAD; ++k) {
    const int64_t e = (int64_t)blockIdx.x * 256 * DOT_PER_THREAD + k * 256 + threadIdx.x;
    if (e >= n) continue;
    const int q = (int)(e % ((int64_t)M * M)), a = q % M, b = q / M;
    if (!dom_u(N, dom, a, b)) continue;
    const double d = u[e] - us[e];
    s += enorm_ahat(N, dom, bh2, ad, a, b) * d * d;
  }
  const double t = block_sum<256>(s, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

// 1^T gp and sum |gp| over the domain's vertices (two partial arrays of nb
// entries): the data are compatible (int g = 0) when the first vanishes
__global__ __launch_bounds__(256) void k_psum_partial(int N, int dom, const double* __restrict__ gp,
                                                      double* partials, int nb) {
  __shared__ double red[4];
  const int n = (N + 1) * (N + 1);
  double s1 = 0.0, s2 = 0.0;
  for (int k = 0; k < 4; ++k) {
    const int e = blockIdx.x * 1024 + k * 256 + threadIdx.x;
    if (e < n && dom_p(N, dom, e % (N + 1), e / (N + 1))) {
      s1 += gp[e];
      s2 += fabs(gp[e]);
    }
  }
  const double t1 = block_sum<256>(s1, red);
  __syncthreads();
  const double t2 = block_sum<256>(s2, red);
  if (threadIdx.x == 0) {
    partials[blockIdx.x] = t1;
    partials[nb + blockIdx.x] = t2;
  }
}

void launch_psum(int N, int dom, const double* gp, double* red, double* out2, hipStream_t s) {
  const int nb = ((N + 1) * (N + 1) + 1023) / 1024;
  k_psum_partial<<<nb, 256, 0, s>>>(N, dom, gp, red, nb);
  k_reduce_final<<<1, 256, 0, s>>>(red, nb, out2);
  k_reduce_final<<<1, 256, 0, s>>>(red + nb, nb, out2 + 1);
}

int enorm_scratch(int N) { return std::max(dot_blocks(N, 0), 2 * ((N + 1) * (N + 1) + 1023) / 1024 + 2); }

// out[0..1]: mean pieces, out[2]: pressure part, out[3]: velocity part
void launch_error_norm(int N, int dom, double bh2, const double* ahat4, const double* sinv, const double* u,
                       const double* p, const double* us, const double* ps, double* red, double* out,
                       hipStream_t s) {
  const int nbp = ((N + 1) * (N + 1) + 1023) / 1024;
  k_enorm_p<<<nbp, 256, 0, s>>>(N, dom, 0, p, ps, sinv, nullptr, red, nbp);
  k_reduce_final<<<1, 256, 0, s>>>(red, nbp, out);
  k_reduce_final<<<1, 256, 0, s>>>(red + nbp, nbp, out + 1);
  k_enorm_p<<<nbp, 256, 0, s>>>(N, dom, 1, p, ps, sinv, out, red, nbp);
  k_reduce_final<<<1, 256, 0, s>>>(red, nbp, out + 2);
  const int nbu = dot_blocks(N, 0);
  k_enorm_u<<<nbu, 256, 0, s>>>(N, dom, bh2, ahat4[0], ahat4[1], ahat4[2], ahat4[3], u, us, red);
  k_reduce_final<<<1, 256, 0, s>>>(red, nbu, out + 3);
}

void launch_dot(int N, int dom, int which, const double* a, const double* b, double* partials,
                double* out, hipStream_t s) {
  const int nb = dot_blocks(N, which);
  k_dot_partial<<<nb, 256, 0, s>>>(N, dom, which, a, b, partials);
  k_reduce_final<<<1, 256, 0, s>>>(partials, nb, out);
}

__global__ __launch_bounds__(256) void k_check(const double* __restrict__ partials, int np,
                                               SolveState* st, double* hist) {
  if (st->done) return;
  __shared__ double red[4];
  double s = 0.0;
  for (int k = threadIdx.x; k < np; k += 256) s += partials[k];
  const double r2 = block_sum<256>(s, red);
  if (threadIdx.x == 0) {
    const double rel = sqrt(r2 / st->fnorm2);
    st->relres = rel;
    const int it = st->iters + 1;
    st->iters = it;
    if (hist) hist[it - 1] = rel;
    if (!(rel == rel) || rel > 1e300) st->done = 3;
    else if (r2 <= st->tol2 * st->fnorm2) st->done = 1;
    else if (rel > 1e6) st->done = 2;
    else if (it >= st->maxit) st->done = 4;
  }
}

void launch_check(const double* partials, int np, SolveState* st, double* hist, hipStream_t s) {
  k_check<<<1, 256, 0, s>>>(partials, np, st, hist);
}

__global__ __launch_bounds__(256) void k_init_state(const double* __restrict__ rpartials, int np,
                                                    const double* __restrict__ fdots,
                                                    SolveState* st) {
  __shared__ double red[4];
  double t = 0.0;
  for (int k = threadIdx.x; k < np; k += 256) t += rpartials[k];
  const double r2 = block_sum<256>(t, red);
  if (threadIdx.x == 0) {
    const double f2 = fdots[0] + fdots[1];
    st->fnorm2 = f2;
    st->iters = 0;
    st->relres = f2 > 0 ? sqrt(r2 / f2) : 0.0;
    st->done = (f2 == 0.0 || r2 <= st->tol2 * f2) ? 1 : 0;
    if (!(r2 == r2) || !(f2 == f2)) st->done = 3;
  }
}

void launch_init_state(const double* rpartials, int np, const double* fdots, SolveState* st,
                       hipStream_t s) {
  k_init_state<<<1, 256, 0, s>>>(rpartials, np, fdots, st);
}

// ---------------------------------------------------------------------------
// elementwise helpers
// ---------------------------------------------------------------------------

template <class T>
__global__ __launch_bounds__(256) void k_fill(T* x, int64_t n, T v) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < n) x[e] = v;
}
void launch_fill(double* x, int64_t n, double v, hipStream_t s) {
  if (n > 0) k_fill<double><<<(unsigned)((n + 255) / 256), 256, 0, s>>>(x, n, v);
}
void launch_fill_f32(float* x, int64_t n, float v, hipStream_t s) {
  if (n > 0) k_fill<float><<<(unsigned)((n + 255) / 256), 256, 0, s>>>(x, n, v);
}

__global__ __launch_bounds__(256) void k_axpy_f32(double* x, const float* __restrict__ d, int64_t n,
                                                  const int* done) {
  if (done && *done) return;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < n) x[e] += (double)d[e];
}
void launch_axpy_f32(double* x, const float* d, int64_t n, const int* done, hipStream_t s) {
  k_axpy_f32<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(x, d, n, done);
}

int ew_tiles(int64_t n) { return (int)((n + 1023) / 1024); }

template <bool PACK>
__global__ __launch_bounds__(256) void k_ew_b(const JobArg<EwJob> A, int mode) {
  int tile;
  const EwJob J = block_job<PACK>(A, (int)blockIdx.x, tile);
  if (J.done && *J.done) return;
  const int64_t base = (int64_t)tile * 1024;
  for (int k = 0; k < 4; ++k) {
    const int64_t e = base + k * 256 + threadIdx.x;
    if (e >= J.n) break;
    if (mode == 1) J.d[e] += (double)J.f[e];
    else J.d[e] = 0.0;
  }
}

void launch_ew_b(const JobArg<EwJob>& A, int nb, int mode, hipStream_t s) {
  if (A.n > 0) k_ew_b<true><<<nb, 256, 0, s>>>(A, mode);
  else k_ew_b<false><<<nb, 256, 0, s>>>(A, mode);
}

}  // namespace smg
