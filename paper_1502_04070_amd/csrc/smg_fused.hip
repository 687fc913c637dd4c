// Fused HIP kernels of the multigrid iterate (gfx950):
//
//   k_ne            one normal-equation smoothing step x <- x + tau L^-1 A L^-1 (F - A x)
//                   (Section 4) in one launch: the intermediate L^-1 (F - A x)
//                   lives only in LDS on the tile plus a halo of one square.
//                   Optionally the coarse-grid correction x += P z (Section 3)
//                   is applied to x while it is staged (the first
//                   post-smoothing step absorbs the prolongation).
//   k_ne2           two normal-equation steps in one launch on levels with
//                   8 x 8 tiles: every intermediate lives in LDS on the tile
//                   plus a halo that shrinks by one square per operator.
//   k_ne2rr         from a zero iterate, two normal-equation steps, the defect
//                   and its restriction in one launch (levels with 8 x 8 tiles).
//   k_ne_res        the last smoothing step of an FP64 iterate on the finest
//                   level together with the solve loop's residual pass (the
//                   residual norm and pressure mean pieces of the new iterate).
//   k_resid_restrict  the defect F - A x and its restriction P^T (F - A x)
//                   (Section 3) in one launch; the fine defect lives only in LDS.
//   k_coarse_cycle  the whole iterate on the coarse levels (N <= 8 by default)
//                   by one workgroup with every vector of those levels in LDS,
//                   including the exact solve on level 0.
//   k_project_partials, k_project_check  the pressure mean projection from
//                   the partial sums of the residual pass, and the
//                   convergence test by the last workgroup.
//
// Bandwidth: an unfused normal-equation step streams x, F and the
// intermediate twice (6 vectors); k_ne streams x and F once and writes x once
// (3 vectors); k_ne2 does two steps for the same three vectors.  k_resid_restrict reads x and F and writes a quarter-size
// coarse vector instead of writing and re-reading the fine defect.
#include <type_traits>

#include "smg_cell.h"
#include "smg_fused.h"

namespace smg {

// ---------------------------------------------------------------------------
// prolongation weights (canonical embedding of coarse P2 functions)
// ---------------------------------------------------------------------------

template <int RA, int RB, class T, class FZ>
__device__ __forceinline__ T pro_w(FZ Z) {
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

// P1 interpolation of coarse pressure zp (Nc+1 per side) at fine vertex (i, j)
template <class T>
__device__ __forceinline__ T pro_p1(const T* zp, int Nc, int i, int j) {
  const int NPc = Nc + 1;
  const int I = i >> 1, J = j >> 1;
  auto Z = [&](int a, int b) -> T { return zp[(size_t)b * NPc + a]; };
  if (!(i & 1) && !(j & 1)) return Z(I, J);
  if ((i & 1) && !(j & 1)) return T(0.5) * (Z(I, J) + Z(I + 1, J));
  if (!(i & 1) && (j & 1)) return T(0.5) * (Z(I, J) + Z(I, J + 1));
  return T(0.5) * (Z(I, J) + Z(I + 1, J + 1));
}

// the same on either grid (union jack: the table of the coarse square's
// diagonal direction)
template <int RA, int RB, class T, int DOM, class FZ>
__device__ __forceinline__ T sq_pro(int Nc, int I, int J, FZ Z) {
  if constexpr (DOM == SMG_DOM_UNIONJACK) {
    const int o = uj_orient_c(Nc, I, J);
    T v = T(0);
#pragma unroll
    for (int k = 0; k < 9; ++k) v += T(smg_stencil::UJ_PRO[o][4 * RB + RA][k]) * Z(k % 3, k / 3);
    return v;
  } else {
    return pro_w<RA, RB, T>(Z);
  }
}

template <class T, int DOM>
__device__ __forceinline__ T sq_pro_p1(const T* zp, int Nc, int i, int j) {
  if constexpr (DOM == SMG_DOM_UNIONJACK) {
    const int NPc = Nc + 1, I = i >> 1, J = j >> 1;
    const int o = uj_orient_c(Nc, I, J), v = 2 * (j & 1) + (i & 1);
    T z = T(0);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int ci = I + (q & 1), cj = J + (q >> 1);
      const double w = smg_stencil::UJ_PP[o][v][q];
      if (w != 0.0 && ci <= Nc && cj <= Nc) z += T(w) * zp[(size_t)cj * NPc + ci];
    }
    return z;
  } else {
    return pro_p1(zp, Nc, i, j);
  }
}

// The same split in two, so that the loads can be issued with the rest of a
// window before any is waited for: pro_p1_fetch reads the coarse values the
// fine vertex (i, j) needs (corners (I, J), (I+1, J), (I, J+1), (I+1, J+1) of
// its coarse square, zero where unused), pro_p1_value combines them with the
// same expressions as sq_pro_p1.
template <class T, int DOM>
__device__ __forceinline__ void pro_p1_fetch(const T* zp, int Nc, int i, int j, T z[4]) {
  const int NPc = Nc + 1, I = i >> 1, J = j >> 1;
  if constexpr (DOM == SMG_DOM_UNIONJACK) {
    const int o = uj_orient_c(Nc, I, J), v = 2 * (j & 1) + (i & 1);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int ci = I + (q & 1), cj = J + (q >> 1);
      z[q] = (smg_stencil::UJ_PP[o][v][q] != 0.0 && ci <= Nc && cj <= Nc) ? zp[(size_t)cj * NPc + ci] : T(0);
    }
  } else {
    z[0] = zp[(size_t)J * NPc + I];
    z[1] = ((i & 1) && !(j & 1)) ? zp[(size_t)J * NPc + I + 1] : T(0);
    z[2] = (!(i & 1) && (j & 1)) ? zp[(size_t)(J + 1) * NPc + I] : T(0);
    z[3] = ((i & 1) && (j & 1)) ? zp[(size_t)(J + 1) * NPc + I + 1] : T(0);
  }
}

template <class T, int DOM>
__device__ __forceinline__ T pro_p1_value(int Nc, int i, int j, const T z[4]) {
  if constexpr (DOM == SMG_DOM_UNIONJACK) {
    const int I = i >> 1, J = j >> 1;
    const int o = uj_orient_c(Nc, I, J), v = 2 * (j & 1) + (i & 1);
    T r = T(0);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int ci = I + (q & 1), cj = J + (q >> 1);
      const double w = smg_stencil::UJ_PP[o][v][q];
      if (w != 0.0 && ci <= Nc && cj <= Nc) r += T(w) * z[q];
    }
    return r;
  } else {
    if (!(i & 1) && !(j & 1)) return z[0];
    if ((i & 1) && !(j & 1)) return T(0.5) * (z[0] + z[1]);
    if (!(i & 1) && (j & 1)) return T(0.5) * (z[0] + z[2]);
    return T(0.5) * (z[0] + z[3]);
  }
}

// Window of the iterate alone on the same squares, staged.
template <class T, int TX, int TY, int H, int NT, int DOM>
struct XWindow {
  static constexpr int XW = 2 * TX + 4 * H, XH = 2 * TY + 4 * H;
  static constexpr int XPW = TX + 2 * H, XPH = TY + 2 * H;
  Staged<XW * XH, NT, 2, T> vel;
  Staged<XPW * XPH, NT, 1, T> pre;
  template <class J_>
  __device__ __forceinline__ void fetch(const J_& J, int i0, int j0, int tid) {
    const int N = J.L.N, M = 2 * N + 1, NP = N + 1;
    vel.fetch(tid, [&](int e, T* v) {
      const int a = 2 * i0 - 2 * H + e % XW, b = 2 * j0 - 2 * H + e / XW;
      const bool in = dom_u(N, DOM, a, b);
      const size_t g = (size_t)b * M + a;
      v[0] = in ? J.xu[g] : T(0);
      v[1] = in ? J.xu[(size_t)M * M + g] : T(0);
    });
    pre.fetch(tid, [&](int e, T* v) {
      const int i = i0 - H + e % XPW, j = j0 - H + e / XPW;
      v[0] = dom_p(N, DOM, i, j) ? J.xp[(size_t)j * NP + i] : T(0);
    });
  }
  __device__ __forceinline__ void put(int tid, T (*U)[XH][XW], T* P) const {
    vel.put(tid, [&](int e, const T* v) {
      U[0][e / XW][e % XW] = v[0];
      U[1][e / XW][e % XW] = v[1];
    });
    pre.put(tid, [&](int e, const T* v) { P[e] = v[0]; });
  }
};

// Window of the iterate plus the prolongated coarse correction, x + P z, on
// the same squares (H even).  fetch() requests the fine window and the coarse
// window of z that covers it; put() writes both to LDS (z to scratch arrays
// ZU[2][2 CH + 1][2 CW + 1] and ZP[(CH + 1) (CW + 1)] that the caller reuses
// later); after a barrier add() forms x + P z in the fine window, with the
// velocity items (coarse square of the window, component, fine row) of four
// fine points each (the fine row slowest, so that a wave mostly shares one
// row class) and the pressure items the window's vertices.  The coarse
// values stay in LDS rather than registers, which keeps the kernels free of
// spills.
template <class T, int TX, int TY, int H, int NT, int DOM>
struct ProWindow {
  static_assert(H % 2 == 0, "the window starts on a coarse square");
  static constexpr int CW = TX / 2 + H, CH = TY / 2 + H;       // coarse squares of the window
  static constexpr int ZW = 2 * CW + 1, ZH = 2 * CH + 1;       // coarse lattice of the window
  static constexpr int ZPW = CW + 1, ZPH = CH + 1;             // coarse vertices of the window
  static constexpr int XPW = TX + 2 * H, XPH = TY + 2 * H;
  XWindow<T, TX, TY, H, NT, DOM> x;
  Staged<ZW * ZH, NT, 2, T> zv;
  Staged<ZPW * ZPH, NT, 1, T> zpv;
  template <class J_>
  __device__ __forceinline__ void fetch(const J_& J, int i0, int j0, int tid) {
    x.fetch(J, i0, j0, tid);
    const int Nc = J.L.N / 2, Mc = 2 * Nc + 1, NPc = Nc + 1;
    // coarse lattice origin (i0 - H, j0 - H), coarse vertex origin ((i0 - H) / 2, (j0 - H) / 2)
    zv.fetch(tid, [&](int e, T* v) {
      const int A = i0 - H + e % ZW, B = j0 - H + e / ZW;
      const bool in = dom_u(Nc, DOM, A, B);
      const size_t g = (size_t)B * Mc + A;
      v[0] = in ? J.zu[g] : T(0);
      v[1] = in ? J.zu[(size_t)Mc * Mc + g] : T(0);
    });
    zpv.fetch(tid, [&](int e, T* v) {
      const int I = (i0 - H) / 2 + e % ZPW, Jc = (j0 - H) / 2 + e / ZPW;
      v[0] = (I >= 0 && Jc >= 0 && I <= Nc && Jc <= Nc) ? J.zp[(size_t)Jc * NPc + I] : T(0);
    });
  }
  template <int XW, int XH>
  __device__ __forceinline__ void put(int tid, T (*U)[XH][XW], T* P, T* ZU, T* ZP) const {
    x.put(tid, U, P);
    zv.put(tid, [&](int e, const T* v) {
      ZU[e] = v[0];
      ZU[ZW * ZH + e] = v[1];
    });
    zpv.put(tid, [&](int e, const T* v) { ZP[e] = v[0]; });
  }
  template <int XW, int XH>
  __device__ __forceinline__ void add(int N, int i0, int j0, int tid, T (*U)[XH][XW], T* P, const T* ZU,
                                      const T* ZP) const {
    const int Nc = N / 2;
    auto interior = [&](int a, int bb) { return dom_u(N, DOM, a, bb); };
    for (int e = tid; e < CW * CH * 8; e += NT) {
      const int rb = e / (2 * CW * CH), rem = e % (2 * CW * CH);
      const int c = rem / (CW * CH), cell = rem % (CW * CH);
      const int ci = cell % CW, cj = cell / CW;
      const int I = i0 / 2 - H / 2 + ci, Jc = j0 / 2 - H / 2 + cj;
      const T* zc = ZU + c * ZW * ZH + (2 * cj) * ZW + 2 * ci;
      auto Z = [&](int dA, int dB) -> T { return zc[dB * ZW + dA]; };
      const int b = 4 * Jc + rb;
      T* row = &U[c][4 * cj + rb][4 * ci];
      T w[4] = {row[0], row[1], row[2], row[3]};
      switch (rb) {
#define SMG_ROW(RB)                                                              \
  case RB:                                                                       \
    if (interior(4 * I + 0, b)) w[0] += sq_pro<0, RB, T, DOM>(Nc, I, Jc, Z);    \
    if (interior(4 * I + 1, b)) w[1] += sq_pro<1, RB, T, DOM>(Nc, I, Jc, Z);    \
    if (interior(4 * I + 2, b)) w[2] += sq_pro<2, RB, T, DOM>(Nc, I, Jc, Z);    \
    if (interior(4 * I + 3, b)) w[3] += sq_pro<3, RB, T, DOM>(Nc, I, Jc, Z);    \
    break;
        SMG_ROW(0) SMG_ROW(1) SMG_ROW(2) SMG_ROW(3)
#undef SMG_ROW
      }
#pragma unroll
      for (int ra = 0; ra < 4; ++ra) row[ra] = w[ra];
    }
    for (int e = tid; e < XPW * XPH; e += NT) {
      const int i = i0 - H + e % XPW, j = j0 - H + e / XPW;
      if (!dom_p(N, DOM, i, j)) continue;
      const int li = (i >> 1) - (i0 - H) / 2, lj = (j >> 1) - (j0 - H) / 2;
      const T z[4] = {ZP[lj * ZPW + li], ZP[lj * ZPW + li + 1], ZP[(lj + 1) * ZPW + li],
                      ZP[(lj + 1) * ZPW + li + 1]};
      P[e] += pro_p1_value<T, DOM>(Nc, i, j, z);
    }
  }
};

// ---------------------------------------------------------------------------
// k_ne: one fused normal-equation step on a TX x TY tile of squares
// ---------------------------------------------------------------------------

template <class T, int TX, int TY, bool ZG, bool PRO, int DOM>
__device__ __forceinline__ void ne_tile(const NEJob<T>& J, int tile) {
  constexpr int NT = 2 * TX * TY;
  constexpr int XW = 2 * TX + 8, XH = 2 * TY + 8;      // x: lattice origin (2 i0 - 4, 2 j0 - 4)
  constexpr int XPW = TX + 4, XPH = TY + 4;            // x pressure: origin (i0 - 2, j0 - 2)
  constexpr int YW = 2 * TX + 4, YH = 2 * TY + 4;      // y: lattice origin (2 i0 - 2, 2 j0 - 2)
  constexpr int YPW = TX + 2, YPH = TY + 2;            // y pressure: origin (i0 - 1, j0 - 1)
  __shared__ T sx[2][XH][XW];
  __shared__ T sxp[XPH * XPW];
  __shared__ T sy[2][YH][YW];
  __shared__ T syp[YPH * YPW];
  __shared__ double red[NT / 64];
  const int N = J.L.N, M = 2 * N + 1, NP = N + 1;
  const int ntx = (N + TX) / TX;
  const int i0 = (tile % ntx) * TX, j0 = (tile / ntx) * TY;
  const int tid = threadIdx.x;
  auto interior = [&](int a, int b) { return dom_u(N, DOM, a, b); };

  // Every global input the workgroup needs is requested before the first
  // wait: the done flag, this thread's stage-1 right-hand side and Shat^-1
  // (one stage-1 square per thread) and its stage-2 Shat^-1, then the
  // iterate window.  The flag is tested once the window is in LDS.
  static_assert((TX + 2) * (TY + 2) <= NT, "one stage-1 square per thread");
  const int dn = J.done ? *J.done : 0;
  const int c1i = tid % (TX + 2), c1j = tid / (TX + 2);
  const int i1 = i0 - 1 + c1i, j1 = j0 - 1 + c1j;
  const bool act1 = tid < (TX + 2) * (TY + 2);
  T f1[9], s1 = T(0);
#pragma unroll
  for (int cls = 0; cls < 4; ++cls) {
    const int a = 2 * i1 + (cls & 1), b = 2 * j1 + (cls >> 1);
    const bool in = act1 && interior(a, b);
#pragma unroll
    for (int c = 0; c < 2; ++c) f1[2 * cls + c] = in ? J.fu[(size_t)c * M * M + (size_t)b * M + a] : T(0);
  }
  const bool inp1 = act1 && dom_p(N, DOM, i1, j1);
  f1[8] = inp1 ? J.fp[(size_t)j1 * NP + i1] : T(0);
  if (inp1) s1 = J.L.sinv[(size_t)j1 * NP + i1];
  T s2 = T(0);
  {
    const int q = tid % (TX * TY), i = i0 + q % TX, j = j0 + q / TX;
    if (tid >= TX * TY && i <= N && j <= N) s2 = J.L.sinv[(size_t)j * NP + i];
  }

  // ---- stage 0: the iterate (plus the prolongated coarse correction with
  // PRO) on the tile plus two squares of halo, every load in flight at once
  if constexpr (!ZG) {
    if constexpr (PRO) {
      // the coarse window of z goes to the storage of y (written in stage 1)
      using PW = ProWindow<T, TX, TY, 2, NT, DOM>;
      static_assert(2 * PW::ZW * PW::ZH <= 2 * YH * YW && PW::ZPW * PW::ZPH <= YPH * YPW, "z window fits");
      PW w;
      w.fetch(J, i0, j0, tid);
      w.put(tid, sx, sxp, &sy[0][0][0], syp);
      __syncthreads();
      w.add(N, i0, j0, tid, sx, sxp, &sy[0][0][0], syp);
    } else {
      XWindow<T, TX, TY, 2, NT, DOM> w;
      w.fetch(J, i0, j0, tid);
      w.put(tid, sx, sxp);
    }
    __syncthreads();
  }

  if (dn) return;   // uniform across the workgroup

  // ---- stage 1: y = L^-1 (F - A x) on the tile plus one square of halo
  double nrm = 0.0;
  if (act1) {
    const int ci = c1i, cj = c1j, i = i1, j = j1;
    T y[9], ad[4];
    auto UA = [&](int c, int da, int db) -> T { return sx[c][2 * cj + 2 + db][2 * ci + 2 + da]; };
    auto PA = [&](int di, int dj) -> T { return sxp[(cj + 1 + dj) * XPW + (ci + 1 + di)]; };
    if constexpr (ZG) sq_rows<T, false, false, DOM>(J.L, i, j, UA, PA, y, ad);
    else sq_rows<T, true, true, DOM>(J.L, i, j, UA, PA, y, ad);
    const bool owned = ci >= 1 && ci <= TX && cj >= 1 && cj <= TY;
#pragma unroll
    for (int cls = 0; cls < 4; ++cls) {
      const int DA = cls & 1, DB = cls >> 1;
      const int a = 2 * i + DA, b = 2 * j + DB;
      const bool in = interior(a, b);
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        T r = T(0);
        if (in) r = f1[2 * cls + c] - y[2 * cls + c];
        if (owned && in) nrm += (double)r * (double)r;
        sy[c][2 * cj + DB][2 * ci + DA] = in ? ad[cls] * r : T(0);
      }
    }
    T rp = T(0);
    if (inp1) rp = f1[8] - y[8];
    if (owned && inp1) nrm += (double)rp * (double)rp;
    syp[cj * YPW + ci] = inp1 ? s1 * rp : T(0);
  }
  __syncthreads();

  // ---- stage 2: x_new = x + tau L^-1 A y on the tile; two threads per square
  {
    const int half = TX * TY;
    const int part = tid / half, q = tid % half;
    const int tx = q % TX, ty = q / TX;
    const int i = i0 + tx, j = j0 + ty;
    if (i <= N && j <= N) {
      auto UA = [&](int c, int da, int db) -> T { return sy[c][2 * ty + 2 + db][2 * tx + 2 + da]; };
      auto PA = [&](int di, int dj) -> T { return syp[(ty + 1 + dj) * YPW + (tx + 1 + di)]; };
      const T tau = J.tau;
      auto emit = [&](int cls, T z0, T z1, T ad) {
        const int DA = cls & 1, DB = cls >> 1;
        const int a = 2 * i + DA, b = 2 * j + DB;
        if (a > 2 * N || b > 2 * N) return;
        const bool in = interior(a, b);
        const size_t g = (size_t)b * M + a;
        T x0 = T(0), x1 = T(0);
        if constexpr (!ZG) {
          x0 = sx[0][2 * ty + 4 + DB][2 * tx + 4 + DA];
          x1 = sx[1][2 * ty + 4 + DB][2 * tx + 4 + DA];
        }
        const T d = ad * tau;
        if constexpr (std::is_same<T, float>::value) {
          if (J.acc_u) {
            // x64 += the new FP32 iterate (zero off the domain: nothing to add)
            if (in) {
              J.acc_u[g] += (double)(x0 + d * z0);
              J.acc_u[(size_t)M * M + g] += (double)(x1 + d * z1);
            }
            return;
          }
        }
        J.ou[g] = in ? x0 + d * z0 : T(0);
        J.ou[(size_t)M * M + g] = in ? x1 + d * z1 : T(0);
      };
      T z0, z1, ad;
      if (part == 0) {
        sq_vel<0, T, true, true, DOM>(J.L, i, j, UA, PA, z0, z1, ad);
        emit(0, z0, z1, ad);
        sq_vel<1, T, true, true, DOM>(J.L, i, j, UA, PA, z0, z1, ad);
        emit(1, z0, z1, ad);
      } else {
        sq_vel<2, T, true, true, DOM>(J.L, i, j, UA, PA, z0, z1, ad);
        emit(2, z0, z1, ad);
        sq_vel<3, T, true, true, DOM>(J.L, i, j, UA, PA, z0, z1, ad);
        emit(3, z0, z1, ad);
        const T zp = sq_prow<T, DOM>(J.L, i, j, UA);
        const size_t g = (size_t)j * NP + i;
        T xo = T(0);
        if constexpr (!ZG) xo = sxp[(ty + 2) * XPW + tx + 2];
        if constexpr (std::is_same<T, float>::value) {
          if (J.acc_p) J.acc_p[g] += (double)(xo + tau * s2 * zp);
          else J.op[g] = xo + tau * s2 * zp;
        } else {
          J.op[g] = xo + tau * s2 * zp;
        }
      }
    }
  }
  if (J.partial) {
    const double s = wg_sum<NT>(nrm, red);
    if (tid == 0) J.partial[tile] = s;
  }
}

// The domain is a template parameter of every fused kernel (chosen by the
// host launchers): a run-time test would cost the square's kernels a few
// percent, and two instantiations inside one kernel would double its static
// LDS.
template <class T, int TX, int TY, bool ZG, bool PRO, int DOM>
__global__ __launch_bounds__(2 * TX* TY) void k_ne(NEJob<T> J) {
  ne_tile<T, TX, TY, ZG, PRO, DOM>(J, xcd_remap(blockIdx.x, gridDim.x));
}

template <class T, int TX, int TY, bool ZG, bool PRO, bool PACK, int DOM>
__global__ __launch_bounds__(2 * TX* TY) void k_ne_b(const JobArg<NEJob<T>> A) {
  int tile;
  const NEJob<T> J = block_job<PACK>(A, xcd_remap(blockIdx.x, gridDim.x), tile);
  ne_tile<T, TX, TY, ZG, PRO, DOM>(J, tile);
}

template <class T, int TX, int TY, bool PACK, int DOM>
static void launch_ne_b_shape(const JobArg<NEJob<T>>& A, int nb, bool zg, bool pro, hipStream_t s) {
  if (zg) k_ne_b<T, TX, TY, true, false, PACK, DOM><<<nb, 2 * TX * TY, 0, s>>>(A);
  else if (pro) k_ne_b<T, TX, TY, false, true, PACK, DOM><<<nb, 2 * TX * TY, 0, s>>>(A);
  else k_ne_b<T, TX, TY, false, false, PACK, DOM><<<nb, 2 * TX * TY, 0, s>>>(A);
}

template <class T, int DOM>
static void launch_ne_b_dom(const JobArg<NEJob<T>>& A, int nb, int tx, bool zg, bool pro, hipStream_t s) {
  if (tx == 16) {
    if (A.n > 0) launch_ne_b_shape<T, 16, 8, true, DOM>(A, nb, zg, pro, s);
    else launch_ne_b_shape<T, 16, 8, false, DOM>(A, nb, zg, pro, s);
  } else {
    if (A.n > 0) launch_ne_b_shape<T, 8, 8, true, DOM>(A, nb, zg, pro, s);
    else launch_ne_b_shape<T, 8, 8, false, DOM>(A, nb, zg, pro, s);
  }
}

template <class T>
void launch_ne_b(const JobArg<NEJob<T>>& A, int nb, int tx, bool zg, bool pro, int dom, hipStream_t s) {
  if (dom == SMG_DOM_LSHAPE) launch_ne_b_dom<T, SMG_DOM_LSHAPE>(A, nb, tx, zg, pro, s);
  else if (dom == SMG_DOM_UNIONJACK) launch_ne_b_dom<T, SMG_DOM_UNIONJACK>(A, nb, tx, zg, pro, s);
  else launch_ne_b_dom<T, SMG_DOM_SQUARE>(A, nb, tx, zg, pro, s);
}
template void launch_ne_b<double>(const JobArg<NEJob<double>>&, int, int, bool, bool, int, hipStream_t);
template void launch_ne_b<float>(const JobArg<NEJob<float>>&, int, int, bool, bool, int, hipStream_t);

TileShape ne_tile_shape(int N) {
  if (N >= 128) return {16, 8};
  return {8, 8};
}

int ne_tiles(int N) {
  const TileShape t = ne_tile_shape(N);
  return ((N + t.tx) / t.tx) * ((N + t.ty) / t.ty);
}

template <class T, int TX, int TY, int DOM>
static void launch_ne_shape(const NEJob<T>& J, bool zg, bool pro, hipStream_t s) {
  const int nb = ((J.L.N + TX) / TX) * ((J.L.N + TY) / TY);
  if (zg)
    k_ne<T, TX, TY, true, false, DOM><<<nb, 2 * TX * TY, 0, s>>>(J);
  else if (pro)
    k_ne<T, TX, TY, false, true, DOM><<<nb, 2 * TX * TY, 0, s>>>(J);
  else
    k_ne<T, TX, TY, false, false, DOM><<<nb, 2 * TX * TY, 0, s>>>(J);
}

template <class T, int DOM>
static void launch_ne_dom(const NEJob<T>& J, bool zg, bool pro, int tx, hipStream_t s) {
  if ((tx ? tx : ne_tile_shape(J.L.N).tx) == 16)
    launch_ne_shape<T, 16, 8, DOM>(J, zg, pro, s);
  else
    launch_ne_shape<T, 8, 8, DOM>(J, zg, pro, s);
}

template <class T>
void launch_ne(const NEJob<T>& J, bool zg, bool pro, int tx, hipStream_t s) {
  if (J.L.dom == SMG_DOM_LSHAPE) launch_ne_dom<T, SMG_DOM_LSHAPE>(J, zg, pro, tx, s);
  else if (J.L.dom == SMG_DOM_UNIONJACK) launch_ne_dom<T, SMG_DOM_UNIONJACK>(J, zg, pro, tx, s);
  else launch_ne_dom<T, SMG_DOM_SQUARE>(J, zg, pro, tx, s);
}
template void launch_ne<double>(const NEJob<double>&, bool, bool, int, hipStream_t);
template void launch_ne<float>(const NEJob<float>&, bool, bool, int, hipStream_t);


// ---------------------------------------------------------------------------
// k_ne_res: the last smoothing step on the finest level together with the
// residual pass of the solve loop.  Stage 0 loads x on the tile + 3 squares;
// stage 1 writes y = L^-1 (F - A x) on the tile + 2; stage 2 forms
// x_new = x + tau L^-1 A y on the tile + 1 (one thread per square, all nine
// rows, the same expressions as k_ne) and writes it over x in LDS (each
// thread reads and writes only its own square's points there) and, on the
// tile, to memory; stage 3 forms F - A x_new on the tile for ||r||^2 and the
// pressure mean pieces of x_new.  16 x 8 tiles, 256 threads.
// ---------------------------------------------------------------------------

template <class T, int DOM>
__device__ __forceinline__ void ne_res_tile(const NEJob<T>& J, int tile) {
  constexpr int TX = 16, TY = 8, NT = 2 * TX * TY;
  using XWn = XWindow<T, TX, TY, 3, NT, DOM>;
  constexpr int XW = XWn::XW, XH = XWn::XH;       // x: lattice origin (2 i0 - 6, 2 j0 - 6)
  constexpr int XPW = XWn::XPW, XPH = XWn::XPH;   // x pressure: origin (i0 - 3, j0 - 3)
  constexpr int YW = 2 * TX + 8, YH = 2 * TY + 8; // y: lattice origin (2 i0 - 4, 2 j0 - 4)
  constexpr int YPW = TX + 4, YPH = TY + 4;       // y pressure: origin (i0 - 2, j0 - 2)
  constexpr int C1W = TX + 4, C1H = TY + 4;       // stage-1 squares (tile + 2)
  constexpr int C2W = TX + 2, C2H = TY + 2;       // stage-2 squares (tile + 1)
  static_assert(C1W * C1H <= NT && C2W * C2H <= NT, "one stage-1 and one stage-2 square per thread");
  __shared__ T sx[2][XH][XW];
  __shared__ T sxp[XPH * XPW];
  __shared__ T sy[2][YH][YW];
  __shared__ T syp[YPH * YPW];
  __shared__ double red[NT / 64];
  const int N = J.L.N, M = 2 * N + 1, NP = N + 1;
  const int ntx = (N + TX) / TX;
  const int i0 = (tile % ntx) * TX, j0 = (tile / ntx) * TY;
  const int tid = threadIdx.x;
  const T tau = J.tau;
  auto interior = [&](int a, int b) { return dom_u(N, DOM, a, b); };

  // every global input requested before the first wait: the done flag,
  // the stage-1 right-hand side and Shat^-1, the stage-2 Shat^-1, the
  // stage-3 right-hand side (two threads per owned square: classes 0, 1 /
  // classes 2, 3 and the pressure row), then the iterate window
  const int dn = J.done ? *J.done : 0;
  const int c1i = tid % C1W, c1j = tid / C1W;
  const int i1 = i0 - 2 + c1i, j1 = j0 - 2 + c1j;
  const bool act1 = tid < C1W * C1H;
  T f1[9], s1 = T(0);
#pragma unroll
  for (int cls = 0; cls < 4; ++cls) {
    const int a = 2 * i1 + (cls & 1), b = 2 * j1 + (cls >> 1);
    const bool in = act1 && interior(a, b);
#pragma unroll
    for (int c = 0; c < 2; ++c) f1[2 * cls + c] = in ? J.fu[(size_t)c * M * M + (size_t)b * M + a] : T(0);
  }
  const bool inp1 = act1 && dom_p(N, DOM, i1, j1);
  f1[8] = inp1 ? J.fp[(size_t)j1 * NP + i1] : T(0);
  if (inp1) s1 = J.L.sinv[(size_t)j1 * NP + i1];
  const int c2i = tid % C2W, c2j = tid / C2W;
  const int i2 = i0 - 1 + c2i, j2 = j0 - 1 + c2j;
  const bool act2 = tid < C2W * C2H && i2 >= 0 && j2 >= 0 && i2 <= N && j2 <= N;
  T s2 = T(0);
  if (act2) s2 = J.L.sinv[(size_t)j2 * NP + i2];
  const int part = tid / (TX * TY), q3 = tid % (TX * TY);
  const int t3x = q3 % TX, t3y = q3 / TX;
  const int i3 = i0 + t3x, j3 = j0 + t3y;
  const bool own3 = i3 <= N && j3 <= N;
  T f3[5];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int cls = 2 * part + k, a = 2 * i3 + (cls & 1), b = 2 * j3 + (cls >> 1);
    const bool in = own3 && a <= 2 * N && b <= 2 * N && interior(a, b);
#pragma unroll
    for (int c = 0; c < 2; ++c) f3[2 * k + c] = in ? J.fu[(size_t)c * M * M + (size_t)b * M + a] : T(0);
  }
  f3[4] = (part == 1 && own3 && dom_p(N, DOM, i3, j3)) ? J.fp[(size_t)j3 * NP + i3] : T(0);
  {
    XWn w;
    w.fetch(J, i0, j0, tid);
    w.put(tid, sx, sxp);
  }
  __syncthreads();
  if (dn) return;   // uniform across the workgroup

  // ---- stage 1: y = L^-1 (F - A x) on the tile + 2
  if (act1) {
    T y[9], ad[4];
    auto UA = [&](int c, int da, int db) -> T { return sx[c][2 * c1j + 2 + db][2 * c1i + 2 + da]; };
    auto PA = [&](int di, int dj) -> T { return sxp[(c1j + 1 + dj) * XPW + (c1i + 1 + di)]; };
    sq_rows<T, true, true, DOM>(J.L, i1, j1, UA, PA, y, ad);
#pragma unroll
    for (int cls = 0; cls < 4; ++cls) {
      const int DA = cls & 1, DB = cls >> 1;
      const int a = 2 * i1 + DA, b = 2 * j1 + DB;
      const bool in = interior(a, b);
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        T r = T(0);
        if (in) r = f1[2 * cls + c] - y[2 * cls + c];
        sy[c][2 * c1j + DB][2 * c1i + DA] = in ? ad[cls] * r : T(0);
      }
    }
    T rp = T(0);
    if (inp1) rp = f1[8] - y[8];
    syp[c1j * YPW + c1i] = inp1 ? s1 * rp : T(0);
  }
  __syncthreads();

  // ---- stage 2: x_new = x + tau L^-1 A y on the tile + 1, over x in LDS
  if (act2) {
    auto UA = [&](int c, int da, int db) -> T { return sy[c][2 * c2j + 2 + db][2 * c2i + 2 + da]; };
    auto PA = [&](int di, int dj) -> T { return syp[(c2j + 1 + dj) * YPW + (c2i + 1 + di)]; };
    const bool mine = c2i >= 1 && c2i <= TX && c2j >= 1 && c2j <= TY;
    auto emit = [&](int cls, T z0, T z1, T ad) {
      const int DA = cls & 1, DB = cls >> 1;
      const int a = 2 * i2 + DA, b = 2 * j2 + DB;
      if (a > 2 * N || b > 2 * N) return;
      const bool in = interior(a, b);
      T& x0 = sx[0][2 * c2j + 4 + DB][2 * c2i + 4 + DA];
      T& x1 = sx[1][2 * c2j + 4 + DB][2 * c2i + 4 + DA];
      const T d = ad * tau;
      const T v0 = in ? x0 + d * z0 : T(0);
      const T v1 = in ? x1 + d * z1 : T(0);
      x0 = v0;
      x1 = v1;
      if (mine) {
        const size_t g = (size_t)b * M + a;
        J.ou[g] = v0;
        J.ou[(size_t)M * M + g] = v1;
      }
    };
    T z0, z1, ad;
    sq_vel<0, T, true, true, DOM>(J.L, i2, j2, UA, PA, z0, z1, ad);
    emit(0, z0, z1, ad);
    sq_vel<1, T, true, true, DOM>(J.L, i2, j2, UA, PA, z0, z1, ad);
    emit(1, z0, z1, ad);
    sq_vel<2, T, true, true, DOM>(J.L, i2, j2, UA, PA, z0, z1, ad);
    emit(2, z0, z1, ad);
    sq_vel<3, T, true, true, DOM>(J.L, i2, j2, UA, PA, z0, z1, ad);
    emit(3, z0, z1, ad);
    const T zp = sq_prow<T, DOM>(J.L, i2, j2, UA);
    T& xo = sxp[(c2j + 2) * XPW + c2i + 2];
    const T vp = xo + tau * s2 * zp;
    xo = vp;
    if (mine) J.op[(size_t)j2 * NP + i2] = vp;
  }
  __syncthreads();

  // ---- stage 3: F - A x_new on the tile (two threads per square), the
  // residual norm over the owned rows and the pressure mean pieces of x_new
  double nrm = 0.0, wp = 0.0, w = 0.0;
  if (own3) {
    auto UA = [&](int c, int da, int db) -> T { return sx[c][2 * t3y + 6 + db][2 * t3x + 6 + da]; };
    auto PA = [&](int di, int dj) -> T { return sxp[(t3y + 3 + dj) * XPW + (t3x + 3 + di)]; };
    auto res = [&](int k, int cls, T z0, T z1) {
      const int DA = cls & 1, DB = cls >> 1;
      const int a = 2 * i3 + DA, b = 2 * j3 + DB;
      if (a > 2 * N || b > 2 * N || !interior(a, b)) return;
      const T r0 = f3[2 * k] - z0, r1 = f3[2 * k + 1] - z1;
      nrm += (double)r0 * (double)r0;
      nrm += (double)r1 * (double)r1;
    };
    T z0, z1, ad;
    if (part == 0) {
      sq_vel<0, T, true, true, DOM>(J.L, i3, j3, UA, PA, z0, z1, ad);
      res(0, 0, z0, z1);
      sq_vel<1, T, true, true, DOM>(J.L, i3, j3, UA, PA, z0, z1, ad);
      res(1, 1, z0, z1);
    } else {
      sq_vel<2, T, true, true, DOM>(J.L, i3, j3, UA, PA, z0, z1, ad);
      res(0, 2, z0, z1);
      sq_vel<3, T, true, true, DOM>(J.L, i3, j3, UA, PA, z0, z1, ad);
      res(1, 3, z0, z1);
      if (dom_p(N, DOM, i3, j3)) {
        const T rp = f3[4] - sq_prow<T, DOM>(J.L, i3, j3, UA);
        nrm += (double)rp * (double)rp;
      }
      w = p1_count_w(N, DOM, i3, j3);
      wp = w * (double)sxp[(t3y + 3) * XPW + t3x + 3];
    }
  }
  if (J.partial) {
    const double s = wg_sum<NT>(nrm, red);
    if (tid == 0) J.partial[tile] = s;
  }
  if (J.mean_partial) {
    __syncthreads();
    const double sw = wg_sum<NT>(wp, red);
    __syncthreads();
    const double s0 = wg_sum<NT>(w, red);
    if (tid == 0) {
      J.mean_partial[2 * tile] = sw;
      J.mean_partial[2 * tile + 1] = s0;
    }
  }
}

template <int DOM>
__global__ __launch_bounds__(256) void k_ne_res(NEJob<double> J) {
  ne_res_tile<double, DOM>(J, xcd_remap(blockIdx.x, gridDim.x));
}

template <bool PACK, int DOM>
__global__ __launch_bounds__(256) void k_ne_res_b(const JobArg<NEJob<double>> A) {
  int tile;
  const NEJob<double> J = block_job<PACK>(A, xcd_remap(blockIdx.x, gridDim.x), tile);
  ne_res_tile<double, DOM>(J, tile);
}

void launch_ne_res(const NEJob<double>& J, hipStream_t s) {
  const int nb = ((J.L.N + 16) / 16) * ((J.L.N + 8) / 8);
  if (J.L.dom == SMG_DOM_LSHAPE) k_ne_res<SMG_DOM_LSHAPE><<<nb, 256, 0, s>>>(J);
  else if (J.L.dom == SMG_DOM_UNIONJACK) k_ne_res<SMG_DOM_UNIONJACK><<<nb, 256, 0, s>>>(J);
  else k_ne_res<SMG_DOM_SQUARE><<<nb, 256, 0, s>>>(J);
}

template <int DOM>
static void launch_ne_res_b_dom(const JobArg<NEJob<double>>& A, int nb, hipStream_t s) {
  if (A.n > 0) k_ne_res_b<true, DOM><<<nb, 256, 0, s>>>(A);
  else k_ne_res_b<false, DOM><<<nb, 256, 0, s>>>(A);
}

void launch_ne_res_b(const JobArg<NEJob<double>>& A, int nb, int dom, hipStream_t s) {
  if (dom == SMG_DOM_LSHAPE) launch_ne_res_b_dom<SMG_DOM_LSHAPE>(A, nb, s);
  else if (dom == SMG_DOM_UNIONJACK) launch_ne_res_b_dom<SMG_DOM_UNIONJACK>(A, nb, s);
  else launch_ne_res_b_dom<SMG_DOM_SQUARE>(A, nb, s);
}

// ---------------------------------------------------------------------------
// k_ne2: two fused normal-equation steps on a TX x TY tile of squares
// ---------------------------------------------------------------------------
// Applying calA on a set of squares needs its argument on the points owned by
// that set plus one square around it.  The second step's result on the tile
// therefore needs the first step's result on the tile plus two squares (X1),
// the first scaled residual on the tile plus three (Y1) and the iterate on the
// tile plus four (X0); F and Shat^-1 are staged on the tile plus three.  The
// second residual (Y2, tile plus one) reuses Y1's storage.  Every window is a
// lattice of the points owned by its squares, zero outside the interior of the
// velocity space and outside the grid.  Each value is computed by the same
// expressions as in two single steps.

template <class T, int TX, int TY, bool ZG, bool PRO, int DOM>
__device__ __forceinline__ void ne2_tile(const NEJob<T>& J, int tile) {
  constexpr int NT = 4 * TX * TY;
  constexpr int W4 = 2 * TX + 16, H4 = 2 * TY + 16, PW4 = TX + 8, PH4 = TY + 8;   // X0: tile + 4
  constexpr int W3 = 2 * TX + 12, H3 = 2 * TY + 12, PW3 = TX + 6, PH3 = TY + 6;   // F, Y1, Shat^-1: + 3
  constexpr int W2 = 2 * TX + 8, H2 = 2 * TY + 8, PW2 = TX + 4, PH2 = TY + 4;     // X1: + 2
  constexpr int W1 = 2 * TX + 4, H1 = 2 * TY + 4, PW1 = TX + 2;                   // Y2: + 1
  static_assert((TX + 6) * (TY + 6) <= NT, "one stage-1 square per thread");
  __shared__ T sx0[ZG ? 1 : 2][ZG ? 1 : H4][ZG ? 1 : W4];
  __shared__ T sx0p[ZG ? 1 : PH4 * PW4];
  __shared__ T sf[2][H3][W3];
  __shared__ T sfp[PH3 * PW3];
  __shared__ T ss[PH3 * PW3];
  __shared__ T sy[2][H3][W3];
  __shared__ T syp[PH3 * PW3];
  __shared__ T sx1[2][H2][W2];
  __shared__ T sx1p[PH2 * PW2];
  const int N = J.L.N, M = 2 * N + 1, NP = N + 1;
  const int ntx = (N + TX) / TX;
  const int i0 = (tile % ntx) * TX, j0 = (tile / ntx) * TY;
  const int tid = threadIdx.x;
  const T tau = J.tau;
  auto interior = [&](int a, int b) { return dom_u(N, DOM, a, b); };
  auto inside = [&](int i, int j) { return dom_p(N, DOM, i, j); };

  // ---- stage 0: F and Shat^-1 on the tile + 3, the iterate on the tile + 4,
  // every load in flight at once
  const int dn = J.done ? *J.done : 0;
  Staged<W3 * H3, NT, 2, T> fw;
  Staged<PW3 * PH3, NT, 2, T> fpw;
  fw.fetch(tid, [&](int e, T* v) {
    const int a = 2 * i0 - 6 + e % W3, b = 2 * j0 - 6 + e / W3;
    const bool in = interior(a, b);
    const size_t g = (size_t)b * M + a;
    v[0] = in ? J.fu[g] : T(0);
    v[1] = in ? J.fu[(size_t)M * M + g] : T(0);
  });
  fpw.fetch(tid, [&](int e, T* v) {
    const int i = i0 - 3 + e % PW3, j = j0 - 3 + e / PW3;
    const bool ok = inside(i, j);
    v[0] = ok ? J.fp[(size_t)j * NP + i] : T(0);
    v[1] = ok ? J.L.sinv[(size_t)j * NP + i] : T(0);
  });
  using PW = ProWindow<T, TX, TY, 4, NT, DOM>;
  std::conditional_t<PRO, PW, XWindow<T, TX, TY, 4, NT, DOM>> xw;
  if constexpr (!ZG) xw.fetch(J, i0, j0, tid);
  fw.put(tid, [&](int e, const T* v) {
    sf[0][e / W3][e % W3] = v[0];
    sf[1][e / W3][e % W3] = v[1];
  });
  fpw.put(tid, [&](int e, const T* v) {
    sfp[e] = v[0];
    ss[e] = v[1];
  });
  if constexpr (!ZG) {
    if constexpr (PRO) {
      // the coarse window of z goes to the storage of Y1 (written in stage 1)
      static_assert(2 * PW::ZW * PW::ZH <= 2 * H3 * W3 && PW::ZPW * PW::ZPH <= PH3 * PW3, "z window fits");
      xw.put(tid, sx0, sx0p, &sy[0][0][0], syp);
      __syncthreads();
      xw.add(N, i0, j0, tid, sx0, sx0p, &sy[0][0][0], syp);
    } else {
      xw.put(tid, sx0, sx0p);
    }
  }
  __syncthreads();
  if (dn) return;   // uniform across the workgroup

  // ---- stage 1: Y1 = L^-1 (F - A X0) on the tile + 3
  for (int e = tid; e < (TX + 6) * (TY + 6); e += NT) {
    const int ci = e % (TX + 6), cj = e / (TX + 6);
    const int i = i0 - 3 + ci, j = j0 - 3 + cj;
    T y[9], ad[4];
    auto UA = [&](int c, int da, int db) -> T {
      if constexpr (ZG) return T(0);
      else return sx0[c][2 * cj + 2 + db][2 * ci + 2 + da];
    };
    auto PA = [&](int di, int dj) -> T {
      if constexpr (ZG) return T(0);
      else return sx0p[(cj + 1 + dj) * PW4 + (ci + 1 + di)];
    };
    if constexpr (ZG) sq_rows<T, false, false, DOM>(J.L, i, j, UA, PA, y, ad);
    else sq_rows<T, true, true, DOM>(J.L, i, j, UA, PA, y, ad);
#pragma unroll
    for (int cls = 0; cls < 4; ++cls) {
      const int DA = cls & 1, DB = cls >> 1;
      const bool in = interior(2 * i + DA, 2 * j + DB);
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const T r = sf[c][2 * cj + DB][2 * ci + DA] - y[2 * cls + c];
        sy[c][2 * cj + DB][2 * ci + DA] = in ? ad[cls] * r : T(0);
      }
    }
    const int q = cj * PW3 + ci;
    syp[q] = inside(i, j) ? ss[q] * (sfp[q] - y[8]) : T(0);
  }
  __syncthreads();

  // ---- stage 2: X1 = X0 + tau L^-1 A Y1 on the tile + 2
  for (int e = tid; e < (TX + 4) * (TY + 4); e += NT) {
    const int ci = e % (TX + 4), cj = e / (TX + 4);
    const int i = i0 - 2 + ci, j = j0 - 2 + cj;
    T z[9], ad[4];
    {
      auto UA = [&](int c, int da, int db) -> T { return sy[c][2 * cj + 2 + db][2 * ci + 2 + da]; };
      auto PA = [&](int di, int dj) -> T { return syp[(cj + 1 + dj) * PW3 + (ci + 1 + di)]; };
      sq_rows<T, true, true, DOM>(J.L, i, j, UA, PA, z, ad);
    }
#pragma unroll
    for (int cls = 0; cls < 4; ++cls) {
      const int DA = cls & 1, DB = cls >> 1;
      const bool in = interior(2 * i + DA, 2 * j + DB);
      const T d = ad[cls] * tau;
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        T x0 = T(0);
        if constexpr (!ZG) x0 = sx0[c][2 * cj + 4 + DB][2 * ci + 4 + DA];
        sx1[c][2 * cj + DB][2 * ci + DA] = in ? x0 + d * z[2 * cls + c] : T(0);
      }
    }
    T x0p = T(0);
    if constexpr (!ZG) x0p = sx0p[(cj + 2) * PW4 + ci + 2];
    sx1p[cj * PW2 + ci] = inside(i, j) ? x0p + tau * ss[(cj + 1) * PW3 + ci + 1] * z[8] : T(0);
  }
  __syncthreads();

  // ---- stage 3: Y2 = L^-1 (F - A X1) on the tile + 1, in Y1's storage
  T (*sy2)[H1][W1] = reinterpret_cast<T (*)[H1][W1]>(&sy[0][0][0]);
  for (int e = tid; e < (TX + 2) * (TY + 2); e += NT) {
    const int ci = e % (TX + 2), cj = e / (TX + 2);
    const int i = i0 - 1 + ci, j = j0 - 1 + cj;
    T y[9], ad[4];
    {
      auto UA = [&](int c, int da, int db) -> T { return sx1[c][2 * cj + 2 + db][2 * ci + 2 + da]; };
      auto PA = [&](int di, int dj) -> T { return sx1p[(cj + 1 + dj) * PW2 + (ci + 1 + di)]; };
      sq_rows<T, true, true, DOM>(J.L, i, j, UA, PA, y, ad);
    }
#pragma unroll
    for (int cls = 0; cls < 4; ++cls) {
      const int DA = cls & 1, DB = cls >> 1;
      const bool in = interior(2 * i + DA, 2 * j + DB);
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const T r = sf[c][2 * cj + 4 + DB][2 * ci + 4 + DA] - y[2 * cls + c];
        sy2[c][2 * cj + DB][2 * ci + DA] = in ? ad[cls] * r : T(0);
      }
    }
    const int q3 = (cj + 2) * PW3 + ci + 2;
    syp[cj * PW1 + ci] = inside(i, j) ? ss[q3] * (sfp[q3] - y[8]) : T(0);
  }
  __syncthreads();

  // ---- stage 4: X2 = X1 + tau L^-1 A Y2 on the tile; four threads per square
  {
    const int part = tid / (TX * TY), q = tid % (TX * TY);
    const int tx = q % TX, ty = q / TX;
    const int i = i0 + tx, j = j0 + ty;
    if (i <= N && j <= N) {
      auto UA = [&](int c, int da, int db) -> T { return sy2[c][2 * ty + 2 + db][2 * tx + 2 + da]; };
      auto PA = [&](int di, int dj) -> T { return syp[(ty + 1 + dj) * PW1 + (tx + 1 + di)]; };
      auto emit = [&](int cls, T z0, T z1, T ad) {
        const int DA = cls & 1, DB = cls >> 1;
        const int a = 2 * i + DA, b = 2 * j + DB;
        if (a > 2 * N || b > 2 * N) return;
        const bool in = interior(a, b);
        const size_t g = (size_t)b * M + a;
        const T d = ad * tau;
        J.ou[g] = in ? sx1[0][2 * ty + 4 + DB][2 * tx + 4 + DA] + d * z0 : T(0);
        J.ou[(size_t)M * M + g] = in ? sx1[1][2 * ty + 4 + DB][2 * tx + 4 + DA] + d * z1 : T(0);
      };
      T z0, z1, ad;
      if (part == 0) {
        sq_vel<0, T, true, true, DOM>(J.L, i, j, UA, PA, z0, z1, ad);
        emit(0, z0, z1, ad);
      } else if (part == 1) {
        sq_vel<1, T, true, true, DOM>(J.L, i, j, UA, PA, z0, z1, ad);
        emit(1, z0, z1, ad);
      } else if (part == 2) {
        sq_vel<2, T, true, true, DOM>(J.L, i, j, UA, PA, z0, z1, ad);
        emit(2, z0, z1, ad);
      } else {
        sq_vel<3, T, true, true, DOM>(J.L, i, j, UA, PA, z0, z1, ad);
        emit(3, z0, z1, ad);
        const T zp = sq_prow<T, DOM>(J.L, i, j, UA);
        J.op[(size_t)j * NP + i] = sx1p[(ty + 2) * PW2 + tx + 2] + tau * ss[(ty + 3) * PW3 + tx + 3] * zp;
      }
    }
  }
}

template <class T, int TX, int TY, bool ZG, bool PRO, int DOM>
__global__ __launch_bounds__(4 * TX* TY) void k_ne2(NEJob<T> J) {
  ne2_tile<T, TX, TY, ZG, PRO, DOM>(J, xcd_remap(blockIdx.x, gridDim.x));
}

template <class T, int TX, int TY, bool ZG, bool PRO, bool PACK, int DOM>
__global__ __launch_bounds__(4 * TX* TY) void k_ne2_b(const JobArg<NEJob<T>> A) {
  int tile;
  const NEJob<T> J = block_job<PACK>(A, xcd_remap(blockIdx.x, gridDim.x), tile);
  ne2_tile<T, TX, TY, ZG, PRO, DOM>(J, tile);
}

template <class T, int DOM>
static void launch_ne2_dom(const NEJob<T>& J, bool zg, bool pro, hipStream_t s) {
  const int nb = ((J.L.N + 8) / 8) * ((J.L.N + 8) / 8);
  if (zg) k_ne2<T, 8, 8, true, false, DOM><<<nb, 256, 0, s>>>(J);
  else if (pro) k_ne2<T, 8, 8, false, true, DOM><<<nb, 256, 0, s>>>(J);
  else k_ne2<T, 8, 8, false, false, DOM><<<nb, 256, 0, s>>>(J);
}

template <class T>
void launch_ne2(const NEJob<T>& J, bool zg, bool pro, hipStream_t s) {
  if (J.L.dom == SMG_DOM_LSHAPE) launch_ne2_dom<T, SMG_DOM_LSHAPE>(J, zg, pro, s);
  else if (J.L.dom == SMG_DOM_UNIONJACK) launch_ne2_dom<T, SMG_DOM_UNIONJACK>(J, zg, pro, s);
  else launch_ne2_dom<T, SMG_DOM_SQUARE>(J, zg, pro, s);
}
template void launch_ne2<double>(const NEJob<double>&, bool, bool, hipStream_t);
template void launch_ne2<float>(const NEJob<float>&, bool, bool, hipStream_t);

template <class T, bool PACK, int DOM>
static void launch_ne2_b_pack(const JobArg<NEJob<T>>& A, int nb, bool zg, bool pro, hipStream_t s) {
  if (zg) k_ne2_b<T, 8, 8, true, false, PACK, DOM><<<nb, 256, 0, s>>>(A);
  else if (pro) k_ne2_b<T, 8, 8, false, true, PACK, DOM><<<nb, 256, 0, s>>>(A);
  else k_ne2_b<T, 8, 8, false, false, PACK, DOM><<<nb, 256, 0, s>>>(A);
}

template <class T, int DOM>
static void launch_ne2_b_dom(const JobArg<NEJob<T>>& A, int nb, bool zg, bool pro, hipStream_t s) {
  if (A.n > 0) launch_ne2_b_pack<T, true, DOM>(A, nb, zg, pro, s);
  else launch_ne2_b_pack<T, false, DOM>(A, nb, zg, pro, s);
}

template <class T>
void launch_ne2_b(const JobArg<NEJob<T>>& A, int nb, bool zg, bool pro, int dom, hipStream_t s) {
  if (dom == SMG_DOM_LSHAPE) launch_ne2_b_dom<T, SMG_DOM_LSHAPE>(A, nb, zg, pro, s);
  else if (dom == SMG_DOM_UNIONJACK) launch_ne2_b_dom<T, SMG_DOM_UNIONJACK>(A, nb, zg, pro, s);
  else launch_ne2_b_dom<T, SMG_DOM_SQUARE>(A, nb, zg, pro, s);
}
template void launch_ne2_b<double>(const JobArg<NEJob<double>>&, int, bool, bool, int, hipStream_t);
template void launch_ne2_b<float>(const JobArg<NEJob<float>>&, int, bool, bool, int, hipStream_t);

// ---------------------------------------------------------------------------
// k_uz: one Uzawa-type smoothing step (Section 4) on a TX x TY tile of squares
// ---------------------------------------------------------------------------
// The three half-steps in one launch:
//   1. u' = u + tau Ahat^-1 (f - A u - B^T p)   on the tile plus two squares
//   2. dp = -sigma Shat^-1 (g - B u')            on the tile's vertices plus one
//   3. u_new = u' - tau Ahat^-1 B^T dp, p_new = p + dp   on the tile
// The velocity row of a node reads u within one square and p at the
// vertices of the squares around it, so step 1 on the tile plus two needs u
// and p on the tile plus three squares; the pressure row of a vertex reads u'
// within one square.  Windows (lattice of the points owned by their squares,
// zero outside the interior of the velocity space and the grid):
//   X  u, squares [i0 - 3, i0 + TX + 2]      XP p, vertices [i0 - 3, i0 + TX + 2]
//   H  u', squares [i0 - 2, i0 + TX + 1]     D  dp, vertices [i0 - 1, i0 + TX]

template <class T, int TX, int TY, bool ZG, int DOM>
__device__ __forceinline__ void uz_tile(const UZJob<T>& J, int tile) {
  constexpr int NT = 2 * TX * TY;
  constexpr int XW = 2 * TX + 12, XH = 2 * TY + 12;     // u: origin (2 i0 - 6, 2 j0 - 6)
  constexpr int PW = TX + 6, PH = TY + 6;               // p: origin (i0 - 3, j0 - 3)
  constexpr int HW = 2 * TX + 8, HH = 2 * TY + 8;       // u': origin (2 i0 - 4, 2 j0 - 4)
  constexpr int DW = TX + 2, DH = TY + 2;               // dp: origin (i0 - 1, j0 - 1)
  constexpr int S1W = TX + 4, S1 = (TX + 4) * (TY + 4); // squares of step 1
  static_assert(S1 <= NT, "one step-1 square per thread");
  __shared__ T sx[2][XH][XW];
  __shared__ T sxp[PH * PW];
  __shared__ T sh[2][HH][HW];
  __shared__ T sd[DH * DW];
  const int N = J.L.N, M = 2 * N + 1, NP = N + 1;
  const int ntx = (N + TX) / TX;
  const int i0 = (tile % ntx) * TX, j0 = (tile / ntx) * TY;
  const int tid = threadIdx.x;
  auto interior = [&](int a, int b) { return dom_u(N, DOM, a, b); };
  // requested before the first wait: the done flag, this thread's step-1
  // right-hand side and its step-2 g and Shat^-1
  const int dn = J.done ? *J.done : 0;
  const int c1i = tid % S1W, c1j = tid / S1W;
  const int s1i = i0 - 2 + c1i, s1j = j0 - 2 + c1j;
  const bool act1 = tid < S1;
  T f1[8];
#pragma unroll
  for (int cls = 0; cls < 4; ++cls) {
    const int a = 2 * s1i + (cls & 1), b = 2 * s1j + (cls >> 1);
    const bool in = act1 && interior(a, b);
#pragma unroll
    for (int c = 0; c < 2; ++c) f1[2 * cls + c] = in ? J.fu[(size_t)c * M * M + (size_t)b * M + a] : T(0);
  }
  const int v2i = tid % DW, v2j = tid / DW;
  const int vi = i0 - 1 + v2i, vj = j0 - 1 + v2j;
  const bool act2 = tid < DW * DH && dom_p(N, DOM, vi, vj);
  const T g2 = act2 ? J.fp[(size_t)vj * NP + vi] : T(0);
  const T s2 = act2 ? J.L.sinv[(size_t)vj * NP + vi] : T(0);

  if constexpr (!ZG) {
    // the iterate on the tile plus three squares, every load in flight at once
    static_assert(XWindow<T, TX, TY, 3, NT, DOM>::XW == XW && XWindow<T, TX, TY, 3, NT, DOM>::XPW == PW,
                  "window shapes");
    XWindow<T, TX, TY, 3, NT, DOM> w;
    w.fetch(J, i0, j0, tid);
    w.put(tid, sx, sxp);
    __syncthreads();
  }
  if (dn) return;   // uniform across the workgroup

  // ---- step 1: u' on the tile plus two squares
  if (act1) {
    T y[9], ad[4];
    auto UA = [&](int c, int da, int db) -> T { return sx[c][2 * c1j + 2 + db][2 * c1i + 2 + da]; };
    auto PA = [&](int di, int dj) -> T { return sxp[(c1j + 1 + dj) * PW + (c1i + 1 + di)]; };
    if constexpr (ZG) sq_rows<T, false, false, DOM>(J.L, s1i, s1j, UA, PA, y, ad);
    else sq_rows<T, true, true, DOM>(J.L, s1i, s1j, UA, PA, y, ad);
#pragma unroll
    for (int cls = 0; cls < 4; ++cls) {
      const int DA = cls & 1, DB = cls >> 1;
      const bool in = interior(2 * s1i + DA, 2 * s1j + DB);
      const T d = J.tau * ad[cls];
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        T x0 = T(0);
        if constexpr (!ZG) x0 = sx[c][2 * c1j + 2 + DB][2 * c1i + 2 + DA];
        sh[c][2 * c1j + DB][2 * c1i + DA] = in ? x0 + d * (f1[2 * cls + c] - y[2 * cls + c]) : T(0);
      }
    }
  }
  __syncthreads();

  // ---- step 2: dp on the tile's vertices plus one
  if (tid < DW * DH) {
    auto UH = [&](int c, int da, int db) -> T { return sh[c][2 * v2j + 2 + db][2 * v2i + 2 + da]; };
    const T bu = sq_prow<T, DOM>(J.L, vi, vj, UH);
    sd[tid] = act2 ? -J.sigma * s2 * (g2 - bu) : T(0);
  }
  __syncthreads();

  // ---- step 3: u_new and p_new on the tile; two threads per square
  {
    const int part = tid / (TX * TY), q = tid % (TX * TY);
    const int tx = q % TX, ty = q / TX;
    const int i = i0 + tx, j = j0 + ty;
    if (i <= N && j <= N) {
      auto PA = [&](int di, int dj) -> T { return sd[(ty + 1 + dj) * DW + (tx + 1 + di)]; };
      auto Un = [&](int c, int da, int db) -> T { return T(0); };
      auto emit = [&](int cls, T z0, T z1, T ad) {
        const int DA = cls & 1, DB = cls >> 1;
        const int a = 2 * i + DA, b = 2 * j + DB;
        if (a > 2 * N || b > 2 * N) return;
        const bool in = interior(a, b);
        const size_t g = (size_t)b * M + a;
        const T d = J.tau * ad;
        J.ou[g] = in ? sh[0][2 * ty + 4 + DB][2 * tx + 4 + DA] - d * z0 : T(0);
        J.ou[(size_t)M * M + g] = in ? sh[1][2 * ty + 4 + DB][2 * tx + 4 + DA] - d * z1 : T(0);
      };
      T z0, z1, ad;
      if (part == 0) {
        sq_vel<0, T, false, true, DOM>(J.L, i, j, Un, PA, z0, z1, ad);
        emit(0, z0, z1, ad);
        sq_vel<1, T, false, true, DOM>(J.L, i, j, Un, PA, z0, z1, ad);
        emit(1, z0, z1, ad);
      } else {
        sq_vel<2, T, false, true, DOM>(J.L, i, j, Un, PA, z0, z1, ad);
        emit(2, z0, z1, ad);
        sq_vel<3, T, false, true, DOM>(J.L, i, j, Un, PA, z0, z1, ad);
        emit(3, z0, z1, ad);
        T p0 = T(0);
        if constexpr (!ZG) p0 = sxp[(ty + 3) * PW + tx + 3];
        J.op[(size_t)j * NP + i] = dom_p(N, DOM, i, j) ? p0 + PA(0, 0) : T(0);
      }
    }
  }
}

template <class T, int TX, int TY, bool ZG, int DOM>
__global__ __launch_bounds__(2 * TX* TY) void k_uz(UZJob<T> J) {
  uz_tile<T, TX, TY, ZG, DOM>(J, xcd_remap(blockIdx.x, gridDim.x));
}

template <class T, int TX, int TY, bool ZG, bool PACK, int DOM>
__global__ __launch_bounds__(2 * TX* TY) void k_uz_b(const JobArg<UZJob<T>> A) {
  int tile;
  const UZJob<T> J = block_job<PACK>(A, xcd_remap(blockIdx.x, gridDim.x), tile);
  uz_tile<T, TX, TY, ZG, DOM>(J, tile);
}

int uz_tiles(int N) { return ((N + 16) / 16) * ((N + 8) / 8); }

template <class T, int DOM>
static void launch_uz_dom(const UZJob<T>& J, bool zg, hipStream_t s) {
  const int nb = uz_tiles(J.L.N);
  if (zg) k_uz<T, 16, 8, true, DOM><<<nb, 256, 0, s>>>(J);
  else k_uz<T, 16, 8, false, DOM><<<nb, 256, 0, s>>>(J);
}

template <class T>
void launch_uz(const UZJob<T>& J, bool zg, hipStream_t s) {
  if (J.L.dom == SMG_DOM_LSHAPE) launch_uz_dom<T, SMG_DOM_LSHAPE>(J, zg, s);
  else if (J.L.dom == SMG_DOM_UNIONJACK) launch_uz_dom<T, SMG_DOM_UNIONJACK>(J, zg, s);
  else launch_uz_dom<T, SMG_DOM_SQUARE>(J, zg, s);
}
template void launch_uz<double>(const UZJob<double>&, bool, hipStream_t);
template void launch_uz<float>(const UZJob<float>&, bool, hipStream_t);

template <class T, int DOM>
static void launch_uz_b_dom(const JobArg<UZJob<T>>& A, int nb, bool zg, hipStream_t s) {
  if (A.n > 0) {
    if (zg) k_uz_b<T, 16, 8, true, true, DOM><<<nb, 256, 0, s>>>(A);
    else k_uz_b<T, 16, 8, false, true, DOM><<<nb, 256, 0, s>>>(A);
  } else {
    if (zg) k_uz_b<T, 16, 8, true, false, DOM><<<nb, 256, 0, s>>>(A);
    else k_uz_b<T, 16, 8, false, false, DOM><<<nb, 256, 0, s>>>(A);
  }
}

template <class T>
void launch_uz_b(const JobArg<UZJob<T>>& A, int nb, bool zg, int dom, hipStream_t s) {
  if (dom == SMG_DOM_LSHAPE) launch_uz_b_dom<T, SMG_DOM_LSHAPE>(A, nb, zg, s);
  else if (dom == SMG_DOM_UNIONJACK) launch_uz_b_dom<T, SMG_DOM_UNIONJACK>(A, nb, zg, s);
  else launch_uz_b_dom<T, SMG_DOM_SQUARE>(A, nb, zg, s);
}
template void launch_uz_b<double>(const JobArg<UZJob<double>>&, int, bool, int, hipStream_t);
template void launch_uz_b<float>(const JobArg<UZJob<float>>&, int, bool, int, hipStream_t);

// ---------------------------------------------------------------------------
// k_resid_restrict: F_c = P^T (F - A x) on an 8 x 8 tile of coarse squares
// ---------------------------------------------------------------------------

template <class T, int DOM>
__device__ __forceinline__ void rr_tile(const RRJob<T>& J, int tile) {
  constexpr int TC = 8, NT = 256;
  constexpr int XW = 4 * TC + 10;      // x: fine lattice origin (4 I0 - 6, 4 J0 - 6)
  constexpr int XPW = 2 * TC + 5;      // x pressure: origin (2 I0 - 3, 2 J0 - 3)
  constexpr int RW = 4 * TC + 6;       // defect: fine lattice origin (4 I0 - 4, 4 J0 - 4)
  constexpr int RPW = 2 * TC + 3;      // defect pressure: origin (2 I0 - 2, 2 J0 - 2)
  constexpr int NC1 = 2 * TC + 3;      // fine squares per side of stage 1
  // the defect window takes the iterate window's storage once stage 1 has
  // read it: half the LDS, so that more workgroups fit on a CU
  constexpr int SXN = 2 * XW * XW + XPW * XPW, SRN = 2 * RW * RW + RPW * RPW;
  __shared__ T buf[SXN > SRN ? SXN : SRN];
  T (*sx)[XW][XW] = reinterpret_cast<T (*)[XW][XW]>(buf);
  T* sxp = buf + 2 * XW * XW;
  T (*sr)[RW][RW] = reinterpret_cast<T (*)[RW][RW]>(buf);
  T* srp = buf + 2 * RW * RW;
  const int N = J.L.N, M = 2 * N + 1, NP = N + 1;
  const int Nc = N / 2, Mc = 2 * Nc + 1, NPc = Nc + 1;
  const int ntx = (Nc + TC) / TC;
  const int I0 = (tile % ntx) * TC, J0 = (tile / ntx) * TC;
  const int tid = threadIdx.x;
  auto interior = [&](int a, int b) { return dom_u(N, DOM, a, b); };
  // the done flag and this thread's stage-1 right-hand sides (at most two
  // squares per thread) are requested together with the iterate window
  static_assert(NC1 * NC1 <= 2 * NT, "at most two stage-1 squares per thread");
  const int dn = J.done ? *J.done : 0;
  T f1[2][9];
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const int e = tid + it * NT, ci = e % NC1, cj = e / NC1;
    const int i = 2 * I0 - 2 + ci, j = 2 * J0 - 2 + cj;
    const bool act = e < NC1 * NC1;
#pragma unroll
    for (int cls = 0; cls < 4; ++cls) {
      const int a = 2 * i + (cls & 1), b = 2 * j + (cls >> 1);
      const bool in = act && interior(a, b);
#pragma unroll
      for (int c = 0; c < 2; ++c) f1[it][2 * cls + c] = in ? J.fu[(size_t)c * M * M + (size_t)b * M + a] : T(0);
    }
    const bool inp = act && dom_p(N, DOM, i, j);
    f1[it][8] = inp ? J.fp[(size_t)j * NP + i] : T(0);
  }
  // the fine iterate window, every load in flight at once
  Staged<XW * XW, NT, 2, T> xw;
  Staged<XPW * XPW, NT, 1, T> xpw;
  xw.fetch(tid, [&](int e, T* v) {
    const int a = 4 * I0 - 6 + e % XW, b = 4 * J0 - 6 + e / XW;
    const bool in = interior(a, b);
    const size_t g = (size_t)b * M + a;
    v[0] = in ? J.xu[g] : T(0);
    v[1] = in ? J.xu[(size_t)M * M + g] : T(0);
  });
  xpw.fetch(tid, [&](int e, T* v) {
    const int i = 2 * I0 - 3 + e % XPW, j = 2 * J0 - 3 + e / XPW;
    v[0] = dom_p(N, DOM, i, j) ? J.xp[(size_t)j * NP + i] : T(0);
  });
  xw.put(tid, [&](int e, const T* v) {
    sx[0][e / XW][e % XW] = v[0];
    sx[1][e / XW][e % XW] = v[1];
  });
  xpw.put(tid, [&](int e, const T* v) { sxp[e] = v[0]; });
  __syncthreads();
  if (dn) return;   // uniform across the workgroup
  // stage 1: fine defect on squares [2 I0 - 2, 2 I0 + 2 TC] per side, kept
  // in registers until every thread has read the window, then stored
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const int e = tid + it * NT;
    if (e >= NC1 * NC1) break;
    const int ci = e % NC1, cj = e / NC1;
    const int i = 2 * I0 - 2 + ci, j = 2 * J0 - 2 + cj;
    T y[9], ad[4];
    {
      auto UA = [&](int c, int da, int db) -> T { return sx[c][2 * cj + 2 + db][2 * ci + 2 + da]; };
      auto PA = [&](int di, int dj) -> T { return sxp[(cj + 1 + dj) * XPW + (ci + 1 + di)]; };
      sq_rows<T, true, true, DOM>(J.L, i, j, UA, PA, y, ad);
    }
#pragma unroll
    for (int cls = 0; cls < 4; ++cls) {
      const int DA = cls & 1, DB = cls >> 1;
      const int a = 2 * i + DA, b = 2 * j + DB;
      const bool in = interior(a, b);
#pragma unroll
      for (int c = 0; c < 2; ++c) f1[it][2 * cls + c] = in ? f1[it][2 * cls + c] - y[2 * cls + c] : T(0);
    }
    const bool inp = dom_p(N, DOM, i, j);
    f1[it][8] = inp ? f1[it][8] - y[8] : T(0);
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const int e = tid + it * NT;
    if (e >= NC1 * NC1) break;
    const int ci = e % NC1, cj = e / NC1;
#pragma unroll
    for (int cls = 0; cls < 4; ++cls) {
      const int DA = cls & 1, DB = cls >> 1;
#pragma unroll
      for (int c = 0; c < 2; ++c) sr[c][2 * cj + DB][2 * ci + DA] = f1[it][2 * cls + c];
    }
    srp[cj * RPW + ci] = f1[it][8];
  }
  __syncthreads();
  // stage 2: one wave per coarse node class, one lane per coarse square
  const int cls = tid >> 6, q = tid & 63;
  const int tx = q % TC, ty = q / TC;
  const int I = I0 + tx, Jc = J0 + ty;
  if (I <= Nc && Jc <= Nc) {
    const int CA = cls & 1, CB = cls >> 1;
    const int A = 2 * I + CA, B = 2 * Jc + CB;
    if (A <= 2 * Nc && B <= 2 * Nc) {
      const bool in = dom_u(Nc, DOM, A, B);
      const int la = 4 * tx + 2 * CA + 4, lb = 4 * ty + 2 * CB + 4;
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        auto R = [&](int fa, int fb) -> T { return sr[c][lb + fb][la + fa]; };
        T v = T(0);
        if (in) {
          switch (cls) {
            case 0: v = sq_res<0, T, DOM>(Nc, I, Jc, R); break;
            case 1: v = sq_res<1, T, DOM>(Nc, I, Jc, R); break;
            case 2: v = sq_res<2, T, DOM>(Nc, I, Jc, R); break;
            default: v = sq_res<3, T, DOM>(Nc, I, Jc, R); break;
          }
        }
        J.cu[(size_t)c * Mc * Mc + (size_t)B * Mc + A] = v;
      }
    }
    if (cls == 3) {
      auto Rp = [&](int di, int dj) -> T { return srp[(2 * ty + 2 + dj) * RPW + (2 * tx + 2 + di)]; };
      J.cp[(size_t)Jc * NPc + I] = dom_p(Nc, DOM, I, Jc) ? sq_resp<T, DOM>(Nc, I, Jc, Rp) : T(0);
    }
  }
}

template <class T, int DOM>
__global__ __launch_bounds__(256) void k_resid_restrict(RRJob<T> J) {
  rr_tile<T, DOM>(J, xcd_remap(blockIdx.x, gridDim.x));
}

template <class T, bool PACK, int DOM>
__global__ __launch_bounds__(256) void k_rr_b(const JobArg<RRJob<T>> A) {
  int tile;
  const RRJob<T> J = block_job<PACK>(A, xcd_remap(blockIdx.x, gridDim.x), tile);
  rr_tile<T, DOM>(J, tile);
}

template <class T, int DOM>
static void launch_rr_b_dom(const JobArg<RRJob<T>>& A, int nb, hipStream_t s) {
  if (A.n > 0) k_rr_b<T, true, DOM><<<nb, 256, 0, s>>>(A);
  else k_rr_b<T, false, DOM><<<nb, 256, 0, s>>>(A);
}

template <class T>
void launch_rr_b(const JobArg<RRJob<T>>& A, int nb, int dom, hipStream_t s) {
  if (dom == SMG_DOM_LSHAPE) launch_rr_b_dom<T, SMG_DOM_LSHAPE>(A, nb, s);
  else if (dom == SMG_DOM_UNIONJACK) launch_rr_b_dom<T, SMG_DOM_UNIONJACK>(A, nb, s);
  else launch_rr_b_dom<T, SMG_DOM_SQUARE>(A, nb, s);
}
template void launch_rr_b<double>(const JobArg<RRJob<double>>&, int, int, hipStream_t);
template void launch_rr_b<float>(const JobArg<RRJob<float>>&, int, int, hipStream_t);

template <class T>
void launch_resid_restrict(const RRJob<T>& J, hipStream_t s) {
  const int Nc = J.L.N / 2;
  const int nb = ((Nc + 8) / 8) * ((Nc + 8) / 8);
  if (J.L.dom == SMG_DOM_LSHAPE) k_resid_restrict<T, SMG_DOM_LSHAPE><<<nb, 256, 0, s>>>(J);
  else if (J.L.dom == SMG_DOM_UNIONJACK) k_resid_restrict<T, SMG_DOM_UNIONJACK><<<nb, 256, 0, s>>>(J);
  else k_resid_restrict<T, SMG_DOM_SQUARE><<<nb, 256, 0, s>>>(J);
}
template void launch_resid_restrict<double>(const RRJob<double>&, hipStream_t);
template void launch_resid_restrict<float>(const RRJob<float>&, hipStream_t);

// ---------------------------------------------------------------------------
// k_ne2rr: from a zero iterate, two normal-equation steps, then the defect
// and its restriction, on a tile of 4 x 4 coarse squares (8 x 8 fine ones)
// ---------------------------------------------------------------------------
// Each stage needs its input on one more square around its own squares, so
// with the fine tile at [i0, i0 + 8) (i0 = 2 I0) the regions of fine squares
// are R1 = [-6, 12] for Y1 = L^-1 F, R2 = [-5, 11] for X1 = tau L^-1 A Y1,
// R3 = [-4, 10] for Y2 = L^-1 (F - A X1), R4 = [-3, 9] for X2 = X1 +
// tau L^-1 A Y2 and R5 = [-2, 8] for the defect R = F - A X2 (what the
// transposed embedding reads for the coarse tile), all relative to i0 (and
// j0).  LDS (64 KB at most): one R1-sized array holds F, then Y1 (in place),
// then Y2, then R; F is kept on R3 (all the later stages read), Shat^-1 on
// R2 (every stage from the second reads it at its own vertices), X1 on R2
// and X2 over it in place (each point of X2 reads X1 at that point only).
// Every value uses the same expressions as two single steps and the
// defect-restriction kernel.

template <class T, int DOM>
__device__ __forceinline__ void ne2rr_tile(const NERRJob<T>& J, int tile) {
  constexpr int TC = 4, FT = 2 * TC, NT = 256;
  constexpr int S1 = FT + 11, S2 = FT + 9, S3 = FT + 7, S4 = FT + 5, S5 = FT + 3;
  constexpr int W1 = 2 * S1, W2 = 2 * S2, W3 = 2 * S3, W5 = 2 * S5;
  __shared__ T sy[2][W1][W1];      // F, Y1, Y2, R
  __shared__ T syp[S1 * S1];       // Y1, Y2, R (pressure)
  __shared__ T sf[2][W3][W3];      // F on R3
  __shared__ T sfp[S3 * S3];
  __shared__ T ss[S2 * S2];        // Shat^-1 on R2
  __shared__ T sx[2][W2][W2];      // X1, X2
  __shared__ T sxp[S2 * S2];
  static_assert(sizeof(T) * (2 * W1 * W1 + S1 * S1 + 2 * W3 * W3 + S3 * S3 + 2 * S2 * S2 + 2 * W2 * W2) <= 65536,
                "LDS of one workgroup");
  const int N = J.L.N, M = 2 * N + 1, NP = N + 1;
  const int Nc = N / 2, Mc = 2 * Nc + 1, NPc = Nc + 1;
  const int ntx = (Nc + TC) / TC;
  const int I0 = (tile % ntx) * TC, J0 = (tile / ntx) * TC;
  const int i0 = 2 * I0, j0 = 2 * J0;
  const int tid = threadIdx.x;
  const T tau = J.tau;
  auto interior = [&](int a, int b) { return dom_u(N, DOM, a, b); };
  auto inside = [&](int i, int j) { return dom_p(N, DOM, i, j); };

  // ---- stage 0: F and Shat^-1 on R1, every load in flight at once; Y1's
  // pressure part L^-1 (F_p - 0) directly
  const int dn = J.done ? *J.done : 0;
  Staged<W1 * W1, NT, 2, T> fw;
  Staged<S1 * S1, NT, 2, T> fpw;
  fw.fetch(tid, [&](int e, T* v) {
    const int a = 2 * i0 - 12 + e % W1, b = 2 * j0 - 12 + e / W1;
    const bool in = interior(a, b);
    const size_t g = (size_t)b * M + a;
    v[0] = in ? J.fu[g] : T(0);
    v[1] = in ? J.fu[(size_t)M * M + g] : T(0);
  });
  fpw.fetch(tid, [&](int e, T* v) {
    const int i = i0 - 6 + e % S1, j = j0 - 6 + e / S1;
    const bool ok = inside(i, j);
    v[0] = ok ? J.fp[(size_t)j * NP + i] : T(0);
    v[1] = ok ? J.L.sinv[(size_t)j * NP + i] : T(0);
  });
  fw.put(tid, [&](int e, const T* v) {
    const int la = e % W1, lb = e / W1;
    sy[0][lb][la] = v[0];
    sy[1][lb][la] = v[1];
    if (la >= 4 && la < 4 + W3 && lb >= 4 && lb < 4 + W3) {
      sf[0][lb - 4][la - 4] = v[0];
      sf[1][lb - 4][la - 4] = v[1];
    }
  });
  fpw.put(tid, [&](int e, const T* v) {
    const int li = e % S1, lj = e / S1;
    syp[e] = inside(i0 - 6 + li, j0 - 6 + lj) ? v[1] * (v[0] - T(0)) : T(0);
    if (li >= 2 && li < 2 + S3 && lj >= 2 && lj < 2 + S3) sfp[(lj - 2) * S3 + li - 2] = v[0];
    if (li >= 1 && li < 1 + S2 && lj >= 1 && lj < 1 + S2) ss[(lj - 1) * S2 + li - 1] = v[1];
  });
  __syncthreads();
  if (dn) return;   // uniform across the workgroup

  // ---- stage 1: Y1 = L^-1 (F - A 0) on R1, in place over F (own points)
  for (int e = tid; e < S1 * S1; e += NT) {
    const int ci = e % S1, cj = e / S1;
    const int i = i0 - 6 + ci, j = j0 - 6 + cj;
    T y[9], ad[4];
    auto Z = [&](int, int, int) -> T { return T(0); };
    auto Zp = [&](int, int) -> T { return T(0); };
    sq_rows<T, false, false, DOM>(J.L, i, j, Z, Zp, y, ad);
#pragma unroll
    for (int cls = 0; cls < 4; ++cls) {
      const int DA = cls & 1, DB = cls >> 1;
      const bool in = interior(2 * i + DA, 2 * j + DB);
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        T& v = sy[c][2 * cj + DB][2 * ci + DA];
        const T r = v - y[2 * cls + c];
        v = in ? ad[cls] * r : T(0);
      }
    }
  }
  __syncthreads();

  // ---- stage 2: X1 = 0 + tau L^-1 A Y1 on R2
  for (int e = tid; e < S2 * S2; e += NT) {
    const int ci = e % S2, cj = e / S2;
    const int i = i0 - 5 + ci, j = j0 - 5 + cj;
    T z[9], ad[4];
    {
      auto UA = [&](int c, int da, int db) -> T { return sy[c][2 * cj + 2 + db][2 * ci + 2 + da]; };
      auto PA = [&](int di, int dj) -> T { return syp[(cj + 1 + dj) * S1 + (ci + 1 + di)]; };
      sq_rows<T, true, true, DOM>(J.L, i, j, UA, PA, z, ad);
    }
#pragma unroll
    for (int cls = 0; cls < 4; ++cls) {
      const int DA = cls & 1, DB = cls >> 1;
      const bool in = interior(2 * i + DA, 2 * j + DB);
      const T d = ad[cls] * tau;
#pragma unroll
      for (int c = 0; c < 2; ++c) sx[c][2 * cj + DB][2 * ci + DA] = in ? T(0) + d * z[2 * cls + c] : T(0);
    }
    sxp[e] = inside(i, j) ? T(0) + tau * ss[e] * z[8] : T(0);
  }
  __syncthreads();

  // ---- stage 3: Y2 = L^-1 (F - A X1) on R3, in the storage of Y1 (no longer read)
  T (*sy2)[W3][W3] = reinterpret_cast<T (*)[W3][W3]>(&sy[0][0][0]);
  for (int e = tid; e < S3 * S3; e += NT) {
    const int ci = e % S3, cj = e / S3;
    const int i = i0 - 4 + ci, j = j0 - 4 + cj;
    T y[9], ad[4];
    {
      auto UA = [&](int c, int da, int db) -> T { return sx[c][2 * cj + 2 + db][2 * ci + 2 + da]; };
      auto PA = [&](int di, int dj) -> T { return sxp[(cj + 1 + dj) * S2 + (ci + 1 + di)]; };
      sq_rows<T, true, true, DOM>(J.L, i, j, UA, PA, y, ad);
    }
#pragma unroll
    for (int cls = 0; cls < 4; ++cls) {
      const int DA = cls & 1, DB = cls >> 1;
      const bool in = interior(2 * i + DA, 2 * j + DB);
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const T r = sf[c][2 * cj + DB][2 * ci + DA] - y[2 * cls + c];
        sy2[c][2 * cj + DB][2 * ci + DA] = in ? ad[cls] * r : T(0);
      }
    }
    syp[e] = inside(i, j) ? ss[(cj + 1) * S2 + ci + 1] * (sfp[e] - y[8]) : T(0);
  }
  __syncthreads();

  // ---- stage 4: X2 = X1 + tau L^-1 A Y2 on R4, in place over X1; the tile's
  // own squares go to the output
  for (int e = tid; e < S4 * S4; e += NT) {
    const int ci = e % S4, cj = e / S4;
    const int i = i0 - 3 + ci, j = j0 - 3 + cj;
    T z[9], ad[4];
    {
      auto UA = [&](int c, int da, int db) -> T { return sy2[c][2 * cj + 2 + db][2 * ci + 2 + da]; };
      auto PA = [&](int di, int dj) -> T { return syp[(cj + 1 + dj) * S3 + (ci + 1 + di)]; };
      sq_rows<T, true, true, DOM>(J.L, i, j, UA, PA, z, ad);
    }
    const bool own = ci >= 3 && ci < 3 + FT && cj >= 3 && cj < 3 + FT && i <= N && j <= N;
#pragma unroll
    for (int cls = 0; cls < 4; ++cls) {
      const int DA = cls & 1, DB = cls >> 1;
      const int a = 2 * i + DA, b = 2 * j + DB;
      const bool in = interior(a, b);
      const T d = ad[cls] * tau;
      T x2[2];
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        T& xv = sx[c][2 * cj + 4 + DB][2 * ci + 4 + DA];
        x2[c] = in ? xv + d * z[2 * cls + c] : T(0);
        xv = x2[c];
      }
      if (own && a <= 2 * N && b <= 2 * N) {
        const size_t g = (size_t)b * M + a;
        J.ou[g] = x2[0];
        J.ou[(size_t)M * M + g] = x2[1];
      }
    }
    const int q2 = (cj + 2) * S2 + ci + 2;
    const T x2p = sxp[q2] + tau * ss[q2] * z[8];
    sxp[q2] = x2p;
    if (own) J.op[(size_t)j * NP + i] = x2p;
  }
  __syncthreads();

  // ---- stage 5: R = F - A X2 on R5, in the storage of Y1 (Y2 no longer read)
  T (*sr)[W5][W5] = reinterpret_cast<T (*)[W5][W5]>(&sy[0][0][0]);
  for (int e = tid; e < S5 * S5; e += NT) {
    const int ci = e % S5, cj = e / S5;
    const int i = i0 - 2 + ci, j = j0 - 2 + cj;
    T y[9], ad[4];
    {
      auto UA = [&](int c, int da, int db) -> T { return sx[c][2 * cj + 6 + db][2 * ci + 6 + da]; };
      auto PA = [&](int di, int dj) -> T { return sxp[(cj + 3 + dj) * S2 + (ci + 3 + di)]; };
      sq_rows<T, true, true, DOM>(J.L, i, j, UA, PA, y, ad);
    }
#pragma unroll
    for (int cls = 0; cls < 4; ++cls) {
      const int DA = cls & 1, DB = cls >> 1;
      const bool in = interior(2 * i + DA, 2 * j + DB);
#pragma unroll
      for (int c = 0; c < 2; ++c)
        sr[c][2 * cj + DB][2 * ci + DA] = in ? sf[c][2 * cj + 4 + DB][2 * ci + 4 + DA] - y[2 * cls + c] : T(0);
    }
    syp[e] = inside(i, j) ? sfp[(cj + 2) * S3 + ci + 2] - y[8] : T(0);
  }
  __syncthreads();

  // ---- stage 6: F_c = P^T R on the coarse tile: one wave per coarse node
  // class, one lane per coarse square
  const int cls = tid >> 6, q = tid & 63;
  const int tx = q % TC, ty = q / TC;
  const int I = I0 + tx, Jc = J0 + ty;
  if (q < TC * TC && I <= Nc && Jc <= Nc) {
    const int CA = cls & 1, CB = cls >> 1;
    const int A = 2 * I + CA, B = 2 * Jc + CB;
    if (A <= 2 * Nc && B <= 2 * Nc) {
      const bool in = dom_u(Nc, DOM, A, B);
      const int la = 4 * tx + 2 * CA + 4, lb = 4 * ty + 2 * CB + 4;
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        auto R = [&](int fa, int fb) -> T { return sr[c][lb + fb][la + fa]; };
        T v = T(0);
        if (in) {
          switch (cls) {
            case 0: v = sq_res<0, T, DOM>(Nc, I, Jc, R); break;
            case 1: v = sq_res<1, T, DOM>(Nc, I, Jc, R); break;
            case 2: v = sq_res<2, T, DOM>(Nc, I, Jc, R); break;
            default: v = sq_res<3, T, DOM>(Nc, I, Jc, R); break;
          }
        }
        J.cu[(size_t)c * Mc * Mc + (size_t)B * Mc + A] = v;
      }
    }
    if (cls == 3) {
      auto Rp = [&](int di, int dj) -> T { return syp[(2 * ty + 2 + dj) * S5 + (2 * tx + 2 + di)]; };
      J.cp[(size_t)Jc * NPc + I] = dom_p(Nc, DOM, I, Jc) ? sq_resp<T, DOM>(Nc, I, Jc, Rp) : T(0);
    }
  }
}

template <class T, int DOM>
__global__ __launch_bounds__(256) void k_ne2rr(NERRJob<T> J) {
  ne2rr_tile<T, DOM>(J, xcd_remap(blockIdx.x, gridDim.x));
}

template <class T, bool PACK, int DOM>
__global__ __launch_bounds__(256) void k_ne2rr_b(const JobArg<NERRJob<T>> A) {
  int tile;
  const NERRJob<T> J = block_job<PACK>(A, xcd_remap(blockIdx.x, gridDim.x), tile);
  ne2rr_tile<T, DOM>(J, tile);
}

int ne2rr_tiles(int Nc) { return ((Nc + 4) / 4) * ((Nc + 4) / 4); }

template <class T>
void launch_ne2rr(const NERRJob<T>& J, hipStream_t s) {
  const int nb = ne2rr_tiles(J.L.N / 2);
  if (J.L.dom == SMG_DOM_LSHAPE) k_ne2rr<T, SMG_DOM_LSHAPE><<<nb, 256, 0, s>>>(J);
  else if (J.L.dom == SMG_DOM_UNIONJACK) k_ne2rr<T, SMG_DOM_UNIONJACK><<<nb, 256, 0, s>>>(J);
  else k_ne2rr<T, SMG_DOM_SQUARE><<<nb, 256, 0, s>>>(J);
}
template void launch_ne2rr<double>(const NERRJob<double>&, hipStream_t);
template void launch_ne2rr<float>(const NERRJob<float>&, hipStream_t);

template <class T, int DOM>
static void launch_ne2rr_b_dom(const JobArg<NERRJob<T>>& A, int nb, hipStream_t s) {
  if (A.n > 0) k_ne2rr_b<T, true, DOM><<<nb, 256, 0, s>>>(A);
  else k_ne2rr_b<T, false, DOM><<<nb, 256, 0, s>>>(A);
}

template <class T>
void launch_ne2rr_b(const JobArg<NERRJob<T>>& A, int nb, int dom, hipStream_t s) {
  if (dom == SMG_DOM_LSHAPE) launch_ne2rr_b_dom<T, SMG_DOM_LSHAPE>(A, nb, s);
  else if (dom == SMG_DOM_UNIONJACK) launch_ne2rr_b_dom<T, SMG_DOM_UNIONJACK>(A, nb, s);
  else launch_ne2rr_b_dom<T, SMG_DOM_SQUARE>(A, nb, s);
}
template void launch_ne2rr_b<double>(const JobArg<NERRJob<double>>&, int, int, hipStream_t);
template void launch_ne2rr_b<float>(const JobArg<NERRJob<float>>&, int, int, hipStream_t);

// ---------------------------------------------------------------------------
constexpr int CC_THREADS = 768;
#include "smg_coarse.inc"

// 12 waves: the five item types of a phase (four node classes, the pressure)
// on the levels up to N = 8 fit in one pass, and the register budget (three
// waves per SIMD) still holds the FP64 stencil rows without spills

template <class T, int DOM>
__global__ __launch_bounds__(CC_THREADS) void k_coarse_cycle(CoarseJob<T> J) {
  coarse_body<T, DOM>(J);
}

template <class T, int DOM>
__global__ __launch_bounds__(CC_THREADS) void k_coarse_cycle_b(const CoarseJob<T>* __restrict__ jobs) {
  // the job (about 1.4 KB of coefficients and pointers) is staged in LDS once;
  // read through global memory, every coefficient access inside the phases
  // would be a vector load
  __shared__ CoarseJob<T> sj;
  {
    const unsigned* src = reinterpret_cast<const unsigned*>(jobs + blockIdx.x);
    unsigned* dst = reinterpret_cast<unsigned*>(&sj);
    for (int e = threadIdx.x; e < (int)(sizeof(CoarseJob<T>) / 4); e += blockDim.x) dst[e] = src[e];
  }
  __syncthreads();
  coarse_body<T, DOM>(sj);
}

template <class T>
void launch_cc_b(const CoarseJob<T>* jobs, int njobs, size_t lds, int dom, hipStream_t s) {
  if (dom == SMG_DOM_LSHAPE) k_coarse_cycle_b<T, SMG_DOM_LSHAPE><<<njobs, CC_THREADS, lds, s>>>(jobs);
  else if (dom == SMG_DOM_UNIONJACK) k_coarse_cycle_b<T, SMG_DOM_UNIONJACK><<<njobs, CC_THREADS, lds, s>>>(jobs);
  else k_coarse_cycle_b<T, SMG_DOM_SQUARE><<<njobs, CC_THREADS, lds, s>>>(jobs);
}
template void launch_cc_b<double>(const CoarseJob<double>*, int, size_t, int, hipStream_t);
template void launch_cc_b<float>(const CoarseJob<float>*, int, size_t, int, hipStream_t);

// ---------------------------------------------------------------------------
// k_ccd: x = K F for the dense coarse map.  One wave per row of K (row-major):
// the lanes take every 64th column, so that each load instruction reads 512
// contiguous bytes, and the lanes' sums are added in a fixed tree.  F is
// staged in LDS by every workgroup.  In FP64 the sums are compensated (the
// product's rounding error by an FMA, the addition's by the two-sum of
// Knuth), so that the map's rows, whose terms cancel strongly for large beta,
// keep the accuracy of the level-by-level computation.
// ---------------------------------------------------------------------------
// s + c += a b with the rounding errors of the product and the sum kept in c
__device__ __forceinline__ void dot2_add(double a, double b, double& s, double& c) {
#pragma clang fp contract(off)
  const double p = a * b;
  const double e = fma(a, b, -p);
  const double t = s + p;
  const double bb = t - s;
  c += ((s - (t - bb)) + (p - bb)) + e;
  s = t;
}
__device__ __forceinline__ void dot2_add(float a, float b, float& s, float&) { s += a * b; }
template <class T>
__device__ __forceinline__ void ccd_body(const DenseJob<T>& J, int rb) {
  static_assert(KD_ROWS * 64 == 256, "256 threads: one wave per row");
  __shared__ T sf[KD_MAX];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int n = J.n, nu = J.nu;
  const int dn = J.done ? *J.done : 0;
  for (int e = tid; e < n; e += 256) sf[e] = e < nu ? J.fu[e] : J.fp[e - nu];
  __syncthreads();
  if (dn) return;   // uniform across the workgroup
  const int row = rb * KD_ROWS + w;
  if (row >= n) return;   // no barrier follows
  const T* k = J.K + (size_t)row * n;
  T z = T(0), zc = T(0);
  int q = lane;
  for (; q + 64 * 7 < n; q += 64 * 8) {
    T kv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) kv[u] = k[q + 64 * u];
#pragma unroll
    for (int u = 0; u < 8; ++u) dot2_add(kv[u], sf[q + 64 * u], z, zc);
  }
  for (; q < n; q += 64) dot2_add(k[q], sf[q], z, zc);
  // lane sums in a fixed tree; each addition's error joins the correction
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const T oz = __shfl_down(z, off, 64);
    const T oc = __shfl_down(zc, off, 64);
    dot2_add(oz, T(1), z, zc);
    zc += oc;
  }
  if (lane == 0) {
    const T v = z + zc;
    if (row < nu) J.xu[row] = v;
    else J.xp[row - nu] = v;
  }
}

template <class T>
__global__ __launch_bounds__(256) void k_ccd(DenseJob<T> J) {
  ccd_body<T>(J, blockIdx.x);
}

template <class T, bool PACK>
__global__ __launch_bounds__(256) void k_ccd_b(const JobArg<DenseJob<T>> A) {
  int tile;
  const DenseJob<T> J = block_job<PACK>(A, (int)blockIdx.x, tile);
  ccd_body<T>(J, tile);
}

template <class T>
void launch_ccd(const DenseJob<T>& J, hipStream_t s) {
  k_ccd<T><<<ccd_blocks(J.n), 256, 0, s>>>(J);
}
template void launch_ccd<double>(const DenseJob<double>&, hipStream_t);
template void launch_ccd<float>(const DenseJob<float>&, hipStream_t);

template <class T>
void launch_ccd_b(const JobArg<DenseJob<T>>& A, int nb, hipStream_t s) {
  if (A.n > 0) k_ccd_b<T, true><<<nb, 256, 0, s>>>(A);
  else k_ccd_b<T, false><<<nb, 256, 0, s>>>(A);
}
template void launch_ccd_b<double>(const JobArg<DenseJob<double>>&, int, hipStream_t);
template void launch_ccd_b<float>(const JobArg<DenseJob<float>>&, int, hipStream_t);

size_t coarse_cycle_lds(int n0, int Lc, size_t elem) {
  size_t tot = 0;
  for (int l = 0; l <= Lc; ++l) {
    const size_t N = (size_t)n0 << l, Mp = 2 * N + 5, NPp = N + 3;
    tot += 3 * (2 * Mp * Mp + NPp * NPp) + (N + 1) * (N + 1);
  }
  return tot * elem;
}

template <class T>
int launch_coarse_cycle(const CoarseJob<T>& J, hipStream_t s) {
  const size_t lds = coarse_cycle_lds(J.n0, J.Lc, sizeof(T));
  if (J.L[0].dom == SMG_DOM_LSHAPE) k_coarse_cycle<T, SMG_DOM_LSHAPE><<<1, CC_THREADS, lds, s>>>(J);
  else if (J.L[0].dom == SMG_DOM_UNIONJACK) k_coarse_cycle<T, SMG_DOM_UNIONJACK><<<1, CC_THREADS, lds, s>>>(J);
  else k_coarse_cycle<T, SMG_DOM_SQUARE><<<1, CC_THREADS, lds, s>>>(J);
  return 0;
}
template int launch_coarse_cycle<double>(const CoarseJob<double>&, hipStream_t);
template int launch_coarse_cycle<float>(const CoarseJob<float>&, hipStream_t);

template <class T>
int coarse_cycle_allow_lds(size_t bytes) {
  const void* fns[6] = {(const void*)k_coarse_cycle<T, SMG_DOM_SQUARE>,
                        (const void*)k_coarse_cycle_b<T, SMG_DOM_SQUARE>,
                        (const void*)k_coarse_cycle<T, SMG_DOM_LSHAPE>,
                        (const void*)k_coarse_cycle_b<T, SMG_DOM_LSHAPE>,
                        (const void*)k_coarse_cycle<T, SMG_DOM_UNIONJACK>,
                        (const void*)k_coarse_cycle_b<T, SMG_DOM_UNIONJACK>};
  for (const void* f : fns) {
    const int e = (int)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != 0) return e;
  }
  return 0;
}
template int coarse_cycle_allow_lds<double>(size_t);
template int coarse_cycle_allow_lds<float>(size_t);

// ---------------------------------------------------------------------------
// pressure mean projection from tile partials (sum_i w_i p_i, sum_i w_i)
// written by the residual-norm pass; every block reduces them in the same
// order and subtracts the mean from its part of p.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_project_partials(const double* __restrict__ mpart, int np, int N,
                                                          int dom, double* p, const int* done) {
  if (done && *done) return;
  __shared__ double red[4];
  __shared__ double sh_mean;
  double s1 = 0.0, s2 = 0.0;
  for (int k = threadIdx.x; k < np; k += 256) {
    s1 += mpart[2 * k];
    s2 += mpart[2 * k + 1];
  }
  const double t1 = wg_sum<256>(s1, red);
  __syncthreads();
  const double t2 = wg_sum<256>(s2, red);
  if (threadIdx.x == 0) sh_mean = t1 / t2;
  __syncthreads();
  const int n = (N + 1) * (N + 1);
  const double m = sh_mean;
  for (int k = 0; k < 4; ++k) {
    const int e = blockIdx.x * 1024 + k * 256 + threadIdx.x;
    if (e < n && dom_p(N, dom, e % (N + 1), e / (N + 1))) p[e] -= m;
  }
}

void launch_project_partials(const double* mpart, int np, int N, int dom, double* p, const int* done,
                             hipStream_t s) {
  const int n = (N + 1) * (N + 1);
  k_project_partials<<<(n + 1023) / 1024, 256, 0, s>>>(mpart, np, N, dom, p, done);
}

// pressure entries per thread of the projection / check kernels: on large
// grids 16, so that few workgroups take a ticket from the one shared counter
// (each ticket is an atomic on the same word); on small grids 4, so that the
// work spreads over more workgroups
__host__ __device__ inline int pc_per_thread(int N) { return N >= 256 ? 16 : 4; }

// Mean projection by every workgroup, then the convergence test by the last
// workgroup to finish (it is last, so every other workgroup has already read
// the flag it is about to set).  The residual pieces are reduced in a fixed
// order, so the test is deterministic.
template <int PER>
__device__ __forceinline__ void project_check_body(const double* __restrict__ mpart,
                                                   const double* __restrict__ rpart, int np, int N,
                                                   int dom, double* p, SolveState* st, double* hist,
                                                   int blk, int nblk) {
  __shared__ double red[4];
  __shared__ double sh_mean;
  __shared__ int sh_last;
  // every global read of the block is issued before the first wait: the done
  // flag, both sets of tile partials, the block's part of p and the state the
  // last workgroup updates (only the last workgroup of this launch writes it,
  // after every workgroup has passed its reads)
  const int done = st->done;
  double fn2 = 0.0, tl2 = 0.0;
  int its = 0, mxit = 0;
  if (threadIdx.x == 0) {
    fn2 = st->fnorm2;
    tl2 = st->tol2;
    its = st->iters;
    mxit = st->maxit;
  }
  // the tile partials in chunks of eight rounds, each chunk's loads issued
  // together; a thread still adds its partials k = tid, tid + 256, ... in
  // increasing order, so every workgroup forms the same sums
  double s1 = 0.0, s2 = 0.0, s3 = 0.0;
  for (int k0 = threadIdx.x; k0 < np; k0 += 8 * 256) {
    double a[8], b[8], c[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const int k = k0 + r * 256;
      const bool ok = k < np;
      a[r] = ok ? mpart[2 * k] : 0.0;
      b[r] = ok ? mpart[2 * k + 1] : 0.0;
      c[r] = ok ? rpart[k] : 0.0;
    }
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      if (k0 + r * 256 < np) {
        s1 += a[r];
        s2 += b[r];
        s3 += c[r];
      }
    }
  }
  const int n = (N + 1) * (N + 1);
  constexpr int BLOCK = PER * 256;
  double pv[PER];
  bool in[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int e = blk * BLOCK + k * 256 + threadIdx.x;
    in[k] = e < n && (dom == SMG_DOM_SQUARE || dom_p(N, dom, e % (N + 1), e / (N + 1)));
    pv[k] = in[k] ? p[e] : 0.0;
  }
  if (done) return;   // the same value in every thread of the block
  const double t1 = wg_sum<256>(s1, red);
  __syncthreads();
  const double t2 = wg_sum<256>(s2, red);
  if (threadIdx.x == 0) sh_mean = t1 / t2;
  __syncthreads();
  const double m = sh_mean;
#pragma unroll
  for (int k = 0; k < PER; ++k)
    if (in[k]) p[blk * BLOCK + k * 256 + threadIdx.x] = pv[k] - m;
  __syncthreads();
  // No fence before the ticket: the last workgroup reads nothing that the
  // others write in this launch (only the partials of the previous launch);
  // the ticket only orders their reads of the done flag before its write.
  if (threadIdx.x == 0) {
    const unsigned ticket = atomicAdd(&st->arrive, 1u);
    sh_last = (ticket == (unsigned)nblk - 1) ? 1 : 0;
  }
  __syncthreads();
  if (!sh_last) return;
  const double r2 = wg_sum<256>(s3, red);
  if (threadIdx.x == 0) {
    const double rel = sqrt(r2 / fn2);
    const int it = its + 1;
    st->relres = rel;
    st->iters = it;
    if (hist) hist[it - 1] = rel;
    st->arrive = 0u;
    if (!(rel == rel) || rel > 1e300) st->done = 3;
    else if (r2 <= tl2 * fn2) st->done = 1;
    else if (rel > 1e6) st->done = 2;
    else if (it >= mxit) st->done = 4;
  }
}

__global__ __launch_bounds__(256) void k_project_check(const double* __restrict__ mpart,
                                                       const double* __restrict__ rpart, int np, int N,
                                                       int dom, double* p, SolveState* st, double* hist) {
  if (pc_per_thread(N) == 16) project_check_body<16>(mpart, rpart, np, N, dom, p, st, hist, blockIdx.x, gridDim.x);
  else project_check_body<4>(mpart, rpart, np, N, dom, p, st, hist, blockIdx.x, gridDim.x);
}

__host__ __device__ int pc_blocks(int N) {
  const int block = pc_per_thread(N) * 256;
  return ((N + 1) * (N + 1) + block - 1) / block;
}

void launch_project_check(const double* mpart, const double* rpart, int np, int N, int dom, double* p,
                          SolveState* st, double* hist, hipStream_t s) {
  k_project_check<<<pc_blocks(N), 256, 0, s>>>(mpart, rpart, np, N, dom, p, st, hist);
}

template <bool PACK>
__global__ __launch_bounds__(256) void k_pc_b(const JobArg<PCJob> A) {
  int tile;
  const PCJob J = block_job<PACK>(A, (int)blockIdx.x, tile);
  if (pc_per_thread(J.N) == 16)
    project_check_body<16>(J.mpart, J.rpart, J.np, J.N, J.dom, J.p, J.st, J.hist, tile, pc_blocks(J.N));
  else
    project_check_body<4>(J.mpart, J.rpart, J.np, J.N, J.dom, J.p, J.st, J.hist, tile, pc_blocks(J.N));
}

void launch_pc_b(const JobArg<PCJob>& A, int nb, hipStream_t s) {
  if (A.n > 0) k_pc_b<true><<<nb, 256, 0, s>>>(A);
  else k_pc_b<false><<<nb, 256, 0, s>>>(A);
}

}  // namespace smg
