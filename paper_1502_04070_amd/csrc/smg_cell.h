// Device helpers shared by the fused kernels: the saddle operator of one
// square of the lattice, evaluated from values staged in LDS windows.
//
// A square (i, j) owns the lattice points V = (2i, 2j), H = (2i+1, 2j),
// E = (2i, 2j+1), D = (2i+1, 2j+1) (both velocity components) and the
// pressure vertex (i, j).  For it, cell_apply computes
//   y[2*cls + c] = (A u + B^T p)_c at the owned point of class cls,
//   y[8]         = (B u) at the vertex,
// from a velocity window U[2][UH][UW] and a pressure window P[PH][PW]; (ua, ub)
// are the window coordinates of the V point and (pa, pb) those of the vertex.
// The windows must hold zeros at lattice points outside the interior of the
// velocity space and at vertices outside the grid.
#pragma once
#include "smg_internal.h"
#include "smg_stage.h"

namespace smg {
#include "stencils.inc"
#include "smg_uj.h"
}

namespace smg {
using namespace smg_stencil;

template <int CLS, class T, class FU, class FC>
__device__ __forceinline__ T cell_a_row(FU U, FC C) {
  if constexpr (CLS == 0) return SMG_A_ROW_V(U, C);
  else if constexpr (CLS == 1) return SMG_A_ROW_H(U, C);
  else if constexpr (CLS == 2) return SMG_A_ROW_E(U, C);
  else return SMG_A_ROW_D(U, C);
}
template <int CLS, class T, class FP>
__device__ __forceinline__ T cell_btx(FP P) {
  if constexpr (CLS == 0) return SMG_BTX_ROW_V(P);
  else if constexpr (CLS == 1) return SMG_BTX_ROW_H(P);
  else if constexpr (CLS == 2) return SMG_BTX_ROW_E(P);
  else return SMG_BTX_ROW_D(P);
}
template <int CLS, class T, class FP>
__device__ __forceinline__ T cell_bty(FP P) {
  if constexpr (CLS == 0) return SMG_BTY_ROW_V(P);
  else if constexpr (CLS == 1) return SMG_BTY_ROW_H(P);
  else if constexpr (CLS == 2) return SMG_BTY_ROW_E(P);
  else return SMG_BTY_ROW_D(P);
}
template <int CLS, class T, class FR>
__device__ __forceinline__ T cell_res(FR R) {
  if constexpr (CLS == 0) return SMG_RES_ROW_V(R);
  else if constexpr (CLS == 1) return SMG_RES_ROW_H(R);
  else if constexpr (CLS == 2) return SMG_RES_ROW_E(R);
  else return SMG_RES_ROW_D(R);
}

// Velocity rows of class CLS (both components) at window position (ua, ub).
template <int CLS, class T, bool HU, bool HP, class UA, class PA>
__device__ __forceinline__ void cell_vel(const LevelCoef<T>& L, UA Uc, PA P, T& y0, T& y1) {
  auto C = [&](int g) -> T { return L.acoef[CLS][g]; };
  T r0 = T(0), r1 = T(0);
  if constexpr (HU) {
    auto U0 = [&](int da, int db) -> T { return Uc(0, da, db); };
    auto U1 = [&](int da, int db) -> T { return Uc(1, da, db); };
    r0 = cell_a_row<CLS, T>(U0, C);
    r1 = cell_a_row<CLS, T>(U1, C);
  }
  if constexpr (HP && CLS != 0) {
    r0 += L.h * cell_btx<CLS, T>(P);
    r1 += L.h * cell_bty<CLS, T>(P);
  }
  y0 = r0;
  y1 = r1;
}

// y[0..7]: velocity rows (class-major, component-minor), y[8]: pressure row.
// UA(c, a, b) reads component c at offset (a, b) from the V point of the
// square, PA(i, j) the pressure at offset (i, j) from its vertex.
template <class T, bool HU, bool HP, class UA, class PA>
__device__ __forceinline__ void cell_apply_acc(const LevelCoef<T>& L, UA U, PA P, T y[9]) {
  {
    auto Uc = [&](int c, int da, int db) -> T { return U(c, da, db); };
    cell_vel<0, T, HU, HP>(L, Uc, P, y[0], y[1]);
  }
  {
    auto Uc = [&](int c, int da, int db) -> T { return U(c, 1 + da, db); };
    auto Pc = [&](int di, int dj) -> T { return P(di, dj); };
    cell_vel<1, T, HU, HP>(L, Uc, Pc, y[2], y[3]);
  }
  {
    auto Uc = [&](int c, int da, int db) -> T { return U(c, da, 1 + db); };
    cell_vel<2, T, HU, HP>(L, Uc, P, y[4], y[5]);
  }
  {
    auto Uc = [&](int c, int da, int db) -> T { return U(c, 1 + da, 1 + db); };
    cell_vel<3, T, HU, HP>(L, Uc, P, y[6], y[7]);
  }
  if constexpr (HU) {
    auto U0 = [&](int da, int db) -> T { return U(0, da, db); };
    auto U1 = [&](int da, int db) -> T { return U(1, da, db); };
    y[8] = L.h * (SMG_BX_ROW(U0) + SMG_BY_ROW(U1));
  } else {
    y[8] = T(0);
  }
}

// The same on fixed-size LDS windows U[2][UH][UW] and P[.][PW].
template <class T, bool HU, bool HP, int UH, int UW, int PW>
__device__ __forceinline__ void cell_apply(const LevelCoef<T>& L, const T (*U)[UH][UW], int ua, int ub,
                                           const T* P, int pa, int pb, T y[9]) {
  auto UA = [&](int c, int da, int db) -> T { return U[c][ub + db][ua + da]; };
  auto PA = [&](int di, int dj) -> T { return P[(pb + dj) * PW + (pa + di)]; };
  cell_apply_acc<T, HU, HP>(L, UA, PA, y);
}

// ---- rows on either grid: DOM = SMG_DOM_UNIONJACK sums them square by
// square (smg_uj.h), every other domain uses the lattice stencils.  (i, j) is
// the square in global indices (the diagonal direction depends on it), U
// reads component c at an offset from the square's V point and P the
// pressure at an offset from its vertex.

// all nine rows of square (i, j) and 1 / Ahat at its four nodes
template <class T, bool HU, bool HP, int DOM, class UA, class PA>
__device__ __forceinline__ void sq_rows(const LevelCoef<T>& L, int i, int j, UA U, PA P, T y[9], T ad[4]) {
  if constexpr (DOM == SMG_DOM_UNIONJACK) {
    const int N = L.N;
    auto OR = [&](int di, int dj) { return uj_orient(N, i + di, j + dj); };
    T d;
    uj_vel_rows<0, T>(L.bh2, L.h, HU, HP, U, P, OR, y[0], y[1], d);
    ad[0] = T(1) / d;
    uj_vel_rows<1, T>(L.bh2, L.h, HU, HP, U, P, OR, y[2], y[3], d);
    ad[1] = T(1) / d;
    uj_vel_rows<2, T>(L.bh2, L.h, HU, HP, U, P, OR, y[4], y[5], d);
    ad[2] = T(1) / d;
    uj_vel_rows<3, T>(L.bh2, L.h, HU, HP, U, P, OR, y[6], y[7], d);
    ad[3] = T(1) / d;
    y[8] = HU ? uj_p_row<T>(L.h, U, OR) : T(0);
  } else {
    cell_apply_acc<T, HU, HP>(L, U, P, y);
#pragma unroll
    for (int k = 0; k < 4; ++k) ad[k] = L.adinv[k];
  }
}

// the two velocity rows of class CLS of square (i, j) and 1 / Ahat there
template <int CLS, class T, bool HU, bool HP, int DOM, class UA, class PA>
__device__ __forceinline__ void sq_vel(const LevelCoef<T>& L, int i, int j, UA U, PA P, T& y0, T& y1, T& ad) {
  if constexpr (DOM == SMG_DOM_UNIONJACK) {
    const int N = L.N;
    auto OR = [&](int di, int dj) { return uj_orient(N, i + di, j + dj); };
    T d;
    uj_vel_rows<CLS, T>(L.bh2, L.h, HU, HP, U, P, OR, y0, y1, d);
    ad = T(1) / d;
  } else {
    constexpr int DA = CLS & 1, DB = CLS >> 1;
    auto Uc = [&](int c, int da, int db) -> T { return U(c, DA + da, DB + db); };
    cell_vel<CLS, T, HU, HP>(L, Uc, P, y0, y1);
    ad = L.adinv[CLS];
  }
}

// the pressure row (B u) at the vertex of square (i, j)
template <class T, int DOM, class UA>
__device__ __forceinline__ T sq_prow(const LevelCoef<T>& L, int i, int j, UA U) {
  if constexpr (DOM == SMG_DOM_UNIONJACK) {
    const int N = L.N;
    auto OR = [&](int di, int dj) { return uj_orient(N, i + di, j + dj); };
    return uj_p_row<T>(L.h, U, OR);
  } else {
    auto U0 = [&](int da, int db) -> T { return U(0, da, db); };
    auto U1 = [&](int da, int db) -> T { return U(1, da, db); };
    return L.h * (SMG_BX_ROW(U0) + SMG_BY_ROW(U1));
  }
}

// restriction (transposed prolongation) at the coarse node of class CLS owned
// by coarse square (I, J) of a grid with Nc squares per side; R(fa, fb) reads
// the fine defect at (2A + fa, 2B + fb), (A, B) the coarse node
template <int CLS, class T, int DOM, class FR>
__device__ __forceinline__ T sq_res(int Nc, int I, int J, FR R) {
  if constexpr (DOM == SMG_DOM_UNIONJACK) {
    constexpr int CA = CLS & 1, CB = CLS >> 1;
    const int A = 2 * I + CA, B = 2 * J + CB;
    T v = T(0);
#pragma unroll
    for (int dj = (CB ? 0 : -1); dj <= 0; ++dj)
#pragma unroll
      for (int di = (CA ? 0 : -1); di <= 0; ++di) {
        const int SI = I + di, SJ = J + dj;
        if (SI < 0 || SJ < 0) continue;
        const int o = uj_orient_c(Nc, SI, SJ);
        const int cl = 3 * (CB - 2 * dj) + (CA - 2 * di);
        for (int f = 0; f < 16; ++f) {
          const double w = smg_stencil::UJ_PRO[o][f][cl];
          if (w != 0.0) v += T(w) * R(4 * SI + (f & 3) - 2 * A, 4 * SJ + (f >> 2) - 2 * B);
        }
      }
    return v;
  } else {
    return cell_res<CLS, T>(R);
  }
}

// pressure restriction at coarse vertex (I, J); Rp(di, dj) reads the fine
// defect at (2I + di, 2J + dj)
template <class T, int DOM, class FR>
__device__ __forceinline__ T sq_resp(int Nc, int I, int J, FR Rp) {
  if constexpr (DOM == SMG_DOM_UNIONJACK) {
    T v = T(0);
    for (int dj = -1; dj <= 0; ++dj)
      for (int di = -1; di <= 0; ++di) {
        const int SI = I + di, SJ = J + dj;
        if (SI < 0 || SJ < 0) continue;
        const int o = uj_orient_c(Nc, SI, SJ), q = 2 * (-dj) + (-di);
        for (int vv = 0; vv < 4; ++vv) {
          const double w = smg_stencil::UJ_PP[o][vv][q];
          if (w != 0.0) v += T(w) * Rp(2 * di + (vv & 1), 2 * dj + (vv >> 1));
        }
      }
    return v;
  } else {
    return Rp(0, 0) + T(0.5) * (Rp(1, 0) + Rp(-1, 0) + Rp(0, 1) + Rp(0, -1) + Rp(1, 1) + Rp(-1, -1));
  }
}

// Sum over the workgroup (NT a multiple of 64); result valid in thread 0.
template <int NT>
__device__ __forceinline__ double wg_sum(double v, double* red) {
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

__device__ __forceinline__ int xcd_remap(int bid, int nb) {
  const int xcd = bid & 7, idx = bid >> 3;
  const int per = nb >> 3, rem = nb & 7;
  return xcd * per + (xcd < rem ? xcd : rem) + idx;
}

}  // namespace smg
