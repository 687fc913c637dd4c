// Rows of the operators on the union-jack grid, summed square by square.
//
// On this grid the diagonal direction changes between the quarters of the
// unit square, so a row is not one constant lattice stencil: it is the sum,
// over the squares that contain the node, of that square's local matrix row
// (Section 2: the Galerkin matrices are sums of element contributions).  The
// square-local matrices of both diagonal directions are exact tables
// (smg_stencil::UJ_*).  Everything here is written for an owner square (i, j)
// and its accessors, so the same code serves the tiled kernels (LDS windows)
// and the host assembly of the coarsest-grid matrix.  Included inside
// namespace smg after stencils.inc.
#pragma once

// Velocity rows at the node of class CLS owned by square (i, j): the
// squares (i + DI, j + DJ) that contain it are DI in {-1, 0} if the node lies
// on the square's left edge (DA = 0), else 0; the same for DJ.
//   U(c, la, lb): u_c at the lattice point (2i + la, 2j + lb)
//   P(pi, pj):    p at the vertex (i + pi, j + pj)
//   OR(di, dj):   diagonal direction of square (i + di, j + dj)
// Accumulates y_c += (A u_c)_row (hu) + h (B_c^T p)_row (hp) and the diagonal
// entry of A (the same for both components).
template <int O, int LN, int DI, int DJ, class T, class UA, class PA>
__host__ __device__ __forceinline__ void uj_vel_sq(T bh2, T h, bool hu, bool hp, UA& U, PA& P, T& y0, T& y1,
                                                   T& diag) {
  using namespace smg_stencil;
  if (hu) {
#pragma unroll
    for (int m = 0; m < 9; ++m) {
      const T a = T(UJ_K[O][LN][m]) + bh2 * T(UJ_M[O][LN][m]);
      if (UJ_K[O][LN][m] != 0.0 || UJ_M[O][LN][m] != 0.0) {
        y0 += a * U(0, 2 * DI + m % 3, 2 * DJ + m / 3);
        y1 += a * U(1, 2 * DI + m % 3, 2 * DJ + m / 3);
      }
    }
  }
  diag += T(UJ_K[O][LN][LN]) + bh2 * T(UJ_M[O][LN][LN]);
  if (hp) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (UJ_BX[O][q][LN] != 0.0) y0 += h * T(UJ_BX[O][q][LN]) * P(DI + q % 2, DJ + q / 2);
      if (UJ_BY[O][q][LN] != 0.0) y1 += h * T(UJ_BY[O][q][LN]) * P(DI + q % 2, DJ + q / 2);
    }
  }
}

template <int DA, int DB, int DI, int DJ, class T, class UA, class PA, class OA>
__host__ __device__ __forceinline__ void uj_vel_part(T bh2, T h, bool hu, bool hp, UA& U, PA& P, OA& OR, T& y0,
                                                     T& y1, T& diag) {
  constexpr int LN = 3 * (DB - 2 * DJ) + (DA - 2 * DI);
  if (OR(DI, DJ) == 0) uj_vel_sq<0, LN, DI, DJ>(bh2, h, hu, hp, U, P, y0, y1, diag);
  else uj_vel_sq<1, LN, DI, DJ>(bh2, h, hu, hp, U, P, y0, y1, diag);
}

template <int CLS, class T, class UA, class PA, class OA>
__host__ __device__ __forceinline__ void uj_vel_rows(T bh2, T h, bool hu, bool hp, UA& U, PA& P, OA& OR, T& y0,
                                                     T& y1, T& diag) {
  constexpr int DA = CLS & 1, DB = CLS >> 1;
  y0 = y1 = diag = T(0);
  uj_vel_part<DA, DB, 0, 0>(bh2, h, hu, hp, U, P, OR, y0, y1, diag);
  if constexpr (DA == 0) uj_vel_part<DA, DB, -1, 0>(bh2, h, hu, hp, U, P, OR, y0, y1, diag);
  if constexpr (DB == 0) uj_vel_part<DA, DB, 0, -1>(bh2, h, hu, hp, U, P, OR, y0, y1, diag);
  if constexpr (DA == 0 && DB == 0) uj_vel_part<DA, DB, -1, -1>(bh2, h, hu, hp, U, P, OR, y0, y1, diag);
}

// Pressure row (B u) at the vertex (i, j): the four squares around it, the
// vertex being corner (-DI, -DJ) of square (i + DI, j + DJ).  Times h.
template <int O, int DI, int DJ, class T, class UA>
__host__ __device__ __forceinline__ T uj_p_sq(UA& U) {
  using namespace smg_stencil;
  constexpr int Q = 2 * (-DJ) + (-DI);
  T y = T(0);
#pragma unroll
  for (int m = 0; m < 9; ++m) {
    if (UJ_BX[O][Q][m] != 0.0) y += T(UJ_BX[O][Q][m]) * U(0, 2 * DI + m % 3, 2 * DJ + m / 3);
    if (UJ_BY[O][Q][m] != 0.0) y += T(UJ_BY[O][Q][m]) * U(1, 2 * DI + m % 3, 2 * DJ + m / 3);
  }
  return y;
}

template <int DI, int DJ, class T, class UA, class OA>
__host__ __device__ __forceinline__ T uj_p_part(UA& U, OA& OR) {
  return OR(DI, DJ) == 0 ? uj_p_sq<0, DI, DJ, T>(U) : uj_p_sq<1, DI, DJ, T>(U);
}

template <class T, class UA, class OA>
__host__ __device__ __forceinline__ T uj_p_row(T h, UA& U, OA& OR) {
  return h * (uj_p_part<0, 0, T>(U, OR) + uj_p_part<-1, 0, T>(U, OR) + uj_p_part<0, -1, T>(U, OR) +
              uj_p_part<-1, -1, T>(U, OR));
}

// Diagonal entry of A at lattice point (a, b) of the N x N union-jack grid
__host__ __device__ inline double uj_adiag(int N, int a, int b, double bh2) {
  using namespace smg_stencil;
  const int DA = a & 1, DB = b & 1, i = a >> 1, j = b >> 1;
  double d = 0.0;
  for (int dj = (DB ? 0 : -1); dj <= 0; ++dj)
    for (int di = (DA ? 0 : -1); di <= 0; ++di) {
      const int o = uj_orient(N, i + di, j + dj);
      const int ln = 3 * (DB - 2 * dj) + (DA - 2 * di);
      d += UJ_K[o][ln][ln] + bh2 * UJ_M[o][ln][ln];
    }
  return d;
}

// P2 mass row at lattice point (a, b) (all nodes: loads and their transpose),
// U(la, lb) reads the scalar field at (2i + la, 2j + lb) of the owner square;
// squares outside the grid contribute nothing.  Unit legs (times h^2 at use).
template <class T, class UA>
__host__ __device__ inline T uj_m_row(int N, int a, int b, UA& U) {
  using namespace smg_stencil;
  const int DA = a & 1, DB = b & 1, i = a >> 1, j = b >> 1;
  T y = T(0);
  for (int dj = (DB ? 0 : -1); dj <= 0; ++dj)
    for (int di = (DA ? 0 : -1); di <= 0; ++di) {
      if (i + di < 0 || i + di >= N || j + dj < 0 || j + dj >= N) continue;
      const int o = uj_orient(N, i + di, j + dj);
      const int ln = 3 * (DB - 2 * dj) + (DA - 2 * di);
      for (int m = 0; m < 9; ++m) y += T(UJ_M[o][ln][m]) * U(2 * di + m % 3, 2 * dj + m / 3);
    }
  return y;
}

// P1 mass row at vertex (i, j); G(pi, pj) reads g at (i + pi, j + pj)
template <class T, class GA>
__host__ __device__ inline T uj_mp_row(int N, int i, int j, GA& G) {
  using namespace smg_stencil;
  T y = T(0);
  for (int dj = -1; dj <= 0; ++dj)
    for (int di = -1; di <= 0; ++di) {
      if (i + di < 0 || i + di >= N || j + dj < 0 || j + dj >= N) continue;
      const int o = uj_orient(N, i + di, j + dj), q = 2 * (-dj) + (-di);
      for (int r = 0; r < 4; ++r) y += T(UJ_MP[o][q][r]) * G(di + r % 2, dj + r / 2);
    }
  return y;
}

// Prolongation from the coarse grid (Nc squares per side): the fine lattice
// point (4I + ra, 4J + rb) owned by coarse square (I, J) (0 <= ra, rb < 4) is
// sum_c PRO[o][4 rb + ra][c] Z(c) over the square's coarse nodes
// (2I + c % 3, 2J + c / 3).  Squares I = Nc or J = Nc own only points on the
// right and top boundary, whose rule (along the edge) does not depend on o.
__host__ __device__ inline int uj_orient_c(int Nc, int I, int J) {
  return uj_orient(Nc, I < Nc ? I : Nc - 1, J < Nc ? J : Nc - 1);
}
