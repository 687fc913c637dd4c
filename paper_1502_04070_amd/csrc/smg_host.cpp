// Host-only part of the runtime (see smg_host.h).
#include "smg_host.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <string>

namespace smg {
#include "stencils.inc"
#include "smg_uj.h"
}

namespace smg {
namespace host {

using smg_stencil::A_K;
using smg_stencil::A_M;
using smg_stencil::DIAG_K;
using smg_stencil::DIAG_M;

namespace {
thread_local std::string g_err = "no error";
}

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

const char* last_error() { return g_err.c_str(); }

int check_params(int N, double beta, const smg_params& prm, int* L) {
  if (prm.smoother != SMG_SMOOTHER_NE && prm.smoother != SMG_SMOOTHER_UZAWA)
    return fail(SMG_EINVAL, "unknown smoother %d", prm.smoother);
  if (!(prm.tau > 0) || !(prm.sigma > 0) || !std::isfinite(prm.tau) || !std::isfinite(prm.sigma))
    return fail(SMG_EINVAL, "tau and sigma must be finite and > 0");
  if (prm.nu_pre < 0 || prm.nu_post < 0 || prm.nu_pre > 64 || prm.nu_post > 64)
    return fail(SMG_EINVAL, "smoothing steps must be in 0..64");
  if (prm.gamma != 1 && prm.gamma != 2) return fail(SMG_EINVAL, "gamma must be 1 or 2");
  if (prm.n0 < 2 || prm.n0 > 8) return fail(SMG_EINVAL, "n0 must be in 2..8");
  if (prm.fuse_depth < 0 || prm.fuse_depth > 2) return fail(SMG_EINVAL, "fuse_depth must be 0, 1 or 2");
  if (prm.coarse_max_n < 0) return fail(SMG_EINVAL, "coarse_max_n must be >= 0");
  if (prm.tile_x != 0 && prm.tile_x != 8 && prm.tile_x != 16) return fail(SMG_EINVAL, "tile_x must be 0, 8 or 16");
  if (prm.domain != SMG_DOM_SQUARE && prm.domain != SMG_DOM_LSHAPE && prm.domain != SMG_DOM_UNIONJACK)
    return fail(SMG_EINVAL, "unknown domain %d", prm.domain);
  if (prm.domain == SMG_DOM_LSHAPE && prm.n0 % 2) return fail(SMG_EINVAL, "the L-shaped domain needs an even n0");
  if (prm.domain == SMG_DOM_UNIONJACK && prm.n0 % 2) return fail(SMG_EINVAL, "the union-jack grid needs an even n0");
  if (!(beta >= 0) || !std::isfinite(beta)) return fail(SMG_EINVAL, "beta must be finite and >= 0");
  int levels = 0;
  int n = N;
  if (n < prm.n0) return fail(SMG_EINVAL, "N=%d below n0=%d", N, prm.n0);
  while (n > prm.n0 && n % 2 == 0) { n /= 2; ++levels; }
  if (n != prm.n0) return fail(SMG_EINVAL, "N=%d is not n0 * 2^L (n0=%d)", N, prm.n0);
  if (N > 8192) return fail(SMG_EINVAL, "N=%d too large", N);
  *L = levels;
  return SMG_OK;
}

void make_coef(int N, int dom, double beta, LevelCoef<double>& c, LevelCoef<float>& c32) {
  const double h = 1.0 / N, bh2 = beta * h * h;
  c.N = c32.N = N;
  c.dom = c32.dom = dom;
  c.h = h;
  c32.h = (float)h;
  c.bh2 = bh2;
  c32.bh2 = (float)bh2;
  for (int k = 0; k < 4; ++k) {
    for (int g = 0; g < 5; ++g) {
      c.acoef[k][g] = A_K[k][g] + bh2 * A_M[k][g];
      c32.acoef[k][g] = (float)c.acoef[k][g];
    }
    c.adinv[k] = 1.0 / (DIAG_K[k] + bh2 * DIAG_M[k]);
    c32.adinv[k] = (float)c.adinv[k];
  }
  c.sinv = nullptr;
  c32.sinv = nullptr;
}

void apply(int N, const LevelCoef<double>& c, const double* u, const double* p, double* yu, double* yp) {
  using T = double;
  const int M = 2 * N + 1, NP = N + 1;
  const T h = c.h;
  auto Ug = [&](int comp, int a, int b) -> T {
    return dom_u(N, c.dom, a, b) ? u[(size_t)comp * M * M + (size_t)b * M + a] : T(0);
  };
  auto Pg = [&](int i, int j) -> T { return dom_p(N, c.dom, i, j) ? p[(size_t)j * NP + i] : T(0); };
  if (c.dom == SMG_DOM_UNIONJACK) {
    // rows summed square by square, as in the kernels
    for (int j = 0; j < NP; ++j)
      for (int i = 0; i < NP; ++i) {
        auto U = [&](int comp, int la, int lb) -> T { return Ug(comp, 2 * i + la, 2 * j + lb); };
        auto P = [&](int di, int dj) -> T { return Pg(i + di, j + dj); };
        auto OR = [&](int di, int dj) { return uj_orient(N, i + di, j + dj); };
        for (int cls = 0; cls < 4; ++cls) {
          const int a = 2 * i + (cls & 1), b = 2 * j + (cls >> 1);
          if (a > 2 * N || b > 2 * N) continue;
          T y0 = T(0), y1 = T(0), d = T(0);
          if (dom_u(N, c.dom, a, b)) {
            switch (cls) {
              case 0: uj_vel_rows<0, T>(c.bh2, h, true, true, U, P, OR, y0, y1, d); break;
              case 1: uj_vel_rows<1, T>(c.bh2, h, true, true, U, P, OR, y0, y1, d); break;
              case 2: uj_vel_rows<2, T>(c.bh2, h, true, true, U, P, OR, y0, y1, d); break;
              default: uj_vel_rows<3, T>(c.bh2, h, true, true, U, P, OR, y0, y1, d); break;
            }
          }
          yu[(size_t)b * M + a] = y0;
          yu[(size_t)M * M + (size_t)b * M + a] = y1;
        }
        yp[(size_t)j * NP + i] = uj_p_row<T>(h, U, OR);
      }
    return;
  }
  for (int comp = 0; comp < 2; ++comp)
    for (int b = 0; b < M; ++b)
      for (int a = 0; a < M; ++a) {
        T y = T(0);
        if (dom_u(N, c.dom, a, b)) {
          const int cls = (a & 1) + 2 * (b & 1), i = a >> 1, j = b >> 1;
          auto U = [&](int da, int db) -> T { return Ug(comp, a + da, b + db); };
          auto C = [&](int g) -> T { return c.acoef[cls][g]; };
          auto P = [&](int di, int dj) -> T { return Pg(i + di, j + dj); };
          switch (cls) {
            case 0: y = SMG_A_ROW_V(U, C) + h * (comp == 0 ? SMG_BTX_ROW_V(P) : SMG_BTY_ROW_V(P)); break;
            case 1: y = SMG_A_ROW_H(U, C) + h * (comp == 0 ? SMG_BTX_ROW_H(P) : SMG_BTY_ROW_H(P)); break;
            case 2: y = SMG_A_ROW_E(U, C) + h * (comp == 0 ? SMG_BTX_ROW_E(P) : SMG_BTY_ROW_E(P)); break;
            default: y = SMG_A_ROW_D(U, C) + h * (comp == 0 ? SMG_BTX_ROW_D(P) : SMG_BTY_ROW_D(P)); break;
          }
        }
        yu[(size_t)comp * M * M + (size_t)b * M + a] = y;
      }
  for (int j = 0; j < NP; ++j)
    for (int i = 0; i < NP; ++i) {
      auto U0 = [&](int da, int db) -> T { return Ug(0, 2 * i + da, 2 * j + db); };
      auto U1 = [&](int da, int db) -> T { return Ug(1, 2 * i + da, 2 * j + db); };
      yp[(size_t)j * NP + i] = dom_p(N, c.dom, i, j) ? h * (SMG_BX_ROW(U0) + SMG_BY_ROW(U1)) : T(0);
    }
}

int coarse_size(int N0) {
  const int ni = 2 * N0 - 1, NP = N0 + 1;
  return 2 * ni * ni + NP * NP + 1;
}

void bordered_matrix(int N0, const LevelCoef<double>& c, std::vector<double>& A) {
  const int M = 2 * N0 + 1, ni = 2 * N0 - 1, nu = ni * ni, NP = N0 + 1;
  const int nc = coarse_size(N0);
  A.assign((size_t)nc * nc, 0.0);
  std::vector<double> u(2 * M * M), p(NP * NP), yu(2 * M * M), yp(NP * NP);
  auto lat_u = [&](int k) {
    const int comp = k / nu, q = k % nu;
    return comp * M * M + (1 + q / ni) * M + (1 + q % ni);
  };
  for (int k = 0; k < nc - 1; ++k) {
    std::fill(u.begin(), u.end(), 0.0);
    std::fill(p.begin(), p.end(), 0.0);
    if (k < 2 * nu) u[lat_u(k)] = 1.0; else p[k - 2 * nu] = 1.0;
    apply(N0, c, u.data(), p.data(), yu.data(), yp.data());
    for (int r = 0; r < 2 * nu; ++r) A[(size_t)r * nc + k] = yu[lat_u(r)];
    for (int r = 0; r < NP * NP; ++r) A[(size_t)(2 * nu + r) * nc + k] = yp[r];
  }
  const double h2 = 1.0 / ((double)N0 * N0);
  for (int j = 0; j < NP; ++j)
    for (int i = 0; i < NP; ++i) {
      const double m = h2 * p1_count_w(N0, c.dom, i, j);
      A[(size_t)(2 * nu + j * NP + i) * nc + (nc - 1)] = m;
      A[(size_t)(nc - 1) * nc + (2 * nu + j * NP + i)] = m;
    }
  // unknowns outside the domain (lattice points and vertices of the removed
  // part) are decoupled: an identity row and column keep them at zero
  for (int k = 0; k < 2 * nu; ++k) {
    const int q = k % nu;
    if (!dom_u(N0, c.dom, 1 + q % ni, 1 + q / ni)) A[(size_t)k * nc + k] = 1.0;
  }
  for (int k = 0; k < NP * NP; ++k)
    if (!dom_p(N0, c.dom, k % NP, k / NP)) A[(size_t)(2 * nu + k) * nc + (2 * nu + k)] = 1.0;
}

int coarse_inverse(int N0, const LevelCoef<double>& c, std::vector<double>& inv_colmajor) {
  const int nc = coarse_size(N0);
  std::vector<double> A;
  bordered_matrix(N0, c, A);
  // symmetric equilibration S A S (s_k = 1 / sqrt(max_q |A_kq|)): the blocks
  // scale like beta h^2, h and h^2, so without it the pivots of the pressure
  // rows fall below any fixed threshold relative to the largest entry once
  // beta h^2 is large; the inverse is S (S A S)^-1 S
  std::vector<double> sc(nc);
  for (int k = 0; k < nc; ++k) {
    double rmax = 0.0;
    for (int q = 0; q < nc; ++q) rmax = std::max(rmax, std::fabs(A[(size_t)k * nc + q]));
    sc[k] = rmax > 0.0 ? 1.0 / std::sqrt(rmax) : 1.0;
  }
  for (int k = 0; k < nc; ++k)
    for (int q = 0; q < nc; ++q) A[(size_t)k * nc + q] *= sc[k] * sc[q];
  double amax = 0.0;
  for (double v : A) amax = std::max(amax, std::fabs(v));
  // LU with partial pivoting, then solve for the identity
  std::vector<int> piv(nc);
  for (int k = 0; k < nc; ++k) {
    int r = k;
    for (int q = k + 1; q < nc; ++q)
      if (std::fabs(A[(size_t)q * nc + k]) > std::fabs(A[(size_t)r * nc + k])) r = q;
    if (!(std::fabs(A[(size_t)r * nc + k]) > 1e-13 * amax))
      return fail(SMG_ESINGULAR, "coarsest-grid matrix singular (pivot %d)", k);
    piv[k] = r;
    if (r != k)
      for (int q = 0; q < nc; ++q) std::swap(A[(size_t)k * nc + q], A[(size_t)r * nc + q]);
    const double d = A[(size_t)k * nc + k];
    for (int q = k + 1; q < nc; ++q) {
      const double l = A[(size_t)q * nc + k] / d;
      A[(size_t)q * nc + k] = l;
      if (l != 0.0)
        for (int w = k + 1; w < nc; ++w) A[(size_t)q * nc + w] -= l * A[(size_t)k * nc + w];
    }
  }
  inv_colmajor.assign((size_t)nc * nc, 0.0);
  std::vector<double> e(nc);
  for (int col = 0; col < nc; ++col) {
    std::fill(e.begin(), e.end(), 0.0);
    e[col] = 1.0;
    for (int k = 0; k < nc; ++k) std::swap(e[k], e[piv[k]]);
    for (int k = 0; k < nc; ++k)
      for (int q = 0; q < k; ++q) e[k] -= A[(size_t)k * nc + q] * e[q];
    for (int k = nc - 1; k >= 0; --k) {
      for (int q = k + 1; q < nc; ++q) e[k] -= A[(size_t)k * nc + q] * e[q];
      e[k] /= A[(size_t)k * nc + k];
    }
    // column `col` of the inverse: Inv[row][col] = s_row e[row] s_col; stored at [col * nc + row]
    for (int row = 0; row < nc; ++row) inv_colmajor[(size_t)col * nc + row] = sc[row] * e[row] * sc[col];
  }
  return SMG_OK;
}

void pack_starts(const std::vector<int>& tiles, int* start) {
  int st = 0;
  for (size_t k = 0; k < tiles.size(); ++k) {
    start[k] = st;
    st += tiles[k];
  }
  start[tiles.size()] = st;
}

std::vector<int> block_map(const std::vector<int>& tiles) {
  std::vector<int> map;
  const long max_job = (1L << (31 - BMAP_SHIFT)) - 1, max_tile = (1L << BMAP_SHIFT) - 1;
  if ((long)tiles.size() - 1 > max_job) return map;
  for (size_t k = 0; k < tiles.size(); ++k) {
    if (tiles[k] < 0 || tiles[k] - 1 > max_tile) return {};
    for (int t = 0; t < tiles[k]; ++t) map.push_back(bmap((int)k, t));
  }
  return map;
}

}  // namespace host
}  // namespace smg
