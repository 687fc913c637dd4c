// Internal interface between the host runtime (smg_capi.hip) and the HIP
// kernels (smg_kernels.hip).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace smg {

// The jobs of one batched launch.  Up to PACK_MAX jobs travel by value in the
// kernel arguments, with the first workgroup of each job, so a workgroup finds
// its job without a round trip to memory.  Larger batches use a device job
// table and a block map ((job << BMAP_SHIFT) | tile per workgroup); then n = 0.
constexpr int PACK_MAX = 8;
constexpr int BMAP_SHIFT = 20;
inline int bmap(int job, int tile) { return (job << BMAP_SHIFT) | tile; }

template <class J>
struct JobArg {
  const J* jobs;
  const int* map;
  int n;
  int start[PACK_MAX + 1];
  J pack[PACK_MAX];
};

// The job of workgroup b (after any block remapping) and its tile index, from
// the packed jobs (PACK) or from the table.  The two sources are separate
// instantiations, so that each reads its job through one address space with
// scalar loads.
template <bool PACK, class J>
__device__ __forceinline__ J block_job(const JobArg<J>& A, int b, int& tile) {
  if constexpr (PACK) {
    int k = 0;
#pragma unroll
    for (int q = 1; q < PACK_MAX; ++q) k += (q < A.n && b >= A.start[q]) ? 1 : 0;
    tile = b - A.start[k];
    return A.pack[k];
  } else {
    const int m = A.map[b];
    tile = m & ((1 << BMAP_SHIFT) - 1);
    return A.jobs[m >> BMAP_SHIFT];
  }
}

// Domains on the grid of N x N squares (lattice point (a, b) at
// (a / 2N, b / 2N), vertex (i, j) at (i / N, j / N)):
//   0: the unit square;
//   1: the L-shape, the unit square without [1/2, 1]^2 (N even);
//   2: the unit square on the union-jack grid (N even): the squares of the
//      lower-left and upper-right quarters are cut by the diagonal from their
//      lower-left to their upper-right corner, the others by the other
//      diagonal, so that the diagonals of the coarsest 2 x 2 grid meet at the
//      centre.
// dom_u: the lattice point carries velocity unknowns (inside, off the boundary);
// dom_p: the vertex belongs to the closed domain (pressure node);
// dom_sq: the square belongs to the domain.
enum { SMG_DOM_SQUARE = 0, SMG_DOM_LSHAPE = 1, SMG_DOM_UNIONJACK = 2 };

// diagonal of square (si, sj) on the union-jack grid: 0 from the lower-left to
// the upper-right corner, 1 from the upper-left to the lower-right corner
__host__ __device__ inline int uj_orient(int N, int si, int sj) {
  return ((2 * si < N) != (2 * sj < N)) ? 1 : 0;
}

__host__ __device__ inline bool dom_u(int N, int dom, int a, int b) {
  return a > 0 && a < 2 * N && b > 0 && b < 2 * N && !(dom == SMG_DOM_LSHAPE && a >= N && b >= N);
}
__host__ __device__ inline bool dom_p(int N, int dom, int i, int j) {
  return i >= 0 && i <= N && j >= 0 && j <= N && !(dom == SMG_DOM_LSHAPE && 2 * i > N && 2 * j > N);
}
__host__ __device__ inline bool dom_sq(int N, int dom, int si, int sj) {
  return si >= 0 && si < N && sj >= 0 && sj < N && !(dom == SMG_DOM_LSHAPE && 2 * si >= N && 2 * sj >= N);
}
// int phi_i / h^2 of the P1 basis function of vertex (i, j): (h^2 / 6) times
// the number of triangles of the domain around it (a square cut from its
// lower-left to its upper-right corner has two triangles at those corners
// and one at the other two; the other diagonal the reverse)
__host__ __device__ inline double p1_count_w(int N, int dom, int i, int j) {
  if (dom == SMG_DOM_UNIONJACK) {
    auto two = [&](int si, int sj, bool main_corner) {
      if (!dom_sq(N, dom, si, sj)) return 0;
      return (uj_orient(N, si, sj) == 0) == main_corner ? 2 : 1;
    };
    return (two(i - 1, j - 1, true) + two(i, j - 1, false) + two(i - 1, j, false) + two(i, j, true)) / 6.0;
  }
  const int c = 2 * dom_sq(N, dom, i - 1, j - 1) + dom_sq(N, dom, i, j - 1) + dom_sq(N, dom, i - 1, j) +
                2 * dom_sq(N, dom, i, j);
  return c / 6.0;
}

// Per-level constants of the operator (Section 2 matrices, Section 6
// preconditioner), in the arithmetic type T of the kernels.
template <class T>
struct LevelCoef {
  int N;             // cells per side
  int dom;           // domain (SMG_DOM_*)
  T acoef[4][5];     // A = K + beta h^2 M, grouped lattice taps per node class
  T adinv[4];        // 1 / Ahat per node class (V, H, E, D)
  T h;               // 1 / N (scales B and B^T)
  T bh2;             // beta h^2 (scales the mass part of A)
  const T* sinv;     // 1 / Shat at every pressure node, (N+1)^2
};

// One application of the generic fused stencil
//   out = base + w * D * (rhs - calA in)          (D = L^-1 rows or identity)
// on the velocity rows (ROWS & 1) and / or the pressure rows (ROWS & 2).
// NULL pointers mean "zero" (in_u, in_p, rhs, base) or "skip" (out).
// in_p_sub, if set, is subtracted from in_p on load (Uzawa pressure update).
// If partial is set, each tile writes its sum of (rhs - calA in)^2 over the
// rows it owns (interior velocity nodes, all pressure nodes).
template <class T>
struct StencilJob {
  LevelCoef<T> L;
  const T* in_u;
  const T* in_p;
  const T* in_p_sub;
  const T* rhs_u;
  const T* rhs_p;
  const T* base_u;
  const T* base_p;
  T* out_u;
  T* out_p;
  float* out32_u;      // if set, the rows' values rounded to FP32 go here
  float* out32_p;      // instead of out_u / out_p
  T w_u, w_p;          // weights of the velocity / pressure rows
  int diag_u, diag_p;  // 1: scale by Ahat^-1 / Shat^-1, 0: no scaling
  double* partial;     // per-tile partial sums, or NULL
  double* mean_partial;  // per tile: (sum w_i p_i, sum w_i) of in_p, or NULL
  const int* done;     // if non-NULL and *done != 0 the launch does nothing
};

enum { ROWS_U = 1, ROWS_P = 2, ROWS_UP = 3 };

// tile shape of the stencil kernels: TX x TY cells per workgroup
struct TileShape { int tx, ty; };
TileShape stencil_tile(int N);
int stencil_tiles(int N);

template <class T>
void launch_stencil(const StencilJob<T>& J, int rows, hipStream_t s);
// operation flags of a job (the compile-time mode of the stencil kernel)
template <class T>
unsigned stencil_flags(const StencilJob<T>& J, int rows);
// batched: jobs with identical flags, one tile shape (tx, ty) for all
template <class T>
void launch_stencil_b(const JobArg<StencilJob<T>>& A, int nb, int tx, int ty,
                      unsigned flags, int dom, hipStream_t s);
int stencil_tiles_shape(int N, int tx, int ty);

// batched prolongation (one job per instance)
template <class T>
struct ProJob {
  int Nc;
  int dom;
  const T* zu;
  const T* zp;
  T* u;
  T* p;
  const int* done;
};
int prolong_tiles(int Nc);
template <class T>
void launch_prolong_b(const JobArg<ProJob<T>>& A, int nb, hipStream_t s);

// batched elementwise: d += f (mode 1), d = 0 (mode 2)
struct EwJob {
  double* d;
  float* f;
  int64_t n;
  const int* done;
};
int ew_tiles(int64_t n);
void launch_ew_b(const JobArg<EwJob>& A, int nb, int mode, hipStream_t s);

// r_c = P^T r_f (velocity P2, pressure P1); also zero (xcu, xcp) if not NULL.
template <class T>
void launch_restrict(int Nc, int dom, const T* rfu, const T* rfp, T* rcu, T* rcp, T* xcu, T* xcp,
                     const int* done, hipStream_t s);
// (u, p) += P (zu, zp)
template <class T>
void launch_prolong_add(int Nc, int dom, const T* zu, const T* zp, T* u, T* p, const int* done,
                        hipStream_t s);
// z = Cinv * [r; 0] on the coarsest grid (FP64 inverse, any T in / out)
template <class T>
void launch_coarse_solve(int N0, int dom, int nc, const double* cinv, const T* ru, const T* rp, T* zu,
                         T* zp, const int* done, hipStream_t s);

// p <- p - (m . p) / sum(m); uses `partials` (>= mean_blocks(N) doubles x 2)
int mean_blocks(int N);
void launch_project_mean(int N, int dom, double* p, double* partials, const int* done, hipStream_t s);
// v <- v - m (sum_i v_i) / (sum_i m_i): the transpose of the mean projection
void launch_project_dual(int N, int dom, double* p, double* partials, hipStream_t s);

// Shat^-1 at setup
template <class T>
void launch_shat_inv(int N, int dom, double bh2, const T* adinv_host4, T* sinv, hipStream_t s);

// load vectors / masses
// mode 0: interior rows from interior values; 1: all rows from interior values;
// 2: interior rows from all values (load vectors of nodal data)
void launch_mass_u(int N, int dom, int mode, const double* u, double* y, hipStream_t s);
// y += scale * (M u) on the rows of `mode` (same modes as launch_mass_u)
void launch_mass_u_acc(int N, int dom, int mode, const double* u, double scale, double* y, hipStream_t s);
void launch_mass_p(int N, int dom, const double* g, double* gp, hipStream_t s);

// deterministic dots: which = 0 velocity interior lattice points, 1 pressure
int dot_blocks(int N, int which);
void launch_dot(int N, int dom, int which, const double* a, const double* b, double* partials,
                double* out, hipStream_t s);
// out[0] = sum of np partials (fixed order)
void launch_reduce(const double* partials, int np, double* out, hipStream_t s);
// Section 6 error measure pieces of (u, p) - (us, ps); scratch of
// enorm_scratch(N) doubles, out: 4 doubles (see the kernels)
int enorm_scratch(int N);
// out2 = (1^T gp, sum |gp|) over the domain's vertices (scratch as enorm_scratch)
void launch_psum(int N, int dom, const double* gp, double* red, double* out2, hipStream_t s);
// relative size of 1^T gp above which the pressure data count as incompatible
constexpr double SMG_COMPAT_TOL = 1e-9;
void launch_error_norm(int N, int dom, double bh2, const double* ahat4, const double* sinv, const double* u,
                       const double* p, const double* us, const double* ps, double* red, double* out,
                       hipStream_t s);

// Convergence bookkeeping of the solve loop (device-side).
struct SolveState {
  int done;        // 0 running, 1 converged, 2 diverged, 3 non-finite, 4 maxit
  int iters;
  int maxit;
  int pad;
  double fnorm2;   // ||F||^2
  double tol2;     // rtol^2
  double relres;   // last relative residual
  unsigned arrive; // workgroups of k_project_check that have finished (reset by the last)
  unsigned pad2;
};
// reduce `np` partials to ||r||^2; record the iterate: iters++, history, done flags.
void launch_check(const double* partials, int np, SolveState* st, double* hist, hipStream_t s);
// set the initial state: ||F||^2 = fdots[0] + fdots[1], ||F - calA x0||^2 from
// np residual partials; done = 1 if x0 already meets the tolerance.
void launch_init_state(const double* rpartials, int np, const double* fdots, SolveState* st,
                       hipStream_t s);

// elementwise helpers
void launch_fill(double* x, int64_t n, double v, hipStream_t s);
void launch_fill_f32(float* x, int64_t n, float v, hipStream_t s);
// x += (double) d ; both with n entries
void launch_axpy_f32(double* x, const float* d, int64_t n, const int* done, hipStream_t s);

}  // namespace smg
