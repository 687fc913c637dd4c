// Jobs of the fused kernels (see smg_fused.hip).
#pragma once
#include "smg_internal.h"

namespace smg {

// one fused normal-equation step: o = x (+ P z) + tau L^-1 A L^-1 (F - A (x (+ P z)))
template <class T>
struct NEJob {
  LevelCoef<T> L;
  const T* xu;
  const T* xp;        // input iterate (not read when it is known to be zero)
  const T* fu;
  const T* fp;        // right-hand side
  T* ou;
  T* op;              // output iterate; must not alias the input
  const T* zu;
  const T* zp;        // coarse correction (coarse layout), added to x first
  T tau;
  double* partial;    // per tile: ||F - A x||^2 over the owned rows, or NULL
  const int* done;
  double* acc_u;      // FP32 steps only: if set, the new iterate is added to
  double* acc_p;      // these FP64 vectors instead of being written to ou / op
  double* mean_partial;  // k_ne_res only: per tile (sum w_i p_i, sum w_i) of the new p
};
TileShape ne_tile_shape(int N);

// One Uzawa-type smoothing step (Section 4), all three half-steps in one
// launch on 16 x 8 tiles (square and L-shaped domains)
template <class T>
struct UZJob {
  LevelCoef<T> L;
  const T* xu;
  const T* xp;        // input iterate (not read when it is known to be zero)
  const T* fu;
  const T* fp;        // right-hand side
  T* ou;
  T* op;              // output iterate; must not alias the input
  T tau, sigma;
  const int* done;
};
int uz_tiles(int N);
template <class T>
void launch_uz(const UZJob<T>& J, bool zero_guess, hipStream_t s);
template <class T>
void launch_uz_b(const JobArg<UZJob<T>>& A, int nb, bool zero_guess, int dom, hipStream_t s);
// two normal-equation steps in one launch (8 x 8 tiles; levels with N < 128):
// the output is the iterate after both steps; the partial field is not used
template <class T>
void launch_ne2(const NEJob<T>& J, bool zero_guess, bool prolong, hipStream_t s);
template <class T>
void launch_ne2_b(const JobArg<NEJob<T>>& A, int nb, bool zero_guess, bool prolong, int dom,
                  hipStream_t s);
int ne_tiles(int N);
template <class T>
void launch_ne(const NEJob<T>& J, bool zero_guess, bool prolong, int tile_x, hipStream_t s);
// one NE step from a non-zero iterate on 16 x 8 tiles, then the residual of
// the result: per tile its ||F - A x_new||^2 (partial) and the pressure mean
// pieces of x_new (mean_partial), as the residual pass of the solve loop
// writes them; tiles as ne_tiles with 16 x 8 tiles
void launch_ne_res(const NEJob<double>& J, hipStream_t s);
inline int ne_res_tiles(int N) { return ((N + 16) / 16) * ((N + 8) / 8); }
// used only for launches of at most this many tiles (about one round of
// workgroups): there the separate residual pass is a launch's latency, while
// on larger grids the fused kernel's extra halo work costs more than the
// pass (64 x 4 batch: 624 us against 344 + 191 us)
constexpr int NE_RES_MAX_TILES = 1024;
void launch_ne_res_b(const JobArg<NEJob<double>>& A, int nb, int dom, hipStream_t s);

// fused defect and restriction: (cu, cp) = P^T (F - A x), L = fine level
template <class T>
struct RRJob {
  LevelCoef<T> L;
  const T* xu;
  const T* xp;
  const T* fu;
  const T* fp;
  T* cu;
  T* cp;
  const int* done;
};
template <class T>
void launch_resid_restrict(const RRJob<T>& J, hipStream_t s);

// From a zero iterate: two normal-equation steps and then the defect and its
// restriction, in one launch (the pre-smoothing of a coarse level with two
// steps, and the right-hand side of the next coarser level).  Tiles of 4 x 4
// coarse squares; the fine level N must be even.
template <class T>
struct NERRJob {
  LevelCoef<T> L;     // fine level
  const T* fu;
  const T* fp;        // right-hand side of the fine level
  T* ou;
  T* op;              // iterate after the two steps (fine level)
  T* cu;
  T* cp;              // P^T (F - A x): right-hand side of the coarse level
  T tau;
  const int* done;
};
int ne2rr_tiles(int Nc);
template <class T>
void launch_ne2rr(const NERRJob<T>& J, hipStream_t s);
template <class T>
void launch_ne2rr_b(const JobArg<NERRJob<T>>& A, int nb, int dom, hipStream_t s);

// the iterate on levels 0..Lc by one workgroup
constexpr int CC_MAX_LEVELS = 5;
enum { CC_NE = 1, CC_UZAWA = 2, CC_RESTRICT = 3, CC_PROLONG = 4, CC_COARSE = 5 };
inline int cc_op(int kind, int level, int zg) { return kind | (level << 8) | (zg << 16); }
constexpr int CC_MAX_OPS = 256;
// level 0's inverse is staged in LDS up to this order (the 27 unknowns of
// n0 = 2 fit); the static LDS of the kernel on top of its level storage
constexpr int CC_CINV_MAX = 32;
constexpr size_t CC_STATIC_LDS = CC_MAX_OPS * sizeof(int) + CC_CINV_MAX * CC_CINV_MAX * sizeof(double);

template <class T>
struct CoarseJob {
  LevelCoef<T> L[CC_MAX_LEVELS + 1];
  int n0, Lc, nc;
  int nops;
  const int* ops;        // device array of nops encoded operations
  const double* cinv;    // bordered inverse of level 0 (column-major, nc x nc)
  const T* fu;
  const T* fp;           // right-hand side of level Lc (global)
  T* xu;
  T* xp;                 // iterate of level Lc (global; read unless zero_guess)
  int zero_guess;
  T tau[CC_MAX_LEVELS + 1], sigma[CC_MAX_LEVELS + 1];   // smoother damping per level
  const int* done;
};
// The coarse part of an iterate from a zero iterate is a linear map of the
// restricted defect F of level Lc: x = K F.  K (row-major, n x n over the
// lattice entries of level Lc: velocity 2 M^2, then pressure) is formed once
// by the coarse-level kernel applied to unit vectors, and k_ccd applies it.
template <class T>
struct DenseJob {
  const T* K;
  int n, nu;              // lattice length of level Lc, its velocity part
  const T* fu;
  const T* fp;
  T* xu;
  T* xp;
  const int* done;
};
constexpr int KD_MAX = 1024;   // largest lattice length given a dense map
constexpr int KD_ROWS = 4;     // rows of K per workgroup (one wave per row)
inline int ccd_blocks(int n) { return (n + KD_ROWS - 1) / KD_ROWS; }
template <class T>
void launch_ccd(const DenseJob<T>& J, hipStream_t s);
template <class T>
void launch_ccd_b(const JobArg<DenseJob<T>>& A, int nb, hipStream_t s);
size_t coarse_cycle_lds(int n0, int Lc, size_t elem);
template <class T>
int launch_coarse_cycle(const CoarseJob<T>& J, hipStream_t s);
template <class T>
int coarse_cycle_allow_lds(size_t bytes);

// p -= mean from partials (sum w p, sum w) pairs of np tiles
void launch_project_partials(const double* mpart, int np, int N, int dom, double* p, const int* done,
                             hipStream_t s);
// the same, then the convergence test of the solve loop from the np residual
// partials (done by the last workgroup to finish)
void launch_project_check(const double* mpart, const double* rpart, int np, int N, int dom, double* p,
                          SolveState* st, double* hist, hipStream_t s);

// ---------------------------------------------------------------------------
// batched launches: many jobs (one per instance and level) in one grid.  A
// block map entry holds (job << 20) | tile; jobs live in device memory.
// ---------------------------------------------------------------------------

template <class T>
void launch_ne_b(const JobArg<NEJob<T>>& A, int nb, int tx, bool zg, bool pro, int dom,
                 hipStream_t s);
template <class T>
void launch_rr_b(const JobArg<RRJob<T>>& A, int nb, int dom, hipStream_t s);
template <class T>
void launch_cc_b(const CoarseJob<T>* jobs, int njobs, size_t lds, int dom, hipStream_t s);

// projection + convergence test per job (one job per instance)
struct PCJob {
  const double* mpart;
  const double* rpart;
  int np, N, dom;
  double* p;
  SolveState* st;
  double* hist;
};
__host__ __device__ int pc_blocks(int N);
void launch_pc_b(const JobArg<PCJob>& A, int nb, hipStream_t s);

}  // namespace smg
