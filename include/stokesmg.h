/*
 * stokesmg — coupled multigrid for the discretized generalized Stokes problem
 * on MI355X (gfx950), C ABI.
 *
 * Problem (paper, Section 1): -Lap u + beta u + grad p = f, div u = g in the
 * unit square, u = 0 on the boundary, int p = int g = 0, discretized with
 * Taylor-Hood P2-P1 elements (Section 2) on a uniformly refined grid of
 * N x N squares, each cut by the diagonal from its lower-left to its
 * upper-right corner.  The discrete system (matrix form, Section 2) is
 *
 *        [ A  B^T ] [u]   [f]      A = K + beta M  (both velocity components)
 *        [ B   0  ] [p] = [g],     B_ij = (div psi_j, phi_i)
 *
 * and is solved by the coupled multigrid iterate of Section 3 with the
 * normal-equation or Uzawa-type smoother of Section 4, preconditioned by
 * L = diag(Ahat, Shat), Ahat = diag A, Shat = diag(B Ahat^-1 B^T) (Section 6).
 *
 * SIGN CONVENTION.  Matrices follow the variational form of Section 2, whose
 * coupling term is +(p, div v).  Integrating by parts, the returned pressure
 * p is therefore the NEGATIVE of the p of the strong form as printed in
 * Section 1 (the two forms of the paper differ in this sign).
 *
 * DATA LAYOUT.  All vectors are caller-owned DEVICE pointers on the device
 * that was current at smg_setup, in the lattice layout of their level
 * (N_l = n0 * 2^l cells per side, M_l = 2 N_l + 1):
 *   velocity  double u[2][M_l][M_l]   component, y index b, x index a; P2 node
 *                                     (a, b) sits at (a/(2N_l), b/(2N_l)).
 *                                     Even/even = vertices, odd entries = edge
 *                                     midpoints.  Entries on the boundary are
 *                                     ignored on input and written 0 on output.
 *   pressure  double p[N_l+1][N_l+1] y index j, x index i; vertex (i/N_l, j/N_l).
 * Load vectors (right-hand sides) use the same layout: fu holds (f, psi) for
 * each interior P2 node, gp holds (g, phi) for each P1 node.  The library
 * never frees or retains caller pointers.  Outputs must not alias inputs
 * unless an entry point says so.
 *
 * STREAMS AND THREADS.  Every entry point enqueues on the given stream and
 * returns without waiting, except these, which wait for their work (and the
 * stream) before they return: smg_setup, smg_destroy, smg_solve,
 * smg_solve_mixed, smg_solve_error, smg_error_norm, smg_implicit_step,
 * smg_implicit_step_mixed, smg_batch_setup, smg_batch_destroy,
 * smg_batch_solve, smg_batch_solve_mixed, smg_batch_implicit_step,
 * smg_batch_implicit_step_mixed, smg_time_kernel, smg_batch_time_kernel and
 * smg_tune.  A handle owns scratch buffers: calls on one handle must not
 * overlap in time (use one stream per handle, or one handle per concurrent
 * stream).
 *
 * ERRORS.  Every function returns an int status.  0 = SMG_OK.  Negative values
 * are hard errors and leave outputs unspecified; positive values are soft
 * results with valid outputs.  smg_last_error() gives a thread-local message.
 */
#ifndef STOKESMG_H
#define STOKESMG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct smg_hier* smg_t;
typedef void* smg_stream_t; /* a hipStream_t; NULL = the default stream */

enum {
  SMG_OK = 0,
  SMG_EINVAL = -1,      /* bad argument: N not n0 * 2^L, beta < 0, NULL, bad level */
  SMG_EHIP = -2,        /* a HIP runtime call failed */
  SMG_ENOMEM = -3,      /* device allocation failed */
  SMG_ESINGULAR = -4,   /* coarsest-grid matrix numerically singular */
  SMG_NOCONV = 1,       /* maxit reached; outputs hold the last iterate */
  SMG_DIVERGED = 2,     /* relative residual above 1e6; last iterate returned */
  SMG_ENONFINITE = 3,   /* NaN or Inf in the residual; last iterate returned */
  SMG_EINCOMPAT = 4     /* no convergence and the pressure data are not
                           compatible: |1^T g_p| > 1e-9 sum |g_p| (the system
                           needs int g = 0, see smg_project_mean); last
                           iterate returned                                   */
};

enum { SMG_SMOOTHER_NE = 0, SMG_SMOOTHER_UZAWA = 1 };

/* Solver parameters (Sections 3, 4 and 6). */
typedef struct {
  int smoother;   /* SMG_SMOOTHER_NE (normal equation) or SMG_SMOOTHER_UZAWA   */
  double tau;     /* damping: 0.35 (normal equation), 0.8 (Uzawa)               */
  double sigma;   /* Uzawa pressure damping: 0.8                                */
  int nu_pre;     /* smoothing steps before the coarse-grid correction          */
  int nu_post;    /* smoothing steps after it                                   */
  int gamma;      /* 1 = V-cycle, 2 = W-cycle                                    */
  int n0;         /* cells per side of the coarsest grid (>= 2); solved exactly */
  int unfused;    /* 0 (default): fused kernels (one or two smoothing steps per
                     launch, defect + restriction in one launch, the coarsest
                     levels in one single-workgroup launch);
                     1: one launch per operator application (reference path) */
  /* Launch schedule of the fused path.  It changes no arithmetic result
   * beyond rounding order; smg_tune searches it.  0 selects the default.    */
  int fuse_depth;   /* normal-equation steps per launch on levels with 8 x 8
                       tiles: 1 or 2 (default 2)                               */
  int coarse_max_n; /* largest grid (squares per side) of the single-workgroup
                       coarse kernel (default 8; the coarsest level always)    */
  int tile_x;       /* squares per tile row of the normal-equation kernels: 8
                       or 16 (default: 16 for N >= 128, else 8)                */
  int domain;       /* SMG_DOMAIN_SQUARE (default): the unit square;
                       SMG_DOMAIN_LSHAPE: the unit square without [1/2, 1]^2, a
                       non-convex domain (Section 1: the method applies, the
                       analysis does not); needs an even n0.  The layouts stay
                       those of the square: entries at points outside the
                       domain are never read, and every entry point writes zero
                       there or leaves them as they were.
                       SMG_DOMAIN_UNIONJACK: the unit square on the grid of the
                       experiments of Section 6 (the coarsest 2 x 2 grid with
                       the diagonals meeting at the centre, refined
                       uniformly); needs an even n0.                           */
} smg_params;

enum { SMG_DOMAIN_SQUARE = 0, SMG_DOMAIN_LSHAPE = 1, SMG_DOMAIN_UNIONJACK = 2 };

/* Defaults: normal equation, tau = 0.35, sigma = 0.8, V(2,2), n0 = 2, fused,
 * default launch schedule. */
int smg_default_params(smg_params* prm);

/* Thread-local description of the last error (never NULL). */
const char* smg_last_error(void);

/*
 * Build the hierarchy for N cells per side (N = n0 * 2^L, L >= 0) and
 * beta >= 0 on the current device: per-level stencil coefficients, the
 * Shat^-1 arrays (Section 6, preconditioner), work vectors, and the inverse of
 * the coarsest-grid saddle matrix bordered by the mean-zero constraint
 * m^T p = 0, m_i = int phi_i (Section 3: level 0 is solved exactly).
 * With the fused path and coarse levels (those the single-workgroup kernel
 * handles, N <= coarse_max_n) below the finest, whose finest has at most 1024
 * lattice entries (N <= 8 with n0 = 2), it also forms the dense coarse map:
 * the coarse part of an iterate entered from a zero iterate is a linear map
 * of the restricted defect, and its matrix (FP64 and FP32, formed by that
 * kernel applied to unit vectors) replaces the level-by-level computation in
 * the iterates of solves with rtol = 0 or rtol >= 1e-11 (its rounding leaves
 * a relative residual floor of about 1e-12; tighter tolerances keep the
 * kernel).  Synchronous.  Errors: SMG_EINVAL, SMG_ENOMEM, SMG_ESINGULAR,
 * SMG_EHIP.
 */
int smg_setup(int N, double beta, const smg_params* prm, smg_t* out);
/* Frees the hierarchy and everything it owns; NULL is accepted (no-op). */
int smg_destroy(smg_t h);

/* Levels are numbered 0 (coarsest, n0 cells) .. L (finest, N cells). */
int smg_num_levels(smg_t h);
int smg_level_size(smg_t h, int level, int* N, int64_t* n_velocity, int64_t* n_pressure);

/*
 * Load vectors of P2 / P1 interpolants (Section 2, right-hand side):
 *   fu = (f, psi_j) at interior P2 nodes, both components, from nodal values
 *        f_nodal[2][M][M] given at ALL lattice points (boundary included);
 *   gp = (g, phi_i) at all P1 nodes, from nodal g_nodal[N+1][N+1].
 * Either output may be NULL to skip it.
 */
int smg_load(smg_t h, int level, const double* f_nodal, const double* g_nodal,
             double* fu, double* gp, smg_stream_t s);

/*
 * Velocity mass: y = M u (both components, M the P2 mass matrix).  If
 * all_nodes = 0 the rows are the interior nodes (boundary rows written 0) and
 * u is read at interior nodes only; if all_nodes = 1 the rows are all
 * lattice points (the transpose of the load map of smg_load: dL/df_nodal from
 * dL/dfu).
 */
int smg_mass(smg_t h, int level, int all_nodes, const double* u, double* y, smg_stream_t s);

/* Pressure mass: gp = M_P g (P1 mass matrix, all nodes). */
int smg_pressure_mass(smg_t h, int level, const double* g, double* gp, smg_stream_t s);

/* y = calA x: yu = A u + B^T p, yp = B u (matrix form, Section 2). */
int smg_apply(smg_t h, int level, const double* u, const double* p,
              double* yu, double* yp, smg_stream_t s);

/*
 * Residual r = F - calA x (Section 3, defect).  If norm2 is not NULL it
 * receives (device pointer, one double) the squared Euclidean norm over the
 * interior velocity and all pressure entries, reduced in a fixed order.
 */
int smg_residual(smg_t h, int level, const double* fu, const double* gp,
                 const double* u, const double* p, double* ru, double* rp,
                 double* norm2, smg_stream_t s);

/* nsteps smoothing steps of the configured smoother (Section 4), in place on (u, p). */
int smg_smooth(smg_t h, int level, int nsteps, const double* fu, const double* gp,
               double* u, double* p, smg_stream_t s);

/* Restriction I_k^{k-1} = (I_{k-1}^k)^T (Section 3) from level fine_level to
 * fine_level - 1.  Coarse outputs use the coarse layout. */
int smg_restrict(smg_t h, int fine_level, const double* ru, const double* rp,
                 double* rcu, double* rcp, smg_stream_t s);

/* Prolongation and add: (u, p) += I_{k-1}^k (zu, zp), the canonical embedding
 * of the coarse P2 / P1 functions (Section 3). */
int smg_prolong_add(smg_t h, int fine_level, const double* zcu, const double* zcp,
                    double* u, double* p, smg_stream_t s);

/* Exact solve on level 0 (Section 3: the coarsest level of the iterate is
 * solved exactly).  The saddle matrix of level 0 is singular on constant
 * pressures (B^T 1 = 0), so it is bordered by the constraint m^T p = 0,
 * m_i = int phi_i (Section 1: int p = 0) and a multiplier; its inverse is
 * formed in FP64 at smg_setup.  z = (zu, zp) receives the solution with a
 * mean-free pressure; r must be compatible (1^T rp = 0) for z to solve the
 * unbordered system.  Level-0 layouts; outputs must not alias inputs. */
int smg_coarse_solve(smg_t h, const double* ru, const double* rp, double* zu, double* zp,
                     smg_stream_t s);

/* p <- p - (sum_i m_i p_i) / (sum_i m_i), m_i = int phi_i: the mean-zero
 * representative of P_k (Section 1 fixes int p = 0). */
int smg_project_mean(smg_t h, int level, double* p, smg_stream_t s);

/* v <- v - m (sum_i v_i) / (sum_i m_i): the transpose of smg_project_mean
 * (maps any pressure cotangent to a compatible adjoint right-hand side). */
int smg_project_dual(smg_t h, int level, double* v, smg_stream_t s);

/* One iterate of Section 3 on the finest level (nu_pre smoothing steps,
 * coarse-grid correction by gamma recursive iterates, nu_post steps),
 * followed by the mean projection; in place on (u, p). */
int smg_cycle(smg_t h, const double* fu, const double* gp, double* u, double* p,
              smg_stream_t s);

/*
 * Error measure of the experiments (Section 6) on the finest level:
 *   *out = ||e||_L = (sum Ahat_k e_u,k^2 + sum Shat_q e_p,q^2)^(1/2),
 * e = (u, p) - (us, ps), its pressure part made mean-free (int e_p = 0)
 * first; Ahat = diag A, Shat = diag(B Ahat^-1 B^T).  Device vectors in, HOST
 * double out; synchronizes the stream.  Errors: SMG_EINVAL, SMG_EHIP.
 */
int smg_error_norm(smg_t h, const double* u, const double* p, const double* us, const double* ps,
                   double* out, smg_stream_t s);

/*
 * The measurement protocol of Section 6: starting from the (u, p) given,
 * repeat iterates on F = (fu, gp) (normally calA (us, ps), see smg_apply)
 * until ||x - x*||_L <= eps ||x0 - x*||_L, with x* = (us, ps).  iters (HOST)
 * receives the number of iterates and rate (HOST) the mean reduction factor
 * (||e_n|| / ||e_0||)^(1/n); either may be NULL.  One synchronization per
 * iterate.  Returns SMG_OK, SMG_NOCONV (maxit reached), SMG_DIVERGED (the
 * error grew by 1e6) or SMG_ENONFINITE (soft), or a hard error.
 */
int smg_solve_error(smg_t h, const double* fu, const double* gp, const double* us, const double* ps,
                    double eps, int maxit, double* u, double* p, int* iters, double* rate,
                    smg_stream_t s);

/*
 * Solve calA x = F on the finest level by repeated iterates of the coupled
 * multigrid method (Section 3, smoothers of Section 4, L of Section 6), each
 * followed by the mean projection (Section 1: int p = 0), until
 * ||F - calA x|| <= rtol ||F|| (2-norm over interior velocity and all
 * pressure entries; the paper's own experiments stop on the error instead,
 * see smg_solve_error).
 * (u, p) are the initial guess on entry and the solution on return (mean-free
 * pressure).  iters, relres and history (maxit doubles, relative residual
 * after each iterate) may be NULL; they are HOST pointers.  Synchronous.
 * rtol = 0 runs exactly maxit iterates (ending with SMG_NOCONV unless the
 * residual is exactly zero); the host then checks the state only at the end.
 * Returns SMG_OK, SMG_NOCONV, SMG_DIVERGED, SMG_ENONFINITE or SMG_EINCOMPAT (soft) or a
 * hard error.
 */
int smg_solve(smg_t h, const double* fu, const double* gp, double rtol, int maxit,
              double* u, double* p, int* iters, double* relres, double* history,
              smg_stream_t s);

/*
 * Same as smg_solve, but each iterate is one FP32 multigrid cycle (the iterate
 * of Section 3 in single precision at every level, an addition beside the
 * paper's FP64 method) applied to the correction equation calA d = r, inside
 * FP64 iterative refinement:
 *   r = F - calA x (FP64); d = cycle_fp32(r) from d = 0 with the FP64 coarse
 *   solve; x += d (FP64); pressure mean removed (FP64).
 * iters counts outer refinement steps (= FP32 cycles).  Synchronous.
 */
int smg_solve_mixed(smg_t h, const double* fu, const double* gp, double rtol, int maxit,
                    double* u, double* p, int* iters, double* relres, double* history,
                    smg_stream_t s);

/*
 * Smoother damping per level (Section 6 remarks that the rates improve
 * slightly when tau and sigma depend on the level and on beta).  Sets tau and
 * sigma of `level` (-1: every level) of h; they start at smg_params' tau and
 * sigma.  The coarsest level (solved exactly) ignores them.  Captured
 * iterates of h are dropped and captured again by the next solve; a batch
 * that holds h (smg_batch_handle) plans and captures its iterates again at
 * its next solve.  A change on a level of the dense coarse map forms the map
 * again (synchronous).  Errors: SMG_EINVAL (values not finite and > 0, bad
 * level), SMG_EHIP.
 */
int smg_set_damping(smg_t h, int level, double tau, double sigma);
int smg_get_damping(smg_t h, int level, double* tau, double* sigma);

/*
 * One implicit (backward) Euler step of the time-dependent Stokes problem,
 * the source of the generalized problem (Section 1: beta grows like 1/dt).
 * h must have been set up with beta = 1/dt.  With u = u^n on input (boundary
 * entries ignored) this solves
 *     calA(beta) x = (M_full f + beta M u^n, M_P g)
 * for x = (u^{n+1}, p^{n+1}) like smg_solve, from the initial guess
 * (u^n, p), and writes the result to u and p.  f_nodal: nodal values at all
 * P2 lattice points, layout of u (NULL: f = 0); g_nodal: P1 nodal values with
 * int g = 0 (NULL: g = 0).  Status codes as smg_solve.  Synchronous.
 */
int smg_implicit_step(smg_t h, const double* f_nodal, const double* g_nodal, double rtol, int maxit,
                      double* u, double* p, int* iters, double* relres, smg_stream_t s);
/* smg_implicit_step solved as smg_solve_mixed: FP32 cycles inside FP64
 * iterative refinement (same arguments and status codes). */
int smg_implicit_step_mixed(smg_t h, const double* f_nodal, const double* g_nodal, double rtol, int maxit,
                            double* u, double* p, int* iters, double* relres, smg_stream_t s);

/*
 * Single-precision cycle (exposed for testing the FP32 kernels): one iterate
 * as in smg_cycle on float vectors of the same layout, coarsest grid solved
 * in FP64.  In place on (u, p).
 */
int smg_cycle_f32(smg_t h, const float* fu, const float* gp, float* u, float* p,
                  smg_stream_t s);

/*
 * Deterministic dot products on a level (device result in out[0]):
 *   which = 0: sum over both velocity components at interior lattice points,
 *   which = 1: sum over all pressure nodes (of the domain: on the L-shaped
 *   domain points outside it are skipped in both sums).
 */
int smg_dot(smg_t h, int level, int which, const double* a, const double* b, double* out,
            smg_stream_t s);

/*
 * Batched solves (many independent instances in one set of launches).  Each
 * instance runs the iterate of Section 3 on its own problem; batching changes
 * which launch computes it, not what is computed.
 *
 * A batch holds n hierarchies built as by smg_setup(N[k], beta[k], prm): the
 * sizes may differ (each N[k] = n0 * 2^L_k with the common n0), beta is per
 * instance, the solver parameters are shared (fused path only).  Each iterate
 * of every instance is computed exactly as by the single-instance solver;
 * one launch serves every instance taking part in a stage (instances are
 * aligned by depth below their own finest level), and the whole iterate of
 * the batch is replayed from captured HIP graphs (one of one iterate, one of
 * four, launched so that a chunk runs exactly its iterates).  Converged
 * instances are skipped by their own convergence flag.  Several right-hand sides of one
 * problem are several instances with the same N and beta.
 */
typedef struct smg_batch_s* smg_batch_t;

int smg_batch_setup(int n, const int* N, const double* beta, const smg_params* prm,
                    smg_batch_t* out);
/* Frees the batch and its hierarchies; NULL is accepted (no-op). */
int smg_batch_destroy(smg_batch_t b);
int smg_batch_size(smg_batch_t b);
/* The hierarchy of instance k (for smg_load, smg_apply, ... on its levels);
 * owned by the batch.  NULL on a bad index. */
smg_t smg_batch_handle(smg_batch_t b, int k);

/*
 * Solve every instance k to ||F_k - calA_k x_k|| <= rtol ||F_k|| by the
 * iterates of Section 3, as smg_solve does for one instance.  fu, gp, u,
 * p are HOST arrays of n DEVICE pointers (layouts as for smg_solve of instance
 * k; u[k], p[k] hold the initial guess and receive the solution).  iters,
 * relres, status (host arrays of n, may be NULL) receive the per-instance
 * iterate count, final relative residual and status.  Returns SMG_OK if all
 * converged, else the largest soft status; synchronous.
 */
int smg_batch_solve(smg_batch_t b, const double* const* fu, const double* const* gp, double rtol,
                    int maxit, double* const* u, double* const* p, int* iters, double* relres,
                    int* status, smg_stream_t s);
/* The same with FP32 cycles inside FP64 iterative refinement (see smg_solve_mixed). */
int smg_batch_solve_mixed(smg_batch_t b, const double* const* fu, const double* const* gp,
                          double rtol, int maxit, double* const* u, double* const* p, int* iters,
                          double* relres, int* status, smg_stream_t s);

/* smg_set_damping for instance `instance` (-1: all) of a batch; the
 * batch's captured iterates are rebuilt by its next solve. */
int smg_batch_set_damping(smg_batch_t b, int instance, int level, double tau, double sigma);

/* smg_implicit_step for every instance of a batch (instance k set up with
 * beta_k = 1/dt_k), solved together; f_nodal / g_nodal may be NULL (all
 * zero) or hold one pointer per instance (NULL entries: zero). */
int smg_batch_implicit_step(smg_batch_t b, const double* const* f_nodal, const double* const* g_nodal,
                            double rtol, int maxit, double* const* u, double* const* p, int* iters,
                            double* relres, int* status, smg_stream_t s);
/* smg_batch_implicit_step solved as smg_batch_solve_mixed (FP32 cycles inside
 * FP64 iterative refinement). */
int smg_batch_implicit_step_mixed(smg_batch_t b, const double* const* f_nodal, const double* const* g_nodal,
                                  double rtol, int maxit, double* const* u, double* const* p, int* iters,
                                  double* relres, int* status, smg_stream_t s);

/*
 * Batched kernel timing (profiling support): `reps` back-to-back launches of
 * the finest-level fused normal-equation step of all instances (which = 0),
 * on the instances' internal work vectors, timed with HIP events on s; mean
 * milliseconds per launch.  Synchronous.
 */
int smg_batch_time_kernel(smg_batch_t b, int which, int reps, double* avg_ms, smg_stream_t s);

/*
 * Kernel timing (profiling support): launches `reps` times, back to back on
 * stream s, one kernel of the finest level on the handle's internal work
 * vectors and returns the mean duration in milliseconds measured with HIP
 * events recorded on s.  which: 0 = normal-equation pass 1 (t = L^-1 (F -
 * calA x)), 1 = normal-equation pass 2 (x += tau L^-1 calA t), 2 = residual
 * (t = F - calA x), 3 = operator (t = calA x).  The work vectors' contents
 * are overwritten.  Synchronous.
 */
int smg_time_kernel(smg_t h, int which, int reps, double* avg_ms, smg_stream_t s);

/*
 * Launch-schedule autotuner (the iterate of Section 3 is the same for every
 * schedule; only its launches differ).  For the n instances (N[k], beta[k])
 * and the parameters `base` (NULL: defaults; must be fused), every candidate
 * schedule -- coarse_max_n in {n0, 4, 8, 16} (limits that select the same
 * levels once), tile_x in {0, 8, 16}, fuse_depth in {1, 2} where it matters
 * (normal equation, tile_x != 16) -- is set up as a batch (one instance when
 * n = 1), and `iters` iterates of f = 1, g = 0 are timed with HIP events on s
 * after three untimed ones, in two passes over all candidates (the faster
 * time of each counts).
 * `best` receives `base` with the fastest schedule and best_ms its time per
 * iterate in milliseconds.  If cap > 0 the first cap candidates tried and
 * their times go to tried / tried_ms; ntried (may be NULL) receives the
 * number of candidates timed.  Candidates that cannot be set up on this
 * device are skipped.  Allocates and frees device memory; synchronous.
 * Errors: SMG_EINVAL (bad sizes, iters outside 1..500, unfused base),
 * SMG_EHIP (no candidate could be timed).
 */
int smg_tune(int n, const int* N, const double* beta, const smg_params* base, int iters,
             smg_params* best, double* best_ms, smg_params* tried, double* tried_ms, int cap,
             int* ntried, smg_stream_t s);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the
 * residual of smg_residual on a grid of N x N squares (N in 2..4096; even N
 * on the L-shaped and union-jack domains) with coefficient beta, without a
 * hierarchy and without any allocation.  fu, gp, u, p, ru, rp: device
 * vectors in the lattice layout of that grid (as for smg_residual); norm2
 * (device, one double, or NULL) receives the squared norm, summed in a
 * fixed order.  The per-tile partial sums live in a fixed device array of
 * 2^17 doubles (1 MiB) that each GPU holds until the process ends; a grid
 * needing more partials than that is refused (SMG_EINVAL).  Every call
 * rewrites every partial it reads, so no clearing is needed; calls that
 * overlap in time on one device race on the array.  Stream-ordered.
 * Errors: SMG_EINVAL, SMG_EHIP.
 */
int smg_residual_noalloc(int N, double beta, int domain, const double* fu, const double* gp,
                         const double* u, const double* p, double* ru, double* rp, double* norm2,
                         smg_stream_t s);

#ifdef __cplusplus
}
#endif

#endif /* STOKESMG_H */
