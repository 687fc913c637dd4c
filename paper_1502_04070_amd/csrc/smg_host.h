// Host-only part of the runtime: no device code and no HIP calls.  It is
// compiled by the host compiler, into the library and, on its own with the
// address and undefined-behaviour sanitizers, into a CPU check program.
//
//   * parameter checks of smg_setup;
//   * the per-level operator coefficients (Section 2 matrices as lattice
//     stencils, Section 6 diagonal);
//   * a host application of calA with the same stencils, which assembles the
//     coarsest-grid matrix column by column;
//   * that matrix bordered by the mean-zero constraint and its inverse
//     (Section 3: level 0 is solved exactly);
//   * the start offsets and block maps of batched launches.
#pragma once
#include <vector>

#include "smg_internal.h"
#include "stokesmg.h"

namespace smg {
namespace host {

// record a thread-local message (printf-style) and return `code`
int fail(int code, const char* fmt, ...);
const char* last_error();

// The parameter and size checks of smg_setup: SMG_OK and *L (levels above
// the coarsest) if N = n0 2^L with valid parameters, else SMG_EINVAL.
int check_params(int N, double beta, const smg_params& prm, int* L);

// coefficients of level N (h = 1/N) in FP64 and rounded to FP32; sinv is
// left unset (it lives on the device)
void make_coef(int N, int dom, double beta, LevelCoef<double>& c, LevelCoef<float>& c32);

// y = calA x on the host with the kernels' stencils (lattice layout of level N)
void apply(int N, const LevelCoef<double>& c, const double* u, const double* p, double* yu, double* yp);

// The unknowns of the coarsest grid in the compact order of the coarse-solve
// kernel: velocity component c at interior lattice point (1 + q % ni, 1 + q / ni)
// (ni = 2 N0 - 1) is unknown c ni^2 + q, pressure vertex (i, j) is
// 2 ni^2 + j (N0 + 1) + i, the multiplier of the constraint is the last.
int coarse_size(int N0);

// [[A, B^T, 0], [B, 0, m], [0, m^T, 0]] in that order (row-major, nc x nc),
// m_i = int phi_i; unknowns outside the domain are decoupled identity rows.
void bordered_matrix(int N0, const LevelCoef<double>& c, std::vector<double>& a_rowmajor);

// Its inverse (column-major) by symmetric equilibration and LU with partial
// pivoting.  SMG_ESINGULAR if a pivot falls below 1e-13 of the largest entry.
int coarse_inverse(int N0, const LevelCoef<double>& c, std::vector<double>& inv_colmajor);

// First workgroup of each job of a batched launch: start[k] = sum of
// tiles[0..k-1], start[n] = the launch's workgroups.  start has n + 1 entries.
void pack_starts(const std::vector<int>& tiles, int* start);
// Block map of a launch that reads its jobs from a table: entry b holds
// (job << BMAP_SHIFT) | tile for workgroup b.  Empty if a job index or a tile
// index does not fit its field.
std::vector<int> block_map(const std::vector<int>& tiles);

}  // namespace host
}  // namespace smg
