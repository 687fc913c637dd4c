// CPU check program for the host-only runtime (paper_1502_04070_amd/csrc/smg_host.cpp).
// Built by tests/test_host_runtime_cpu.py with the address and undefined-behaviour
// sanitizers; any sanitizer report ends it with a non-zero status.
//
//   host_check selftest
//       parameter checks, launch start offsets and block maps, and the host
//       operator (symmetry of calA, zero rows outside the unknowns); prints
//       "selftest ok" or the first failure and exits 1.
//   host_check coarse N0 BETA DOMAIN OUT
//       writes the bordered coarsest-grid matrix (row-major) and its inverse
//       (column-major) in the compact order of smg_host.h to OUT:
//       int32 nc, int32 status, nc*nc doubles (matrix), nc*nc doubles
//       (inverse; zeros if the status is not 0).
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <string>
#include <vector>

#include "smg_host.h"

using namespace smg;

static int failures = 0;
#define CHECK(cond)                                                        \
  do {                                                                     \
    if (!(cond)) {                                                         \
      std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
      ++failures;                                                          \
    }                                                                      \
  } while (0)

static smg_params defaults() {
  smg_params p{};
  p.smoother = SMG_SMOOTHER_NE;
  p.tau = 0.35;
  p.sigma = 0.8;
  p.nu_pre = p.nu_post = 2;
  p.gamma = 1;
  p.n0 = 2;
  p.domain = SMG_DOMAIN_SQUARE;
  return p;
}

static void selftest_params() {
  int L = -1;
  smg_params p = defaults();
  CHECK(host::check_params(128, 1.0, p, &L) == SMG_OK && L == 6);
  CHECK(host::check_params(2, 0.0, p, &L) == SMG_OK && L == 0);
  CHECK(host::check_params(96, 1.0, p, &L) == SMG_EINVAL);        // 96 = 3 * 2^5, n0 = 2
  p.n0 = 3;
  CHECK(host::check_params(96, 1.0, p, &L) == SMG_OK && L == 5);
  CHECK(host::check_params(2, 1.0, p, &L) == SMG_EINVAL);         // below n0
  p.domain = SMG_DOMAIN_LSHAPE;
  CHECK(host::check_params(96, 1.0, p, &L) == SMG_EINVAL);        // odd n0
  p.domain = SMG_DOMAIN_UNIONJACK;
  CHECK(host::check_params(96, 1.0, p, &L) == SMG_EINVAL);
  p = defaults();
  CHECK(host::check_params(16384, 1.0, p, &L) == SMG_EINVAL);     // too large
  CHECK(host::check_params(16, -1.0, p, &L) == SMG_EINVAL);
  CHECK(host::check_params(16, NAN, p, &L) == SMG_EINVAL);
  CHECK(host::check_params(16, INFINITY, p, &L) == SMG_EINVAL);
  smg_params q = defaults();
  q.tau = 0.0;
  CHECK(host::check_params(16, 1.0, q, &L) == SMG_EINVAL);
  q = defaults();
  q.sigma = INFINITY;
  CHECK(host::check_params(16, 1.0, q, &L) == SMG_EINVAL);
  q = defaults();
  q.gamma = 3;
  CHECK(host::check_params(16, 1.0, q, &L) == SMG_EINVAL);
  q = defaults();
  q.nu_pre = -1;
  CHECK(host::check_params(16, 1.0, q, &L) == SMG_EINVAL);
  q = defaults();
  q.tile_x = 12;
  CHECK(host::check_params(16, 1.0, q, &L) == SMG_EINVAL);
  q = defaults();
  q.smoother = 7;
  CHECK(host::check_params(16, 1.0, q, &L) == SMG_EINVAL);
  q = defaults();
  q.domain = 9;
  CHECK(host::check_params(16, 1.0, q, &L) == SMG_EINVAL);
  CHECK(host::last_error()[0] != '\0');
}

static void selftest_maps() {
  std::vector<int> tiles = {3, 1, 4, 0, 2};
  int start[6];
  host::pack_starts(tiles, start);
  const int want[6] = {0, 3, 4, 8, 8, 10};
  for (int k = 0; k < 6; ++k) CHECK(start[k] == want[k]);
  std::vector<int> map = host::block_map(tiles);
  CHECK(map.size() == 10);
  int b = 0;
  for (size_t j = 0; j < tiles.size(); ++j)
    for (int t = 0; t < tiles[j]; ++t, ++b) {
      CHECK(map[b] >> BMAP_SHIFT == (int)j);
      CHECK((map[b] & ((1 << BMAP_SHIFT) - 1)) == t);
    }
  // a job index beyond the field of the map is refused
  std::vector<int> many((1 << (31 - BMAP_SHIFT)) + 1, 1);
  CHECK(host::block_map(many).empty());
  std::vector<int> wide = {(1 << BMAP_SHIFT) + 1, 1};   // tile index 2^20 does not fit
  CHECK(host::block_map(wide).empty());
}

// calA is symmetric: v . (calA w) = w . (calA v) on the unknowns, and the
// host operator writes zero at every entry that is not an unknown
static void selftest_apply() {
  std::mt19937_64 rng(7);
  std::normal_distribution<double> nd;
  for (int dom : {SMG_DOM_SQUARE, SMG_DOM_LSHAPE, SMG_DOM_UNIONJACK})
    for (int N : {2, 4, 8})
      for (double beta : {0.0, 3.0, 1e6}) {
        LevelCoef<double> c;
        LevelCoef<float> c32;
        host::make_coef(N, dom, beta, c, c32);
        const int M = 2 * N + 1, NP = N + 1;
        std::vector<double> u1(2 * M * M), p1(NP * NP), u2(2 * M * M), p2(NP * NP);
        for (double& v : u1) v = nd(rng);
        for (double& v : p1) v = nd(rng);
        for (double& v : u2) v = nd(rng);
        for (double& v : p2) v = nd(rng);
        std::vector<double> yu1(2 * M * M, 7.0), yp1(NP * NP, 7.0), yu2(2 * M * M, 7.0), yp2(NP * NP, 7.0);
        host::apply(N, c, u1.data(), p1.data(), yu1.data(), yp1.data());
        host::apply(N, c, u2.data(), p2.data(), yu2.data(), yp2.data());
        double s12 = 0, s21 = 0, scale = 0;
        for (int comp = 0; comp < 2; ++comp)
          for (int bb = 0; bb < M; ++bb)
            for (int a = 0; a < M; ++a) {
              const size_t g = (size_t)comp * M * M + (size_t)bb * M + a;
              if (!dom_u(N, dom, a, bb)) {
                CHECK(yu1[g] == 0.0);
                continue;
              }
              s12 += u1[g] * yu2[g];
              s21 += u2[g] * yu1[g];
              scale += std::fabs(u1[g] * yu2[g]);
            }
        for (int j = 0; j < NP; ++j)
          for (int i = 0; i < NP; ++i) {
            const size_t g = (size_t)j * NP + i;
            if (!dom_p(N, dom, i, j)) {
              CHECK(yp1[g] == 0.0);
              continue;
            }
            s12 += p1[g] * yp2[g];
            s21 += p2[g] * yp1[g];
            scale += std::fabs(p1[g] * yp2[g]);
          }
        CHECK(std::fabs(s12 - s21) <= 1e-12 * scale);
      }
}

int main(int argc, char** argv) {
  if (argc >= 2 && std::string(argv[1]) == "selftest") {
    selftest_params();
    selftest_maps();
    selftest_apply();
    if (failures) return 1;
    std::printf("selftest ok\n");
    return 0;
  }
  if (argc == 6 && std::string(argv[1]) == "coarse") {
    const int n0 = std::atoi(argv[2]);
    const double beta = std::atof(argv[3]);
    const int dom = std::atoi(argv[4]);
    LevelCoef<double> c;
    LevelCoef<float> c32;
    host::make_coef(n0, dom, beta, c, c32);
    std::vector<double> a, inv;
    host::bordered_matrix(n0, c, a);
    const int status = host::coarse_inverse(n0, c, inv);
    const int32_t nc = host::coarse_size(n0);
    if (inv.empty()) inv.assign((size_t)nc * nc, 0.0);
    FILE* f = std::fopen(argv[5], "wb");
    if (!f) return 2;
    const int32_t st = status;
    bool ok = std::fwrite(&nc, sizeof nc, 1, f) == 1 && std::fwrite(&st, sizeof st, 1, f) == 1 &&
              std::fwrite(a.data(), sizeof(double), a.size(), f) == a.size() &&
              std::fwrite(inv.data(), sizeof(double), inv.size(), f) == inv.size();
    ok = (std::fclose(f) == 0) && ok;
    return ok ? 0 : 2;
  }
  std::fprintf(stderr, "usage: host_check selftest | coarse N0 BETA DOMAIN OUT\n");
  return 2;
}
