// Staging of LDS windows for the grid kernels.
#pragma once
#include <hip/hip_runtime.h>

namespace smg {

// LDS windows staged with every global load of the workgroup in flight
// before the first wait.  A window of COUNT items is walked by NT threads in
// IT = ceil(COUNT / NT) rounds: fetch() reads a thread's items of all rounds
// into registers (unrolled, no wait between rounds), put() writes them to LDS
// afterwards.  A loop `for (e = tid; e < COUNT; e += NT) lds[e] = g[e]` waits
// for each round's loads before it issues the next round's, so a window of
// four rounds pays the memory latency four times.  ld(e, v) must set all V
// values of item e (zero outside the domain).
template <int COUNT, int NT, int V, class T>
struct Staged {
  static constexpr int IT = (COUNT + NT - 1) / NT;
  T v[IT][V];
  template <class LD>
  __device__ __forceinline__ void fetch(int tid, LD ld) {
#pragma unroll
    for (int k = 0; k < IT; ++k) {
      const int e = tid + k * NT;
      if (COUNT % NT == 0 || e < COUNT) ld(e, v[k]);
    }
  }
  template <class ST>
  __device__ __forceinline__ void put(int tid, ST st) const {
#pragma unroll
    for (int k = 0; k < IT; ++k) {
      const int e = tid + k * NT;
      if (COUNT % NT == 0 || e < COUNT) st(e, v[k]);
    }
  }
};

}  // namespace smg
