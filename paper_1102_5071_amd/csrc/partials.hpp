// Per-thread share of a block's re-sum of per-block partial sums written by
// an earlier kernel: thread t adds part[t], part[t + THREADS], ... in that
// order.  The loads of the first MAXNP values are issued together, with no
// branch between them (a wait after each load would cost one memory round
// trip per value): an index past the end loads the last value and the select
// after the loads drops it.  The values are then added in the same order, so
// the result is the number the plain strided loop gives.
#pragma once

#include <hip/hip_runtime.h>

namespace cfet {

template <int THREADS, int MAXNP = 2048>
__device__ __forceinline__ double thread_partials(const double* __restrict__ part, int np) {
  constexpr int PER = (MAXNP + THREADS - 1) / THREADS;
  if (np <= 0) return 0.0;
  double v[PER];
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int i = (int)threadIdx.x + j * THREADS;
    v[j] = part[i < np ? i : np - 1];
  }
  double s = 0.0;
#pragma unroll
  for (int j = 0; j < PER; ++j)
    if ((int)threadIdx.x + j * THREADS < np) s += v[j];
  for (int i = (int)threadIdx.x + PER * THREADS; i < np; i += THREADS) s += part[i];
  return s;
}

}  // namespace cfet
