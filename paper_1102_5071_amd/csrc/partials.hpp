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

// The same sum for lane `lane` of `THREADS` lanes when the count has no useful
// bound: chunks of PER values per lane, each chunk's loads issued together
// (one memory round trip per chunk instead of per value), in the same order.
template <int THREADS, int PER>
__device__ __forceinline__ double thread_partials_chunked(const double* __restrict__ part, int np,
                                                          int lane) {
  double s = 0.0;
  if (np <= 0) return s;
  for (int c = 0; c < np; c += PER * THREADS) {
    double v[PER];
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const int i = c + lane + j * THREADS;
      v[j] = part[i < np ? i : np - 1];
    }
#pragma unroll
    for (int j = 0; j < PER; ++j)
      if (c + lane + j * THREADS < np) s += v[j];
  }
  return s;
}

}  // namespace cfet
