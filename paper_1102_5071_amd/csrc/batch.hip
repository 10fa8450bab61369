// Batched CFET kernels: one launch per Lanczos phase over every instance of
// the batch (layout and grouping: batch_internal.h).
//
// Per exponential (paper Sec. 8.1, for each instance independently):
//   START     beta_0 = ||psi||, the instance is idle if psi = 0
//   for k = 0, 1, ...:
//     SPMM    y = H_w v_k on all rows, partial sums of Re<v_k, y>
//     ALPHA   alpha_k; at k = min(m, n) - 1 the basis is complete
//     AXPY    w = y - alpha_k v_k - beta_{k-1} v_{k-1} (stored unnormalised
//             as basis vector k + 1), partial sums of ||w||^2
//     BETA    beta_k; the basis is complete when the breakdown rule fires or,
//             with tol > 0, when dt beta_k |e_k^T exp(-i dt T) e_1| <= tol
//   COMBINE   psi = beta_0 sum_l c_l v_l, partial sums of ||psi||^2 (for the
//             next START)
// An instance whose basis is complete idles (its lanes skip) until COMBINE;
// a block whose instances are all idle returns at once.  All reductions are
// fixed-order: per-block tree sums, then one wavefront per instance adds the
// block partials in block order.
#include <hip/hip_runtime.h>

#include "batch_internal.h"
#include "partials.hpp"
#include "tridiag.hpp"

namespace cfet {

namespace {

struct RowMap {
  int g;        // group
  int64_t r0;   // first row of the block
  int64_t r1;   // one past the last row
  int j;        // instance within the group (lane % lpr)
  int sub;      // row offset of the lane within its wavefront's row set
  int rpw;      // rows per wavefront pass
  bool lane_ok; // j < B
};

__device__ __forceinline__ int find_group(const BGroup* G, int ng, int b) {
  int lo = 0, hi = ng - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (G[mid].block0 <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ int find_group_of_slot(const BGroup* G, int ng, int slot) {
  int lo = 0, hi = ng - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (G[mid].slot0 <= slot) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Blocks take the (group, row) space in launch order.  (Renumbering them so
// that each XCD sweeps one contiguous eighth measured slower here than the
// plain order, in which the XCDs work on neighbouring rows at the same time
// and share the lines they fetch through the memory-side cache.)
__device__ __forceinline__ int logical_block(int) { return blockIdx.x; }

__device__ __forceinline__ RowMap row_map(const BGroup& gr, int g, int lb) {
  RowMap m;
  m.g = g;
  const int local = lb - gr.block0;
  m.r0 = (int64_t)local * gr.rows_per_block;
  m.r1 = min(gr.n, m.r0 + gr.rows_per_block);
  const int lane = threadIdx.x & 63;
  m.j = lane & (gr.lpr - 1);
  m.rpw = 64 / gr.lpr;
  m.sub = (threadIdx.x >> 6) * m.rpw + lane / gr.lpr;
  m.lane_ok = m.j < gr.B;
  return m;
}

// Sum v over the lanes of this block that serve instance j (fixed order) and
// write it to the partial of (slot, block within the group): the partials of
// one instance are contiguous, so its reduction reads them coalesced.
template <int W>
__device__ void block_partial(double v, const BGroup& gr, double* red, const BLaunch& L,
                              int lb) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1)
    if (off >= gr.lpr) v += __shfl_xor(v, off, 64);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane < gr.lpr) red[w * 64 + lane] = v;
  __syncthreads();
  if (threadIdx.x < gr.B) {
    double t = 0.0;
    for (int i = 0; i < W; ++i) t += red[i * 64 + threadIdx.x];
    L.part[(int64_t)(gr.slot0 + threadIdx.x) * L.pstride + (lb - gr.block0)] = t;
  }
}

// true if every instance of the group has completed its basis
__device__ __forceinline__ bool group_idle(const BGroup& gr, const int* done) {
  const int lane = threadIdx.x & 63;
  const int d = (lane < gr.B) ? done[gr.slot0 + lane] : 1;
  return __ballot(d == 0) == 0ull;
}

// ---- START / COMBINE partial sums: ||V_0||^2 of every instance
template <int W>
__global__ __launch_bounds__(64 * W) void k_b_norm(BLaunch L) {
  __shared__ double red[W * 64];
  const int lb = logical_block(L.total_blocks);
  if (lb >= L.total_blocks) return;
  const int g = find_group(L.groups, L.ngroups, lb);
  const BGroup gr = L.groups[g];
  const RowMap M = row_map(gr, g, lb);
  double s = 0.0;
  if (M.lane_ok) {
    const double2* __restrict__ x = L.V + gr.voff;
    for (int64_t r = M.r0 + M.sub; r < M.r1; r += W * M.rpw) {
      const double2 v = x[r * gr.B + M.j];
      s += v.x * v.x + v.y * v.y;
    }
  }
  block_partial<W>(s, gr, red, L, lb);
}

// ---- y = H_w v_k (v_k = V_k * inv_k) and partials of Re<v_k, y>
template <int W>
__global__ __launch_bounds__(64 * W) void k_b_spmm(BLaunch L, int k) {
  __shared__ double red[W * 64];
  __shared__ double wl[kBatchMaxGroup][kBatchMaxK1];
  const int lb = logical_block(L.total_blocks);
  if (lb >= L.total_blocks) return;
  const int g = find_group(L.groups, L.ngroups, lb);
  const BGroup gr = L.groups[g];
  if (group_idle(gr, L.S.done)) return;
  const RowMap M = row_map(gr, g, lb);
  const BState* st = L.st;
  const int K1 = st->K1;
  const long long cur = st->cursor;
  for (int t = threadIdx.x; t < gr.B * K1; t += 64 * W) {
    const int jj = t / K1, tt = t % K1;
    wl[jj][tt] = st->wts[((int64_t)cur * st->nslots + gr.slot0 + jj) * K1 + tt];
  }
  __syncthreads();
  const int slot = gr.slot0 + M.j;
  const bool act = M.lane_ok && L.S.done[slot] == 0;
  double s = 0.0;
  if (act) {
    const double invk = L.S.inv[(int64_t)slot * kMaxM + k];
    const double2* __restrict__ x = L.V + (int64_t)k * L.ntot + gr.voff;
    double2* __restrict__ y = L.Y + gr.voff;
    const int B = gr.B;
    const int j = M.j;
    const double* __restrict__ wt = wl[j];
    for (int64_t r = M.r0 + M.sub; r < M.r1; r += W * M.rpw) {
      double ar = 0.0, ai = 0.0;
      int64_t e = gr.rowptr[r];
      const int64_t e1 = gr.rowptr[r + 1];
      // entries in fours: the column loads, then the gathers, then the products,
      // so each lane has several independent loads in flight
      for (; e + 4 <= e1; e += 4) {
        uint32_t ct[4];
        double2 v[4], xv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          ct[u] = gr.colt[e + u];
          v[u] = gr.val[e + u];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) xv[u] = x[(int64_t)(ct[u] & kColMask) * B + j];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const double w = wt[ct[u] >> kTermShift];
          ar += w * (v[u].x * xv[u].x - v[u].y * xv[u].y);
          ai += w * (v[u].x * xv[u].y + v[u].y * xv[u].x);
        }
      }
      for (; e < e1; ++e) {
        const uint32_t ct = gr.colt[e];
        const double2 v = gr.val[e];
        const double2 xv = x[(int64_t)(ct & kColMask) * B + j];
        const double w = wt[ct >> kTermShift];
        ar += w * (v.x * xv.x - v.y * xv.y);
        ai += w * (v.x * xv.y + v.y * xv.x);
      }
      const double2 xo = x[r * B + j];
      if (!gr.shared_h0) {
        typedef double dv2 __attribute__((ext_vector_type(2)));
        const dv2 d = __builtin_nontemporal_load(reinterpret_cast<const dv2*>(gr.diag) + r * B + j);
        double hr = d.x * xo.x - d.y * xo.y, hi = d.x * xo.y + d.y * xo.x;
        if (gr.orp) {
          const int64_t* rp = gr.orp + (int64_t)j * (gr.n + 1);
          for (int64_t e = rp[r]; e < rp[r + 1]; ++e) {
            const double2 v = gr.oval[e];
            const double2 xv = x[(int64_t)gr.ocol[e] * B + j];
            hr += v.x * xv.x - v.y * xv.y;
            hi += v.x * xv.y + v.y * xv.x;
          }
        }
        ar += wt[0] * hr;
        ai += wt[0] * hi;
      }
      const double2 yv = make_double2(ar * invk, ai * invk);
      typedef double dv2 __attribute__((ext_vector_type(2)));
      __builtin_nontemporal_store(dv2{yv.x, yv.y}, reinterpret_cast<dv2*>(y) + r * B + j);
      s += (xo.x * yv.x + xo.y * yv.y) * invk;
    }
  }
  block_partial<W>(s, gr, red, L, lb);
}

// ---- w = y - alpha_k v_k - beta_{k-1} v_{k-1}, stored as V_{k+1}; partials of ||w||^2
template <int W>
__global__ __launch_bounds__(64 * W) void k_b_axpy(BLaunch L, int k) {
  __shared__ double red[W * 64];
  const int lb = logical_block(L.total_blocks);
  if (lb >= L.total_blocks) return;
  const int g = find_group(L.groups, L.ngroups, lb);
  const BGroup gr = L.groups[g];
  if (group_idle(gr, L.S.done)) return;
  const RowMap M = row_map(gr, g, lb);
  const int slot = gr.slot0 + M.j;
  const bool act = M.lane_ok && L.S.done[slot] == 0;
  double s = 0.0;
  if (act) {
    const int64_t sb = (int64_t)slot * kMaxM;
    const double ca = L.S.alpha[sb + k] * L.S.inv[sb + k];
    const double cb = (k > 0) ? L.S.beta[sb + k - 1] * L.S.inv[sb + k - 1] : 0.0;
    const double2* __restrict__ vk = L.V + (int64_t)k * L.ntot + gr.voff;
    const double2* __restrict__ vm = L.V + (int64_t)(k > 0 ? k - 1 : 0) * L.ntot + gr.voff;
    const double2* __restrict__ y = L.Y + gr.voff;
    double2* __restrict__ w = L.V + (int64_t)(k + 1) * L.ntot + gr.voff;
    const int B = gr.B;
    typedef double dv2 __attribute__((ext_vector_type(2)));
    for (int64_t r = M.r0 + M.sub; r < M.r1; r += W * M.rpw) {
      const int64_t i = r * B + M.j;
      const dv2 a = __builtin_nontemporal_load(reinterpret_cast<const dv2*>(vk) + i);
      const dv2 yv = __builtin_nontemporal_load(reinterpret_cast<const dv2*>(y) + i);
      double wr = yv.x - ca * a.x, wi = yv.y - ca * a.y;
      if (k > 0) {
        const dv2 b = __builtin_nontemporal_load(reinterpret_cast<const dv2*>(vm) + i);
        wr -= cb * b.x;
        wi -= cb * b.y;
      }
      __builtin_nontemporal_store(dv2{wr, wi}, reinterpret_cast<dv2*>(w) + i);
      s += wr * wr + wi * wi;
    }
  }
  block_partial<W>(s, gr, red, L, lb);
}

// ---- psi = sum_l coef_l V_l; partials of ||psi||^2
template <int W>
__global__ __launch_bounds__(64 * W) void k_b_combine(BLaunch L) {
  __shared__ double red[W * 64];
  const int lb = logical_block(L.total_blocks);
  if (lb >= L.total_blocks) return;
  const int g = find_group(L.groups, L.ngroups, lb);
  const BGroup gr = L.groups[g];
  const RowMap M = row_map(gr, g, lb);
  double s = 0.0;
  if (M.lane_ok) {
    const int slot = gr.slot0 + M.j;
    const int meff = L.S.m_eff[slot];
    const double2* __restrict__ cf = L.S.coef + (int64_t)slot * kMaxM;
    double2* __restrict__ psi = L.V + gr.voff;
    const int B = gr.B;
    for (int64_t r = M.r0 + M.sub; r < M.r1; r += W * M.rpw) {
      const int64_t i = r * B + M.j;
      double ar = 0.0, ai = 0.0;
      typedef double dv2 __attribute__((ext_vector_type(2)));
      for (int l = 0; l < meff; ++l) {
        const dv2 v = __builtin_nontemporal_load(reinterpret_cast<const dv2*>(L.V) + (int64_t)l * L.ntot + gr.voff + i);
        const double2 c = cf[l];
        ar += c.x * v.x - c.y * v.y;
        ai += c.x * v.y + c.y * v.x;
      }
      __builtin_nontemporal_store(dv2{ar, ai}, reinterpret_cast<dv2*>(psi) + i);
      s += ar * ar + ai * ai;
    }
  }
  block_partial<W>(s, gr, red, L, lb);
}

// Fixed-order sum of instance j's block partials by one wavefront.
__device__ double slot_sum(const BLaunch& L, const BGroup& gr, int j) {
  const int lane = threadIdx.x & 63;
  const double* __restrict__ p = L.part + (int64_t)(gr.slot0 + j) * L.pstride;
  double s = thread_partials_chunked<64, 16>(p, gr.nblocks, lane);
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
  return lane_read(s, 0);
}

// Complete instance slot's basis at size mm: c = exp(-i dt T_mm) e_1 (computed
// here unless given), recombination coefficients, statistics.
__device__ void finish_slot(const BLaunch& L, int slot, int mm, double dt, double* lds,
                            bool have_c, double2 c, int why) {
  const int lane = threadIdx.x & 63;
  const int64_t sb = (int64_t)slot * kMaxM;
  const double beta0 = L.S.beta0[slot];
  int status = CFET_OK;
  if (!have_c) {
    const double a = (lane < mm) ? L.S.alpha[sb + lane] : 0.0;
    const double b = (lane < mm - 1) ? L.S.beta[sb + lane] : 0.0;
    const bool bad = !(isfinite(a) && isfinite(b));
    if (__ballot(bad) != 0ull) {
      status = CFET_ENONFINITE;
      c = make_double2(__builtin_nan(""), __builtin_nan(""));
    } else {
      status = tridiag_exp_e1(a, b, mm, dt, lds, c);
    }
  }
  if (lane < mm) {
    const double sc = beta0 * L.S.inv[sb + lane];
    L.S.coef[sb + lane] = make_double2(c.x * sc, c.y * sc);
  }
  if (lane == 0) {
    L.S.m_eff[slot] = mm;
    L.S.done[slot] = 1;
    L.S.matvecs[slot] += mm;
    L.S.expos[slot] += 1;
    if (why == 1) L.S.breakdowns[slot] += 1;
    if (why == 2) L.S.early[slot] += 1;
    if (mm < L.S.min_m[slot]) L.S.min_m[slot] = mm;
    if (mm > L.S.max_m[slot]) L.S.max_m[slot] = mm;
    if (status != CFET_OK && L.st->status == CFET_OK) L.st->status = status;
  }
}

__global__ __launch_bounds__(64) void k_b_scalars(BLaunch L, int mode, int k) {
  __shared__ double lds[kChebMaxTerms];
  const int slot = blockIdx.x;
  const int lane = threadIdx.x;
  const int g = find_group_of_slot(L.groups, L.ngroups, slot);
  const BGroup gr = L.groups[g];
  const int j = slot - gr.slot0;
  const int64_t sb = (int64_t)slot * kMaxM;
  const double dt = L.st->dt;
  if (mode == kBStart) {
    const double b0 = sqrt(slot_sum(L, gr, j));
    if (lane == 0) {
      L.S.beta0[slot] = b0;
      L.S.inv[sb] = (b0 > 0.0) ? 1.0 / b0 : 0.0;
      L.S.m_eff[slot] = 0;
      L.S.done[slot] = (b0 > 0.0) ? 0 : 1;
      if (!(b0 > 0.0)) {
        L.S.expos[slot] += 1;
        L.S.breakdowns[slot] += 1;
        L.S.min_m[slot] = 0;
        if (!isfinite(b0) && L.st->status == CFET_OK) L.st->status = CFET_ENONFINITE;
      }
    }
    return;
  }
  if (L.S.done[slot]) return;
  const int mcap = L.S.mcap[slot];
  if (mode == kBAlpha) {
    const double a = slot_sum(L, gr, j);
    if (lane == 0) L.S.alpha[sb + k] = a;
    wave_sync();
    if (k == mcap - 1) finish_slot(L, slot, k + 1, dt, lds, false, make_double2(0.0, 0.0), 0);
    return;
  }
  // kBBeta
  const double b = sqrt(slot_sum(L, gr, j));
  if (lane == 0) L.S.beta[sb + k] = b;
  wave_sync();
  const double al = (lane <= k) ? L.S.alpha[sb + lane] : 0.0;
  const double be = (lane < k) ? L.S.beta[sb + lane] : 0.0;
  double sc = (lane <= k) ? fabs(al) + ((lane < k) ? be : b) : 0.0;
  sc = wave_max(sc);
  if (b <= kBreakdownRel * sc) {
    finish_slot(L, slot, k + 1, dt, lds, false, make_double2(0.0, 0.0), 1);
    return;
  }
  const double tol = L.st->tol;
  if (tol > 0.0) {
    double2 c = make_double2(0.0, 0.0);
    const int mm = k + 1;
    const double a = (lane < mm) ? al : 0.0;
    const double bb = (lane < mm - 1) ? be : 0.0;
    const bool bad = !(isfinite(a) && isfinite(bb) && isfinite(b));
    if (__ballot(bad) == 0ull) {
      const int status = tridiag_exp_e1(a, bb, mm, dt, lds, c);
      const double ck = lane_read(sqrt(c.x * c.x + c.y * c.y), k);
      if (status == CFET_OK && fabs(dt) * b * ck <= tol) {
        finish_slot(L, slot, mm, dt, lds, true, c, 2);
        return;
      }
    }
  }
  if (lane == 0) L.S.inv[sb + k + 1] = 1.0 / b;
}

__global__ void k_b_advance(BState* st) {
  if (threadIdx.x == 0) st->cursor += 1;
}

__global__ void k_b_set_cursor(BState* st, long long v) {
  if (threadIdx.x == 0) st->cursor = v;
}

template <int W>
__global__ __launch_bounds__(64 * W) void k_b_pack(BLaunch L, const double2* __restrict__ user,
                                                        const int64_t* __restrict__ uoff, int dir) {
  const int lb = logical_block(L.total_blocks);
  if (lb >= L.total_blocks) return;
  const int g = find_group(L.groups, L.ngroups, lb);
  const BGroup gr = L.groups[g];
  const RowMap M = row_map(gr, g, lb);
  if (!M.lane_ok) return;
  const int64_t uo = uoff[gr.slot0 + M.j];
  double2* __restrict__ x = L.V + gr.voff;
  double2* __restrict__ u = const_cast<double2*>(user) + uo;
  for (int64_t r = M.r0 + M.sub; r < M.r1; r += W * M.rpw) {
    if (dir == 0) x[r * gr.B + M.j] = u[r];
    else u[r] = x[r * gr.B + M.j];
  }
}

__global__ void k_b_stats_reset(BSlots S, int nslots) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nslots) {
    S.matvecs[i] = 0;
    S.expos[i] = 0;
    S.breakdowns[i] = 0;
    S.early[i] = 0;
    S.min_m[i] = 1 << 30;
    S.max_m[i] = 0;
  }
}

}  // namespace

static inline int row_grid(const BLaunch& L) { return L.total_blocks; }

// launch a row kernel with the batch's block layout (L.waves wavefronts)
#define CFET_ROW_LAUNCH(KERNEL, ...)                                                        \
  do {                                                                                     \
    switch (L.waves) {                                                                     \
      case 2: hipLaunchKernelGGL(KERNEL<2>, dim3(row_grid(L)), dim3(128), 0, s, __VA_ARGS__); break; \
      case 8: hipLaunchKernelGGL(KERNEL<8>, dim3(row_grid(L)), dim3(512), 0, s, __VA_ARGS__); break; \
      default: hipLaunchKernelGGL(KERNEL<4>, dim3(row_grid(L)), dim3(256), 0, s, __VA_ARGS__); break; \
    }                                                                                      \
  } while (0)

hipError_t batch_norm(const BLaunch& L, hipStream_t s) {
  CFET_ROW_LAUNCH(k_b_norm, L);
  return hipGetLastError();
}

hipError_t batch_scalars(const BLaunch& L, int mode, int k, hipStream_t s) {
  hipLaunchKernelGGL(k_b_scalars, dim3(L.nslots), dim3(64), 0, s, L, mode, k);
  return hipGetLastError();
}

hipError_t batch_spmm(const BLaunch& L, int k, hipStream_t s) {
  CFET_ROW_LAUNCH(k_b_spmm, L, k);
  return hipGetLastError();
}

hipError_t batch_axpy(const BLaunch& L, int k, hipStream_t s) {
  CFET_ROW_LAUNCH(k_b_axpy, L, k);
  return hipGetLastError();
}

hipError_t batch_combine(const BLaunch& L, hipStream_t s) {
  CFET_ROW_LAUNCH(k_b_combine, L);
  return hipGetLastError();
}

hipError_t batch_advance(const BLaunch& L, hipStream_t s) {
  hipLaunchKernelGGL(k_b_advance, dim3(1), dim3(64), 0, s, L.st);
  return hipGetLastError();
}

hipError_t batch_set_cursor(const BLaunch& L, long long v, hipStream_t s) {
  hipLaunchKernelGGL(k_b_set_cursor, dim3(1), dim3(64), 0, s, L.st, v);
  return hipGetLastError();
}

hipError_t batch_pack(const BLaunch& L, const double2* user, const int64_t* uoff, hipStream_t s) {
  CFET_ROW_LAUNCH(k_b_pack, L, user, uoff, 0);
  return hipGetLastError();
}

hipError_t batch_unpack(const BLaunch& L, double2* user, const int64_t* uoff, hipStream_t s) {
  CFET_ROW_LAUNCH(k_b_pack, L, user, uoff, 1);
  return hipGetLastError();
}

hipError_t batch_stats_reset(const BLaunch& L, hipStream_t s) {
  hipLaunchKernelGGL(k_b_stats_reset, dim3((L.nslots + 255) / 256), dim3(256), 0, s, L.S,
                     L.nslots);
  return hipGetLastError();
}

}  // namespace cfet
