// Sliced-ELL (SELL-64) weighted apply for large dimensions (multi-kernel path).
//
// Layout: rows are cut into slices of 64 consecutive rows, one wavefront per
// slice and one lane per row.  Slice s stores its entries column-major,
// padded to the longest row of the slice: entry k of row 64 s + l sits at
// slice_ptr[s] + 64 k + l.  So every load of values and columns by a
// wavefront is one contiguous 1 KiB (values) / 256 B (columns) request.
// Within a row the driven terms come first (H_1 .. H_K, then H0), each in the
// caller's order; for operators built from site terms (the same local flip in
// every row) entry k of 64 consecutive rows then gathers 64 consecutive x
// values.  Matrix streams are read non-temporally so they do not evict x from
// the caches; padded slots are skipped (row lengths are stored per row).
// Optionally the entries that many rows of a slice hold with the same column
// offset (column = row XOR offset), term and value, such as a site term's
// flip with a uniform coupling, are stored once per slice with a 64-bit mask
// of the rows holding them, ahead of the per-row slots, so their values and
// columns are not streamed per row.
#include <hip/hip_runtime.h>

#include "cfet_internal.h"
#include "partials.hpp"

namespace cfet {

namespace {

constexpr int kSellBlock = 256;  // 4 slices per block
// The row kernels are held to 80 VGPRs (6 wavefronts per SIMD): the gathers of
// x are latency-bound and more resident wavefronts keep more of them in
// flight (8 per SIMD spills and runs slower).
#define CFET_SELL_OCCUPANCY __attribute__((amdgpu_waves_per_eu(6, 6)))
constexpr int kSellMaxBlocks = 3072;

typedef double dvec2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ double s_wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ double s_block_sum(double v, double* red) {
  v = s_wave_sum(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) red[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < kSellBlock / 64; ++i) t += red[i];
    red[16] = t;
  }
  __syncthreads();
  return red[16];
}

__device__ double s_sum_partials(const double* __restrict__ part, int np, double* red) {
  return s_block_sum(thread_partials<kSellBlock>(part, np), red);
}

template <int NT>
__device__ __forceinline__ void sell_acc(uint32_t ct, dvec2 v, double2 xv, const double* wl,
                                         double& a0r, double& a0i, double& a1r, double& a1i) {
  const double pr = v.x * xv.x - v.y * xv.y;
  const double pi = v.x * xv.y + v.y * xv.x;
  if (NT == 1) {
    if (ct >> kTermShift) { a1r += pr; a1i += pi; } else { a0r += pr; a0i += pi; }
  } else {
    const double wt = wl[ct >> kTermShift];
    a0r += wt * pr;
    a0i += wt * pi;
  }
}

// Shared entries of a slice: entry k is (offset | term, value) held by the
// rows of mask um[k] (bit = lane); a holding lane gathers x[row ^ offset],
// the others gather x[xr] (a valid row) and add a zero product, so the
// wavefront issues one gather per entry.
template <int NT>
__device__ __forceinline__ void shared_acc(const uint32_t* __restrict__ uc,
                                           const dvec2* __restrict__ uv,
                                           const uint64_t* __restrict__ um, int nu, int lane,
                                           int64_t row, int64_t xr, const double2* __restrict__ x,
                                           const double* wl, double& a0r, double& a0i,
                                           double& a1r, double& a1i) {
  int k = 0;
  for (; k + 4 <= nu; k += 4) {
    uint32_t ct[4];
    dvec2 v[4];
    bool on[4];
    double2 xv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      ct[u] = uc[k + u];
      v[u] = uv[k + u];
      on[u] = (um[k + u] >> lane) & 1ull;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) xv[u] = x[on[u] ? row ^ (int64_t)(ct[u] & kColMask) : xr];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (!on[u]) v[u] = dvec2{0.0, 0.0};
      sell_acc<NT>(ct[u], v[u], xv[u], wl, a0r, a0i, a1r, a1i);
    }
  }
  for (; k < nu; ++k) {
    const uint32_t ct = uc[k];
    const bool on = (um[k] >> lane) & 1ull;
    const double2 xv = x[on ? row ^ (int64_t)(ct & kColMask) : xr];
    const dvec2 v = on ? uv[k] : dvec2{0.0, 0.0};
    sell_acc<NT>(ct, v, xv, wl, a0r, a0i, a1r, a1i);
  }
}

// y_row = sum_k w_{term} val x[col] over the row's entries (lane = row; the
// slice index is the same for the whole wavefront).
template <int NT>
__device__ __forceinline__ double2 sell_row(const DevSELL& S, int64_t slice_in, int lane, int64_t row,
                                            const double2* __restrict__ x, const double* wl) {
  // slices number below 2^23 (rows below 2^29): the index fits a scalar register
  const int64_t slice = __builtin_amdgcn_readfirstlane((int)slice_in);
  const int64_t base = S.slice_ptr[slice];
  const int width = S.slice_width[slice];
  const bool valid = row < S.n;
  int len = valid ? (int)S.rowlen[row] : 0;
  double a0r = 0.0, a0i = 0.0, a1r = 0.0, a1i = 0.0;
  // shared entries: one (offset, term, value) for the rows in its mask,
  // column = row ^ offset; the other rows gather x[row] and drop the product
  const int nu = S.nuni ? S.nuni[slice] : 0;
  if (nu > 0) {
    const int64_t ub = S.uptr[slice];
    shared_acc<NT>(S.ucolt + ub, reinterpret_cast<const dvec2*>(S.uval) + ub, S.umask + ub, nu,
                   lane, row, valid ? row : 0, x, wl, a0r, a0i, a1r, a1i);
  }
  const uint32_t* __restrict__ cp = S.colt + base + lane;
  const dvec2* __restrict__ vp = reinterpret_cast<const dvec2*>(S.val) + base + lane;
  int k = 0;
  // padded slots (k >= len) are neither loaded nor gathered
  for (; k + 4 <= width; k += 4) {
    uint32_t ct[4];
    dvec2 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (k + u < len) {
        ct[u] = __builtin_nontemporal_load(cp + (int64_t)(k + u) * 64);
        v[u] = __builtin_nontemporal_load(vp + (int64_t)(k + u) * 64);
      } else {
        ct[u] = 0u;
        v[u] = dvec2{0.0, 0.0};
      }
    }
    double2 xv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) xv[u] = (k + u < len) ? x[ct[u] & kColMask] : make_double2(0.0, 0.0);
#pragma unroll
    for (int u = 0; u < 4; ++u) sell_acc<NT>(ct[u], v[u], xv[u], wl, a0r, a0i, a1r, a1i);
  }
  for (; k < len; ++k) {
    const uint32_t ct = __builtin_nontemporal_load(cp + (int64_t)k * 64);
    const dvec2 v = __builtin_nontemporal_load(vp + (int64_t)k * 64);
    sell_acc<NT>(ct, v, x[ct & kColMask], wl, a0r, a0i, a1r, a1i);
  }
  if (NT == 1) return make_double2(wl[0] * a0r + wl[1] * a1r, wl[0] * a0i + wl[1] * a1i);
  return make_double2(a0r, a0i);
}

// Slice schedule: workgroups are dealt to the 8 XCDs round-robin, so block b
// runs on XCD b % 8.  Each XCD is given one contiguous eighth of the slices,
// swept by its own blocks in lock-step, so the x lines gathered for nearby
// rows stay in that XCD's L2.  (Any grid size is valid; for a grid that is not
// a multiple of 8 the plain grid-stride order is used.)
struct SliceRange {
  int64_t first, end, stride;
};

__device__ __forceinline__ SliceRange slice_range(int64_t nslices) {
  constexpr int kXcds = 8;
  constexpr int kWaves = kSellBlock / 64;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave index (uniform)
  const int nb = gridDim.x;
  if (nb % kXcds != 0) {
    return {(int64_t)blockIdx.x * kWaves + w, nslices, (int64_t)nb * kWaves};
  }
  const int xcd = blockIdx.x % kXcds;
  const int rank = blockIdx.x / kXcds;
  const int64_t per = (nslices + kXcds - 1) / kXcds;
  const int64_t beg = min(nslices, (int64_t)xcd * per);
  const int64_t end = min(nslices, beg + per);
  return {beg + (int64_t)rank * kWaves + w, end, (int64_t)(nb / kXcds) * kWaves};
}

template <int NT>
__global__ __launch_bounds__(kSellBlock) CFET_SELL_OCCUPANCY void k_sell_apply(DevSELL S, TermWeights tw,
                                                           const double2* __restrict__ x,
                                                           double2* __restrict__ y) {
  __shared__ double wl[kMaxTerms + 1];
  if (threadIdx.x <= kMaxTerms) wl[threadIdx.x] = tw.w[threadIdx.x];
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const SliceRange R = slice_range((S.n + 63) / 64);
  for (int64_t sl = R.first; sl < R.end; sl += R.stride) {
    const int64_t row = sl * 64 + lane;
    const double2 r = sell_row<NT>(S, sl, lane, row, x, wl);
    if (row < S.n) y[row] = r;
  }
}

// Lanczos SpMV on the SELL layout; same contract as the CSR kernel: finishes
// the pending norm reduction, applies the early-stop rule, y = H_w v_j and
// partials of Re<v_j, y>.
template <int NT>
__global__ __launch_bounds__(kSellBlock) CFET_SELL_OCCUPANCY void k_sell_lz_spmv(
    DevSELL S, TermWeights tw, const double2* __restrict__ x, double2* __restrict__ y,
    const double* __restrict__ part_in, int np_in, double* __restrict__ part_out, LzScalars* L,
    int j) {
  __shared__ double red[17];
  __shared__ double wl[kMaxTerms + 1];
  if (j > 0 && L->brk[j - 1]) {
    if (blockIdx.x == 0 && threadIdx.x == 0) L->brk[j] = 1;
    return;
  }
  const double nrm2 = s_sum_partials(part_in, np_in, red);
  double inv;
  const bool b0 = (blockIdx.x == 0 && threadIdx.x == 0);
  if (j == 0) {
    const double beta0 = sqrt(nrm2);
    const bool stop = (beta0 == 0.0);
    if (b0) {
      L->beta0 = beta0;
      L->inv_nrm[0] = stop ? 0.0 : 1.0 / beta0;
      L->brk[0] = stop ? 1 : 0;
      if (stop) L->m_eff = 0;
    }
    if (stop) return;
    inv = 1.0 / beta0;
  } else {
    const double b = sqrt(nrm2);
    double sc = 0.0;
    for (int k = 0; k < j - 1; ++k) sc = fmax(sc, fabs(L->alpha[k]) + L->beta[k]);
    sc = fmax(sc, fabs(L->alpha[j - 1]) + b);
    const bool stop = (b <= kBreakdownRel * sc);
    if (b0) {
      L->beta[j - 1] = b;
      L->brk[j] = stop ? 1 : 0;
      if (stop) L->m_eff = j;
      else L->inv_nrm[j] = 1.0 / b;
    }
    if (stop) return;
    inv = 1.0 / b;
  }
  if (threadIdx.x <= kMaxTerms) wl[threadIdx.x] = tw.w[threadIdx.x];
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const SliceRange R = slice_range((S.n + 63) / 64);
  double apart = 0.0;
  for (int64_t sl = R.first; sl < R.end; sl += R.stride) {
    const int64_t row = sl * 64 + lane;
    double2 r = sell_row<NT>(S, sl, lane, row, x, wl);
    if (row < S.n) {
      r.x *= inv;
      r.y *= inv;
      // the product is read by the next kernel only: stream it past the caches
      if (y) __builtin_nontemporal_store(*reinterpret_cast<const dvec2*>(&r),
                                         reinterpret_cast<dvec2*>(y) + row);
      const double2 xr = x[row];
      apart += (xr.x * r.x + xr.y * r.y) * inv;
    }
  }
  apart = s_block_sum(apart, red);
  if (threadIdx.x == 0) part_out[blockIdx.x] = apart;
}


}  // namespace

int sell_grid(int64_t n) {
  const int64_t nslices = (n + 63) / 64;
  const int64_t want = (nslices + (kSellBlock / 64) - 1) / (kSellBlock / 64);
  return (int)std::max<int64_t>(1, std::min<int64_t>(want, kSellMaxBlocks));
}

hipError_t launch_sell_apply(const DevSELL& S, int nterms, const TermWeights& tw, const double2* x,
                             double2* y, hipStream_t st) {
  const int nb = sell_grid(S.n);
  if (nterms == 1)
    hipLaunchKernelGGL(k_sell_apply<1>, dim3(nb), dim3(kSellBlock), 0, st, S, tw, x, y);
  else
    hipLaunchKernelGGL(k_sell_apply<0>, dim3(nb), dim3(kSellBlock), 0, st, S, tw, x, y);
  return hipGetLastError();
}

hipError_t launch_sell_lz_spmv(const DevSELL& S, int nterms, const TermWeights& tw,
                               const double2* x, double2* y, const double* pin, int npin,
                               double* pout, LzScalars* L, int j, hipStream_t st) {
  const int nb = sell_grid(S.n);
  if (nterms == 1)
    hipLaunchKernelGGL(k_sell_lz_spmv<1>, dim3(nb), dim3(kSellBlock), 0, st, S, tw, x, y, pin,
                       npin, pout, L, j);
  else
    hipLaunchKernelGGL(k_sell_lz_spmv<0>, dim3(nb), dim3(kSellBlock), 0, st, S, tw, x, y, pin,
                       npin, pout, L, j);
  return hipGetLastError();
}

}  // namespace cfet
