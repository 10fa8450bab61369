// HIP kernels for the CFET propagator on gfx950 (multi-kernel path).
//
// One exponential psi <- exp(-i dt H_w) psi, H_w = w0 H0 + sum_k w_k H_k, is
// the Krylov (Lanczos) technique of paper Sec. 8.1, split into kernels that
// stay on the device between launches (no host synchronisation):
//
//   K0 k_norm_start   partials of ||psi||^2                  (first exponential only)
//   K1 k_lz_spmv<G>   y = H_w v_j (v_j = w_j / nrm_j) and partials of Re<v_j, y>;
//                     it first finishes the pending norm reduction (beta_{j-1} or
//                     beta_0) and applies the early-stop rule
//   K2 k_lz_axpy      w_{j+1} = y - alpha_j v_j - beta_{j-1} v_{j-1}, partials of ||w||^2
//   K3 k_lz_small     T = tridiag(beta; alpha) -> c = exp(-i dt T) e_1 (one wavefront,
//                     implicit symmetric QR with Wilkinson shift, Z in LDS)
//   K4 k_lz_combine   psi <- beta_0 sum_j c_j v_j, partials of ||psi||^2 for the next one
//
// Basis vectors are stored unnormalised (w_j with scale inv_nrm[j]), so no
// kernel rewrites a vector just to normalise it; w_0 is psi itself.
// Reductions are deterministic: per-block tree sums written to a partials
// array, and every consumer block re-reduces the partials in a fixed order.
#include <hip/hip_runtime.h>

#include <algorithm>

#include <cmath>

#include "cfet_internal.h"
#include "partials.hpp"
#include "tridiag.hpp"

namespace cfet {

namespace {

constexpr int kBlock = 256;
constexpr int kMaxBlocks = 2048;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum over the block; every thread receives thread 0's result.
__device__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if (l == 0) red[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < nw; ++i) t += red[i];
    red[16] = t;
  }
  __syncthreads();
  return red[16];
}

// THREADS: the kernel's block size
template <int THREADS>
__device__ double sum_partials(const double* __restrict__ part, int np, double* red) {
  return block_sum(thread_partials<THREADS>(part, np), red);
}

__device__ __forceinline__ bool block0_thread0() { return blockIdx.x == 0 && threadIdx.x == 0; }

// out[i] = in[idx[i]] (a row permutation of a vector; out and in distinct)
__global__ __launch_bounds__(kBlock) void k_permute(double2* __restrict__ out,
                                                    const double2* __restrict__ in,
                                                    const int32_t* __restrict__ idx, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    out[i] = in[idx[i]];
}

__global__ __launch_bounds__(kBlock) void k_norm_start(const double2* __restrict__ psi, int64_t n,
                                                       double* __restrict__ part) {
  __shared__ double red[17];
  double s = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += stride) {
    const double2 v = psi[r];
    s += v.x * v.x + v.y * v.y;
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// part[block] = sum over the block's rows of |a_r - b_r|^2 (the distance of
// two states, taken on their difference so that it keeps full relative
// accuracy when the states agree to many digits)
__global__ __launch_bounds__(kBlock) void k_dist2(const double2* __restrict__ a,
                                                  const double2* __restrict__ b, int64_t n,
                                                  double* __restrict__ part) {
  __shared__ double red[17];
  double s = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += stride) {
    const double2 u = a[r], v = b[r];
    const double dx = u.x - v.x, dy = u.y - v.y;
    s += dx * dx + dy * dy;
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// Chebyshev exponential (Sec. 8.1): start of the series.  v0 = psi,
// psi = c0 psi; block 0 counts the exponential and its K products.
__global__ __launch_bounds__(kBlock) void k_cheb_start(double2* __restrict__ psi,
                                                       double2* __restrict__ v0, int64_t n,
                                                       double2 c0, int K,
                                                       DevStats* __restrict__ st) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += stride) {
    const double2 p = psi[r];
    v0[r] = p;
    psi[r] = make_double2(c0.x * p.x - c0.y * p.y, c0.x * p.y + c0.y * p.x);
  }
  if (block0_thread0()) {
    st->exponentials += 1;
    st->matvecs += (unsigned long long)K;
    if (K < st->min_m_eff) st->min_m_eff = K;
  }
}

// One term of the series: w = scale (y - sigma v) - prev  (prev omitted for
// the first term), prev <- w (the next polynomial), psi += ck w.  y = H_w v
// from the apply kernels; scale is 1/h for T_1 and 2/h after it.
__global__ __launch_bounds__(kBlock) void k_cheb_update(const double2* __restrict__ y,
                                                        const double2* __restrict__ v,
                                                        double2* __restrict__ prev,
                                                        double2* __restrict__ psi, int64_t n,
                                                        double scale, double sigma, int first,
                                                        double2 ck) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += stride) {
    const double2 yy = y[r], vv = v[r];
    double wr = scale * (yy.x - sigma * vv.x);
    double wi = scale * (yy.y - sigma * vv.y);
    if (!first) {
      const double2 pp = prev[r];
      wr -= pp.x;
      wi -= pp.y;
    }
    prev[r] = make_double2(wr, wi);
    const double2 p = psi[r];
    psi[r] = make_double2(p.x + ck.x * wr - ck.y * wi, p.y + ck.x * wi + ck.y * wr);
  }
}

// y = H_w x for one row handled by a group of G lanes; NT = 1 specialises the
// single-drive case (term bit selects the accumulator), NT = 0 is generic.
template <int G, int NT>
__device__ __forceinline__ double2 row_apply(const int64_t* __restrict__ rowptr,
                                             const uint32_t* __restrict__ colt,
                                             const double2* __restrict__ val,
                                             const double2* __restrict__ x, int64_t row, int lane,
                                             const double* wl, double w0, double w1) {
  const int64_t beg = rowptr[row], end = rowptr[row + 1];
  double a0r = 0.0, a0i = 0.0, a1r = 0.0, a1i = 0.0;
  for (int64_t e = beg + lane; e < end; e += G) {
    const uint32_t ct = colt[e];
    const double2 v = val[e];
    const double2 xv = x[ct & kColMask];
    const double pr = v.x * xv.x - v.y * xv.y;
    const double pi = v.x * xv.y + v.y * xv.x;
    if (NT == 1) {
      if (ct >> kTermShift) {
        a1r += pr;
        a1i += pi;
      } else {
        a0r += pr;
        a0i += pi;
      }
    } else {
      const double wt = wl[ct >> kTermShift];
      a0r += wt * pr;
      a0i += wt * pi;
    }
  }
  double yr, yi;
  if (NT == 1) {
    yr = w0 * a0r + w1 * a1r;
    yi = w0 * a0i + w1 * a1i;
  } else {
    yr = a0r;
    yi = a0i;
  }
#pragma unroll
  for (int off = G / 2; off >= 1; off >>= 1) {
    yr += __shfl_xor(yr, off, G);
    yi += __shfl_xor(yi, off, G);
  }
  return make_double2(yr, yi);
}

template <int G, int NT>
__global__ __launch_bounds__(kBlock) void k_apply(const int64_t* __restrict__ rowptr,
                                                  const uint32_t* __restrict__ colt,
                                                  const double2* __restrict__ val, int64_t n,
                                                  TermWeights tw, const double2* __restrict__ x,
                                                  double2* __restrict__ y) {
  __shared__ double wl[kMaxTerms + 1];
  if (threadIdx.x <= kMaxTerms) wl[threadIdx.x] = tw.w[threadIdx.x];
  __syncthreads();
  const int lane = threadIdx.x % G;
  const int64_t ngroups = (int64_t)gridDim.x * blockDim.x / G;
  for (int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G; row < n; row += ngroups) {
    const double2 r = row_apply<G, NT>(rowptr, colt, val, x, row, lane, wl, tw.w[0], tw.w[1]);
    if (lane == 0) y[row] = r;
  }
}

template <int G, int NT>
__global__ __launch_bounds__(kBlock) void k_lz_spmv(
    const int64_t* __restrict__ rowptr, const uint32_t* __restrict__ colt,
    const double2* __restrict__ val, int64_t n, TermWeights tw, const TermWeights* twp,
    const double2* __restrict__ x, double2* __restrict__ y, const double* __restrict__ part_in,
    int np_in, double* __restrict__ part_out, LzScalars* S, int j) {
  __shared__ double red[17];
  __shared__ double wl[kMaxTerms + 1];
  if (twp) tw = *twp;  // weights from device memory (replayed graphs)
  // stopped at an earlier step: pass the flag on and do nothing
  if (j > 0 && S->brk[j - 1]) {
    if (block0_thread0()) S->brk[j] = 1;
    return;
  }
  const double nrm2 = sum_partials<kBlock>(part_in, np_in, red);
  double inv;
  if (j == 0) {
    const double b0 = sqrt(nrm2);
    const bool stop = (b0 == 0.0);
    if (block0_thread0()) {
      S->beta0 = b0;
      S->inv_nrm[0] = stop ? 0.0 : 1.0 / b0;
      S->brk[0] = stop ? 1 : 0;
      if (stop) S->m_eff = 0;
    }
    if (stop) return;
    inv = 1.0 / b0;
  } else {
    const double b = sqrt(nrm2);
    double sc = 0.0;
    for (int k = 0; k < j - 1; ++k) sc = fmax(sc, fabs(S->alpha[k]) + S->beta[k]);
    sc = fmax(sc, fabs(S->alpha[j - 1]) + b);
    const bool stop = (b <= kBreakdownRel * sc);
    if (block0_thread0()) {
      S->beta[j - 1] = b;
      S->brk[j] = stop ? 1 : 0;
      if (stop) {
        S->m_eff = j;
      } else {
        S->inv_nrm[j] = 1.0 / b;
      }
    }
    if (stop) return;
    inv = 1.0 / b;
  }
  if (threadIdx.x <= kMaxTerms) wl[threadIdx.x] = tw.w[threadIdx.x];
  __syncthreads();
  const int lane = threadIdx.x % G;
  const int64_t ngroups = (int64_t)gridDim.x * blockDim.x / G;
  double apart = 0.0;
  for (int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G; row < n; row += ngroups) {
    double2 r = row_apply<G, NT>(rowptr, colt, val, x, row, lane, wl, tw.w[0], tw.w[1]);
    r.x *= inv;
    r.y *= inv;
    if (lane == 0) {
      if (y) y[row] = r;
      const double2 xr = x[row];
      apart += (xr.x * r.x + xr.y * r.y) * inv;
    }
  }
  apart = block_sum(apart, red);
  if (threadIdx.x == 0) part_out[blockIdx.x] = apart;
}

__global__ __launch_bounds__(kBlock) void k_lz_axpy(int64_t n, const double2* __restrict__ wj,
                                                    const double2* __restrict__ wjm1,
                                                    double2* __restrict__ wnext,
                                                    const double* __restrict__ part_in, int np_in,
                                                    double* __restrict__ part_out, LzScalars* S,
                                                    int j) {
  __shared__ double red[17];
  if (S->brk[j]) return;
  const double alpha = sum_partials<kBlock>(part_in, np_in, red);
  if (block0_thread0()) S->alpha[j] = alpha;
  const double ca = alpha * S->inv_nrm[j];
  const double cb = (j > 0) ? S->beta[j - 1] * S->inv_nrm[j - 1] : 0.0;
  double s = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  // the three vectors stream through once (each larger than the caches at
  // the sizes where this path runs): non-temporal loads and store
  typedef double dv2 __attribute__((ext_vector_type(2)));
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += stride) {
    const dv2 y = __builtin_nontemporal_load(reinterpret_cast<const dv2*>(wnext) + r);
    const dv2 a = __builtin_nontemporal_load(reinterpret_cast<const dv2*>(wj) + r);
    double wr = y.x - ca * a.x, wi = y.y - ca * a.y;
    if (j > 0) {
      const dv2 b = __builtin_nontemporal_load(reinterpret_cast<const dv2*>(wjm1) + r);
      wr -= cb * b.x;
      wi -= cb * b.y;
    }
    __builtin_nontemporal_store(dv2{wr, wi}, reinterpret_cast<dv2*>(wnext) + r);
    s += wr * wr + wi * wi;
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) part_out[blockIdx.x] = s;
}

__global__ __launch_bounds__(64) void k_lz_small(const double* __restrict__ part_in, int np_in,
                                                 LzScalars* S, int m, double dt, DevStats* stats) {
  __shared__ double lds[kChebMaxTerms];
  __shared__ double red[17];
  const int lane = threadIdx.x;
  const int done = S->brk[m - 1];
  int meff;
  double alast = 0.0;
  if (!done) {
    alast = sum_partials<64>(part_in, np_in, red);
    meff = m;
  } else {
    meff = S->m_eff;
  }
  double a = 0.0, b = 0.0;
  if (lane < meff) a = (!done && lane == m - 1) ? alast : S->alpha[lane];
  if (lane < meff - 1) b = S->beta[lane];
  const double beta0 = S->beta0;
  int status = CFET_OK;
  double2 c = make_double2(0.0, 0.0);
  if (meff > 0) {
    const bool bad = !(isfinite(a) && isfinite(b) && isfinite(beta0));
    if (__ballot(bad) != 0ull) {
      status = CFET_ENONFINITE;
    } else {
      status = tridiag_exp_e1(a, b, meff, dt, lds, c);
    }
  }
  if (lane < meff) {
    const double sc = beta0 * S->inv_nrm[lane];
    S->coef[2 * lane] = c.x * sc;
    S->coef[2 * lane + 1] = c.y * sc;
  }
  if (lane == 0) {
    if (!done) {
      S->alpha[m - 1] = alast;
      S->m_eff = meff;
    }
    stats->exponentials += 1;
    stats->matvecs += (unsigned long long)meff;
    if (meff < stats->min_m_eff) stats->min_m_eff = meff;
    if (done) stats->breakdowns += 1;
    if (status != CFET_OK && stats->status == CFET_OK) stats->status = status;
    stats->last_norm2 = beta0 * beta0;
  }
}

// basis vector j >= 1 lives at basis + (j-1)*n; vector 0 is psi itself
__global__ __launch_bounds__(kBlock) void k_lz_combine(double2* __restrict__ psi,
                                                       const double2* __restrict__ basis, int64_t n,
                                                       const LzScalars* __restrict__ S,
                                                       double* __restrict__ part_out) {
  __shared__ double red[17];
  __shared__ double2 cf[kMaxM];
  const int meff = S->m_eff;
  if (threadIdx.x < meff)
    cf[threadIdx.x] = make_double2(S->coef[2 * threadIdx.x], S->coef[2 * threadIdx.x + 1]);
  __syncthreads();
  double s = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += stride) {
    double accr = 0.0, acci = 0.0;
    // the basis vectors and psi stream through once: non-temporal accesses
    typedef double dv2 __attribute__((ext_vector_type(2)));
    for (int jj = 0; jj < meff; ++jj) {
      const dv2* src = (jj == 0) ? reinterpret_cast<const dv2*>(psi) + r
                                 : reinterpret_cast<const dv2*>(basis) + (int64_t)(jj - 1) * n + r;
      const dv2 v = __builtin_nontemporal_load(src);
      const double2 k = cf[jj];
      accr += k.x * v.x - k.y * v.y;
      acci += k.x * v.y + k.y * v.x;
    }
    __builtin_nontemporal_store(dv2{accr, acci}, reinterpret_cast<dv2*>(psi) + r);
    s += accr * accr + acci * acci;
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) part_out[blockIdx.x] = s;
}

__global__ __launch_bounds__(64) void k_tridiag_expm(const double* __restrict__ alpha,
                                                     const double* __restrict__ beta, int k,
                                                     double dt, double2* __restrict__ c_out,
                                                     int32_t* status_out) {
  __shared__ double lds[kChebMaxTerms];
  const int lane = threadIdx.x;
  const double a = (lane < k) ? alpha[lane] : 0.0;
  const double b = (lane < k - 1) ? beta[lane] : 0.0;
  double2 c = make_double2(0.0, 0.0);
  int status;
  const bool bad = !(isfinite(a) && isfinite(b));
  if (__ballot(bad) != 0ull) {
    status = CFET_ENONFINITE;
  } else {
    status = tridiag_exp_e1(a, b, k, dt, lds, c);
  }
  if (lane < k) c_out[lane] = c;
  if (lane == 0 && status_out) *status_out = status;
}

__global__ void k_stats_init(DevStats* st) {
  st->exponentials = 0;
  st->matvecs = 0;
  st->min_m_eff = 1 << 30;
  st->breakdowns = 0;
  st->status = CFET_OK;
  st->last_norm2 = 0.0;
  for (int i = 0; i < 4; ++i) st->seg[i] = 0;
}

__global__ __launch_bounds__(kBlock) void k_final_norm(const double* __restrict__ part, int np,
                                                       DevStats* st) {
  __shared__ double red[17];
  const double s = sum_partials<kBlock>(part, np, red);
  if (threadIdx.x == 0) st->last_norm2 = s;
}

template <int NT>
hipError_t dispatch_apply(int G, const DevCSR& A, int nb, const TermWeights& tw,
                          const double2* x, double2* y, hipStream_t st) {
#define CFET_APPLY_CASE(GG)                                                                  \
  case GG:                                                                                  \
    hipLaunchKernelGGL((k_apply<GG, NT>), dim3(nb), dim3(kBlock), 0, st, A.rowptr, A.colt, \
                       A.val, A.n, tw, x, y);                                               \
    break;
  switch (G) {
    CFET_APPLY_CASE(1)
    CFET_APPLY_CASE(2)
    CFET_APPLY_CASE(4)
    CFET_APPLY_CASE(8)
    CFET_APPLY_CASE(16)
    CFET_APPLY_CASE(32)
    default:
      return hipErrorInvalidValue;
  }
#undef CFET_APPLY_CASE
  return hipGetLastError();
}

template <int NT>
hipError_t dispatch_spmv(int G, const DevCSR& A, int nb, const TermWeights& tw,
                         const TermWeights* twp, const double2* x, double2* y, const double* pin,
                         int npin, double* pout, LzScalars* S, int j, hipStream_t st) {
#define CFET_SPMV_CASE(GG)                                                                      \
  case GG:                                                                                     \
    hipLaunchKernelGGL((k_lz_spmv<GG, NT>), dim3(nb), dim3(kBlock), 0, st, A.rowptr, A.colt,  \
                       A.val, A.n, tw, twp, x, y, pin, npin, pout, S, j);                     \
    break;
  switch (G) {
    CFET_SPMV_CASE(1)
    CFET_SPMV_CASE(2)
    CFET_SPMV_CASE(4)
    CFET_SPMV_CASE(8)
    CFET_SPMV_CASE(16)
    CFET_SPMV_CASE(32)
    default:
      return hipErrorInvalidValue;
  }
#undef CFET_SPMV_CASE
  return hipGetLastError();
}

}  // namespace

LaunchPlan make_plan(int64_t n, int64_t nnz) {
  LaunchPlan p;
  const double avg = n > 0 ? double(nnz) / double(n) : 1.0;
  int G = 1;
  while (G < 32 && 2.0 * G <= avg / 2.0) G *= 2;
  p.G = G;
  const int64_t want_spmv = (n * G + kBlock - 1) / kBlock;
  const int64_t want_vec = (n + kBlock - 1) / kBlock;
  p.nb_spmv = (int)std::max<int64_t>(1, std::min<int64_t>(want_spmv, kMaxBlocks));
  p.nb_vec = (int)std::max<int64_t>(1, std::min<int64_t>(want_vec, kMaxBlocks));
  return p;
}

hipError_t launch_apply(const DevCSR& A, int nterms, const LaunchPlan& plan, const TermWeights& tw,
                        const double2* x, double2* y, hipStream_t st) {
  if (nterms == 1) return dispatch_apply<1>(plan.G, A, plan.nb_spmv, tw, x, y, st);
  return dispatch_apply<0>(plan.G, A, plan.nb_spmv, tw, x, y, st);
}

hipError_t launch_permute(double2* out, const double2* in, const int32_t* idx, int64_t n,
                          hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int nb = (int)std::min<int64_t>((n + kBlock - 1) / kBlock, 4096);
  hipLaunchKernelGGL(k_permute, dim3(nb), dim3(kBlock), 0, st, out, in, idx, n);
  return hipGetLastError();
}

hipError_t launch_norm_start(const double2* psi, int64_t n, const LaunchPlan& plan, double* part,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_norm_start, dim3(plan.nb_vec), dim3(kBlock), 0, st, psi, n, part);
  return hipGetLastError();
}

hipError_t launch_lanczos(const DevCSR& A, int nterms, const LaunchPlan& plan,
                              const TermWeights& tw, double dt, int m, const ExpWork& wk,
                              hipStream_t st) {
  LzScalars* S = wk.S;
  hipError_t e = hipSuccess;
  // partial sums of alpha: one per block of the SpMV (of each of its passes)
  const int np_alpha = (wk.sell && wk.hi) ? 2 * wk.nb_tile : plan.nb_spmv;
  for (int j = 0; j < m; ++j) {
    const double2* x = wk.W_host[j];
    double2* y = (j + 1 < m) ? wk.W_host[j + 1] : nullptr;
    EventPool* ev = (wk.events && wk.events->used < wk.events->cap) ? wk.events : nullptr;
    if (ev) (void)hipEventRecord(ev->begin[ev->used], st);
    if (wk.sell && wk.hi)
      e = launch_tile_lz_spmv(*wk.sell, *wk.hi, wk.tbits, wk.nb_tile, nterms, wk.tile_real, tw, x,
                              y, wk.partA, plan.nb_vec, wk.partB, S, j, st);
    else if (wk.sell)
      e = launch_sell_lz_spmv(*wk.sell, nterms, tw, x, y, wk.partA, plan.nb_vec, wk.partB, S, j, st);
    else if (nterms == 1)
      e = dispatch_spmv<1>(plan.G, A, plan.nb_spmv, tw, wk.twp, x, y, wk.partA, plan.nb_vec,
                           wk.partB, S, j, st);
    else
      e = dispatch_spmv<0>(plan.G, A, plan.nb_spmv, tw, wk.twp, x, y, wk.partA, plan.nb_vec,
                           wk.partB, S, j, st);
    if (e != hipSuccess) return e;
    if (ev) {
      (void)hipEventRecord(ev->end[ev->used], st);
      ev->used += 1;
    }
    if (j + 1 < m) {
      const double2* wm1 = (j > 0) ? wk.W_host[j - 1] : nullptr;
      hipLaunchKernelGGL(k_lz_axpy, dim3(plan.nb_vec), dim3(kBlock), 0, st, A.n, x, wm1,
                         wk.W_host[j + 1], wk.partB, np_alpha, wk.partA, S, j);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
  }
  hipLaunchKernelGGL(k_lz_small, dim3(1), dim3(64), 0, st, wk.partB, np_alpha, S, m, dt,
                     wk.stats);
  return hipGetLastError();
}

hipError_t launch_combine(int64_t n, const LaunchPlan& plan, const ExpWork& wk, hipStream_t st) {
  hipLaunchKernelGGL(k_lz_combine, dim3(plan.nb_vec), dim3(kBlock), 0, st, wk.W_host[0],
                     (const double2*)wk.W_host[1], n, wk.S, wk.partA);
  return hipGetLastError();
}

hipError_t launch_exponential(const DevCSR& A, int nterms, const LaunchPlan& plan,
                              const TermWeights& tw, double dt, int m, const ExpWork& wk,
                              hipStream_t st) {
  const hipError_t e = launch_lanczos(A, nterms, plan, tw, dt, m, wk, st);
  if (e != hipSuccess) return e;
  return launch_combine(A.n, plan, wk, st);
}

hipError_t launch_final_norm(const double* part, int np, DevStats* st_dev, hipStream_t st) {
  hipLaunchKernelGGL(k_final_norm, dim3(1), dim3(kBlock), 0, st, part, np, st_dev);
  return hipGetLastError();
}

hipError_t launch_cheb_start(double2* psi, double2* v0, int64_t n, double2 c0, int K,
                             DevStats* st_dev, hipStream_t st) {
  const int nb = (int)std::max<int64_t>(1, std::min<int64_t>((n + kBlock - 1) / kBlock, kMaxBlocks));
  hipLaunchKernelGGL(k_cheb_start, dim3(nb), dim3(kBlock), 0, st, psi, v0, n, c0, K, st_dev);
  return hipGetLastError();
}

hipError_t launch_cheb_update(const double2* y, const double2* v, double2* prev, double2* psi,
                              int64_t n, double scale, double sigma, bool first, double2 ck,
                              hipStream_t st) {
  const int nb = (int)std::max<int64_t>(1, std::min<int64_t>((n + kBlock - 1) / kBlock, kMaxBlocks));
  hipLaunchKernelGGL(k_cheb_update, dim3(nb), dim3(kBlock), 0, st, y, v, prev, psi, n, scale,
                     sigma, first ? 1 : 0, ck);
  return hipGetLastError();
}

int dist2_blocks(int64_t n) {
  return (int)std::max<int64_t>(1, std::min<int64_t>((n + kBlock - 1) / kBlock, kMaxBlocks));
}

hipError_t launch_dist2(const double2* a, const double2* b, int64_t n, double* part,
                        hipStream_t st) {
  hipLaunchKernelGGL(k_dist2, dim3(dist2_blocks(n)), dim3(kBlock), 0, st, a, b, n, part);
  return hipGetLastError();
}

hipError_t launch_tridiag_expm(const double* alpha, const double* beta, int k, double dt,
                               double2* c, int32_t* status, hipStream_t st) {
  hipLaunchKernelGGL(k_tridiag_expm, dim3(1), dim3(64), 0, st, alpha, beta, k, dt, c, status);
  return hipGetLastError();
}

hipError_t launch_stats_init(DevStats* st_dev, hipStream_t st) {
  hipLaunchKernelGGL(k_stats_init, dim3(1), dim3(1), 0, st, st_dev);
  return hipGetLastError();
}

}  // namespace cfet
