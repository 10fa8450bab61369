// Device kernels of the fidelity gradient (cfet_gradient).
//
// For one exponential E = exp(-i dt H_i) of the CFET step, with the Lanczos
// bases of H_i started from the state psi before E (stored vectors w_j,
// v_j = w_j inv_j, tridiagonal T) and from the adjoint state lam after E
// (vectors u_k, tridiagonal S), the derivative of <lam|E|psi> along H_k* is
// taken from the block-triangular augmented operator projected onto the two
// Krylov spaces:
//     g = beta_lam beta_psi e_1^T exp(M) e_{m_lam + 1},
//     M = -i dt [[S, C], [0, T]],   C_kj = <v_lam,k | H_k* | v_psi,j>.
// k_frechet_c forms C (partials per block, fixed-order reduction after), and
// k_frechet_small exponentiates M against one unit vector by a Taylor series
// with substeps and accumulates g into dz/du.
#include <hip/hip_runtime.h>

#include "cfet_internal.h"
#include <algorithm>

namespace cfet {

namespace {

constexpr int kCRows = 16;      // rows per tile of k_frechet_c
constexpr int kCBlock = 256;
constexpr int kSmallThreads = 128;
constexpr int kSmallC = 32;  // C held in LDS by k_frechet_small up to 32 x 32

__device__ __forceinline__ const double2* basis_vec(const double2* w0, const double2* rest,
                                                    int64_t n, int j) {
  return (j == 0) ? w0 : rest + (int64_t)(j - 1) * n;
}

// Partial C_kj (raw: stored vectors, no inv scaling) over the rows of this
// block's tiles, for the ml x mp pairs in use (pair = k * mp + j).
// part: [gridDim.x][kMaxM * kMaxM] complex.
constexpr int kCPairsPerThread = (kMaxM * kMaxM + kCBlock - 1) / kCBlock;

__global__ __launch_bounds__(kCBlock) void k_frechet_c(
    const int64_t* __restrict__ rowptr, const uint32_t* __restrict__ colt,
    const double2* __restrict__ val, int64_t n, int term, const double2* __restrict__ psi0,
    const double2* __restrict__ psi_rest, const double2* __restrict__ lam0,
    const double2* __restrict__ lam_rest, const LzScalars* __restrict__ Spsi,
    const LzScalars* __restrict__ Slam, double2* __restrict__ part) {
  __shared__ double2 Y[kCRows][kMaxM];
  __shared__ double2 U[kCRows][kMaxM];
  const int mp = Spsi->m_eff, ml = Slam->m_eff;
  const int mx = max(mp, ml);
  const int npairs = ml * mp;
  double2 acc[kCPairsPerThread];
#pragma unroll
  for (int q = 0; q < kCPairsPerThread; ++q) acc[q] = make_double2(0, 0);
  const int64_t ntiles = (n + kCRows - 1) / kCRows;
  for (int64_t tile = blockIdx.x; tile < ntiles && mx > 0; tile += gridDim.x) {
    const int64_t r0 = tile * kCRows;
    __syncthreads();
    for (int t = threadIdx.x; t < kCRows * mx; t += blockDim.x) {
      const int rl = t / mx, j = t % mx;
      const int64_t r = r0 + rl;
      double2 y = make_double2(0.0, 0.0), u = make_double2(0.0, 0.0);
      if (r < n) {
        if (j < mp) {
          const double2* x = basis_vec(psi0, psi_rest, n, j);
          for (int64_t e = rowptr[r]; e < rowptr[r + 1]; ++e) {
            const uint32_t ct = colt[e];
            if ((int)(ct >> kTermShift) != term) continue;
            const double2 v = val[e];
            const double2 xv = x[ct & kColMask];
            y.x += v.x * xv.x - v.y * xv.y;
            y.y += v.x * xv.y + v.y * xv.x;
          }
        }
        if (j < ml) u = basis_vec(lam0, lam_rest, n, j)[r];
      }
      Y[rl][j] = y;
      U[rl][j] = u;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kCPairsPerThread; ++q) {
      const int pair = threadIdx.x + q * kCBlock;
      if (pair < npairs) {
        const int k = pair / mp, j = pair % mp;
        double2 a = acc[q];
        for (int rl = 0; rl < kCRows; ++rl) {
          const double2 uu = U[rl][k], yy = Y[rl][j];
          // conj(u) * y
          a.x += uu.x * yy.x + uu.y * yy.y;
          a.y += uu.x * yy.y - uu.y * yy.x;
        }
        acc[q] = a;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < kCPairsPerThread; ++q) {
    const int pair = threadIdx.x + q * kCBlock;
    if (pair < npairs) part[(int64_t)blockIdx.x * kMaxM * kMaxM + pair] = acc[q];
  }
}

// C[k][j] = inv_lam[k] inv_psi[j] * sum over blocks of the partials (fixed
// order; one thread per pair, consecutive pairs read consecutive partials).
__global__ __launch_bounds__(256) void k_frechet_c_reduce(const double2* __restrict__ part,
                                                          int nb, const LzScalars* Spsi,
                                                          const LzScalars* Slam,
                                                          double2* __restrict__ C) {
  const int pair = blockIdx.x * blockDim.x + threadIdx.x;
  const int mp = Spsi->m_eff, ml = Slam->m_eff;
  if (pair >= kMaxM * kMaxM) return;
  double sr = 0.0, si = 0.0;
  int k = pair / kMaxM, j = pair % kMaxM;  // pairs past the used ones clear C
  if (pair < ml * mp) {
    k = pair / mp;
    j = pair % mp;
    for (int b = 0; b < nb; ++b) {
      const double2 v = part[(int64_t)b * kMaxM * kMaxM + pair];
      sr += v.x;
      si += v.y;
    }
    const double sc = Slam->inv_nrm[k] * Spsi->inv_nrm[j];
    sr *= sc;
    si *= sc;
    C[k * kMaxM + j] = make_double2(sr, si);
  }
}

// g = beta_lam beta_psi [exp(M) e_{ml}]_0,  M = -i dt [[S, C], [0, T]] of order
// ml + mp, by v <- exp(M / q) v repeated q times (Taylor series of each factor
// summed until the terms are below 1e-18 of the sum), then dz[p] += w * g for
// the (piece, weight) pairs of this exponential.
__global__ __launch_bounds__(kSmallThreads) void k_frechet_small(
    const LzScalars* __restrict__ Spsi, const LzScalars* __restrict__ Slam,
    const double2* __restrict__ C, double dt, int npairs, int p0, double w0, int p1, double w1,
    int p2, double w2, int p3, double w3, double2* __restrict__ dz, DevStats* stats,
    const GradRec* __restrict__ rec) {
  __shared__ double2 v[2 * kMaxM], term[2 * kMaxM];
  __shared__ double2 Cs[kSmallC][kSmallC];  // C when ml, mp <= kSmallC
  __shared__ double red[2];
  __shared__ int again;
  const int ml = Slam->m_eff, mp = Spsi->m_eff;
  const int nm = ml + mp;
  const int r = threadIdx.x;
  if (ml == 0 || mp == 0) return;  // a zero state: no contribution
  const bool lds_c = ml <= kSmallC && mp <= kSmallC;
  if (lds_c) {
    for (int t = r; t < ml * mp; t += blockDim.x) Cs[t / mp][t % mp] = C[(t / mp) * kMaxM + t % mp];
    __syncthreads();
  }
  // row r of M: coefficients (times -i dt) and the infinity norm
  double rowsum = 0.0;
  if (r < ml) {
    rowsum = fabs(Slam->alpha[r]) + (r > 0 ? Slam->beta[r - 1] : 0.0) +
             (r + 1 < ml ? Slam->beta[r] : 0.0);
    for (int j = 0; j < mp; ++j) rowsum += hypot(C[r * kMaxM + j].x, C[r * kMaxM + j].y);
  } else if (r < nm) {
    const int q = r - ml;
    rowsum = fabs(Spsi->alpha[q]) + (q > 0 ? Spsi->beta[q - 1] : 0.0) +
             (q + 1 < mp ? Spsi->beta[q] : 0.0);
  }
  rowsum *= fabs(dt);
  // block maximum of rowsum
  double mx = rowsum;
  for (int off = 32; off >= 1; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
  if ((r & 63) == 0) red[r >> 6] = mx;
  __syncthreads();
  const double nrm = fmax(red[0], red[1]);
  const int nsub = max(1, (int)ceil(2.0 * nrm));
  const double h = dt / nsub;
  if (r < 2 * kMaxM) v[r] = make_double2(r == ml ? 1.0 : 0.0, 0.0);
  __syncthreads();
  for (int sub = 0; sub < nsub; ++sub) {
    if (r < 2 * kMaxM) term[r] = v[r];
    __syncthreads();
    for (int kk = 1; kk < 60; ++kk) {
      // nxt = (M/nsub) term / kk, M x = -i h (K x) with K = [[S, C], [0, T]]
      double2 kx = make_double2(0.0, 0.0);
      if (r < ml) {
        double ar = Slam->alpha[r] * term[r].x, ai = Slam->alpha[r] * term[r].y;
        if (r > 0) { ar += Slam->beta[r - 1] * term[r - 1].x; ai += Slam->beta[r - 1] * term[r - 1].y; }
        if (r + 1 < ml) { ar += Slam->beta[r] * term[r + 1].x; ai += Slam->beta[r] * term[r + 1].y; }
        for (int j = 0; j < mp; ++j) {
          const double2 c = lds_c ? Cs[r][j] : C[r * kMaxM + j], x = term[ml + j];
          ar += c.x * x.x - c.y * x.y;
          ai += c.x * x.y + c.y * x.x;
        }
        kx = make_double2(ar, ai);
      } else if (r < nm) {
        const int q = r - ml;
        double ar = Spsi->alpha[q] * term[r].x, ai = Spsi->alpha[q] * term[r].y;
        if (q > 0) { ar += Spsi->beta[q - 1] * term[r - 1].x; ai += Spsi->beta[q - 1] * term[r - 1].y; }
        if (q + 1 < mp) { ar += Spsi->beta[q] * term[r + 1].x; ai += Spsi->beta[q] * term[r + 1].y; }
        kx = make_double2(ar, ai);
      }
      // -i h kx / kk
      const double2 nt = make_double2(h * kx.y / kk, -h * kx.x / kk);
      __syncthreads();
      if (r < nm) {
        v[r].x += nt.x;
        v[r].y += nt.y;
      }
      if (r == 0) again = 0;
      __syncthreads();
      if (r < nm) {
        const double tn = fabs(nt.x) + fabs(nt.y);
        const double vn = fabs(v[r].x) + fabs(v[r].y);
        if (tn > 1e-18 * (vn + 1e-300)) again = 1;
        term[r] = nt;
      }
      __syncthreads();
      if (!again) break;
    }
    __syncthreads();
  }
  if (r == 0) {
    const double bb = Slam->beta0 * Spsi->beta0;
    const double2 g = make_double2(bb * v[0].x, bb * v[0].y);
    int ps[4] = {p0, p1, p2, p3};
    double ws[4] = {w0, w1, w2, w3};
    if (rec) {  // pairs from device memory (replayed graphs)
      npairs = rec->np;
      for (int q = 0; q < 4; ++q) {
        ps[q] = rec->p[q];
        ws[q] = rec->w[q];
      }
    }
    for (int q = 0; q < npairs; ++q) {
      dz[ps[q]].x += ws[q] * g.x;
      dz[ps[q]].y += ws[q] * g.y;
    }
    if (!(isfinite(g.x) && isfinite(g.y)) && stats->status == CFET_OK)
      stats->status = CFET_ENONFINITE;
  }
}

// conj(a) . b partial sums per block (complex).
__global__ __launch_bounds__(256) void k_zdot(const double2* __restrict__ a,
                                              const double2* __restrict__ b, int64_t n,
                                              double2* __restrict__ part) {
  __shared__ double rr[256], ri[256];
  double sr = 0.0, si = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double2 x = a[i], y = b[i];
    sr += x.x * y.x + x.y * y.y;
    si += x.x * y.y - x.y * y.x;
  }
  rr[threadIdx.x] = sr;
  ri[threadIdx.x] = si;
  __syncthreads();
  for (int s = 128; s >= 1; s >>= 1) {
    if (threadIdx.x < s) {
      rr[threadIdx.x] += rr[threadIdx.x + s];
      ri[threadIdx.x] += ri[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = make_double2(rr[0], ri[0]);
}

__global__ void k_zdot_reduce(const double2* __restrict__ part, int nb, double2* out) {
  if (threadIdx.x != 0) return;
  double sr = 0.0, si = 0.0;
  for (int b = 0; b < nb; ++b) {
    sr += part[b].x;
    si += part[b].y;
  }
  *out = make_double2(sr, si);
}

// Start of one replayed backward exponential: take record *cursor and the
// state before that exponential into fixed buffers.
__global__ __launch_bounds__(256) void k_grad_prologue(const GradRec* __restrict__ recs,
                                                       const int* __restrict__ cursor,
                                                       GradRec* __restrict__ cur,
                                                       const double2* __restrict__ before,
                                                       int64_t n, double2* __restrict__ pb,
                                                       const double2* __restrict__ lam,
                                                       double2* __restrict__ lam_copy) {
  const int idx = *cursor;
  if (blockIdx.x == 0 && threadIdx.x == 0) *cur = recs[idx];
  const double2* __restrict__ src = before + (int64_t)idx * n;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    pb[i] = src[i];
    if (lam_copy) lam_copy[i] = lam[i];
  }
}

__global__ void k_grad_epilogue(int* cursor) {
  if (threadIdx.x == 0) *cursor -= 1;
}

__global__ void k_zero2(double2* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = make_double2(0.0, 0.0);
}

}  // namespace

int frechet_c_blocks(int64_t n) {
  const int64_t tiles = (n + kCRows - 1) / kCRows;
  return (int)std::max<int64_t>(1, std::min<int64_t>(tiles, 128));
}

hipError_t launch_frechet_c(const DevCSR& A, int term, const double2* psi0,
                            const double2* psi_rest, const double2* lam0, const double2* lam_rest,
                            const LzScalars* Spsi, const LzScalars* Slam, double2* part,
                            double2* C, hipStream_t st) {
  const int nb = frechet_c_blocks(A.n);
  hipLaunchKernelGGL(k_frechet_c, dim3(nb), dim3(kCBlock), 0, st, A.rowptr, A.colt, A.val, A.n,
                     term, psi0, psi_rest, lam0, lam_rest, Spsi, Slam, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_frechet_c_reduce, dim3((kMaxM * kMaxM + 255) / 256), dim3(256), 0, st,
                     part, nb, Spsi, Slam, C);
  return hipGetLastError();
}

hipError_t launch_frechet_small(const LzScalars* Spsi, const LzScalars* Slam, const double2* C,
                                double dt, int npairs, const int* p, const double* w,
                                double2* dz, DevStats* stats, hipStream_t st) {
  hipLaunchKernelGGL(k_frechet_small, dim3(1), dim3(kSmallThreads), 0, st, Spsi, Slam, C, dt,
                     npairs, p[0], w[0], p[1], w[1], p[2], w[2], p[3], w[3], dz, stats,
                     (const GradRec*)nullptr);
  return hipGetLastError();
}

hipError_t launch_frechet_small_rec(const LzScalars* Spsi, const LzScalars* Slam,
                                    const double2* C, double dt, const GradRec* cur,
                                    double2* dz, DevStats* stats, hipStream_t st) {
  hipLaunchKernelGGL(k_frechet_small, dim3(1), dim3(kSmallThreads), 0, st, Spsi, Slam, C, dt, 0,
                     0, 0.0, 0, 0.0, 0, 0.0, 0, 0.0, dz, stats, cur);
  return hipGetLastError();
}

hipError_t launch_grad_prologue(const GradRec* recs, const int* cursor, GradRec* cur,
                                const double2* before, int64_t n, double2* pb,
                                const double2* lam, double2* lam_copy, hipStream_t st) {
  const int nb = (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 1024));
  hipLaunchKernelGGL(k_grad_prologue, dim3(nb), dim3(256), 0, st, recs, cursor, cur, before, n,
                     pb, lam, lam_copy);
  return hipGetLastError();
}

hipError_t launch_grad_epilogue(int* cursor, hipStream_t st) {
  hipLaunchKernelGGL(k_grad_epilogue, dim3(1), dim3(64), 0, st, cursor);
  return hipGetLastError();
}

int zdot_blocks(int64_t n) {
  return (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 1024));
}

hipError_t launch_zdot(const double2* a, const double2* b, int64_t n, double2* part,
                       double2* out, hipStream_t st) {
  const int nb = zdot_blocks(n);
  hipLaunchKernelGGL(k_zdot, dim3(nb), dim3(256), 0, st, a, b, n, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_zdot_reduce, dim3(1), dim3(64), 0, st, part, nb, out);
  return hipGetLastError();
}

hipError_t launch_zero2(double2* p, int n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero2, dim3((n + 255) / 256), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

}  // namespace cfet
