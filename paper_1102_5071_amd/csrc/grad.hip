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
// k_frechet_c forms C from the operator (partials per block, fixed-order
// reduction after); k_frechet_dots forms it from Y_j = H_k* w_psi,j when the
// recurrence from psi has stored those; k_frechet_small (one wavefront:
// k_frechet_small_wave, for m <= 32) exponentiates M against one unit vector
// by a Taylor series with substeps and accumulates g into dz/du.
#include <hip/hip_runtime.h>

#include "cfet_internal.h"
#include <algorithm>

namespace cfet {

namespace {

constexpr int kCRows = 16;      // rows per tile of k_frechet_c
constexpr int kCBlock = 256;
constexpr int kSmallThreads = 128;
constexpr int kSmallC = 32;  // k_frechet_small keeps a row of C in registers up to 32 wide

__device__ __forceinline__ const double2* basis_vec(const double2* w0, const double2* rest,
                                                    int64_t n, int j) {
  return (j == 0) ? w0 : rest + (int64_t)(j - 1) * n;
}

// Partial C_kj (raw: stored vectors, no inv scaling) over the rows of this
// block's tiles, for the ml x mp pairs in use (pair = k * mp + j).
// part: [gridDim.x][ml * mp] complex.
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
    if (pair < npairs) part[(int64_t)blockIdx.x * npairs + pair] = acc[q];
  }
}

// The same partials from stored vectors: Y_j = H_k* w_psi,j (j < mp, at
// Y + j n) and the lambda basis.  Each block takes one contiguous range of
// rows in tiles of kDRows staged in LDS.
constexpr int kDRows = 32;

__global__ __launch_bounds__(kCBlock) void k_frechet_dots(
    int64_t n, const double2* __restrict__ lam0, const double2* __restrict__ lam_rest,
    const double2* __restrict__ Y, const LzScalars* __restrict__ Spsi,
    const LzScalars* __restrict__ Slam, double2* __restrict__ part) {
  __shared__ double2 Ys[kDRows][kMaxM];
  __shared__ double2 Us[kDRows][kMaxM];
  const int mp = Spsi->m_eff, ml = Slam->m_eff;
  const int mx = max(mp, ml);
  const int npairs = ml * mp;
  double2 acc[kCPairsPerThread];
#pragma unroll
  for (int q = 0; q < kCPairsPerThread; ++q) acc[q] = make_double2(0, 0);
  const int64_t ntiles = (n + kDRows - 1) / kDRows;
  const int64_t per = (ntiles + gridDim.x - 1) / gridDim.x;
  const int64_t t0 = (int64_t)blockIdx.x * per, t1 = min(ntiles, t0 + per);
  for (int64_t tile = t0; tile < t1 && mx > 0; ++tile) {
    const int64_t r0 = tile * kDRows;
    __syncthreads();
    // consecutive threads take consecutive rows of one vector
    for (int t = threadIdx.x; t < kDRows * mx; t += blockDim.x) {
      const int j = t / kDRows, rl = t % kDRows;
      const int64_t r = r0 + rl;
      double2 y = make_double2(0.0, 0.0), u = make_double2(0.0, 0.0);
      if (r < n) {
        if (j < mp) y = Y[(int64_t)j * n + r];
        if (j < ml) u = basis_vec(lam0, lam_rest, n, j)[r];
      }
      Ys[rl][j] = y;
      Us[rl][j] = u;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kCPairsPerThread; ++q) {
      const int pair = threadIdx.x + q * kCBlock;
      if (pair < npairs) {
        const int k = pair / mp, j = pair % mp;
        double2 a = acc[q];
        for (int rl = 0; rl < kDRows; ++rl) {
          const double2 uu = Us[rl][k], yy = Ys[rl][j];
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
    if (pair < npairs) part[(int64_t)blockIdx.x * npairs + pair] = acc[q];
  }
}

// C[k][j] = inv_lam[k] inv_psi[j] * sum over blocks of the partials, one
// wavefront per pair: lane l adds blocks l, l + 64, ... in order, then a fixed
// butterfly over the lanes (the same order on every run).
__global__ __launch_bounds__(256) void k_frechet_c_reduce(const double2* __restrict__ part,
                                                          int nb, const LzScalars* Spsi,
                                                          const LzScalars* Slam,
                                                          double2* __restrict__ C) {
  const int mp = Spsi->m_eff, ml = Slam->m_eff;
  const int npairs = ml * mp;
  const int pair = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  const int l = threadIdx.x & 63;
  if (pair >= npairs) return;  // whole wavefronts leave together
  double sr = 0.0, si = 0.0;
  for (int b = l; b < nb; b += 64) {
    const double2 v = part[(int64_t)b * npairs + pair];
    sr += v.x;
    si += v.y;
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    sr += __shfl_xor(sr, off, 64);
    si += __shfl_xor(si, off, 64);
  }
  if (l == 0) {
    const int k = pair / mp, j = pair % mp;
    const double sc = Slam->inv_nrm[k] * Spsi->inv_nrm[j];
    C[k * kMaxM + j] = make_double2(sr * sc, si * sc);
  }
}

// g = beta_lam beta_psi [exp(M) e_{ml}]_0,  M = -i dt [[S, C], [0, T]] of order
// ml + mp, by v <- exp(M / q) v repeated q times (Taylor series of each factor
// summed until the terms are below 1e-18 of the sum), then dz[p] += w * g for
// the (piece, weight) pairs of this exponential.
__global__ __launch_bounds__(kSmallThreads) void k_frechet_small(
    const LzScalars* __restrict__ Spsi, const LzScalars* __restrict__ Slam,
    const double2* __restrict__ C, double dt, double2* __restrict__ dz, DevStats* stats,
    const GradRec* __restrict__ rec, int* cursor) {
  __shared__ double2 tb[2][2 * kMaxM];
  __shared__ double red[2];
  const int ml = Slam->m_eff, mp = Spsi->m_eff;
  const int nm = ml + mp;
  const int r = threadIdx.x;
  // the record of this exponential was taken by the prologue: step the cursor
  // to the one before it (also for a zero state)
  if (cursor && r == 0) *cursor -= 1;
  if (ml == 0 || mp == 0) return;  // a zero state: no contribution
  // row r of C in registers when mp <= kSmallC (the Taylor loop then reads
  // only the term vector from LDS)
  const bool reg_c = mp <= kSmallC;
  double2 creg[kSmallC];
#pragma unroll
  for (int j = 0; j < kSmallC; ++j)
    creg[j] = (reg_c && r < ml && j < mp) ? C[r * kMaxM + j] : make_double2(0.0, 0.0);
  // row r of K = [[S, C], [0, T]]: tridiagonal part in registers (read once),
  // and the infinity norm
  double ad = 0.0, bl = 0.0, bu = 0.0;
  bool hasl = false, hasu = false;
  if (r < ml) {
    ad = Slam->alpha[r];
    hasl = r > 0;
    hasu = r + 1 < ml;
    if (hasl) bl = Slam->beta[r - 1];
    if (hasu) bu = Slam->beta[r];
  } else if (r < nm) {
    const int q = r - ml;
    ad = Spsi->alpha[q];
    hasl = q > 0;
    hasu = q + 1 < mp;
    if (hasl) bl = Spsi->beta[q - 1];
    if (hasu) bu = Spsi->beta[q];
  }
  double rowsum = fabs(ad) + bl + bu;
  if (r < ml && reg_c) {
#pragma unroll
    for (int j = 0; j < kSmallC; ++j) rowsum += hypot(creg[j].x, creg[j].y);  // zero past mp
  } else if (r < ml) {
    for (int j = 0; j < mp; ++j) rowsum += hypot(C[r * kMaxM + j].x, C[r * kMaxM + j].y);
  }
  rowsum *= fabs(dt);
  // block maximum of rowsum
  double mx = rowsum;
  for (int off = 32; off >= 1; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
  if ((r & 63) == 0) red[r >> 6] = mx;
  __syncthreads();
  const double nrm = fmax(red[0], red[1]);
  // substeps of infinity norm nu <= 1: term k is then bounded by nu^k / k!
  // times the substep's start (no cancellation), and the series stops after
  // the K-th term with nu^(K+1) / (K+1)! <= 1e-18
  const int nsub = max(1, (int)ceil(nrm));
  const double h = dt / nsub;
  const double nu = nrm / nsub;
  int nterms = 1;
  for (double nxt = 0.5 * nu * nu; nterms < 59 && nxt > 1e-18; nxt *= nu / (nterms + 1)) ++nterms;
  // thread r < nm owns entry r of v; the Taylor terms alternate between two
  // LDS buffers, so one barrier per term publishes the new term
  double2 vr = make_double2(r == ml ? 1.0 : 0.0, 0.0);
  for (int sub = 0; sub < nsub; ++sub) {
    if (r < nm) tb[0][r] = vr;
    __syncthreads();
    int cur = 0;
    for (int kk = 1; kk <= nterms; ++kk) {
      // next term = (-i h / kk) K term, K = [[S, C], [0, T]]
      const double2* __restrict__ t = tb[cur];
      if (r < nm) {
        double ar = ad * t[r].x, ai = ad * t[r].y;
        if (hasl) { ar += bl * t[r - 1].x; ai += bl * t[r - 1].y; }
        if (hasu) { ar += bu * t[r + 1].x; ai += bu * t[r + 1].y; }
        if (r < ml && reg_c) {
          double er = 0.0, ei = 0.0, orr = 0.0, oi = 0.0;  // even / odd j
#pragma unroll
          for (int j = 0; j < kSmallC; j += 2) {
            if (j < mp) {
              const double2 c = creg[j], x = t[ml + j];
              er += c.x * x.x - c.y * x.y;
              ei += c.x * x.y + c.y * x.x;
            }
            if (j + 1 < mp) {
              const double2 c = creg[j + 1], x = t[ml + j + 1];
              orr += c.x * x.x - c.y * x.y;
              oi += c.x * x.y + c.y * x.x;
            }
          }
          ar += er + orr;
          ai += ei + oi;
        } else if (r < ml) {
          for (int j = 0; j < mp; ++j) {
            const double2 c = C[r * kMaxM + j], x = t[ml + j];
            ar += c.x * x.x - c.y * x.y;
            ai += c.x * x.y + c.y * x.x;
          }
        }
        const double hk = h / kk;
        const double2 nt = make_double2(hk * ai, -hk * ar);
        vr.x += nt.x;
        vr.y += nt.y;
        tb[cur ^ 1][r] = nt;
      }
      __syncthreads();
      cur ^= 1;
    }
    __syncthreads();
  }
  if (r == 0) {
    const double bb = Slam->beta0 * Spsi->beta0;
    const double2 g = make_double2(bb * vr.x, bb * vr.y);
    // (piece, weight) pairs of this exponential from its record
    const int npairs = rec->np;
    for (int q = 0; q < npairs; ++q) {
      dz[rec->p[q]].x += rec->w[q] * g.x;
      dz[rec->p[q]].y += rec->w[q] * g.y;
    }
    if (!(isfinite(g.x) && isfinite(g.y)) && stats->status == CFET_OK)
      stats->status = CFET_ENONFINITE;
  }
}

// The same on one wavefront, for m_lam + m_psi <= 64 and m_psi <= kSmallC:
// entry r of the term in lane r, neighbours by DPP lane shifts, the term
// published in LDS for the C product after a wavefront barrier, and the
// same term count from the norm bound (|Re| + |Im| bounds each modulus in
// the norm here).  A count fixed in advance, rather than a test of each
// entry's last term, matters: entries far down the tridiagonal blocks only
// begin to move after as many terms as their distance from the start.
__device__ __forceinline__ double lane_below(double v) {  // lane r receives lane r-1 (0 in lane 0)
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x138, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x138, 0xf, 0xf, true);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double lane_above(double v) {  // lane r receives lane r+1 (0 in lane 63)
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x130, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x130, 0xf, 0xf, true);
  return __hiloint2double(hi, lo);
}

__global__ __launch_bounds__(64) void k_frechet_small_wave(
    const LzScalars* __restrict__ Spsi, const LzScalars* __restrict__ Slam,
    const double2* __restrict__ C, double dt, double2* __restrict__ dz, DevStats* stats,
    const GradRec* __restrict__ rec, int* cursor) {
  __shared__ double2 tw[64];
  const int ml = Slam->m_eff, mp = Spsi->m_eff;
  const int nm = ml + mp;
  const int r = threadIdx.x;
  if (cursor && r == 0) *cursor -= 1;
  if (ml == 0 || mp == 0) return;  // a zero state: no contribution
  double2 creg[kSmallC];
#pragma unroll
  for (int j = 0; j < kSmallC; ++j)
    creg[j] = (r < ml && j < mp) ? C[r * kMaxM + j] : make_double2(0.0, 0.0);
  double ad = 0.0, bl = 0.0, bu = 0.0;
  if (r < ml) {
    ad = Slam->alpha[r];
    if (r > 0) bl = Slam->beta[r - 1];
    if (r + 1 < ml) bu = Slam->beta[r];
  } else if (r < nm) {
    const int q = r - ml;
    ad = Spsi->alpha[q];
    if (q > 0) bl = Spsi->beta[q - 1];
    if (q + 1 < mp) bu = Spsi->beta[q];
  }
  double rowsum = fabs(ad) + bl + bu;
  if (r < ml) {
#pragma unroll
    for (int j = 0; j < kSmallC; ++j) rowsum += fabs(creg[j].x) + fabs(creg[j].y);  // zero past mp
  }
  rowsum *= fabs(dt);
  double nrm = rowsum;
  for (int off = 32; off >= 1; off >>= 1) nrm = fmax(nrm, __shfl_xor(nrm, off, 64));
  const int nsub = __builtin_amdgcn_readfirstlane(max(1, (int)ceil(nrm)));
  const double h = dt / nsub;
  const double nu = nrm / nsub;
  int nterms = 1;
  for (double nxt = 0.5 * nu * nu; nterms < 59 && nxt > 1e-18; nxt *= nu / (nterms + 1)) ++nterms;
  nterms = __builtin_amdgcn_readfirstlane(nterms);
  double2 vr = make_double2(r == ml ? 1.0 : 0.0, 0.0);
  for (int sub = 0; sub < nsub; ++sub) {
    double2 t = vr;
    for (int kk = 1; kk <= nterms; ++kk) {
      // publish the term for the C product (the previous term's reads are
      // complete: their values fed the term written here)
      tw[r] = t;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      const double tlx = lane_below(t.x), tly = lane_below(t.y);
      const double tux = lane_above(t.x), tuy = lane_above(t.y);
      double ar = ad * t.x, ai = ad * t.y;
      ar += bl * tlx;
      ai += bl * tly;
      ar += bu * tux;
      ai += bu * tuy;
      if (r < ml) {
        double er = 0.0, ei = 0.0, orr = 0.0, oi = 0.0;  // even / odd j
#pragma unroll
        for (int j = 0; j < kSmallC; j += 2) {
          if (j < mp) {
            const double2 c = creg[j], x = tw[ml + j];
            er += c.x * x.x - c.y * x.y;
            ei += c.x * x.y + c.y * x.x;
          }
          if (j + 1 < mp) {
            const double2 c = creg[j + 1], x = tw[ml + j + 1];
            orr += c.x * x.x - c.y * x.y;
            oi += c.x * x.y + c.y * x.x;
          }
        }
        ar += er + orr;
        ai += ei + oi;
      }
      const double hk = h / kk;
      const double2 nt = (r < nm) ? make_double2(hk * ai, -hk * ar) : make_double2(0.0, 0.0);
      vr.x += nt.x;
      vr.y += nt.y;
      t = nt;
    }
  }
  if (r == 0) {
    const double bb = Slam->beta0 * Spsi->beta0;
    const double2 g = make_double2(bb * vr.x, bb * vr.y);
    const int npairs = rec->np;
    for (int q = 0; q < npairs; ++q) {
      dz[rec->p[q]].x += rec->w[q] * g.x;
      dz[rec->p[q]].y += rec->w[q] * g.y;
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
                                                       double2* __restrict__ lam_copy,
                                                       unsigned long long* __restrict__ bar,
                                                       int bar_words, int* __restrict__ fault) {
  // cursor == nullptr: only the lambda copy and the barrier state
  const int idx = cursor ? *cursor : 0;
  if (cursor && blockIdx.x == 0 && threadIdx.x == 0) *cur = recs[idx];
  // barrier state of the persistent launches that follow (they skip their own reset)
  if (bar && blockIdx.x == 0) {
    for (int i = threadIdx.x; i < bar_words; i += blockDim.x) bar[i] = 0ull;
    if (threadIdx.x == 0) *fault = 0;
  }
  const double2* __restrict__ src = cursor ? before + (int64_t)idx * n : nullptr;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (src) pb[i] = src[i];
    if (lam_copy) lam_copy[i] = lam[i];
  }
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

static int frechet_dots_blocks(int64_t n) {
  const int64_t tiles = (n + kDRows - 1) / kDRows;
  return (int)std::max<int64_t>(1, std::min<int64_t>(tiles, 256));
}

int frechet_part_blocks(int64_t n) {
  return std::max(frechet_c_blocks(n), frechet_dots_blocks(n));
}

static hipError_t launch_c_reduce(const double2* part, int nb, const LzScalars* Spsi,
                                  const LzScalars* Slam, double2* C, hipStream_t st) {
  // one wavefront per pair in use (at most kMaxM^2; the kernel reads m_eff)
  hipLaunchKernelGGL(k_frechet_c_reduce, dim3((kMaxM * kMaxM + 3) / 4), dim3(256), 0, st, part,
                     nb, Spsi, Slam, C);
  return hipGetLastError();
}

hipError_t launch_frechet_dots(int64_t n, const double2* lam0, const double2* lam_rest,
                               const double2* Y, const LzScalars* Spsi, const LzScalars* Slam,
                               double2* part, double2* C, hipStream_t st) {
  const int nb = frechet_dots_blocks(n);
  hipLaunchKernelGGL(k_frechet_dots, dim3(nb), dim3(kCBlock), 0, st, n, lam0, lam_rest, Y, Spsi,
                     Slam, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_c_reduce(part, nb, Spsi, Slam, C, st);
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
  return launch_c_reduce(part, nb, Spsi, Slam, C, st);
}

hipError_t launch_frechet_small_rec(const LzScalars* Spsi, const LzScalars* Slam,
                                    const double2* C, double dt, const GradRec* cur,
                                    double2* dz, DevStats* stats, int* cursor, int mmax,
                                    hipStream_t st) {
  if (!cur) return hipErrorInvalidValue;
  if (mmax >= 1 && mmax <= kSmallC && 2 * mmax <= 64) {
    hipLaunchKernelGGL(k_frechet_small_wave, dim3(1), dim3(64), 0, st, Spsi, Slam, C, dt, dz,
                       stats, cur, cursor);
  } else {
    hipLaunchKernelGGL(k_frechet_small, dim3(1), dim3(kSmallThreads), 0, st, Spsi, Slam, C, dt,
                       dz, stats, cur, cursor);
  }
  return hipGetLastError();
}

hipError_t launch_grad_prologue(const GradRec* recs, const int* cursor, GradRec* cur,
                                const double2* before, int64_t n, double2* pb,
                                const double2* lam, double2* lam_copy, unsigned long long* bar,
                                int bar_words, int* fault, hipStream_t st) {
  const int nb = (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 1024));
  hipLaunchKernelGGL(k_grad_prologue, dim3(nb), dim3(256), 0, st, recs, cursor, cur, before, n,
                     pb, lam, lam_copy, bar, bar_words, fault);
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
