// Persistent CFET propagation: one kernel launch runs every step, every
// exponential and every Lanczos iteration of a cfet_propagate call.
//
// Work split.  Block b owns a contiguous row range for the whole launch.  A
// group of G lanes works on one row; lane 0 of the group owns that row's
// Lanczos quantities.  At launch start every lane copies its share of the
// matrix rows it will ever touch (up to PMAX rows x QMAX entries) into
// registers, so after that the SpMV reads only the vector it multiplies
// (longer rows fall back to global loads for their tail).
//
// One Lanczos iteration (paper Sec. 8.1):
//     SpMV  y = H_w v_j in registers, partial Re<v_j, y>   -> reduce -> alpha_j
//     axpy  w_{j+1} = y - alpha_j v_j - beta_{j-1} v_{j-1} in registers,
//           store w_{j+1} (the next SpMV gathers it), partial ||w||^2
//                                                         -> reduce -> beta_j
// y is never stored.  A reduction across blocks is a block sum, a store of the
// partial, a grid barrier and a fixed-order re-sum of all partials by every
// block, so all blocks hold bit-identical alpha/beta, take identical
// decisions (early stop) and evaluate the small exponential exp(-i dt T) e_1
// themselves (one wave per block) without another barrier.
//
// Cross-block data -- the basis vectors, psi and the partial sums -- is
// written and read with device-scope (agent) accesses, which bypass the
// per-XCD L2s, so the barrier needs no cache write-back or invalidation: each
// wave waits for its own memory operations to complete, the block meets at
// __syncthreads, and thread 0 bumps a monotone 64-bit arrival counter and
// polls it.  Waiting is bounded by a wall-clock limit; a block that times out
// raises a fault flag, every block that sees the flag leaves the kernel, and
// the status is latched as CFET_EDEVICE.  The launch is cooperative, so all
// blocks are co-resident.
//
// SINGLE = true is the one-workgroup variant for small dimensions: the block
// barrier is the whole synchronisation, no partials, ordinary memory accesses.
#include <hip/hip_runtime.h>

#include "cfet_internal.h"
#include "tridiag.hpp"

namespace cfet {

namespace {

// Register-holding presets (G lanes per row, P rows per lane group, Q
// entries per lane and row).  A block of kPersistBlock threads holds
// P * kPersistBlock / G rows; rows longer than G*Q read their tail from memory.
struct Preset {
  int G, P, Q;
};
constexpr Preset kPresets[] = {{1, 2, 12}, {1, 1, 8}, {2, 2, 8}, {4, 1, 8}};
constexpr int kNumPresets = sizeof(kPresets) / sizeof(kPresets[0]);

__device__ __forceinline__ double p_wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Block sum; every thread receives the value thread 0 formed.
__device__ double p_block_sum(double v, double* red) {
  v = p_wave_sum(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int nw = blockDim.x >> 6;
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

// device-scope (agent) accesses of cross-block data
template <bool SINGLE>
__device__ __forceinline__ double2 vload(const double2* p) {
  if (SINGLE) return *p;
  const unsigned long long* q = reinterpret_cast<const unsigned long long*>(p);
  const unsigned long long a = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const unsigned long long b =
      __hip_atomic_load(q + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return make_double2(__longlong_as_double((long long)a), __longlong_as_double((long long)b));
}

template <bool SINGLE>
__device__ __forceinline__ void vstore(double2* p, double2 v) {
  if (SINGLE) {
    *p = v;
    return;
  }
  unsigned long long* q = reinterpret_cast<unsigned long long*>(p);
  __hip_atomic_store(q, (unsigned long long)__double_as_longlong(v.x), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(q + 1, (unsigned long long)__double_as_longlong(v.y), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ double dload(const double* p) {
  const unsigned long long v = __hip_atomic_load(reinterpret_cast<const unsigned long long*>(p),
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return __longlong_as_double((long long)v);
}

__device__ __forceinline__ void dstore(double* p, double v) {
  __hip_atomic_store(reinterpret_cast<unsigned long long*>(p),
                     (unsigned long long)__double_as_longlong(v), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}

__device__ bool grid_barrier(unsigned long long* bar, int* fault, unsigned long long& epoch,
                             long long limit, int* s_ok) {
  // all memory operations of this wave (device-scope stores included) are done
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    int ok = 1;
    epoch += 1ull;
    const unsigned long long target = epoch * (unsigned long long)gridDim.x;
    unsigned long long v =
        __hip_atomic_fetch_add(bar, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1ull;
    if (v < target) {
      const long long t0 = wall_clock64();
      for (;;) {
        v = __hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (v >= target) break;
        if (__hip_atomic_load(fault, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
          ok = 0;
          break;
        }
        if (wall_clock64() - t0 > limit) {
          __hip_atomic_store(fault, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          ok = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    }
    *s_ok = ok;
  }
  __syncthreads();
  return *s_ok != 0;
}

struct Shared {
  double cheb[kChebMaxTerms];
  double red[18];
  double alpha[kMaxM];
  double beta[kMaxM];
  double inv[kMaxM];
  double2 coef[kMaxM];
  double w[kMaxTerms + 1];
  int ok;
};

// u_k from the three stored vectors at one index: the Lanczos three-term
// recurrence written for unnormalised vectors,
//     u_k = (z_{k-1} - alpha_{k-1} u_{k-1}) / nu_{k-1} - (nu_{k-1} / nu_{k-2}) u_{k-2},
// with explicit fused multiply-adds so that every block forms bit-identical
// values for the same index.
__device__ __forceinline__ double2 form_u(double2 z, double2 u1, double2 u2, double c1, double c2,
                                          double c3) {
  double2 r;
  r.x = fma(c1, z.x, fma(-c2, u1.x, -c3 * u2.x));
  r.y = fma(c1, z.y, fma(-c2, u1.y, -c3 * u2.y));
  return r;
}

// Two block sums at once (every thread receives thread 0's values).
__device__ void p_block_sum2(double& a, double& b, double* red) {
  a = p_wave_sum(a);
  b = p_wave_sum(b);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int nw = blockDim.x >> 6;
  __syncthreads();
  if (l == 0) {
    red[w] = a;
    red[8 + w] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double ta = 0.0, tb = 0.0;
    for (int i = 0; i < nw; ++i) {
      ta += red[i];
      tb += red[8 + i];
    }
    red[16] = ta;
    red[17] = tb;
  }
  __syncthreads();
  a = red[16];
  b = red[17];
}

// Global sums of (a, b) over all threads of all blocks.  Returns false on a fault.
template <bool SINGLE>
__device__ __forceinline__ bool all_reduce2(double& a, double& b, const PersistArgs& A, Shared& sh,
                                            unsigned long long& epoch, int& pc) {
  p_block_sum2(a, b, sh.red);
  if (SINGLE) return true;
  double* P = A.part + (size_t)(pc & 1) * 2 * gridDim.x;
  if (threadIdx.x == 0) {
    dstore(P + 2 * blockIdx.x, a);
    dstore(P + 2 * blockIdx.x + 1, b);
  }
  if (!grid_barrier(A.bar, A.fault, epoch, A.spin_limit, &sh.ok)) return false;
  pc += 1;
  double sa = 0.0, sb = 0.0;
  for (int i = threadIdx.x; i < (int)gridDim.x; i += blockDim.x) {
    sa += dload(P + 2 * i);
    sb += dload(P + 2 * i + 1);
  }
  a = sa;
  b = sb;
  p_block_sum2(a, b, sh.red);
  return true;
}

template <int G, int PMAX, int QMAX, int NT, bool SINGLE>
__global__ __launch_bounds__(kPersistBlock) void k_propagate(PersistArgs A) {
  constexpr int BLOCK = kPersistBlock;
  __shared__ Shared sh;
  const int nb = gridDim.x;
  const int64_t n = A.n;
  const int64_t per = (n + nb - 1) / nb;
  const int64_t r0 = min(n, (int64_t)blockIdx.x * per);
  const int64_t r1 = min(n, r0 + per);
  const int nt1 = A.nterms + 1;
  const int lane = threadIdx.x % G;
  const int grp = threadIdx.x / G;
  constexpr int NGRP = BLOCK / G;
  unsigned long long epoch = 0;
  int pc = 0;
  bool ok = true;
  double2* __restrict__ psi = A.psi;
  // u_0 = psi, u_k (k >= 1) in the basis storage; z_k alternates between two buffers
  auto U = [&](int k) -> double2* {
    return (k == 0) ? psi : A.basis + (size_t)(k - 1) * (size_t)n;
  };
  auto Zb = [&](int k) -> double2* { return A.zbuf + (size_t)(k & 1) * (size_t)n; };

  // ---- the matrix entries this lane will use, kept in registers
  int64_t rowp[PMAX];
  int64_t tail_beg[PMAX], tail_end[PMAX];
  int cnt[PMAX];
  uint32_t ccol[PMAX][QMAX];
  double2 cval[PMAX][QMAX];
#pragma unroll
  for (int p = 0; p < PMAX; ++p) {
    const int64_t row = r0 + grp + (int64_t)p * NGRP;
    rowp[p] = (row < r1) ? row : -1;
    int64_t beg = 0, end = 0;
    if (row < r1) {
      beg = A.rowptr[row];
      end = A.rowptr[row + 1];
    }
#pragma unroll
    for (int q = 0; q < QMAX; ++q) {
      const int64_t e = beg + lane + (int64_t)q * G;
      if (e < end) {
        ccol[p][q] = A.colt[e];
        cval[p][q] = A.val[e];
      } else {
        ccol[p][q] = 0u;
        cval[p][q] = make_double2(0.0, 0.0);
      }
    }
    tail_beg[p] = beg + (int64_t)QMAX * G + lane;
    tail_end[p] = end;
    const int64_t len = end - beg;
    cnt[p] = (len > lane) ? (int)min<int64_t>(QMAX, (len - lane + G - 1) / G) : 0;
  }

  // own-row state (lane 0 of each group): u_{k-1}, u_{k-2}, z_{k-1}
  double2 u1[PMAX], u2[PMAX], zp[PMAX];
#pragma unroll
  for (int p = 0; p < PMAX; ++p) {
    u1[p] = u2[p] = zp[p] = make_double2(0.0, 0.0);
    if (lane == 0 && rowp[p] >= 0) u1[p] = vload<SINGLE>(psi + rowp[p]);  // becomes u_0
  }

  for (int64_t step = 0; ok && step < A.nsteps; ++step) {
    for (int i = A.s - 1; ok && i >= 0; --i) {
      if (threadIdx.x < nt1)
        sh.w[threadIdx.x] = A.wts[((size_t)step * A.s + i) * nt1 + threadIdx.x];
      __syncthreads();
      const double w0 = sh.w[0], w1 = (NT == 1) ? sh.w[1] : 0.0;
      const int m = A.m;
      int meff = m;
      bool zero = false;
      double nu0 = 0.0;
      // recurrence coefficients of the phase (uniform)
      double c1 = 0.0, c2 = 0.0, c3 = 0.0;
      for (int k = 0; k < m; ++k) {
        const double2* __restrict__ zprev = Zb(k + 1);   // z_{k-1}
        const double2* __restrict__ um1 = (k >= 1) ? U(k - 1) : psi;
        const double2* __restrict__ um2 = (k >= 2) ? U(k - 2) : psi;
        double2* __restrict__ uk = U(k);
        double2* __restrict__ zk = Zb(k);
        // ---- own rows: u_k (k >= 1; u_0 = psi is already stored)
        double s_uz = 0.0, s_uu = 0.0;
        double2 ucur[PMAX];
#pragma unroll
        for (int p = 0; p < PMAX; ++p) {
          ucur[p] = u1[p];
          if (k >= 1 && lane == 0 && rowp[p] >= 0) {
            ucur[p] = form_u(zp[p], u1[p], u2[p], c1, c2, (k >= 2) ? c3 : 0.0);
            vstore<SINGLE>(uk + rowp[p], ucur[p]);
          }
        }
        // ---- z_k = H_w u_k, u_k gathered (formed on the fly for k >= 1)
#pragma unroll
        for (int p = 0; p < PMAX; ++p) {
          double a0r = 0.0, a0i = 0.0, a1r = 0.0, a1i = 0.0;
          if (rowp[p] >= 0) {
#pragma unroll
            for (int q = 0; q < QMAX + 1; ++q) {
              // q < QMAX: register-held entries; q == QMAX: tail loop from memory
              const int64_t tb = (q == QMAX) ? tail_beg[p] : 0;
              const int64_t te = (q == QMAX) ? tail_end[p] : ((q < cnt[p]) ? 1 : 0);
              for (int64_t e = tb; e < te; e += G) {
                const uint32_t ct = (q == QMAX) ? A.colt[e] : ccol[p][q < QMAX ? q : 0];
                const double2 v = (q == QMAX) ? A.val[e] : cval[p][q < QMAX ? q : 0];
                const int64_t c = ct & kColMask;
                double2 xv = vload<SINGLE>(um1 + c);
                if (k >= 1) {
                  const double2 zc = vload<SINGLE>(zprev + c);
                  const double2 u2c = (k >= 2) ? vload<SINGLE>(um2 + c) : make_double2(0.0, 0.0);
                  xv = form_u(zc, xv, u2c, c1, c2, (k >= 2) ? c3 : 0.0);
                }
                const double pr = v.x * xv.x - v.y * xv.y;
                const double pi = v.x * xv.y + v.y * xv.x;
                if (NT == 1) {
                  if (ct >> kTermShift) { a1r += pr; a1i += pi; } else { a0r += pr; a0i += pi; }
                } else {
                  const double wt = sh.w[ct >> kTermShift];
                  a0r += wt * pr;
                  a0i += wt * pi;
                }
              }
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
          if (lane == 0 && rowp[p] >= 0) {
            const double2 zv = make_double2(yr, yi);
            if (k + 1 < m) vstore<SINGLE>(zk + rowp[p], zv);
            s_uz += ucur[p].x * zv.x + ucur[p].y * zv.y;
            s_uu += ucur[p].x * ucur[p].x + ucur[p].y * ucur[p].y;
            u2[p] = u1[p];
            u1[p] = ucur[p];
            zp[p] = zv;
          }
        }
        ok = all_reduce2<SINGLE>(s_uz, s_uu, A, sh, epoch, pc);
        if (!ok) break;
        const double nu = sqrt(s_uu);
        if (k == 0) {
          nu0 = nu;
          if (nu == 0.0) {  // psi == 0 stays 0
            zero = true;
            break;
          }
        } else {
          // beta_{k-1} = nu_k: the early-stop rule of the recurrence
          double sc = 0.0;
          for (int t = 0; t < k - 1; ++t) sc = fmax(sc, fabs(sh.alpha[t]) + sh.beta[t]);
          sc = fmax(sc, fabs(sh.alpha[k - 1]) + nu);
          __syncthreads();
          if (threadIdx.x == 0) sh.beta[k - 1] = nu;
          __syncthreads();
          if (nu <= kBreakdownRel * sc) {
            meff = k;
            break;
          }
        }
        const double inv = 1.0 / nu;
        const double alpha = s_uz * inv * inv;
        __syncthreads();
        if (threadIdx.x == 0) {
          sh.alpha[k] = alpha;
          sh.inv[k] = inv;
        }
        __syncthreads();
        // coefficients of u_{k+1} = (z_k - alpha_k u_k)/nu_k - (nu_k/nu_{k-1}) u_{k-1}
        c1 = inv;
        c2 = alpha * inv;
        c3 = (k >= 1) ? nu * sh.inv[k - 1] : 0.0;
      }
      if (!ok) break;
      if (zero) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
          A.stats->exponentials += 1;
          A.stats->breakdowns += 1;
          A.stats->min_m_eff = 0;
        }
        // u1 already holds psi = 0; restore the own-row state and go on
        continue;
      }
      __syncthreads();
      // ---- small exponential (wave 0; identical in every block)
      const double beta0 = nu0;
      if (threadIdx.x < 64) {
        const int l = threadIdx.x;
        const double a = (l < meff) ? sh.alpha[l] : 0.0;
        const double b = (l < meff - 1) ? sh.beta[l] : 0.0;
        double2 c = make_double2(0.0, 0.0);
        int status;
        const bool bad = !(isfinite(a) && isfinite(b) && isfinite(beta0));
        if (__ballot(bad) != 0ull) status = CFET_ENONFINITE;
        else status = tridiag_exp_e1(a, b, meff, A.dt, sh.cheb, c);
        if (l < meff) {
          const double scl = beta0 * sh.inv[l];
          sh.coef[l] = make_double2(c.x * scl, c.y * scl);
        }
        if (l == 0 && blockIdx.x == 0) {
          DevStats* st = A.stats;
          st->exponentials += 1;
          st->matvecs += (unsigned long long)meff;
          if (meff < st->min_m_eff) st->min_m_eff = meff;
          if (meff < m) st->breakdowns += 1;
          if (status != CFET_OK && st->status == CFET_OK) st->status = status;
          st->last_norm2 = beta0 * beta0;
        }
      }
      __syncthreads();
      // ---- recombination psi = sum_k coef_k u_k on own rows
      double dummy = 0.0, rp = 0.0;
#pragma unroll
      for (int p = 0; p < PMAX; ++p) {
        if (lane == 0 && rowp[p] >= 0) {
          double accr = 0.0, acci = 0.0;
          for (int kk = 0; kk < meff; ++kk) {
            const double2 v = vload<SINGLE>(U(kk) + rowp[p]);
            const double2 cf = sh.coef[kk];
            accr += cf.x * v.x - cf.y * v.y;
            acci += cf.x * v.y + cf.y * v.x;
          }
          const double2 nv = make_double2(accr, acci);
          vstore<SINGLE>(psi + rowp[p], nv);
          u1[p] = nv;
          rp += accr * accr + acci * acci;
        }
      }
      // the next exponential gathers psi: every block must have written it
      ok = all_reduce2<SINGLE>(dummy, rp, A, sh, epoch, pc);
      if (ok && blockIdx.x == 0 && threadIdx.x == 0) A.stats->last_norm2 = rp;
    }
  }
  if (!ok && threadIdx.x == 0) {
    // a barrier timed out somewhere: latch a device error
    __hip_atomic_store(&A.stats->status, (int)CFET_EDEVICE, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  }
}

__global__ void k_persist_reset(unsigned long long* bar, int* fault) {
  *bar = 0ull;
  *fault = 0;
}

template <int G, int P, int Q, bool SINGLE>
const void* pick_nt(int NT) {
  return NT == 1 ? (const void*)&k_propagate<G, P, Q, 1, SINGLE>
                 : (const void*)&k_propagate<G, P, Q, 0, SINGLE>;
}

template <bool SINGLE>
const void* pick_kernel(int preset, int NT) {
  switch (preset) {
    case 0: return pick_nt<kPresets[0].G, kPresets[0].P, kPresets[0].Q, SINGLE>(NT);
    case 1: return pick_nt<kPresets[1].G, kPresets[1].P, kPresets[1].Q, SINGLE>(NT);
    case 2: return pick_nt<kPresets[2].G, kPresets[2].P, kPresets[2].Q, SINGLE>(NT);
    case 3: return pick_nt<kPresets[3].G, kPresets[3].P, kPresets[3].Q, SINGLE>(NT);
    default: return nullptr;
  }
}

}  // namespace

int persistent_rows_per_block(int preset) {
  if (preset < 0 || preset >= kNumPresets) return 0;
  return kPresets[preset].P * (kPersistBlock / kPresets[preset].G);
}

// Preset for a matrix: prefer one that holds the longest row in registers,
// then the one holding the fewest entries per lane (register pressure), among
// those whose block capacity is at least min_rows_per_block.
int persistent_choose_preset(int max_row, int64_t min_rows_per_block) {
  int best = -1;
  for (int pass = 0; pass < 2 && best < 0; ++pass) {
    int best_cost = 1 << 30;
    for (int i = 0; i < kNumPresets; ++i) {
      const Preset& q = kPresets[i];
      if (pass == 0 && q.G * q.Q < max_row) continue;
      if (persistent_rows_per_block(i) < min_rows_per_block) continue;
      const int cost = q.P * q.Q;
      if (cost < best_cost) {
        best_cost = cost;
        best = i;
      }
    }
  }
  return best;
}

const void* persistent_kernel(int preset, int nterms, bool single) {
  const int NT = (nterms == 1) ? 1 : 0;
  return single ? pick_kernel<true>(preset, NT) : pick_kernel<false>(preset, NT);
}

hipError_t launch_persistent(const PersistArgs& args, int preset, bool single, int nblocks,
                             hipStream_t st) {
  const void* fn = persistent_kernel(preset, args.nterms, single);
  if (!fn) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_persist_reset, dim3(1), dim3(1), 0, st, args.bar, args.fault);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  PersistArgs a = args;
  void* kargs[] = {&a};
  if (single) {
    e = hipLaunchKernel(fn, dim3(1), dim3(kPersistBlock), kargs, 0, st);
  } else {
    e = hipLaunchCooperativeKernel(fn, dim3(nblocks), dim3(kPersistBlock), kargs, 0, st);
  }
  return e;
}

hipError_t persistent_max_blocks(int preset, int nterms, int* out) {
  const void* fn = persistent_kernel(preset, nterms, false);
  if (!fn) return hipErrorInvalidValue;
  int dev = 0, cus = 0, per = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, kPersistBlock, 0);
  if (e != hipSuccess) return e;
  *out = cus * per;
  return hipSuccess;
}

}  // namespace cfet
