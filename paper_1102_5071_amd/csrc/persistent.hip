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

#include <type_traits>

namespace cfet {

namespace {

// Register-holding presets (G lanes per row, P rows per lane group, Q
// entries per lane and row, B threads per block).  A block holds P * B / G
// rows; rows longer than G*Q read their tail from memory.
struct Preset {
  int G, P, Q, B;
};
// cooperative kernel (gathers prefetched into registers).  With eight entries
// per lane a 512-thread block needs more than the 256 registers a wavefront
// gets at two wavefronts per SIMD and spills to scratch; at 256 threads (one
// wavefront per SIMD) the overflow goes to accumulation registers instead,
// so those presets come first and the 512-thread ones serve only larger
// blocks.  (The single-workgroup kernel is faster with 512 threads in spite
// of its spills: it needs the wavefronts to spread its rows.)
constexpr Preset kCoopPresets[] = {{1, 1, 5, 512}, {1, 1, 8, 256}, {2, 1, 8, 256}, {4, 1, 8, 256},
                                   {1, 1, 8, 512}, {2, 1, 8, 512}, {4, 1, 8, 512}};
// single-workgroup kernel (working vectors in LDS, n <= kSingleMaxRows)
constexpr Preset kSinglePresets[] = {{1, 2, 12, 512}, {2, 2, 8, 512}, {4, 2, 8, 512}};
constexpr int kNumCoopPresets = sizeof(kCoopPresets) / sizeof(kCoopPresets[0]);
constexpr int kNumSinglePresets = sizeof(kSinglePresets) / sizeof(kSinglePresets[0]);
constexpr int kSingleMaxRows = 1024;
constexpr int kCoopMaxRows = 512;  // rows of one cooperative block, at most (P * B / G)

// One DPP step of the wavefront sum: v + (v moved by the DPP pattern), rows
// outside row_mask add 0.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_add(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWMASK, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWMASK, 0xf, false);
  return v + __hiloint2double(hi, lo);
}

// Sum over the 64 lanes in a fixed order with DPP moves (pair swap, quad
// swap, half-row and row mirrors, then row broadcasts 15 and 31); the total
// lands in lane 63 and is broadcast from there.
__device__ __forceinline__ double p_wave_sum(double v) {
  v = dpp_add<0xB1, 0xf>(v);   // quad_perm [1,0,3,2]
  v = dpp_add<0x4E, 0xf>(v);   // quad_perm [2,3,0,1]
  v = dpp_add<0x141, 0xf>(v);  // row_half_mirror
  v = dpp_add<0x140, 0xf>(v);  // row_mirror
  v = dpp_add<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
  v = dpp_add<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
  return lane_read(v, 63);
}

// Device-scope accesses of cross-block vectors: one 16-byte buffer load or
// store carrying the device-coherence cache policy, addressed as (base,
// element index) so the buffer descriptor stays uniform.  The descriptor's
// record count is the vector's byte size, so an index outside [0, n) reads 0
// and drops the write instead of touching other memory.
constexpr int kBufWord3 = 0x00020000;  // descriptor word 3 on gfx9: 32-bit data format
constexpr int kCpolDevice = 16;        // cache-policy operand: device scope

__device__ __forceinline__ __amdgpu_buffer_rsrc_t vec_rsrc(const double2* base, int64_t n) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<double2*>(base), (short)0, (int)(n * 16),
                                           kBufWord3);
}

template <bool SINGLE>
__device__ __forceinline__ double2 vld(const double2* base, int64_t i, int64_t n) {
  if (SINGLE) return base[i];
  const auto v = __builtin_amdgcn_raw_buffer_load_b128(vec_rsrc(base, n), (int)(i * 16), 0,
                                                       kCpolDevice);
  return make_double2(__hiloint2double((int)v[1], (int)v[0]),
                      __hiloint2double((int)v[3], (int)v[2]));
}

template <bool SINGLE>
__device__ __forceinline__ void vst(double2* base, int64_t i, int64_t n, double2 x) {
  if (SINGLE) {
    base[i] = x;
    return;
  }
  typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
  u32x4 v;
  v[0] = (unsigned)__double2loint(x.x);
  v[1] = (unsigned)__double2hiint(x.x);
  v[2] = (unsigned)__double2loint(x.y);
  v[3] = (unsigned)__double2hiint(x.y);
  __builtin_amdgcn_raw_buffer_store_b128(v, vec_rsrc(base, n), (int)(i * 16), 0, kCpolDevice);
}

// Barrier state: words kBarGroupStride*(1+g) = arrival counter of group g
// (blocks b with b % groups == g), one 128-byte line each, so arrivals of
// different groups do not serialise on one address; word 0 is unused.
constexpr int kBarGroups = 16;
constexpr int kBarGroupStride = 16;  // 64-bit words per 128-byte line

__device__ bool grid_barrier(unsigned long long* bar, int* fault, unsigned long long& epoch,
                             long long limit, int* s_ok) {
  // all memory operations of this wave (device-scope stores included) are done
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  epoch += 1ull;
  const int nb = gridDim.x;
  const int ng = nb < kBarGroups ? nb : kBarGroups;
  // arrive on the group counter (no return value is needed)
  if (threadIdx.x == 0)
    __hip_atomic_fetch_add(bar + kBarGroupStride * (1 + blockIdx.x % ng), 1ull,
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (threadIdx.x < 64) {
    // wavefront 0 watches every group counter at once (lane g: group g) and,
    // in the same round, the fault flag (lane ng)
    const int l = threadIdx.x;
    const unsigned long long members =
        (l < ng) ? (unsigned long long)((nb - 1 - l) / ng + 1) : 0ull;
    const unsigned long long target = epoch * members;
    int ok = 1;
    const long long t0 = wall_clock64();
    for (;;) {
      bool waiting = false, faulted = false;
      if (l < ng)
        waiting = __hip_atomic_load(bar + kBarGroupStride * (1 + l), __ATOMIC_RELAXED,
                                    __HIP_MEMORY_SCOPE_AGENT) < target;
      else if (l == ng)
        faulted = __hip_atomic_load(fault, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
      if (__ballot(waiting) == 0ull) break;
      if (__ballot(faulted) != 0ull) {
        ok = 0;
        break;
      }
      if (wall_clock64() - t0 > limit) {
        if (l == 0) __hip_atomic_store(fault, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    if (l == 0) *s_ok = ok;
  }
  __syncthreads();
  return *s_ok != 0;
}

constexpr int kRedB = 16;      // offset of the second sum's per-wavefront values
constexpr int kRedA = 2 * kRedB;  // the two results

struct Shared {
  double cheb[kChebMaxTerms];
  // block reductions: per-wavefront values of the first sum at red[w], of the
  // second at red[kRedB + w] (up to 16 wavefronts), results at red[2 kRedB + 0/1]
  double red[2 * kRedB + 2];
  // the single workgroup's per-iteration sums: two alternating sets of
  // per-wavefront values (first sum at [w], second at [kRedB + w])
  double red2[2][2 * kRedB];
  // per-wavefront values of the cross-block re-sum (first sum at [w], second at [kRedB + w])
  double pr[2 * kRedB];
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
    red[kRedB + w] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double ta = 0.0, tb = 0.0;
    for (int i = 0; i < nw; ++i) {
      ta += red[i];
      tb += red[kRedB + i];
    }
    red[kRedA] = ta;
    red[kRedA + 1] = tb;
  }
  __syncthreads();
  a = red[kRedA];
  b = red[kRedA + 1];
}

// The same two block sums with one block barrier: the per-wavefront values go
// to the set `parity` of red2 and every thread adds them in the order thread
// 0 uses above (so the results are the same bit for bit).  Two calls in a row
// use different sets; a set is rewritten only two calls later, after a block
// barrier that every thread passes once it has read the set.
// NW: wavefronts of the block, a compile-time constant, so that the reads of
// the per-wavefront values are issued together (and no block size is loaded).
template <int NW>
__device__ __forceinline__ void p_block_sum2_1b(double& a, double& b, double (*red2)[2 * kRedB],
                                                int& parity) {
  a = p_wave_sum(a);
  b = p_wave_sum(b);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  double* R = red2[parity];
  if (l == 0) {
    R[w] = a;
    R[kRedB + w] = b;
  }
  __syncthreads();
  double ta = 0.0, tb = 0.0;
#pragma unroll
  for (int i = 0; i < NW; ++i) {
    ta += R[i];
    tb += R[kRedB + i];
  }
  a = ta;
  b = tb;
  parity ^= 1;
}

// Cross-block sums.  Each block publishes its two partial sums as one
// 16-byte record (set `ph & 1` of A.part, record blockIdx.x); after the grid
// barrier every block re-sums all records in the same fixed order: thread t
// loads record t (the launch has at most as many blocks as a block has
// threads), the wavefronts reduce with the DPP sum, and every thread adds the
// per-wavefront values in wavefront order, so all blocks hold bit-identical
// totals.  The record load is issued before the gathers of the next phase,
// which are issued unconditionally, so waiting for the record does not wait
// for them.
__device__ __forceinline__ void publish_partial(const PersistArgs& A, int ph, double a, double b) {
  double2* P = reinterpret_cast<double2*>(A.part) + (size_t)(ph & 1) * gridDim.x;
  vst<false>(P, blockIdx.x, gridDim.x, make_double2(a, b));
}

__device__ __forceinline__ void resum_issue(const PersistArgs& A, int ph, double2& pv) {
  const double2* P = reinterpret_cast<const double2*>(A.part) + (size_t)(ph & 1) * gridDim.x;
  // threads past the last record read 0 (outside the buffer's records)
  pv = vld<false>(P, threadIdx.x, gridDim.x);
}

// BLOCK: the block size (a compile-time constant: reading blockDim is a
// memory load, and waiting for it would wait for the gathers in flight)
template <int BLOCK>
__device__ __forceinline__ void resum_finish(double2 pv, Shared& sh, double& a, double& b) {
  double sa = pv.x, sb = pv.y;
  sa = p_wave_sum(sa);
  sb = p_wave_sum(sb);
  if ((threadIdx.x & 63) == 0) {
    sh.pr[threadIdx.x >> 6] = sa;
    sh.pr[kRedB + (threadIdx.x >> 6)] = sb;
  }
  __syncthreads();
  double ta = 0.0, tb = 0.0;
  for (int w = 0; w < BLOCK / 64; ++w) {
    ta += sh.pr[w];
    tb += sh.pr[kRedB + w];
  }
  a = ta;
  b = tb;
}

// Segment timer (block 0, thread 0, only when A.timing is set).
// Accumulated in registers and written once at the end of the launch, so that
// timing adds no memory round trip to the path it measures.
struct SegTimer {
  long long last;
  long long acc[4];
  bool on;
  __device__ void start(bool enable) {
    on = enable && blockIdx.x == 0 && threadIdx.x == 0;
    acc[0] = acc[1] = acc[2] = acc[3] = 0;
    if (on) last = wall_clock64();
  }
  __device__ void lap(DevStats*, int seg) {
    if (!on) return;
    const long long t = wall_clock64();
    acc[seg] += t - last;
    last = t;
  }
  __device__ void flush(DevStats* st) {
    if (!on) return;
    for (int i = 0; i < 4; ++i) st->seg[i] += acc[i];
  }
};

// Statistics of the launch, kept by thread 0 of block 0 and added to the
// device statistics once at the end.
struct LaunchStats {
  unsigned long long expo = 0, mv = 0;
  int minm = 1 << 30, brk = 0, status = CFET_OK;
  __device__ void flush(DevStats* st) {
    if (expo == 0) return;
    st->exponentials += expo;
    st->matvecs += mv;
    if (minm < st->min_m_eff) st->min_m_eff = minm;
    st->breakdowns += brk;
    if (status != CFET_OK && st->status == CFET_OK) st->status = status;
  }
};

// RV: every stored value is real (imaginary parts exactly 0), so the
// register-held entries keep only their real parts (half the registers; the
// products are the same numbers, a zero imaginary part contributing exact
// zeros).
template <int G, int PMAX, int QMAX, int NT, bool SINGLE, int BLOCK, bool RV = false>
__global__ __launch_bounds__(BLOCK) void k_propagate(PersistArgs A) {
  static_assert(BLOCK % 64 == 0 && BLOCK <= 64 * kRedB, "block of whole wavefronts, at most 16");
  static_assert(SINGLE || PMAX * BLOCK / G <= kCoopMaxRows, "rows of a block exceed the ring");
  __shared__ Shared sh;
  // u_k ring (k mod 3) of this block's own rows in LDS, indexed by row - r0:
  // the single workgroup reads every gathered value from here, the cooperative
  // blocks the entries whose column is one of their own rows
  constexpr int LN = SINGLE ? kSingleMaxRows : kCoopMaxRows;
  __shared__ double2 lu[3][LN];
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
  int rpar = 0;  // set of sh.red2 the next single-workgroup sum uses
  bool ok = true;
  double2* __restrict__ psi = A.psi;
  // u_0 = psi, u_k (k >= 1) in the basis storage; z_k alternates between two buffers
  auto U = [&](int k) -> double2* {
    return (k <= 0) ? psi : A.basis + (size_t)(k - 1) * (size_t)n;
  };
  auto Zb = [&](int k) -> double2* { return A.zbuf + (size_t)(k & 1) * (size_t)n; };

  // ---- the matrix entries this lane will use, kept in registers
  int64_t rowp[PMAX];
  int64_t tail_beg[PMAX], tail_end[PMAX];
  int cnt[PMAX];
  uint32_t ccol[PMAX][QMAX];
  std::conditional_t<RV, double, double2> cval[PMAX][QMAX];
  uint32_t lmask[PMAX];  // bit q: entry q's column is a row of this block (read from LDS)
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
        ccol[p][q] = A.colt[e] ;
        if constexpr (RV) cval[p][q] = A.val[e].x;
        else cval[p][q] = A.val[e];
      } else {
        ccol[p][q] = 0u;
        if constexpr (RV) cval[p][q] = 0.0;
        else cval[p][q] = make_double2(0.0, 0.0);
      }
    }
    tail_beg[p] = beg + (int64_t)QMAX * G + lane;
    tail_end[p] = end;
    lmask[p] = 0u;
#pragma unroll
    for (int q = 0; q < QMAX; ++q) {
      const int64_t c = ccol[p][q] & kColMask;
      if (SINGLE || (c >= r0 && c < r1)) lmask[p] |= (1u << q);
    }
    const int64_t len = end - beg;
    cnt[p] = (len > lane) ? (int)min<int64_t>(QMAX, (len - lane + G - 1) / G) : 0;
  }

  // own-row state (lane 0 of each group): u_{k-1}, u_{k-2}, z_{k-1}
  double2 u1[PMAX], u2[PMAX], zp[PMAX];
  // other blocks' columns of the register-held entries: running copies of
  // u_{k-1} (g1), u_{k-2} (g2), and z_{k-1} gathered for the current phase
  double2 g1[PMAX][QMAX], g2[PMAX][QMAX], gz[PMAX][QMAX];
#pragma unroll
  for (int p = 0; p < PMAX; ++p) {
    u1[p] = u2[p] = zp[p] = make_double2(0.0, 0.0);
    if (lane == 0 && rowp[p] >= 0) u1[p] = vld<SINGLE>(psi, rowp[p], n);  // becomes u_0
  }
  // issue the gathers of phase k at the register-held entries whose column is
  // another block's row: phase 0 takes u_0 = psi, phase k >= 1 only z_{k-1}.
  // u_{k-1} and u_{k-2} of such a column are the running copies g1, g2 that
  // this lane formed itself in the two phases before, with the same fused
  // multiply-adds as the column's owner, so they equal the owner's values bit
  // for bit (by induction from u_0).  Every entry issues its load (no branch,
  // so the compiler can count the loads in flight): an entry that needs none
  // reads index n, outside the buffer's records, which returns 0 without a
  // memory access; its register is never read.  live = false: no entry needs
  // a value (the phase after the last product).
  auto gather = [&](int k, bool live) {
    if (SINGLE) return;
    const double2* __restrict__ a0 = psi;
    const double2* __restrict__ az = Zb(k - 1);
#pragma unroll
    for (int p = 0; p < PMAX; ++p) {
#pragma unroll
      for (int q = 0; q < QMAX; ++q) {
        const bool need = live && rowp[p] >= 0 && q < cnt[p] && !((lmask[p] >> q) & 1u);
        const int64_t c = need ? (int64_t)(ccol[p][q] & kColMask) : n;
        if (k == 0) g1[p][q] = vld<SINGLE>(a0, c, n);
        else gz[p][q] = vld<SINGLE>(az, c, n);
      }
    }
  };

  SegTimer tm;
  tm.start(A.timing != 0);
  LaunchStats ls;
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
      double c1 = 0.0, c2 = 0.0, c3 = 0.0;
      double S1 = 0.0, S2 = 0.0;  // block sums of <u, z> and ||u||^2 of the last phase
      double scale = 0.0, alpha_prev = 0.0, inv_prev = 0.0;
      // index of this exponential in application order within the call
      const int64_t eidx = step * A.s + (A.s - 1 - i);
      LzScalars* const XT = (A.export_T && A.export_each) ? A.export_T + eidx : A.export_T;
      double2* const XY =
          (A.export_Y && A.export_each) ? A.export_Y + (size_t)eidx * (size_t)m * (size_t)n
                                        : A.export_Y;
      // u_0 = psi on the own rows (the previous exponential's barrier or the
      // weights' __syncthreads above ended every read of the ring)
#pragma unroll
      for (int p = 0; p < PMAX; ++p)
        if (lane == 0 && rowp[p] >= 0) {
          lu[0][rowp[p] - r0] = u1[p];
          if (A.save) A.save[eidx * n + rowp[p]] = u1[p];  // the state before this exponential
        }
      __syncthreads();
      gather(0, true);
      for (int k = 0; k <= m; ++k) {
        if (k >= 1) {
          tm.lap(A.stats, 1);
          // ---- reduction of phase k-1; the gathers of phase k fly meanwhile
          if (!SINGLE) {
            // every block re-sums the block partials in the same fixed order
            double2 pv;
            resum_issue(A, pc - 1, pv);
            gather(k, k < m);
            resum_finish<BLOCK>(pv, sh, S1, S2);
          }
          const double nu = sqrt(S2);
          if (k == 1) {
            nu0 = nu;
            if (nu == 0.0) {  // psi == 0 stays 0
              zero = true;
              break;
            }
          } else {
            // beta_{k-2} = nu_{k-1}: early-stop rule of the recurrence, with the
            // running max over t <= k-2 of |alpha_t| + beta_t
            scale = fmax(scale, fabs(alpha_prev) + nu);
            if (threadIdx.x == 0) sh.beta[k - 2] = nu;
            if (nu <= kBreakdownRel * scale) {
              meff = k - 1;
              break;
            }
          }
          const double inv = 1.0 / nu;
          const double alpha = S1 * inv * inv;
          if (threadIdx.x == 0) {
            sh.alpha[k - 1] = alpha;
            sh.inv[k - 1] = inv;
          }
          // u_k = (z_{k-1} - alpha_{k-1} u_{k-1})/nu_{k-1} - (nu_{k-1}/nu_{k-2}) u_{k-2}
          c3 = (k >= 2) ? nu * inv_prev : 0.0;
          inv_prev = inv;
          alpha_prev = alpha;
          if (k == m) break;
          c1 = inv;
          c2 = alpha * inv;
        }
        // ---- phase k: u_k on own rows, z_k = H_w u_k, partial sums
        double2* __restrict__ uk = U(k);
        double2* __restrict__ zk = Zb(k);
        const double2* __restrict__ um1 = U(k - 1);
        const double2* __restrict__ zm1 = Zb(k - 1);
        const double2* __restrict__ um2 = U(k - 2);
        double s_uz = 0.0, s_uu = 0.0;
        // u_k on the own rows first; after one block barrier every column that
        // is a row of this block reads it from LDS (the value its owner formed)
        double2 ucurs[PMAX];
#pragma unroll
        for (int p = 0; p < PMAX; ++p) {
          ucurs[p] = u1[p];
          if (k >= 1 && lane == 0 && rowp[p] >= 0) {
            ucurs[p] = form_u(zp[p], u1[p], u2[p], c1, c2, c3);
            vst<SINGLE>(uk, rowp[p], n, ucurs[p]);
            lu[k % 3][rowp[p] - r0] = ucurs[p];
          }
        }
        __syncthreads();
#pragma unroll
        for (int p = 0; p < PMAX; ++p) {
          const double2 ucur = ucurs[p];
          double a0r = 0.0, a0i = 0.0, a1r = 0.0, a1i = 0.0;
          if (rowp[p] >= 0) {
            // the ring values of all register-held entries are read first,
            // with nothing between the reads, so that they are in flight
            // together (an entry whose column is another block's row reads
            // index 0 and does not use it; in the single workgroup an entry
            // past the row's length holds value 0 and column 0, a valid index
            // of the ring, and adds a zero product)
            double2 xs[QMAX];
#pragma unroll
            for (int q = 0; q < QMAX; ++q) {
              const int li =
                  SINGLE ? (int)(ccol[p][q] & kColMask)
                         : (((lmask[p] >> q) & 1u) ? (int)((int64_t)(ccol[p][q] & kColMask) - r0)
                                                   : 0);
              xs[q] = lu[k % 3][li];
            }
#pragma unroll
            for (int q = 0; q < QMAX; ++q) {
              if (SINGLE || q < cnt[p]) {
                const uint32_t ct = ccol[p][q];
                const auto v = cval[p][q];
                double2 xv;
                if (SINGLE || ((lmask[p] >> q) & 1u)) {
                  xv = xs[q];  // u_k of a row of this block
                } else {
                  const double2 xg2 = (k >= 2) ? g2[p][q] : make_double2(0.0, 0.0);
                  xv = (k >= 1) ? form_u(gz[p][q], g1[p][q], xg2, c1, c2, c3) : g1[p][q];
                  if (k >= 1) {  // the running copies move on: u_{k-1}, u_k
                    g2[p][q] = g1[p][q];
                    g1[p][q] = xv;
                  }
                }
                double pr, pi;
                if constexpr (RV) {
                  pr = v * xv.x;
                  pi = v * xv.y;
                } else {
                  pr = v.x * xv.x - v.y * xv.y;
                  pi = v.x * xv.y + v.y * xv.x;
                }
                if (NT == 1) {
                  if (ct >> kTermShift) { a1r += pr; a1i += pi; } else { a0r += pr; a0i += pi; }
                } else {
                  const double wt = sh.w[ct >> kTermShift];
                  a0r += wt * pr;
                  a0i += wt * pi;
                }
              }
            }
            for (int64_t e = tail_beg[p]; e < tail_end[p]; e += G) {
              const uint32_t ct = A.colt[e];
              const double2 v = A.val[e];
              const int64_t c = ct & kColMask;
              double2 xv;
              if (SINGLE) {
                xv = lu[k % 3][c];  // u_k (every row is the block's own)
              } else {
                xv = vld<SINGLE>(um1, c, n);
                if (k >= 1) {
                  const double2 zc = vld<SINGLE>(zm1, c, n);
                  const double2 u2c = (k >= 2) ? vld<SINGLE>(um2, c, n) : make_double2(0.0, 0.0);
                  xv = form_u(zc, xv, u2c, c1, c2, c3);
                }
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
          if (NT == 1 && XY) {
            // H_1 u_k on this row (the driven term alone, before weighting)
            double hr = a1r, hi = a1i;
#pragma unroll
            for (int off = G / 2; off >= 1; off >>= 1) {
              hr += __shfl_xor(hr, off, G);
              hi += __shfl_xor(hi, off, G);
            }
            if (lane == 0 && rowp[p] >= 0) XY[(size_t)k * (size_t)n + rowp[p]] = make_double2(hr, hi);
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
            if (!SINGLE && k + 1 < m) vst<SINGLE>(zk, rowp[p], n, zv);
            s_uz += ucur.x * zv.x + ucur.y * zv.y;
            s_uu += ucur.x * ucur.x + ucur.y * ucur.y;
            u2[p] = u1[p];
            u1[p] = ucur;
            zp[p] = zv;
          }
        }
        tm.lap(A.stats, 0);
        if (SINGLE) {
          p_block_sum2_1b<BLOCK / 64>(s_uz, s_uu, sh.red2, rpar);
          S1 = s_uz;
          S2 = s_uu;
        } else {
          // wave sums to LDS, thread 0 adds them in order and publishes the
          // block partial (the barrier's own __syncthreads follows)
          s_uz = p_wave_sum(s_uz);
          s_uu = p_wave_sum(s_uu);
          if ((threadIdx.x & 63) == 0) {
            sh.red[threadIdx.x >> 6] = s_uz;
            sh.red[kRedB + (threadIdx.x >> 6)] = s_uu;
          }
          __syncthreads();
          if (threadIdx.x == 0) {
            double ta = 0.0, tb = 0.0;
            for (int wv = 0; wv < BLOCK / 64; ++wv) {
              ta += sh.red[wv];
              tb += sh.red[kRedB + wv];
            }
            publish_partial(A, pc, ta, tb);
          }
          if (!grid_barrier(A.bar, A.fault, epoch, A.spin_limit, &sh.ok)) {
            ok = false;
            break;
          }
          pc += 1;
        }
      }
      if (!ok) break;
      if (zero) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
          ls.expo += 1;
          ls.brk += 1;
          ls.minm = 0;
          if (XT) {
            XT->beta0 = 0.0;
            XT->m_eff = 0;
          }
        }
        continue;
      }
      __syncthreads();
      if (XT && blockIdx.x == 0) {
        // the projection of this exponential: u_j = nu_j v_j, so inv_nrm = 1 / nu
        LzScalars* X = XT;
        const int t = threadIdx.x;
        if (t < meff) {
          X->alpha[t] = sh.alpha[t];
          X->inv_nrm[t] = sh.inv[t];
        }
        if (t < meff - 1) X->beta[t] = sh.beta[t];
        if (t == 0) {
          X->beta0 = nu0;
          X->m_eff = meff;
        }
      }
      if (A.no_combine) continue;
      tm.lap(A.stats, 1);
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
          ls.expo += 1;
          ls.mv += (unsigned long long)meff;
          if (meff < ls.minm) ls.minm = meff;
          if (meff < m) ls.brk += 1;
          if (status != CFET_OK && ls.status == CFET_OK) ls.status = status;
        }
      }
      __syncthreads();
      tm.lap(A.stats, 2);
      // ---- recombination psi = sum_k coef_k u_k on own rows
#pragma unroll
      for (int p = 0; p < PMAX; ++p) {
        if (lane == 0 && rowp[p] >= 0) {
          double accr = 0.0, acci = 0.0;
          int kk = 0;
          // eight basis entries in flight at a time, summed in order
          for (; kk + 8 <= meff; kk += 8) {
            double2 v[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) v[q] = vld<SINGLE>(U(kk + q), rowp[p], n);
#pragma unroll
            for (int q = 0; q < 8; ++q) {
              const double2 cf = sh.coef[kk + q];
              accr += cf.x * v[q].x - cf.y * v[q].y;
              acci += cf.x * v[q].y + cf.y * v[q].x;
            }
          }
          for (; kk < meff; ++kk) {
            const double2 v = vld<SINGLE>(U(kk), rowp[p], n);
            const double2 cf = sh.coef[kk];
            accr += cf.x * v.x - cf.y * v.y;
            acci += cf.x * v.y + cf.y * v.x;
          }
          const double2 nv = make_double2(accr, acci);
          vst<SINGLE>(psi, rowp[p], n, nv);
          u1[p] = nv;
        }
      }
      // the next exponential gathers psi: every block must have written it
      if (SINGLE) {
        __syncthreads();
      } else if (!grid_barrier(A.bar, A.fault, epoch, A.spin_limit, &sh.ok)) {
        ok = false;
      }
      tm.lap(A.stats, 3);
    }
  }
  if (ok) {
    // ||psi||^2 after the last exponential, for the statistics
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int p = 0; p < PMAX; ++p)
      if (lane == 0 && rowp[p] >= 0) s1 += u1[p].x * u1[p].x + u1[p].y * u1[p].y;
    p_block_sum2(s0, s1, sh.red);
    if (!SINGLE) {
      if (threadIdx.x == 0) publish_partial(A, pc, s0, s1);
      if (grid_barrier(A.bar, A.fault, epoch, A.spin_limit, &sh.ok)) {
        double2 pv;
        resum_issue(A, pc, pv);
        resum_finish<BLOCK>(pv, sh, s0, s1);
      } else {
        ok = false;
      }
    }
    if (ok && blockIdx.x == 0 && threadIdx.x == 0 && A.nsteps > 0) A.stats->last_norm2 = s1;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ls.flush(A.stats);
    tm.flush(A.stats);
  }
  if (!ok && threadIdx.x == 0) {
    // a barrier timed out somewhere: latch a device error
    __hip_atomic_store(&A.stats->status, (int)CFET_EDEVICE, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  }
}

__global__ void k_persist_reset(unsigned long long* bar, int* fault) {
  for (int i = threadIdx.x; i < kBarGroupStride * (1 + kBarGroups); i += blockDim.x) bar[i] = 0ull;
  if (threadIdx.x == 0) *fault = 0;
}

template <int G, int P, int Q, bool SINGLE, int B, bool RV = false>
const void* pick_nt(int NT) {
  return NT == 1 ? (const void*)&k_propagate<G, P, Q, 1, SINGLE, B, RV>
                 : (const void*)&k_propagate<G, P, Q, 0, SINGLE, B, RV>;
}

static_assert(kNumCoopPresets == 7 && kNumSinglePresets == 3,
              "pick_coop and pick_single list every preset");

const void* pick_coop(int preset, int NT, bool real) {
#define CFET_CP(I)                                                                        \
  case I:                                                                                 \
    return real ? pick_nt<kCoopPresets[I].G, kCoopPresets[I].P, kCoopPresets[I].Q, false, \
                          kCoopPresets[I].B, true>(NT)                                    \
                : pick_nt<kCoopPresets[I].G, kCoopPresets[I].P, kCoopPresets[I].Q, false, \
                          kCoopPresets[I].B>(NT);
  switch (preset) {
    CFET_CP(0)
    CFET_CP(1)
    CFET_CP(2)
    CFET_CP(3)
    CFET_CP(4)
    CFET_CP(5)
    CFET_CP(6)
    default: return nullptr;
  }
#undef CFET_CP
}

const void* pick_single(int preset, int NT, bool real) {
#define CFET_SP(I)                                                                        \
  case I:                                                                                 \
    return real ? pick_nt<kSinglePresets[I].G, kSinglePresets[I].P, kSinglePresets[I].Q,  \
                          true, kSinglePresets[I].B, true>(NT)                            \
                : pick_nt<kSinglePresets[I].G, kSinglePresets[I].P, kSinglePresets[I].Q,  \
                          true, kSinglePresets[I].B>(NT);
  switch (preset) {
    CFET_SP(0)
    CFET_SP(1)
    CFET_SP(2)
    default: return nullptr;
  }
#undef CFET_SP
}

}  // namespace

int persistent_block_threads(int preset, bool single) {
  const Preset* t = single ? kSinglePresets : kCoopPresets;
  const int np = single ? kNumSinglePresets : kNumCoopPresets;
  return (preset < 0 || preset >= np) ? 0 : t[preset].B;
}

int persistent_rows_per_block(int preset, bool single) {
  const Preset* t = single ? kSinglePresets : kCoopPresets;
  const int np = single ? kNumSinglePresets : kNumCoopPresets;
  if (preset < 0 || preset >= np) return 0;
  const int rows = t[preset].P * (t[preset].B / t[preset].G);
  return single ? std::min(rows, kSingleMaxRows) : rows;
}

// Preset for a matrix: prefer one that holds the longest row in registers,
// then the one holding the fewest entries per lane (register pressure), among
// those whose block capacity is at least min_rows_per_block.
int persistent_choose_preset(int max_row, int64_t min_rows_per_block, bool single) {
  const Preset* t = single ? kSinglePresets : kCoopPresets;
  const int np = single ? kNumSinglePresets : kNumCoopPresets;
  int best = -1;
  for (int pass = 0; pass < 2 && best < 0; ++pass) {
    int best_cost = 1 << 30;
    for (int i = 0; i < np; ++i) {
      const Preset& q = t[i];
      if (pass == 0 && q.G * q.Q < max_row) continue;
      if (persistent_rows_per_block(i, single) < min_rows_per_block) continue;
      const int cost = q.P * q.Q;
      if (cost < best_cost) {
        best_cost = cost;
        best = i;
      }
    }
  }
  return best;
}

// real: the real-valued form (every stored value has imaginary part 0)
const void* persistent_kernel(int preset, int nterms, bool single, bool real) {
  const int NT = (nterms == 1) ? 1 : 0;
  return single ? pick_single(preset, NT, real) : pick_coop(preset, NT, real);
}

hipError_t launch_persistent(const PersistArgs& args, int preset, bool single, int nblocks,
                             hipStream_t st, bool reset) {
  const void* fn = persistent_kernel(preset, args.nterms, single, args.real_vals != 0);
  if (!fn) return hipErrorInvalidValue;
  hipError_t e = hipSuccess;
  if (reset) {
    hipLaunchKernelGGL(k_persist_reset, dim3(1), dim3(64), 0, st, args.bar, args.fault);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  PersistArgs a = args;
  void* kargs[] = {&a};
  const int block = persistent_block_threads(preset, single);
  // the cross-block re-sum loads one partial record per thread
  if (!single && nblocks > block) return hipErrorInvalidValue;
  if (single) {
    e = hipLaunchKernel(fn, dim3(1), dim3(block), kargs, 0, st);
  } else {
    e = hipLaunchCooperativeKernel(fn, dim3(nblocks), dim3(block), kargs, 0, st);
  }
  return e;
}

hipError_t persistent_max_blocks(int preset, int nterms, bool real, int* out) {
  const void* fn = persistent_kernel(preset, nterms, false, real);
  if (!fn) return hipErrorInvalidValue;
  int dev = 0, cus = 0, per = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn,
                                                     persistent_block_threads(preset, false), 0);
  if (e != hipSuccess) return e;
  *out = cus * per;
  return hipSuccess;
}

int persistent_barrier_words() { return kBarGroupStride * (1 + kBarGroups); }

}  // namespace cfet
