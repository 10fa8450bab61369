// LDS-tiled Lanczos SpMV for the split shared-part layout (two passes).
//
// Both passes walk the rows in tiles of 2^tbits consecutive indices of their
// order (the identity for the first pass, the bit-permuted order of DevSELLHi
// for the second).  A workgroup copies the tile's x values into LDS with
// coalesced loads, then its wavefronts run the tile's 64-row slices: a shared
// entry whose offset stays inside the tile (offset < 2^tbits in that order)
// reads x from LDS, every other column is gathered from memory.  In the
// second pass every offset stays inside the tile (the layout is built so); in
// the first the out-of-tile entries of a slice are stored first, so the first
// batch of a slice issues its gathers before its LDS reads.
//
// The entries' metadata is uniform across a wavefront and read with scalar
// loads; an entry held by every row of its slice (a site flip) skips the
// per-lane mask test, and operators whose stored values are all real
// accumulate real products only (half the floating-point work).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "cfet_internal.h"
#include "partials.hpp"

namespace cfet {

namespace {

// Two workgroups share a CU (64 KiB tiles in LDS); the block size sets the
// resident wavefronts: 12 per workgroup for the first pass (its registers
// allow 6 per SIMD), 16 for the second (8 per SIMD).  More resident
// wavefronts hide more of each slice's chain of metadata, LDS and gather
// latencies.
constexpr int kPass1Threads = 768;
constexpr int kPass2Threads = 1024;
constexpr int kMaxTileWaves = 16;
// tile elements each thread stages (the index is masked into the tile, so a
// count that does not divide it reads some elements twice)
template <int THREADS>
constexpr int tile_loads() {
  return ((1 << kTileBitsMax) + THREADS - 1) / THREADS;
}
// The tile is staged through named registers per thread (an array here is
// kept in scratch memory across the barrier by the compiler).
static_assert(tile_loads<kPass1Threads>() <= 8 && tile_loads<kPass2Threads>() <= 8,
              "tile staging is written out for at most eight loads per thread");
#define CFET_TILE_8(M) M(0) M(1) M(2) M(3) M(4) M(5) M(6) M(7)
#define CFET_TS(u) \
  if constexpr (u < LOADS) xt[((int)threadIdx.x + u * THREADS) & (T - 1)] = b##u;
constexpr int kTileScratch = 32;   // doubles after the tile: block sums and term weights

typedef double dvec2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ double t_wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <int WAVES>
__device__ double t_block_sum(double v, double* red) {
  static_assert(WAVES <= kMaxTileWaves, "block sums hold 16 wavefronts");
  v = t_wave_sum(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) red[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < WAVES; ++i) t += red[i];
    red[16] = t;
  }
  __syncthreads();
  return red[16];
}

template <int WAVES>
__device__ double t_sum_partials(const double* __restrict__ part, int np, double* red) {
  return t_block_sum<WAVES>(thread_partials<64 * WAVES>(part, np), red);
}

// The layout arrays are not written while the kernels run: reading them
// through the constant address space lets uniform reads use scalar loads.
#define CFET_CONST __attribute__((address_space(4)))
template <class T>
__device__ __forceinline__ const CFET_CONST T* as_const(const T* p) {
  return (const CFET_CONST T*)(p);
}

// Term weights as the kernels read them: NT = 1 (one driven term): w0, w1
// in scalar registers; otherwise the table wl in LDS.
struct Wts {
  double w0, w1;
  const double* wl;
};

// (ar, ai) += w_term v xv, the weight folded into the value (RV: the
// imaginary part of v is zero).  ct is uniform for shared entries and
// per-lane for per-row slots.
template <int NT, bool RV>
__device__ __forceinline__ void t_acc(uint32_t ct, dvec2 v, double2 xv, const Wts& W, double& ar,
                                      double& ai) {
  const double w = (NT == 1) ? ((ct >> kTermShift) ? W.w1 : W.w0) : W.wl[ct >> kTermShift];
  const double er = w * v.x;
  if (RV) {
    ar = fma(er, xv.x, ar);
    ai = fma(er, xv.y, ai);
  } else {
    const double ei = w * v.y;
    ar = fma(er, xv.x, fma(-ei, xv.y, ar));
    ai = fma(er, xv.y, fma(ei, xv.x, ai));
  }
}

typedef __attribute__((address_space(3))) const dvec2* lds_cptr;

// x of the tile-local index qloc ^ offset: qb = LDS byte address of the lane's
// own element (tile base + 16 qloc), ob = 16 (offset & tile mask)
// (wavefront-uniform, formed with scalar operations).  The tile base is
// aligned to the tile's byte size (it is the start of the dynamic LDS), so
// qb ^ ob stays in the tile: one vector XOR per entry, no add of the base.
__device__ __forceinline__ double2 t_lds(const double2*, uint32_t qb, uint32_t ob) {
  const dvec2 v = *(lds_cptr)(uintptr_t)(qb ^ ob);
  return make_double2(v.x, v.y);
}

// LDS byte address of the lane's element, kept opaque to the compiler so that
// it does not fold the per-entry XOR back into (qloc ^ offset) & mask,
// shifted, plus the base (several vector operations per entry)
__device__ __forceinline__ uint32_t t_lane_bytes(const double2* xt, int qloc) {
  uint32_t qb = (uint32_t)(uintptr_t)((lds_cptr)xt) + ((uint32_t)qloc << 4);
  asm volatile("" : "+v"(qb));
  return qb;
}

// One group of a slice's shared entries (count cnt, a multiple of four) into
// (ar, ai) without weights.  FULL: every row holds every entry (no lane test).
// Offsets up to tmask read the tile in LDS; larger ones (GLOBAL: first pass,
// identity order) gather x[row ^ offset]; the host stores them first in the
// group, in whole batches of four.  The metadata of four entries is
// read (scalar loads) before any of it is used: one latency per four.
template <bool FULL, bool RV, bool GLOBAL>
__device__ __forceinline__ void t_group(const CFET_CONST uint32_t* uc, const CFET_CONST dvec2* uv,
                                        const CFET_CONST uint64_t* um, int k0, int cnt,
                                        uint64_t lanebit, uint32_t qb, int64_t row,
                                        uint32_t tmask, const double2* xt,
                                        const double2* __restrict__ x, double& ar, double& ai) {
  for (int k = k0; k < k0 + cnt; k += 4) {
    uint32_t off[4];
    uint64_t m[4];
    dvec2 v[4];
    double2 xv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      off[u] = uc[k + u] & kColMask;
      m[u] = FULL ? ~0ull : um[k + u];
      v[u].x = uv[k + u].x;
      v[u].y = RV ? 0.0 : uv[k + u].y;
    }
    // a batch is all gathers or all tile reads (the host orders and pads the
    // lists so): one decision per batch, no per-entry branch
    if (GLOBAL && off[0] > tmask) {
#pragma unroll
      for (int u = 0; u < 4; ++u)
        xv[u] = x[(FULL || (m[u] & lanebit)) ? row ^ (int64_t)off[u] : row];
    } else {
#pragma unroll
      for (int u = 0; u < 4; ++u) xv[u] = t_lds(xt, qb, (off[u] & tmask) << 4);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (FULL || (m[u] & lanebit)) {
        if (RV) {
          ar = fma(v[u].x, xv[u].x, ar);
          ai = fma(v[u].x, xv[u].y, ai);
        } else {
          ar = fma(v[u].x, xv[u].x, fma(-v[u].y, xv[u].y, ar));
          ai = fma(v[u].x, xv[u].y, fma(v[u].y, xv[u].x, ai));
        }
      }
    }
  }
}

// Unweighted sums of a slice's shared entries, by term: (a0r, a0i) over H0's
// entries, (a1r, a1i) over the driven term's (one driven term: NT = 1).
// t_group for real values from 64-byte records (one scalar load per batch
// of four; record k / 4 holds entries k .. k + 3, k a multiple of four).
template <bool FULL, bool GLOBAL>
__device__ __forceinline__ void t_group_rec(const CFET_CONST Rec4* rec,
                                            const CFET_CONST uint64_t* um, int k0, int cnt,
                                            uint64_t lanebit, uint32_t qb, int64_t row,
                                            uint32_t tmask, const double2* xt,
                                            const double2* __restrict__ x, double& ar,
                                            double& ai) {
  typedef uint32_t u32x16 __attribute__((ext_vector_type(16)));
  for (int k = k0; k < k0 + cnt; k += 4) {
    // the whole record in one load
    const u32x16 w = *reinterpret_cast<const CFET_CONST u32x16*>(rec + (k >> 2));
    uint32_t off[4];
    uint64_t m[4];
    double v[4];
    double2 xv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      off[u] = w[u] & kColMask;
      m[u] = FULL ? ~0ull : um[k + u];
      v[u] = __builtin_bit_cast(double, (uint64_t)w[4 + 2 * u] | ((uint64_t)w[5 + 2 * u] << 32));
    }
    if (GLOBAL && off[0] > tmask) {
#pragma unroll
      for (int u = 0; u < 4; ++u)
        xv[u] = x[(FULL || (m[u] & lanebit)) ? row ^ (int64_t)off[u] : row];
    } else {
#pragma unroll
      for (int u = 0; u < 4; ++u) xv[u] = t_lds(xt, qb, (off[u] & tmask) << 4);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (FULL || (m[u] & lanebit)) {
        ar = fma(v[u], xv[u].x, ar);
        ai = fma(v[u], xv[u].y, ai);
      }
    }
  }
}

// Entries of a slice's list: the sum of its four group sizes.
__device__ __forceinline__ int group_total(uint64_t g) {
  return (int)(g & 0xFFFF) + (int)((g >> 16) & 0xFFFF) + (int)((g >> 32) & 0xFFFF) +
         (int)(g >> 48);
}

// The common entries (held by every row of every slice), unweighted by term:
// (a1r, a1i) driven, (a0r, a0i) H0.  Every wavefront reads the same few
// entries, so their scalar loads hit the scalar cache.
template <bool RV, bool GLOBAL>
__device__ __forceinline__ void t_common_nt1(const uint32_t* cc, const double2* cv,
                                             const Rec4* crec, int ncd, int nch,
                                             uint64_t lanebit, uint32_t qb, int64_t row,
                                             uint32_t tmask, const double2* xt,
                                             const double2* __restrict__ x, double& a0r,
                                             double& a0i, double& a1r, double& a1i) {
  if (RV) {
    const CFET_CONST Rec4* rc = as_const(crec);
    t_group_rec<true, GLOBAL>(rc, nullptr, 0, ncd, lanebit, qb, row, tmask, xt, x, a1r, a1i);
    t_group_rec<true, GLOBAL>(rc, nullptr, ncd, nch, lanebit, qb, row, tmask, xt, x, a0r, a0i);
    return;
  }
  const CFET_CONST uint32_t* uc = as_const(cc);
  const CFET_CONST dvec2* uv = as_const(reinterpret_cast<const dvec2*>(cv));
  t_group<true, RV, GLOBAL>(uc, uv, nullptr, 0, ncd, lanebit, qb, row, tmask, xt, x, a1r, a1i);
  t_group<true, RV, GLOBAL>(uc, uv, nullptr, ncd, nch, lanebit, qb, row, tmask, xt, x, a0r, a0i);
}

// The common entries, any number of driven terms: (ar, ai) += w v x.
template <bool RV, bool GLOBAL>
__device__ __forceinline__ void t_common_any(const uint32_t* cc, const double2* cv, int nc,
                                             uint32_t qb, int64_t row, uint32_t tmask,
                                             const double2* xt, const double2* __restrict__ x,
                                             const double* wl, double& ar, double& ai) {
  const CFET_CONST uint32_t* uc = as_const(cc);
  const CFET_CONST dvec2* uv = as_const(reinterpret_cast<const dvec2*>(cv));
  for (int k = 0; k < nc; ++k) {
    const uint32_t ct = uc[k];
    const uint32_t off = ct & kColMask;
    const double2 xv = (GLOBAL && off > tmask) ? x[row ^ (int64_t)off]
                                               : t_lds(xt, qb, (off & tmask) << 4);
    const double w = wl[ct >> kTermShift];
    const double er = w * uv[k].x, ei = RV ? 0.0 : w * uv[k].y;
    ar = fma(er, xv.x, fma(-ei, xv.y, ar));
    ai = fma(er, xv.y, fma(ei, xv.x, ai));
  }
}

template <bool RV, bool GLOBAL>
__device__ __forceinline__ void t_shared_nt1(const CFET_CONST uint32_t* uc,
                                             const CFET_CONST dvec2* uv,
                                             const CFET_CONST uint64_t* um,
                                             const CFET_CONST Rec4* rec, uint64_t groups,
                                             uint64_t lanebit, uint32_t qb, int64_t row,
                                             uint32_t tmask, const double2* xt,
                                             const double2* __restrict__ x, double& a0r,
                                             double& a0i, double& a1r, double& a1i) {
  const int c0 = (int)(groups & 0xFFFF), c1 = (int)((groups >> 16) & 0xFFFF);
  const int c2 = (int)((groups >> 32) & 0xFFFF), c3 = (int)(groups >> 48);
  if (RV) {
    t_group_rec<true, GLOBAL>(rec, um, 0, c0, lanebit, qb, row, tmask, xt, x, a1r, a1i);
    t_group_rec<false, GLOBAL>(rec, um, c0, c1, lanebit, qb, row, tmask, xt, x, a1r, a1i);
    t_group_rec<true, GLOBAL>(rec, um, c0 + c1, c2, lanebit, qb, row, tmask, xt, x, a0r, a0i);
    t_group_rec<false, GLOBAL>(rec, um, c0 + c1 + c2, c3, lanebit, qb, row, tmask, xt, x, a0r,
                               a0i);
    return;
  }
  t_group<true, RV, GLOBAL>(uc, uv, um, 0, c0, lanebit, qb, row, tmask, xt, x, a1r, a1i);
  t_group<false, RV, GLOBAL>(uc, uv, um, c0, c1, lanebit, qb, row, tmask, xt, x, a1r, a1i);
  t_group<true, RV, GLOBAL>(uc, uv, um, c0 + c1, c2, lanebit, qb, row, tmask, xt, x, a0r, a0i);
  t_group<false, RV, GLOBAL>(uc, uv, um, c0 + c1 + c2, c3, lanebit, qb, row, tmask, xt, x, a0r,
                             a0i);
}

// Weighted sum of a slice's shared entries, any number of driven terms (the
// weight of each entry's term from the LDS table): (ar, ai) += w v x.
template <bool RV, bool GLOBAL>
__device__ __forceinline__ void t_shared_any(const CFET_CONST uint32_t* uc,
                                             const CFET_CONST dvec2* uv,
                                             const CFET_CONST uint64_t* um, int nu,
                                             uint64_t lanebit, uint32_t qb, int64_t row,
                                             uint32_t tmask, const double2* xt,
                                             const double2* __restrict__ x, const double* wl,
                                             double& ar, double& ai) {
  for (int k = 0; k < nu; ++k) {
    const uint32_t ct = uc[k];
    const uint32_t off = ct & kColMask;
    const uint64_t m = um[k];
    if (!(m & lanebit)) continue;
    const double2 xv = (GLOBAL && off > tmask) ? x[row ^ (int64_t)off]
                                               : t_lds(xt, qb, (off & tmask) << 4);
    const double w = wl[ct >> kTermShift];
    const double er = w * uv[k].x, ei = RV ? 0.0 : w * uv[k].y;
    ar = fma(er, xv.x, fma(-ei, xv.y, ar));
    ai = fma(er, xv.y, fma(ei, xv.x, ai));
  }
}

// Tile schedule: blocks are dealt to the 8 XCDs round-robin (block b on XCD
// b % 8); each XCD takes a contiguous eighth of the tiles, swept by its
// blocks together, so out-of-tile neighbours gathered by nearby tiles stay in
// that XCD's L2.
struct TileRange {
  int64_t first, end, stride;
};

__device__ __forceinline__ TileRange tile_range(int64_t ntiles) {
  constexpr int kXcds = 8;
  const int nb = gridDim.x;
  if (nb % kXcds != 0 || ntiles < nb) return {(int64_t)blockIdx.x, ntiles, (int64_t)nb};
  const int xcd = blockIdx.x % kXcds;
  const int rank = blockIdx.x / kXcds;
  const int64_t per = (ntiles + kXcds - 1) / kXcds;
  const int64_t beg = min(ntiles, (int64_t)xcd * per);
  const int64_t end = min(ntiles, beg + per);
  return {beg + rank, end, (int64_t)(nb / kXcds)};
}

// Row of the index q of the permuted order (pos: row position of bit b of q;
// bits 0 .. nbits-1 of q, nbits <= MAXB).
template <int MAXB>
__device__ __forceinline__ int64_t perm_row(const int32_t* pos, int nbits, int64_t q) {
  int64_t r = 0;
#pragma unroll
  for (int b = 0; b < MAXB; ++b)
    if (b < nbits) r |= ((q >> b) & 1) << pos[b];
  return r;
}

// Finishes the pending norm reduction of Lanczos step j and applies the early
// stop rule (the contract of the first SpMV launch of a step); returns false
// when the recurrence has stopped, else 1/||w_j|| in *inv.
template <int WAVES>
__device__ bool t_lanczos_start(const double* __restrict__ part_in, int np_in, LzScalars* L,
                                int j, double* red, double* inv) {
  if (j > 0 && L->brk[j - 1]) {
    if (blockIdx.x == 0 && threadIdx.x == 0) L->brk[j] = 1;
    return false;
  }
  const double nrm2 = t_sum_partials<WAVES>(part_in, np_in, red);
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
    if (stop) return false;
    *inv = 1.0 / beta0;
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
    if (stop) return false;
    *inv = 1.0 / b;
  }
  return true;
}

// First pass over tiles of consecutive rows: shared entries (in-tile from
// LDS, the rest gathered) and per-row slots.  LZ: Lanczos form (scale by
// inv, partials of Re<v_j, y>); else y = H x.
template <int NT, bool LZ, bool RV, int THREADS = kPass1Threads>
__global__ __launch_bounds__(THREADS) void k_tile_pass1(
    DevSELL S, int tbits, TermWeights tw, const double2* __restrict__ x, double2* __restrict__ y,
    const double* __restrict__ part_in, int np_in, double* __restrict__ part_out, LzScalars* L,
    int j) {
  extern __shared__ double2 xt[];
  const int T = 1 << tbits;
  double* red = reinterpret_cast<double*>(xt + T);
  double* wl = red + 20;
  double inv = 1.0;
  constexpr int WAVES = THREADS / 64;
  constexpr int LOADS = tile_loads<THREADS>();
  if (LZ && !t_lanczos_start<WAVES>(part_in, np_in, L, j, red, &inv)) return;
  if (threadIdx.x <= kMaxTerms) wl[threadIdx.x] = tw.w[threadIdx.x];
  const Wts W{tw.w[0], tw.w[1], wl};
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform: scalar metadata loads
  const uint64_t lanebit = 1ull << lane;
  const uint32_t tmask = (uint32_t)(T - 1);
  const TileRange R = tile_range(S.n >> tbits);
  double apart = 0.0;
  for (int64_t tile = R.first; tile < R.end; tile += R.stride) {
    const int64_t r0 = tile << tbits;
    // all loads in flight at once; a tile smaller than the block's share
    // (small operators) is read several times over (index masked into it)
#define CFET_TL(u)   \
  double2 b##u;      \
  if constexpr (u < LOADS) b##u = x[r0 + (((int)threadIdx.x + u * THREADS) & (T - 1))];
    CFET_TILE_8(CFET_TL)
#undef CFET_TL
    __syncthreads();  // the previous tile's readers are done (and wl is set)
    CFET_TILE_8(CFET_TS)
    __syncthreads();
    // the diagonal is read one slice ahead (latency overlap)
    double dn = (S.diag && wave < (T >> 6)) ? __builtin_nontemporal_load(S.diag + r0 + wave * 64 + lane)
                                            : 0.0;
    for (int sl = wave; sl < (T >> 6); sl += WAVES) {
      const int qloc = sl * 64 + lane;
      const int64_t row = r0 + qloc;
      const int64_t slice = (r0 >> 6) + sl;
      const double d = dn;
      if (S.diag && sl + WAVES < (T >> 6))
        dn = __builtin_nontemporal_load(S.diag + row + WAVES * 64);
      // the first per-row slot is read before the shared entries, so its
      // latency overlaps them
      // (operators whose entries are all shared or diagonal have no slots)
      const int width = S.slots > 0 ? as_const(S.slice_width)[slice] : 0;
      const int len = width > 0 ? S.rowlen[row] : 0;
      const int64_t base = width > 0 ? as_const(S.slice_ptr)[slice] : 0;
      const uint32_t* __restrict__ cp = S.colt + base + lane;
      const dvec2* __restrict__ vp = reinterpret_cast<const dvec2*>(S.val) + base + lane;
      uint32_t ct0 = 0u;
      dvec2 v0 = dvec2{0.0, 0.0};
      if (len > 0) {
        ct0 = __builtin_nontemporal_load(cp);
        v0 = __builtin_nontemporal_load(vp);
      }
      const uint32_t qb = t_lane_bytes(xt, qloc);
      double a0r = 0.0, a0i = 0.0, a1r = 0.0, a1i = 0.0;  // unweighted, by term (NT = 1)
      double ar = 0.0, ai = 0.0;                          // weighted
      if (NT == 1)
        t_common_nt1<RV, true>(S.ccolt, S.cval, S.crec, S.ncd, S.nch, lanebit, qb, row, tmask,
                               xt, x, a0r, a0i, a1r, a1i);
      else
        t_common_any<RV, true>(S.ccolt, S.cval, S.ncd + S.nch, qb, row, tmask, xt, x, wl, ar, ai);
      const int64_t ub = (int64_t)as_const(S.uhdr)[2 * slice];
      const uint64_t groups = as_const(S.uhdr)[2 * slice + 1];
      if (groups != 0) {
        const CFET_CONST uint32_t* uc = as_const(S.ucolt + ub);
        const CFET_CONST dvec2* uv = as_const(reinterpret_cast<const dvec2*>(S.uval) + ub);
        const CFET_CONST uint64_t* um = as_const(S.umask + ub);
        if (NT == 1)
          t_shared_nt1<RV, true>(uc, uv, um, as_const(S.urec + (ub >> 2)), groups, lanebit, qb,
                                 row, tmask, xt, x, a0r, a0i, a1r, a1i);
        else
          t_shared_any<RV, true>(uc, uv, um, group_total(groups), lanebit, qb, row, tmask, xt, x,
                                 wl, ar, ai);
      }
      for (int k = 0; k < len; ++k) {
        uint32_t ct = ct0;
        dvec2 v = v0;
        if (k > 0) {
          ct = __builtin_nontemporal_load(cp + (int64_t)k * 64);
          v = __builtin_nontemporal_load(vp + (int64_t)k * 64);
        }
        const int64_t col = (int64_t)(ct & kColMask);
        const double2 xv = ((col >> tbits) == (row >> tbits)) ? xt[col & tmask] : x[col];
        t_acc<NT, RV>(ct, v, xv, W, ar, ai);
      }
      if (S.diag) {
        const uint32_t dt = (uint32_t)S.diag_term << kTermShift;
        t_acc<NT, true>(dt, dvec2{d, 0.0}, xt[qloc], W, ar, ai);
      }
      if (NT == 1) {
        ar += W.w0 * a0r + W.w1 * a1r;
        ai += W.w0 * a0i + W.w1 * a1i;
      }
      if (LZ) {
        ar *= inv;
        ai *= inv;
        if (y) __builtin_nontemporal_store(dvec2{ar, ai}, reinterpret_cast<dvec2*>(y) + row);
        const double2 xr = xt[qloc];
        apart += (xr.x * ar + xr.y * ai) * inv;
      } else {
        y[row] = make_double2(ar, ai);
      }
    }
  }
  if (LZ) {
    apart = t_block_sum<WAVES>(apart, red);
    if (threadIdx.x == 0) part_out[blockIdx.x] = apart;
  }
}

// Second pass over tiles of the permuted order (every offset inside the tile):
// y[row] += H_hi x.  LZ: Lanczos form (state of the first pass, partials).
// Without LZ and with ct.psi set, the row's complete y feeds one term of the
// Chebyshev series (ChebTerm) instead of being stored.
template <int NT, bool LZ, bool RV, int THREADS = kPass2Threads>
__global__ __launch_bounds__(THREADS) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_tile_pass2(
    DevSELLHi H, int tbits, TermWeights tw, const double2* __restrict__ x,
    double2* __restrict__ y, double* __restrict__ part_out, const LzScalars* L, int j,
    ChebTerm ct) {
  extern __shared__ double2 xt[];
  const int T = 1 << tbits;
  double* red = reinterpret_cast<double*>(xt + T);
  double* wl = red + 20;
  double inv = 1.0;
  constexpr int WAVES = THREADS / 64;
  constexpr int LOADS = tile_loads<THREADS>();
  if (LZ) {
    if (L->brk[j]) return;
    inv = L->inv_nrm[j];
  }
  if (threadIdx.x <= kMaxTerms) wl[threadIdx.x] = tw.w[threadIdx.x];
  const Wts W{tw.w[0], tw.w[1], wl};
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform: scalar metadata loads
  const uint64_t lanebit = 1ull << lane;
  const uint32_t tmask = (uint32_t)(T - 1);
  // row bits (inside a tile) of the indices this thread loads and of this
  // lane inside a slice: the same for every tile
#define CFET_LOC(u) \
  const int64_t loc##u = perm_row<kTileBitsMax>(H.pos, tbits, ((int)threadIdx.x + u * THREADS) & (T - 1));
  CFET_TILE_8(CFET_LOC)
#undef CFET_LOC
  const int64_t lane_bits = perm_row<6>(H.pos, 6, lane);
  const TileRange R = tile_range(H.n >> tbits);
  double apart = 0.0;
  for (int64_t tile = R.first; tile < R.end; tile += R.stride) {
    const int64_t q0 = tile << tbits;
    const int64_t rbase = as_const(H.tile_row)[tile];
#define CFET_TL(u) \
  double2 b##u;    \
  if constexpr (u < LOADS) b##u = x[rbase | loc##u];
    CFET_TILE_8(CFET_TL)
#undef CFET_TL
    __syncthreads();
    CFET_TILE_8(CFET_TS)
    __syncthreads();
    // row of this lane in slice sl of the tile
    auto slice_row = [&](int sl) {
      int64_t srow = 0;  // row bits of the slice inside the tile (bits 6 .. tbits-1)
      for (int b = 6; b < tbits; ++b) srow |= (int64_t)((sl >> (b - 6)) & 1) << H.pos[b];
      return rbase | srow | lane_bits;
    };
    // the first pass's part of y is read one slice ahead (latency overlap)
    dvec2 y1n = dvec2{0.0, 0.0};
    if (wave < (T >> 6) && (!LZ || y)) {
      const int64_t r = slice_row(wave);
      y1n = LZ ? __builtin_nontemporal_load(reinterpret_cast<const dvec2*>(y) + r)
               : dvec2{y[r].x, y[r].y};
    }
    for (int sl = wave; sl < (T >> 6); sl += WAVES) {
      const int qloc = sl * 64 + lane;
      const int64_t slice = (q0 >> 6) + sl;
      const int64_t row = slice_row(sl);
      const dvec2 y1 = y1n;
      if (sl + WAVES < (T >> 6) && (!LZ || y)) {
        const int64_t r = slice_row(sl + WAVES);
        y1n = LZ ? __builtin_nontemporal_load(reinterpret_cast<const dvec2*>(y) + r)
                 : dvec2{y[r].x, y[r].y};
      }
      const uint32_t qb = t_lane_bytes(xt, qloc);
      double ar = 0.0, ai = 0.0;
      const int64_t ub = (int64_t)as_const(H.uhdr)[2 * slice];
      const uint64_t groups = as_const(H.uhdr)[2 * slice + 1];
      const CFET_CONST uint32_t* uc = as_const(H.ucolt + ub);
      const CFET_CONST dvec2* uv = as_const(reinterpret_cast<const dvec2*>(H.uval) + ub);
      const CFET_CONST uint64_t* um = as_const(H.umask + ub);
      if (NT == 1) {
        double a0r = 0.0, a0i = 0.0, a1r = 0.0, a1i = 0.0;
        t_common_nt1<RV, false>(H.ccolt, H.cval, H.crec, H.ncd, H.nch, lanebit, qb, row, tmask,
                                xt, x, a0r, a0i, a1r, a1i);
        if (groups != 0)
          t_shared_nt1<RV, false>(uc, uv, um, as_const(H.urec + (ub >> 2)), groups, lanebit, qb,
                                  row, tmask, xt, x, a0r, a0i, a1r, a1i);
        ar = W.w0 * a0r + W.w1 * a1r;
        ai = W.w0 * a0i + W.w1 * a1i;
      } else {
        t_common_any<RV, false>(H.ccolt, H.cval, H.ncd + H.nch, qb, row, tmask, xt, x, wl, ar,
                                ai);
        if (groups != 0)
          t_shared_any<RV, false>(uc, uv, um, group_total(groups), lanebit, qb, row, tmask, xt,
                                  x, wl, ar, ai);
      }
      if (LZ) {
        ar *= inv;
        ai *= inv;
        if (y)
          __builtin_nontemporal_store(dvec2{y1.x + ar, y1.y + ai},
                                      reinterpret_cast<dvec2*>(y) + row);
        const double2 xr = xt[qloc];
        apart += (xr.x * ar + xr.y * ai) * inv;
      } else if (ct.psi) {
        const double2 xr = xt[qloc];
        double wr = ct.scale * ((y1.x + ar) - ct.sigma * xr.x);
        double wi = ct.scale * ((y1.y + ai) - ct.sigma * xr.y);
        if (!ct.first) {
          const double2 pp = ct.prev[row];
          wr -= pp.x;
          wi -= pp.y;
        }
        ct.prev[row] = make_double2(wr, wi);
        const double2 p = ct.psi[row];
        ct.psi[row] = make_double2(p.x + ct.ck.x * wr - ct.ck.y * wi,
                                   p.y + ct.ck.x * wi + ct.ck.y * wr);
      } else {
        y[row] = make_double2(y1.x + ar, y1.y + ai);
      }
    }
  }
  if (LZ) {
    apart = t_block_sum<WAVES>(apart, red);
    if (threadIdx.x == 0) part_out[blockIdx.x] = apart;
  }
}

size_t tile_lds_bytes(int tbits) {
  return (size_t(1) << tbits) * sizeof(double2) + kTileScratch * sizeof(double);
}

template <class K>
hipError_t allow_lds(K kernel, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <int NT, bool LZ, bool RV>
hipError_t allow_pair() {
  const size_t b = tile_lds_bytes(kTileBitsMax);
  hipError_t e = allow_lds(k_tile_pass1<NT, LZ, RV>, b);
  if (e == hipSuccess) e = allow_lds(k_tile_pass2<NT, LZ, RV>, b);
  return e;
}

template <int NT, bool RV>
void launch_lz(const DevSELL& S, const DevSELLHi& H, int tbits, int nb, const TermWeights& tw,
               const double2* x, double2* y, const double* pin, int npin, double* pout,
               LzScalars* L, int j, hipStream_t st) {
  const size_t lds = tile_lds_bytes(tbits);
  hipLaunchKernelGGL((k_tile_pass1<NT, true, RV>), dim3(nb), dim3(kPass1Threads), lds, st, S,
                     tbits, tw, x, y, pin, npin, pout, L, j);
  hipLaunchKernelGGL((k_tile_pass2<NT, true, RV>), dim3(nb), dim3(kPass2Threads), lds, st, H,
                     tbits, tw, x, y, pout + nb, L, j, ChebTerm{});
}

template <int NT, bool RV>
void launch_ap(const DevSELL& S, const DevSELLHi& H, int tbits, int nb, const TermWeights& tw,
               const double2* x, double2* y, const ChebTerm& ct, hipStream_t st) {
  const size_t lds = tile_lds_bytes(tbits);
  hipLaunchKernelGGL((k_tile_pass1<NT, false, RV>), dim3(nb), dim3(kPass1Threads), lds, st, S,
                     tbits, tw, x, y, nullptr, 0, nullptr, nullptr, 0);
  hipLaunchKernelGGL((k_tile_pass2<NT, false, RV>), dim3(nb), dim3(kPass2Threads), lds, st, H,
                     tbits, tw, x, y, nullptr, nullptr, 0, ct);
}

}  // namespace

int tile_grid(int64_t n, int tbits, int num_cus) {
  const int64_t ntiles = n >> tbits;
  const int64_t want = std::max<int64_t>(1, int64_t(2) * std::max(num_cus, 1));
  return (int)std::max<int64_t>(1, std::min<int64_t>(ntiles, want));
}

hipError_t tile_prepare() {
  hipError_t e = allow_pair<1, true, true>();
  if (e == hipSuccess) e = allow_pair<1, true, false>();
  if (e == hipSuccess) e = allow_pair<0, true, true>();
  if (e == hipSuccess) e = allow_pair<0, true, false>();
  if (e == hipSuccess) e = allow_pair<1, false, false>();
  if (e == hipSuccess) e = allow_pair<0, false, false>();
  if (e == hipSuccess) e = allow_pair<1, false, true>();
  if (e == hipSuccess) e = allow_pair<0, false, true>();
  return e;
}

hipError_t launch_tile_lz_spmv(const DevSELL& S, const DevSELLHi& H, int tbits, int nb,
                               int nterms, bool real_vals, const TermWeights& tw,
                               const double2* x, double2* y, const double* pin, int npin,
                               double* pout, LzScalars* L, int j, hipStream_t st) {
  if (nterms == 1 && real_vals)
    launch_lz<1, true>(S, H, tbits, nb, tw, x, y, pin, npin, pout, L, j, st);
  else if (nterms == 1)
    launch_lz<1, false>(S, H, tbits, nb, tw, x, y, pin, npin, pout, L, j, st);
  else if (real_vals)
    launch_lz<0, true>(S, H, tbits, nb, tw, x, y, pin, npin, pout, L, j, st);
  else
    launch_lz<0, false>(S, H, tbits, nb, tw, x, y, pin, npin, pout, L, j, st);
  return hipGetLastError();
}

hipError_t launch_tile_apply(const DevSELL& S, const DevSELLHi& H, int tbits, int nb, int nterms,
                             bool real_vals, const TermWeights& tw, const double2* x, double2* y,
                             hipStream_t st) {
  const ChebTerm none{};
  if (nterms == 1 && real_vals) launch_ap<1, true>(S, H, tbits, nb, tw, x, y, none, st);
  else if (nterms == 1) launch_ap<1, false>(S, H, tbits, nb, tw, x, y, none, st);
  else if (real_vals) launch_ap<0, true>(S, H, tbits, nb, tw, x, y, none, st);
  else launch_ap<0, false>(S, H, tbits, nb, tw, x, y, none, st);
  return hipGetLastError();
}

hipError_t launch_tile_cheb(const DevSELL& S, const DevSELLHi& H, int tbits, int nb, int nterms,
                            bool real_vals, const TermWeights& tw, const double2* x, double2* y,
                            const ChebTerm& ct, hipStream_t st) {
  if (nterms == 1 && real_vals) launch_ap<1, true>(S, H, tbits, nb, tw, x, y, ct, st);
  else if (nterms == 1) launch_ap<1, false>(S, H, tbits, nb, tw, x, y, ct, st);
  else if (real_vals) launch_ap<0, true>(S, H, tbits, nb, tw, x, y, ct, st);
  else launch_ap<0, false>(S, H, tbits, nb, tw, x, y, ct, st);
  return hipGetLastError();
}

}  // namespace cfet
