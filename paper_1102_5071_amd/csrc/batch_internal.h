// Internal declarations of the batched path: many independent trajectories
// advanced together, one kernel per Lanczos phase over all of them.
//
// Instances that share their driven operators (and the dimension) form a
// group of at most 64; a group's vectors are stored interleaved, element
// (row r, instance j) at voff + r * B + j, so one wavefront lane per instance
// gathers the same column of all instances in one contiguous request and the
// shared operator row is read once for the whole group (an SpMM over the
// group).  The instances' own H0 is kept as a dense diagonal plus, if any, an
// off-diagonal CSR per instance.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "cfet_internal.h"

namespace cfet {

constexpr int kBatchMaxGroup = 64;  // instances per group (one wavefront lane each)
// wavefronts per block of the row kernels: chosen at create among these
// (with the rows each lane covers); every row kernel of a batch uses the
// same block layout, since the block partials follow it
constexpr int kBatchWaveChoices[] = {2, 4, 8};
constexpr int kBatchDefaultWaves = 4;
constexpr int kBatchMaxK1 = 8;      // 1 + driven terms

struct BGroup {
  int64_t n;            // rows
  int64_t voff;         // element offset of the group's vectors
  int B;                // instances in the group
  int lpr;              // lanes per row: smallest power of two >= B
  int rows_per_block;   // rows handled by one block of the row kernels
  int nblocks;          // blocks of the group in the row-kernel grid
  int block0;           // first block of the group in that grid
  int slot0;            // first instance slot of the group
  int shared_h0;        // 1: H0 is term 0 of the shared operator
  int pad;
  const int64_t* rowptr;  // shared operator, n + 1 row pointers
  const uint32_t* colt;   // column | term << kTermShift
  const double2* val;
  const double2* diag;    // [n][B] H0 diagonal of each instance (shared_h0 == 0)
  const int64_t* orp;     // [B][n + 1] H0 off-diagonal rows per instance, or null
  const int32_t* ocol;
  const double2* oval;
};

// Per-slot Lanczos state and statistics (slot = instance in group order).
struct BSlots {
  double* alpha;    // [slot][kMaxM]
  double* beta;     // [slot][kMaxM]
  double* inv;      // [slot][kMaxM] 1 / norm of stored basis vector l
  double2* coef;    // [slot][kMaxM] recombination coefficients
  double* beta0;    // [slot]
  int* m_eff;       // [slot]
  int* done;        // [slot] 1 once the running exponential's basis is complete
  int* mcap;        // [slot] min(m, n)
  long long* matvecs;     // [slot] cumulative
  long long* expos;       // [slot]
  long long* breakdowns;  // [slot] stopped by the breakdown rule
  long long* early;       // [slot] stopped by the error estimate
  int* min_m;             // [slot]
  int* max_m;             // [slot]
};

// Parameters read by every launch from device memory, so that a captured
// step graph stays valid across calls.
struct BState {
  const double* wts;   // [expo][slot][K1] weights in application order
  long long cursor;    // exponential index into wts (advanced on the device)
  double dt;
  double tol;
  int nslots;
  int K1;
  int status;          // latched device status: last field, never rewritten by the
                       // per-call parameter upload (cleared when reported)
};

struct BLaunch {
  const BGroup* groups;  // device array
  int ngroups;
  int total_blocks;
  int nslots;
  int64_t ntot;          // elements of one packed vector
  double2* V;            // basis: vector l at V + l * ntot (vector 0 = psi)
  double2* Y;            // H v_k
  double* part;          // [slot][pstride] partial sums: instance slot, block of its group
  int64_t pstride;
  int waves;             // wavefronts per block of the row kernels (2, 4 or 8)
  BSlots S;
  BState* st;
};

enum BScalarMode { kBStart = 0, kBAlpha = 1, kBBeta = 2 };

hipError_t batch_norm(const BLaunch& L, hipStream_t s);
hipError_t batch_scalars(const BLaunch& L, int mode, int k, hipStream_t s);
hipError_t batch_spmm(const BLaunch& L, int k, hipStream_t s);
hipError_t batch_axpy(const BLaunch& L, int k, hipStream_t s);
hipError_t batch_combine(const BLaunch& L, hipStream_t s);
hipError_t batch_advance(const BLaunch& L, hipStream_t s);
hipError_t batch_set_cursor(const BLaunch& L, long long v, hipStream_t s);
hipError_t batch_pack(const BLaunch& L, const double2* user, const int64_t* uoff, hipStream_t s);
hipError_t batch_unpack(const BLaunch& L, double2* user, const int64_t* uoff, hipStream_t s);
hipError_t batch_stats_reset(const BLaunch& L, hipStream_t s);

}  // namespace cfet
