// Internal declarations shared by the host driver and the device code.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/cfet.h"

namespace cfet {

constexpr int kMaxStages = 11;  // CF8:11 has the most exponentials
constexpr int kMaxTerms = CFET_MAX_TERMS;
constexpr int kMaxM = CFET_MAX_KRYLOV;
constexpr int kTermShift = 29;  // merged CSR: column | (term << 29)
constexpr uint32_t kColMask = (1u << kTermShift) - 1u;
constexpr int64_t kMaxDim = (int64_t(1) << kTermShift);
constexpr double kBreakdownRel = 1e-12;

struct SchemeTable {
  int s, M, order;
  double x[4], w[4];
  double g[kMaxStages][4];
};

struct DriveSpec {
  int kind;
  double A, omega, phi, Tp, tc, tau;
  std::vector<double> edges, u;
};

bool scheme_build(int id, SchemeTable* out);
double drive_eval(const DriveSpec& d, double t);
void step_weights(const SchemeTable& sc, const std::vector<DriveSpec>& drives, double t_n,
                  double dt, double* a, double* b);

// Per-exponential Lanczos scalars, written by block 0 of one kernel and read
// by all blocks of later kernels only (kernel boundaries order the accesses;
// no launch reads a field that the same launch writes).
struct LzScalars {
  double alpha[kMaxM];
  double beta[kMaxM];        // beta[j] = ||w_{j+1}||  (off-diagonal of T)
  double inv_nrm[kMaxM];     // stored basis vector j is w_j, v_j = w_j * inv_nrm[j]
  double beta0;
  double coef[2 * kMaxM];    // recombination: psi = sum_j coef_j w_j
  int32_t brk[kMaxM];        // brk[j] = 1: the recursion stopped at or before step j
  int32_t m_eff;             // effective Krylov dimension (final after the small exponential)
  int32_t pad;
};

// Device-side statistics and latched status.
struct DevStats {
  unsigned long long exponentials;
  unsigned long long matvecs;
  int32_t min_m_eff;
  int32_t breakdowns;
  int32_t status;
  int32_t pad;
  double last_norm2;
  long long seg[4];  // persistent kernels with timing on: wall-clock ticks of block 0 in
                     // SpMV phases, reductions/barriers, small exponentials, recombinations
};

// Term weights of one exponential: w[0] multiplies H0, w[1+k] multiplies H_k.
struct TermWeights {
  double w[kMaxTerms + 1];
};

// Device copy of the merged operator.
struct DevCSR {
  int64_t n = 0, nnz = 0;
  int64_t* rowptr = nullptr;   // int64[n+1]
  uint32_t* colt = nullptr;    // column | term << kTermShift
  double2* val = nullptr;      // complex128[nnz]
};

// Device copy of the operator in sliced-ELL form (sell.hip): slices of 64
// consecutive rows stored column-major and padded to the slice's longest row.
// Four entries of a shared list in one 64-byte record (the tiled kernels'
// real-valued form reads a batch of four with one scalar load): offsets |
// term, real values.
struct alignas(64) Rec4 {
  uint32_t col[4];
  double val[4];
  uint32_t pad[4];
};

struct DevSELL {
  int64_t n = 0;
  int64_t* slice_ptr = nullptr;  // first slot of each slice
  int32_t* slice_width = nullptr;
  int32_t* rowlen = nullptr;     // per-row entries of each row (slots in use)
  uint32_t* colt = nullptr;      // column | term << kTermShift (padding: 0)
  double2* val = nullptr;        // padding: 0
  int64_t slots = 0;
  // Optional shared part (null nuni: none).  nuni[s] entries of slice s, each
  // a column offset (column = row XOR offset), term and value that the rows
  // of umask (bit l: row 64 s + l) hold, are stored once at uptr[s]; rowlen
  // and the slots above count only the remaining per-row entries.
  int32_t* nuni = nullptr;
  int64_t* uptr = nullptr;
  uint32_t* ucolt = nullptr;     // offset | term << kTermShift
  double2* uval = nullptr;
  uint64_t* umask = nullptr;
  int64_t uslots = 0;
  // Optional (split layout only): the diagonal of one term, real-valued, one
  // double per row (rows without a diagonal entry hold 0); the per-row slots
  // then leave the diagonal out.
  double* diag = nullptr;
  int32_t diag_term = 0;
  // Split layout only: per slice the padded sizes of its four list groups
  // (driven terms held by all rows / by some rows, H0 all / some), 16 bits
  // each, group g at bits 16 g.
  uint64_t* ugroups = nullptr;
  // Split layout only: the entries every row of every slice holds with the
  // same offset, term and value (e.g. a driven sum of sigma_x with one
  // coefficient), stored once: ncd of driven terms, then nch of H0, each part
  // with the entries outside the tile first, padded to whole batches of four.
  uint32_t* ccolt = nullptr;
  double2* cval = nullptr;
  int32_t ncd = 0, nch = 0;
  // Split layout only: per slice {uptr, ugroups} side by side (one scalar
  // load for both).
  uint64_t* uhdr = nullptr;
  // Split layout with real values only: the shared lists (record i holds
  // entries 4 i .. 4 i + 3) and the common list as records.
  Rec4* urec = nullptr;
  Rec4* crec = nullptr;
};

// Second pass of the split shared-part layout (operators on 2^nbits rows whose
// shared entries connect rows that differ in a few bits, e.g. spin chains).
// Shared entries whose column offset (row XOR column) has a bit at or above a
// split bit are taken out of the first pass (DevSELL above) and stored here
// for slices of a bit-permuted row order: permuted index q has its bit b at
// position pos[b] of the row, row = sum_b bit_b(q) << pos[b], and slice s holds
// the 64 rows q = 64 s .. 64 s + 63.  The low permuted bits are the three
// lowest row bits (8 consecutive rows, 128 bytes of a vector) and then every
// bit that such an offset uses, so the rows one slice gathers from lie in the
// same small block of permuted indices as the slice itself: a tile of 2^tbits
// permuted indices holds every column its rows read.  Every entry of this
// pass is shared (mask of the slice rows holding it) and stores its offset in
// the permuted order (column index q ^ offset).
struct DevSELLHi {
  int64_t n = 0;
  int64_t nslices = 0;
  int nbits = 0;
  int32_t pos[32] = {};
  int32_t* nuni = nullptr;
  int64_t* uptr = nullptr;
  uint32_t* ucolt = nullptr;     // permuted offset | term << kTermShift
  double2* uval = nullptr;
  uint64_t* umask = nullptr;     // bit l: row of permuted index 64 s + l
  int64_t uslots = 0;
  uint64_t* ugroups = nullptr;   // per slice the four group sizes, as in DevSELL
  int64_t* tile_row = nullptr;   // row of the first index of each tile of 2^tbits
                                 // permuted indices (the tile's row bits above tbits)
  uint32_t* ccolt = nullptr;     // common entries of every slice, as in DevSELL
  double2* cval = nullptr;
  int32_t ncd = 0, nch = 0;
  uint64_t* uhdr = nullptr;      // per slice {uptr, ugroups}, as in DevSELL
  Rec4* urec = nullptr;          // records, as in DevSELL
  Rec4* crec = nullptr;
};

int sell_grid(int64_t n);
// LDS-tiled SpMV of the split layout (tile.hip): tiles of 2^tbits indices of
// each pass's order (tbits <= kTileBitsMax); both passes in one call.
constexpr int kTileBitsMax = 12;
int tile_grid(int64_t n, int tbits, int num_cus);
// Allows the tile kernels their LDS (once per process and device).
hipError_t tile_prepare();
// One term of the Chebyshev series fused into the second pass's epilogue:
// w = scale (y - sigma x) - prev (prev omitted when first), prev <- w,
// psi += ck w, with y = H x complete for the row (y itself is not written).
struct ChebTerm {
  double2* prev;
  double2* psi;
  double scale;
  double sigma;
  double2 ck;
  int first;
};
// y = H x, then the Chebyshev term on the split layout (the first pass writes
// y, the second applies the term instead of storing y).
hipError_t launch_tile_cheb(const DevSELL& S, const DevSELLHi& H, int tbits, int nb, int nterms,
                            bool real_vals, const TermWeights& tw, const double2* x, double2* y,
                            const ChebTerm& ct, hipStream_t st);
// y = H x (real_vals: every stored value is real; real products only).
hipError_t launch_tile_apply(const DevSELL& S, const DevSELLHi& H, int tbits, int nb, int nterms,
                             bool real_vals, const TermWeights& tw, const double2* x, double2* y,
                             hipStream_t st);
// Lanczos SpMV, same contract as launch_sell_lz_spmv; the alpha partials of
// the two passes go to pout[0 .. 2 nb).
// real_vals: every stored value of both passes has imaginary part 0.
hipError_t launch_tile_lz_spmv(const DevSELL& S, const DevSELLHi& H, int tbits, int nb,
                               int nterms, bool real_vals, const TermWeights& tw,
                               const double2* x, double2* y, const double* pin, int npin,
                               double* pout, LzScalars* L, int j, hipStream_t st);
hipError_t launch_sell_apply(const DevSELL& S, int nterms, const TermWeights& tw, const double2* x,
                             double2* y, hipStream_t st);
hipError_t launch_sell_lz_spmv(const DevSELL& S, int nterms, const TermWeights& tw,
                               const double2* x, double2* y, const double* pin, int npin,
                               double* pout, LzScalars* L, int j, hipStream_t st);

// Launch helpers (device.hip).
struct LaunchPlan {
  int G;        // lanes per row in the SpMV
  int nb_spmv;  // blocks of the SpMV kernels
  int nb_vec;   // blocks of the elementwise kernels
};

LaunchPlan make_plan(int64_t n, int64_t nnz);

hipError_t launch_apply(const DevCSR& A, int nterms, const LaunchPlan& plan, const TermWeights& tw,
                        const double2* x, double2* y, hipStream_t st);

// Multi-kernel exponential: psi <- exp(-i dt H_w) psi using m Lanczos vectors.
struct EventPool {
  hipEvent_t* begin = nullptr;
  hipEvent_t* end = nullptr;
  int cap = 0;
  int used = 0;
};

struct ExpWork {
  double2* const* W_host;  // basis pointers: W[0] = psi, W[j] = workspace (W[j] = W[1] + (j-1) n)
  const DevSELL* sell;   // SELL layout for the SpMV (null: CSR)
  const DevSELLHi* hi = nullptr;  // second pass of a split SELL layout (null: none)
  int tbits = 0;                  // its tile size (2^tbits indices)
  int nb_tile = 0;                // and grid
  bool tile_real = false;         // its stored values are all real
  EventPool* events;     // optional SpMV timing (null: off)
  double* partA;         // partial sums (norms)
  double* partB;         // partial sums (alpha)
  LzScalars* S;          // scalar block of the exponential
  DevStats* stats;
  const TermWeights* twp = nullptr;  // if set, the SpMV reads the weights here (device)
};

// out[i] = in[idx[i]] for i < n (idx a permutation of 0..n-1; out and in distinct)
hipError_t launch_permute(double2* out, const double2* in, const int32_t* idx, int64_t n,
                          hipStream_t st);
hipError_t launch_norm_start(const double2* psi, int64_t n, const LaunchPlan& plan, double* part,
                             hipStream_t st);
hipError_t launch_exponential(const DevCSR& A, int nterms, const LaunchPlan& plan,
                              const TermWeights& tw, double dt, int m, const ExpWork& wk,
                              hipStream_t st);
// The exponential in two parts: the Lanczos recurrence with the small
// exponential (basis W[1..], scalars S; W[0] is only read), then the
// recombination W[0] <- sum_j coef_j W[j].
hipError_t launch_lanczos(const DevCSR& A, int nterms, const LaunchPlan& plan,
                          const TermWeights& tw, double dt, int m, const ExpWork& wk,
                          hipStream_t st);
hipError_t launch_combine(int64_t n, const LaunchPlan& plan, const ExpWork& wk, hipStream_t st);
hipError_t launch_final_norm(const double* part, int np, DevStats* st_dev, hipStream_t st);

// Fidelity gradient (grad.hip).
// One exponential of the backward sweep, as read by its replayed kernel graph.
struct GradRec {
  TermWeights tw;  // weights of H0 and the driven terms
  int np;          // (piece, weight) pairs of db/du
  int p[4];
  double w[4];
};
// Copies record *cursor to cur, the state before that exponential to pb and,
// if lam_copy is set, lam to lam_copy.
hipError_t launch_grad_prologue(const GradRec* recs, const int* cursor, GradRec* cur,
                                const double2* before, int64_t n, double2* pb,
                                const double2* lam, double2* lam_copy, unsigned long long* bar,
                                int bar_words, int* fault, hipStream_t st);
// mmax: bound on both Krylov dimensions (one wavefront serves m <= 32)
hipError_t launch_frechet_small_rec(const LzScalars* Spsi, const LzScalars* Slam,
                                    const double2* C, double dt, const GradRec* cur,
                                    double2* dz, DevStats* stats, int* cursor, int mmax,
                                    hipStream_t st);
int frechet_c_blocks(int64_t n);
int frechet_part_blocks(int64_t n);  // blocks of partials either C kernel writes, at most
// C from the stored lambda basis and Y_j = H_k* w_psi,j (exported by the
// persistent recurrence from psi), same output as launch_frechet_c
hipError_t launch_frechet_dots(int64_t n, const double2* lam0, const double2* lam_rest,
                               const double2* Y, const LzScalars* Spsi, const LzScalars* Slam,
                               double2* part, double2* C, hipStream_t st);
hipError_t launch_frechet_c(const DevCSR& A, int term, const double2* psi0,
                            const double2* psi_rest, const double2* lam0, const double2* lam_rest,
                            const LzScalars* Spsi, const LzScalars* Slam, double2* part,
                            double2* C, hipStream_t st);
// Chebyshev series: v0 = psi, psi = c0 psi (and the statistics of one
// exponential of K products); one term: w = scale (y - sigma v) - prev (no prev
// when first), prev = w, psi += ck w.
hipError_t launch_cheb_start(double2* psi, double2* v0, int64_t n, double2 c0, int K,
                             DevStats* st_dev, hipStream_t st);
hipError_t launch_cheb_update(const double2* y, const double2* v, double2* prev, double2* psi,
                              int64_t n, double scale, double sigma, bool first, double2 ck,
                              hipStream_t st);
// part[0 .. dist2_blocks(n) - 1] = block partial sums of ||a - b||^2
int dist2_blocks(int64_t n);
hipError_t launch_dist2(const double2* a, const double2* b, int64_t n, double* part,
                        hipStream_t st);
int zdot_blocks(int64_t n);
hipError_t launch_zdot(const double2* a, const double2* b, int64_t n, double2* part,
                       double2* out, hipStream_t st);
hipError_t launch_zero2(double2* p, int n, hipStream_t st);
// Persistent propagation (persistent.hip): one launch for a whole call.

struct PersistArgs {
  const int64_t* rowptr;
  const uint32_t* colt;
  const double2* val;
  int64_t n;
  int nterms;
  const double* wts;        // [(step*s + i)*(1+nterms) + t]: t = 0 -> a_i, t > 0 -> b_{i,t-1}
  int s;
  int64_t nsteps;
  int m;
  double dt;
  double2* psi;
  double2* basis;           // basis vector j >= 1 at basis + (j-1)*n
  double2* zbuf;            // 2 * n: H u_k of the last two Lanczos steps
  double* part;             // 2 parities x gridDim records of two partial sums
  unsigned long long* bar;  // barrier counters (persistent_barrier_words(), reset per launch)
  int* fault;               // set when a barrier wait times out
  DevStats* stats;
  long long spin_limit;     // barrier wait limit in wall-clock ticks
  int timing;               // accumulate per-segment wall-clock time (block 0)
  double2* save;            // optional: psi before exponential e of the call at save + e*n
  LzScalars* export_T;      // optional: Lanczos scalars of the (last) exponential, with the
                            // stored basis psi, basis[..] scaled as v_j = w_j * inv_nrm[j]
  int no_combine;           // 1: stop after the Lanczos recurrence (psi unchanged)
  double2* export_Y;        // optional, one driven term only: H_1 w_k of every stored
                            // Lanczos vector w_k (k < m) at export_Y + k*n
  int export_each;          // 1: export_T / export_Y hold one record per exponential of
                            // the call (application order e: export_T + e,
                            // export_Y + e*m*n) instead of the last one only
  int real_vals;            // 1: every imaginary part of val is 0 (real-valued kernels)
};

// reset = false: the caller has cleared args.bar and args.fault on the stream
hipError_t launch_persistent(const PersistArgs& args, int preset, bool single, int nblocks,
                             hipStream_t st, bool reset = true);
// real: occupancy of the real-valued form (the one launched for real operators)
hipError_t persistent_max_blocks(int preset, int nterms, bool real, int* out);
int persistent_rows_per_block(int preset, bool single);
int persistent_block_threads(int preset, bool single);
int persistent_barrier_words();
int persistent_choose_preset(int max_row, int64_t min_rows_per_block, bool single);

// File-scope device array of the allocation-free entry point (noalloc.hip):
// its size, and its address on `device` (looked up once per device; the
// device must be current).
size_t static_scratch_bytes();
hipError_t static_scratch(int device, void** out);

hipError_t launch_tridiag_expm(const double* alpha, const double* beta, int k, double dt,
                               double2* c, int32_t* status, hipStream_t st);
hipError_t launch_stats_init(DevStats* st_dev, hipStream_t st);

}  // namespace cfet
