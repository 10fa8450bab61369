// Host side of libcfet: argument validation, CSR merge and upload, workspace
// management and the CFET step loop that enqueues the device kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstddef>
#include <cstring>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "cfet_internal.h"
#include "host_common.h"

using cfet::DevCSR;
using cfet::DevStats;
using cfet::DriveSpec;
using cfet::LzScalars;
using cfet::SchemeTable;

struct cfet_ctx {
  int device = 0;
  int64_t n = 0;
  int nterms = 0;
  DevCSR A;
  cfet::DevSELL sell;
  cfet::DevSELLHi hi;       // second pass of the split layout (hi.nuni null: none)
  int tbits = 0;            // tile size of its LDS-tiled kernels (2^tbits rows)
  int nb_tile = 0;          // and their grid
  bool tile_real = false;   // every value stored in the split layout is real
  bool use_sell = false;
  int64_t sell_bytes = 0;   // stored SELL data one application reads
  // row order of the CSR paths (null: the caller's): row i of the stored
  // operator is the caller's row perm[i], caller row j is row iperm[j];
  // pv, pv2 hold vectors in that order
  int32_t* perm = nullptr;
  int32_t* iperm = nullptr;
  double2* pv = nullptr;
  double2* pv2 = nullptr;
  cfet::LaunchPlan plan{};
  std::vector<DriveSpec> drives;
  // Krylov workspace (grown on demand)
  int m_alloc = 0;
  double2* basis = nullptr;         // (m_alloc - 1) * n vectors
  std::vector<double2*> h_W;        // host copy of the pointers (W[0] patched per call)
  double* partA = nullptr;
  double* partB = nullptr;
  LzScalars* S = nullptr;           // Lanczos scalars of the running exponential
  DevStats* stats = nullptr;
  DevStats* stats_host = nullptr;   // pinned mirror, refreshed at the end of each call
  hipStream_t last_stream = nullptr;
  cfet::EventPool events;
  bool profiling = false;
  bool seg_timers = false;          // profiling also runs the persistent segment timers
  int64_t timed_launches = 0;
  double timed_ms = 0.0;
  bool have_work = false;
  int last_path = 0;
  uint32_t flags = 0;
  // persistent paths
  double* d_wts = nullptr;          // per-call weight table on the device
  size_t wts_cap = 0;               // doubles
  double* h_wts = nullptr;          // pinned staging buffer
  size_t h_wts_cap = 0;
  hipEvent_t wts_copied = nullptr;  // the staging buffer may be rewritten once this fired
  bool wts_pending = false;
  double* d_part = nullptr;         // 4 * blocks partial sums (2 parities x 2 sums)
  double2* zbuf = nullptr;          // 2 * n: H u_k of the last two Lanczos steps
  int part_cap = 0;
  unsigned long long* d_bar = nullptr;
  int* d_fault = nullptr;
  long long spin_limit = 0;
  int num_cus = 0;
  int max_row = 0;                  // longest row of the merged operator
  bool real_vals = false;           // every stored value has imaginary part 0
  int preset_single = -1;           // register preset of the one-workgroup kernel (-1: none)
  int preset_coop = -1;             // register preset of the cooperative kernel (-1: none)
  int coop_blocks = 0;              // grid of the cooperative kernel
  // Gershgorin interval of each term (0: H0, 1 + k: H_k), for the Chebyshev
  // exponential's spectral bounds
  std::vector<double> glo, ghi;
  std::string err;
};

namespace {

thread_local std::string g_err;

// automatic path choice by dimension
constexpr int64_t kAutoSingleMaxN = 4096;
constexpr int64_t kAutoCoopMaxN = int64_t(1) << 22;
// Grid of the cooperative kernel: one block per CU, but at least ~128 rows per
// block; each block owns ceil(n / blocks) consecutive rows.
int64_t coop_grid_blocks(int64_t n, int cus) {
  return std::max<int64_t>(1, std::min<int64_t>(cus, (n + 127) / 128));
}

// device bytes the gradient may spend on keeping the recomputed projections
constexpr size_t kGradStoreMax = size_t(16) << 30;
static_assert(sizeof(cfet_dt_choice) == 96 && offsetof(cfet_dt_choice, rounds) == 92,
              "cfet_dt_choice layout is part of the ABI");
static_assert(sizeof(cfet_stats_t) == 120 && offsetof(cfet_stats_t, matrix_bytes) == 112,
              "cfet_stats_t layout is part of the ABI");

int fail(cfet_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  g_err = msg;
  return code;
}

int hip_fail(cfet_ctx* c, hipError_t e, const char* what) {
  std::string msg = std::string(what) + ": " + hipGetErrorString(e);
  const int code = (e == hipErrorOutOfMemory) ? CFET_ENOMEM : CFET_EDEVICE;
  return fail(c, code, msg);
}

using cfet::HostCSR;

int load_csr(cfet_ctx* c, const cfet_csr* m, const char* name, HostCSR* h) {
  const int rc = cfet::load_csr(c->err, m, name, h);
  if (rc != CFET_OK) g_err = c->err;
  return rc;
}

int validate_csr(cfet_ctx* c, const HostCSR& h, const char* name) {
  const int rc = cfet::validate_csr(c->err, h, name);
  if (rc != CFET_OK) g_err = c->err;
  return rc;
}

int check_hermitian(cfet_ctx* c, const HostCSR& h, const char* name) {
  const int rc = cfet::check_hermitian(c->err, h, name);
  if (rc != CFET_OK) g_err = c->err;
  return rc;
}

int copy_drive(cfet_ctx* c, const cfet_drive& d, DriveSpec* out) {
  const int rc = cfet::copy_drive(c->err, d, out);
  if (rc != CFET_OK) g_err = c->err;
  return rc;
}

using cfet::is_device_ptr;

void free_events(cfet_ctx* c) {
  for (int i = 0; i < c->events.cap; ++i) {
    if (c->events.begin[i]) (void)hipEventDestroy(c->events.begin[i]);
    if (c->events.end[i]) (void)hipEventDestroy(c->events.end[i]);
  }
  delete[] c->events.begin;
  delete[] c->events.end;
  c->events = cfet::EventPool();
}

// Sum the durations of the recorded event pairs (their stream must be done).
void harvest_events(cfet_ctx* c) {
  for (int i = 0; i < c->events.used; ++i) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, c->events.begin[i], c->events.end[i]) == hipSuccess) {
      c->timed_ms += ms;
      c->timed_launches += 1;
    } else {
      (void)hipGetLastError();
    }
  }
  c->events.used = 0;
}

void free_ctx(cfet_ctx* c) {
  if (!c) return;
  free_events(c);
  if (c->A.rowptr) (void)hipFree(c->A.rowptr);
  if (c->A.colt) (void)hipFree(c->A.colt);
  if (c->A.val) (void)hipFree(c->A.val);
  if (c->perm) (void)hipFree(c->perm);
  if (c->iperm) (void)hipFree(c->iperm);
  if (c->pv) (void)hipFree(c->pv);
  if (c->pv2) (void)hipFree(c->pv2);
  if (c->sell.slice_ptr) (void)hipFree(c->sell.slice_ptr);
  if (c->sell.slice_width) (void)hipFree(c->sell.slice_width);
  if (c->sell.rowlen) (void)hipFree(c->sell.rowlen);
  if (c->sell.colt) (void)hipFree(c->sell.colt);
  if (c->sell.val) (void)hipFree(c->sell.val);
  if (c->sell.nuni) (void)hipFree(c->sell.nuni);
  if (c->sell.uptr) (void)hipFree(c->sell.uptr);
  if (c->sell.ucolt) (void)hipFree(c->sell.ucolt);
  if (c->sell.uval) (void)hipFree(c->sell.uval);
  if (c->sell.umask) (void)hipFree(c->sell.umask);
  if (c->sell.diag) (void)hipFree(c->sell.diag);
  if (c->sell.ugroups) (void)hipFree(c->sell.ugroups);
  if (c->hi.ugroups) (void)hipFree(c->hi.ugroups);
  if (c->hi.nuni) (void)hipFree(c->hi.nuni);
  if (c->hi.uptr) (void)hipFree(c->hi.uptr);
  if (c->hi.ucolt) (void)hipFree(c->hi.ucolt);
  if (c->hi.uval) (void)hipFree(c->hi.uval);
  if (c->hi.umask) (void)hipFree(c->hi.umask);
  if (c->hi.tile_row) (void)hipFree(c->hi.tile_row);
  if (c->sell.urec) (void)hipFree(c->sell.urec);
  if (c->hi.urec) (void)hipFree(c->hi.urec);
  if (c->sell.crec) (void)hipFree(c->sell.crec);
  if (c->hi.crec) (void)hipFree(c->hi.crec);
  if (c->sell.uhdr) (void)hipFree(c->sell.uhdr);
  if (c->hi.uhdr) (void)hipFree(c->hi.uhdr);
  if (c->sell.ccolt) (void)hipFree(c->sell.ccolt);
  if (c->sell.cval) (void)hipFree(c->sell.cval);
  if (c->hi.ccolt) (void)hipFree(c->hi.ccolt);
  if (c->hi.cval) (void)hipFree(c->hi.cval);
  if (c->basis) (void)hipFree(c->basis);
  if (c->partA) (void)hipFree(c->partA);
  if (c->partB) (void)hipFree(c->partB);
  if (c->S) (void)hipFree(c->S);
  if (c->stats) (void)hipFree(c->stats);
  if (c->stats_host) (void)hipHostFree(c->stats_host);
  if (c->d_wts) (void)hipFree(c->d_wts);
  if (c->h_wts) (void)hipHostFree(c->h_wts);
  if (c->wts_copied) (void)hipEventDestroy(c->wts_copied);
  if (c->d_part) (void)hipFree(c->d_part);
  if (c->zbuf) (void)hipFree(c->zbuf);
  if (c->d_bar) (void)hipFree(c->d_bar);
  if (c->d_fault) (void)hipFree(c->d_fault);
  delete c;
}

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) == hipSuccess && prev != dev) (void)hipSetDevice(dev);
    else prev = -1;
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

int ensure_workspace(cfet_ctx* c, int m) {
  if (m <= c->m_alloc) return CFET_OK;
  hipError_t e;
  if (c->basis) {
    e = hipFree(c->basis);
    c->basis = nullptr;
    c->m_alloc = 0;
  }
  const size_t bytes = size_t(m - 1) * size_t(c->n) * sizeof(double2);
  if (bytes > 0) {
    e = hipMalloc(&c->basis, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      c->basis = nullptr;
      return fail(c, CFET_ENOMEM, "cannot allocate the Krylov basis (" +
                                      std::to_string(bytes >> 20) + " MiB)");
    }
  }
  c->h_W.assign(cfet::kMaxM, nullptr);
  for (int j = 1; j < m; ++j) c->h_W[j] = c->basis + size_t(j - 1) * size_t(c->n);
  c->m_alloc = m;
  return CFET_OK;
}

// The last index K of the Chebyshev series kept for tol: the smallest K >= 0
// with 2 (|theta|/2)^(K+1) / (K+1)! / (1 - q) <= tol, q = |theta| / (2 (K+2)) < 1
// (|J_k(theta)| <= (|theta|/2)^k / k! and |T_k| <= 1 on [-1, 1]).
int cheb_terms(double theta, double tol) {
  const double x = std::fabs(theta) / 2.0;
  if (x == 0.0) return 0;
  const double lt = std::log(tol);
  for (int k = 0;; ++k) {
    const double q = x / double(k + 2);
    if (q < 1.0) {
      const double lg = std::log(2.0) + double(k + 1) * std::log(x) - std::lgamma(double(k + 2)) -
                        std::log1p(-q);
      if (lg <= lt) return k;
    }
  }
}

// J_0(theta) .. J_K(theta): the power series for |theta| <= 1, Miller's
// backward recurrence J_{k-1} = (2k/x) J_k - J_{k+1} from far above K,
// normalised by J_0 + 2 sum J_2k = 1, otherwise; J_k(-x) = (-1)^k J_k(x).
void bessel_j(double theta, int K, double* J) {
  const double x = std::fabs(theta);
  if (x <= 1.0) {
    for (int k = 0; k <= K; ++k) {
      // (x/2)^k / k! sum_m (-(x/2)^2)^m / (m! (m+k)!)
      double term = 1.0;
      for (int i = 1; i <= k; ++i) term *= (x / 2.0) / double(i);
      double sum = 0.0;
      const double q = -(x / 2.0) * (x / 2.0);
      for (int m = 0; m < 40 && term != 0.0; ++m) {
        sum += term;
        term *= q / (double(m + 1) * double(m + 1 + k));
      }
      J[k] = sum;
    }
  } else {
    const double top = std::max(double(K), x);
    int M = int(top + 2.0 * std::sqrt(40.0 * (top + 1.0))) + 20;
    M += M & 1;
    double jp = 0.0, jk = 1e-30, norm = 0.0;
    for (int k = M; k >= 1; --k) {
      const double jm = (2.0 * double(k) / x) * jk - jp;
      jp = jk;
      jk = jm;                              // jk = J_{k-1} (unnormalised)
      if (k - 1 <= K) J[k - 1] = jk;
      if ((k - 1) % 2 == 0 && k - 1 > 0) norm += 2.0 * jk;
      if (std::fabs(jk) > 1e200) {
        jk *= 1e-200;
        jp *= 1e-200;
        norm *= 1e-200;
        for (int i = k - 1; i <= K; ++i) J[i] *= 1e-200;
      }
    }
    norm += jk;                             // + J_0
    for (int k = 0; k <= K; ++k) J[k] /= norm;
  }
  if (theta < 0.0)
    for (int k = 1; k <= K; k += 2) J[k] = -J[k];
}

// 1: one kernel per phase, 2: one workgroup, 3: cooperative grid
bool single_fits(const cfet_ctx* c) { return c->preset_single >= 0; }

bool coop_fits(const cfet_ctx* c) { return c->preset_coop >= 0 && c->coop_blocks > 0; }

int choose_path(const cfet_ctx* c) {
  if (c->flags & CFET_FORCE_MULTIKERNEL) return 1;
  if ((c->flags & CFET_FORCE_SINGLE) && single_fits(c)) return 2;
  if ((c->flags & CFET_FORCE_COOPERATIVE) && coop_fits(c)) return 3;
  if (c->flags & (CFET_FORCE_SINGLE | CFET_FORCE_COOPERATIVE)) return 1;
  if (c->n <= kAutoSingleMaxN && single_fits(c)) return 2;
  if (c->n <= kAutoCoopMaxN && coop_fits(c)) return 3;
  return 1;
}

int propagate_persistent(cfet_ctx* c, void* psi_dev, double t0, double dt, int64_t nsteps,
                         const SchemeTable& sc, int m, int path, hipStream_t st,
                         double2* save = nullptr, LzScalars* export_T = nullptr,
                         double2* export_Y = nullptr) {
  const int nt1 = c->nterms + 1;
  if (c->profiling && c->events.used > 0) {
    (void)hipStreamSynchronize(c->last_stream);
    harvest_events(c);
  }
  const size_t need = size_t(nsteps) * sc.s * nt1;
  hipError_t e;
  // the pinned staging buffer is reused: wait for its previous upload
  if (c->wts_pending) {
    e = hipEventSynchronize(c->wts_copied);
    if (e != hipSuccess) return hip_fail(c, e, "wait for the weight upload");
    c->wts_pending = false;
  }
  if (need > c->h_wts_cap) {
    if (c->h_wts) (void)hipHostFree(c->h_wts);
    c->h_wts = nullptr;
    c->h_wts_cap = 0;
    e = hipHostMalloc(&c->h_wts, need * sizeof(double));
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(c, CFET_ENOMEM, "cannot allocate the pinned weight table");
    }
    c->h_wts_cap = need;
  }
  if (need > c->wts_cap) {
    if (c->d_wts) (void)hipFree(c->d_wts);
    c->d_wts = nullptr;
    c->wts_cap = 0;
    e = hipMalloc(&c->d_wts, need * sizeof(double));
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(c, CFET_ENOMEM, "cannot allocate the device weight table");
    }
    c->wts_cap = need;
  }
  std::vector<double> a(sc.s), b(sc.s * c->nterms);
  for (int64_t n = 0; n < nsteps; ++n) {
    cfet::step_weights(sc, c->drives, t0 + double(n) * dt, dt, a.data(), b.data());
    double* row = c->h_wts + size_t(n) * sc.s * nt1;
    for (int i = 0; i < sc.s; ++i) {
      row[i * nt1] = a[i];
      for (int k = 0; k < c->nterms; ++k) row[i * nt1 + 1 + k] = b[i * c->nterms + k];
    }
  }
  e = hipMemcpyAsync(c->d_wts, c->h_wts, need * sizeof(double), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipEventRecord(c->wts_copied, st);
  if (e != hipSuccess) return hip_fail(c, e, "upload the weight table");
  c->wts_pending = true;
  int nblocks = 1;
  if (path == 3) {
    nblocks = c->coop_blocks;
    if (4 * nblocks > c->part_cap) {
      if (c->d_part) (void)hipFree(c->d_part);
      c->d_part = nullptr;
      c->part_cap = 0;
      e = hipMalloc(&c->d_part, 4 * nblocks * sizeof(double));
      if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(c, CFET_ENOMEM, "cannot allocate partial sums");
      }
      c->part_cap = 4 * nblocks;
    }
  }
  if (!c->zbuf) {
    e = hipMalloc(&c->zbuf, 2 * size_t(c->n) * sizeof(double2));
    if (e != hipSuccess) {
      (void)hipGetLastError();
      c->zbuf = nullptr;
      return fail(c, CFET_ENOMEM, "cannot allocate the persistent z buffers");
    }
  }
  cfet::PersistArgs pa{};
  pa.rowptr = c->A.rowptr;
  pa.colt = c->A.colt;
  pa.val = c->A.val;
  pa.real_vals = c->real_vals ? 1 : 0;
  pa.n = c->n;
  pa.nterms = c->nterms;
  pa.wts = c->d_wts;
  pa.s = sc.s;
  pa.nsteps = nsteps;
  pa.m = m;
  pa.dt = dt;
  pa.psi = static_cast<double2*>(psi_dev);
  pa.basis = c->basis;
  pa.zbuf = c->zbuf;
  pa.part = c->d_part;
  pa.bar = c->d_bar;
  pa.fault = c->d_fault;
  pa.stats = c->stats;
  pa.spin_limit = c->spin_limit;
  pa.timing = (c->profiling && c->seg_timers) ? 1 : 0;
  pa.save = save;
  pa.export_T = export_T;  // one record per exponential of the call
  pa.no_combine = 0;
  pa.export_Y = export_Y;
  pa.export_each = (export_T || export_Y) ? 1 : 0;
  const bool timed = c->profiling && c->events.used < c->events.cap;
  if (timed) (void)hipEventRecord(c->events.begin[c->events.used], st);
  e = cfet::launch_persistent(pa, path == 2 ? c->preset_single : c->preset_coop, path == 2,
                             nblocks, st);
  if (timed && e == hipSuccess) {
    (void)hipEventRecord(c->events.end[c->events.used], st);
    c->events.used += 1;
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->stats_host, c->stats, sizeof(DevStats), hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return hip_fail(c, e, "persistent propagation launch");
  c->last_stream = st;
  c->have_work = true;
  c->last_path = path;
  return CFET_OK;
}

// One exponential exp(-i dt H_w) on the persistent path for the gradient's
// backward sweep: weights read from the device (wts_dev, 1 + nterms values),
// Lanczos basis kept in psi (vector 0) and basis, the projection exported to
// X; with no_combine psi is left unchanged.
hipError_t persistent_exponential(cfet_ctx* c, int path, double2* psi, double2* basis,
                                  const double* wts_dev, double dt, int m, LzScalars* X,
                                  bool no_combine, hipStream_t st, double2* Y = nullptr,
                                  unsigned long long* bar = nullptr) {
  cfet::PersistArgs pa{};
  pa.rowptr = c->A.rowptr;
  pa.colt = c->A.colt;
  pa.val = c->A.val;
  pa.real_vals = c->real_vals ? 1 : 0;
  pa.n = c->n;
  pa.nterms = c->nterms;
  pa.wts = wts_dev;
  pa.s = 1;
  pa.nsteps = 1;
  pa.m = m;
  pa.dt = dt;
  pa.psi = psi;
  pa.basis = basis;
  pa.zbuf = c->zbuf;
  pa.part = c->d_part;
  pa.bar = c->d_bar;
  pa.fault = c->d_fault;
  pa.stats = c->stats;
  pa.spin_limit = c->spin_limit;
  pa.timing = 0;
  pa.save = nullptr;
  pa.export_T = X;
  pa.no_combine = no_combine ? 1 : 0;
  pa.export_Y = Y;
  if (bar) pa.bar = bar;  // cleared by the caller on the stream
  const bool timed = c->profiling && c->events.used < c->events.cap;
  if (timed) (void)hipEventRecord(c->events.begin[c->events.used], st);
  const hipError_t e = cfet::launch_persistent(pa, path == 2 ? c->preset_single : c->preset_coop,
                                               path == 2, path == 3 ? c->coop_blocks : 1, st,
                                               bar == nullptr);
  if (timed && e == hipSuccess) {
    (void)hipEventRecord(c->events.end[c->events.used], st);
    c->events.used += 1;
  }
  return e;
}

}  // namespace

namespace {

// Device buffers of one cfet_gradient call (freed when the call returns).
struct GradBuffers {
  std::vector<void*> ptrs;
  ~GradBuffers() {
    for (void* p : ptrs) (void)hipFree(p);
  }
  template <class T>
  hipError_t get(T** p, size_t count) {
    hipError_t e = hipMalloc(reinterpret_cast<void**>(p), std::max<size_t>(count, 1) * sizeof(T));
    if (e == hipSuccess) ptrs.push_back(*p);
    return e;
  }
};

// Host staging of the SELL-64 layout.  Row r lists the driven terms' entries
// (H1, H2, ... each in the caller's order) and then H0's.  With `uniform`,
// every (row XOR column, term, value) that at least kSharedMinRows rows of a
// slice hold (all of them, in a slice of fewer rows) becomes one shared entry
// of the slice with a 64-bit mask of those rows, in order of first
// appearance (rows in order); the per-row slots keep the rest.
constexpr int kSharedMinRows = 8;

struct SellStage {
  std::vector<int64_t> sptr;
  std::vector<int32_t> swid;
  std::vector<int32_t> rlen;   // per-row slots in use
  std::vector<uint32_t> scol;
  std::vector<double> sval;
  std::vector<int32_t> nuni;
  std::vector<int64_t> uptr;
  std::vector<uint32_t> ucol;
  std::vector<double> uval;
  std::vector<uint64_t> umask;
  std::vector<double> diag;    // extracted diagonal of term diag_term (empty: none)
  int diag_term = 0;
};

template <class F>
void for_sell_row(const std::vector<HostCSR>& mats, int nterms, int64_t r, F f) {
  for (int tt = 1; tt <= nterms + 1; ++tt) {
    const int term = (tt == nterms + 1) ? 0 : tt;  // driven terms first, then H0
    const HostCSR& h = mats[term];
    for (int64_t q = h.rp[r]; q < h.rp[r + 1]; ++q) f(term, h.col[q], &h.val[2 * q]);
  }
}

// Shared entries of one slice: (row XOR column | term << kTermShift, value
// bits) keys in a small open-addressing table, with the mask of rows holding
// each (a row holds a key at most once: columns of one term are distinct).
struct SliceShared {
  struct Cand {
    uint32_t key;
    uint64_t re, im;
    uint64_t mask;
    int count;
  };
  std::vector<Cand> cand;
  std::vector<char> keep;
  std::vector<int32_t> table;  // candidate index + 1, 0 = empty
  uint32_t tmask = 0;

  static uint32_t make_key(int64_t r, int32_t col, int term) {
    return uint32_t(int64_t(col) ^ r) | (uint32_t(term) << cfet::kTermShift);
  }
  static uint64_t bits(double v) {
    uint64_t u;
    std::memcpy(&u, &v, sizeof(u));
    return u;
  }
  uint32_t slot(uint32_t key, uint64_t re, uint64_t im) const {
    uint64_t h = uint64_t(key) * 0x9E3779B97F4A7C15ull;
    h ^= (re + 0x632BE59BD9B4E019ull) * 0xC2B2AE3D27D4EB4Full;
    h ^= (im + 0x94D049BB133111EBull) * 0x165667B19E3779F9ull;
    return uint32_t(h >> 32) & tmask;
  }
  int find(uint32_t key, uint64_t re, uint64_t im) const {
    if (table.empty()) return -1;
    for (uint32_t h = slot(key, re, im);; h = (h + 1) & tmask) {
      const int i = table[h] - 1;
      if (i < 0) return -1;
      if (cand[i].key == key && cand[i].re == re && cand[i].im == im) return i;
    }
  }

  // Shared entries of the rows rows[0 .. nr) (at most 64; bit l of a mask is
  // rows[l]), over the entries that keep(row, col) accepts.  A candidate is
  // kept when at least min(need, nr) of the rows hold it.  Returns the number
  // kept.
  template <class Keep>
  int run(const std::vector<HostCSR>& mats, int nterms, const int64_t* rows, int nr, int need,
          Keep keep_entry) {
    cand.clear();
    int64_t total = 0;
    for (int l = 0; l < nr; ++l)
      for (int k = 0; k <= nterms; ++k) total += mats[k].rp[rows[l] + 1] - mats[k].rp[rows[l]];
    table.clear();
    // (a slice of very long rows keeps everything per row)
    if (total == 0 || total > (int64_t(1) << 29)) return 0;
    uint32_t size = 2;
    while (size < 2 * uint64_t(total)) size <<= 1;
    tmask = size - 1;
    table.assign(size, 0);
    for (int l = 0; l < nr; ++l) {
      const int64_t r = rows[l];
      const uint64_t bit = uint64_t(1) << l;
      for_sell_row(mats, nterms, r, [&](int term, int32_t col, const double* v) {
        if (!keep_entry(r, col)) return;
        const uint32_t key = make_key(r, col, term);
        const uint64_t re = bits(v[0]), im = bits(v[1]);
        uint32_t h = slot(key, re, im);
        for (;; h = (h + 1) & tmask) {
          const int i = table[h] - 1;
          if (i < 0) {
            table[h] = int32_t(cand.size()) + 1;
            cand.push_back({key, re, im, bit, 1});
            break;
          }
          if (cand[i].key == key && cand[i].re == re && cand[i].im == im) {
            cand[i].mask |= bit;
            cand[i].count += 1;
            break;
          }
        }
      });
    }
    const int need_rows = std::min(need, nr);
    keep.assign(cand.size(), 0);
    int ns = 0;
    for (size_t i = 0; i < cand.size(); ++i)
      if (cand[i].count >= need_rows) {
        keep[i] = 1;
        ++ns;
      }
    return ns;
  }

  bool shared(int64_t r, int32_t col, int term, const double* v) const {
    const int i = find(make_key(r, col, term), bits(v[0]), bits(v[1]));
    return i >= 0 && keep[i];
  }
};

// An entry (row, col) belongs to the first pass unless the split bit is set
// (split_bit > 0) and its offset row ^ col has a bit at or above it.
inline bool low_entry(int64_t r, int32_t col, int split_bit) {
  return split_bit <= 0 || ((r ^ int64_t(col)) >> split_bit) == 0;
}

template <class Body>
void run_threads(int64_t count, unsigned nth, Body body) {
  if (nth <= 1) {
    body(int64_t(0), count);
    return;
  }
  std::vector<std::thread> pool;
  for (unsigned t = 0; t < nth; ++t)
    pool.emplace_back([&, t]() { body(count * t / nth, count * (t + 1) / nth); });
  for (auto& th : pool) th.join();
}

// Gershgorin interval of one Hermitian CSR matrix (Sec. 8.1: the Chebyshev
// technique needs a-priori bounds on the spectrum): row r contributes
// [d_r - R_r, d_r + R_r], d_r the real part of its diagonal entries, R_r the
// sum of |H_rc| over its other entries.
void gershgorin(const cfet::HostCSR& h, unsigned nth, double* lo, double* hi) {
  std::vector<double> tlo(std::max(1u, nth), 1e300), thi(std::max(1u, nth), -1e300);
  std::atomic<unsigned> next{0};
  auto body = [&](int64_t r0, int64_t r1) {
    const unsigned t = next.fetch_add(1);
    double l = 1e300, u = -1e300;
    for (int64_t r = r0; r < r1; ++r) {
      double d = 0.0, R = 0.0;
      for (int64_t e = h.rp[r]; e < h.rp[r + 1]; ++e) {
        const double re = h.val[2 * e], im = h.val[2 * e + 1];
        if (int64_t(h.col[e]) == r)
          d += re;
        else
          R += std::hypot(re, im);
      }
      l = std::min(l, d - R);
      u = std::max(u, d + R);
    }
    tlo[t] = l;
    thi[t] = u;
  };
  run_threads(h.n, nth, body);
  *lo = *std::min_element(tlo.begin(), tlo.end());
  *hi = *std::max_element(thi.begin(), thi.end());
  if (h.n == 0) *lo = *hi = 0.0;
}

// Stage the SELL-64 layout of the first pass: all entries, or with split_bit
// > 0 only the low-offset ones (the others go to the second pass).  Returns
// false when the host buffers cannot be allocated.
// With diag_term >= 0 the diagonal entries (all of that term and real) are
// stored apart, one double per row, and left out of the slots.
bool stage_sell(const std::vector<HostCSR>& mats, int nterms, int64_t n,
                const std::vector<int32_t>& rowlen_all, bool uniform, int split_bit,
                int tbits, int diag_term, unsigned nth, SellStage* S) {
  const int64_t nsl = (n + 63) / 64;
  const bool xdiag = diag_term >= 0;
  auto keep = [split_bit, xdiag](int64_t r, int32_t col) {
    return low_entry(r, col, split_bit) && !(xdiag && int64_t(col) == r);
  };
  if (xdiag) {
    try {
      S->diag.assign(n, 0.0);
    } catch (const std::bad_alloc&) {
      return false;
    }
    S->diag_term = diag_term;
    const HostCSR& h = mats[diag_term];
    run_threads(n, nth, [&](int64_t r0, int64_t r1) {
      for (int64_t r = r0; r < r1; ++r)
        for (int64_t q = h.rp[r]; q < h.rp[r + 1]; ++q)
          if (int64_t(h.col[q]) == r) S->diag[r] = h.val[2 * q];
    });
  }
  try {
    S->sptr.assign(nsl + 1, 0);
    S->swid.assign(nsl, 0);
    S->rlen = rowlen_all;
    if (uniform) {
      S->nuni.assign(nsl, 0);
      S->uptr.assign(nsl + 1, 0);
    }
  } catch (const std::bad_alloc&) {
    return false;
  }
  if (split_bit > 0 || xdiag) {
    // per-row counts of the first pass's entries
    run_threads(n, nth, [&](int64_t r0, int64_t r1) {
      for (int64_t r = r0; r < r1; ++r) {
        int32_t len = 0;
        for_sell_row(mats, nterms, r, [&](int, int32_t col, const double*) {
          if (keep(r, col)) ++len;
        });
        S->rlen[r] = len;
      }
    });
  }
  if (uniform) {
    // shared entries per slice, and each row's count of the rest
    run_threads(nsl, nth, [&](int64_t s0, int64_t s1) {
      SliceShared U;
      int64_t rows[64];
      for (int64_t sl = s0; sl < s1; ++sl) {
        const int64_t r0 = sl * 64, r1 = std::min<int64_t>(n, sl * 64 + 64);
        for (int64_t r = r0; r < r1; ++r) rows[r - r0] = r;
        S->nuni[sl] = U.run(mats, nterms, rows, int(r1 - r0), kSharedMinRows, keep);
        for (size_t i = 0; i < U.cand.size(); ++i) {
          if (!U.keep[i]) continue;
          for (int64_t r = r0; r < r1; ++r)
            if ((U.cand[i].mask >> (r - r0)) & 1u) S->rlen[r] -= 1;
        }
      }
    });
  }
  for (int64_t sl = 0; sl < nsl; ++sl) {
    int w = 0;
    for (int64_t r = sl * 64; r < std::min<int64_t>(n, sl * 64 + 64); ++r) w = std::max(w, S->rlen[r]);
    S->swid[sl] = w;
    S->sptr[sl + 1] = S->sptr[sl] + 64 * int64_t(w);
    if (uniform) S->uptr[sl + 1] = S->uptr[sl] + S->nuni[sl];
  }
  const int64_t slots = S->sptr[nsl];
  const int64_t uslots = uniform ? S->uptr[nsl] : 0;
  try {
    S->scol.assign(slots, 0u);
    S->sval.assign(2 * slots, 0.0);
    S->ucol.assign(uslots, 0u);
    S->uval.assign(2 * uslots, 0.0);
    S->umask.assign(uslots, 0ull);
  } catch (const std::bad_alloc&) {
    return false;
  }
  run_threads(nsl, nth, [&](int64_t s0, int64_t s1) {
    SliceShared U;
    int64_t rows[64];
    for (int64_t sl = s0; sl < s1; ++sl) {
      const int64_t r0 = sl * 64, r1 = std::min<int64_t>(n, sl * 64 + 64);
      const bool uni = uniform && S->nuni[sl] > 0;
      if (uni) {
        for (int64_t r = r0; r < r1; ++r) rows[r - r0] = r;
        U.run(mats, nterms, rows, int(r1 - r0), kSharedMinRows, keep);
        int64_t u = S->uptr[sl];
        // with tiles (tbits > 0) the entries reaching outside the tile first
        for (int round = (tbits > 0 ? 0 : 1); round < 2; ++round) {
          for (size_t i = 0; i < U.cand.size(); ++i) {
            if (!U.keep[i]) continue;
            const SliceShared::Cand& cd = U.cand[i];
            const bool outside = tbits > 0 && (cd.key & cfet::kColMask) >> tbits;
            if (round == 0 && !outside) continue;
            if (round == 1 && tbits > 0 && outside) continue;
            S->ucol[u] = cd.key;
            std::memcpy(&S->uval[2 * u], &cd.re, sizeof(double));
            std::memcpy(&S->uval[2 * u + 1], &cd.im, sizeof(double));
            S->umask[u] = cd.mask;
            ++u;
          }
        }
      }
      for (int64_t r = r0; r < r1; ++r) {
        const int64_t lane = r - r0;
        int64_t k = 0;
        for_sell_row(mats, nterms, r, [&](int term, int32_t col, const double* v) {
          if (!keep(r, col)) return;
          if (uni && U.shared(r, col, term, v)) return;
          const int64_t pos = S->sptr[sl] + 64 * k + lane;
          S->scol[pos] = uint32_t(col) | (uint32_t(term) << cfet::kTermShift);
          S->sval[2 * pos] = v[0];
          S->sval[2 * pos + 1] = v[1];
          ++k;
        });
      }
    }
  });
  return true;
}

// Shared lists of slices, made compact: each slice's list (entries at
// uptr[s], nuni[s] of them) is padded with empty entries (mask 0, which no
// row holds) to a multiple of `pad`, and slices whose padded lists are equal
// (same offsets, terms, values and masks -- the common case for site terms of
// spin systems, whose lists depend on a few bits of the slice index) point to
// one stored copy.  Afterwards uptr[s] is the start of slice s's list (no
// longer increasing) and uptr[nsl] the number of stored entries.
bool compact_shared_lists(int64_t nsl, int pad, std::vector<int32_t>* nuni,
                          std::vector<int64_t>* uptr, std::vector<uint32_t>* ucol,
                          std::vector<double>* uval, std::vector<uint64_t>* umask) {
  std::vector<uint32_t> oc;
  std::vector<double> ov;
  std::vector<uint64_t> om;
  std::vector<int64_t> optr;
  try {
    optr.assign(nsl + 1, 0);
    oc.reserve(ucol->size() / 4 + 64);
    ov.reserve(uval->size() / 4 + 128);
    om.reserve(umask->size() / 4 + 64);
  } catch (const std::bad_alloc&) {
    return false;
  }
  // hash of a padded list -> slices whose stored list has that hash
  std::unordered_map<uint64_t, std::vector<int64_t>> seen;
  std::vector<uint32_t> lc;
  std::vector<double> lv;
  std::vector<uint64_t> lm;
  for (int64_t sl = 0; sl < nsl; ++sl) {
    const int64_t b = (*uptr)[sl];
    int cnt = (*nuni)[sl];
    lc.assign(ucol->begin() + b, ucol->begin() + b + cnt);
    lv.assign(uval->begin() + 2 * b, uval->begin() + 2 * (b + cnt));
    lm.assign(umask->begin() + b, umask->begin() + b + cnt);
    while (pad > 1 && cnt % pad) {
      lc.push_back(0u);
      lv.push_back(0.0);
      lv.push_back(0.0);
      lm.push_back(0ull);
      ++cnt;
    }
    uint64_t h = 0x9E3779B97F4A7C15ull ^ uint64_t(cnt);
    for (int i = 0; i < cnt; ++i) {
      uint64_t re, im;
      std::memcpy(&re, &lv[2 * i], 8);
      std::memcpy(&im, &lv[2 * i + 1], 8);
      for (uint64_t w : {uint64_t(lc[i]), re, im, lm[i]}) {
        h ^= w + 0x9E3779B97F4A7C15ull + (h << 6) + (h >> 2);
        h *= 0xBF58476D1CE4E5B9ull;
      }
    }
    int64_t at = -1;
    std::vector<int64_t>& cands = seen[h];
    for (int64_t other : cands) {
      if ((*nuni)[other] != cnt) continue;
      const int64_t ob = optr[other];
      if (std::equal(lc.begin(), lc.end(), oc.begin() + ob) &&
          std::memcmp(lv.data(), ov.data() + 2 * ob, lv.size() * sizeof(double)) == 0 &&
          std::equal(lm.begin(), lm.end(), om.begin() + ob)) {
        at = ob;
        break;
      }
    }
    if (at < 0) {
      at = int64_t(oc.size());
      oc.insert(oc.end(), lc.begin(), lc.end());
      ov.insert(ov.end(), lv.begin(), lv.end());
      om.insert(om.end(), lm.begin(), lm.end());
      cands.push_back(sl);
    }
    (*nuni)[sl] = cnt;
    optr[sl] = at;
  }
  optr[nsl] = int64_t(oc.size());
  ucol->swap(oc);
  uval->swap(ov);
  umask->swap(om);
  uptr->swap(optr);
  return true;
}

// Shared lists of the tiled kernels: each slice's list is arranged in four
// groups -- entries of the driven terms held by all 64 rows, the other
// driven-term entries, then the same two for H0 -- each keeping the order it
// had (entries reaching outside the tile first) and padded to a multiple of
// four with entries that add nothing (value 0; mask all rows in the
// all-rows groups, no row in the others).  groups[s] packs the four padded
// counts in 16 bits each (group g at bits 16 g).  Returns false when a group
// would not fit 16 bits or memory runs out.
bool arrange_tiled_lists(int64_t nsl, uint32_t tmask, std::vector<int32_t>* nuni,
                         std::vector<int64_t>* uptr, std::vector<uint32_t>* ucol,
                         std::vector<double>* uval, std::vector<uint64_t>* umask,
                         std::vector<uint64_t>* groups) {
  std::vector<uint32_t> oc;
  std::vector<double> ov;
  std::vector<uint64_t> om;
  std::vector<int64_t> optr;
  try {
    optr.assign(nsl + 1, 0);
    groups->assign(nsl, 0);
    oc.reserve(ucol->size() + 16 * nsl);
    ov.reserve(uval->size() + 32 * nsl);
    om.reserve(umask->size() + 16 * nsl);
  } catch (const std::bad_alloc&) {
    return false;
  }
  for (int64_t sl = 0; sl < nsl; ++sl) {
    const int64_t b = (*uptr)[sl];
    const int cnt = (*nuni)[sl];
    optr[sl] = int64_t(oc.size());
    uint64_t packed = 0;
    for (int g = 0; g < 4; ++g) {
      const bool driven = g < 2, full = (g % 2) == 0;
      const uint32_t pad_term = driven ? (1u << cfet::kTermShift) : 0u;
      int64_t taken = 0;
      // entries outside the tile (offset above tmask) first, then the others,
      // each part padded to whole batches of four (zero value, offset 0): a
      // batch is either all gathers or all tile reads
      for (int outside = 1; outside >= 0; --outside) {
        for (int i = 0; i < cnt; ++i) {
          const uint32_t ct = (*ucol)[b + i];
          const uint64_t m = (*umask)[b + i];
          if (((ct >> cfet::kTermShift) != 0) != driven || (m == ~0ull) != full) continue;
          if (((ct & cfet::kColMask) > tmask) != (outside == 1)) continue;
          oc.push_back(ct);
          ov.push_back((*uval)[2 * (b + i)]);
          ov.push_back((*uval)[2 * (b + i) + 1]);
          om.push_back(m);
          ++taken;
        }
        while (taken % 4) {
          oc.push_back(pad_term);
          ov.push_back(0.0);
          ov.push_back(0.0);
          om.push_back(full ? ~0ull : 0ull);
          ++taken;
        }
      }
      if (taken >= 65536) return false;
      packed |= uint64_t(taken) << (16 * g);
    }
    (*groups)[sl] = packed;
    (*nuni)[sl] = int32_t(int64_t(oc.size()) - optr[sl]);
  }
  optr[nsl] = int64_t(oc.size());
  ucol->swap(oc);
  uval->swap(ov);
  umask->swap(om);
  uptr->swap(optr);
  return true;
}

// The entries that every slice's shared list holds with a full row mask and
// the same offset, term and value (a driven sum of site operators with one
// coefficient: every sigma_x flip), moved out of the per-slice lists into one
// common list.  The tiled kernels then read them from one place, where the
// scalar cache keeps them, instead of from every slice's own list.  The
// common list is arranged as the kernels read it: driven terms, then H0;
// each part with the entries outside the tile (offset above tmask) first,
// each run padded to whole batches of four (zero value, offset 0).
constexpr int kCommonMax = 64;

struct CommonList {
  std::vector<uint32_t> col;
  std::vector<double> val;   // re, im
  int nd = 0, nh = 0;
};

bool extract_common(int64_t nsl, uint32_t tmask, unsigned nth, std::vector<int32_t>* nuni,
                    std::vector<int64_t>* uptr, std::vector<uint32_t>* ucol,
                    std::vector<double>* uval, std::vector<uint64_t>* umask, CommonList* C) {
  struct Key {
    uint32_t ct;
    uint64_t re, im;
    bool operator<(const Key& o) const {
      if (ct != o.ct) return ct < o.ct;
      if (re != o.re) return re < o.re;
      return im < o.im;
    }
    bool operator==(const Key& o) const { return ct == o.ct && re == o.re && im == o.im; }
  };
  auto key_of = [&](int64_t e) {
    Key k;
    k.ct = (*ucol)[e];
    std::memcpy(&k.re, &(*uval)[2 * e], 8);
    std::memcpy(&k.im, &(*uval)[2 * e + 1], 8);
    return k;
  };
  *C = CommonList();
  if (nsl <= 0) return true;
  std::vector<Key> cand;
  for (int64_t e = (*uptr)[0]; e < (*uptr)[1]; ++e)
    if ((*umask)[e] == ~0ull) cand.push_back(key_of(e));
  std::sort(cand.begin(), cand.end());
  cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
  if (cand.empty()) return true;
  const unsigned T = std::max(1u, nth);
  std::vector<std::vector<int64_t>> cnt(T, std::vector<int64_t>(cand.size(), 0));
  std::atomic<unsigned> next{0};
  auto find = [&](const Key& k) -> int64_t {
    auto it = std::lower_bound(cand.begin(), cand.end(), k);
    return (it != cand.end() && *it == k) ? int64_t(it - cand.begin()) : -1;
  };
  run_threads(nsl, T, [&](int64_t s0, int64_t s1) {
    std::vector<int64_t>& my = cnt[next.fetch_add(1)];
    for (int64_t sl = s0; sl < s1; ++sl)
      for (int64_t e = (*uptr)[sl]; e < (*uptr)[sl + 1]; ++e)
        if ((*umask)[e] == ~0ull) {
          const int64_t i = find(key_of(e));
          if (i >= 0) ++my[size_t(i)];
        }
  });
  std::vector<char> common(cand.size(), 0);
  int ncommon = 0;
  for (size_t i = 0; i < cand.size(); ++i) {
    int64_t tot = 0;
    for (unsigned t = 0; t < T; ++t) tot += cnt[t][i];
    if (tot == nsl && ncommon < kCommonMax) {
      common[i] = 1;
      ++ncommon;
    }
  }
  if (ncommon == 0) return true;
  // every slice must hold each common entry exactly once (the shared lists
  // hold a key at most once per slice); otherwise leave the lists as they are
  std::atomic<bool> once{true};
  run_threads(nsl, T, [&](int64_t s0, int64_t s1) {
    for (int64_t sl = s0; sl < s1 && once.load(std::memory_order_relaxed); ++sl) {
      int found = 0;
      for (int64_t e = (*uptr)[sl]; e < (*uptr)[sl + 1]; ++e)
        if ((*umask)[e] == ~0ull) {
          const int64_t i = find(key_of(e));
          if (i >= 0 && common[size_t(i)]) ++found;
        }
      if (found != ncommon) once.store(false);
    }
  });
  if (!once.load()) return true;
  // the common list, in the kernels' order
  for (int driven = 1; driven >= 0; --driven) {
    int taken = 0;
    for (int outside = 1; outside >= 0; --outside) {
      for (size_t i = 0; i < cand.size(); ++i) {
        if (!common[i]) continue;
        if (((cand[i].ct >> cfet::kTermShift) != 0) != (driven == 1)) continue;
        if (((cand[i].ct & cfet::kColMask) > tmask) != (outside == 1)) continue;
        double re, im;
        std::memcpy(&re, &cand[i].re, 8);
        std::memcpy(&im, &cand[i].im, 8);
        C->col.push_back(cand[i].ct);
        C->val.push_back(re);
        C->val.push_back(im);
        ++taken;
      }
      while (taken % 4) {
        C->col.push_back(driven ? (1u << cfet::kTermShift) : 0u);
        C->val.push_back(0.0);
        C->val.push_back(0.0);
        ++taken;
      }
    }
    (driven ? C->nd : C->nh) = taken;
  }
  // the per-slice lists without them (each slice holds each common entry once)
  std::vector<int64_t> nptr(nsl + 1, 0);
  for (int64_t sl = 0; sl < nsl; ++sl) nptr[sl + 1] = nptr[sl] + ((*nuni)[sl] - ncommon);
  std::vector<uint32_t> oc;
  std::vector<double> ov;
  std::vector<uint64_t> om;
  try {
    oc.resize(size_t(nptr[nsl]));
    ov.resize(2 * size_t(nptr[nsl]));
    om.resize(size_t(nptr[nsl]));
  } catch (const std::bad_alloc&) {
    return false;
  }
  run_threads(nsl, T, [&](int64_t s0, int64_t s1) {
    for (int64_t sl = s0; sl < s1; ++sl) {
      int64_t w = nptr[sl];
      for (int64_t e = (*uptr)[sl]; e < (*uptr)[sl + 1]; ++e) {
        if ((*umask)[e] == ~0ull) {
          const int64_t i = find(key_of(e));
          if (i >= 0 && common[size_t(i)]) continue;
        }
        oc[size_t(w)] = (*ucol)[e];
        ov[2 * size_t(w)] = (*uval)[2 * e];
        ov[2 * size_t(w) + 1] = (*uval)[2 * e + 1];
        om[size_t(w)] = (*umask)[e];
        ++w;
      }
      (*nuni)[sl] = int32_t(nptr[sl + 1] - nptr[sl]);
    }
  });
  ucol->swap(oc);
  uval->swap(ov);
  umask->swap(om);
  uptr->swap(nptr);
  return true;
}

// Split of the shared-part layout into two passes (see DevSELLHi).  Applies to
// operators on 2^nbits rows (nbits >= 8): entries whose offset row ^ col has a
// bit at or above split_bit = min(16, nbits - 2) leave the first pass, whose
// gathers then stay within 2^16 rows (1 MiB of a vector) of the row.
constexpr int kSplitBitMax = 16;
constexpr int kSplitMinBits = 8;

struct SplitPlan {
  int nbits = 0;
  int split_bit = 0;      // 0: no split
  int tbits = 0;          // tile of both passes: 2^tbits indices
  int pos[32] = {};       // row position of permuted bit b
  int64_t high = 0;       // entries of the second pass
};

// The permuted order: the three lowest row bits first (8 consecutive rows),
// then every bit that a second-pass offset uses, then the remaining bits, each
// group in increasing order.  Returns false if nothing would move.
bool plan_split(const std::vector<HostCSR>& mats, int nterms, int64_t n, unsigned nth,
                SplitPlan* P) {
  int nbits = 0;
  while ((int64_t(1) << nbits) < n) ++nbits;
  if ((int64_t(1) << nbits) != n || nbits < kSplitMinBits) return false;
  const int S = std::min(kSplitBitMax, nbits - 2);
  std::vector<uint64_t> used(nth, 0);
  std::vector<int64_t> cnt(nth, 0);
  std::vector<std::thread> pool;
  for (unsigned t = 0; t < nth; ++t)
    pool.emplace_back([&, t]() {
      const int64_t r0 = n * t / nth, r1 = n * (t + 1) / nth;
      uint64_t u = 0;
      int64_t c = 0;
      for (int64_t r = r0; r < r1; ++r)
        for_sell_row(mats, nterms, r, [&](int, int32_t col, const double*) {
          if (!low_entry(r, col, S)) {
            u |= uint64_t(r ^ int64_t(col));
            ++c;
          }
        });
      used[t] = u;
      cnt[t] = c;
    });
  for (auto& th : pool) th.join();
  uint64_t u = 0;
  int64_t c = 0;
  for (unsigned t = 0; t < nth; ++t) {
    u |= used[t];
    c += cnt[t];
  }
  if (c == 0) return false;
  // the second pass's tile must hold every column its rows read: the three
  // low bits and the bits of its offsets
  const int tb = std::min(cfet::kTileBitsMax, nbits);
  int nb2 = 3;
  for (int b = 3; b < nbits; ++b) nb2 += int((u >> b) & 1u);
  if (nb2 > tb) return false;
  P->nbits = nbits;
  P->split_bit = S;
  P->tbits = tb;
  P->high = c;
  int k = 0;
  for (int b = 0; b < 3; ++b) P->pos[k++] = b;
  for (int b = 3; b < nbits; ++b)
    if ((u >> b) & 1u) P->pos[k++] = b;
  for (int b = 3; b < nbits; ++b)
    if (!((u >> b) & 1u)) P->pos[k++] = b;
  return true;
}

inline int64_t permuted_row(const SplitPlan& P, int64_t q) {
  int64_t r = 0;
  for (int b = 0; b < P.nbits; ++b) r |= ((q >> b) & 1) << P.pos[b];
  return r;
}

// The offset in the permuted order: bit pos[b] of off becomes bit b.
inline uint32_t permuted_offset(const SplitPlan& P, uint32_t off) {
  uint32_t q = 0;
  for (int b = 0; b < P.nbits; ++b) q |= ((off >> P.pos[b]) & 1u) << b;
  return q;
}

struct SellHiStage {
  std::vector<int32_t> nuni;
  std::vector<int64_t> uptr;
  std::vector<uint32_t> ucol;
  std::vector<double> uval;
  std::vector<uint64_t> umask;
};

// Stage the second pass: every high-offset entry, shared per permuted slice.
bool stage_sell_hi(const std::vector<HostCSR>& mats, int nterms, int64_t n, const SplitPlan& P,
                   unsigned nth, SellHiStage* H) {
  const int64_t nsl = n / 64;
  const int S = P.split_bit;
  auto keep = [S](int64_t r, int32_t col) { return !low_entry(r, col, S); };
  try {
    H->nuni.assign(nsl, 0);
    H->uptr.assign(nsl + 1, 0);
  } catch (const std::bad_alloc&) {
    return false;
  }
  auto slice_rows = [&](int64_t sl, int64_t* rows) {
    for (int l = 0; l < 64; ++l) rows[l] = permuted_row(P, sl * 64 + l);
  };
  run_threads(nsl, nth, [&](int64_t s0, int64_t s1) {
    SliceShared U;
    int64_t rows[64];
    for (int64_t sl = s0; sl < s1; ++sl) {
      slice_rows(sl, rows);
      H->nuni[sl] = U.run(mats, nterms, rows, 64, 1, keep);
    }
  });
  for (int64_t sl = 0; sl < nsl; ++sl) H->uptr[sl + 1] = H->uptr[sl] + H->nuni[sl];
  const int64_t us = H->uptr[nsl];
  try {
    H->ucol.assign(us, 0u);
    H->uval.assign(2 * us, 0.0);
    H->umask.assign(us, 0ull);
  } catch (const std::bad_alloc&) {
    return false;
  }
  run_threads(nsl, nth, [&](int64_t s0, int64_t s1) {
    SliceShared U;
    int64_t rows[64];
    for (int64_t sl = s0; sl < s1; ++sl) {
      slice_rows(sl, rows);
      U.run(mats, nterms, rows, 64, 1, keep);
      int64_t u = H->uptr[sl];
      for (size_t i = 0; i < U.cand.size(); ++i) {
        const SliceShared::Cand& cd = U.cand[i];
        H->ucol[u] = permuted_offset(P, cd.key & cfet::kColMask) |
                     (cd.key & ~cfet::kColMask);
        std::memcpy(&H->uval[2 * u], &cd.re, sizeof(double));
        std::memcpy(&H->uval[2 * u + 1], &cd.im, sizeof(double));
        H->umask[u] = cd.mask;
        ++u;
      }
    }
  });
  return true;
}

// Piece of a piecewise-constant drive containing t, or -1 outside.
int pwc_piece(const DriveSpec& d, double t) {
  const std::vector<double>& e = d.edges;
  if (e.size() < 2 || t < e.front() || t >= e.back()) return -1;
  const size_t p = size_t(std::upper_bound(e.begin(), e.end(), t) - e.begin()) - 1;
  return int(std::min(p, e.size() - 2));
}

}  // namespace

extern "C" {

int cfet_version(void) { return CFET_VERSION; }

const char* cfet_last_error(const cfet_ctx* c) {
  if (c) return c->err.c_str();
  return g_err.c_str();
}

int cfet_create(const cfet_csr* H0, int32_t nterms, const cfet_csr* Hk, const cfet_drive* fk,
                uint32_t flags, cfet_ctx** out) {
  if (!out) return fail(nullptr, CFET_EINVAL, "out is null");
  *out = nullptr;
  if (nterms < 1 || nterms > CFET_MAX_TERMS)
    return fail(nullptr, CFET_EINVAL, "nterms must be in 1..7");
  if (!H0 || !Hk || !fk) return fail(nullptr, CFET_EINVAL, "null H0, Hk or fk");
  cfet_ctx* c = new (std::nothrow) cfet_ctx();
  if (!c) return fail(nullptr, CFET_ENOMEM, "cannot allocate context");
  int rc;
  hipError_t e = hipGetDevice(&c->device);
  if (e != hipSuccess) {
    free_ctx(c);
    return hip_fail(nullptr, e, "hipGetDevice");
  }
  std::vector<HostCSR> mats(nterms + 1);
  rc = load_csr(c, H0, "H0", &mats[0]);
  for (int k = 0; rc == CFET_OK && k < nterms; ++k) rc = load_csr(c, &Hk[k], "Hk", &mats[k + 1]);
  if (rc != CFET_OK) {
    g_err = c->err;
    free_ctx(c);
    return rc;
  }
  const int64_t n = mats[0].n;
  for (int k = 1; k <= nterms; ++k)
    if (mats[k].n != n) {
      rc = fail(c, CFET_EINVAL, "all matrices must have the same n");
      free_ctx(c);
      return rc;
    }
  if (n >= cfet::kMaxDim) {
    rc = fail(c, CFET_EUNSUPPORTED, "dimension must be below 2^29");
    free_ctx(c);
    return rc;
  }
  for (int k = 0; k <= nterms && rc == CFET_OK; ++k) {
    rc = validate_csr(c, mats[k], k == 0 ? "H0" : "Hk");
    if (rc == CFET_OK && (flags & CFET_VALIDATE_HERMITIAN))
      rc = check_hermitian(c, mats[k], k == 0 ? "H0" : "Hk");
  }
  c->drives.resize(nterms);
  for (int k = 0; k < nterms && rc == CFET_OK; ++k) rc = copy_drive(c, fk[k], &c->drives[k]);
  if (rc != CFET_OK) {
    g_err = c->err;
    free_ctx(c);
    return rc;
  }
  c->n = n;
  c->nterms = nterms;
  c->flags = flags;
  {
    const unsigned nth = (n < 65536) ? 1u
                                     : std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    c->glo.assign(nterms + 1, 0.0);
    c->ghi.assign(nterms + 1, 0.0);
    for (int k = 0; k <= nterms; ++k) gershgorin(mats[k], nth, &c->glo[k], &c->ghi[k]);
  }

  // Device layouts.  CSR (row r: entries of H0, then H1, ...) serves the
  // persistent paths and small problems; SELL (row r: H1.., then H0) serves the
  // multi-kernel path for large dimensions, where CSR is not kept.
  int64_t nnz = 0;
  for (int k = 0; k <= nterms; ++k) nnz += mats[k].nnz;
  std::vector<int32_t> rowlen;
  try {
    rowlen.resize(n);
  } catch (const std::bad_alloc&) {
    rc = fail(c, CFET_ENOMEM, "cannot stage row lengths on the host");
    free_ctx(c);
    return rc;
  }
  for (int64_t r = 0; r < n; ++r) {
    int64_t len = 0;
    for (int k = 0; k <= nterms; ++k) len += mats[k].rp[r + 1] - mats[k].rp[r];
    rowlen[r] = int32_t(std::min<int64_t>(len, INT32_MAX));
    c->max_row = std::max<int>(c->max_row, rowlen[r]);
  }
  const bool use_sell =
      (flags & (CFET_LAYOUT_SELL | CFET_LAYOUT_SELL_UNIFORM | CFET_LAYOUT_SELL_SPLIT)) ||
      n > kAutoCoopMaxN;
  const bool need_csr = !use_sell || n <= kAutoCoopMaxN || (flags & CFET_KEEP_CSR);
  c->A.n = n;
  c->A.nnz = nnz;
  const unsigned nth_all = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  // Row order of the CSR paths: reverse Cuthill-McKee when it leaves at least
  // a quarter fewer entries whose column lies in another block of the
  // cooperative kernel (those are the values a block gathers from other
  // blocks each Lanczos step).  Only above the single-workgroup size, and not
  // when the multi-kernel path runs on SELL.
  std::vector<int32_t> perm, iperm;
  if (need_csr && !use_sell && n > kAutoSingleMaxN && !(flags & CFET_NO_REORDER)) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device) ==
            hipSuccess && cus > 0) {
      const int64_t nbw = coop_grid_blocks(n, cus);
      const int64_t per = (n + nbw - 1) / nbw;
      try {
        std::vector<int32_t> ord = cfet::rcm_order(mats, n);
        std::vector<int32_t> inv(n);
        for (int64_t i = 0; i < n; ++i) inv[ord[i]] = int32_t(i);
        const int64_t nat = cfet::cross_block_entries(mats, n, per, nullptr);
        const int64_t rcm = cfet::cross_block_entries(mats, n, per, inv.data());
        if (4 * rcm <= 3 * nat) {
          perm.swap(ord);
          iperm.swap(inv);
        }
      } catch (const std::bad_alloc&) {
        perm.clear();  // keep the caller's order
        iperm.clear();
      }
    }
  }
  const bool reorder = !perm.empty();
  if (need_csr) {
    std::vector<int64_t> rp;
    std::vector<uint32_t> colt;
    std::vector<double> val;
    try {
      rp.resize(n + 1);
      colt.resize(nnz);
      val.resize(2 * nnz);
    } catch (const std::bad_alloc&) {
      rc = fail(c, CFET_ENOMEM, "cannot stage the merged matrix on the host");
      free_ctx(c);
      return rc;
    }
    // stored row i is the caller's row perm[i] (i itself without reordering),
    // columns relabelled by iperm; entries keep the caller's order
    rp[0] = 0;
    for (int64_t i = 0; i < n; ++i) rp[i + 1] = rp[i] + rowlen[reorder ? perm[i] : i];
    const unsigned nth = (n < 65536) ? 1u : nth_all;
    std::vector<std::thread> pool;
    for (unsigned t = 0; t < nth; ++t) {
      pool.emplace_back([&, t]() {
        const int64_t i0 = n * t / nth, i1 = n * (t + 1) / nth;
        for (int64_t i = i0; i < i1; ++i) {
          const int64_t r = reorder ? perm[i] : i;
          int64_t pos = rp[i];
          for (int k = 0; k <= nterms; ++k) {
            const HostCSR& h = mats[k];
            for (int64_t q = h.rp[r]; q < h.rp[r + 1]; ++q, ++pos) {
              const uint32_t col = uint32_t(reorder ? iperm[h.col[q]] : h.col[q]);
              colt[pos] = col | (uint32_t(k) << cfet::kTermShift);
              val[2 * pos] = h.val[2 * q];
              val[2 * pos + 1] = h.val[2 * q + 1];
            }
          }
        }
      });
    }
    for (auto& th : pool) th.join();
    c->real_vals = true;
    for (int64_t q = 0; q < nnz && c->real_vals; ++q) c->real_vals = (val[2 * q + 1] == 0.0);
    e = hipMalloc(&c->A.rowptr, (n + 1) * sizeof(int64_t));
    if (e == hipSuccess) e = hipMalloc(&c->A.colt, std::max<int64_t>(nnz, 1) * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMalloc(&c->A.val, std::max<int64_t>(nnz, 1) * sizeof(double2));
    if (e == hipSuccess)
      e = hipMemcpy(c->A.rowptr, rp.data(), (n + 1) * sizeof(int64_t), hipMemcpyHostToDevice);
    if (e == hipSuccess && nnz)
      e = hipMemcpy(c->A.colt, colt.data(), nnz * sizeof(uint32_t), hipMemcpyHostToDevice);
    if (e == hipSuccess && nnz)
      e = hipMemcpy(c->A.val, val.data(), nnz * sizeof(double2), hipMemcpyHostToDevice);
    if (e == hipSuccess && reorder) {
      e = hipMalloc(&c->perm, n * sizeof(int32_t));
      if (e == hipSuccess) e = hipMalloc(&c->iperm, n * sizeof(int32_t));
      if (e == hipSuccess) e = hipMalloc(&c->pv, n * sizeof(double2));
      if (e == hipSuccess) e = hipMalloc(&c->pv2, n * sizeof(double2));
      if (e == hipSuccess)
        e = hipMemcpy(c->perm, perm.data(), n * sizeof(int32_t), hipMemcpyHostToDevice);
      if (e == hipSuccess)
        e = hipMemcpy(c->iperm, iperm.data(), n * sizeof(int32_t), hipMemcpyHostToDevice);
    }
  }
  if (e == hipSuccess && use_sell) {
    const int64_t nsl = (n + 63) / 64;
    // large dimensions default to the uniform-part layout; CFET_LAYOUT_SELL
    // alone asks for plain SELL-64
    const bool auto_layout =
        !(flags & (CFET_LAYOUT_SELL | CFET_LAYOUT_SELL_UNIFORM | CFET_LAYOUT_SELL_SPLIT)) &&
        n > kAutoCoopMaxN;
    const bool uniform =
        (flags & (CFET_LAYOUT_SELL_UNIFORM | CFET_LAYOUT_SELL_SPLIT)) || auto_layout;
    const unsigned nth = (n < 65536) ? 1u : nth_all;
    // the split into two passes: asked for, or the automatic large-dimension
    // layout; kept when the second pass's entries are shared by at least
    // kSharedMinRows rows on average (site operators of spin systems)
    SplitPlan sp;
    SellHiStage HS;
    bool split = false;
    if (((flags & CFET_LAYOUT_SELL_SPLIT) || auto_layout) &&
        plan_split(mats, nterms, n, nth, &sp)) {
      if (!stage_sell_hi(mats, nterms, n, sp, nth, &HS)) {
        rc = fail(c, CFET_ENOMEM, "cannot stage the SELL matrix on the host");
        free_ctx(c);
        return rc;
      }
      split = HS.uptr.back() * kSharedMinRows <= sp.high;
      if (!split) HS = SellHiStage();
    }
    // the tiled kernels take the diagonal apart when it lies in one term and is
    // real (a disordered field: one value per row)
    int diag_term = -1;
    if (split) {
      std::atomic<int32_t> terms_seen{0};
      std::atomic<bool> real{true};
      run_threads(n, nth, [&](int64_t r0, int64_t r1) {
        int32_t tm = 0;
        bool good = true;
        for (int64_t r = r0; r < r1 && good; ++r)
          for_sell_row(mats, nterms, r, [&](int term, int32_t col, const double* v) {
            if (int64_t(col) != r) return;
            tm |= 1 << term;
            if (v[1] != 0.0) good = false;
          });
        terms_seen.fetch_or(tm);
        if (!good) real.store(false);
      });
      const int32_t tm = terms_seen.load();
      if (real.load() && tm != 0 && (tm & (tm - 1)) == 0)
        for (int k = 0; k <= nterms; ++k)
          if (tm == (1 << k)) diag_term = k;
    }
    SellStage S;
    bool staged = stage_sell(mats, nterms, n, rowlen, uniform, split ? sp.split_bit : 0,
                             split ? sp.tbits : 0, diag_term, nth, &S);
    // compact shared lists; the tiled kernels of the split layout read them in
    // groups of four entries
    std::vector<uint64_t> groups1, groups2;
    CommonList common1, common2;
    if (staged && split)
      staged = extract_common(nsl, (1u << sp.tbits) - 1u, nth, &S.nuni, &S.uptr, &S.ucol,
                              &S.uval, &S.umask, &common1) &&
               extract_common(n / 64, 0xFFFFFFFFu, nth, &HS.nuni, &HS.uptr, &HS.ucol, &HS.uval,
                              &HS.umask, &common2);
    if (staged && split)
      staged = arrange_tiled_lists(nsl, (1u << sp.tbits) - 1u, &S.nuni, &S.uptr, &S.ucol,
                                   &S.uval, &S.umask, &groups1) &&
               arrange_tiled_lists(n / 64, 0xFFFFFFFFu, &HS.nuni, &HS.uptr, &HS.ucol, &HS.uval,
                                   &HS.umask, &groups2);
    if (staged && uniform)
      staged = compact_shared_lists(nsl, 1, &S.nuni, &S.uptr, &S.ucol, &S.uval, &S.umask);
    if (staged && split)
      staged = compact_shared_lists(n / 64, 1, &HS.nuni, &HS.uptr, &HS.ucol, &HS.uval, &HS.umask);
    if (!staged) {
      rc = fail(c, CFET_ENOMEM, "cannot stage the SELL matrix on the host");
      free_ctx(c);
      return rc;
    }
    const int64_t slots = S.sptr[nsl];
    c->sell.n = n;
    c->sell.slots = slots;
    e = hipMalloc(&c->sell.slice_ptr, (nsl + 1) * sizeof(int64_t));
    if (e == hipSuccess) e = hipMalloc(&c->sell.slice_width, nsl * sizeof(int32_t));
    if (e == hipSuccess) e = hipMalloc(&c->sell.rowlen, n * sizeof(int32_t));
    if (e == hipSuccess) e = hipMalloc(&c->sell.colt, std::max<int64_t>(slots, 1) * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMalloc(&c->sell.val, std::max<int64_t>(slots, 1) * sizeof(double2));
    if (e == hipSuccess)
      e = hipMemcpy(c->sell.slice_ptr, S.sptr.data(), (nsl + 1) * sizeof(int64_t), hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = hipMemcpy(c->sell.slice_width, S.swid.data(), nsl * sizeof(int32_t), hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = hipMemcpy(c->sell.rowlen, S.rlen.data(), n * sizeof(int32_t), hipMemcpyHostToDevice);
    if (e == hipSuccess && slots)
      e = hipMemcpy(c->sell.colt, S.scol.data(), slots * sizeof(uint32_t), hipMemcpyHostToDevice);
    if (e == hipSuccess && slots)
      e = hipMemcpy(c->sell.val, S.sval.data(), slots * sizeof(double2), hipMemcpyHostToDevice);
    int64_t stored = 0;  // per-row entries actually present (padding excluded)
    for (int64_t r = 0; r < n; ++r) stored += S.rlen[r];
    // row lengths are read only in slices with per-row slots
    int64_t rows_with_slots = 0;
    for (int64_t sl = 0; sl < nsl; ++sl)
      if (S.swid[sl] > 0) rows_with_slots += std::min<int64_t>(64, n - sl * 64);
    c->sell_bytes = 20 * stored + 4 * rows_with_slots + 12 * nsl;
    if (!S.diag.empty()) {
      if (e == hipSuccess) e = hipMalloc(&c->sell.diag, n * sizeof(double));
      if (e == hipSuccess)
        e = hipMemcpy(c->sell.diag, S.diag.data(), n * sizeof(double), hipMemcpyHostToDevice);
      c->sell.diag_term = S.diag_term;
      c->sell_bytes += 8 * n;
    }
    if (uniform) {
      const int64_t us = S.uptr[nsl];
      c->sell.uslots = us;
      if (e == hipSuccess) e = hipMalloc(&c->sell.nuni, nsl * sizeof(int32_t));
      if (e == hipSuccess) e = hipMalloc(&c->sell.uptr, (nsl + 1) * sizeof(int64_t));
      if (e == hipSuccess) e = hipMalloc(&c->sell.ucolt, std::max<int64_t>(us, 1) * sizeof(uint32_t));
      if (e == hipSuccess) e = hipMalloc(&c->sell.uval, std::max<int64_t>(us, 1) * sizeof(double2));
      if (e == hipSuccess) e = hipMalloc(&c->sell.umask, std::max<int64_t>(us, 1) * sizeof(uint64_t));
      if (e == hipSuccess)
        e = hipMemcpy(c->sell.nuni, S.nuni.data(), nsl * sizeof(int32_t), hipMemcpyHostToDevice);
      if (e == hipSuccess)
        e = hipMemcpy(c->sell.uptr, S.uptr.data(), (nsl + 1) * sizeof(int64_t), hipMemcpyHostToDevice);
      if (e == hipSuccess && us)
        e = hipMemcpy(c->sell.ucolt, S.ucol.data(), us * sizeof(uint32_t), hipMemcpyHostToDevice);
      if (e == hipSuccess && us)
        e = hipMemcpy(c->sell.uval, S.uval.data(), us * sizeof(double2), hipMemcpyHostToDevice);
      if (e == hipSuccess && us)
        e = hipMemcpy(c->sell.umask, S.umask.data(), us * sizeof(uint64_t), hipMemcpyHostToDevice);
      c->sell_bytes += 28 * us + 12 * nsl;
    }
    if (split) {
      if (e == hipSuccess) e = hipMalloc(&c->sell.ugroups, nsl * sizeof(uint64_t));
      if (e == hipSuccess)
        e = hipMemcpy(c->sell.ugroups, groups1.data(), nsl * sizeof(uint64_t),
                      hipMemcpyHostToDevice);
      if (e == hipSuccess) e = hipMalloc(&c->hi.ugroups, (n / 64) * sizeof(uint64_t));
      if (e == hipSuccess)
        e = hipMemcpy(c->hi.ugroups, groups2.data(), (n / 64) * sizeof(uint64_t),
                      hipMemcpyHostToDevice);
      // per slice {uptr, ugroups} side by side for the tiled kernels (the group
      // sizes replace the 8-byte uptr and 4-byte nuni they read otherwise)
      for (int p = 0; p < 2 && e == hipSuccess; ++p) {
        const int64_t ns = p == 0 ? nsl : n / 64;
        const std::vector<int64_t>& up = p == 0 ? S.uptr : HS.uptr;
        const std::vector<uint64_t>& gr = p == 0 ? groups1 : groups2;
        std::vector<uint64_t> hdr(2 * size_t(ns));
        for (int64_t sl = 0; sl < ns; ++sl) {
          hdr[2 * size_t(sl)] = uint64_t(up[size_t(sl)]);
          hdr[2 * size_t(sl) + 1] = gr[size_t(sl)];
        }
        uint64_t** dh = p == 0 ? &c->sell.uhdr : &c->hi.uhdr;
        e = hipMalloc(dh, hdr.size() * sizeof(uint64_t));
        if (e == hipSuccess)
          e = hipMemcpy(*dh, hdr.data(), hdr.size() * sizeof(uint64_t), hipMemcpyHostToDevice);
      }
      c->sell_bytes += 8 * nsl + 8 * (n / 64);
      // the common lists (read once per slice from the scalar cache; counted once)
      const CommonList* cl[2] = {&common1, &common2};
      for (int p = 0; p < 2 && e == hipSuccess; ++p) {
        const size_t nc = cl[p]->col.size();
        if (nc == 0) continue;
        uint32_t** dc = p == 0 ? &c->sell.ccolt : &c->hi.ccolt;
        double2** dv = p == 0 ? &c->sell.cval : &c->hi.cval;
        e = hipMalloc(dc, nc * sizeof(uint32_t));
        if (e == hipSuccess) e = hipMalloc(dv, nc * sizeof(double2));
        if (e == hipSuccess)
          e = hipMemcpy(*dc, cl[p]->col.data(), nc * sizeof(uint32_t), hipMemcpyHostToDevice);
        if (e == hipSuccess)
          e = hipMemcpy(*dv, cl[p]->val.data(), nc * sizeof(double2), hipMemcpyHostToDevice);
        (p == 0 ? c->sell.ncd : c->hi.ncd) = cl[p]->nd;
        (p == 0 ? c->sell.nch : c->hi.nch) = cl[p]->nh;
        c->sell_bytes += 20 * int64_t(nc);
      }
    }
    if (split) {
      const int64_t hsl = n / 64;
      const int64_t us = HS.uptr[hsl];
      c->hi.n = n;
      c->hi.nslices = hsl;
      c->hi.nbits = sp.nbits;
      for (int b = 0; b < 32; ++b) c->hi.pos[b] = sp.pos[b];
      c->hi.uslots = us;
      if (e == hipSuccess) e = hipMalloc(&c->hi.nuni, hsl * sizeof(int32_t));
      if (e == hipSuccess) e = hipMalloc(&c->hi.uptr, (hsl + 1) * sizeof(int64_t));
      if (e == hipSuccess) e = hipMalloc(&c->hi.ucolt, std::max<int64_t>(us, 1) * sizeof(uint32_t));
      if (e == hipSuccess) e = hipMalloc(&c->hi.uval, std::max<int64_t>(us, 1) * sizeof(double2));
      if (e == hipSuccess) e = hipMalloc(&c->hi.umask, std::max<int64_t>(us, 1) * sizeof(uint64_t));
      if (e == hipSuccess)
        e = hipMemcpy(c->hi.nuni, HS.nuni.data(), hsl * sizeof(int32_t), hipMemcpyHostToDevice);
      if (e == hipSuccess)
        e = hipMemcpy(c->hi.uptr, HS.uptr.data(), (hsl + 1) * sizeof(int64_t), hipMemcpyHostToDevice);
      if (e == hipSuccess && us)
        e = hipMemcpy(c->hi.ucolt, HS.ucol.data(), us * sizeof(uint32_t), hipMemcpyHostToDevice);
      if (e == hipSuccess && us)
        e = hipMemcpy(c->hi.uval, HS.uval.data(), us * sizeof(double2), hipMemcpyHostToDevice);
      if (e == hipSuccess && us)
        e = hipMemcpy(c->hi.umask, HS.umask.data(), us * sizeof(uint64_t), hipMemcpyHostToDevice);
      c->sell_bytes += 28 * us + 12 * hsl;
      c->tbits = sp.tbits;
      {
        const int64_t ntiles = n >> sp.tbits;
        std::vector<int64_t> trow(ntiles);
        for (int64_t t = 0; t < ntiles; ++t) trow[t] = permuted_row(sp, t << sp.tbits);
        if (e == hipSuccess) e = hipMalloc(&c->hi.tile_row, ntiles * sizeof(int64_t));
        if (e == hipSuccess)
          e = hipMemcpy(c->hi.tile_row, trow.data(), ntiles * sizeof(int64_t),
                        hipMemcpyHostToDevice);
      }
      bool real = true;
      for (size_t q = 1; q < S.sval.size() && real; q += 2) real = (S.sval[q] == 0.0);
      for (size_t q = 1; q < S.uval.size() && real; q += 2) real = (S.uval[q] == 0.0);
      for (size_t q = 1; q < HS.uval.size() && real; q += 2) real = (HS.uval[q] == 0.0);
      for (size_t q = 1; q < common1.val.size() && real; q += 2) real = (common1.val[q] == 0.0);
      for (size_t q = 1; q < common2.val.size() && real; q += 2) real = (common2.val[q] == 0.0);
      c->tile_real = real;
      // real values: the lists also as 64-byte records of four entries
      auto records = [&](const std::vector<uint32_t>& col, const std::vector<double>& val,
                         cfet::Rec4** out) -> hipError_t {
        const size_t nrec = (col.size() + 3) / 4;
        if (nrec == 0) return hipSuccess;
        std::vector<cfet::Rec4> rec(nrec);
        for (size_t i = 0; i < nrec; ++i) {
          std::memset(&rec[i], 0, sizeof(cfet::Rec4));
          for (int u = 0; u < 4; ++u) {
            const size_t e = 4 * i + size_t(u);
            if (e >= col.size()) break;
            rec[i].col[u] = col[e];
            rec[i].val[u] = val[2 * e];
          }
        }
        hipError_t er = hipMalloc(out, nrec * sizeof(cfet::Rec4));
        if (er == hipSuccess)
          er = hipMemcpy(*out, rec.data(), nrec * sizeof(cfet::Rec4), hipMemcpyHostToDevice);
        return er;
      };
      if (real) {
        if (e == hipSuccess) e = records(S.ucol, S.uval, &c->sell.urec);
        if (e == hipSuccess) e = records(HS.ucol, HS.uval, &c->hi.urec);
        if (e == hipSuccess) e = records(common1.col, common1.val, &c->sell.crec);
        if (e == hipSuccess) e = records(common2.col, common2.val, &c->hi.crec);
      }
      if (e == hipSuccess) e = cfet::tile_prepare();
    }
    c->use_sell = true;
  }
  c->plan = cfet::make_plan(n, nnz);
  if (c->use_sell) c->plan.nb_spmv = cfet::sell_grid(n);
  // alpha partials: one per SpMV block and pass
  const int np = std::max(2 * c->plan.nb_spmv, c->plan.nb_vec);
  if (e == hipSuccess) e = hipMalloc(&c->partA, np * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&c->partB, np * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&c->S, sizeof(LzScalars));
  if (e == hipSuccess) e = hipMalloc(&c->stats, sizeof(DevStats));
  if (e == hipSuccess) e = hipHostMalloc(&c->stats_host, sizeof(DevStats));
  if (e == hipSuccess)
    e = hipMalloc(&c->d_bar, cfet::persistent_barrier_words() * sizeof(unsigned long long));
  if (e == hipSuccess) e = hipMalloc(&c->d_fault, sizeof(int));
  if (e == hipSuccess) e = hipEventCreateWithFlags(&c->wts_copied, hipEventDisableTiming);
  if (e == hipSuccess)
    e = hipDeviceGetAttribute(&c->num_cus, hipDeviceAttributeMultiprocessorCount, c->device);
  if (e == hipSuccess) {
    int khz = 0;
    e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, c->device);
    if (khz <= 0) khz = 100000;
    c->spin_limit = (long long)khz * 1000LL * 10LL;  // 10 s
  }
  if (c->hi.nuni) c->nb_tile = cfet::tile_grid(n, c->tbits, c->num_cus);
  c->preset_single = need_csr ? cfet::persistent_choose_preset(c->max_row, n, true) : -1;
  if (e == hipSuccess && c->num_cus > 0 && need_csr) {
    const int64_t nbw = coop_grid_blocks(n, c->num_cus);
    const int64_t rows = (n + nbw - 1) / nbw;
    c->preset_coop = cfet::persistent_choose_preset(c->max_row, rows, false);
    if (c->preset_coop >= 0) {
      int maxb = 0;
      e = cfet::persistent_max_blocks(c->preset_coop, nterms, c->real_vals, &maxb);
      c->coop_blocks = (maxb >= nbw) ? int(nbw) : 0;
      if (c->coop_blocks == 0) c->preset_coop = -1;
    }
  }
  // set up this device's scratch of cfet_propagate_static (first context on
  // the device only): the runtime materialises the array here, not in a call
  // that must not allocate
  if (e == hipSuccess) {
    void* scratch_ptr = nullptr;
    e = cfet::static_scratch(c->device, &scratch_ptr);
  }
  if (e == hipSuccess) e = cfet::launch_stats_init(c->stats, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    rc = hip_fail(c, e, "cfet_create: device setup");
    (void)hipGetLastError();
    g_err = c->err;
    free_ctx(c);
    return rc;
  }
  std::memset(c->stats_host, 0, sizeof(DevStats));
  c->h_W.assign(cfet::kMaxM, nullptr);
  *out = c;
  return CFET_OK;
}

int cfet_destroy(cfet_ctx* c) {
  if (!c) return fail(nullptr, CFET_EINVAL, "null context");
  DeviceGuard g(c->device);
  if (c->have_work) (void)hipStreamSynchronize(c->last_stream);
  free_ctx(c);
  return CFET_OK;
}

int cfet_scheme_info(int32_t scheme, int32_t* s, int32_t* M, double* x, double* g) {
  SchemeTable t;
  if (!cfet::scheme_build(scheme, &t)) return fail(nullptr, CFET_EINVAL, "unknown scheme");
  if (s) *s = t.s;
  if (M) *M = t.M;
  if (x)
    for (int m = 0; m < t.M; ++m) x[m] = t.x[m];
  if (g)
    for (int i = 0; i < t.s; ++i)
      for (int m = 0; m < t.M; ++m) g[i * t.M + m] = t.g[i][m];
  return CFET_OK;
}

int cfet_step_weights(const cfet_ctx* c, double t0, double dt, int64_t nsteps, int32_t scheme,
                      double* a, double* b) {
  if (!c) return fail(nullptr, CFET_EINVAL, "null context");
  SchemeTable t;
  if (!cfet::scheme_build(scheme, &t)) return fail(nullptr, CFET_EINVAL, "unknown scheme");
  if (nsteps < 0 || !a || (nsteps > 0 && !b)) return fail(nullptr, CFET_EINVAL, "bad arguments");
  std::vector<double> bb(t.s * c->nterms);
  for (int64_t n = 0; n < nsteps; ++n) {
    cfet::step_weights(t, c->drives, t0 + double(n) * dt, dt, a, bb.data());
    std::memcpy(b + n * t.s * c->nterms, bb.data(), bb.size() * sizeof(double));
  }
  if (nsteps == 0) {
    for (int i = 0; i < t.s; ++i) {
      double sa = 0.0;
      for (int m = 0; m < t.M; ++m) sa += t.g[i][m];
      a[i] = sa;
    }
  }
  return CFET_OK;
}

int cfet_apply(cfet_ctx* c, const void* x_dev, void* y_dev, double a, const double* b,
               void* hip_stream) {
  if (!c) return fail(nullptr, CFET_EINVAL, "null context");
  if (!x_dev || !y_dev || !b) return fail(c, CFET_EINVAL, "null x, y or b");
  if (x_dev == y_dev) return fail(c, CFET_EINVAL, "x and y must not overlap");
  if (!is_device_ptr(x_dev) || !is_device_ptr(y_dev))
    return fail(c, CFET_EINVAL, "x and y must be device memory");
  DeviceGuard g(c->device);
  cfet::TermWeights tw;
  std::memset(&tw, 0, sizeof(tw));
  tw.w[0] = a;
  for (int k = 0; k < c->nterms; ++k) tw.w[k + 1] = b[k];
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  hipError_t e;
  if (c->use_sell && c->hi.nuni) {
    e = cfet::launch_tile_apply(c->sell, c->hi, c->tbits, c->nb_tile, c->nterms, c->tile_real,
                                tw, static_cast<const double2*>(x_dev),
                                static_cast<double2*>(y_dev), st);
  } else if (c->use_sell) {
    e = cfet::launch_sell_apply(c->sell, c->nterms, tw, static_cast<const double2*>(x_dev),
                                static_cast<double2*>(y_dev), st);
  } else if (c->perm) {  // the stored row order: permute x in and y out
    e = cfet::launch_permute(c->pv, static_cast<const double2*>(x_dev), c->perm, c->n, st);
    if (e == hipSuccess) e = cfet::launch_apply(c->A, c->nterms, c->plan, tw, c->pv, c->pv2, st);
    if (e == hipSuccess)
      e = cfet::launch_permute(static_cast<double2*>(y_dev), c->pv2, c->iperm, c->n, st);
  } else {
    e = cfet::launch_apply(c->A, c->nterms, c->plan, tw, static_cast<const double2*>(x_dev),
                           static_cast<double2*>(y_dev), st);
  }
  if (e != hipSuccess) return hip_fail(c, e, "cfet_apply launch");
  c->last_stream = st;
  c->have_work = true;
  return CFET_OK;
}

}  // extern "C"

namespace {

// The multi-kernel path over nsteps steps on W[0] (the state, stored row
// order), with the Krylov basis W[1..m-1], partial sums partA/partB and
// Lanczos scalars S supplied by the caller (the context's workspace, or the
// static scratch of cfet_propagate_static).  Allocates nothing.
int run_multi(cfet_ctx* c, double t0, double dt, int64_t nsteps, const SchemeTable& sc, int m,
              double2* const* W, double* partA, double* partB, LzScalars* S, bool timed,
              hipStream_t st) {
  hipError_t e;
  cfet::ExpWork wk;
  wk.W_host = W;
  wk.partA = partA;
  wk.partB = partB;
  wk.S = S;
  wk.stats = c->stats;
  wk.sell = c->use_sell ? &c->sell : nullptr;
  wk.hi = (c->use_sell && c->hi.nuni) ? &c->hi : nullptr;
  wk.tbits = c->tbits;
  wk.nb_tile = c->nb_tile;
  wk.tile_real = c->tile_real;
  if (timed) {
    if (c->events.used > 0) {
      (void)hipStreamSynchronize(c->last_stream);
      harvest_events(c);
    }
    wk.events = &c->events;
  } else {
    wk.events = nullptr;
  }
  e = cfet::launch_norm_start(W[0], c->n, c->plan, partA, st);
  if (e != hipSuccess) return hip_fail(c, e, "norm kernel");
  double a[cfet::kMaxStages], b[cfet::kMaxStages * cfet::kMaxTerms];
  cfet::TermWeights tw;
  std::memset(&tw, 0, sizeof(tw));
  for (int64_t n = 0; n < nsteps; ++n) {
    const double tn = t0 + double(n) * dt;
    cfet::step_weights(sc, c->drives, tn, dt, a, b);
    for (int i = sc.s - 1; i >= 0; --i) {
      tw.w[0] = a[i];
      for (int k = 0; k < c->nterms; ++k) tw.w[k + 1] = b[i * c->nterms + k];
      e = cfet::launch_exponential(c->A, c->nterms, c->plan, tw, dt, m, wk, st);
      if (e != hipSuccess) return hip_fail(c, e, "exponential kernels");
    }
  }
  e = cfet::launch_final_norm(partA, c->plan.nb_vec, c->stats, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->stats_host, c->stats, sizeof(DevStats), hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return hip_fail(c, e, "final kernels");
  c->last_stream = st;
  c->have_work = true;
  c->last_path = 1;
  return CFET_OK;
}

// y = H_w x in the stored row order on the layout of the multi-kernel path.
hipError_t apply_stored(cfet_ctx* c, const cfet::TermWeights& tw, const double2* x, double2* y,
                        hipStream_t st) {
  if (c->use_sell && c->hi.nuni)
    return cfet::launch_tile_apply(c->sell, c->hi, c->tbits, c->nb_tile, c->nterms, c->tile_real,
                                   tw, x, y, st);
  if (c->use_sell) return cfet::launch_sell_apply(c->sell, c->nterms, tw, x, y, st);
  return cfet::launch_apply(c->A, c->nterms, c->plan, tw, x, y, st);
}

// The CFET step loop with Chebyshev exponentials on psi (stored row order):
// per exponential the interval of H_i = a_i H0 + sum_k b_ik H_k from the terms'
// Gershgorin intervals (a negative weight swaps the ends), sigma and h its
// centre and half-width, theta = dt h, K terms for tol, and
//   psi <- e^{-i dt sigma} sum_{k<=K} (2 - delta_k0) (-i)^k J_k(theta) T_k(H~) psi,
// H~ = (H_i - sigma) / h, by the three-term recurrence of T_k.
int run_cheb(cfet_ctx* c, double t0, double dt, int64_t nsteps, const SchemeTable& sc, double tol,
             double2* psi, hipStream_t st) {
  hipError_t e = hipSuccess;
  double2* V[3] = {c->h_W[1], c->h_W[2], c->h_W[3]};
  const bool timed = c->profiling;
  if (timed && c->events.used > 0) {
    (void)hipStreamSynchronize(c->last_stream);
    harvest_events(c);
  }
  double a[cfet::kMaxStages], b[cfet::kMaxStages * cfet::kMaxTerms];
  std::vector<double> J;
  cfet::TermWeights tw;
  std::memset(&tw, 0, sizeof(tw));
  for (int64_t n = 0; n < nsteps; ++n) {
    const double tn = t0 + double(n) * dt;
    cfet::step_weights(sc, c->drives, tn, dt, a, b);
    for (int i = sc.s - 1; i >= 0; --i) {
      tw.w[0] = a[i];
      for (int k = 0; k < c->nterms; ++k) tw.w[k + 1] = b[i * c->nterms + k];
      double lo = 0.0, hi = 0.0;
      for (int k = 0; k <= c->nterms; ++k) {
        const double w = tw.w[k];
        if (w >= 0.0) {
          lo += w * c->glo[k];
          hi += w * c->ghi[k];
        } else {
          lo += w * c->ghi[k];
          hi += w * c->glo[k];
        }
      }
      const double sigma = 0.5 * (lo + hi), h = 0.5 * (hi - lo);
      const double ph = -dt * sigma;
      const double2 phase = make_double2(std::cos(ph), std::sin(ph));
      const int K = h > 0.0 ? cheb_terms(dt * h, tol) : 0;
      J.assign(size_t(K) + 1, 0.0);
      if (h > 0.0)
        bessel_j(dt * h, K, J.data());
      else
        J[0] = 1.0;
      // c_k = (2 - delta_k0) (-i)^k J_k e^{-i dt sigma}
      auto coef = [&](int k) {
        const double m = (k == 0 ? 1.0 : 2.0) * J[size_t(k)];
        double re = 0.0, im = 0.0;   // (-i)^k m
        switch (k & 3) {
          case 0: re = m; break;
          case 1: im = -m; break;
          case 2: re = -m; break;
          default: im = m; break;
        }
        return make_double2(re * phase.x - im * phase.y, re * phase.y + im * phase.x);
      };
      e = cfet::launch_cheb_start(psi, V[0], c->n, coef(0), K, c->stats, st);
      if (e != hipSuccess) return hip_fail(c, e, "Chebyshev start");
      double2* cur = V[0];
      double2* prev = V[1];
      double2* y = V[2];
      for (int k = 1; k <= K; ++k) {
        const bool ev = timed && c->events.used < c->events.cap;
        const double scale = (k == 1 ? 1.0 : 2.0) / h;
        if (ev) (void)hipEventRecord(c->events.begin[c->events.used], st);
        if (c->use_sell && c->hi.nuni) {
          // split layout: the term is applied in the second pass's epilogue
          const cfet::ChebTerm ct{prev, psi, scale, sigma, coef(k), k == 1 ? 1 : 0};
          e = cfet::launch_tile_cheb(c->sell, c->hi, c->tbits, c->nb_tile, c->nterms,
                                     c->tile_real, tw, cur, y, ct, st);
          if (e != hipSuccess) return hip_fail(c, e, "Chebyshev apply");
        } else {
          e = apply_stored(c, tw, cur, y, st);
          if (e != hipSuccess) return hip_fail(c, e, "Chebyshev apply");
        }
        if (ev) {
          (void)hipEventRecord(c->events.end[c->events.used], st);
          c->events.used += 1;
        }
        if (!(c->use_sell && c->hi.nuni)) {
          e = cfet::launch_cheb_update(y, cur, prev, psi, c->n, scale, sigma, k == 1, coef(k), st);
          if (e != hipSuccess) return hip_fail(c, e, "Chebyshev update");
        }
        std::swap(cur, prev);
      }
    }
  }
  e = hipMemcpyAsync(c->stats_host, c->stats, sizeof(DevStats), hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return hip_fail(c, e, "statistics");
  c->last_stream = st;
  c->have_work = true;
  c->last_path = 1;
  return CFET_OK;
}

// cfet_propagate on psi_dev in the stored row order (user_order false: the
// gradient's own buffers) or in the caller's order (permuted in and out when
// the CSR paths run on a row order of their own).
int propagate_impl(cfet_ctx* c, void* psi_dev, double t0, double dt, int64_t nsteps,
                   int32_t scheme, int32_t krylov_m, void* hip_stream, bool user_order) {
  if (!c) return fail(nullptr, CFET_EINVAL, "null context");
  if (!psi_dev) return fail(c, CFET_EINVAL, "null psi");
  if (nsteps < 0) return fail(c, CFET_EINVAL, "nsteps < 0");
  if (krylov_m < 1 || krylov_m > CFET_MAX_KRYLOV)
    return fail(c, CFET_EINVAL, "krylov_m must be in 1..64");
  if (!std::isfinite(t0) || !std::isfinite(dt)) return fail(c, CFET_EINVAL, "non-finite t0/dt");
  SchemeTable sc;
  if (!cfet::scheme_build(scheme, &sc)) return fail(c, CFET_EINVAL, "unknown scheme");
  if (!is_device_ptr(psi_dev)) return fail(c, CFET_EINVAL, "psi must be device memory");
  DeviceGuard g(c->device);
  // report a fault latched by earlier work that has already finished
  if (c->have_work && hipStreamQuery(c->last_stream) == hipSuccess &&
      c->stats_host->status != CFET_OK) {
    const int st = c->stats_host->status;
    c->stats_host->status = CFET_OK;
    return fail(c, st, "device fault latched by an earlier call (see cfet_stats)");
  }
  if (nsteps == 0) return CFET_OK;
  const int m = int(std::min<int64_t>(krylov_m, c->n));
  int rc = ensure_workspace(c, m);
  if (rc != CFET_OK) return rc;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const int path = choose_path(c);
  void* const user_psi = psi_dev;
  const bool permute = user_order && c->perm;
  if (permute) {
    const hipError_t ep = cfet::launch_permute(c->pv, static_cast<const double2*>(user_psi),
                                               c->perm, c->n, st);
    if (ep != hipSuccess) return hip_fail(c, ep, "permute psi in");
    psi_dev = c->pv;
  }
  auto permute_out = [&]() -> int {
    if (!permute) return CFET_OK;
    const hipError_t ep =
        cfet::launch_permute(static_cast<double2*>(user_psi), c->pv, c->iperm, c->n, st);
    return ep == hipSuccess ? CFET_OK : hip_fail(c, ep, "permute psi out");
  };
  if (path != 1) {
    const int rp = propagate_persistent(c, psi_dev, t0, dt, nsteps, sc, m, path, st);
    return rp == CFET_OK ? permute_out() : rp;
  }
  c->h_W[0] = static_cast<double2*>(psi_dev);
  const int rm = run_multi(c, t0, dt, nsteps, sc, m, c->h_W.data(), c->partA, c->partB, c->S,
                           c->profiling, st);
  return rm == CFET_OK ? permute_out() : rm;
}

}  // namespace

extern "C" {

int cfet_propagate(cfet_ctx* c, void* psi_dev, double t0, double dt, int64_t nsteps,
                   int32_t scheme, int32_t krylov_m, void* hip_stream) {
  return propagate_impl(c, psi_dev, t0, dt, nsteps, scheme, krylov_m, hip_stream, true);
}

int cfet_propagate_static(cfet_ctx* c, void* psi_dev, double t0, double dt, int64_t nsteps,
                          int32_t scheme, int32_t krylov_m, void* hip_stream) {
  if (!c) return fail(nullptr, CFET_EINVAL, "null context");
  if (!psi_dev) return fail(c, CFET_EINVAL, "null psi");
  if (nsteps < 0) return fail(c, CFET_EINVAL, "nsteps < 0");
  if (krylov_m < 1 || krylov_m > CFET_MAX_KRYLOV)
    return fail(c, CFET_EINVAL, "krylov_m must be in 1..64");
  if (!std::isfinite(t0) || !std::isfinite(dt)) return fail(c, CFET_EINVAL, "non-finite t0/dt");
  SchemeTable sc;
  if (!cfet::scheme_build(scheme, &sc)) return fail(c, CFET_EINVAL, "unknown scheme");
  if (!is_device_ptr(psi_dev)) return fail(c, CFET_EINVAL, "psi must be device memory");
  DeviceGuard g(c->device);
  if (c->have_work && hipStreamQuery(c->last_stream) == hipSuccess &&
      c->stats_host->status != CFET_OK) {
    const int st = c->stats_host->status;
    c->stats_host->status = CFET_OK;
    return fail(c, st, "device fault latched by an earlier call (see cfet_stats)");
  }
  const int m = int(std::min<int64_t>(krylov_m, c->n));
  // scratch layout: Lanczos scalars, two partial-sum arrays, the state in
  // the stored row order (reordered operators only), the basis vectors 1..m-1
  auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
  const size_t np = size_t(std::max(2 * c->plan.nb_spmv, c->plan.nb_vec));
  const size_t nn = size_t(c->n);
  const size_t off_a = up(sizeof(LzScalars));
  const size_t off_b = off_a + up(np * sizeof(double));
  const size_t off_pv = off_b + up(np * sizeof(double));
  const size_t off_basis = off_pv + (c->perm ? up(nn * sizeof(double2)) : 0);
  const size_t need = off_basis + size_t(m - 1) * nn * sizeof(double2);
  if (need > cfet::static_scratch_bytes())
    return fail(c, CFET_EINVAL,
                "cfet_propagate_static: the problem needs " + std::to_string(need) +
                    " bytes of scratch (Krylov basis of n (m - 1) complex values), more than "
                    "the " + std::to_string(cfet::static_scratch_bytes()) + " it has");
  if (nsteps == 0) return CFET_OK;
  void* base = nullptr;
  hipError_t e = cfet::static_scratch(c->device, &base);
  if (e != hipSuccess) return hip_fail(c, e, "cfet_propagate_static: scratch address");
  char* sb = static_cast<char*>(base);
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  double2* W[cfet::kMaxM] = {};
  W[0] = static_cast<double2*>(psi_dev);
  if (c->perm) {
    W[0] = reinterpret_cast<double2*>(sb + off_pv);
    e = cfet::launch_permute(W[0], static_cast<const double2*>(psi_dev), c->perm, c->n, st);
    if (e != hipSuccess) return hip_fail(c, e, "permute psi in");
  }
  for (int j = 1; j < m; ++j)
    W[j] = reinterpret_cast<double2*>(sb + off_basis) + size_t(j - 1) * nn;
  int rc = run_multi(c, t0, dt, nsteps, sc, m, W, reinterpret_cast<double*>(sb + off_a),
                     reinterpret_cast<double*>(sb + off_b), reinterpret_cast<LzScalars*>(sb),
                     false, st);
  if (rc == CFET_OK && c->perm) {
    e = cfet::launch_permute(static_cast<double2*>(psi_dev), W[0], c->iperm, c->n, st);
    if (e != hipSuccess) rc = hip_fail(c, e, "permute psi out");
  }
  return rc;
}

int cfet_propagate_chebyshev(cfet_ctx* c, void* psi_dev, double t0, double dt, int64_t nsteps,
                             int32_t scheme, double tol, void* hip_stream) {
  if (!c) return fail(nullptr, CFET_EINVAL, "null context");
  if (!psi_dev) return fail(c, CFET_EINVAL, "null psi");
  if (nsteps < 0) return fail(c, CFET_EINVAL, "nsteps < 0");
  if (!(tol > 0.0 && tol < 1.0)) return fail(c, CFET_EINVAL, "tol must be in (0, 1)");
  if (!std::isfinite(t0) || !std::isfinite(dt)) return fail(c, CFET_EINVAL, "non-finite t0/dt");
  SchemeTable sc;
  if (!cfet::scheme_build(scheme, &sc)) return fail(c, CFET_EINVAL, "unknown scheme");
  if (!is_device_ptr(psi_dev)) return fail(c, CFET_EINVAL, "psi must be device memory");
  DeviceGuard g(c->device);
  if (c->have_work && hipStreamQuery(c->last_stream) == hipSuccess &&
      c->stats_host->status != CFET_OK) {
    const int st = c->stats_host->status;
    c->stats_host->status = CFET_OK;
    return fail(c, st, "device fault latched by an earlier call (see cfet_stats)");
  }
  if (nsteps == 0) return CFET_OK;
  int rc = ensure_workspace(c, 4);
  if (rc != CFET_OK) return rc;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  double2* psi = static_cast<double2*>(psi_dev);
  hipError_t e;
  if (c->perm) {
    e = cfet::launch_permute(c->pv, psi, c->perm, c->n, st);
    if (e != hipSuccess) return hip_fail(c, e, "permute psi in");
    psi = c->pv;
  }
  rc = run_cheb(c, t0, dt, nsteps, sc, tol, psi, st);
  if (rc == CFET_OK && c->perm) {
    e = cfet::launch_permute(static_cast<double2*>(psi_dev), c->pv, c->iperm, c->n, st);
    if (e != hipSuccess) rc = hip_fail(c, e, "permute psi out");
  }
  return rc;
}

int cfet_profile(cfet_ctx* c, int32_t enable, int32_t max_launches) {
  if (!c) return fail(nullptr, CFET_EINVAL, "null context");
  DeviceGuard g(c->device);
  if (c->have_work) (void)hipStreamSynchronize(c->last_stream);
  harvest_events(c);
  free_events(c);
  c->profiling = false;
  c->seg_timers = false;
  c->timed_launches = 0;
  c->timed_ms = 0.0;
  if (!enable) return CFET_OK;
  if (max_launches < 1 || max_launches > (1 << 20))
    return fail(c, CFET_EINVAL, "max_launches must be in 1..2^20");
  c->events.begin = new (std::nothrow) hipEvent_t[max_launches]();
  c->events.end = new (std::nothrow) hipEvent_t[max_launches]();
  if (!c->events.begin || !c->events.end) {
    free_events(c);
    return fail(c, CFET_ENOMEM, "cannot allocate the event pool");
  }
  c->events.cap = max_launches;
  for (int i = 0; i < max_launches; ++i) {
    hipError_t e = hipEventCreate(&c->events.begin[i]);
    if (e == hipSuccess) e = hipEventCreate(&c->events.end[i]);
    if (e != hipSuccess) {
      free_events(c);
      return hip_fail(c, e, "hipEventCreate");
    }
  }
  c->profiling = true;
  c->seg_timers = (enable != 2);
  return CFET_OK;
}

int cfet_gradient(cfet_ctx* c, const void* psi0_dev, const void* target_dev, double t0,
                  double dt, int64_t nsteps, int32_t scheme, int32_t krylov_m, const double* u,
                  int32_t K, double* F_out, double* dFdu_out, void* hip_stream) {
  if (!c) return fail(nullptr, CFET_EINVAL, "null context");
  if (!psi0_dev || !target_dev || !F_out) return fail(c, CFET_EINVAL, "null psi0, target or F");
  if (K < 1 || !dFdu_out) return fail(c, CFET_EINVAL, "K must be >= 1 with an output array");
  if (nsteps < 0) return fail(c, CFET_EINVAL, "nsteps < 0");
  if (krylov_m < 1 || krylov_m > CFET_MAX_KRYLOV)
    return fail(c, CFET_EINVAL, "krylov_m must be in 1..64");
  if (!std::isfinite(t0) || !std::isfinite(dt)) return fail(c, CFET_EINVAL, "non-finite t0/dt");
  SchemeTable sc;
  if (!cfet::scheme_build(scheme, &sc)) return fail(c, CFET_EINVAL, "unknown scheme");
  if (!is_device_ptr(psi0_dev) || !is_device_ptr(target_dev))
    return fail(c, CFET_EINVAL, "psi0 and target must be device memory");
  if (!c->A.rowptr)
    return fail(c, CFET_EUNSUPPORTED,
                "cfet_gradient needs the CSR operator (dimension <= 2^22, or CFET_KEEP_CSR)");
  int kstar = -1;
  for (int k = 0; k < c->nterms && kstar < 0; ++k)
    if (c->drives[k].kind == CFET_DRIVE_PWC) kstar = k;
  if (kstar < 0) return fail(c, CFET_EINVAL, "no driven term has a piecewise-constant drive");
  if (int(c->drives[kstar].u.size()) != K)
    return fail(c, CFET_EINVAL, "K differs from the number of pieces of the drive");
  std::vector<DriveSpec> dmod = c->drives;
  if (u) {
    for (int p = 0; p < K; ++p)
      if (!std::isfinite(u[p])) return fail(c, CFET_EINVAL, "non-finite amplitude");
    dmod[kstar].u.assign(u, u + K);
  }
  DeviceGuard g(c->device);
  const int64_t n = c->n;
  const int m = int(std::min<int64_t>(krylov_m, n));
  int rc = ensure_workspace(c, m);
  if (rc != CFET_OK) return rc;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  // the call propagates with the given amplitudes: swap them in for its duration
  struct DriveSwap {
    cfet_ctx* c;
    std::vector<DriveSpec>& d;
    DriveSwap(cfet_ctx* c_, std::vector<DriveSpec>& d_) : c(c_), d(d_) { std::swap(c->drives, d); }
    ~DriveSwap() { std::swap(c->drives, d); }
  } swap_guard(c, dmod);

  const int64_t N = nsteps;
  const int64_t seg = (N > 0) ? std::max<int64_t>(1, int64_t(std::ceil(std::sqrt(double(N))))) : 1;
  const int64_t nseg = (N + seg - 1) / seg;
  GradBuffers gb;
  double2 *psi = nullptr, *lam = nullptr, *vpsi = nullptr, *vlam = nullptr, *ckpt = nullptr,
          *before = nullptr, *cpart = nullptr, *cmat = nullptr, *dz = nullptr, *zval = nullptr,
          *zpart = nullptr;
  LzScalars *Spsi = nullptr, *Slam = nullptr;
  const size_t nn = size_t(n);
  // The segment recomputation and the backward exponentials run on the
  // persistent path when the operator fits it; otherwise exponential by
  // exponential on the multi-kernel path.  With one driven term on a
  // persistent path the recomputation also keeps, for every exponential, its
  // projection and Y_j = H_1 w_j (the kernel forms that term apart anyway):
  // the backward sweep then runs no Lanczos recurrence from psi.  That store
  // takes seg * s * m vectors; above kGradStoreMax (or half the free device
  // memory) the recurrence from psi is rerun instead, with the same result.
  const int rpath = choose_path(c);
  const size_t ystore = size_t(seg) * size_t(sc.s) * size_t(m) * nn * sizeof(double2);
  bool keep = rpath != 1 && c->nterms == 1 && ystore <= kGradStoreMax;
  if (keep) {
    size_t free_b = 0, total_b = 0;
    keep = hipMemGetInfo(&free_b, &total_b) == hipSuccess && ystore <= free_b / 2;
  }
  double2* Yall = nullptr;
  LzScalars* Tall = nullptr;
  hipError_t e = gb.get(&psi, nn);
  if (e == hipSuccess) e = gb.get(&lam, nn);
  if (e == hipSuccess) e = gb.get(&vpsi, size_t(std::max(m - 1, 1)) * nn);
  if (e == hipSuccess) e = gb.get(&vlam, size_t(std::max(m - 1, 1)) * nn);
  if (e == hipSuccess) e = gb.get(&ckpt, size_t(std::max<int64_t>(nseg, 1)) * nn);
  if (e == hipSuccess && !keep) e = gb.get(&before, size_t(seg) * size_t(sc.s) * nn);
  if (e == hipSuccess && keep) e = gb.get(&Yall, size_t(seg) * size_t(sc.s) * size_t(m) * nn);
  if (e == hipSuccess && keep) e = gb.get(&Tall, size_t(seg) * size_t(sc.s));
  if (e == hipSuccess)
    e = gb.get(&cpart, size_t(cfet::frechet_part_blocks(n)) * cfet::kMaxM * cfet::kMaxM);
  if (e == hipSuccess) e = gb.get(&cmat, size_t(cfet::kMaxM) * cfet::kMaxM);
  if (e == hipSuccess) e = gb.get(&dz, size_t(K));
  if (e == hipSuccess) e = gb.get(&zval, 1);
  if (e == hipSuccess) e = gb.get(&zpart, size_t(cfet::zdot_blocks(n)));
  if (e == hipSuccess) e = gb.get(&Spsi, 1);
  if (e == hipSuccess) e = gb.get(&Slam, 1);
  if (e != hipSuccess) return hip_fail(c, e, "cfet_gradient: workspace");
  const size_t vb = nn * sizeof(double2);
  // ---- forward pass, keeping psi at the start of every segment
  // psi and lambda live in the stored row order
  e = c->perm ? cfet::launch_permute(psi, static_cast<const double2*>(psi0_dev), c->perm, n, st)
              : hipMemcpyAsync(psi, psi0_dev, vb, hipMemcpyDeviceToDevice, st);
  for (int64_t sg = 0; sg < nseg && e == hipSuccess; ++sg) {
    e = hipMemcpyAsync(ckpt + size_t(sg) * nn, psi, vb, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) break;
    const int64_t s0 = sg * seg, len = std::min(seg, N - s0);
    rc = propagate_impl(c, psi, t0 + double(s0) * dt, dt, len, scheme, m, st, false);
    if (rc != CFET_OK) return rc;
  }
  if (e == hipSuccess)
    e = c->perm ? cfet::launch_permute(lam, static_cast<const double2*>(target_dev), c->perm, n, st)
                : hipMemcpyAsync(lam, target_dev, vb, hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess) e = cfet::launch_zdot(lam, psi, n, zpart, zval, st);
  if (e == hipSuccess) e = cfet::launch_zero2(dz, K, st);
  if (e != hipSuccess) return hip_fail(c, e, "cfet_gradient: forward pass");

  // ---- backward sweep, one segment at a time
  std::vector<double2*> Wf(cfet::kMaxM, nullptr), Wp(cfet::kMaxM, nullptr),
      Wl(cfet::kMaxM, nullptr);
  for (int j = 1; j < m; ++j) {
    Wf[j] = c->h_W[j];
    Wp[j] = vpsi + size_t(j - 1) * nn;
    Wl[j] = vlam + size_t(j - 1) * nn;
  }
  cfet::ExpWork wf{}, wp{}, wl{};
  wf.W_host = Wf.data();
  wp.W_host = Wp.data();
  wl.W_host = Wl.data();
  wf.partA = wp.partA = wl.partA = c->partA;
  wf.partB = wp.partB = wl.partB = c->partB;
  wf.S = c->S;
  wp.S = Spsi;
  wl.S = Slam;
  wf.stats = wp.stats = wl.stats = c->stats;
  wf.sell = wp.sell = wl.sell = nullptr;
  wf.events = wp.events = wl.events = nullptr;
  const DriveSpec& dk = c->drives[kstar];
  std::vector<double> a(sc.s), b(size_t(sc.s) * c->nterms);
  Wl[0] = lam;
  // One backward exponential: Lanczos from psi (before the exponential) and
  // from lambda, the Frechet term, lambda moved back.  It reads its weights,
  // its db/du pairs and the state before it from device memory (record
  // *cursor, uploaded once per segment), so the same launches serve every
  // exponential.  (Replaying them as a captured graph measured 9 % slower than
  // enqueueing them: the kernels, not their submission, set the time.)
  cfet::GradRec *d_recs = nullptr, *d_cur = nullptr;
  int* d_cursor = nullptr;
  double2* pb = nullptr;
  double2* lam0 = nullptr;  // lambda after the exponential, kept as the first basis vector
  if (e == hipSuccess) e = gb.get(&d_recs, size_t(seg) * sc.s);
  if (e == hipSuccess) e = gb.get(&lam0, nn);
  if (e == hipSuccess) e = gb.get(&d_cur, 1);
  if (e == hipSuccess) e = gb.get(&d_cursor, 1);
  if (e == hipSuccess) e = gb.get(&pb, nn);
  if (e != hipSuccess) return hip_fail(c, e, "cfet_gradient: workspace");
  cfet::GradRec* h_recs = nullptr;  // pinned staging of one segment's records and cursor
  e = hipHostMalloc(reinterpret_cast<void**>(&h_recs), (size_t(seg) * sc.s + 1) * sizeof(cfet::GradRec));
  if (e != hipSuccess) return hip_fail(c, e, "cfet_gradient: pinned staging");
  struct PinnedGuard {
    void* p;
    ~PinnedGuard() { (void)hipHostFree(p); }
  } pin_guard{h_recs};
  const cfet::TermWeights* dtw = reinterpret_cast<const cfet::TermWeights*>(
      reinterpret_cast<const char*>(d_cur) + offsetof(cfet::GradRec, tw));
  Wp[0] = pb;
  wp.twp = dtw;
  wl.twp = dtw;
  cfet::TermWeights tw0;
  std::memset(&tw0, 0, sizeof(tw0));
  const double* dw = reinterpret_cast<const double*>(dtw);
  // one driven term without the store: the recurrence from psi still exports
  // Y_j, and C is the product of two stored blocks of vectors
  double2* vY = nullptr;
  if (rpath != 1 && c->nterms == 1 && !keep) {
    e = gb.get(&vY, size_t(m) * nn);
    if (e != hipSuccess) return hip_fail(c, e, "cfet_gradient: workspace");
  }
  // barrier state of the two persistent launches per exponential, cleared by
  // the prologue (one launch fewer each)
  const int bw = cfet::persistent_barrier_words();
  unsigned long long* gbar = nullptr;
  if (rpath != 1) {
    e = gb.get(&gbar, size_t(2) * bw);
    if (e != hipSuccess) return hip_fail(c, e, "cfet_gradient: workspace");
  }
  auto enqueue_back = [&](hipStream_t s_, size_t ix) -> hipError_t {
    // the persistent exponential of lambda overwrites lambda with its result:
    // its first basis vector is then read from the copy lam0
    if (keep) {
      // record ix: weights, pieces, and the projection and Y of the recurrence
      // from psi kept by the recomputation
      const cfet::GradRec* rx = d_recs + ix;
      const double* wx = reinterpret_cast<const double*>(reinterpret_cast<const char*>(rx) +
                                                         offsetof(cfet::GradRec, tw));
      LzScalars* Tx = Tall + ix;
      hipError_t x = cfet::launch_grad_prologue(nullptr, nullptr, nullptr, nullptr, n, nullptr,
                                                lam, lam0, gbar, bw, c->d_fault, s_);
      if (x == hipSuccess)
        x = persistent_exponential(c, rpath, lam, vlam, wx, -dt, m, Slam, false, s_, nullptr,
                                   gbar);
      if (x == hipSuccess)
        x = cfet::launch_frechet_dots(n, lam0, vlam, Yall + ix * size_t(m) * nn, Tx, Slam, cpart,
                                      cmat, s_);
      if (x == hipSuccess)
        x = cfet::launch_frechet_small_rec(Tx, Slam, cmat, dt, rx, dz, c->stats, nullptr, m, s_);
      return x;
    }
    hipError_t x = cfet::launch_grad_prologue(d_recs, d_cursor, d_cur, before, n, pb, lam,
                                              rpath != 1 ? lam0 : nullptr, gbar, 2 * bw,
                                              c->d_fault, s_);
    if (rpath != 1) {
      // two persistent launches: the recurrence from psi (kept, not combined)
      // and the exponential of lambda (with -dt), both exporting their projection
      if (x == hipSuccess)
        x = persistent_exponential(c, rpath, pb, vpsi, dw, dt, m, Spsi, true, s_, vY, gbar);
      if (x == hipSuccess)
        x = persistent_exponential(c, rpath, lam, vlam, dw, -dt, m, Slam, false, s_, nullptr,
                                   gbar + bw);
    } else {
      if (x == hipSuccess) x = cfet::launch_norm_start(pb, n, c->plan, c->partA, s_);
      if (x == hipSuccess) x = cfet::launch_lanczos(c->A, c->nterms, c->plan, tw0, dt, m, wp, s_);
      if (x == hipSuccess) x = cfet::launch_norm_start(lam, n, c->plan, c->partA, s_);
      if (x == hipSuccess) x = cfet::launch_lanczos(c->A, c->nterms, c->plan, tw0, -dt, m, wl, s_);
    }
    if (x == hipSuccess && vY)
      x = cfet::launch_frechet_dots(n, lam0, vlam, vY, Spsi, Slam, cpart, cmat, s_);
    else if (x == hipSuccess)
      x = cfet::launch_frechet_c(c->A, kstar + 1, pb, vpsi, rpath != 1 ? lam0 : lam, vlam, Spsi,
                                 Slam, cpart, cmat, s_);
    if (x == hipSuccess)
      x = cfet::launch_frechet_small_rec(Spsi, Slam, cmat, dt, d_cur, dz, c->stats, d_cursor, m,
                                          s_);
    if (x == hipSuccess && rpath == 1) x = cfet::launch_combine(n, c->plan, wl, s_);
    return x;
  };
  hipEvent_t staged = nullptr;
  e = hipEventCreateWithFlags(&staged, hipEventDisableTiming);
  if (e != hipSuccess) return hip_fail(c, e, "cfet_gradient: event");
  struct EventGuard {
    hipEvent_t ev;
    ~EventGuard() { (void)hipEventDestroy(ev); }
  } ev_guard{staged};
  bool staged_pending = false;

  for (int64_t sg = nseg - 1; sg >= 0 && e == hipSuccess; --sg) {
    const int64_t s0 = sg * seg, s1 = std::min(N, s0 + seg);
    e = hipMemcpyAsync(psi, ckpt + size_t(sg) * nn, vb, hipMemcpyDeviceToDevice, st);
    Wf[0] = psi;
    if (e == hipSuccess && rpath != 1) {
      rc = propagate_persistent(c, psi, t0 + double(s0) * dt, dt, s1 - s0, sc, m, rpath, st,
                                before, Tall, Yall);
      if (rc != CFET_OK) return rc;
    } else if (e == hipSuccess) {
      e = cfet::launch_norm_start(psi, n, c->plan, c->partA, st);
    }
    // records of this segment's exponentials (application order)
    if (staged_pending) (void)hipEventSynchronize(staged);
    staged_pending = false;
    size_t idx = 0;
    for (int64_t q = s0; q < s1 && e == hipSuccess; ++q) {
      const double tn = t0 + double(q) * dt;
      cfet::step_weights(sc, c->drives, tn, dt, a.data(), b.data());
      for (int i = sc.s - 1; i >= 0 && e == hipSuccess; --i, ++idx) {
        cfet::GradRec& r = h_recs[idx];
        std::memset(&r, 0, sizeof(r));
        r.tw.w[0] = a[i];
        for (int k = 0; k < c->nterms; ++k) r.tw.w[k + 1] = b[size_t(i) * c->nterms + k];
        r.np = 0;
        for (int mm = 0; mm < sc.M; ++mm) {
          const int p = pwc_piece(dk, tn + sc.x[mm] * dt);
          if (p < 0) continue;
          int slot = 0;
          while (slot < r.np && r.p[slot] != p) ++slot;
          if (slot == r.np) {
            r.p[r.np] = p;
            r.w[r.np] = 0.0;
            r.np += 1;
          }
          r.w[slot] += sc.g[i][mm];
        }
        if (rpath == 1) {
          e = hipMemcpyAsync(before + idx * nn, psi, vb, hipMemcpyDeviceToDevice, st);
          if (e == hipSuccess)
            e = cfet::launch_exponential(c->A, c->nterms, c->plan, r.tw, dt, m, wf, st);
        }
      }
    }
    // the cursor starts at the last exponential of the segment
    int* hcur = reinterpret_cast<int*>(&h_recs[idx]);
    *hcur = int(idx) - 1;
    if (e == hipSuccess)
      e = hipMemcpyAsync(d_recs, h_recs, idx * sizeof(cfet::GradRec), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(d_cursor, hcur, sizeof(int), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipEventRecord(staged, st);
    if (e == hipSuccess) staged_pending = true;
    for (size_t x = idx; x-- > 0 && e == hipSuccess;) e = enqueue_back(st, x);
  }
  if (e != hipSuccess) return hip_fail(c, e, "cfet_gradient: backward sweep");
  std::vector<double2> hz(size_t(K) + 1);
  e = hipMemcpyAsync(hz.data(), dz, sizeof(double2) * K, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipMemcpyAsync(&hz[K], zval, sizeof(double2), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->stats_host, c->stats, sizeof(DevStats), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(c, e, "cfet_gradient: results");
  c->last_stream = st;
  c->have_work = true;
  const double2 z = hz[K];
  *F_out = z.x * z.x + z.y * z.y;
  for (int p = 0; p < K; ++p) dFdu_out[p] = 2.0 * (z.x * hz[p].x + z.y * hz[p].y);
  if (c->stats_host->status != CFET_OK) {
    const int code = c->stats_host->status;
    return fail(c, code, "cfet_gradient: device fault (non-finite values or no convergence)");
  }
  return CFET_OK;
}

int cfet_select_dt(cfet_ctx* c, const void* psi0_dev, double t0, double window, int32_t n1,
                   int32_t checkpoints, double ratio, int32_t scheme, int32_t krylov_m,
                   double T_total, double eps, int32_t verify, int32_t refine,
                   cfet_dt_choice* out, void* hip_stream) {
  if (!c) return fail(nullptr, CFET_EINVAL, "null context");
  if (!psi0_dev || !out) return fail(c, CFET_EINVAL, "null psi0 or output");
  if (!(window > 0.0) || !(T_total > 0.0) || !(eps > 0.0) || !(ratio > 1.0) ||
      !std::isfinite(window) || !std::isfinite(T_total) || !std::isfinite(ratio) ||
      !std::isfinite(t0))
    return fail(c, CFET_EINVAL, "window, T_total and eps must be positive, ratio > 1, all finite");
  const int J = checkpoints;
  if (J < 1 || n1 < 1 || n1 % J != 0)
    return fail(c, CFET_EINVAL, "n1 must be a positive multiple of checkpoints >= 1");
  if (refine < 0 || (refine > 0 && !verify))
    return fail(c, CFET_EINVAL, "refine must be >= 0 and needs verify");
  SchemeTable sc;
  if (!cfet::scheme_build(scheme, &sc)) return fail(c, CFET_EINVAL, "unknown scheme");
  if (!is_device_ptr(psi0_dev)) return fail(c, CFET_EINVAL, "psi0 must be device memory");
  DeviceGuard g(c->device);
  const int N = sc.order;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const size_t nn = size_t(c->n);
  const int nbp = cfet::dist2_blocks(c->n);
  GradBuffers gb;
  double2 *xa = nullptr, *xb = nullptr;
  double* part = nullptr;
  hipError_t e = gb.get(&xa, nn);
  if (e == hipSuccess) e = gb.get(&xb, nn);
  if (e == hipSuccess) e = gb.get(&part, size_t(nbp));
  if (e != hipSuccess) return hip_fail(c, e, "cfet_select_dt: workspace");
  std::vector<double> hpart(static_cast<size_t>(nbp), 0.0);
  // n2 = J round((n1 / J) ratio^(1/N)), at least n1 + J
  auto probe = [&](int64_t na) {
    const int64_t nb = int64_t(J) * int64_t(std::llround(double(na / J) *
                                                         std::pow(ratio, 1.0 / N)));
    return std::max<int64_t>(nb, na + J);
  };
  // largest distance over the J checkpoints of runs of [t0, t0 + W] with
  // na and nb steps, both started from psi0
  auto max_distance = [&](double W, int64_t na, int64_t nb, double* d_out) -> int {
    hipError_t ec = hipMemcpyAsync(xa, psi0_dev, nn * sizeof(double2), hipMemcpyDeviceToDevice, st);
    if (ec == hipSuccess)
      ec = hipMemcpyAsync(xb, psi0_dev, nn * sizeof(double2), hipMemcpyDeviceToDevice, st);
    if (ec != hipSuccess) return hip_fail(c, ec, "cfet_select_dt: copy psi0");
    const double dta = W / double(na), dtb = W / double(nb);
    const int64_t ka = na / J, kb = nb / J;
    double d = 0.0;
    for (int j = 0; j < J; ++j) {
      int rc = propagate_impl(c, xa, t0 + double(j * ka) * dta, dta, ka, scheme, krylov_m,
                              hip_stream, true);
      if (rc == CFET_OK)
        rc = propagate_impl(c, xb, t0 + double(j * kb) * dtb, dtb, kb, scheme, krylov_m,
                            hip_stream, true);
      if (rc != CFET_OK) return rc;
      ec = cfet::launch_dist2(xa, xb, c->n, part, st);
      if (ec == hipSuccess)
        ec = hipMemcpyAsync(hpart.data(), part, size_t(nbp) * sizeof(double),
                            hipMemcpyDeviceToHost, st);
      if (ec == hipSuccess) ec = hipStreamSynchronize(st);
      if (ec != hipSuccess) return hip_fail(c, ec, "cfet_select_dt: distance");
      if (c->stats_host->status != CFET_OK) {
        const int code = c->stats_host->status;
        c->stats_host->status = CFET_OK;
        return fail(c, code, "cfet_select_dt: device fault in a probe run (see cfet_stats)");
      }
      double s2 = 0.0;
      for (int i = 0; i < nbp; ++i) s2 += hpart[size_t(i)];
      d = std::max(d, std::sqrt(s2));
    }
    *d_out = d;
    return CFET_OK;
  };
  cfet_dt_choice r{};
  r.order = N;
  r.n1 = n1;
  const int64_t n2 = probe(n1);
  if (n2 > INT32_MAX) return fail(c, CFET_EINVAL, "probe step count overflows");
  r.n2 = int32_t(n2);
  r.dt1 = window / double(n1);
  r.dt2 = window / double(n2);
  int rc = max_distance(window, n1, n2, &r.diff);
  if (rc != CFET_OK) return rc;
  // dt for eps over T_total from the constant cc, capped at T_total and
  // rounded down to whole steps
  auto whole_steps = [&](double cc) -> int {
    double dt_raw = cc > 0.0 ? std::pow(eps / (cc * T_total), 1.0 / N) : T_total;
    dt_raw = std::min(dt_raw, T_total);
    const double ns = std::ceil(T_total / dt_raw * (1.0 - 1e-12));
    if (!(ns < 9.0e18)) return fail(c, CFET_EINVAL, "selected step count overflows");
    r.c = cc;
    r.nsteps = std::max<int64_t>(1, int64_t(ns));
    r.dt = T_total / double(r.nsteps);
    r.err_est = cc * T_total * std::pow(r.dt, N);
    return CFET_OK;
  };
  rc = whole_steps(r.diff / (window * std::fabs(std::pow(r.dt1, N) - std::pow(r.dt2, N))));
  if (rc != CFET_OK) return rc;
  r.err_check = std::nan("");
  for (int round = 0; verify; ++round) {
    // the window stretched to whole multiples of J steps of dt, run with dt
    // and with the smaller step of the same ratio
    const double blocks = std::ceil(window / (double(J) * r.dt) * (1.0 - 1e-12));
    if (!(blocks * J < 2.0e9)) return fail(c, CFET_EINVAL, "verification step count overflows");
    const int64_t na = int64_t(J) * std::max<int64_t>(1, int64_t(blocks));
    const int64_t nb = probe(na);
    if (nb > INT32_MAX) return fail(c, CFET_EINVAL, "verification step count overflows");
    const double Wc = double(na) * r.dt;
    double d = 0.0;
    rc = max_distance(Wc, na, nb, &d);
    if (rc != CFET_OK) return rc;
    const double db = Wc / double(nb);
    const double pa = std::pow(r.dt, N), pb = std::pow(db, N);
    r.check_window = Wc;
    r.check_n1 = int32_t(na);
    r.check_n2 = int32_t(nb);
    r.err_check = d * pa / (pa - pb) * T_total / Wc;
    r.rounds = round;
    if (r.err_check <= eps || round >= refine) break;
    rc = whole_steps(d / (Wc * std::fabs(pa - pb)));
    if (rc != CFET_OK) return rc;
  }
  *out = r;
  return CFET_OK;
}

int cfet_stats(cfet_ctx* c, cfet_stats_t* s) {
  if (!c || !s) return fail(c, CFET_EINVAL, "null argument");
  DeviceGuard g(c->device);
  hipError_t e = hipSuccess;
  if (c->have_work) e = hipStreamSynchronize(c->last_stream);
  if (e != hipSuccess) return hip_fail(c, e, "synchronise");
  DevStats d;
  e = hipMemcpy(&d, c->stats, sizeof(d), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(c, e, "read statistics");
  std::memset(s, 0, sizeof(*s));
  s->n = c->n;
  s->nnz_stored = c->A.nnz;
  s->exponentials = int64_t(d.exponentials);
  s->matvecs = int64_t(d.matvecs);
  s->min_m_eff = d.exponentials ? d.min_m_eff : 0;
  s->breakdowns = d.breakdowns;
  s->path = c->last_path;
  s->layout = !c->use_sell ? 0 : (c->hi.nuni ? 3 : (c->sell.nuni ? 2 : 1));
  s->reordered = c->perm ? 1 : 0;
  s->matrix_bytes = c->use_sell ? c->sell_bytes : 20 * c->A.nnz + 8 * (c->n + 1);
  s->status = d.status;
  s->last_norm = std::sqrt(d.last_norm2);
  harvest_events(c);
  s->timed_launches = c->timed_launches;
  s->timed_ms = c->timed_ms;
  {
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, c->device) != hipSuccess ||
        khz <= 0)
      khz = 100000;
    for (int i = 0; i < 4; ++i) s->segment_us[i] = double(d.seg[i]) * 1000.0 / double(khz);
  }
  if (d.status != CFET_OK) {
    const int32_t ok = CFET_OK;
    e = hipMemcpy(reinterpret_cast<char*>(c->stats) + offsetof(DevStats, status), &ok,
                  sizeof(ok), hipMemcpyHostToDevice);
    c->stats_host->status = CFET_OK;
    if (e != hipSuccess) return hip_fail(c, e, "clear status");
  }
  return CFET_OK;
}

int cfet_tridiag_expm(const double* alpha_dev, const double* beta_dev, int32_t k, double dt,
                      void* c_dev, int32_t* status_dev, void* hip_stream) {
  if (k < 1 || k > CFET_MAX_KRYLOV) return fail(nullptr, CFET_EINVAL, "k must be in 1..64");
  if (!alpha_dev || !c_dev || (k > 1 && !beta_dev))
    return fail(nullptr, CFET_EINVAL, "null argument");
  if (!std::isfinite(dt)) return fail(nullptr, CFET_EINVAL, "non-finite dt");
  const hipError_t e =
      cfet::launch_tridiag_expm(alpha_dev, beta_dev, k, dt, static_cast<double2*>(c_dev),
                                status_dev, static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return hip_fail(nullptr, e, "tridiagonal exponential launch");
  return CFET_OK;
}

}  // extern "C"
