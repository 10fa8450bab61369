// Host side of the batched path: operator table upload, grouping of the
// instances, launch autotuning, step-graph capture and the step loop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "batch_internal.h"
#include "cfet_internal.h"
#include "host_common.h"

using cfet::BGroup;
using cfet::BLaunch;
using cfet::BSlots;
using cfet::BState;
using cfet::DriveSpec;
using cfet::HostCSR;
using cfet::SchemeTable;

struct cfet_batch {
  int device = 0;
  int ninst = 0;
  int K1 = 1;
  uint32_t flags = 0;
  std::vector<int> inst_of;        // slot -> caller instance
  std::vector<int64_t> dims;       // per slot
  std::vector<int64_t> user_off;   // per slot: offset of the instance in the caller's buffer
  int64_t user_total = 0;
  std::vector<int> nterms;                     // per slot
  std::vector<std::vector<DriveSpec>> drives;  // per slot
  std::vector<BGroup> groups;
  BGroup* d_groups = nullptr;
  std::vector<void*> allocs;       // operator arrays
  int64_t ntot = 0;
  int total_blocks = 0;
  int64_t pstride = 0;             // partial sums per instance (most blocks of a group)
  int unroll = 1;                  // rows per lane and pass (autotuned)
  int waves = cfet::kBatchDefaultWaves;  // wavefronts per block of the row kernels (autotuned)
  std::vector<double> tune_us;     // timing of each candidate (autotune), [waves][unroll]
  // workspace
  int m_alloc = 0;
  double2* V = nullptr;
  double2* Y = nullptr;
  double* part = nullptr;
  BSlots S{};
  BState* st = nullptr;
  int64_t* d_uoff = nullptr;
  double* d_wts = nullptr;
  size_t wts_cap = 0;
  double* h_wts = nullptr;
  size_t h_wts_cap = 0;
  BState* h_state = nullptr;       // pinned staging of the device parameters
  int* h_mcap = nullptr;           // pinned staging of per-slot Krylov caps
  hipEvent_t staged = nullptr;     // staging buffers are free once this fired
  bool staged_pending = false;
  int mcap_m = 0;                  // m the device caps were written for
  // step graph
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t exec = nullptr;
  int graph_m = 0, graph_s = 0;
  bool graph_used = false;
  hipStream_t last_stream = nullptr;
  bool have_work = false;
  std::string err;
};

namespace {

thread_local std::string g_berr;

constexpr int kTuneCandidates[] = {2, 4, 8, 16};
constexpr double kTuneSlack = 0.03;  // relative window around the fastest candidate
constexpr size_t kWtsBudget = size_t(64) << 20;  // bytes of weights per upload chunk

int bfail(cfet_batch* b, int code, const std::string& msg) {
  if (b) b->err = msg;
  g_berr = msg;
  return code;
}

int bhip(cfet_batch* b, hipError_t e, const char* what) {
  return bfail(b, e == hipErrorOutOfMemory ? CFET_ENOMEM : CFET_EDEVICE,
               std::string(what) + ": " + hipGetErrorString(e));
}

template <class T>
hipError_t dalloc(T** p, size_t count) {
  return hipMalloc(reinterpret_cast<void**>(p), std::max<size_t>(count, 1) * sizeof(T));
}

void free_batch(cfet_batch* b) {
  if (!b) return;
  if (b->have_work) (void)hipDeviceSynchronize();
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  for (void* p : b->allocs) (void)hipFree(p);
  void* dev[] = {b->d_groups, b->V, b->Y, b->part, b->st, b->d_uoff, b->d_wts,
                 b->S.alpha, b->S.beta, b->S.inv, b->S.coef, b->S.beta0, b->S.m_eff,
                 b->S.done, b->S.mcap, b->S.matvecs, b->S.expos, b->S.breakdowns,
                 b->S.early, b->S.min_m, b->S.max_m};
  for (void* p : dev)
    if (p) (void)hipFree(p);
  if (b->h_wts) (void)hipHostFree(b->h_wts);
  if (b->h_state) (void)hipHostFree(b->h_state);
  if (b->h_mcap) (void)hipHostFree(b->h_mcap);
  if (b->staged) (void)hipEventDestroy(b->staged);
  (void)hipGetLastError();
  delete b;
}

static_assert(sizeof(cfet_batch_stats_t) == 168 && offsetof(cfet_batch_stats_t, tune_us) == 72,
              "cfet_batch_stats_t layout is part of the ABI");

// Block layout of the row kernels for a given unroll: fills rows_per_block,
// nblocks, block0 and returns the total number of blocks.
int layout_blocks(std::vector<BGroup>& G, int unroll, int waves) {
  int total = 0;
  for (auto& g : G) {
    g.rows_per_block = waves * (64 / g.lpr) * unroll;
    g.nblocks = int((g.n + g.rows_per_block - 1) / g.rows_per_block);
    g.block0 = total;
    total += g.nblocks;
  }
  return total;
}

BLaunch launch_of(const cfet_batch* b) {
  BLaunch L;
  L.groups = b->d_groups;
  L.ngroups = int(b->groups.size());
  L.total_blocks = b->total_blocks;
  L.nslots = b->ninst;
  L.ntot = b->ntot;
  L.V = b->V;
  L.Y = b->Y;
  L.part = b->part;
  L.pstride = b->pstride;
  L.waves = b->waves;
  L.S = b->S;
  L.st = b->st;
  return L;
}

hipError_t ensure_basis(cfet_batch* b, int m) {
  if (b->m_alloc >= m) return hipSuccess;
  if (b->have_work) (void)hipDeviceSynchronize();
  if (b->V) (void)hipFree(b->V);
  b->V = nullptr;
  b->m_alloc = 0;
  if (b->exec) {
    (void)hipGraphExecDestroy(b->exec);
    b->exec = nullptr;
  }
  hipError_t e = dalloc(&b->V, size_t(m) * size_t(b->ntot));
  if (e == hipSuccess) b->m_alloc = m;
  return e;
}

hipError_t enqueue_exponential(const BLaunch& L, int m, hipStream_t s) {
  hipError_t e = cfet::batch_scalars(L, cfet::kBStart, 0, s);
  for (int k = 0; k < m && e == hipSuccess; ++k) {
    e = cfet::batch_spmm(L, k, s);
    if (e == hipSuccess) e = cfet::batch_scalars(L, cfet::kBAlpha, k, s);
    if (k < m - 1) {
      if (e == hipSuccess) e = cfet::batch_axpy(L, k, s);
      if (e == hipSuccess) e = cfet::batch_scalars(L, cfet::kBBeta, k, s);
    }
  }
  if (e == hipSuccess) e = cfet::batch_combine(L, s);
  if (e == hipSuccess) e = cfet::batch_advance(L, s);
  return e;
}

hipError_t enqueue_step(const BLaunch& L, int m, int s_count, hipStream_t s) {
  hipError_t e = hipSuccess;
  for (int i = 0; i < s_count && e == hipSuccess; ++i) e = enqueue_exponential(L, m, s);
  return e;
}

// Time the first Lanczos iteration's product, its reduction and the
// three-term update per layout candidate (wavefronts per block x rows per
// lane) on the real operators.  Among the candidates within kTuneSlack of the
// fastest, keep the one whose blocks cover the most rows, and of those the one
// with the fewest wavefronts per block: the other kernels of a step (the
// second reduction, the recombination) pay per block and per partial, and a
// smaller block waits at its barrier for fewer wavefronts, none of which this
// timing shows.
int autotune(cfet_batch* b) {
  hipError_t e = hipSuccess;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  e = ensure_basis(b, 2);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  // one exponential of unit weights, every instance active with inv = 1
  std::vector<double> w(size_t(b->ninst) * b->K1, 1.0);
  std::vector<double> inv(size_t(b->ninst) * cfet::kMaxM, 1.0);
  BState hs{};
  hs.wts = b->d_wts;
  hs.nslots = b->ninst;
  hs.K1 = b->K1;
  hs.dt = 0.0;
  if (e == hipSuccess) e = hipMemcpy(b->d_wts, w.data(), w.size() * sizeof(double), hipMemcpyHostToDevice);
  hs.status = CFET_OK;
  if (e == hipSuccess) e = hipMemcpy(b->st, &hs, sizeof(BState), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(b->S.inv, inv.data(), inv.size() * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(b->S.done, 0, sizeof(int) * b->ninst);
  {
    std::vector<int> caps(size_t(b->ninst), cfet::kMaxM);  // no instance completes at k = 0
    if (e == hipSuccess)
      e = hipMemcpy(b->S.mcap, caps.data(), caps.size() * sizeof(int), hipMemcpyHostToDevice);
  }
  if (e == hipSuccess) e = hipMemset(b->V, 0, sizeof(double2) * b->ntot);
  b->tune_us.clear();
  for (int wv : cfet::kBatchWaveChoices)
  for (int u : kTuneCandidates) {
    if (e != hipSuccess) break;
    std::vector<BGroup> G = b->groups;
    const int tb = layout_blocks(G, u, wv);
    e = hipMemcpy(b->d_groups, G.data(), G.size() * sizeof(BGroup), hipMemcpyHostToDevice);
    if (e != hipSuccess) break;
    BLaunch L = launch_of(b);
    L.total_blocks = tb;
    L.waves = wv;
    e = cfet::batch_spmm(L, 0, nullptr);  // warm-up
    if (e == hipSuccess) e = cfet::batch_scalars(L, cfet::kBAlpha, 0, nullptr);
    if (e == hipSuccess) e = cfet::batch_axpy(L, 0, nullptr);
    if (e == hipSuccess) e = hipEventRecord(e0, nullptr);
    for (int r = 0; r < 3 && e == hipSuccess; ++r) {
      e = cfet::batch_spmm(L, 0, nullptr);
      if (e == hipSuccess) e = cfet::batch_scalars(L, cfet::kBAlpha, 0, nullptr);
      if (e == hipSuccess) e = cfet::batch_axpy(L, 0, nullptr);
    }
    if (e == hipSuccess) e = hipEventRecord(e1, nullptr);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    b->tune_us.push_back(1e3 * ms / 3.0);
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (e != hipSuccess) return bhip(b, e, "cfet_batch_create: autotune");
  double fastest = 1e300;
  for (double us : b->tune_us) fastest = std::min(fastest, us);
  int best_u = 1, best_w = cfet::kBatchDefaultWaves, best_rows = 0;
  size_t i = 0;
  for (int wv : cfet::kBatchWaveChoices)
    for (int u : kTuneCandidates) {
      const double us = b->tune_us[i++];
      if (us > fastest * (1.0 + kTuneSlack)) continue;
      const int rows = wv * u;  // rows per block, per lane of a row
      if (rows > best_rows || (rows == best_rows && wv < best_w)) {
        best_rows = rows;
        best_u = u;
        best_w = wv;
      }
    }
  b->unroll = best_u;
  b->waves = best_w;
  return CFET_OK;
}

int weights_for_chunk(cfet_batch* b, const SchemeTable& sc, double t0, double dt, int64_t n0,
                      int64_t nst) {
  const size_t per_expo = size_t(b->ninst) * b->K1;
  const size_t need = size_t(nst) * sc.s * per_expo;
  if (need > b->h_wts_cap) {
    if (b->staged_pending) (void)hipEventSynchronize(b->staged);
    b->staged_pending = false;
    if (b->h_wts) (void)hipHostFree(b->h_wts);
    b->h_wts = nullptr;
    b->h_wts_cap = 0;
    if (hipHostMalloc(reinterpret_cast<void**>(&b->h_wts), need * sizeof(double)) != hipSuccess)
      return bfail(b, CFET_ENOMEM, "cfet_batch_propagate: pinned weight staging");
    b->h_wts_cap = need;
  }
  std::vector<double> a(cfet::kMaxStages), bb(cfet::kMaxStages * cfet::kMaxTerms);
  for (int64_t q = 0; q < nst; ++q) {
    const double tn = t0 + double(n0 + q) * dt;
    for (int slot = 0; slot < b->ninst; ++slot) {
      const int K = b->nterms[slot];
      cfet::step_weights(sc, b->drives[slot], tn, dt, a.data(), bb.data());
      for (int ii = 0; ii < sc.s; ++ii) {
        const int i = sc.s - 1 - ii;  // exponential s is applied first
        double* w = b->h_wts + (size_t(q) * sc.s + ii) * per_expo + size_t(slot) * b->K1;
        w[0] = a[i];
        for (int k = 1; k < b->K1; ++k) w[k] = (k <= K) ? bb[size_t(i) * K + (k - 1)] : 0.0;
      }
    }
  }
  return CFET_OK;
}

}  // namespace

extern "C" {

CFET_API int cfet_batch_create(int32_t nops, const cfet_csr* ops, int32_t ninst,
                               const cfet_instance* inst, uint32_t flags, cfet_batch** out) {
  if (!out) return bfail(nullptr, CFET_EINVAL, "cfet_batch_create: null out");
  *out = nullptr;
  if (nops < 1 || !ops) return bfail(nullptr, CFET_EINVAL, "cfet_batch_create: no operators");
  if (ninst < 1 || !inst) return bfail(nullptr, CFET_EINVAL, "cfet_batch_create: no instances");
  cfet_batch* b = new (std::nothrow) cfet_batch();
  if (!b) return bfail(nullptr, CFET_ENOMEM, "cfet_batch_create: host allocation");
  b->flags = flags;
  hipError_t e = hipSuccess;
  int rc = CFET_OK;
  std::vector<HostCSR> mats(nops);
  for (int i = 0; i < nops && rc == CFET_OK; ++i) {
    rc = cfet::load_csr(b->err, &ops[i], "operator", &mats[i]);
    if (rc == CFET_OK && mats[i].n >= cfet::kMaxDim)
      rc = bfail(b, CFET_EUNSUPPORTED, "operator dimension must be below 2^29");
    if (rc == CFET_OK) rc = cfet::validate_csr(b->err, mats[i], "operator");
    if (rc == CFET_OK && (flags & CFET_VALIDATE_HERMITIAN))
      rc = cfet::check_hermitian(b->err, mats[i], "operator");
  }
  // instances
  std::vector<int> h0_refs(nops, 0);
  for (int t = 0; t < ninst && rc == CFET_OK; ++t) {
    const cfet_instance& I = inst[t];
    if (I.h0 < 0 || I.h0 >= nops) {
      rc = bfail(b, CFET_EINVAL, "instance: h0 out of range");
      break;
    }
    if (I.nterms < 0 || I.nterms > CFET_MAX_TERMS) {
      rc = bfail(b, CFET_EINVAL, "instance: nterms out of range");
      break;
    }
    for (int k = 0; k < I.nterms && rc == CFET_OK; ++k) {
      if (I.hk[k] < 0 || I.hk[k] >= nops)
        rc = bfail(b, CFET_EINVAL, "instance: hk out of range");
      else if (mats[I.hk[k]].n != mats[I.h0].n)
        rc = bfail(b, CFET_EINVAL, "instance: operators of one instance must have the same n");
    }
    h0_refs[I.h0] += 1;
  }
  if (rc != CFET_OK) {
    g_berr = b->err;
    free_batch(b);
    return rc;
  }
  // group key: dimension, driven operators, and H0 when it is shared
  typedef std::tuple<int64_t, std::vector<int>, int> Key;
  std::vector<std::pair<Key, int>> order;
  for (int t = 0; t < ninst; ++t) {
    const cfet_instance& I = inst[t];
    std::vector<int> hk(I.hk, I.hk + I.nterms);
    const int sh = (h0_refs[I.h0] >= 2) ? I.h0 : -1;
    order.push_back({Key(mats[I.h0].n, hk, sh), t});
  }
  std::stable_sort(order.begin(), order.end(),
                   [](const std::pair<Key, int>& x, const std::pair<Key, int>& y) {
                     return x.first < y.first;
                   });
  b->ninst = ninst;
  b->inst_of.resize(ninst);
  b->dims.resize(ninst);
  b->nterms.resize(ninst);
  b->drives.resize(ninst);
  int maxK = 0;
  for (int slot = 0; slot < ninst && rc == CFET_OK; ++slot) {
    const int t = order[slot].second;
    b->inst_of[slot] = t;
    b->dims[slot] = mats[inst[t].h0].n;
    b->nterms[slot] = inst[t].nterms;
    maxK = std::max(maxK, int(inst[t].nterms));
    b->drives[slot].resize(inst[t].nterms);
    for (int k = 0; k < inst[t].nterms && rc == CFET_OK; ++k)
      rc = cfet::copy_drive(b->err, inst[t].fk[k], &b->drives[slot][k]);
  }
  if (rc != CFET_OK) {
    g_berr = b->err;
    free_batch(b);
    return rc;
  }
  b->K1 = maxK + 1;
  e = hipGetDevice(&b->device);
  if (e != hipSuccess) {
    rc = bhip(b, e, "hipGetDevice");
    free_batch(b);
    return rc;
  }
  // caller layout: instances concatenated in their own order
  {
    std::vector<int64_t> off(ninst + 1, 0);
    for (int t = 0; t < ninst; ++t) off[t + 1] = off[t] + mats[inst[t].h0].n;
    b->user_total = off[ninst];
    b->user_off.resize(ninst);
    for (int slot = 0; slot < ninst; ++slot) b->user_off[slot] = off[b->inst_of[slot]];
  }
  // shared operators, one per key
  std::map<Key, std::tuple<int64_t*, uint32_t*, double2*>> shared;
  int slot = 0;
  int64_t voff = 0;
  while (slot < ninst && rc == CFET_OK) {
    const Key key = order[slot].first;
    // groups of a power-of-two size (at most 64): every lane of a wavefront
    // serves an instance, and a row's B complex values fill whole cache lines
    int same = slot;
    while (same < ninst && order[same].first == key) ++same;
    int take = 1;
    while (take * 2 <= std::min(same - slot, cfet::kBatchMaxGroup)) take *= 2;
    const int end = slot + take;
    const int t0 = order[slot].second;
    const int64_t n = mats[inst[t0].h0].n;
    const int sh = std::get<2>(key);
    const std::vector<int>& hk = std::get<1>(key);
    if (!shared.count(key)) {
      // merged rows: H0 (term 0, if shared), then H_1 .. H_K
      std::vector<const HostCSR*> terms;
      std::vector<int> tid;
      if (sh >= 0) {
        terms.push_back(&mats[sh]);
        tid.push_back(0);
      }
      for (size_t k = 0; k < hk.size(); ++k) {
        terms.push_back(&mats[hk[k]]);
        tid.push_back(int(k) + 1);
      }
      std::vector<int64_t> rp(n + 1, 0);
      for (int64_t r = 0; r < n; ++r) {
        int64_t len = 0;
        for (auto* h : terms) len += h->rp[r + 1] - h->rp[r];
        rp[r + 1] = rp[r] + len;
      }
      const int64_t nnz = rp[n];
      std::vector<uint32_t> colt(std::max<int64_t>(nnz, 1));
      std::vector<double> val(2 * std::max<int64_t>(nnz, 1));
      for (int64_t r = 0; r < n; ++r) {
        int64_t pos = rp[r];
        for (size_t q = 0; q < terms.size(); ++q) {
          const HostCSR& h = *terms[q];
          for (int64_t x = h.rp[r]; x < h.rp[r + 1]; ++x, ++pos) {
            colt[pos] = uint32_t(h.col[x]) | (uint32_t(tid[q]) << cfet::kTermShift);
            val[2 * pos] = h.val[2 * x];
            val[2 * pos + 1] = h.val[2 * x + 1];
          }
        }
      }
      int64_t* drp = nullptr;
      uint32_t* dcol = nullptr;
      double2* dval = nullptr;
      e = dalloc(&drp, n + 1);
      if (e == hipSuccess) b->allocs.push_back(drp);
      if (e == hipSuccess) e = dalloc(&dcol, colt.size());
      if (e == hipSuccess) b->allocs.push_back(dcol);
      if (e == hipSuccess) e = dalloc(&dval, colt.size());
      if (e == hipSuccess) b->allocs.push_back(dval);
      if (e == hipSuccess) e = hipMemcpy(drp, rp.data(), (n + 1) * sizeof(int64_t), hipMemcpyHostToDevice);
      if (e == hipSuccess) e = hipMemcpy(dcol, colt.data(), colt.size() * sizeof(uint32_t), hipMemcpyHostToDevice);
      if (e == hipSuccess) e = hipMemcpy(dval, val.data(), val.size() * sizeof(double), hipMemcpyHostToDevice);
      if (e != hipSuccess) {
        rc = bhip(b, e, "cfet_batch_create: operator upload");
        break;
      }
      shared[key] = std::make_tuple(drp, dcol, dval);
    }
    BGroup g{};
    g.n = n;
    g.voff = voff;
    g.B = end - slot;
    g.lpr = 1;
    while (g.lpr < g.B) g.lpr <<= 1;
    g.slot0 = slot;
    g.shared_h0 = sh >= 0 ? 1 : 0;
    g.rowptr = std::get<0>(shared[key]);
    g.colt = std::get<1>(shared[key]);
    g.val = std::get<2>(shared[key]);
    if (sh < 0) {
      // per-instance H0: dense diagonal [n][B] and off-diagonal rows [B][n + 1]
      const int B = g.B;
      std::vector<double> diag(size_t(2) * n * B, 0.0);
      std::vector<int64_t> orp(size_t(B) * (n + 1), 0);
      std::vector<int32_t> ocol;
      std::vector<double> oval;
      bool any_off = false;
      for (int j = 0; j < B; ++j) {
        const HostCSR& h = mats[inst[order[slot + j].second].h0];
        int64_t* rpj = orp.data() + size_t(j) * (n + 1);
        for (int64_t r = 0; r < n; ++r) {
          rpj[r] = int64_t(ocol.size());
          for (int64_t x = h.rp[r]; x < h.rp[r + 1]; ++x) {
            if (h.col[x] == r) {
              diag[2 * (size_t(r) * B + j)] = h.val[2 * x];
              diag[2 * (size_t(r) * B + j) + 1] = h.val[2 * x + 1];
            } else {
              ocol.push_back(h.col[x]);
              oval.push_back(h.val[2 * x]);
              oval.push_back(h.val[2 * x + 1]);
              any_off = true;
            }
          }
        }
        rpj[n] = int64_t(ocol.size());
      }
      double2* dd = nullptr;
      e = dalloc(&dd, size_t(n) * B);
      if (e == hipSuccess) b->allocs.push_back(dd);
      if (e == hipSuccess)
        e = hipMemcpy(dd, diag.data(), diag.size() * sizeof(double), hipMemcpyHostToDevice);
      g.diag = dd;
      if (e == hipSuccess && any_off) {
        int64_t* drp = nullptr;
        int32_t* dcol = nullptr;
        double2* dval = nullptr;
        e = dalloc(&drp, orp.size());
        if (e == hipSuccess) b->allocs.push_back(drp);
        if (e == hipSuccess) e = dalloc(&dcol, ocol.size());
        if (e == hipSuccess) b->allocs.push_back(dcol);
        if (e == hipSuccess) e = dalloc(&dval, ocol.size());
        if (e == hipSuccess) b->allocs.push_back(dval);
        if (e == hipSuccess) e = hipMemcpy(drp, orp.data(), orp.size() * sizeof(int64_t), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(dcol, ocol.data(), ocol.size() * sizeof(int32_t), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(dval, oval.data(), oval.size() * sizeof(double), hipMemcpyHostToDevice);
        g.orp = drp;
        g.ocol = dcol;
        g.oval = dval;
      }
      if (e != hipSuccess) {
        rc = bhip(b, e, "cfet_batch_create: H0 upload");
        break;
      }
    }
    b->groups.push_back(g);
    voff += n * g.B;
    slot = end;
  }
  if (rc != CFET_OK) {
    g_berr = b->err;
    free_batch(b);
    return rc;
  }
  b->ntot = voff;
  // partial-sum rows sized for the layout with the most blocks (the smallest
  // block and rows per lane among the candidates)
  layout_blocks(b->groups, kTuneCandidates[0], cfet::kBatchWaveChoices[0]);
  for (const auto& g : b->groups) b->pstride = std::max<int64_t>(b->pstride, g.nblocks);
  // per-slot state and workspace
  const size_t ns = size_t(ninst), nm = ns * cfet::kMaxM;
  e = dalloc(&b->d_groups, b->groups.size());
  if (e == hipSuccess) e = dalloc(&b->Y, size_t(b->ntot));
  if (e == hipSuccess) e = dalloc(&b->part, size_t(ninst) * size_t(b->pstride));
  if (e == hipSuccess) e = dalloc(&b->st, 1);
  if (e == hipSuccess) e = dalloc(&b->d_uoff, ns);
  if (e == hipSuccess) e = dalloc(&b->S.alpha, nm);
  if (e == hipSuccess) e = dalloc(&b->S.beta, nm);
  if (e == hipSuccess) e = dalloc(&b->S.inv, nm);
  if (e == hipSuccess) e = dalloc(&b->S.coef, nm);
  if (e == hipSuccess) e = dalloc(&b->S.beta0, ns);
  if (e == hipSuccess) e = dalloc(&b->S.m_eff, ns);
  if (e == hipSuccess) e = dalloc(&b->S.done, ns);
  if (e == hipSuccess) e = dalloc(&b->S.mcap, ns);
  if (e == hipSuccess) e = dalloc(&b->S.matvecs, ns);
  if (e == hipSuccess) e = dalloc(&b->S.expos, ns);
  if (e == hipSuccess) e = dalloc(&b->S.breakdowns, ns);
  if (e == hipSuccess) e = dalloc(&b->S.early, ns);
  if (e == hipSuccess) e = dalloc(&b->S.min_m, ns);
  if (e == hipSuccess) e = dalloc(&b->S.max_m, ns);
  if (e == hipSuccess) {
    b->wts_cap = std::max<size_t>(ns * b->K1, 1);
    e = dalloc(&b->d_wts, b->wts_cap);
  }
  if (e == hipSuccess) e = ensure_basis(b, 1);
  if (e == hipSuccess)
    e = hipMemcpy(b->d_uoff, b->user_off.data(), ns * sizeof(int64_t), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&b->h_state), sizeof(BState));
  if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&b->h_mcap), ns * sizeof(int));
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->staged, hipEventDisableTiming);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking);
  if (e == hipSuccess) {
    // the device parameters, with the latched status cleared: the per-call
    // upload never rewrites the status, so it must start at CFET_OK whether
    // or not the layouts are timed below
    BState hs{};
    hs.wts = b->d_wts;
    hs.nslots = b->ninst;
    hs.K1 = b->K1;
    hs.status = CFET_OK;
    e = hipMemcpy(b->st, &hs, sizeof(BState), hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) {
    rc = bhip(b, e, "cfet_batch_create: device setup");
    g_berr = b->err;
    free_batch(b);
    return rc;
  }
  if (flags & CFET_BATCH_NO_AUTOTUNE) {
    b->unroll = 8;
    b->waves = cfet::kBatchDefaultWaves;
  } else {
    rc = autotune(b);
    if (rc != CFET_OK) {
      g_berr = b->err;
      free_batch(b);
      return rc;
    }
  }
  b->total_blocks = layout_blocks(b->groups, b->unroll, b->waves);
  e = hipMemcpy(b->d_groups, b->groups.data(), b->groups.size() * sizeof(BGroup),
                hipMemcpyHostToDevice);
  if (e == hipSuccess) e = cfet::batch_stats_reset(launch_of(b), nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    rc = bhip(b, e, "cfet_batch_create: device setup");
    g_berr = b->err;
    free_batch(b);
    return rc;
  }
  *out = b;
  return CFET_OK;
}

CFET_API int cfet_batch_propagate(cfet_batch* b, void* psi_dev, double t0, double dt,
                                  int64_t nsteps, int32_t scheme, int32_t krylov_m, double tol,
                                  void* hip_stream) {
  if (!b) return bfail(nullptr, CFET_EINVAL, "cfet_batch_propagate: null batch");
  if (!psi_dev) return bfail(b, CFET_EINVAL, "cfet_batch_propagate: null psi");
  if (nsteps < 0) return bfail(b, CFET_EINVAL, "cfet_batch_propagate: nsteps < 0");
  if (krylov_m < 1 || krylov_m > CFET_MAX_KRYLOV)
    return bfail(b, CFET_EINVAL, "cfet_batch_propagate: krylov_m out of range");
  if (!std::isfinite(t0) || !std::isfinite(dt) || !std::isfinite(tol) || tol < 0.0)
    return bfail(b, CFET_EINVAL, "cfet_batch_propagate: t0, dt and tol must be finite, tol >= 0");
  SchemeTable sc;
  if (!cfet::scheme_build(scheme, &sc))
    return bfail(b, CFET_EINVAL, "cfet_batch_propagate: unknown scheme");
  if (!cfet::is_device_ptr(psi_dev))
    return bfail(b, CFET_EINVAL, "cfet_batch_propagate: psi must be device memory");
  if (nsteps == 0) return CFET_OK;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  b->last_stream = s;
  hipError_t e = ensure_basis(b, krylov_m);
  if (e != hipSuccess) return bhip(b, e, "cfet_batch_propagate: basis allocation");
  // weights in chunks of whole steps
  const size_t per_step = size_t(sc.s) * b->ninst * b->K1;
  const int64_t chunk = std::max<int64_t>(
      1, std::min<int64_t>(nsteps, int64_t(kWtsBudget / (per_step * sizeof(double)))));
  if (size_t(chunk) * per_step > b->wts_cap) {
    if (b->have_work) (void)hipDeviceSynchronize();
    (void)hipFree(b->d_wts);
    b->d_wts = nullptr;
    b->wts_cap = 0;
    e = dalloc(&b->d_wts, size_t(chunk) * per_step);
    if (e != hipSuccess) return bhip(b, e, "cfet_batch_propagate: weight table");
    b->wts_cap = size_t(chunk) * per_step;
  }
  // device parameters and per-slot caps (pinned staging, stream-ordered copies)
  if (b->staged_pending) (void)hipEventSynchronize(b->staged);
  b->staged_pending = false;
  BState hs{};
  hs.wts = b->d_wts;
  hs.cursor = 0;
  hs.dt = dt;
  hs.tol = tol;
  hs.nslots = b->ninst;
  hs.K1 = b->K1;
  *b->h_state = hs;
  for (int slot = 0; slot < b->ninst; ++slot)
    b->h_mcap[slot] = int(std::min<int64_t>(krylov_m, b->dims[slot]));
  e = hipMemcpyAsync(b->st, b->h_state, offsetof(BState, status), hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->S.mcap, b->h_mcap, sizeof(int) * b->ninst, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipEventRecord(b->staged, s);
  if (e != hipSuccess) return bhip(b, e, "cfet_batch_propagate: parameter upload");
  b->staged_pending = true;
  BLaunch L = launch_of(b);
  e = cfet::batch_pack(L, static_cast<const double2*>(psi_dev), b->d_uoff, s);
  if (e == hipSuccess) e = cfet::batch_norm(L, s);
  if (e != hipSuccess) return bhip(b, e, "cfet_batch_propagate: launch");
  // the step graph: one CFET step (all exponentials, all Lanczos phases)
  const bool want_graph = !(b->flags & CFET_BATCH_NO_GRAPH);
  if (want_graph && (!b->exec || b->graph_m != krylov_m || b->graph_s != sc.s)) {
    if (b->exec) {
      (void)hipGraphExecDestroy(b->exec);
      b->exec = nullptr;
    }
    hipGraph_t graph = nullptr;
    e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeRelaxed);
    if (e == hipSuccess) {
      const hipError_t e2 = enqueue_step(L, krylov_m, sc.s, b->cap_stream);
      e = hipStreamEndCapture(b->cap_stream, &graph);
      if (e2 != hipSuccess) e = e2;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
      b->exec = nullptr;
      return bhip(b, e, "cfet_batch_propagate: step graph");
    }
    b->graph_m = krylov_m;
    b->graph_s = sc.s;
  }
  b->graph_used = want_graph;
  for (int64_t n0 = 0; n0 < nsteps; n0 += chunk) {
    const int64_t nst = std::min<int64_t>(chunk, nsteps - n0);
    if (b->staged_pending) (void)hipEventSynchronize(b->staged);
    b->staged_pending = false;
    int rc = weights_for_chunk(b, sc, t0, dt, n0, nst);
    if (rc != CFET_OK) return rc;
    e = hipMemcpyAsync(b->d_wts, b->h_wts, size_t(nst) * per_step * sizeof(double),
                       hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipEventRecord(b->staged, s);
    if (e == hipSuccess) e = cfet::batch_set_cursor(L, 0, s);
    if (e != hipSuccess) return bhip(b, e, "cfet_batch_propagate: weight upload");
    b->staged_pending = true;
    for (int64_t q = 0; q < nst && e == hipSuccess; ++q)
      e = want_graph ? hipGraphLaunch(b->exec, s) : enqueue_step(L, krylov_m, sc.s, s);
    if (e != hipSuccess) return bhip(b, e, "cfet_batch_propagate: step launch");
  }
  e = cfet::batch_unpack(L, static_cast<double2*>(psi_dev), b->d_uoff, s);
  if (e != hipSuccess) return bhip(b, e, "cfet_batch_propagate: launch");
  b->have_work = true;
  return CFET_OK;
}

CFET_API int cfet_batch_set_layout(cfet_batch* b, int32_t block_threads, int32_t rows_per_lane) {
  if (!b) return bfail(nullptr, CFET_EINVAL, "cfet_batch_set_layout: null batch");
  int waves = 0;
  for (int wv : cfet::kBatchWaveChoices)
    if (64 * wv == block_threads) waves = wv;
  bool rows_ok = false;
  for (int u : kTuneCandidates) rows_ok = rows_ok || u == rows_per_lane;
  if (waves == 0 || !rows_ok)
    return bfail(b, CFET_EINVAL,
                 "cfet_batch_set_layout: block_threads must be 128, 256 or 512 and "
                 "rows_per_lane 2, 4, 8 or 16");
  hipError_t e = b->have_work ? hipStreamSynchronize(b->last_stream) : hipSuccess;
  if (e != hipSuccess) return bhip(b, e, "cfet_batch_set_layout: synchronise");
  b->waves = waves;
  b->unroll = rows_per_lane;
  // the partial rows (pstride) were sized at create for the layout with the most blocks
  b->total_blocks = layout_blocks(b->groups, b->unroll, b->waves);
  e = hipMemcpy(b->d_groups, b->groups.data(), b->groups.size() * sizeof(BGroup),
                hipMemcpyHostToDevice);
  if (e != hipSuccess) return bhip(b, e, "cfet_batch_set_layout: upload");
  if (b->exec) {  // recorded with the old grid: re-record on the next call
    (void)hipGraphExecDestroy(b->exec);
    b->exec = nullptr;
  }
  return CFET_OK;
}

CFET_API int cfet_batch_stats(cfet_batch* b, cfet_batch_stats_t* out) {
  if (!b || !out) return bfail(b, CFET_EINVAL, "cfet_batch_stats: null argument");
  hipError_t e = b->have_work ? hipStreamSynchronize(b->last_stream) : hipSuccess;
  if (e != hipSuccess) return bhip(b, e, "cfet_batch_stats: synchronize");
  const size_t ns = size_t(b->ninst);
  std::vector<long long> mv(ns), ex(ns), br(ns), ea(ns);
  std::vector<int> mn(ns), mx(ns);
  BState hs{};
  e = hipMemcpy(mv.data(), b->S.matvecs, ns * sizeof(long long), hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(ex.data(), b->S.expos, ns * sizeof(long long), hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(br.data(), b->S.breakdowns, ns * sizeof(long long), hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(ea.data(), b->S.early, ns * sizeof(long long), hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(mn.data(), b->S.min_m, ns * sizeof(int), hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(mx.data(), b->S.max_m, ns * sizeof(int), hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(&hs, b->st, sizeof(BState), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return bhip(b, e, "cfet_batch_stats: copy");
  std::memset(out, 0, sizeof(*out));
  out->ninst = b->ninst;
  out->ngroups = int32_t(b->groups.size());
  out->total_dim = b->user_total;
  out->min_m_eff = 1 << 30;
  out->max_m_eff = 0;
  for (size_t i = 0; i < ns; ++i) {
    out->matvecs += mv[i];
    out->exponentials += ex[i];
    out->breakdowns += br[i];
    out->early_stops += ea[i];
    if (ex[i] > 0) {
      out->min_m_eff = std::min(out->min_m_eff, mn[i]);
      out->max_m_eff = std::max(out->max_m_eff, mx[i]);
    }
  }
  if (out->exponentials == 0) out->min_m_eff = 0;
  out->status = hs.status;
  if (hs.status != CFET_OK) {  // reported: clear the latch
    const int ok = CFET_OK;
    (void)hipMemcpy(&b->st->status, &ok, sizeof(int), hipMemcpyHostToDevice);
  }
  out->unroll = b->unroll;
  out->graph = b->graph_used ? 1 : 0;
  out->block_threads = 64 * b->waves;
  for (size_t i = 0; i < b->tune_us.size() && i < 12; ++i) out->tune_us[i] = b->tune_us[i];
  return hs.status;
}

CFET_API int cfet_batch_instance_matvecs(cfet_batch* b, int64_t* out) {
  if (!b || !out) return bfail(b, CFET_EINVAL, "cfet_batch_instance_matvecs: null argument");
  hipError_t e = b->have_work ? hipStreamSynchronize(b->last_stream) : hipSuccess;
  std::vector<long long> mv(b->ninst);
  if (e == hipSuccess)
    e = hipMemcpy(mv.data(), b->S.matvecs, mv.size() * sizeof(long long), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return bhip(b, e, "cfet_batch_instance_matvecs");
  for (int slot = 0; slot < b->ninst; ++slot) out[b->inst_of[slot]] = mv[slot];
  return CFET_OK;
}

CFET_API int cfet_batch_destroy(cfet_batch* b) {
  if (!b) return CFET_OK;
  free_batch(b);
  return CFET_OK;
}

CFET_API const char* cfet_batch_last_error(const cfet_batch* b) {
  return b ? b->err.c_str() : g_berr.c_str();
}

}  // extern "C"
