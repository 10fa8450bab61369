// Host-side input handling shared by the entry points (see host_common.h).
#include "host_common.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <thread>

namespace cfet {

namespace {

int fail(std::string& err, int code, const std::string& msg) {
  err = msg;
  return code;
}

}  // namespace

bool is_device_ptr(const void* p) {
  if (!p) return false;
  hipPointerAttribute_t attr;
  const hipError_t e = hipPointerGetAttributes(&attr, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
}

namespace {

template <class T>
bool fetch_to_host(const T* p, size_t count, std::vector<T>& out, const T** view) {
  if (count == 0) {
    *view = p;
    return true;
  }
  if (is_device_ptr(p)) {
    try {
      out.resize(count);
    } catch (const std::bad_alloc&) {
      return false;
    }
    if (hipMemcpy(out.data(), p, count * sizeof(T), hipMemcpyDeviceToHost) != hipSuccess)
      return false;
    *view = out.data();
  } else {
    *view = p;
  }
  return true;
}

}  // namespace

int load_csr(std::string& err, const cfet_csr* m, const char* name, HostCSR* h) {
  if (!m) return fail(err, CFET_EINVAL, std::string(name) + ": null matrix");
  if (m->n <= 0 || m->nnz < 0) return fail(err, CFET_EINVAL, std::string(name) + ": bad n/nnz");
  if (!m->row_ptr) return fail(err, CFET_EINVAL, std::string(name) + ": null row_ptr");
  if (m->nnz > 0 && (!m->col || !m->val))
    return fail(err, CFET_EINVAL, std::string(name) + ": null col/val");
  h->n = m->n;
  h->nnz = m->nnz;
  if (!fetch_to_host(m->row_ptr, size_t(m->n + 1), h->rp_buf, &h->rp) ||
      !fetch_to_host(m->col, size_t(m->nnz), h->col_buf, &h->col) ||
      !fetch_to_host(m->val, size_t(2 * m->nnz), h->val_buf, &h->val))
    return fail(err, CFET_ENOMEM, std::string(name) + ": cannot stage matrix on the host");
  return CFET_OK;
}

// Structure and value checks, split over threads by rows.
int validate_csr(std::string& err, const HostCSR& h, const char* name) {
  if (h.rp[0] != 0 || h.rp[h.n] != h.nnz)
    return fail(err, CFET_EINVAL, std::string(name) + ": row_ptr[0] != 0 or row_ptr[n] != nnz");
  const int64_t n = h.n;
  unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  if (n < 65536) nth = 1;
  std::vector<int> bad(nth, 0);
  std::vector<std::thread> pool;
  for (unsigned t = 0; t < nth; ++t) {
    pool.emplace_back([&, t]() {
      const int64_t r0 = n * t / nth, r1 = n * (t + 1) / nth;
      std::vector<int64_t> seen;  // duplicate detection by marking columns with the row id
      for (int64_t r = r0; r < r1 && !bad[t]; ++r) {
        const int64_t b = h.rp[r], e = h.rp[r + 1];
        if (e < b || e > h.nnz) {
          bad[t] = 1;
          break;
        }
        for (int64_t k = b; k < e; ++k) {
          const int32_t col = h.col[k];
          if (col < 0 || col >= n) {
            bad[t] = 2;
            break;
          }
          if (!std::isfinite(h.val[2 * k]) || !std::isfinite(h.val[2 * k + 1])) {
            bad[t] = 3;
            break;
          }
          for (int64_t k2 = b; k2 < k && (e - b) <= 64; ++k2)
            if (h.col[k2] == col) {
              bad[t] = 4;
              break;
            }
        }
        if (!bad[t] && (e - b) > 64) {  // long rows: sort a copy
          seen.assign(h.col + b, h.col + e);
          std::sort(seen.begin(), seen.end());
          if (std::adjacent_find(seen.begin(), seen.end()) != seen.end()) bad[t] = 4;
        }
      }
    });
  }
  for (auto& th : pool) th.join();
  for (unsigned t = 0; t < nth; ++t) {
    switch (bad[t]) {
      case 1: return fail(err, CFET_EINVAL, std::string(name) + ": row_ptr not non-decreasing");
      case 2: return fail(err, CFET_EINVAL, std::string(name) + ": column index out of range");
      case 3: return fail(err, CFET_ENONFINITE, std::string(name) + ": non-finite value");
      case 4: return fail(err, CFET_EINVAL, std::string(name) + ": repeated column in a row");
      default: break;
    }
  }
  return CFET_OK;
}

int check_hermitian(std::string& err, const HostCSR& h, const char* name) {
  for (int64_t r = 0; r < h.n; ++r) {
    for (int64_t k = h.rp[r]; k < h.rp[r + 1]; ++k) {
      const int64_t col = h.col[k];
      bool found = false;
      for (int64_t k2 = h.rp[col]; k2 < h.rp[col + 1]; ++k2) {
        if (h.col[k2] == r) {
          const double dr = h.val[2 * k] - h.val[2 * k2];
          const double di = h.val[2 * k + 1] + h.val[2 * k2 + 1];
          const double sc = std::fabs(h.val[2 * k]) + std::fabs(h.val[2 * k + 1]) + 1e-300;
          if (std::fabs(dr) > 1e-12 * sc || std::fabs(di) > 1e-12 * sc)
            return fail(err, CFET_EINVAL, std::string(name) + ": not Hermitian");
          found = true;
          break;
        }
      }
      const bool zero = h.val[2 * k] == 0.0 && h.val[2 * k + 1] == 0.0;
      if (!found && !zero) return fail(err, CFET_EINVAL, std::string(name) + ": not Hermitian");
    }
  }
  return CFET_OK;
}

int copy_drive(std::string& err, const cfet_drive& d, DriveSpec* out) {
  out->kind = d.kind;
  out->A = d.A;
  out->omega = d.omega;
  out->phi = d.phi;
  out->Tp = d.Tp;
  out->tc = d.tc;
  out->tau = d.tau;
  switch (d.kind) {
    case CFET_DRIVE_COS:
      if (!std::isfinite(d.A) || !std::isfinite(d.omega) || !std::isfinite(d.phi))
        return fail(err, CFET_EINVAL, "drive: non-finite parameter");
      break;
    case CFET_DRIVE_SIN2_COS:
      if (!(d.Tp > 0.0) || !std::isfinite(d.Tp) || !std::isfinite(d.A) ||
          !std::isfinite(d.omega) || !std::isfinite(d.phi))
        return fail(err, CFET_EINVAL, "drive: SIN2_COS needs finite parameters and Tp > 0");
      break;
    case CFET_DRIVE_PWC: {
      if (d.npieces < 1 || !d.t_edges || !d.u)
        return fail(err, CFET_EINVAL, "drive: PWC needs npieces >= 1 and edges/u arrays");
      out->edges.assign(d.t_edges, d.t_edges + d.npieces + 1);
      out->u.assign(d.u, d.u + d.npieces);
      for (int j = 0; j < d.npieces; ++j)
        if (!(out->edges[j] < out->edges[j + 1]) || !std::isfinite(out->u[j]))
          return fail(err, CFET_EINVAL, "drive: PWC edges must increase and u be finite");
      if (!std::isfinite(out->edges[0]) || !std::isfinite(out->edges[d.npieces]))
        return fail(err, CFET_EINVAL, "drive: PWC edges must be finite");
      break;
    }
    case CFET_DRIVE_SECH_COS:
      if (!(d.tau != 0.0) || !std::isfinite(d.tau) || !std::isfinite(d.A) ||
          !std::isfinite(d.omega) || !std::isfinite(d.phi) || !std::isfinite(d.tc))
        return fail(err, CFET_EINVAL, "drive: SECH_COS needs finite parameters and tau != 0");
      break;
    default:
      return fail(err, CFET_EINVAL, "drive: unknown kind");
  }
  return CFET_OK;
}

std::vector<int32_t> rcm_order(const std::vector<HostCSR>& mats, int64_t n) {
  std::vector<int32_t> deg(n, 0);
  for (int64_t r = 0; r < n; ++r) {
    int64_t d = 0;
    for (const HostCSR& h : mats) d += h.rp[r + 1] - h.rp[r];
    deg[r] = int32_t(std::min<int64_t>(d, INT32_MAX));
  }
  auto for_nb = [&](int32_t u, auto f) {
    for (const HostCSR& h : mats)
      for (int64_t q = h.rp[u]; q < h.rp[u + 1]; ++q) f(h.col[q]);
  };
  std::vector<char> done(n, 0);           // placed in the order
  std::vector<int32_t> lvl(n, -1), q;     // level scratch of one search
  // breadth-first search over rows not yet placed; returns the last level's
  // row of smallest degree and sets ecc to its level
  auto bfs = [&](int32_t s, int& ecc) -> int32_t {
    q.clear();
    q.push_back(s);
    lvl[s] = 0;
    for (size_t h = 0; h < q.size(); ++h) {
      const int32_t u = q[h];
      for_nb(u, [&](int32_t v) {
        if (!done[v] && lvl[v] < 0) {
          lvl[v] = lvl[u] + 1;
          q.push_back(v);
        }
      });
    }
    ecc = lvl[q.back()];
    int32_t best = q.back();
    for (size_t h = q.size(); h-- > 0 && lvl[q[h]] == ecc;)
      if (deg[q[h]] < deg[best]) best = q[h];
    for (int32_t u : q) lvl[u] = -1;
    return best;
  };
  std::vector<int32_t> order;
  order.reserve(n);
  std::vector<int32_t> nbrs;
  for (int64_t s0 = 0; s0 < n; ++s0) {
    if (done[s0]) continue;
    // pseudo-peripheral root: repeat the search from the far end while the
    // eccentricity grows (at most a few rounds)
    int32_t root = int32_t(s0);
    int ecc = 0;
    int32_t far = bfs(root, ecc);
    for (int it = 0; it < 4; ++it) {
      int e2 = 0;
      const int32_t far2 = bfs(far, e2);
      if (e2 <= ecc) break;
      root = far;
      ecc = e2;
      far = far2;
    }
    // Cuthill-McKee from the root
    const size_t first = order.size();
    order.push_back(root);
    done[root] = 1;
    for (size_t h = first; h < order.size(); ++h) {
      const int32_t u = order[h];
      nbrs.clear();
      for_nb(u, [&](int32_t v) {
        if (!done[v]) {
          done[v] = 1;
          nbrs.push_back(v);
        }
      });
      std::stable_sort(nbrs.begin(), nbrs.end(),
                       [&](int32_t a, int32_t b) { return deg[a] < deg[b]; });
      order.insert(order.end(), nbrs.begin(), nbrs.end());
    }
  }
  std::reverse(order.begin(), order.end());
  return order;
}

int64_t cross_block_entries(const std::vector<HostCSR>& mats, int64_t n, int64_t per,
                            const int32_t* inv) {
  int64_t cross = 0;
  for (int64_t r = 0; r < n; ++r) {
    const int64_t br = (inv ? inv[r] : r) / per;
    for (const HostCSR& h : mats)
      for (int64_t q = h.rp[r]; q < h.rp[r + 1]; ++q) {
        const int64_t c = h.col[q];
        cross += ((inv ? inv[c] : c) / per) != br;
      }
  }
  return cross;
}

}  // namespace cfet
