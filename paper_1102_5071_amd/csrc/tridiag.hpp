// exp(-i dt T) e_1 for a real symmetric tridiagonal T of order k <= 64,
// computed by one 64-lane wavefront (the small exponential of paper Sec. 8.1).
//
// Method: implicit symmetric QR iteration with Wilkinson shift (bulge chasing
// with Givens rotations), deflating from the bottom, accumulating the
// rotations into Z so that T = Z diag(lambda) Z^T.  Then
//     c = Z exp(-i dt lambda) Z^T e_1,  c_r = sum_l Z[r][l] e^{-i dt lambda_l} Z[0][l].
// Lane r holds T's diagonal entry a_r and sub-diagonal entry b_r (b_r couples
// rows r and r+1) in registers and row r of Z in LDS (column-major,
// Z[col*64 + row], so every lane touches only its own bank).  Uniform scalars
// of the sweep are read with v_readlane; deflation flags for all positions
// are formed in parallel and combined with a ballot.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

namespace cfet {

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ double lane_read(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// Diagonalise T in place: on return lane l's a holds eigenvalue l and column l
// of Z (LDS) its eigenvector.  Returns 0 or CFET_ENOCONV.
__device__ inline int tridiag_eig_wave(double& a, double& b, int k, double* Z) {
  const int lane = threadIdx.x & 63;
  for (int col = 0; col < k; ++col) Z[col * 64 + lane] = (lane == col) ? 1.0 : 0.0;
  if (lane >= k - 1) b = 0.0;
  if (lane >= k) a = 0.0;
  const double eps = 2.220446049250313e-16;
  const double tnorm = wave_max(fabs(a) + fabs(b));
  const double floor_abs = 1e-2 * eps * tnorm;
  int q = k - 1;
  int iters = 0;
  const int maxit = 40 * k;
  while (q > 0) {
    const double anext = __shfl_down(a, 1, 64);
    const bool neg = (lane < k - 1) && (fabs(b) <= eps * (fabs(a) + fabs(anext)) + floor_abs);
    const unsigned long long mask = __ballot(neg);
    if (neg) b = 0.0;
    while (q > 0 && ((mask >> (q - 1)) & 1ull)) --q;
    if (q == 0) break;
    const unsigned long long below = (q >= 2) ? (mask & ((1ull << (q - 1)) - 1ull)) : 0ull;
    const int p = below ? (64 - __clzll(below)) : 0;
    if (++iters > maxit) return CFET_ENOCONV;
    // Wilkinson shift from the trailing 2x2 block of [p..q]
    const double aq = lane_read(a, q), aq1 = lane_read(a, q - 1), bq = lane_read(b, q - 1);
    const double d = 0.5 * (aq1 - aq);
    const double h = sqrt(d * d + bq * bq);
    const double mu = aq - bq * bq / (d + (d >= 0.0 ? h : -h));
    // chase the bulge from p to q
    double ak = lane_read(a, p), bk = lane_read(b, p);
    double bprev = 0.0, bulge = 0.0;
    double zk = Z[p * 64 + lane];
    for (int kk = p; kk < q; ++kk) {
      const double ak1 = lane_read(a, kk + 1);
      const double bk1 = (kk + 1 < q) ? lane_read(b, kk + 1) : 0.0;
      const double xr = (kk == p) ? ak - mu : bprev;
      const double zr = (kk == p) ? bk : bulge;
      const double r = sqrt(xr * xr + zr * zr);
      double c = 1.0, s = 0.0;
      if (r != 0.0) {
        const double ir = 1.0 / r;
        c = xr * ir;
        s = zr * ir;
      }
      if (kk > p && lane == kk - 1) b = r;
      const double cc = c * c, ss = s * s, cs = c * s;
      const double nak = cc * ak + 2.0 * cs * bk + ss * ak1;
      const double nak1 = ss * ak - 2.0 * cs * bk + cc * ak1;
      const double nbk = cs * (ak1 - ak) + (cc - ss) * bk;
      bulge = s * bk1;
      const double nbk1 = c * bk1;
      if (lane == kk) a = nak;
      ak = nak1;
      bk = nbk1;
      bprev = nbk;
      const double zk1 = Z[(kk + 1) * 64 + lane];
      Z[kk * 64 + lane] = c * zk + s * zk1;
      zk = c * zk1 - s * zk;
    }
    if (lane == q) a = ak;
    if (lane == q - 1) b = bprev;
    Z[q * 64 + lane] = zk;
  }
  return 0;
}

// c (lane r holds c_r) = exp(-i dt T) e_1 by diagonalisation.  a, b as above
// (taken by value).  Z: 64*64 doubles of LDS, phi: 64 complex of LDS.
// Returns 0 or CFET_ENOCONV.
__device__ inline int tridiag_exp_e1_qr(double a, double b, int k, double dt, double* Z,
                                        double2* phi, double2& c) {
  const int lane = threadIdx.x & 63;
  const int status = tridiag_eig_wave(a, b, k, Z);
  double sn, cs;
  sincos(dt * a, &sn, &cs);
  const double z0 = Z[lane * 64];  // row 0 of eigenvector 'lane'
  if (lane < k) phi[lane] = make_double2(cs * z0, -sn * z0);
  wave_sync();
  double cr = 0.0, ci = 0.0;
  for (int l = 0; l < k; ++l) {
    const double z = Z[l * 64 + lane];
    const double2 p = phi[l];
    cr += z * p.x;
    ci += z * p.y;
  }
  c = (lane < k) ? make_double2(cr, ci) : make_double2(0.0, 0.0);
  wave_sync();
  return status;
}

}  // namespace cfet

namespace cfet {

// Values of the neighbouring lanes (wavefront-wide DPP shifts; 0 past the ends).
__device__ __forceinline__ double from_lane_below(double v) {  // lane r receives lane r-1
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x138, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x138, 0xf, 0xf, true);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double from_lane_above(double v) {  // lane r receives lane r+1
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x130, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x130, 0xf, 0xf, true);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
  return v;
}

// Number of eigenvalues of T below x (Sylvester inertia of the LDL^T
// factorisation of T - x I); x may differ per lane.
__device__ inline int sturm_count(double a, double b, int k, double x) {
  // q_r = det(T_r - x I) = (a_r - x) q_{r-1} - b_{r-1}^2 q_{r-2}, q_0 = 1: the
  // count is the number of sign changes along q_0..q_k (no division: both
  // terms are rescaled together when |q_r| leaves [1e-100, 1e100]; an exact
  // zero takes the sign opposite to its predecessor)
  int cnt = 0;
  double q = 1.0, qp = 0.0;
  for (int r = 0; r < k; ++r) {
    const double ar = lane_read(a, r);
    const double br = (r > 0) ? lane_read(b, r - 1) : 0.0;
    double qn = (ar - x) * q - (br * br) * qp;
    if (qn == 0.0) qn = (q < 0.0) ? 1e-300 : -1e-300;
    cnt += ((qn < 0.0) != (q < 0.0)) ? 1 : 0;
    const double aq = fabs(qn);
    const double sc = (aq > 1e100) ? 1e-100 : ((aq < 1e-100) ? 1e100 : 1.0);
    qp = q * sc;
    q = qn * sc;
  }
  return cnt;
}

// Miller's backward recurrence for the Bessel values fused with Clenshaw's
// for the Chebyshev sum (used by tridiag_exp_e1_cheb).  Miller: f_{Nm+1} = 0,
// f_{Nm} = tiny, f_{j-1} = (2j/theta) f_j - f_{j+1}, with Nm >= N + 16 (J_Nm is
// then below J_N by orders of magnitude, so the start leaves no trace in
// f_0 .. f_N); f_j = J_j(theta) / S with S = f_0 + 2 sum_{k >= 1} f_2k (the
// Bessel sum J_0 + 2 sum J_2k = 1).  The sum sum_{j <= N} w_j f_j T_j(X) e_1,
// w_0 = 1 and w_j = 2 (sgn i)^j, is taken by Clenshaw's recurrence
// y_j = w_j f_j e_1 + 2 X y_{j+1} - y_{j+2} (sum = y_0 - X y_1), which runs
// downwards in j like Miller's, so both advance in one loop as independent
// chains whose latencies overlap.  X is real: the even j feed the real part,
// the odd j the imaginary part.  PACKED: both parts in one vector (real rows
// in lanes 0..31, imaginary rows in lanes 32..63; wre, wim are nonzero in
// lane 0 and lane 32), else in two (yr, yi; wre, wim nonzero in lane 0).
// On return f0 = f_0, S without its f_0 term, and y1, y2 (yi1, yi2) = y_1, y_2.
template <bool PACKED>
__device__ __forceinline__ void miller_clenshaw(int N, int Nm, double theta, double ax, double blo,
                                                double bhi, double wre, double wim, double& f0,
                                                double& S, double& yr1, double& yr2, double& yi1,
                                                double& yi2) {
  const double it2 = 2.0 / theta;
  const double a2 = 2.0 * ax, b2lo = 2.0 * blo, b2hi = 2.0 * bhi;
  double f1 = 0.0;
  f0 = 1e-30;
  S = 0.0;
  yr1 = yr2 = yi1 = yi2 = 0.0;
  // f0 <- f_{j-1}, f1 <- f_j
  auto miller = [&](int j) {
    const double fm = ((double)j * it2) * f0 - f1;
    f1 = f0;
    f0 = fm;
  };
  // Clenshaw step j (phase PH = j mod 4) with f0 = f_j
  auto clenshaw = [&](auto ph) {
    constexpr int PH = decltype(ph)::value;
    if (PH == 0 || PH == 2) S += 2.0 * f0;
    if constexpr (PACKED) {
      const double lo = from_lane_below(yr1), hi = from_lane_above(yr1);
      double r = a2 * yr1 - yr2;
      if (PH == 0) r = wre * f0 + r;
      if (PH == 2) r = r - wre * f0;
      if (PH == 1) r = wim * f0 + r;
      if (PH == 3) r = r - wim * f0;
      r = b2lo * lo + r;
      yr2 = yr1;
      yr1 = b2hi * hi + r;
    } else {
      const double lr = from_lane_below(yr1), hr = from_lane_above(yr1);
      const double li = from_lane_below(yi1), hi = from_lane_above(yi1);
      double r = a2 * yr1 - yr2;
      double q = a2 * yi1 - yi2;
      if (PH == 0) r = wre * f0 + r;
      if (PH == 2) r = r - wre * f0;
      if (PH == 1) q = wim * f0 + q;
      if (PH == 3) q = q - wim * f0;
      r = b2lo * lr + r;
      q = b2lo * li + q;
      yr2 = yr1;
      yi2 = yi1;
      yr1 = b2hi * hr + r;
      yi1 = b2hi * hi + q;
    }
  };
  using P0 = std::integral_constant<int, 0>;
  using P1 = std::integral_constant<int, 1>;
  using P2 = std::integral_constant<int, 2>;
  using P3 = std::integral_constant<int, 3>;
  auto clenshaw_any = [&](int j) {
    switch (j & 3) {
      case 0: clenshaw(P0{}); break;
      case 1: clenshaw(P1{}); break;
      case 2: clenshaw(P2{}); break;
      default: clenshaw(P3{}); break;
    }
  };
  // |f| grows by at most 2 Nm/theta + 1 <= 1e8 per step (theta >= 1e-6 here),
  // so tests every 4 steps (and once after the first 16..31) at 1e150 keep
  // every value far below the overflow threshold; everything is scaled alike
  auto rescale = [&]() {
    if (__builtin_amdgcn_readfirstlane(fabs(f0) > 1e150 ? 1 : 0)) {
      f0 *= 1e-200;
      f1 *= 1e-200;
      S *= 1e-200;
      yr1 *= 1e-200;
      yr2 *= 1e-200;
      yi1 *= 1e-200;
      yi2 *= 1e-200;
    }
  };
  int j = Nm;
  for (; j > N; --j) miller(j);  // f_N, f_{N+1}
  rescale();
  for (; j >= 1 && (j & 3) != 3; --j) {
    clenshaw_any(j);
    miller(j);
  }
  // j = 3 mod 4 at the top: phases 3, 2, 1, 0
  for (; j >= 4; j -= 4) {
    clenshaw(P3{});
    miller(j);
    clenshaw(P2{});
    miller(j - 1);
    clenshaw(P1{});
    miller(j - 2);
    clenshaw(P0{});
    miller(j - 3);
    rescale();
  }
  for (; j >= 1; --j) {
    clenshaw_any(j);
    miller(j);
  }
}

constexpr int kChebMaxTerms = 8192;      // LDS doubles a caller reserves (the QR path's Z and phi)
constexpr double kChebMaxTheta = 7000.0; // beyond this the QR path is cheaper

// c = exp(-i dt T) e_1 by the Chebyshev expansion of exp(-i theta x) on the
// spectral interval of T (Jacobi-Anger: exp(-i theta x) = J_0(theta)
// + 2 sum_k (-i)^k J_k(theta) T_k(x)), with X = (T - sigma)/h.  The Bessel
// values J_k(theta) come from Miller's backward recurrence normalised by
// J_0 + 2 sum J_2k = 1, and the series is summed by Clenshaw's backward
// recurrence in the same loop.  lds is not used here (the QR path uses it).
// Returns 0, or 1 if theta is too large for this path (the caller then
// diagonalises).
__device__ inline int tridiag_exp_e1_cheb(double a, double b, int k, double dt, double* lds,
                                          double2& c) {
  const int lane = threadIdx.x & 63;
  // k and the term counts are the same in every lane: keep them (and the loops
  // over them) scalar so that the recurrences below run without exec masking
  k = __builtin_amdgcn_readfirstlane(k);
  if (lane >= k - 1) b = 0.0;
  if (lane >= k) a = 0.0;
  const double bl = from_lane_below(b);      // b_{r-1}
  // Gershgorin interval
  double lo = (lane < k) ? a - fabs(bl) - fabs(b) : 1e300;
  double hi = (lane < k) ? a + fabs(bl) + fabs(b) : -1e300;
  lo = wave_min(lo);
  hi = wave_max(hi);
  double theta = fabs(dt) * 0.5 * (hi - lo);
  // A multisection round (one Sturm recurrence of length k per lane) costs
  // about as much as 60 terms of the expansion below, and a tighter interval
  // saves (theta_Gershgorin - theta) terms: worth it only for large theta
  // (Gershgorin overestimates the half-width of Lanczos matrices by some tens
  // of per cent).
  if (theta > 256.0 && k > 1) {
    // Two rounds of 64-point multisection on the Sturm count tighten both
    // ends: round 0 spans the Gershgorin interval, round 1 spends 32 points
    // on each end within one round-0 spacing.  Every update keeps a valid
    // bound (count == k: all eigenvalues below x; count == 0: none below x).
    const double w0 = (hi - lo) / 64.0;
    for (int round = 0; round < 2; ++round) {
      const double x = (round == 0) ? lo + w0 * (double)(lane + 1)
                       : (lane < 32) ? lo + w0 * (double)(lane + 1) / 32.0
                                     : hi - w0 * (double)(64 - lane) / 32.0;
      const int cnt = sturm_count(a, b, k, x);
      const double nhi = wave_min((cnt == k) ? x : 1e300);
      const double nlo = wave_max((cnt == 0) ? x : -1e300);
      if (nhi < 1e299) hi = fmin(hi, nhi);
      if (nlo > -1e299) lo = fmax(lo, nlo);
    }
    // rounding in the counts can misplace a bound by a few ulps
    const double pad = 1e-10 * (fabs(hi) + fabs(lo)) + 1e-300;
    hi += pad;
    lo -= pad;
  }
  const double sigma = 0.5 * (hi + lo);
  const double h = 0.5 * (hi - lo);
  theta = fabs(dt) * h;
  if (theta > kChebMaxTheta) return 1;
  // phase of exp(-i dt sigma)
  double sn, cs;
  sincos(dt * sigma, &sn, &cs);
  if (!(theta > 1e-300)) {  // T = sigma I
    c = (lane == 0) ? make_double2(cs, -sn) : make_double2(0.0, 0.0);
    return 0;
  }
  const double inv_h = 1.0 / h;
  const double ax = (lane < k) ? (a - sigma) * inv_h : 0.0;
  const double blo = bl * inv_h, bhi = b * inv_h;
  if (theta < 1e-6) {
    // exp(-i s X) e_1 = e_1 - i s X e_1 - (s^2 / 2) X^2 e_1 + O(s^3), s = dt h
    const double sx = dt * h;
    const double e1 = (lane == 0) ? 1.0 : 0.0;
    const double x1 = ax * e1 + blo * from_lane_below(e1) + bhi * from_lane_above(e1);
    const double x2 = ax * x1 + blo * from_lane_below(x1) + bhi * from_lane_above(x1);
    const double cr = e1 - 0.5 * sx * sx * x2, ci = -sx * x1;
    c = (lane < k) ? make_double2(cs * cr + sn * ci, cs * ci - sn * cr) : make_double2(0.0, 0.0);
    return 0;
  }
  // truncation after N terms: 2 sum_{j > N} |J_j(theta)| stays below 4e-19
  // for 0.04 <= theta <= 7000 and below 3e-16 for smaller theta
  const int N = __builtin_amdgcn_readfirstlane((int)ceil(theta + 12.0 * cbrt(theta) + 2.0));
  const int Nm = (N + 16 + 15) & ~15;
  const double sgn = (dt >= 0.0) ? -1.0 : 1.0;   // phase (sgn i)^j
  double cr, ci, S;
  if (k <= 32) {
    // real part in lanes 0..31, imaginary part in lanes 32..63 (row = lane & 31);
    // the rows past k have zero coefficients, so nothing crosses between halves
    const int src = lane & 31;
    const double pax = __shfl(ax, src, 64), pblo = __shfl(blo, src, 64), pbhi = __shfl(bhi, src, 64);
    double y1, y2, unused1 = 0.0, unused2 = 0.0, f0;
    miller_clenshaw<true>(N, Nm, theta, pax, pblo, pbhi, (lane == 0) ? 2.0 : 0.0,
                          (lane == 32) ? 2.0 * sgn : 0.0, f0, S, y1, y2, unused1, unused2);
    S += f0;
    double sum = pax * y1 + pblo * from_lane_below(y1) + pbhi * from_lane_above(y1) - y2;
    sum = ((lane == 0) ? f0 : 0.0) + sum;
    cr = sum;
    ci = __shfl(sum, src + 32, 64);
  } else {
    const double e1 = (lane == 0) ? 1.0 : 0.0;
    double yr1, yr2, yi1, yi2, f0;
    miller_clenshaw<false>(N, Nm, theta, ax, blo, bhi, 2.0 * e1, 2.0 * sgn * e1, f0, S, yr1, yr2,
                           yi1, yi2);
    S += f0;
    cr = ax * yr1 + blo * from_lane_below(yr1) + bhi * from_lane_above(yr1) - yr2;
    ci = ax * yi1 + blo * from_lane_below(yi1) + bhi * from_lane_above(yi1) - yi2;
    cr = e1 * f0 + cr;
  }
  const double invS = 1.0 / S;
  cr *= invS;
  ci *= invS;
  // multiply by exp(-i dt sigma) = cs - i sn
  c = (lane < k) ? make_double2(cs * cr + sn * ci, cs * ci - sn * cr) : make_double2(0.0, 0.0);
  wave_sync();
  return 0;
}

// Dispatcher: Chebyshev when cheap, diagonalisation otherwise.  lds must hold
// kChebMaxTerms doubles (it also hosts Z and phi of the QR path).  Kept out of
// line: it runs once per exponential, and inlining it would raise the register
// count of the whole persistent kernel.
__device__ __noinline__ int tridiag_exp_e1(double a, double b, int k, double dt, double* lds,
                                           double2& c) {
  if (k == 1) {
    double sn, cs;
    sincos(dt * a, &sn, &cs);
    c = ((threadIdx.x & 63) == 0) ? make_double2(cs, -sn) : make_double2(0.0, 0.0);
    return 0;
  }
  if (tridiag_exp_e1_cheb(a, b, k, dt, lds, c) == 0) return 0;
  return tridiag_exp_e1_qr(a, b, k, dt, lds, reinterpret_cast<double2*>(lds + 64 * 64), c);
}

}  // namespace cfet
