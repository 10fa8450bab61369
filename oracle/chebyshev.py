"""Plain CPU FP64 CFET propagator with the Chebyshev exponential (oracle).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: imported by tests,
``__graft_entry__.smoke()`` and ``bench.py``'s CPU baseline, never by the
product path, and sharing no code with the HIP library.

The Chebyshev technique (Sec. 8.1, compared with Krylov in Sec. 8.2) expands
the exponential in Chebyshev polynomials of the operator mapped onto [-1, 1];
it needs a-priori bounds on the spectrum.  With bounds [e_lo, e_hi] of the
Hermitian H, sigma = (e_lo + e_hi)/2, h = (e_hi - e_lo)/2, H~ = (H - sigma)/h
and theta = dt h, the Jacobi-Anger expansion gives

    exp(-i dt H) psi = e^{-i dt sigma} sum_{k>=0} (2 - delta_k0) (-i)^k J_k(theta) T_k(H~) psi,

with T_0 psi = psi, T_1 psi = H~ psi, T_{k+1} psi = 2 H~ T_k psi - T_{k-1} psi.

Readings where the paper leaves the choice (each stated in the design notes):
* bounds: Gershgorin discs of each operator (row r: diagonal d_r, radius
  R_r = sum_{c != r} |H_rc|; [min(d - R), max(d + R)]), combined for
  H_i = a_i H0 + sum_k b_ik H_k by interval arithmetic (a negative weight swaps
  the ends); the sum of intervals contains the spectrum of the sum (Weyl);
* truncation: the series stops after term K, the smallest K whose tail bound
  2 (|theta|/2)^(K+1) / (K+1)! / (1 - q), q = |theta| / (2 (K+2)) < 1, from
  |J_k(theta)| <= (|theta|/2)^k / k! and |T_k| <= 1 on [-1, 1], is at most tol
  (the error is then at most tol ||psi||);
* a zero-width interval (H = sigma I on the whole space) gives e^{-i dt sigma} psi.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.special as ssp

from .cfet import _as_matrix, step_weights
from .schemes import scheme as get_scheme

__all__ = ["gershgorin_bounds", "weighted_bounds", "chebyshev_terms", "chebyshev_expv",
           "propagate_chebyshev"]


def gershgorin_bounds(H) -> tuple[float, float]:
    """[min_r (d_r - R_r), max_r (d_r + R_r)] of a Hermitian matrix."""
    H = _as_matrix(H, False)
    d = np.real(H.diagonal())
    R = np.asarray(abs(H).sum(axis=1)).ravel() - np.abs(H.diagonal())
    R = np.maximum(R, 0.0)
    return float(np.min(d - R)), float(np.max(d + R))


def weighted_bounds(bounds, weights) -> tuple[float, float]:
    """Interval containing the spectrum of sum_j w_j H_j from the intervals of
    the H_j (w_j >= 0: w [lo, hi]; w_j < 0: w [hi, lo])."""
    lo = hi = 0.0
    for (l, h), w in zip(bounds, weights):
        if w >= 0.0:
            lo += w * l
            hi += w * h
        else:
            lo += w * h
            hi += w * l
    return lo, hi


def chebyshev_terms(theta: float, tol: float) -> int:
    """The last index K kept: the smallest K >= 0 whose tail bound is <= tol."""
    x = abs(theta) / 2.0
    if x == 0.0:
        return 0
    k = 0
    while True:
        q = x / (k + 2)
        if q < 1.0:
            log_tail = (math.log(2.0) + (k + 1) * math.log(x) - math.lgamma(k + 2)
                        - math.log1p(-q))
            if log_tail <= math.log(tol):
                return k
        k += 1


def chebyshev_expv(H, psi, dt: float, lo: float, hi: float, tol: float,
                   return_terms: bool = False):
    """exp(-i dt H) psi by the Chebyshev series on the interval [lo, hi]."""
    H = _as_matrix(H, False)
    psi = np.asarray(psi, dtype=np.complex128)
    sigma = 0.5 * (lo + hi)
    h = 0.5 * (hi - lo)
    phase = np.exp(-1j * dt * sigma)
    if h <= 0.0:
        out = phase * psi
        return (out, 0) if return_terms else out
    theta = dt * h
    K = chebyshev_terms(theta, tol)
    # coefficients (2 - delta_k0) (-i)^k J_k(theta), J from scipy
    ks = np.arange(K + 1)
    coef = (2.0 - (ks == 0)) * ((-1j) ** ks) * ssp.jv(ks, theta)

    def Ht(v):
        return (H @ v - sigma * v) / h

    t_prev = psi
    out = coef[0] * t_prev
    if K >= 1:
        t_cur = Ht(psi)
        out = out + coef[1] * t_cur
        for k in range(2, K + 1):
            t_next = 2.0 * Ht(t_cur) - t_prev
            out = out + coef[k] * t_next
            t_prev, t_cur = t_cur, t_next
    out = phase * out
    return (out, K) if return_terms else out


def propagate_chebyshev(H0, Hk, drives, psi0, t0: float, dt: float, nsteps: int,
                        scheme_name: str, tol: float, stats: dict | None = None):
    """The CFET step loop of oracle.cfet.propagate (Omega_s first) with every
    exponential taken by the Chebyshev series; the spectral interval of
    H_i = a_i H0 + sum_k b_ik H_k from the terms' Gershgorin intervals."""
    sc = get_scheme(scheme_name)
    if len(Hk) != len(drives):
        raise ValueError("one drive per driven term")
    H0 = _as_matrix(H0, False)
    Hk = [_as_matrix(h, False) for h in Hk]
    bounds = [gershgorin_bounds(H0)] + [gershgorin_bounds(h) for h in Hk]
    psi = np.array(psi0, dtype=np.complex128, copy=True)
    n_matvec = 0
    for n in range(nsteps):
        t_n = t0 + n * dt
        a, b = step_weights(sc, drives, t_n, dt)
        for i in range(sc.s - 1, -1, -1):
            Hi = a[i] * H0
            for k in range(len(Hk)):
                Hi = Hi + b[i, k] * Hk[k]
            lo, hi = weighted_bounds(bounds, [a[i]] + [b[i, k] for k in range(len(Hk))])
            psi, K = chebyshev_expv(Hi, psi, dt, lo, hi, tol, return_terms=True)
            n_matvec += K
            if stats is not None:
                stats.setdefault("terms", []).append(K)
    if stats is not None:
        stats["n_matvec"] = n_matvec
    return psi
