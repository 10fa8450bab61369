"""Plain CPU FP64 CFET propagator with a Lanczos-Krylov exponential (oracle).

TEST INFRASTRUCTURE ONLY.  Imported by ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py``; never by the product path.  It
shares no code with the HIP library (no kernels, tables, helpers or
pre/post-processing) and does not import it.

What it computes, step by step and in the paper's order:

1. Drive H(t) = H0 + sum_k f_k(t) H_k, A(t) = -i H(t)          (Sec. 1, eq. DGL)
2. Per time step t_n = t0 + n dt (computed fresh, not accumulated), for each
   exponential i = s, s-1, ..., 1 (Omega_s acts on psi first because
   U~ = exp(Omega_1) ... exp(Omega_s), Sec. 4 eq. Ucf):
       a_i      = sum_m g[i,m]
       b_{i,k}  = sum_m g[i,m] f_k(t_n + x_m dt)
       Omega_i  = -i dt (a_i H0 + sum_k b_{i,k} H_k)           (Sec. 7, eq. OmGLeg)
       psi     <- exp(Omega_i) psi
3. exp(-i dt H_i) psi by the Krylov (Lanczos) technique of Sec. 8.1: an
   orthonormal basis v_1..v_m of span{psi, H psi, ..., H^(m-1) psi} built by
   the three-term recurrence, the tridiagonal projection T, and
   psi <- |psi| V exp(-i dt T) e_1.
   The small exponential uses LAPACK's symmetric tridiagonal eigensolver
   (scipy.linalg.eigh_tridiagonal): exp(-i dt T) e_1 = Q exp(-i dt Lambda) Q^T e_1.

Readings where the paper is silent (listed with reasons in the design notes):
* no re-orthogonalisation, alpha_j = Re <v_j, H v_j>, beta_j = ||w||_2;
* breakdown: stop at j < m when beta_j <= 1e-12 * max_{k<=j}(|alpha_k| + beta_k),
  and the Krylov dimension never exceeds the matrix dimension;
* Lanczos runs on H_i and dt enters only in exp(-i dt T);
* psi is never renormalised.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .schemes import Scheme, gl_weights, scheme as get_scheme

BREAKDOWN_REL_TOL = 1e-12

__all__ = ["apply_rows", "drive_value", "step_weights", "lanczos", "tridiag_expm_e1", "expv",
           "expv_adaptive", "expv_dense", "propagate", "propagate_batch", "LanczosInfo",
           "BREAKDOWN_REL_TOL"]


# --------------------------------------------------------------------------
# drive functions f_k(t)
# --------------------------------------------------------------------------
def drive_value(d: dict, t: float) -> float:
    """Evaluate one drive function at time t.

    kinds: 'cos'      A cos(w t + phi)
           'sin2cos'  A sin^2(pi t / Tp) cos(w t + phi) on [0, Tp], 0 outside
                      (a pulsed field as used for the hydrogen atom, Sec. 11.2)
           'pwc'      u[k] for t_edges[k] <= t < t_edges[k+1], 0 outside
           'sechcos'  A cos(w t + phi) / cosh((t - tc)/tau)  (pulse shape of
                      Sec. 11.1, eq. BPulse, real part)
    """
    kind = d["kind"]
    if kind == "cos":
        return d["A"] * math.cos(d["omega"] * t + d.get("phi", 0.0))
    if kind == "sin2cos":
        Tp = d["Tp"]
        if t < 0.0 or t > Tp:
            return 0.0
        s = math.sin(math.pi * t / Tp)
        return d["A"] * s * s * math.cos(d["omega"] * t + d.get("phi", 0.0))
    if kind == "pwc":
        edges = d["t_edges"]
        u = d["u"]
        if t < edges[0] or t >= edges[-1]:
            return 0.0
        # plain linear scan: the piece k with edges[k] <= t < edges[k+1]
        for k in range(len(u)):
            if edges[k] <= t < edges[k + 1]:
                return float(u[k])
        return 0.0
    if kind == "sechcos":
        return d["A"] * math.cos(d["omega"] * t + d.get("phi", 0.0)) / math.cosh(
            (t - d["tc"]) / d["tau"])
    raise ValueError(f"unknown drive kind {kind}")


def step_weights(sc: Scheme, drives, t_n: float, dt: float):
    """(a, b) for one time step: a[i] = sum_m g[i,m] (weight of H0),
    b[i,k] = sum_m g[i,m] f_k(t_n + x_m dt) (weight of H_k).  Sec. 7."""
    x, g = gl_weights(sc)
    a = np.zeros(sc.s)
    b = np.zeros((sc.s, len(drives)))
    fvals = np.array([[drive_value(d, t_n + x[m] * dt) for d in drives]
                      for m in range(sc.M)]).reshape(sc.M, len(drives))
    for i in range(sc.s):
        acc = 0.0
        for m in range(sc.M):
            acc += g[i, m]
        a[i] = acc
        for k in range(len(drives)):
            acc = 0.0
            for m in range(sc.M):
                acc += g[i, m] * fvals[m, k]
            b[i, k] = acc
    return a, b


# --------------------------------------------------------------------------
# Lanczos-Krylov exponential (Sec. 8.1)
# --------------------------------------------------------------------------
@dataclass
class LanczosInfo:
    m_eff: int = 0
    beta0: float = 0.0
    alpha: np.ndarray = field(default_factory=lambda: np.zeros(0))
    beta: np.ndarray = field(default_factory=lambda: np.zeros(0))
    near_breakdown: bool = False


def lanczos(matvec, psi: np.ndarray, m: int, dim: int):
    """Three-term Lanczos recurrence started from psi.

    Returns (V, alpha, beta, info): V has m_eff orthonormal columns,
    alpha[0..m_eff-1] the diagonal of T, beta[0..m_eff-2] its off-diagonal.
    """
    info = LanczosInfo()
    beta0 = float(np.linalg.norm(psi))
    info.beta0 = beta0
    m = min(m, dim)
    if beta0 == 0.0:
        info.m_eff = 0
        return np.zeros((dim, 0), complex), np.zeros(0), np.zeros(0), info
    V = np.zeros((dim, m), dtype=np.complex128)
    alpha = np.zeros(m)
    beta = np.zeros(m)
    V[:, 0] = psi / beta0
    scale = 0.0
    m_eff = m
    for j in range(m):
        w = matvec(V[:, j])
        alpha[j] = float(np.real(np.vdot(V[:, j], w)))
        if j == m - 1:
            # the last basis vector needs only its alpha: T is m x m
            break
        w = w - alpha[j] * V[:, j]
        if j > 0:
            w = w - beta[j - 1] * V[:, j - 1]
        beta[j] = float(np.linalg.norm(w))
        scale = max(scale, abs(alpha[j]) + beta[j])
        tau = BREAKDOWN_REL_TOL * scale
        if beta[j] <= 10.0 * tau:
            info.near_breakdown = True
        if beta[j] <= tau:
            m_eff = j + 1
            break
        V[:, j + 1] = w / beta[j]
    info.m_eff = m_eff
    info.alpha = alpha[:m_eff].copy()
    info.beta = beta[:m_eff - 1].copy()
    return V[:, :m_eff], info.alpha, info.beta, info


def tridiag_expm_e1(alpha: np.ndarray, beta: np.ndarray, dt: float) -> np.ndarray:
    """c = exp(-i dt T) e_1 for the real symmetric tridiagonal T with diagonal
    alpha and off-diagonal beta, via T = Q diag(lam) Q^T (LAPACK)."""
    k = len(alpha)
    if k == 1:
        return np.array([np.exp(-1j * dt * alpha[0])])
    lam, Q = sla.eigh_tridiagonal(alpha, beta)
    return Q @ (np.exp(-1j * dt * lam) * Q[0, :])


def expv(H, psi: np.ndarray, dt: float, m: int, return_info: bool = False):
    """Krylov approximation of exp(-i dt H) psi with m Lanczos vectors."""
    dim = psi.shape[0]
    if hasattr(H, "to_scipy"):
        H = H.to_scipy()
    matvec = (lambda v: H @ v)
    V, alpha, beta, info = lanczos(matvec, psi, m, dim)
    if info.m_eff == 0:
        out = np.zeros_like(psi)
    else:
        c = tridiag_expm_e1(alpha, beta, dt)
        out = info.beta0 * (V @ c)
    return (out, info) if return_info else out


def expv_adaptive(H, psi: np.ndarray, dt: float, m_max: int, tol: float,
                  return_info: bool = False):
    """Krylov exponential with the basis size chosen per call.

    The Lanczos recurrence of ``lanczos`` runs until, after j basis vectors
    (j < m_max), either the breakdown rule fires or the a-posteriori estimate
    of the Krylov error relative to ||psi||,

        est_j = |dt| * beta_j * | e_j^T exp(-i dt T_j) e_1 |,

    is at most tol (T_j: the j x j tridiagonal projection, beta_j: the norm of
    the residual after j steps).  It is the leading term of the expansion of
    the Krylov error in the residual direction v_{j+1}, with phi_1 replaced by
    the exponential itself, and like the Krylov approximation it is invariant
    under H -> c H, dt -> dt / c.  The paper fixes m per run; its conclusions
    leave the automatic choice of the Krylov dimension open (Sec. 12).  At
    j = m_max the recurrence stops in any case, exactly as ``expv``.
    tol <= 0 gives ``expv`` with m = m_max.
    """
    dim = psi.shape[0]
    if hasattr(H, "to_scipy"):
        H = H.to_scipy()
    info = LanczosInfo()
    beta0 = float(np.linalg.norm(psi))
    info.beta0 = beta0
    m = min(m_max, dim)
    if beta0 == 0.0:
        out = np.zeros_like(psi)
        return (out, info) if return_info else out
    V = np.zeros((dim, m), dtype=np.complex128)
    alpha = np.zeros(m)
    beta = np.zeros(m)
    V[:, 0] = psi / beta0
    scale = 0.0
    m_eff = m
    c = None
    for j in range(m):
        w = H @ V[:, j]
        alpha[j] = float(np.real(np.vdot(V[:, j], w)))
        if j == m - 1:
            break
        w = w - alpha[j] * V[:, j]
        if j > 0:
            w = w - beta[j - 1] * V[:, j - 1]
        beta[j] = float(np.linalg.norm(w))
        scale = max(scale, abs(alpha[j]) + beta[j])
        if beta[j] <= BREAKDOWN_REL_TOL * scale:
            m_eff = j + 1
            break
        if tol > 0.0:
            cj = tridiag_expm_e1(alpha[:j + 1], beta[:j], dt)
            if abs(dt) * beta[j] * abs(cj[j]) <= tol:
                m_eff = j + 1
                c = cj
                break
        V[:, j + 1] = w / beta[j]
    info.m_eff = m_eff
    info.alpha = alpha[:m_eff].copy()
    info.beta = beta[:m_eff - 1].copy()
    if c is None:
        c = tridiag_expm_e1(info.alpha, info.beta, dt)
    out = beta0 * (V[:, :m_eff] @ c)
    return (out, info) if return_info else out


def expv_dense(H, psi: np.ndarray, dt: float) -> np.ndarray:
    """exp(-i dt H) psi by scipy.linalg.expm on the dense matrix (small dims)."""
    Hd = _as_matrix(H, True)
    return sla.expm(-1j * dt * Hd) @ psi


# --------------------------------------------------------------------------
# CFET time stepping (Secs. 4, 6.1, 7)
# --------------------------------------------------------------------------
def apply_rows(H0, Hk, a: float, b, x: np.ndarray, rows) -> np.ndarray:
    """Entries ``rows`` of y = (a H0 + sum_k b_k H_k) x, one row at a time from
    the CSR rows (for spot checks of operators too large to apply whole).
    The matrices are CSR containers with row_ptr / col / val arrays."""
    out = np.zeros(len(rows), dtype=np.complex128)
    mats = [(a, H0)] + [(bk, h) for bk, h in zip(b, Hk)]
    for i, r in enumerate(rows):
        acc = 0.0 + 0.0j
        for w, h in mats:
            lo, hi = int(h.row_ptr[r]), int(h.row_ptr[r + 1])
            acc += w * np.dot(h.val[lo:hi], x[h.col[lo:hi]])
        out[i] = acc
    return out


def _as_matrix(H, dense: bool):
    """Accept a scipy sparse matrix, a dense array, or any object with a
    ``to_scipy()`` method (the CSR container of the input generators)."""
    if hasattr(H, "to_scipy"):
        H = H.to_scipy()
    if dense:
        return H.toarray() if sp.issparse(H) else np.asarray(H)
    return sp.csr_matrix(H)


def propagate(H0, Hk, drives, psi0, t0: float, dt: float, nsteps: int,
              scheme_name: str, m: int | None = None, dense: bool = False,
              stats: dict | None = None, tol: float = 0.0):
    """Propagate psi0 over nsteps CFET steps of size dt starting at t0.

    H0: sparse/dense Hermitian matrix, Hk: list of matrices, drives: list of
    drive dicts (one per H_k).  With dense=True every exponential is taken
    exactly (expm), otherwise by Lanczos with m vectors (tol > 0: at most m,
    chosen per exponential by ``expv_adaptive``).
    """
    sc = get_scheme(scheme_name)
    if len(Hk) != len(drives):
        raise ValueError("one drive per driven term")
    psi = np.array(psi0, dtype=np.complex128, copy=True)
    H0 = _as_matrix(H0, dense)
    Hk = [_as_matrix(h, dense) for h in Hk]
    n_matvec = 0
    for n in range(nsteps):
        t_n = t0 + n * dt
        a, b = step_weights(sc, drives, t_n, dt)
        for i in range(sc.s - 1, -1, -1):
            Hi = a[i] * H0
            for k in range(len(Hk)):
                Hi = Hi + b[i, k] * Hk[k]
            if dense:
                psi = expv_dense(Hi, psi, dt)
            else:
                if tol > 0.0:
                    psi, info = expv_adaptive(Hi, psi, dt, m, tol, return_info=True)
                else:
                    psi, info = expv(Hi, psi, dt, m, return_info=True)
                n_matvec += info.m_eff
                if stats is not None:
                    stats.setdefault("m_eff", []).append(info.m_eff)
                    if info.near_breakdown:
                        stats["near_breakdown"] = stats.get("near_breakdown", 0) + 1
    if stats is not None:
        stats["n_matvec"] = n_matvec
    return psi


def propagate_batch(instances, t0: float, dt: float, nsteps: int, scheme_name: str,
                    m: int, tol: float = 0.0, stats: list | None = None):
    """Independent trajectories, one after another: each instance is a dict
    with keys H0, Hk, drives, psi0 and is propagated by ``propagate`` with the
    same scheme, time grid, m (the upper bound when tol > 0) and tol.
    Returns the list of final states (and per-instance stats when asked)."""
    out = []
    for inst in instances:
        st = {} if stats is not None else None
        out.append(propagate(inst["H0"], inst["Hk"], inst["drives"], inst["psi0"], t0, dt,
                             nsteps, scheme_name, m=m, stats=st, tol=tol))
        if stats is not None:
            stats.append(st)
    return out
