"""Plain CPU FP64 gradient of the final-state fidelity of a CFET run (oracle).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: imported by tests,
``__graft_entry__.smoke()`` and ``bench.py``'s CPU baseline, never by the
product path, and sharing no code with the HIP library.

Quantity.  For psi_N = U_N ... U_1 psi_0, each step
U_n = E_{n,1} ... E_{n,s} (exp(Omega_{n,s}) acts first, Sec. 4 eq. Ucf) with
Omega_{n,i} = -i dt (a_i H0 + sum_k b_{n,i,k} H_k) (Sec. 7, eq. OmGLeg) and one
driven term k* piecewise constant, f(t) = u_p on [t_p, t_{p+1}):

    F = |<phi|psi_N>|^2,   dF/du_p = 2 Re( conj(z) dz/du_p ),  z = <phi|psi_N>,

where b_{n,i,k*} = sum_m g_{i,m} f(t_n + x_m dt), so
db_{n,i}/du_p = sum of g_{i,m} over the Gauss points x_m whose time falls in
piece p, and

    dz/du_p = sum_{n,i} db_{n,i}/du_p  <lambda_{n,i}| L(Omega_{n,i}, -i dt H_k*) |psi_{n,i}>

with psi_{n,i} the state before E_{n,i}, lambda_{n,i} = (later factors)^H phi
the adjoint state after it, and L(A, D) = int_0^1 e^{sA} D e^{(1-s)A} ds the
Frechet derivative of the exponential, the top-right block of
exp([[A, D], [0, A]]) (the block-triangular augmented operator).

Discretisation of each term (the same Krylov technique as the forward
exponential, Sec. 8.1).  With Lanczos bases of H_i started from psi_{n,i}
(V, T, beta_psi = ||psi||) and from lambda_{n,i} (W, S, beta_lam), the
augmented operator is projected onto span(W) + span(V):

    <lambda| L |psi>  ~  beta_lam beta_psi  e_1^T  exp(M)[top-right]  e_1,
    M = [[-i dt S, -i dt C], [0, -i dt T]],  C = W^H H_k* V,

which is exact when both Krylov spaces are invariant (e.g. m >= dim).  The
adjoint state moves back by the same Lanczos basis:
lambda_{n,i-before} = E^H lambda = beta_lam W exp(+i dt S) e_1.

A second, independent route (route="augmented") takes each term straight
from the definition: the Krylov technique of Sec. 8.1 applied to the
2n-dimensional block-triangular operator  A = [[X, D], [0, X]]  (X = Omega,
D = -i dt H_k*) started from [0; psi]: exp(A) [0; psi] = [L(X, D) psi;
exp(X) psi], so <lambda| L |psi> is <lambda| with the top half of the Krylov
approximation of exp(A) [0; psi].  A is not skew-Hermitian, so the basis is
built by Arnoldi with full (modified Gram-Schmidt) orthogonalisation and the
small exponential is scipy's expm of the Hessenberg matrix; m_aug = 2 m
vectors by default (the augmented space holds both chains).

Memory: psi is kept at every ceil(sqrt(N))-th step; each segment is recomputed
forward (storing the states before each exponential) when the backward sweep
reaches it.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla

from .cfet import _as_matrix, drive_value, expv, lanczos, step_weights, tridiag_expm_e1
from .schemes import gl_weights, scheme as get_scheme

__all__ = ["piece_of", "weight_derivatives", "fidelity", "fidelity_gradient",
           "frechet_term", "frechet_term_augmented", "arnoldi_expv"]


def piece_of(d: dict, t: float) -> int:
    """Index p of the piece of a 'pwc' drive containing t, or -1 outside."""
    edges = d["t_edges"]
    if t < edges[0] or t >= edges[-1]:
        return -1
    for p in range(len(edges) - 1):
        if edges[p] <= t < edges[p + 1]:
            return p
    return -1


def weight_derivatives(sc, d: dict, t_n: float, dt: float):
    """For one step: list over exponentials i of {p: db_{n,i}/du_p}."""
    x, g = gl_weights(sc)
    out = []
    for i in range(sc.s):
        acc = {}
        for m in range(sc.M):
            p = piece_of(d, t_n + x[m] * dt)
            if p >= 0:
                acc[p] = acc.get(p, 0.0) + g[i, m]
        out.append(acc)
    return out


def _lanczos_basis(H, v, m):
    """Lanczos basis of H from v: (V with orthonormal columns, alpha, beta, beta0)."""
    V, alpha, beta, info = lanczos(lambda x: H @ x, v, m, v.shape[0])
    return V, alpha, beta, info.beta0


def frechet_term(Hi, Hk, psi, lam, dt: float, m: int):
    """<lam| L(-i dt Hi, -i dt Hk) |psi> by the projected augmented operator,
    and the adjoint state moved back, lam_before = exp(+i dt Hi) lam (Lanczos)."""
    V, a_psi, b_psi, beta_psi = _lanczos_basis(Hi, psi, m)
    W, a_lam, b_lam, beta_lam = _lanczos_basis(Hi, lam, m)
    if beta_psi == 0.0 or beta_lam == 0.0:
        lam_before = np.zeros_like(lam) if beta_lam == 0.0 else \
            beta_lam * (W @ tridiag_expm_e1(a_lam, b_lam, -dt))
        return 0.0 + 0.0j, lam_before
    ml, mp = W.shape[1], V.shape[1]
    S = np.diag(a_lam) + np.diag(b_lam, 1) + np.diag(b_lam, -1)
    T = np.diag(a_psi) + np.diag(b_psi, 1) + np.diag(b_psi, -1)
    C = W.conj().T @ (Hk @ V)
    M = np.zeros((ml + mp, ml + mp), dtype=np.complex128)
    M[:ml, :ml] = -1j * dt * S
    M[:ml, ml:] = -1j * dt * C
    M[ml:, ml:] = -1j * dt * T
    E = sla.expm(M)
    g = beta_lam * beta_psi * E[0, ml]
    lam_before = beta_lam * (W @ tridiag_expm_e1(a_lam, b_lam, -dt))
    return g, lam_before


def arnoldi_expv(matvec, b: np.ndarray, m: int, dim: int, info: dict | None = None):
    """Krylov approximation of exp(A) b for a general (non-normal) A given by
    matvec: Arnoldi with modified Gram-Schmidt, ||b|| Q_k expm(H_k) e_1 with
    k <= m the basis size reached (stops early when the next vector vanishes,
    relative to the Hessenberg entries so far, as the Lanczos rule).
    info (optional) receives k and the a-posteriori estimate of the error,
    ||b|| h_{k+1,k} |e_k^T expm(H_k) e_1| (zero when the space is invariant)."""
    beta = float(np.linalg.norm(b))
    if beta == 0.0:
        if info is not None:
            info.update(k=0, estimate=0.0)
        return np.zeros_like(b)
    m = min(m, dim)
    Q = np.zeros((b.shape[0], m), dtype=np.complex128)
    Hh = np.zeros((m, m), dtype=np.complex128)
    Q[:, 0] = b / beta
    k = m
    scale = 0.0
    h_next = 0.0
    for j in range(m):
        w = matvec(Q[:, j])
        for i in range(j + 1):
            Hh[i, j] = np.vdot(Q[:, i], w)
            w = w - Hh[i, j] * Q[:, i]
        nw = float(np.linalg.norm(w))
        scale = max(scale, float(np.max(np.abs(Hh[:j + 1, j]))) + nw)
        if nw <= 1e-12 * scale:
            k = j + 1
            break
        if j == m - 1:
            h_next = nw
            break
        Hh[j + 1, j] = nw
        Q[:, j + 1] = w / nw
    c = sla.expm(Hh[:k, :k])[:, 0]
    if info is not None:
        info.update(k=k, estimate=beta * h_next * abs(c[k - 1]))
    return beta * (Q[:, :k] @ c)


def frechet_term_augmented(Hi, Hk, psi, lam, dt: float, m: int, m_aug: int | None = None,
                           info: dict | None = None):
    """<lam| L(-i dt Hi, -i dt Hk) |psi> by Arnoldi on the augmented operator
    [[X, D], [0, X]] from [0; psi] (m_aug vectors, default 2 m), and the adjoint
    state moved back by the Lanczos exponential with m vectors.  info receives
    the Arnoldi basis size and error estimate (of the whole 2n-vector)."""
    n = psi.shape[0]
    m_aug = 2 * m if m_aug is None else m_aug

    def aug(v):
        top, bot = v[:n], v[n:]
        return np.concatenate([-1j * dt * (Hi @ top) - 1j * dt * (Hk @ bot),
                               -1j * dt * (Hi @ bot)])

    b = np.concatenate([np.zeros(n, dtype=np.complex128), np.asarray(psi, np.complex128)])
    y = arnoldi_expv(aug, b, m_aug, 2 * n, info)
    g = np.vdot(lam, y[:n])
    lam_before = expv(Hi, lam, -dt, m)
    return g, lam_before


def _exponentials_of_step(sc, H0, Hk, drives, t_n, dt):
    """The step's exponent operators in application order: list of (i, H_i)."""
    a, b = step_weights(sc, drives, t_n, dt)
    out = []
    for i in range(sc.s - 1, -1, -1):
        Hi = a[i] * H0
        for k in range(len(Hk)):
            Hi = Hi + b[i, k] * Hk[k]
        out.append((i, Hi))
    return out


def fidelity(H0, Hk, drives, psi0, target, t0, dt, nsteps, scheme_name, m):
    """F = |<target|psi_N>|^2 with the Lanczos CFET propagator (same as
    oracle.cfet.propagate)."""
    from .cfet import propagate
    psi = propagate(H0, Hk, drives, psi0, t0, dt, nsteps, scheme_name, m=m)
    return abs(np.vdot(target, psi)) ** 2


def fidelity_gradient(H0, Hk, drives, psi0, target, t0: float, dt: float, nsteps: int,
                      scheme_name: str, m: int, term: int = 0, stats: dict | None = None,
                      route: str = "projected", m_aug: int | None = None):
    """(F, dF/du) for the pieces u of the 'pwc' drive of driven term ``term``.
    route: "projected" (the augmented operator projected on the two Lanczos
    spaces) or "augmented" (Arnoldi on the augmented operator, m_aug vectors)."""
    if route not in ("projected", "augmented"):
        raise ValueError("route is 'projected' or 'augmented'")
    sc = get_scheme(scheme_name)
    d = drives[term]
    if d["kind"] != "pwc":
        raise ValueError("the differentiated term must have a piecewise-constant drive")
    K = len(d["u"])
    H0 = _as_matrix(H0, False)
    Hk = [_as_matrix(h, False) for h in Hk]
    H1 = Hk[term]
    psi = np.array(psi0, dtype=np.complex128, copy=True)
    N = nsteps
    seg = max(1, math.ceil(math.sqrt(N))) if N > 0 else 1
    # forward pass, keeping psi at the start of every segment
    ckpt = {}
    for n in range(N):
        if n % seg == 0:
            ckpt[n] = psi.copy()
        for i, Hi in _exponentials_of_step(sc, H0, Hk, drives, t0 + n * dt, dt):
            psi = expv(Hi, psi, dt, m)
    z = np.vdot(target, psi)
    F = abs(z) ** 2
    dz = np.zeros(K, dtype=np.complex128)
    lam = np.array(target, dtype=np.complex128, copy=True)
    starts = sorted(ckpt)
    for s0 in reversed(starts):
        s1 = min(N, s0 + seg)
        # recompute the segment, keeping the state before each exponential
        psi = ckpt[s0].copy()
        before = []
        for n in range(s0, s1):
            t_n = t0 + n * dt
            exps = _exponentials_of_step(sc, H0, Hk, drives, t_n, dt)
            db = weight_derivatives(sc, d, t_n, dt)
            for i, Hi in exps:
                before.append((n, i, Hi, psi.copy(), db[i]))
                psi = expv(Hi, psi, dt, m)
        for n, i, Hi, psi_b, dbi in reversed(before):
            if route == "projected":
                g, lam = frechet_term(Hi, H1, psi_b, lam, dt, m)
            else:
                g, lam = frechet_term_augmented(Hi, H1, psi_b, lam, dt, m, m_aug)
            for p, w in dbi.items():
                dz[p] += w * g
    grad = 2.0 * np.real(np.conj(z) * dz)
    if stats is not None:
        stats["z"] = z
        stats["segments"] = len(starts)
        stats["segment_steps"] = seg
    return F, grad
