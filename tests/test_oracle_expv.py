"""Pins for the oracle's Lanczos-Krylov exponential (Sec. 8.1).

The references are library routines on cases where the Krylov approximation is
exact or converged (scipy.linalg.expm), the closed form of the harmonic
oscillator example of Sec. 8.2 (H_nn = n w  =>  psi_n(t) = exp(-i t w n) psi_n),
and invariants of the recurrence (orthonormal basis, T = V^H H V).
"""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import cfet as O
from paper_1102_5071_amd import inputs as I


def _rand_herm(n, seed, scale=1.0):
    return I.random_hermitian(n, np.random.default_rng(seed), scale=scale).toarray()


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8])
def test_full_krylov_equals_expm(n):
    H = _rand_herm(n, 10 + n)
    psi = I.random_state(n, np.random.default_rng(n))
    dt = 0.7
    out = O.expv(H, psi, dt, m=16)          # m > n: clipped / breaks down at n
    ref = sla.expm(-1j * dt * H) @ psi
    assert np.linalg.norm(out - ref) < 1e-13


@pytest.mark.parametrize("n,m", [(40, 24), (64, 30), (64, 40)])
def test_converged_krylov_equals_expm(n, m):
    H = _rand_herm(n, n, scale=0.3)
    psi = I.random_state(n, np.random.default_rng(3))
    dt = 0.5
    out = O.expv(H, psi, dt, m=m)
    ref = sla.expm(-1j * dt * H) @ psi
    assert np.linalg.norm(out - ref) < 1e-12


def test_harmonic_oscillator_closed_form():
    # Sec. 8.2: diagonal 50 x 50 H_nn = n w, random psi, t = pi/(10 w)
    w = 1.0
    n = 50
    H = np.diag(np.arange(n) * w).astype(complex)
    psi = np.random.default_rng(7).random(n).astype(complex)
    psi /= np.linalg.norm(psi)
    t = np.pi / (10 * w)
    exact = np.exp(-1j * t * w * np.arange(n)) * psi
    errs = []
    for K in (6, 10, 14, 20, 26):
        errs.append(np.linalg.norm(O.expv(H, psi, t, m=K) - exact))
    # error falls fast with the number of Krylov vectors and reaches rounding
    assert all(errs[i + 1] < errs[i] for i in range(3))
    assert errs[-1] < 1e-12


def test_lanczos_basis_and_projection():
    n, m = 30, 12
    H = _rand_herm(n, 5)
    psi = I.random_state(n, np.random.default_rng(5))
    V, a, b, info = O.lanczos(lambda v: H @ v, psi, m, n)
    assert info.m_eff == m
    assert np.allclose(V.conj().T @ V, np.eye(m), atol=1e-12)
    T = V.conj().T @ H @ V
    Tref = np.diag(a) + np.diag(b, 1) + np.diag(b, -1)
    assert np.allclose(T, Tref, atol=1e-12)
    assert np.allclose(V[:, 0], psi / np.linalg.norm(psi))
    assert np.all(b > 0)


def test_breakdown_two_level():
    # dim 2 with m = 16: the Krylov space is exhausted after two vectors
    H = np.array([[0.5, 0.3 - 0.2j], [0.3 + 0.2j, -0.5]])
    psi = np.array([1.0, 0.0], dtype=complex)
    out, info = O.expv(H, psi, 0.4, m=16, return_info=True)
    assert info.m_eff == 2
    assert np.linalg.norm(out - sla.expm(-0.4j * H) @ psi) < 1e-15


def test_eigenvector_start_breaks_down_at_one():
    n = 6
    H = _rand_herm(n, 9)
    lam, Q = np.linalg.eigh(H)
    psi = Q[:, 2].astype(complex) * 1.7
    out, info = O.expv(H, psi, 0.9, m=5, return_info=True)
    assert info.m_eff == 1
    assert np.allclose(out, np.exp(-0.9j * lam[2]) * psi, atol=1e-13)


def test_zero_vector():
    H = _rand_herm(4, 1)
    out = O.expv(H, np.zeros(4, complex), 0.3, m=3)
    assert np.all(out == 0)


@pytest.mark.parametrize("k", [1, 2, 7, 30, 64])
def test_tridiagonal_exponential_matches_expm(k):
    rng = np.random.default_rng(k)
    a = rng.standard_normal(k) * 3
    b = np.abs(rng.standard_normal(k - 1)) + 0.1
    T = np.diag(a) + np.diag(b, 1) + np.diag(b, -1)
    for dt in (0.01, 0.7, 5.0):
        c = O.tridiag_expm_e1(a, b, dt)
        ref = sla.expm(-1j * dt * T)[:, 0]
        assert np.linalg.norm(c - ref) < 1e-13 * max(1, dt * np.abs(T).max())


def test_unitarity_of_krylov_step():
    # Sec. 8.2: the Krylov exponential preserves the norm even when inexact
    n = 200
    H = I.random_hermitian(n, np.random.default_rng(2), density=0.05).to_scipy()
    psi = I.random_state(n, np.random.default_rng(3))
    out = O.expv(H, psi, 2.0, m=6)        # far from converged
    assert abs(np.linalg.norm(out) - 1.0) < 1e-13
