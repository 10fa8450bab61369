"""Pins of the oracle's Chebyshev exponential and CFET propagator
(oracle.chebyshev; Sec. 8.1-8.2).

* Against scipy's expm (48-dim random Hermitian, five dt including negative
  and long ones, three tolerances): error <= tol ||psi||.
* The paper's own comparison case (Sec. 8.2): the harmonic oscillator
  H_nn = n w on 50 levels with a random psi, exact psi_n(t) = e^{-i t w n} psi_n;
  at t = pi / (10 w) the error falls below tol after 10-30 terms (the paper:
  fast decay after the first 10-20 terms), and a full period returns psi.
* Gershgorin intervals contain the spectrum (random, spin-chain, hydrogen
  operators and weighted sums with negative weights, by eigvalsh).
* The truncation rule: the chosen K meets the tail bound and K - 1 does not;
  the true tail 2 sum_{k>K} |J_k(theta)| (scipy's Bessel functions) is below tol.
* A zero-width interval (H = c I) gives the pure phase.
* The CFET propagator with Chebyshev exponentials equals the one with exact
  exponentials within (number of exponentials) x tol, and conserves the norm
  to the same accuracy.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.special as ssp

from oracle import cfet as O
from oracle import chebyshev as C
from paper_1102_5071_amd import inputs as I


def _random(n, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    return I.random_hermitian(n, rng, 0.4, scale).to_scipy(), I.random_state(n, rng)


@pytest.mark.parametrize("dt", [0.05, 0.3, 1.0, -0.7, 5.0])
@pytest.mark.parametrize("tol", [1e-6, 1e-10, 1e-14])
def test_error_below_tol(dt, tol):
    H, psi = _random(48, 1)
    lo, hi = C.gershgorin_bounds(H)
    out, K = C.chebyshev_expv(H, psi, dt, lo, hi, tol, return_terms=True)
    ex = sla.expm(-1j * dt * H.toarray()) @ psi
    # rounding of K terms of norm <= 2 each adds a few 1e-16 per term
    assert np.linalg.norm(out - ex) <= tol * np.linalg.norm(psi) + 1e-15 * (K + 1)
    assert K >= 1


def test_harmonic_oscillator_of_the_comparison():
    w, n = 1.0, 50
    rng = np.random.default_rng(8)
    psi = rng.standard_normal(n).astype(complex)
    psi /= np.linalg.norm(psi)
    H = I.diagonal(np.arange(n) * w)
    lo, hi = C.gershgorin_bounds(H)
    assert (lo, hi) == (0.0, (n - 1) * w)
    t = math.pi / (10 * w)
    exact = np.exp(-1j * t * w * np.arange(n)) * psi
    Ks = []
    for tol in (1e-4, 1e-8, 1e-12):
        out, K = C.chebyshev_expv(H, psi, t, lo, hi, tol, return_terms=True)
        assert np.linalg.norm(out - exact) <= tol
        Ks.append(K)
    assert 10 <= Ks[0] < Ks[1] < Ks[2] <= 30
    # a full period: e^{-i 2 pi n} = 1
    out = C.chebyshev_expv(H, psi, 2 * math.pi / w, lo, hi, 1e-13)
    assert np.linalg.norm(out - psi) <= 1e-12


def test_gershgorin_contains_the_spectrum():
    rng = np.random.default_rng(4)
    mats = [I.random_hermitian(40, rng, 0.3, 1.0), I.heisenberg_chain(6, 1.0, rng.uniform(-1, 1, 6)),
            I.sigma_x_sum(6), I.ising_chain(6, 1.0, rng.uniform(-1, 1, 6))]
    for M in mats:
        lo, hi = C.gershgorin_bounds(M)
        ev = np.linalg.eigvalsh(M.to_scipy().toarray())
        assert lo <= ev[0] + 1e-12 and ev[-1] <= hi + 1e-12
    H0, H1 = mats[1], mats[2]
    b0, b1 = C.gershgorin_bounds(H0), C.gershgorin_bounds(H1)
    for a, b in ((0.3, 0.7), (0.5, -1.2), (-0.2, 0.4), (0.0, -2.0)):
        lo, hi = C.weighted_bounds([b0, b1], [a, b])
        ev = np.linalg.eigvalsh((a * H0.to_scipy() + b * H1.to_scipy()).toarray())
        assert lo <= ev[0] + 1e-12 and ev[-1] <= hi + 1e-12 and lo <= hi


def _tail_bound(theta, K):
    x = abs(theta) / 2
    q = x / (K + 2)
    if q >= 1:
        return math.inf
    return 2 * x ** (K + 1) / math.factorial(K + 1) / (1 - q)


@pytest.mark.parametrize("theta", [0.01, 0.5, 3.0, -7.5, 20.0, 64.0])
@pytest.mark.parametrize("tol", [1e-4, 1e-10, 1e-15])
def test_truncation_rule(theta, tol):
    K = C.chebyshev_terms(theta, tol)
    assert _tail_bound(theta, K) <= tol * (1 + 1e-12)
    if K > 0:
        assert _tail_bound(theta, K - 1) > tol * (1 - 1e-12)
    ks = np.arange(K + 1, K + 200)
    assert 2 * np.sum(np.abs(ssp.jv(ks, theta))) <= tol
    assert C.chebyshev_terms(0.0, tol) == 0


def test_zero_width_interval_is_a_phase():
    H = I.diagonal(np.full(16, 3.0))
    rng = np.random.default_rng(2)
    psi = I.random_state(16, rng)
    lo, hi = C.gershgorin_bounds(H)
    out, K = C.chebyshev_expv(H, psi, 0.4, lo, hi, 1e-12, return_terms=True)
    assert K == 0 and np.allclose(out, np.exp(-1.2j) * psi, atol=1e-15, rtol=0)


@pytest.mark.parametrize("case", ["two_level", "ising5"])
def test_propagate_equals_exact_exponentials(case):
    if case == "two_level":
        H0, Hk, drives = I.two_level(2.0, 0.5, 1.0)
        psi0 = np.array([0.6, 0.8j])
        scheme, dt, N = "CF8:11", 0.2, 25
    else:
        rng = np.random.default_rng(5)
        H0 = I.ising_chain(5, 1.0, rng.uniform(-0.5, 0.5, 5))
        Hk = [I.sigma_x_sum(5)]
        drives = [{"kind": "cos", "A": 0.8, "omega": 2.0, "phi": 0.0}]
        psi0 = I.random_state(32, rng)
        scheme, dt, N = "CF6:5Opt", 0.05, 20
    tol = 1e-12
    st = {}
    out = C.propagate_chebyshev(H0, Hk, drives, psi0, 0.1, dt, N, scheme, tol, stats=st)
    ref = O.propagate(H0, Hk, drives, psi0, 0.1, dt, N, scheme, dense=True)
    nexp = len(st["terms"])
    assert nexp == N * {"CF8:11": 11, "CF6:5Opt": 5}[scheme]
    assert np.linalg.norm(out - ref) <= nexp * tol + 1e-13
    assert abs(np.linalg.norm(out) - np.linalg.norm(psi0)) <= nexp * tol + 1e-13
    assert st["n_matvec"] == sum(st["terms"])
