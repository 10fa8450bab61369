"""Pins for the oracle's CFET step loop (Secs. 4, 6, 7 and 11).

References: the closed-form propagator of the circularly driven two-level
system (Sec. 6.2, eq. TwoLevelU); its tensor product for non-interacting spins;
the Rosen-Zener transition probability (Sec. 11.1); an independent ODE solver
(scipy DOP853) for the convergence order N of every scheme; exactness for a
constant Hamiltonian; time reversibility of the symmetric schemes (Sec. 4.1,
rule R1); norm conservation; and the drive functions.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla
from scipy.integrate import solve_ivp

from oracle import cfet as O
from oracle import schemes as S
from paper_1102_5071_amd import inputs as I
from tests.closed_forms import two_level_U


def _H_of_t(H0, Hk, drives):
    H0 = H0.toarray()
    Hk = [h.toarray() for h in Hk]

    def H(t):
        M = H0.copy()
        for h, d in zip(Hk, drives):
            M = M + O.drive_value(d, t) * h
        return M
    return H


def _ode_reference(H, psi0, T):
    def rhs(t, y):
        return -1j * (H(t) @ y)
    sol = solve_ivp(rhs, (0.0, T), psi0.astype(complex), method="DOP853",
                    rtol=1e-13, atol=1e-14)
    return sol.y[:, -1]


def test_two_level_closed_form_against_ode():
    # the typed closed form itself is checked first against an ODE solve
    Delta, V, w = 0.5, 0.7, 1.0
    H0, Hk, drives = I.two_level(Delta, V, w)
    psi0 = np.array([0.6, 0.8j])
    T = 3.3
    ref = _ode_reference(_H_of_t(H0, Hk, drives), psi0, T)
    assert np.linalg.norm(two_level_U(T, Delta, V, w) @ psi0 - ref) < 1e-11


@pytest.mark.parametrize("name", list(S.SCHEMES))
def test_two_level_closed_form(name):
    Delta, V, w = 0.5, 0.5, 1.0
    H0, Hk, drives = I.two_level(Delta, V, w)
    psi0 = np.array([1.0, 0.0], dtype=complex)
    T = 2 * math.pi / w
    order = S.scheme(name).order
    nsteps = {2: 4000, 4: 400, 6: 120, 8: 80}[order]
    dt = T / nsteps
    out_dense = O.propagate(H0, Hk, drives, psi0, 0.0, dt, nsteps, name, dense=True)
    out_kry = O.propagate(H0, Hk, drives, psi0, 0.0, dt, nsteps, name, m=2)
    exact = two_level_U(T, Delta, V, w) @ psi0
    assert np.linalg.norm(out_dense - exact) < 2e-6
    # dim 2: two Lanczos vectors span everything, Krylov == dense
    assert np.linalg.norm(out_kry - out_dense) < 1e-12


def _random_problem(seed, n=6):
    rng = np.random.default_rng(seed)
    H0 = I.random_hermitian(n, rng, scale=0.8)
    H1 = I.random_hermitian(n, rng, scale=0.8)
    drives = [{"kind": "cos", "A": 1.5, "omega": 2.0, "phi": 0.3}]
    psi0 = I.random_state(n, rng)
    return H0, [H1], drives, psi0


@pytest.mark.parametrize("name", list(S.SCHEMES))
def test_global_convergence_order(name):
    # Sec. 6.1: the global error of an N-th order CFET scales as dt^N
    H0, Hk, drives, psi0 = _random_problem(11)
    T = 1.0
    ref = _ode_reference(_H_of_t(H0, Hk, drives), psi0, T)
    order = S.scheme(name).order
    n1 = {2: 32, 4: 8, 6: 4, 8: 3}[order]
    errs = []
    for n in (n1, 2 * n1):
        out = O.propagate(H0, Hk, drives, psi0, 0.0, T / n, n, name, dense=True)
        errs.append(np.linalg.norm(out - ref))
    slope = math.log2(errs[0] / errs[1])
    assert errs[1] > 1e-12, "error hit the reference floor; enlarge dt"
    # optimised schemes have small leading constants, so the pre-asymptotic
    # slope may exceed N a little; a lost order gives a slope near N - 1 or less
    assert order - 0.5 < slope < order + 1.2, (name, errs, slope)


def test_reversed_exponential_order_loses_order():
    # Sec. 4, eq. Ucf: exp(Omega_s) acts first.  Applying exp(Omega_1) first is
    # a plausible mistake; it must show up as a lost order.
    H0, Hk, drives, psi0 = _random_problem(11)
    T = 1.0
    ref = _ode_reference(_H_of_t(H0, Hk, drives), psi0, T)
    sc = S.scheme("CF4:2")
    x, g = S.gl_weights(sc)
    H0d, H1d = H0.toarray(), Hk[0].toarray()
    errs = []
    for n in (16, 32):
        dt = T / n
        psi = psi0.copy()
        for k in range(n):
            t = k * dt
            for i in range(sc.s):          # wrong order: Omega_1 first
                b = sum(g[i, m] * O.drive_value(drives[0], t + x[m] * dt) for m in range(sc.M))
                psi = sla.expm(-1j * dt * (g[i].sum() * H0d + b * H1d)) @ psi
        errs.append(np.linalg.norm(psi - ref))
    assert math.log2(errs[0] / errs[1]) < 2.6


@pytest.mark.parametrize("name", ["CF4:2", "CF6:5Opt", "CF8:11"])
def test_constant_hamiltonian_is_exact(name):
    # with f constant, every step is exp(-i dt H) because sum_i f_{i,1} = 1
    H0, Hk, _, psi0 = _random_problem(3)
    drives = [{"kind": "cos", "A": 0.7, "omega": 0.0, "phi": 0.0}]
    dt, n = 0.3, 5
    out = O.propagate(H0, Hk, drives, psi0, 0.0, dt, n, name, dense=True)
    H = H0.toarray() + 0.7 * Hk[0].toarray()
    ref = sla.expm(-1j * dt * n * H) @ psi0
    assert np.linalg.norm(out - ref) < 1e-13


@pytest.mark.parametrize("name", ["CF4:2", "CF4:3Opt", "CF6:5Opt", "CF6:6Opt", "CF8:11"])
def test_time_reversibility(name):
    # rule R1 (Sec. 4.1): a step dt from t followed by a step -dt from t+dt
    # returns the initial state
    H0, Hk, drives, psi0 = _random_problem(5)
    dt = 0.37
    fwd = O.propagate(H0, Hk, drives, psi0, 0.2, dt, 1, name, dense=True)
    back = O.propagate(H0, Hk, drives, fwd, 0.2 + dt, -dt, 1, name, dense=True)
    assert np.linalg.norm(back - psi0) < 1e-13


def test_norm_conservation_krylov():
    rng = np.random.default_rng(4)
    n = 120
    H0 = I.random_hermitian(n, rng, density=0.05)
    H1 = I.random_hermitian(n, rng, density=0.05)
    drives = [{"kind": "cos", "A": 1.0, "omega": 1.3, "phi": 0.0}]
    psi0 = I.random_state(n, rng)
    out = O.propagate(H0, [H1], drives, psi0, 0.0, 0.05, 200, "CF6:5Opt", m=8)
    assert abs(np.linalg.norm(out) - 1.0) < 1e-12


def test_restart_equals_continuous_run():
    H0, Hk, drives, psi0 = _random_problem(8, n=10)
    dt, n = 0.05, 20
    full = O.propagate(H0, Hk, drives, psi0, 0.0, dt, 2 * n, "CF6:5Opt", m=6)
    half = O.propagate(H0, Hk, drives, psi0, 0.0, dt, n, "CF6:5Opt", m=6)
    rest = O.propagate(H0, Hk, drives, half, n * dt, dt, n, "CF6:5Opt", m=6)
    assert np.linalg.norm(full - rest) < 1e-13


def test_noninteracting_spins_tensor_product():
    L, Delta, V, w = 3, 0.4, 0.6, 0.9
    H0, Hk, drives = I.noninteracting_spins(L, Delta, V, w)
    rng = np.random.default_rng(2)
    sites = [I.random_state(2, rng) for _ in range(L)]
    psi0 = I.product_state(sites)
    T = 2.0
    out = O.propagate(H0, Hk, drives, psi0, 0.0, T / 40, 40, "CF6:5Opt", m=8)
    U = two_level_U(T, Delta, V, w)
    exact = I.product_state([U @ s for s in sites])
    assert np.linalg.norm(out - exact) < 1e-8


def test_rosen_zener_transition_probability():
    # Sec. 11.1, eq. BPulse: V(t) = V e^{-2iwt}/cosh(t/tau); P_inf closed form
    Delta, w, tau, V = 1.0, 0.9, 1.0, 0.3
    H0 = I.diagonal([Delta, -Delta])
    _, Hk, _ = I.two_level(Delta, V, w)
    drives = [{"kind": "sechcos", "A": V, "omega": 2 * w, "phi": 0.0, "tc": 0.0, "tau": tau},
              {"kind": "sechcos", "A": V, "omega": 2 * w, "phi": -math.pi / 2, "tc": 0.0,
               "tau": tau}]
    psi0 = np.array([0.0, 1.0], dtype=complex)     # spin down
    t0, t1 = -30.0 * tau, 30.0 * tau
    n = 3000
    out = O.propagate(H0, Hk, drives, psi0, t0, (t1 - t0) / n, n, "CF6:5Opt", m=2)
    P = abs(out[0]) ** 2
    P_exact = math.sin(math.pi * V * tau) ** 2 / math.cosh(math.pi * (Delta - w) * tau) ** 2
    assert abs(P - P_exact) < 1e-9


def test_drive_functions():
    assert O.drive_value({"kind": "cos", "A": 2.0, "omega": 3.0, "phi": 0.5}, 0.7) == \
        pytest.approx(2.0 * math.cos(2.6))
    d = {"kind": "sin2cos", "A": 0.05, "omega": 0.5, "phi": 0.0, "Tp": 200.0}
    assert O.drive_value(d, 100.0) == pytest.approx(0.05 * math.cos(50.0))
    assert O.drive_value(d, -1.0) == 0.0 and O.drive_value(d, 200.5) == 0.0
    p = {"kind": "pwc", "t_edges": [0.0, 0.1, 0.2], "u": [3.0, -1.0]}
    assert O.drive_value(p, 0.0) == 3.0
    assert O.drive_value(p, 0.1) == -1.0
    assert O.drive_value(p, 0.2) == 0.0 and O.drive_value(p, -0.01) == 0.0
    s = {"kind": "sechcos", "A": 1.0, "omega": 0.0, "phi": 0.0, "tc": 1.0, "tau": 2.0}
    assert O.drive_value(s, 3.0) == pytest.approx(1.0 / math.cosh(1.0))


def test_piecewise_constant_drive_step_aligned():
    # a step that lies inside one piece sees a constant H: exp(-i dt H(u_k))
    H0, Hk, _, psi0 = _random_problem(6)
    drives = [{"kind": "pwc", "t_edges": [0.0, 0.5, 1.0], "u": [0.4, -0.9]}]
    dt = 0.25
    out = O.propagate(H0, Hk, drives, psi0, 0.0, dt, 4, "CF6:5Opt", dense=True)
    Ha = H0.toarray() + 0.4 * Hk[0].toarray()
    Hb = H0.toarray() - 0.9 * Hk[0].toarray()
    ref = sla.expm(-0.5j * Hb) @ (sla.expm(-0.5j * Ha) @ psi0)
    assert np.linalg.norm(out - ref) < 1e-13


def test_apply_rows_matches_sparse_product():
    # spot rows of y = a H0 x + b1 H1 x + b2 H2 x against scipy's whole product,
    # on a ragged random operator (empty rows included) and a spin chain
    rng = np.random.default_rng(21)
    H0 = I.random_hermitian(90, rng, density=0.05)
    H1 = I.random_hermitian(90, rng, density=0.1)
    H2 = I.diagonal(rng.standard_normal(90))
    x = I.random_state(90, rng)
    a, b = -0.7, [1.3, 0.25]
    full = a * (H0.to_scipy() @ x) + b[0] * (H1.to_scipy() @ x) + b[1] * (H2.to_scipy() @ x)
    rows = [0, 5, 44, 89] + list(rng.choice(90, 10, replace=False))
    got = O.apply_rows(H0, [H1, H2], a, b, x, rows)
    assert np.allclose(got, full[rows], rtol=1e-14, atol=1e-14)
    p = I.config_heisenberg(L=8)
    x = I.random_state(p.dim, rng)
    full = 0.4 * (p.H0.to_scipy() @ x) - 2.0 * (p.Hk[0].to_scipy() @ x)
    rows = list(range(0, p.dim, 17))
    assert np.allclose(O.apply_rows(p.H0, p.Hk, 0.4, [-2.0], x, rows), full[rows],
                       rtol=1e-14, atol=1e-14)
