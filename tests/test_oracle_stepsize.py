"""Pins of the oracle's time-step selection (oracle.stepsize, Sec. 6.6) and of
the order comparison (Sec. 6.5, eq. ErrOrder).

* The paper's printed accuracy windows (tests/golden/order_windows.txt) follow
  from eq. ErrOrder with cbar = s.
* An exactly modelled error x(t) = exact(t) + c (t - t0) dt^N v: the two-run
  estimate must return c to rounding, the selected step must satisfy
  c T dt^N <= eps with equality before rounding to whole steps, and the
  verification run must reproduce c T dt^N (a dropped factor, a wrong power or
  swapped steps all break these).
* The circularly driven two-level system, whose exact propagator is
  eq. TwoLevelU (Sec. 6.2; omega = 1, Delta = 2, V = 0.5 as in the paper's
  error-effort plot, T = 5 pi): the step chosen for eps from two probe runs on
  the first fifth of the time gives a true error (max over the run, against
  the closed form) of at most eps and at least eps / 10, for orders 4, 6 and 8
  and eps from 1e-6 to 1e-10; the verification estimate is within a factor 4
  of the true error; and cbar = s c^(1/N) of the estimated c agrees with the
  measured (s / dt) (eps / T)^(1/N) (Sec. 6.3) within the accuracy of c.
* Refinement from the verification pair (a reading, not in the paper): on a
  modelled error that saturates above a step a, the plain procedure misses
  the goal and its verification says so; refinement meets it.
"""
import math
import os

import numpy as np
import pytest

from oracle import cfet as O
from oracle import schemes as S
from oracle import stepsize as SS
from paper_1102_5071_amd import inputs as I
from tests.closed_forms import two_level_U

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _windows():
    rows = []
    with open(os.path.join(GOLDEN, "order_windows.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                a, b, s1, s2, v = line.split()
                rows.append((int(a), int(b), float(s1), float(s2), float(v)))
    return rows


def test_order_windows_printed_in_the_paper():
    rows = _windows()
    assert len(rows) == 3
    for N1, N2, s1, s2, printed in rows:
        x = (s1 / s2) ** (N1 * N2 / (N2 - N1))
        assert float(f"{x:.0e}") == printed, (N1, N2, x)
        assert SS.lower_order_preferred(s1, N1, s2, N2, 1.01 * x, 1.0)
        assert not SS.lower_order_preferred(s1, N1, s2, N2, 0.99 * x, 1.0)
        # the same crossing from the efforts s T / dt of eq. BarC
        c1, c2 = (s1 / s1) ** N1, (s2 / s2) ** N2    # cbar = s c^(1/N) with c = 1
        for eps in (0.5 * x, 2.0 * x):
            e1 = s1 * (c1 / eps) ** (1 / N1)
            e2 = s2 * (c2 / eps) ** (1 / N2)
            assert (e1 <= e2) == SS.lower_order_preferred(s1, N1, s2, N2, eps, 1.0)
    with pytest.raises(ValueError):
        SS.lower_order_preferred(1.0, 6, 1.0, 4, 1e-6, 1.0)


def test_effective_constant_of_eq_barc():
    # s N_s = s T / dt at the step dt = (eps / (c T))^(1/N) equals
    # cbar T^(1 + 1/N) eps^(-1/N)
    for s, N, c in ((2, 4, 3e-3), (5, 6, 7e-5), (11, 8, 2e-6)):
        T, eps = 7.0, 1e-9
        dt = SS.step_for(eps, c, T, N)
        cbar = SS.effective_error_constant(c, s, N)
        assert abs(s * T / dt - cbar * T ** (1 + 1 / N) * eps ** (-1 / N)) <= 1e-12 * s * T / dt


def _model_run(c, N, w, u, v, t0):
    # x(t) = e^{-i w t} (u + c (t - t0) dt^N v): the error grows linearly in t
    def run(psi, t, dt, nsteps):
        tau = nsteps * dt
        return np.exp(-1j * w * tau) * psi + c * tau * dt ** N * np.exp(-1j * w * (t + tau)) * v
    return run


@pytest.mark.parametrize("N,J", [(4, 1), (6, 3), (8, 5)])
def test_exact_error_model(N, J):
    rng = np.random.default_rng(N)
    u = I.random_state(8, rng)
    v = I.random_state(8, rng)
    w, t0, W, T = 0.9, 0.25, 1.5, 12.0
    # distances of about 1e-5 between the probes (far above rounding), and a
    # goal that asks for about a third of the probe step
    c = 1e-5 / (W * (W / (10 * J)) ** N)
    eps = 0.97 * c * T * (W / (30 * J)) ** N
    x0 = np.exp(-1j * w * t0) * u
    run = _model_run(c, N, w, u, v, t0)
    r = SS.select_dt_from_runs(run, N, x0, t0, W, 10 * J, T, eps, J=J)
    assert r["n1"] == 10 * J and r["n2"] % J == 0 and r["n2"] > r["n1"]
    assert 2.0 <= (r["n2"] / r["n1"]) ** N <= 3.2
    # rounding of states of norm 1 limits the distance to about 1e-16
    den = W * abs(r["dt1"] ** N - r["dt2"] ** N)
    assert abs(r["c"] - c) <= 1e-9 * c + 1e-15 / den
    dt_raw = (eps / (c * T)) ** (1 / N)
    assert r["dt"] <= dt_raw * (1 + 1e-12)
    assert r["nsteps"] == math.ceil(T / dt_raw * (1 - 1e-12))
    assert abs(r["dt"] * r["nsteps"] - T) <= 1e-12 * T
    assert r["err_est"] <= eps * (1 + 1e-9)
    assert abs(r["err_check"] - c * T * r["dt"] ** N) <= 1e-4 * r["err_check"]


def test_refinement_recovers_from_a_probe_outside_the_asymptotic_range():
    # error c (t - t0) g(dt) with g = dt^N / (1 + (dt / a)^(N - 2)): dt^N below
    # a, only dt^2 above it.  Probes far above a see a much smaller difference
    # than the dt^N law implies, so the first c is far too small; the
    # verification pair (at the extrapolated step) exposes it, and refinement
    # brings the step below a, where the law holds.
    N, a, c, w, t0 = 6, 0.05, 2e-3, 0.7, 0.0
    W, T, eps = 4.0, 10.0, 1e-12
    rng = np.random.default_rng(17)
    u, v = I.random_state(4, rng), I.random_state(4, rng)

    def g(dt):
        return dt ** N / (1.0 + (dt / a) ** (N - 2))

    def run(psi, t, dt, nsteps):
        tau = nsteps * dt
        return np.exp(-1j * w * tau) * psi + c * tau * g(dt) * np.exp(-1j * w * (t + tau)) * v

    plain = SS.select_dt_from_runs(run, N, u, t0, W, 8, T, eps)
    assert plain["rounds"] == 0 and plain["err_check"] > 10 * eps
    r = SS.select_dt_from_runs(run, N, u, t0, W, 8, T, eps, refine=6)
    assert 1 <= r["rounds"] <= 4
    assert r["err_check"] <= eps
    assert r["dt"] < plain["dt"]
    assert c * T * g(r["dt"]) <= 1.1 * eps                 # the model's own error
    with pytest.raises(ValueError):
        SS.select_dt_from_runs(run, N, u, t0, W, 8, T, eps, verify=False, refine=1)


def test_exact_propagator_gives_the_whole_time_in_one_step():
    # f = 0, diagonal H0: every CFET step is exact (the weights of H0 sum to
    # one), the probes agree to rounding and the cap dt <= T applies
    rng = np.random.default_rng(3)
    H0 = I.diagonal(rng.uniform(-1, 1, 16))
    H1 = I.sigma_x_sum(4)
    drives = [{"kind": "cos", "A": 0.0, "omega": 1.0, "phi": 0.0}]
    r = SS.select_dt(H0, [H1], drives, I.random_state(16, rng), 0.0, 0.5, 4, "CF4:2", 8,
                     3.0, 1e-8, dense=True)
    assert r["diff"] <= 1e-14
    assert r["nsteps"] == 1 and r["dt"] == 3.0


def test_probe_step_counts():
    assert SS.probe_steps(20, 2.5, 6, 4) == 24
    assert SS.probe_steps(4, 2.5, 8, 4) == 8         # at least one more checkpoint block
    for N in (2, 4, 6, 8):
        n2 = SS.probe_steps(100, 2.5, N)
        assert 2.3 <= (n2 / 100) ** N <= 2.7
    with pytest.raises(ValueError):
        SS.probe_steps(10, 2.5, 4, 3)
    with pytest.raises(ValueError):
        SS.error_constant(1e-8, 1.0, 0.1, 0.1, 4)


DELTA, V, W_DRIVE = 2.0, 0.5, 1.0


def _true_error(scheme, dt, n, phi, K=10):
    H0, Hk, dr = I.two_level(DELTA, V, W_DRIVE)
    x, done, emax = phi.copy(), 0, 0.0
    for k in range(1, K + 1):
        tgt = (n * k) // K
        x = O.propagate(H0, Hk, dr, x, done * dt, dt, tgt - done, scheme, dense=True)
        done = tgt
        emax = max(emax, np.linalg.norm(x - two_level_U(done * dt, DELTA, V, W_DRIVE) @ phi))
    return emax


@pytest.mark.parametrize("scheme", ["CF4:3Opt", "CF6:5Opt", "CF8:11"])
@pytest.mark.parametrize("eps", [1e-6, 1e-8, 1e-10])
def test_two_level_selected_step_meets_goal(scheme, eps):
    H0, Hk, dr = I.two_level(DELTA, V, W_DRIVE)
    phi = np.array([1.0, 0.0], dtype=complex)
    T = 5 * math.pi / W_DRIVE
    r = SS.select_dt(H0, Hk, dr, phi, 0.0, T / 5, 20, scheme, 2, T, eps, J=4, dense=True)
    assert r["rounds"] == 0
    sc = S.scheme(scheme)
    assert r["order"] == sc.order
    err = _true_error(scheme, r["dt"], r["nsteps"], phi)
    assert eps / 10 <= err <= eps, (err, eps)
    assert err / 4 <= r["err_check"] <= 4 * err
    # eq. BarC against the measured effective constant (Sec. 6.3's definition)
    cbar_meas = (sc.s / r["dt"]) * (err / T) ** (1 / sc.order)
    cbar_est = SS.effective_error_constant(r["c"], sc.s, sc.order)
    assert cbar_meas <= cbar_est <= 1.35 * cbar_meas
