"""Time-step selection and error tracking for CFET runs (oracle).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: imported by tests,
``__graft_entry__.smoke()`` and ``bench.py``'s CPU baseline, never by the
product path, and sharing no code with the HIP library.

What the paper fixes (Sec. 6.6 on time-step selection; Sec. 6.1, eq. BarC;
Sec. 6.5, eq. ErrOrder):

* the global error of an order-N CFET over a time T scales as eps = c T dt^N
  (Sec. 6.1);
* two runs with steps dt1 != dt2 over the same time give the constant c from
  the largest distance between their states,
      max_t ||x1(t) - x2(t)|| = c T |dt1^N - dt2^N|,
  without the exact solution; a ratio (dt1/dt2)^N of 2 to 3 is recommended;
* from c the step for an accuracy goal eps follows, dt = (eps / (c T))^(1/N),
  and one more run at a smaller step gives a reliable estimate of the error;
* the effective error constant of a scheme with s exponentials is
  cbar = s c^(1/N) (eq. BarC; measured as (s / dt) (eps / T)^(1/N), Sec. 6.3); of two
  orders N1 < N2 the lower one needs fewer exponentials for a goal eps over T
  when (cbar1 / cbar2)^(N1 N2 / (N2 - N1)) <= eps / T (eq. ErrOrder).

Readings where the paper leaves a choice (each one a parameter here):
* "max over t" is taken over J checkpoints t0 + j W / J (j = 1..J) of a probe
  window of length W, which both step grids hit: the probe step counts are
  n1 and n2 = J round((n1 / J) ratio^(1/N)), both multiples of J, n2 > n1;
* T in the relation for c is the window length W (the error grows with the
  time propagated, so its maximum over the window is reached near its end);
* the selected step is capped at the total time T_total and rounded down so
  that T_total is a whole number of steps;
* the additional run (the paper's recommendation) propagates the window,
  stretched to W' = a whole number of selected steps (a multiple of J), with
  the selected step dt and with dt' of the same ratio (again on J
  checkpoints) and scales their largest distance d to the error of dt over
  the total time:  err(dt) = d dt^N / (dt^N - dt'^N) * T_total / W';
* refinement (optional, `refine` rounds at most): when that estimate exceeds
  eps, the verification pair becomes the probe -- c from d and W' by the same
  relation, a new dt, a new verification -- until the estimate meets eps.
  This guards against probes taken outside the asymptotic range of dt^N
  (the distance of the probes then underestimates c); the step only shrinks.
"""
from __future__ import annotations

import math

import numpy as np

from .cfet import propagate
from .schemes import scheme as get_scheme

__all__ = ["error_constant", "step_for", "effective_error_constant",
           "lower_order_preferred", "probe_steps", "select_dt_from_runs", "select_dt"]


def error_constant(max_diff: float, W: float, dt1: float, dt2: float, N: int) -> float:
    """c from max_t ||x1 - x2|| = c W |dt1^N - dt2^N| (Sec. 6.6)."""
    den = W * abs(dt1 ** N - dt2 ** N)
    if den <= 0.0:
        raise ValueError("the two probe steps must differ and W must be positive")
    return max_diff / den


def step_for(eps: float, c: float, T: float, N: int) -> float:
    """dt with c T dt^N = eps (infinite for c = 0)."""
    if c <= 0.0:
        return math.inf
    return (eps / (c * T)) ** (1.0 / N)


def effective_error_constant(c: float, s: int, N: int) -> float:
    """cbar = (s / dt) (eps / T)^(1/N) with eps = c T dt^N, i.e. s c^(1/N)."""
    return s * c ** (1.0 / N)


def lower_order_preferred(cbar1: float, N1: int, cbar2: float, N2: int, eps: float,
                          T: float) -> bool:
    """eq. ErrOrder: the order-N1 scheme (N1 < N2) needs no more exponentials
    than the order-N2 one for the goal eps over T."""
    if not N1 < N2:
        raise ValueError("N1 < N2")
    return (cbar1 / cbar2) ** (N1 * N2 / (N2 - N1)) <= eps / T


def probe_steps(n1: int, ratio: float, N: int, J: int = 1) -> int:
    """n2 = J round((n1 / J) ratio^(1/N)), at least n1 + J."""
    if n1 <= 0 or J <= 0 or n1 % J:
        raise ValueError("n1 must be a positive multiple of J")
    n2 = J * int(round((n1 // J) * ratio ** (1.0 / N)))
    return max(n2, n1 + J)


def _max_distance(run, psi0, t0: float, W: float, n_a: int, n_b: int, J: int) -> float:
    """Largest ||x_a - x_b|| over the J checkpoints of two runs of the window
    with n_a and n_b steps."""
    xa = np.array(psi0, dtype=np.complex128, copy=True)
    xb = xa.copy()
    dta, dtb = W / n_a, W / n_b
    d = 0.0
    for j in range(J):
        xa = run(xa, t0 + j * (n_a // J) * dta, dta, n_a // J)
        xb = run(xb, t0 + j * (n_b // J) * dtb, dtb, n_b // J)
        d = max(d, float(np.linalg.norm(xa - xb)))
    return d


def _whole_steps(c: float, eps: float, T_total: float, N: int):
    """(dt, nsteps): the step for eps, capped at T_total, rounded down to
    T_total / nsteps."""
    dt_raw = min(step_for(eps, c, T_total, N), T_total)
    nsteps = max(1, math.ceil(T_total / dt_raw * (1.0 - 1e-12)))
    return T_total / nsteps, nsteps


def select_dt_from_runs(run, N: int, psi0, t0: float, W: float, n1: int, T_total: float,
                        eps: float, ratio: float = 2.5, J: int = 1, verify: bool = True,
                        refine: int = 0) -> dict:
    """The procedure of Sec. 6.6 for any propagator run(psi, t, dt, nsteps) -> psi
    of order N: probe the window [t0, t0 + W] with n1 and n2 steps, estimate c,
    extrapolate the step for eps over T_total, optionally check it with one
    more pair of runs (and refine from that pair up to `refine` times)."""
    if not (W > 0 and T_total > 0 and eps > 0 and ratio > 1) or refine < 0:
        raise ValueError("W, T_total, eps must be positive, ratio > 1, refine >= 0")
    if refine and not verify:
        raise ValueError("refinement needs the verification runs")
    n2 = probe_steps(n1, ratio, N, J)
    dt1, dt2 = W / n1, W / n2
    diff = _max_distance(run, psi0, t0, W, n1, n2, J)
    c = error_constant(diff, W, dt1, dt2, N)
    dt, nsteps = _whole_steps(c, eps, T_total, N)
    out = {"dt": dt, "nsteps": nsteps, "c": c, "order": N, "n1": n1, "n2": n2,
           "dt1": dt1, "dt2": dt2, "diff": diff, "err_est": c * T_total * dt ** N,
           "err_check": None, "rounds": 0}
    rounds = 0
    while verify:
        # the window stretched to whole steps of dt (J checkpoints), run with dt
        # and with the smaller step of the same ratio
        na = J * max(1, math.ceil(W / (J * dt) * (1.0 - 1e-12)))
        Wc = na * dt
        nb = probe_steps(na, ratio, N, J)
        d = _max_distance(run, psi0, t0, Wc, na, nb, J)
        db = Wc / nb
        err_check = d * dt ** N / (dt ** N - db ** N) * T_total / Wc
        out.update(dt=dt, nsteps=nsteps, c=c, err_est=c * T_total * dt ** N, rounds=rounds,
                   check_window=Wc, check_steps=(na, nb), check_diff=d, err_check=err_check)
        if err_check <= eps or rounds >= refine:
            break
        rounds += 1
        c = error_constant(d, Wc, dt, db, N)
        dt, nsteps = _whole_steps(c, eps, T_total, N)
    return out


def select_dt(H0, Hk, drives, psi0, t0: float, W: float, n1: int, scheme_name: str, m: int,
              T_total: float, eps: float, ratio: float = 2.5, J: int = 1, verify: bool = True,
              dense: bool = False, refine: int = 0) -> dict:
    """select_dt_from_runs with the oracle's CFET propagator (Lanczos with m
    vectors, or exact exponentials with dense=True)."""
    sc = get_scheme(scheme_name)

    def run(psi, t, dt, nsteps):
        return propagate(H0, Hk, drives, psi, t, dt, nsteps, scheme_name, m=m, dense=dense)

    return select_dt_from_runs(run, sc.order, psi0, t0, W, n1, T_total, eps, ratio, J, verify,
                               refine)
