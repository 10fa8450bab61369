"""Write the stored expected states of the large parity tests.

Every value written here comes from the CPU oracle (``oracle/``) run on the
seeded inputs of ``paper_1102_5071_amd/inputs.py``; nothing is read from the
HIP library.  Usage (from the repository root):

    python tests/golden/make_goldens.py heisenberg --L 18 --steps 200
    python tests/golden/make_goldens.py heisenberg --L 24 --steps 2
    python tests/golden/make_goldens.py heisenberg --L 24 --steps 1 --dt-window 4 --dt-steps 19
    python tests/golden/make_goldens.py hydrogen

Heisenberg chain (disordered, J = 1, h_i ~ U[-1, 1] from seed 0, H1 = sum sx,
f = 0.5 sin 1.3t, random product state, CF6:5Opt, dt = 0.02, m = 24; the
spin-chain workload of Sec. 11.1 at the dimensions of the at-scale
configuration): up to L = 18 the whole final state is stored; above, the
entries at seeded sample rows (with the slice and half-space edges), the norm
and the projections onto seeded complex Gaussian vectors (which involve every
entry), so the file stays small.  With --dt-window T --dt-steps N the step
is T / N instead of 0.02 (the benchmark runs the step selected for a state
error of 1e-8 over T = 4: 4 / 19) and the file name carries the step.

Hydrogen (radial grid Nr = 2000, dr = 0.1, l <= 63, CF8:11, m = 30, 1s start):
the 30 steps of dt = 0.002 from t0 = 40 that the hydrogen benchmark runs
(10 warm-up steps, then 20 timed).

The oracle forms a_i H0 + b_i H1 for every exponential (one sparse matrix of
612 M entries at L = 24); L = 24 needs about 45 GB of host memory and about
15 minutes on one core.
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import cfet as O  # noqa: E402
from paper_1102_5071_amd import inputs as I  # noqa: E402

FULL_STATE_MAX_L = 18
SAMPLE_SEED = 20240
NPROJ = 4


def sample_rows(n: int) -> np.ndarray:
    """Seeded sample rows plus the edges of 64-row slices, of the two halves
    and of the four quarters of the index space."""
    rng = np.random.default_rng(SAMPLE_SEED)
    k = min(n, 4096)
    rows = set(int(r) for r in rng.choice(n, size=k, replace=False))
    for e in (0, n // 4, n // 2, 3 * n // 4, n):
        for d in range(-65, 66):
            if 0 <= e + d < n:
                rows.add(e + d)
    return np.array(sorted(rows), dtype=np.int64)


def projection_vectors(n: int):
    """Seeded complex Gaussian vectors r_k (not normalised); the tests compare
    <r_k|psi> = sum_j conj(r_k[j]) psi[j]."""
    rng = np.random.default_rng(SAMPLE_SEED + 1)
    for _ in range(NPROJ):
        yield rng.standard_normal(n) + 1j * rng.standard_normal(n)


def golden_path(name: str) -> str:
    return os.path.join(HERE, name)


def heisenberg(L: int, steps: int, dt: float | None = None) -> str:
    p = I.config_heisenberg(L=L, nsteps=steps)
    if dt is not None:
        p.dt = dt
    n = p.dim
    H0 = p.H0.to_scipy()
    H1 = p.Hk[0].to_scipy()
    psi0 = p.psi0
    del p.H0, p.Hk
    t = time.time()
    stats = {}
    psi = O.propagate(H0, [H1], p.drives, psi0, 0.0, p.dt, steps, p.scheme, m=p.m, stats=stats)
    el = time.time() - t
    out = {"L": L, "steps": steps, "dt": p.dt, "m": p.m, "scheme": p.scheme, "t0": 0.0,
           "norm": np.linalg.norm(psi), "n_matvec": stats["n_matvec"],
           "min_m_eff": min(stats["m_eff"]), "oracle_seconds": el}
    if L <= FULL_STATE_MAX_L:
        out["psi"] = psi
    else:
        rows = sample_rows(n)
        out["rows"] = rows
        out["psi_rows"] = psi[rows]
        out["proj"] = np.array([np.vdot(r, psi) for r in projection_vectors(n)])
    tag = "" if dt is None else f"_dt{dt:.6f}"
    path = golden_path(f"heisenberg_L{L}_{steps}steps{tag}.npz")
    np.savez(path, **out)
    print(f"heisenberg L={L}: {steps} steps in {el:.0f} s, |psi| = {out['norm']:.15f}, "
          f"matvecs {stats['n_matvec']} -> {path}", flush=True)
    return path


def hydrogen() -> str:
    p = I.config_hydrogen()
    t0, dt, steps = 40.0, 0.002, 30
    t = time.time()
    stats = {}
    psi = O.propagate(p.H0, p.Hk, p.drives, p.psi0, t0, dt, steps, p.scheme, m=p.m, stats=stats)
    el = time.time() - t
    path = golden_path("hydrogen_t40_dt0.002_30steps.npz")
    np.savez(path, psi=psi, t0=t0, dt=dt, steps=steps, m=p.m, scheme=p.scheme,
             n_matvec=stats["n_matvec"], oracle_seconds=el)
    print(f"hydrogen: {steps} steps in {el:.0f} s -> {path}", flush=True)
    return path


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("which", choices=["heisenberg", "hydrogen"])
    ap.add_argument("--L", type=int, default=18)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--dt-window", type=float, default=0.0)
    ap.add_argument("--dt-steps", type=int, default=0)
    a = ap.parse_args()
    if a.which == "heisenberg":
        dt = a.dt_window / a.dt_steps if a.dt_steps > 0 else None
        heisenberg(a.L, a.steps, dt)
    else:
        hydrogen()


if __name__ == "__main__":
    main()
