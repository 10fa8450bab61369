#!/usr/bin/env python3
"""Benchmark: CFET steps/s on one MI355X, with roofline and CPU-oracle baseline.

Default workload: disordered Heisenberg chain of L = 24 spins (dim 2^24 =
16 777 216, complex128; J = 1, h_i ~ U[-1, 1], H1 = sum sx with
f(t) = 0.5 sin(1.3 t), random product state), CF6:5Opt, dt = 0.02, Lanczos
m = 24 -- the spin-chain workload of the paper's Sec. 11.1 at the largest
size one GPU holds.  A "step" is one CFET step: 5 exponentials, each 24
Lanczos iterations (SpMV + reductions), the small tridiagonal exponential and
the recombination -- the whole path, on inputs already resident in HBM.

The time step is chosen for the accuracy goal (default 1e-8 over the
workload's time span) by the library's two-run selection (cfet_select_dt,
Sec. 6.6) on a probe window, unless --dt fixes it; the choice, its estimated
error constant and its verification estimate are reported.  The state error
over the timed window is measured against a run at dt/4 with m = 40 and
reported with the window length.  Other workloads:
--workload hydrogen | ising | batched | adjoint.

Prints ONE JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PROFILES = os.path.join(ROOT, "profiles")
DEFAULT_CHUNK = {"hydrogen": 10, "ising": 50, "heisenberg": 1, "batched": 0, "adjoint": 0}
# (timed steps, warm-up steps) when not given on the command line; the plain
# workloads time the selected number of steps instead (unless --dt fixes dt)
DEFAULT_STEPS = {"hydrogen": (200, 20), "ising": (1000, 100), "heisenberg": (20, 2),
                 "batched": (200, 20), "adjoint": (200, 20)}
# the roofline each plain workload's dominant kernel is measured against: the
# Heisenberg chain's SpMV streams its vectors and layout from HBM (1.7 GB of
# counted traffic per SpMV on the split layout, 13 GB in complex-CSR terms;
# its first pass runs below that ceiling, held by per-slice latency chains);
# the hydrogen and Ising operators and Krylov bases stay in the caches and
# their persistent kernels wait on grid-wide round trips
BOUND = {"heisenberg": "hbm", "hydrogen": "latency", "ising": "latency"}
# step selection per plain workload: (probe window start, probe window length,
# probe steps n1, time span T the accuracy goal refers to).  The probe steps
# are a few times the selected ones, so the distance of the two probe runs
# (1e-11 .. 1e-6) stands well above rounding; the spans: the table's 200 steps
# of 0.02 (Heisenberg), 1000 of 0.01 (Ising), and for hydrogen a window of 0.4
# inside the pulse.  Without --steps the timed run covers the span: the
# selected number of steps.
SELECT = {"heisenberg": (0.0, 1.0, 8, 4.0), "ising": (0.0, 0.8, 8, 10.0),
          "hydrogen": (40.0, 0.4, 40, 0.4)}
# refinement rounds from the verification pair when its estimate misses the goal
SELECT_REFINE = 4


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def spmv_algorithmic_bytes(dim, nnz_total, ncsr):
    """Bytes one weighted SpMV must move: each stored non-zero once (16 B value
    + 4 B column), the row pointers of every CSR once, x read once and y
    written once."""
    return 20 * nnz_total + 8 * (dim + 1) * ncsr + 32 * dim


def exponential_algorithmic_bytes(dim, nnz_total, ncsr, m):
    """One Lanczos exponential: m SpMVs, m-1 three-term updates with norm
    (read y, v_j, v_{j-1}, write w: 64 B per row) and the recombination
    (read m basis vectors, write psi: (m+1)*16 B per row)."""
    return (m * spmv_algorithmic_bytes(dim, nnz_total, ncsr) + (m - 1) * 64 * dim
            + (m + 1) * 16 * dim)


def measured_traffic(kernel, key, chunk):
    """HBM bytes per launch of `kernel` from the committed counter summary
    profiles/<kernel>__<key>.txt ('+' of a kernel pair written '_and_';
    FETCH_SIZE + WRITE_SIZE, scaled by a copy
    kernel of known size), or None when there is none, when it was taken on
    other library sources (digest mismatch) or with another launch size."""
    from paper_1102_5071_amd.build import source_digest
    path = os.path.join(PROFILES, f"{kernel.replace('+', '_and_')}__{key}.txt")
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith((" ", "#")):
                k, v = line.split(":", 1)
                fields[k.strip()] = v.strip()
    try:
        if fields.get("source_digest") != source_digest():
            return None
        if int(fields.get("steps_per_launch", "0")) != chunk:
            return None
        return float(fields["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def copy_calibration(nbytes, reps):
    """Plain device copy of a known size (torch elementwise kernel), for the
    scale factor of the FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    n = nbytes // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.mul(src, 1.0, out=dst)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        torch.mul(src, 1.0, out=dst)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    print(json.dumps({"copy_calibration": {"bytes_read": n * 8, "bytes_written": n * 8,
                                           "launches": reps + 1, "avg_ms": round(ms, 4),
                                           "GB/s": round(2 * n * 8 / (ms * 1e-3) / 1e9, 1)}}),
          flush=True)


def make_workload(name, L):
    from paper_1102_5071_amd import inputs as I
    if name == "hydrogen":
        p = I.config_hydrogen()
        p.t0 = 40.0           # inside the pulse
        label = "hydrogen-fd Nr=2000 dr=0.1 l<=63 dim=128000 CF8:11 m=30"
        key = "hydrogen"
    elif name == "ising":
        p = I.config_ising(L=L or 10)
        label = f"ising L={p.meta['L']} dim={p.dim} CF4:2 m=16"
        key = f"ising_L{p.meta['L']}"
    elif name == "heisenberg":
        p = I.config_heisenberg(L=L or 24)
        label = f"heisenberg L={p.meta['L']} dim={p.dim} CF6:5Opt m=24"
        key = f"heisenberg_L{p.meta['L']}"
    else:
        raise SystemExit(f"unknown workload {name}")
    return p, label, key


def cpu_baseline(p, nsteps_sample, state0):
    """Time the CPU oracle on a bounded sample of the same workload."""
    from oracle import cfet as O
    try:
        from threadpoolctl import threadpool_limits
        limiter = threadpool_limits(limits=1)
    except Exception:       # pragma: no cover
        limiter = None
    t = time.perf_counter()
    O.propagate(p.H0, p.Hk, p.drives, state0, p.t0, p.dt, nsteps_sample, p.scheme, m=p.m)
    el = time.perf_counter() - t
    if limiter is not None:
        limiter.unregister() if hasattr(limiter, "unregister") else None
    return nsteps_sample / el, el


def cpu_baseline_scaled(args, p, nnz_total):
    """The oracle on one step of the same recipe at a smaller chain length
    (the full chain needs about 45 GB of host memory and minutes per step on
    the oracle), its time scaled to the benchmarked size by the ratio of
    stored non-zeros: the oracle's cost per step is the sparse products,
    linear in the non-zeros."""
    from paper_1102_5071_amd import inputs as I
    Ls = min(args.cpu_L, p.meta["L"])
    q = I.config_heisenberg(L=Ls, nsteps=1)
    nnz_s = q.H0.nnz + sum(h.nnz for h in q.Hk)
    log(f"timing the CPU oracle on 1 step at L={Ls} (nnz {nnz_s}) ...")
    cps_s, el = cpu_baseline(q, 1, q.psi0)
    scale = nnz_s / nnz_total
    cps = cps_s * scale
    log(f"oracle: {cps_s:.4f} steps/s at L={Ls} -> {cps:.3e} steps/s scaled to nnz {nnz_total}")
    return {"value": float(f"{cps:.4g}"), "unit": "steps/s", "cores": 1, "kind": "oracle",
            "sample": f"1 step of the same recipe at L={Ls} (dim {q.dim}, {nnz_s} non-zeros; "
                      f"{el:.1f} s, numpy/scipy FP64, BLAS limited to 1 thread), scaled by the "
                      f"non-zero ratio {scale:.4g} to L={p.meta['L']}"}


def run_batched(args):
    """Many-trajectory workload: 256 driven Ising chains, L ~ U{12..18}, CF4:2,
    dt = 0.01, adaptive m <= 32 at tol 1e-10, all in one batch (one kernel per
    Lanczos phase over every trajectory, step replayed from a HIP graph).
    Reports trajectory-steps/s, and the plain single-trajectory path on one
    chain of each length for comparison (same steps, m fixed at the largest
    Krylov dimension the batch used)."""
    import numpy as np
    import torch
    from paper_1102_5071_amd import binding as B
    from paper_1102_5071_amd import inputs as I

    Bt = I.config_batched(n_traj=args.ntraj, seed=0)
    K, W = args.steps, args.warmup
    nin = len(Bt.instances)
    label = (f"batched {nin} ising chains L={Bt.meta['L_min']}..{Bt.meta['L_max']} "
             f"CF4:2 dt={Bt.dt} adaptive m<={Bt.m} tol={Bt.tol}")
    log(f"workload {label}, steps={K}, warmup={W}")
    t = time.perf_counter()
    P = B.BatchPropagator(Bt.ops, Bt.instances)
    log(f"batch created in {time.perf_counter() - t:.1f}s (total dim {P.total})")
    psi = torch.from_numpy(np.concatenate([i["psi0"] for i in Bt.instances])).to("cuda")
    P.propagate(psi, 0.0, Bt.dt, W, Bt.scheme, Bt.m, Bt.tol)
    torch.cuda.synchronize()
    st0 = P.stats()
    mv0 = P.instance_matvecs()
    t_start = W * Bt.dt
    psi_start = psi.clone()
    torch.cuda.synchronize()
    t = time.perf_counter()
    P.propagate(psi, t_start, Bt.dt, K, Bt.scheme, Bt.m, Bt.tol)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t
    st1 = P.stats()
    mv = P.instance_matvecs() - mv0
    rate = nin * K / elapsed
    log(f"timed: {elapsed * 1e3:.1f} ms for {K} steps x {nin} trajectories -> "
        f"{rate:.1f} trajectory-steps/s; Krylov dimension {st1['min_m_eff']}..{st1['max_m_eff']}, "
        f"{mv.sum() / (nin * K * 2):.2f} H applications per exponential, unroll {st1['unroll']}, "
        f"block {st1['block_threads']} threads, graph {st1['graph']}, "
        f"create-time layout timing {st1['tune_us']}")
    # algorithmic bytes, vectors only (shared operators excluded: a lower bound)
    dims = np.array(P.dims, dtype=np.float64)
    expos = 2 * K
    vec_bytes = float(np.sum(mv * (48.0 + 64.0) * dims)
                      + np.sum(expos * dims * 16.0 * (mv / expos + 2.0)))
    achieved = vec_bytes / elapsed / 1e9
    # measured HBM traffic of one whole step (all kernels), when the committed
    # counter summary matches these sources
    traffic = measured_traffic("batched_step", f"batched_{nin}", 1)
    if traffic is not None:
        log(f"batched step: measured traffic {traffic / 1e9:.1f} GB per step "
            f"({traffic / (vec_bytes / K):.2f} x the vector bytes)")
    psi_end = psi.clone()
    state_error = None
    if not args.no_error:
        ref = psi_start.clone()
        P.propagate(ref, t_start, Bt.dt / 4, 4 * K, Bt.scheme, 40, 1e-13)
        torch.cuda.synchronize()
        errs = [float(torch.linalg.vector_norm(a - b).item())
                for a, b in zip(P.split(psi_end), P.split(ref))]
        state_error = max(errs)
        log(f"state error vs dt/4, m<=40, tol 1e-13: max over trajectories {state_error:.3e}")
    # plain path on one chain per length
    m_plain = int(st1["max_m_eff"])
    plain_per_L = {}
    Ks = min(K, args.plain_steps)
    for t_i, inst in enumerate(Bt.instances if Ks > 0 else []):
        L = inst["L"]
        if L in plain_per_L:
            continue
        Pp = B.Propagator(Bt.ops[inst["h0"]], [Bt.ops[k] for k in inst["hk"]], inst["drives"])
        x = P.split(psi_start)[t_i].clone()
        Pp.propagate(x, t_start, Bt.dt, 2, Bt.scheme, m_plain)
        torch.cuda.synchronize()
        x = P.split(psi_start)[t_i].clone()
        tt = time.perf_counter()
        Pp.propagate(x, t_start, Bt.dt, Ks, Bt.scheme, m_plain)
        torch.cuda.synchronize()
        el = time.perf_counter() - tt
        path = B.PATH_NAMES[Pp.stats()["path"]]
        plain_per_L[L] = (Ks / el, path)
        Pp.close()
    plain_rate = None
    if plain_per_L:
        per_step_plain = sum(1.0 / plain_per_L[i["L"]][0] for i in Bt.instances)
        plain_rate = nin / per_step_plain
        log("plain path (m=%d): " % m_plain + ", ".join(
            f"L={L}: {r:.0f} steps/s ({p})" for L, (r, p) in sorted(plain_per_L.items()))
            + f" -> {plain_rate:.1f} trajectory-steps/s for the batch one after another; "
            f"batched/plain = {rate / plain_rate:.2f}")
    cpu = None
    if args.cpu_steps != 0:
        from oracle import cfet as O
        try:
            from threadpoolctl import threadpool_limits
            limiter = threadpool_limits(limits=1)
        except Exception:       # pragma: no cover
            limiter = None
        n_cpu = 2 if args.cpu_steps < 0 else args.cpu_steps
        sample = [i for i in Bt.instances if i["L"] <= 14][:4]
        tt = time.perf_counter()
        for inst in sample:
            O.propagate(Bt.ops[inst["h0"]], [Bt.ops[k] for k in inst["hk"]], inst["drives"],
                        inst["psi0"], 0.0, Bt.dt, n_cpu, Bt.scheme, m=Bt.m, tol=Bt.tol)
        el = time.perf_counter() - tt
        # scale by dimension: the oracle's cost per step is linear in the dimension
        dim_sample = sum(1 << i["L"] for i in sample)
        cps = n_cpu * dim_sample / el / float(np.sum(dims)) * nin
        cpu = {"value": round(cps, 4), "unit": "trajectory-steps/s", "cores": 1,
               "kind": "oracle",
               "sample": f"{len(sample)} chains with L<=14, {n_cpu} steps each ({el:.1f} s), "
                         f"scaled to the batch by total dimension"}
        log(f"oracle: {cps:.3f} trajectory-steps/s (scaled)")
    out = {
        "metric": "CFET trajectory-steps/s at 1e-8 state error (batched)",
        "value": round(rate, 3), "unit": "trajectory-steps/s", "n_gpus": 1, "steps": K,
        "warmup": W, "ms_per_step": round(elapsed * 1e3 / K, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "c128", "data": "synthetic",
        "config": {"workload": label, "trajectories": nin, "total_dim": P.total,
                   "state_error": state_error, "matvecs_per_exponential":
                       round(float(mv.sum()) / (nin * K * 2), 3),
                   "plain_path_trajectory_steps_per_s": (round(plain_rate, 3)
                                                         if plain_rate else None),
                   "batched_over_plain": round(rate / plain_rate, 3) if plain_rate else None,
                   "launch_layout": {"block_threads": st1["block_threads"],
                                     "rows_per_lane": st1["unroll"]}},
        "roofline": {"bound": "hbm", "kernel": "batched step (all kernels, vector bytes only)",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "bytes_per_launch": vec_bytes / K, "launch": "one step",
                     "traffic_GBps": (round(traffic * K / elapsed / 1e9, 1)
                                      if traffic is not None else None)},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    P.close()


def run_adjoint(args):
    """Fidelity gradient of a controlled Ising chain (L = 14, dim 16384): K = 200
    piecewise-constant amplitudes on sum sx over T = 20, CF6:5Opt, dt = 0.01
    (2000 steps), m = 20.  Reports gradient steps/s (steps of the forward map
    per second of the whole gradient), the plain forward path on the same
    problem, and central finite differences of a few components."""
    import numpy as np
    import torch
    from paper_1102_5071_amd import binding as B
    from paper_1102_5071_amd import inputs as I

    p = I.config_adjoint(L=args.L or 14)
    N = p.nsteps if not args.steps_override else args.steps_override
    label = (f"adjoint ising L={p.meta['L']} dim={p.dim} K={p.meta['K']} T={N * p.dt:g} "
             f"CF6:5Opt dt={p.dt} m={p.m}")
    log(f"workload {label}, {N} steps")
    P = B.Propagator(p.H0, p.Hk, p.drives)
    psi0 = torch.from_numpy(p.psi0).to("cuda")
    target = torch.from_numpy(p.meta["target"]).to("cuda")
    F, g = P.gradient(psi0, target, 0.0, p.dt, min(N, 10), p.scheme, p.m)   # warm-up
    reps = max(1, args.grad_reps)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        F, g = P.gradient(psi0, target, 0.0, p.dt, N, p.scheme, p.m)
    elapsed = (time.perf_counter() - t) / reps
    rate = N / elapsed
    log(f"gradient: {elapsed:.3f} s for {N} steps -> {rate:.1f} steps/s; F = {F:.6e}, "
        f"|dF/du| = {np.linalg.norm(g):.3e}")
    x = psi0.clone()
    P.propagate(x, 0.0, p.dt, 10, p.scheme, p.m)
    torch.cuda.synchronize()
    x = psi0.clone()
    t = time.perf_counter()
    P.propagate(x, 0.0, p.dt, N, p.scheme, p.m)
    torch.cuda.synchronize()
    el_f = time.perf_counter() - t
    path = B.PATH_NAMES[P.stats()["path"]]
    log(f"plain forward ({path} path): {el_f * 1e3:.1f} ms -> {N / el_f:.1f} steps/s; "
        f"gradient / forward time = {elapsed / el_f:.2f}")
    # the roofline of the gradient's dominant kernel: the persistent launches
    # (forward, segment recomputation, adjoint exponentials) timed with events
    # over one more gradient call; each of the three sweeps runs N s
    # exponentials of m vectors
    s_exp = B.scheme_info(p.scheme)[1].shape[0]
    P.profile(True, max_launches=1 << 14, segments=False)
    st_a = P.stats()
    P.gradient(psi0, target, 0.0, p.dt, N, p.scheme, p.m)
    st_b = P.stats()
    P.profile(False)
    launches = st_b["timed_launches"] - st_a["timed_launches"]
    timed_ms = st_b["timed_ms"] - st_a["timed_ms"]
    nnz_total = p.H0.nnz + sum(h.nnz for h in p.Hk)
    grad_bytes = 3 * N * s_exp * exponential_algorithmic_bytes(p.dim, nnz_total, 1 + len(p.Hk),
                                                                min(p.m, p.dim))
    grad_achieved = grad_bytes / (timed_ms * 1e-3) / 1e9 if timed_ms > 0 else None
    log(f"k_propagate in the gradient: {launches} launches, {timed_ms:.1f} ms, "
        f"{grad_bytes / 1e9:.1f} GB algorithmic -> {grad_achieved:.0f} GB/s")
    # central differences of a few components with the GPU forward map: h = 1e-6
    # (rounding-limited) and the fourth-order stencil at h = 1e-3
    scale = float(np.max(np.abs(g)))

    def F_at(q, d):
        u = p.drives[0]["u"].copy()
        u[q] += d
        Pq = B.Propagator(p.H0, p.Hk, [dict(p.drives[0], u=u)])
        y = psi0.clone()
        Pq.propagate(y, 0.0, p.dt, N, p.scheme, p.m)
        val = abs(torch.vdot(target, y).item()) ** 2
        Pq.close()
        return val

    fd_err = fd4_err = 0.0
    for q in (0, p.meta["K"] // 2, p.meta["K"] - 1):
        h = 1e-6
        fd = (F_at(q, h) - F_at(q, -h)) / (2 * h)
        fd_err = max(fd_err, abs(fd - g[q]) / scale)
        h = 1e-3
        fd4 = (-F_at(q, 2 * h) + 8 * F_at(q, h) - 8 * F_at(q, -h) + F_at(q, -2 * h)) / (12 * h)
        fd4_err = max(fd4_err, abs(fd4 - g[q]) / scale)
    log(f"finite differences (3 components): central h = 1e-6 {fd_err:.2e}, fourth order "
        f"h = 1e-3 {fd4_err:.2e} of max |dF/du|")
    cpu = None
    if args.cpu_steps != 0:
        from oracle import adjoint as OA
        try:
            from threadpoolctl import threadpool_limits
            threadpool_limits(limits=1)
        except Exception:       # pragma: no cover
            pass
        n_cpu = 4 if args.cpu_steps < 0 else args.cpu_steps
        tt = time.perf_counter()
        OA.fidelity_gradient(p.H0, p.Hk, p.drives, p.psi0, p.meta["target"], 0.0, p.dt, n_cpu,
                             p.scheme, p.m)
        el = time.perf_counter() - tt
        cpu = {"value": round(n_cpu / el, 4), "unit": "steps/s", "cores": 1, "kind": "oracle",
               "sample": f"gradient over the first {n_cpu} steps ({el:.1f} s, numpy/scipy FP64)"}
        log(f"oracle gradient: {n_cpu / el:.3f} steps/s")
    out = {
        "metric": "CFET gradient steps/s (adjoint, fidelity wrt 200 drive amplitudes)",
        "value": round(rate, 3), "unit": "steps/s", "n_gpus": 1, "steps": N,
        "warmup": 1, "ms_per_step": round(elapsed * 1e3 / N, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "c128", "data": "synthetic",
        "config": {"workload": label, "plain_forward_steps_per_s": round(N / el_f, 3),
                   "gradient_over_forward_time": round(elapsed / el_f, 3),
                   "fd_max_rel_error": fd_err, "fd4_max_rel_error": fd4_err, "F": F},
        "roofline": ({"bound": "latency",
                      "kernel": "k_propagate (forward, recomputation and adjoint exponentials)",
                      "achieved": round(grad_achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                      "frac": round(grad_achieved / HBM_PEAK_GBS, 4), "traffic": None,
                      "bytes_per_launch": grad_bytes / max(1, launches), "launches": launches,
                      "avg_launch_us": round(timed_ms * 1e3 / max(1, launches), 3)}
                     if grad_achieved else None),
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    P.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--workload", default="heisenberg",
                    choices=["heisenberg", "hydrogen", "ising", "batched", "adjoint"])
    ap.add_argument("--ntraj", type=int, default=256, help="batched: number of trajectories")
    ap.add_argument("--grad-reps", type=int, default=1, help="adjoint: timed gradient calls")
    ap.add_argument("--steps-override", type=int, default=0,
                    help="adjoint: steps of the control window (default T/dt)")
    ap.add_argument("--plain-steps", type=int, default=20,
                    help="batched: steps timed on the plain path per chain length "
                         "(0: no plain comparison)")
    ap.add_argument("--L", type=int, default=0)
    ap.add_argument("--dt", type=float, default=0.0,
                    help="fix the time step (skips the step selection)")
    ap.add_argument("--eps", type=float, default=1e-8,
                    help="accuracy goal of the step selection over the workload's time span")
    ap.add_argument("--cpu-steps", type=int, default=-1,
                    help="oracle sample length (steps); 0 disables")
    ap.add_argument("--cpu-L", type=int, default=20,
                    help="heisenberg: chain length of the scaled oracle sample")
    ap.add_argument("--no-error", action="store_true", help="skip the state-error run")
    ap.add_argument("--path", default=None, choices=["multi", "single", "coop"],
                    help="force an execution path (default: chosen by dimension)")
    ap.add_argument("--layout", default=None, choices=["sell", "sell_uniform", "sell_split"],
                    help="operator layout of the multi-kernel path (default: by dimension)")
    ap.add_argument("--chunk", type=int, default=0,
                    help="steps per propagate call (default per workload); every launch "
                         "of the timed kernel then covers the same work")
    ap.add_argument("--exp", default="lanczos", choices=["lanczos", "chebyshev"],
                    help="plain workloads: exponential by Lanczos (m vectors) or by the "
                         "Chebyshev series (cfet_propagate_chebyshev)")
    ap.add_argument("--cheb-tol", type=float, default=1e-12,
                    help="Chebyshev: series truncation per exponential")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of this size (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py: the library runs on one GPU (it has no multi-GPU path); "
              "use --gpus 1", file=sys.stderr)
        sys.exit(2)
    dsteps, dwarm = DEFAULT_STEPS[args.workload]
    args.steps_given = args.steps is not None
    if args.steps is None:
        args.steps = dsteps
    if args.warmup is None:
        args.warmup = dwarm

    import torch

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    try:
        if args.copy_calibration:
            copy_calibration(args.copy_calibration << 20, max(1, args.steps))
        elif args.workload == "batched":
            run_batched(args)
        elif args.workload == "adjoint":
            run_adjoint(args)
        else:
            run_plain(args)
    finally:
        # release every device object before the interpreter exits: contexts
        # are closed by the runners; here the cached tensors go, and the device
        # is idle when the runtime (and a profiler attached to it) tears down
        import gc
        gc.collect()
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        torch.cuda.synchronize()


def run_plain(args):
    import numpy as np
    import torch
    from paper_1102_5071_amd import binding as B

    p, label, key = make_workload(args.workload, args.L)
    dt_table = p.dt
    if args.dt:
        p.dt = args.dt
    chunk = args.chunk or DEFAULT_CHUNK[args.workload]
    K = max(chunk, (args.steps + chunk - 1) // chunk * chunk)
    W = (args.warmup + chunk - 1) // chunk * chunk

    cheb = args.exp == "chebyshev"

    def run(psi, t0, dt, nsteps, m):
        for c in range(0, nsteps, chunk):
            if cheb and m == p.m:
                P.propagate_chebyshev(psi, t0 + c * dt, dt, chunk, p.scheme, args.cheb_tol)
            else:
                P.propagate(psi, t0 + c * dt, dt, chunk, p.scheme, m)

    t = time.perf_counter()
    P = B.Propagator(p.H0, p.Hk, p.drives, path=args.path, layout=args.layout)
    log(f"context created in {time.perf_counter() - t:.1f}s")
    nnz_total = p.H0.nnz + sum(h.nnz for h in p.Hk)
    ncsr = 1 + len(p.Hk)
    s = B.scheme_info(p.scheme)[1].shape[0]

    psi = torch.from_numpy(np.ascontiguousarray(p.psi0)).to("cuda")
    # the time step for the accuracy goal (Sec. 6.6), unless given
    selection = None
    if not args.dt:
        t0s, Wp, n1p, T_span = SELECT[args.workload]
        t = time.perf_counter()
        sel = P.select_dt(psi, t0s, Wp, n1p, p.scheme, p.m, T_span, args.eps,
                          refine=SELECT_REFINE)
        sel_s = time.perf_counter() - t
        p.dt = sel["dt"]
        if not args.steps_given:
            K = max(chunk, (sel["nsteps"] + chunk - 1) // chunk * chunk)
        selection = {"eps": args.eps, "T": T_span, "probe_window": [t0s, t0s + Wp],
                     "probe_steps": [sel["n1"], sel["n2"]], "probe_distance": sel["diff"],
                     "c": sel["c"], "order": sel["order"], "nsteps_for_T": sel["nsteps"],
                     "err_est": sel["err_est"], "err_check": sel["err_check"],
                     "check_steps": [sel["check_n1"], sel["check_n2"]],
                     "refine_rounds": sel["rounds"],
                     "dt_table": dt_table,
                     "err_est_at_dt_table": sel["c"] * T_span * dt_table ** sel["order"],
                     "seconds": round(sel_s, 2)}
        log(f"step selection for eps={args.eps:g} over T={T_span:g}: probes n1={sel['n1']} "
            f"n2={sel['n2']} on [{t0s:g}, {t0s + Wp:g}], distance {sel['diff']:.3e}, "
            f"c={sel['c']:.3e} -> dt={p.dt:.6g} ({sel['nsteps']} steps), "
            f"estimate {sel['err_est']:.2e}, check {sel['err_check']:.2e}, "
            f"{sel['rounds']} refinement rounds ({sel_s:.1f}s)")
    log(f"workload {label}, dt={p.dt:.6g}, steps={K}, warmup={W}, {chunk} steps per call")
    # warm-up
    run(psi, p.t0, p.dt, W, p.m)
    torch.cuda.synchronize()
    t_start = p.t0 + W * p.dt
    psi_start = psi.clone()
    st0 = P.stats()

    # timed region
    torch.cuda.synchronize()
    t = time.perf_counter()
    run(psi, t_start, p.dt, K, p.m)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t
    st1 = P.stats()
    steps_per_s = K / elapsed
    matvecs = st1["matvecs"] - st0["matvecs"]
    log(f"timed: {elapsed * 1e3:.1f} ms for {K} steps -> {steps_per_s:.2f} steps/s; "
        f"matvecs {matvecs} ({'Chebyshev terms' if cheb else f'expected {K * s * min(p.m, p.dim)}'}), "
        f"min m_eff {st1['min_m_eff']}")
    psi_end = psi.clone()

    path = B.PATH_NAMES[st1["path"]]
    m_eff = min(p.m, p.dim)
    # kernel timing pass: HIP events on the propagation stream around every
    # launch of the dominant kernel (the SpMV on the multi-kernel path, the
    # whole-call kernel on the persistent paths)
    psi.copy_(psi_start)
    P.profile(True, max_launches=(1 << 18) if cheb else min(K * s * p.m, 1 << 18),
              segments=False)
    run(psi, t_start, p.dt, K, p.m)
    torch.cuda.synchronize()
    stp = P.stats()
    P.profile(False)
    avg_ms = stp["timed_ms"] / max(1, stp["timed_launches"])
    layout = B.LAYOUT_NAMES[stp["layout"]]
    csr_bytes = spmv_algorithmic_bytes(p.dim, nnz_total, ncsr)
    extra = {}
    if path == "multi":
        kernel = B.SPMV_KERNEL_NAMES[stp["layout"]]
        if layout in ("sell_uniform", "sell_split"):
            # the stored bytes of this layout (per-slice shared entries once)
            # plus x read once and y written once
            bytes_per_launch = stp["matrix_bytes"] + 32 * p.dim
            key += "_" + layout.replace("sell_", "")
            extra["csr_equivalent_bytes_per_spmv"] = csr_bytes
            extra["csr_equivalent_GBps"] = round(csr_bytes / (avg_ms * 1e-3) / 1e9, 1)
        else:
            bytes_per_launch = csr_bytes
        if cheb:
            # the Chebyshev path times its applies (no Lanczos epilogue)
            key += "_cheb"
            kernel = {"k_lz_spmv": "k_apply", "k_sell_lz_spmv": "k_sell_apply"}.get(kernel, kernel)
    else:
        kernel = "k_propagate"
        bytes_per_launch = chunk * s * exponential_algorithmic_bytes(p.dim, nnz_total, ncsr, m_eff)
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    log(f"path {path} ({layout}): {kernel} {stp['timed_launches']} timed, avg {avg_ms * 1e3:.2f} us, "
        f"{bytes_per_launch / 1e6:.2f} MB algorithmic -> {achieved:.0f} GB/s")
    if path != "multi":
        # where block 0's time goes: a third pass with the segment timers on
        # (they lengthen the kernel slightly, so the pass above runs without)
        psi.copy_(psi_start)
        st2 = P.stats()
        P.profile(True, max_launches=16, segments=True)
        run(psi, t_start, p.dt, K, p.m)
        torch.cuda.synchronize()
        st3 = P.stats()
        P.profile(False)
        seg = [a - b for a, b in zip(st3["segment_us"], st2["segment_us"])]
        log("persistent segments (block 0, us per step): spmv %.1f, reduce/barrier %.1f, "
            "small exp %.1f, recombination %.1f" % tuple(x / K for x in seg))

    # state error over the timed window: reference at dt/4 with m = 40
    state_error = None
    if not args.no_error:
        ref = psi_start.clone()
        run(ref, t_start, p.dt / 4, 4 * K, max(40, p.m))
        torch.cuda.synchronize()
        state_error = float(torch.linalg.vector_norm(psi_end - ref).item())
        log(f"state error over the window [{t_start:g}, {t_start + K * p.dt:g}] vs dt/4, "
            f"m=40: {state_error:.3e}")
        del ref

    traffic = measured_traffic(kernel, key, chunk)
    if traffic is not None:
        log(f"{kernel}: measured HBM traffic {traffic / 1e6:.2f} MB per launch "
            f"({traffic / bytes_per_launch:.3f} x algorithmic)")

    # CPU oracle baseline on a bounded sample
    cpu = None
    n_cpu = args.cpu_steps
    if args.workload == "heisenberg" and p.dim > (1 << 20):
        if n_cpu != 0:
            cpu = cpu_baseline_scaled(args, p, nnz_total)
    else:
        if n_cpu < 0:
            n_cpu = {"hydrogen": 15, "ising": 200, "heisenberg": 1}[args.workload]
        if n_cpu > 0:
            log(f"timing the CPU oracle on {n_cpu} steps ...")
            cps, cel = cpu_baseline(p, n_cpu, psi_start.cpu().numpy())
            cpu = {"value": round(cps, 4), "unit": "steps/s", "cores": 1, "kind": "oracle",
                   "sample": f"{n_cpu} steps of the same workload from the same start state "
                             f"({cel:.1f} s, numpy/scipy FP64, BLAS limited to 1 thread)"}
            log(f"oracle: {cps:.3f} steps/s")

    roof = {"bound": BOUND[args.workload], "kernel": kernel, "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic, "bytes_per_launch": bytes_per_launch,
            "avg_launch_us": round(avg_ms * 1e3, 3)}
    roof.update(extra)
    if traffic is not None:
        roof["traffic_GBps"] = round(traffic / (avg_ms * 1e-3) / 1e9, 1)
    out = {
        "metric": "CFET steps/s at 1e-8 state error (batched/adjoint vs plain); SpMV HBM GB/s",
        "value": round(steps_per_s, 3),
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": round(elapsed * 1e3 / K, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128",
        "data": "synthetic",
        "config": {"workload": label, "dim": p.dim, "nnz": nnz_total, "scheme": p.scheme,
                   "krylov_m": None if cheb else p.m,
                   "exponential": (f"chebyshev tol={args.cheb_tol:g}" if cheb
                                   else f"lanczos m={p.m}"),
                   "dt": p.dt, "dt_selection": selection,
                   "t0": t_start, "path": path,
                   "layout": layout if path == "multi" else "csr",
                   "steps_per_call": chunk,
                   "state_error": state_error,
                   "state_error_window": [t_start, t_start + K * p.dt],
                   "seconds_for_T": (round(selection["nsteps_for_T"] * elapsed / K, 4)
                                     if selection else None),
                   "matvecs_per_step": matvecs / K},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    P.close()
    del psi, psi_start, psi_end


if __name__ == "__main__":
    main()
