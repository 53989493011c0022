#!/usr/bin/env python3
"""Benchmark of the Parareal hot path for 2D Rayleigh-Benard convection on
one MI355X.

Workload: Ra = 1e6, Pr = 1, aspect ratio 2, fine grid 256 x 64, 32 time
slices over t in [0, 50], fine step 2e-4 (7813 steps per slice), coarse grid
128 x 32 at step 2e-3, ARS(4,4,3), mixed precision (FP32 transforms and
products, FP64 state, solves, correction, defect and Nusselt numbers).

One timed step is one Parareal iteration.  The timed region is one whole
Parareal run from the seeded initial state: the coarse prediction, then
`--steps` iterations in the pipelined schedule (each slice's fine run starts
as soon as its initial state is corrected and advances in one batch with
every other run in flight; the serial coarse sweep overlaps them), with the
correction U_{n+1} = G(U_n^new) + F(U_n^old) - G(U_n^old), the defect and
Nusselt samples every 50 fine steps.  Iteration k runs F on slices k-1..S-1.
`value` is the fine DOF-steps computed (grid points x fine steps x fine
runs) per second of that wall time, so the coarse sweeps count against it.
The same run in the sweep-then-batch order (bit-identical results) and the
fine propagator alone at full batch are reported beside it.

The roofline object describes the dominant kernel (the per-mode stage
kernel): algorithmic bytes per launch from the byte model below (per state
times the mean number of states in the timed launches), divided by its
mean launch duration measured with HIP events on the stream it runs on
during the timed run.  The cpu_baseline object times the FP64
CPU oracle on one host core over a bounded number of fine steps of one slice.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import rbc_inputs as I  # noqa: E402

HBM_PEAK_GBS = 8000.0
NU_STRIDE = 50
TIMING_EVERY = 97


def stage_kernel_bytes_per_dof_step(s: int, rb: int) -> float:
    """Compulsory HBM bytes of the stage kernel per grid point and slice over
    one fine step (all s stage launches).  Per launch i = 1..s it reads the
    two product fields on the padded grid (2 x 1.5 values per point of Real),
    the old state (2 doubles per point), the i-1 stored explicit terms (Real)
    and i-1 stored implicit terms (FP64), and writes the explicit term and
    the implicit term for later stages (i < s), the new state (i = s) and the
    six padded-grid fields of the next x-pass (6 x 1.5 Real per point)."""
    tot = 0.0
    for i in range(1, s + 1):
        tot += 2 * 1.5 * rb + 2 * 8 + (i - 1) * 2 * rb + (i - 1) * 2 * 8
        if i < s:
            tot += 2 * rb + 2 * 8
        else:
            tot += 2 * 8
        tot += 6 * 1.5 * rb
    return tot


def xpass_bytes_per_dof_step(s: int, rb: int) -> float:
    """x-pass: reads six padded-grid fields and writes two (per stage)."""
    return s * (6 * 1.5 * rb + 2 * 1.5 * rb)


def measured_traffic(workload: str):
    """HBM bytes per state of a stage-kernel launch from the committed PMC
    summary (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy, over the states
    of the profiled launches), or None when the summary is for another
    workload or the kernel source has changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "stage_kernel_traffic.txt")
    src = os.path.join(ROOT, "paper_2001_01609_amd", "csrc", "rbc_kernels.hip")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if ":" in line:
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    with open(src, "rb") as f:
        cur = hashlib.sha256(f.read()).hexdigest()[:16]
    if kv.get("workload") != workload or kv.get("kernel_source_sha256_16") != cur:
        return None
    return float(kv["bytes_per_launch"]) / float(kv["states_per_launch"])


def cpu_baseline(w, seconds: float):
    """Time the FP64 oracle's fine steps on one slice, one host thread."""
    from threadpoolctl import threadpool_limits

    from oracle import rbc_oracle as O
    n, dt = O.steps_per_slice(w.t0, w.t_end, w.n_slices, w.dt_f)
    g = O.Grid(w.Ra, w.Pr, w.Lx, w.Lz, w.Nx, w.Nz, dt, scheme=w.scheme)
    with threadpool_limits(limits=1):
        st = O.Stepper(g)
        X = O.initial_state(g, I.gaussian_noise(w.seed, w.Nx, w.Nz), w.noise_amp)
        X = st.step(X)
        steps = 0
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < seconds:
            X = st.step(X)
            steps += 1
        el = time.perf_counter() - t0
    return {"value": w.Nx * w.Nz * steps / el, "unit": "DOF-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"{steps} FP64 fine steps of one {w.Nx}x{w.Nz} slice (ARS443, dt {dt:.6g}) "
                      f"from the seeded initial state; {el:.1f} s on one thread"}


def q_visc(w) -> float:
    """Viscosity in free-fall units."""
    return math.sqrt(w.Pr / w.Ra)


def diag_time_averages(rec: np.ndarray, visc: float) -> np.ndarray:
    """Time averages of diagnostic records (Nu_V, Nu_b, Nu_t, KE, eps_U, P)
    in the library's order: Nu_V, Nu_b, Nu_t, Nu_int, KE, Re, eps_U, P,
    |P - eps_U| / P (section 2.2)."""
    nv, nb, nt, ke, eps, P = rec.mean(axis=0)
    re = float(np.mean(np.sqrt(2.0 * rec[:, 3]))) / visc
    nu_int = max(abs(nb - nv), abs(nb - nt), abs(nv - nt)) / nv
    return np.array([nv, nb, nt, nu_int, ke, re, eps, P, abs(P - eps) / P])


def time_to_solution(w, tol: float = 1e-8):
    """Parareal (this workload's precision with the FP64 switch, pipelined
    schedule) to a defect <= tol, against the serial FP64 fine stepper on one
    run over the same horizon and fine step.  Both report time-averaged
    Nusselt numbers over the whole horizon (samples every NU_STRIDE fine
    steps)."""
    import torch

    from paper_2001_01609_amd import rbc as R
    dev = torch.device("cuda:0")
    st = torch.cuda.current_stream(dev).cuda_stream
    S = w.n_slices
    # Parareal
    p = R.params_from_workload(w, nu_stride=NU_STRIDE, nu_t_start=w.t0)
    h = R.rbc_create(p, st)
    try:
        n = R.rbc_state_size(h, 0)
        U = torch.zeros((S + 1) * n, dtype=torch.float64, device=dev)
        R.rbc_init_state(h, w.seed, w.noise_amp, U)
        torch.cuda.synchronize()
        print("[bench] time to solution: Parareal", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        status, kd, defects, nu = R.parareal_iterate(h, U, S, tol, want_nu=True)
        torch.cuda.synchronize()
        t_para = time.perf_counter() - t0
        k64 = R.rbc_fine_fp64_from(h)
        report_at = R.rbc_get_pipeline_stats(h)["report_at_s"][: kd + 1] if p.pipelined else None
        u_end = U[S * n:].clone()
    finally:
        R.rbc_destroy(h)
    # serial FP64 stepper: one run over the whole horizon
    q = R.params_from_workload(w, n_slices=1, precision=R.RBC_FP64, nu_stride=NU_STRIDE, nu_t_start=w.t0)
    q.dt_f = (w.t_end - w.t0) / S / math.ceil((w.t_end - w.t0) / S / w.dt_f - 1e-9)   # the Parareal fine step
    q.dt_c = q.dt_f
    h = R.rbc_create(q, st)
    try:
        ns, dts = R.rbc_steps_per_slice(h, 0)
        V = torch.zeros(n, dtype=torch.float64, device=dev)
        R.rbc_init_state(h, w.seed, w.noise_amp, V)
        nus = torch.zeros((ns // NU_STRIDE) * R.RBC_DIAG, dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        print(f"[bench] time to solution: serial FP64 ({ns} steps)", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        R.rbc_fine_step_batch(h, V, V, 1, ns, nus)
        torch.cuda.synchronize()
        t_ser = time.perf_counter() - t0
        nu_ser = diag_time_averages(nus.view(-1, R.RBC_DIAG).cpu().numpy(), q_visc(w))
        rel = float(torch.linalg.norm(u_end - V) / torch.linalg.norm(V))
    finally:
        R.rbc_destroy(h)
    nu_par = nu[-1]
    fields = R.DIAG_AVG_FIELDS
    return {"parareal_s": t_para, "serial_fp64_s": t_ser, "speedup": t_ser / t_para,
            "iterations": kd, "fp64_from_iteration": k64, "iteration_done_at_s": report_at,
            "status": status, "tol": tol, "defects": [float(d) for d in defects],
            "serial_steps": ns,
            "averages_parareal": {f: float(v) for f, v in zip(fields, nu_par)},
            "averages_serial_fp64": {f: float(v) for f, v in zip(fields, nu_ser)},
            "nu_V_rel_diff": float(abs(nu_par[0] - nu_ser[0]) / abs(nu_ser[0])),
            "final_state_rel_l2_vs_serial_fp64": rel}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default=I.C2.name, choices=sorted(I.WORKLOADS))
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="oracle sample length (0 = skip)")
    ap.add_argument("--no-tts", action="store_true",
                    help="skip the Parareal vs serial FP64 time-to-solution comparison")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the sweep-then-batch run and the full-batch fine propagator (profiling: the "
                         "fine kernels then run only in the timed pipelined run)")
    ap.add_argument("--profile-steps", type=int, default=0, metavar="N",
                    help="counter-collection mode: only N batched fine steps (same kernels and launch "
                         "shapes as the timed run), no Parareal iteration, no JSON line")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="also run one plain device-to-device copy of MIB MiB (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the slices of a run would shard "
              "across GPUs as described in the design notes, but no multi-GPU path is built.",
              file=sys.stderr)
        return 2

    import torch

    from paper_2001_01609_amd import rbc as R

    w = I.WORKLOADS[args.workload]
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    S = w.n_slices
    K = args.steps
    # the measured configuration: mixed precision throughout (no FP64 switch),
    # Nu samples every NU_STRIDE fine steps, pipelined schedule
    p = R.params_from_workload(w, nu_stride=NU_STRIDE, nu_t_start=w.t0, promote_fp64=0, pipelined=1)
    h = R.rbc_create(p, stream.cuda_stream)
    try:
        n = R.rbc_state_size(h, 0)
        nf, dtf = R.rbc_steps_per_slice(h, 0)
        ncs, dtc = R.rbc_steps_per_slice(h, 1)
        U = torch.zeros((S + 1) * n, dtype=torch.float64, device=dev)

        def calibrate():
            # reference kernels of known traffic for the HBM byte counters:
            # a fill (writes N bytes), an elementwise scale by 1 into another
            # buffer (reads N, writes N) and the runtime's device copy
            if args.calibrate_copy > 0:
                a = torch.empty(args.calibrate_copy * (1 << 20) // 8, dtype=torch.float64, device=dev)
                b = torch.empty_like(a)
                a.fill_(1.0)
                torch.mul(a, 1.0, out=b)
                b.copy_(a)
                torch.cuda.synchronize()
                del a, b

        if args.profile_steps > 0:
            # the fine propagator's kernels at full batch from the seeded state
            F = torch.zeros(S * n, dtype=torch.float64, device=dev)
            R.rbc_init_state(h, w.seed, w.noise_amp, F)
            F.view(S, n)[1:] = F.view(S, n)[0]
            R.rbc_fine_step_batch(h, F, F, S, args.profile_steps, None)
            torch.cuda.synchronize()
            calibrate()
            print(f"[bench] profile mode: {args.profile_steps} batched fine steps done", file=sys.stderr)
            return 0

        def parareal(k):
            U.zero_()
            R.rbc_init_state(h, w.seed, w.noise_amp, U)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st, kd, defects, nu = R.parareal_iterate(h, U, k, 0.0, want_nu=True)
            torch.cuda.synchronize()
            return time.perf_counter() - t0, kd, defects, nu

        for it in range(args.warmup):
            parareal(1)
            print(f"[bench] warmup Parareal run {it + 1}/{args.warmup} (1 iteration) done", file=sys.stderr,
                  flush=True)
        R.rbc_kernel_timing_enable(h, 0, TIMING_EVERY)
        el, kd, defects, nu_hist = parareal(K)
        k_ms, k_cnt, k_batch = R.rbc_kernel_timing(h)
        R.rbc_kernel_timing_enable(h, -1, 0)
        pstats = R.rbc_get_pipeline_stats(h)
        print(f"[bench] timed pipelined Parareal: {K} iterations in {el:.2f} s", file=sys.stderr, flush=True)
        u_pipe = U.cpu().numpy()
        finite = bool(np.isfinite(u_pipe).all())
        # fine propagator alone at full batch (events around one batched F
        # call; the stage kernel timed inside it as well)
        full = None
        if not args.no_compare:
            F = U[:S * n].clone()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            R.rbc_kernel_timing_enable(h, 0, TIMING_EVERY)
            e0.record(stream)
            R.rbc_fine_step_batch(h, F, F, S, nf, None)
            e1.record(stream)
            torch.cuda.synchronize()
            f_ms = e0.elapsed_time(e1)
            kf_ms, kf_cnt, kf_batch = R.rbc_kernel_timing(h)
            R.rbc_kernel_timing_enable(h, -1, 0)
            full = (f_ms, kf_ms, kf_cnt, kf_batch)
            calibrate()
    finally:
        # one handle at a time: each holds two streams, and a process has few
        # hardware queues (two live handles can leave the fine and coarse
        # streams of the next one on a shared queue, without overlap)
        R.rbc_destroy(h)
    # the same K iterations in the sweep-then-batch order (same results, bit for bit)
    seq = None
    if not args.no_compare:
        q = R.params_from_workload(w, nu_stride=NU_STRIDE, nu_t_start=w.t0, promote_fp64=0, pipelined=0)
        h = R.rbc_create(q, stream.cuda_stream)
        try:
            U.zero_()
            R.rbc_init_state(h, w.seed, w.noise_amp, U)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            R.parareal_iterate(h, U, K, 0.0, want_nu=True)
            torch.cuda.synchronize()
            el_seq = time.perf_counter() - t0
            seq = (el_seq, bool(np.array_equal(U.cpu().numpy(), u_pipe)))
            print(f"[bench] sweep-then-batch Parareal: {K} iterations in {el_seq:.2f} s", file=sys.stderr,
                  flush=True)
        finally:
            R.rbc_destroy(h)
    return emit(args, w, K, el, kd, defects, nu_hist, finite, k_ms, k_cnt, k_batch, pstats, nf, ncs, seq, full)


def emit(args, w, K, el, kd, defects, nu_hist, finite, k_ms, k_cnt, k_batch, pstats, nf, ncs, seq, full):
    """Prints the JSON line (the timed run's figures and the optional legs)."""
    from paper_2001_01609_amd import rbc as R
    S = w.n_slices

    dof = w.Nx * w.Nz
    runs = sum(S - k + 1 for k in range(1, K + 1))      # fine runs of iterations 1..K
    fine_dof_steps = dof * nf * runs
    value = fine_dof_steps / el
    rb = 4 if w.mixed else 8
    s = w.scheme
    per_state = stage_kernel_bytes_per_dof_step(s, rb) / s * dof
    per_launch = per_state * k_batch
    achieved = per_launch / (k_ms * 1e-3) / 1e9 if k_ms > 0 else 0.0
    traffic_state = measured_traffic(w.name)
    out = {
        "metric": "fine-step DOF-steps/s (%HBM roofline); Parareal vs serial time-to-solution",
        "value": value,
        "unit": "DOF-steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * el / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if w.mixed else "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "Ra": w.Ra, "Pr": w.Pr, "grid": [w.Nx, w.Nz],
                   "coarse_grid": [w.Nx_c, w.Nz_c], "slices": S, "t": [w.t0, w.t_end],
                   "fine_steps_per_slice": nf, "coarse_steps_per_slice": ncs,
                   "scheme": "ARS443" if s == 4 else "ARS222",
                   "step": "one Parareal iteration (pipelined schedule; the timed run is the coarse "
                           "prediction and `steps` iterations from the seeded state, fine runs of "
                           "iteration k on slices k-1..S-1)"},
        "roofline": {"bound": "hbm", "kernel": "stage_kernel", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic_state * k_batch if traffic_state else None,
                     "bytes_per_launch": per_launch, "mean_launch_ms": k_ms, "timed_launches": k_cnt,
                     "mean_slices_per_launch": k_batch},
        "parareal": {"iterations": kd, "defects": [float(d) for d in defects], "fine_runs": runs,
                     "averages_last": {f: float(v) for f, v in zip(R.DIAG_AVG_FIELDS, nu_hist[-1])},
                     "finite": finite,
                     "scheduler": {k: v for k, v in pstats.items() if k != "report_at_s"}},
    }
    if seq is not None:
        el_seq, same = seq
        out["parareal"].update({"sweep_then_batch_s": el_seq, "sweep_then_batch_value": fine_dof_steps / el_seq,
                                "pipelined_speedup": el_seq / el, "bitwise_equal_to_sweep_then_batch": same})
    if full is not None:
        f_ms, kf_ms, kf_cnt, kf_batch = full
        achieved_full = per_state * kf_batch / (kf_ms * 1e-3) / 1e9 if kf_ms > 0 else 0.0
        out["fine_propagator"] = {
            "dof_steps_per_s": dof * S * nf / (f_ms * 1e-3), "ms_per_call": f_ms,
            "us_per_batched_step": 1e3 * f_ms / nf, "slices": S,
            "stage_kernel": {"mean_launch_ms": kf_ms, "timed_launches": kf_cnt,
                             "bytes_per_launch": per_state * kf_batch, "achieved_gbs": achieved_full,
                             "frac": achieved_full / HBM_PEAK_GBS,
                             "traffic": traffic_state * kf_batch if traffic_state else None},
            "bytes_per_dof_step_model": stage_kernel_bytes_per_dof_step(s, rb) + xpass_bytes_per_dof_step(s, rb)}
    if not args.no_tts:
        out["time_to_solution"] = time_to_solution(w)
    if args.cpu_seconds > 0:
        print("[bench] timing the CPU oracle", file=sys.stderr, flush=True)
        cb = cpu_baseline(w, args.cpu_seconds)
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
