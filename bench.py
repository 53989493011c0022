#!/usr/bin/env python3
"""Benchmark of the Parareal hot path for 2D Rayleigh-Benard convection on
one MI355X.

Headline (one bench "step" = one batched fine step of the whole fine
propagator F over every time slice): Ra = 1e8, Pr = 1, aspect ratio 2, fine
grid 1024 x 256, 64 slices of [0, 20] (fine step 2e-5), ARS(4,4,3), mixed
precision (FP32 transforms and products on FP32 MFMA / vector units, FP64
state, banded solves and Nusselt numbers).  The slice states are the coarse
prediction (256 x 64 grid) of the seeded initial state, so every slice
starts from its own state of the trajectory; Nusselt records are sampled
every 50 fine steps inside the timed region.  `value` is fine DOF-steps per
second: 64 slices x 1024 x 256 points x `--steps` batched steps over the
wall time (inputs resident in HBM; events and a device synchronise on both
sides).

The roofline object is the per-mode stage of the step (forward transform,
stage right-hand side and banded solves, inverse transform: the
fwd_gemm, stage and inv_gemm kernels of one stage), timed with HIP events
on the stream they run on around every stage of the timed steps, against
the 3-pass minimum of 176 bytes per grid point and stage (mixed, ARS443):
the 6 padded-grid fields it writes and the 2 it reads (12 x 4 bytes) and a
quarter of the 64 FP64 stage-data values per grid point and step (state,
right-hand-side history, stage writes).  The whole step's 896 bytes per
DOF-step is reported beside it, with the x-pass.

Legs beside the headline (skippable):
  ensemble          24 independent runs of different Rayleigh numbers and
                    grids (128 x 32, 256 x 64, 512 x 128; 16 slices each)
                    advanced together by the ensemble engine;
  serving           a Poisson stream of Parareal requests served with
                    continuous batching (throughput, p50 / p99 latency);
  parareal_c2       one pipelined Parareal run at Ra 1e6, 256 x 64, 32
                    slices (coarse prediction + 3 iterations) and the same
                    run in the sweep-then-batch order (bit-identical);
  time_to_solution  Parareal at that workload (FP64 switch on) to a defect
                    of 1e-8 against the serial FP64 GPU stepper over the
                    same window and fine step;
  cpu_baseline      the FP64 CPU oracle on one host core: fine steps of one
                    1024 x 256 slice (the headline's unit), and one
                    64 x 32 slice.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import rbc_inputs as I  # noqa: E402
from paper_2001_01609_amd.studies import time_averages  # noqa: E402

HBM_PEAK_GBS = 8000.0
NU_STRIDE = 50


def stage_data_values(s: int) -> int:
    """FP64 stage data per grid point and fine step (3-pass model): the old
    state read by each of the s stages (2 fields), the right-hand-side
    history of stage i (2 + 4 (i - 1) fields), and the writes of Y_i, E_i
    and L Y_i (2 fields each) per stage."""
    return 2 * s + sum(2 + 4 * (i - 1) for i in range(1, s + 1)) + 6 * s


def bytes_per_dof_step(s: int, b_bulk: int, b_state: int = 8) -> float:
    """3-pass minimum HBM bytes per grid point and fine step: per stage the
    inverse transform writes 6 padded-grid fields (1.5 values per point
    each), the x-pass reads them and writes 2, the forward transform reads
    those 2 (24 x 1.5 ... = 24 bulk values per point), plus the stage data."""
    return 24 * s * b_bulk + stage_data_values(s) * b_state


def stage_bytes_per_dof_launch(s: int, b_bulk: int, b_state: int = 8) -> float:
    """The per-mode stage's share per stage: 8 of the 16 padded-grid field
    passes (6 written, 2 read, 1.5 values per point each) and 1/s of the
    stage data."""
    return 12 * b_bulk + stage_data_values(s) * b_state / s


def xpass_bytes_per_dof_launch(b_bulk: int) -> float:
    """The x-pass per stage: reads 6 padded-grid fields, writes 2."""
    return 12 * b_bulk


def measured_traffic(workload: str):
    """HBM bytes per state of one stage (the per-mode kernels of that stage)
    from the committed PMC summary (FETCH_SIZE + WRITE_SIZE scaled by a
    plain copy), or None when the summary is for another workload or the
    kernel source has changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"stage_traffic_{workload}.txt")
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
    return float(kv["bytes_per_stage"]) / float(kv["states_per_launch"])


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_oracle_rate(w, seconds: float):
    """The FP64 oracle's fine steps on one slice of workload w, one host
    thread, for about `seconds` (setup not timed)."""
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
        while time.perf_counter() - t0 < seconds or steps == 0:
            X = st.step(X)
            steps += 1
        el = time.perf_counter() - t0
    return w.Nx * w.Nz * steps / el, steps, el, dt


def cpu_baseline(seconds: float):
    """The oracle timed on the host: the headline's unit (one 1024 x 256
    slice, ARS443) and the small plain case (one 64 x 32 slice, ARS222)."""
    v3, n3, e3, dt3 = cpu_oracle_rate(I.C3, seconds)
    v1, n1, e1, dt1 = cpu_oracle_rate(I.C1, max(seconds / 3, 2.0))
    return {"value": v3, "unit": "DOF-steps/s", "cores": 1, "kind": "oracle", "cpu": cpu_model(),
            "host_cpus": os.cpu_count(),
            "sample": f"{n3} FP64 fine steps of one 1024x256 slice (Ra 1e8, ARS443, dt {dt3:.3g}) from the "
                      f"seeded initial state, {e3:.1f} s on one thread (operator setup not timed)",
            "small_case": {"value": v1, "unit": "DOF-steps/s",
                           "sample": f"{n1} FP64 fine steps of one 64x32 slice (Ra 1e4, ARS222, dt {dt1:.3g}), "
                                     f"{e1:.1f} s on one thread"}}


def q_visc(w) -> float:
    """Viscosity in free-fall units."""
    return math.sqrt(w.Pr / w.Ra)


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


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
    p = R.params_from_workload(w, nu_stride=NU_STRIDE, nu_t_start=w.t0)
    h = R.rbc_create(p, st)
    try:
        n = R.rbc_state_size(h, 0)
        U = torch.zeros((S + 1) * n, dtype=torch.float64, device=dev)
        R.rbc_init_state(h, w.seed, w.noise_amp, U)
        torch.cuda.synchronize()
        log("time to solution: Parareal")
        t0 = time.perf_counter()
        status, kd, defects, nu = R.parareal_iterate(h, U, S, tol, want_nu=True)
        torch.cuda.synchronize()
        t_para = time.perf_counter() - t0
        k64 = R.rbc_fine_fp64_from(h)
        report_at = R.rbc_get_pipeline_stats(h)["report_at_s"][: kd + 1] if p.pipelined else None
        u_end = U[S * n:].clone()
    finally:
        R.rbc_destroy(h)
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
        log(f"time to solution: serial FP64 ({ns} steps)")
        t0 = time.perf_counter()
        R.rbc_fine_step_batch(h, V, V, 1, ns, nus)
        torch.cuda.synchronize()
        t_ser = time.perf_counter() - t0
        nu_ser = time_averages(nus.view(-1, R.RBC_DIAG).cpu().numpy(), q_visc(w))
        rel = float(torch.linalg.norm(u_end - V) / torch.linalg.norm(V))
    finally:
        R.rbc_destroy(h)
    nu_par = nu[-1]
    fields = R.DIAG_AVG_FIELDS
    return {"workload": w.name, "parareal_s": t_para, "serial_fp64_s": t_ser, "speedup": t_ser / t_para,
            "iterations": kd, "fp64_from_iteration": k64, "iteration_done_at_s": report_at,
            "status": status, "tol": tol, "defects": [float(d) for d in defects],
            "serial_steps": ns,
            "averages_parareal": {f: float(v) for f, v in zip(fields, nu_par)},
            "averages_serial_fp64": {f: float(v) for f, v in zip(fields, nu_ser)},
            "nu_V_rel_diff": float(abs(nu_par[0] - nu_ser[0]) / abs(nu_ser[0])),
            "final_state_rel_l2_vs_serial_fp64": rel}


def parareal_leg(w, K: int):
    """One pipelined Parareal run (coarse prediction + K iterations, Nusselt
    samples every NU_STRIDE fine steps, no FP64 switch) and the same run in
    the sweep-then-batch order."""
    import torch

    from paper_2001_01609_amd import rbc as R
    dev = torch.device("cuda:0")
    st = torch.cuda.current_stream(dev).cuda_stream
    S = w.n_slices
    out = {"workload": w.name, "iterations": K}
    finals = []
    for pipelined in (1, 0):
        p = R.params_from_workload(w, nu_stride=NU_STRIDE, nu_t_start=w.t0, promote_fp64=0, pipelined=pipelined)
        h = R.rbc_create(p, st)
        try:
            n = R.rbc_state_size(h, 0)
            nf, _ = R.rbc_steps_per_slice(h, 0)
            U = torch.zeros((S + 1) * n, dtype=torch.float64, device=dev)
            R.rbc_init_state(h, w.seed, w.noise_amp, U)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, kd, defects, nu = R.parareal_iterate(h, U, K, 0.0, want_nu=True)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            finals.append(U.cpu().numpy())
            runs = sum(S - k + 1 for k in range(1, kd + 1))
            key = "pipelined" if pipelined else "sweep_then_batch"
            out[key] = {"s": el, "fine_dof_steps_per_s": w.Nx * w.Nz * nf * runs / el, "defects": defects.tolist()}
            if pipelined:
                stats = R.rbc_get_pipeline_stats(h)
                out[key]["scheduler"] = {k: v for k, v in stats.items() if k != "report_at_s"}
                out[key]["averages_last"] = {f: float(v) for f, v in zip(R.DIAG_AVG_FIELDS, nu[-1])}
            log(f"parareal leg ({key}): {K} iterations in {el:.2f} s")
        finally:
            R.rbc_destroy(h)
    out["pipelined_speedup"] = out["sweep_then_batch"]["s"] / out["pipelined"]["s"]
    out["bitwise_equal_to_sweep_then_batch"] = bool(np.array_equal(finals[0], finals[1]))
    return out


def ensemble_leg(t_end: float = 0.5, k_max: int = 3):
    """The 24-run ensemble (Ra log-uniform in [1e5, 1e7], grids 128x32 /
    256x64 / 512x128, 16 slices each, mixed precision) advanced together to
    k_max iterations: aggregate fine DOF-steps per second of the whole
    job (predictions and coarse sweeps included)."""
    import torch

    from paper_2001_01609_amd import rbc as R
    runs = I.ensemble_runs(t_end=t_end)
    dev = torch.device("cuda:0")
    st = torch.cuda.current_stream(dev).cuda_stream
    e = R.rbc_ensemble_create(st)
    try:
        ids, plist = [], []
        t_setup = time.perf_counter()
        for w in runs:
            p = R.params_from_workload(w, promote_fp64=0, pipelined=0)
            U0 = torch.zeros(4 * (w.Nx // 2) * w.Nz, dtype=torch.float64, device=dev)
            R.rbc_initial_state(p, w.seed, w.noise_amp, U0, st)
            ids.append(R.rbc_ensemble_add(e, p, U0, k_max, w.tol))
            plist.append(p)
        t_setup = time.perf_counter() - t_setup
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        t0 = time.perf_counter()
        n_steps = 0
        while R.rbc_ensemble_step(e) > 0:
            n_steps += 1
        n_steps += 1
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        dof_steps = 0.0
        for w, rid in zip(runs, ids):
            _, kd, _, _ = R.rbc_ensemble_run_info(e, rid, 0)
            nf = math.ceil((w.t_end - w.t0) / w.n_slices / w.dt_f - 1e-9)
            dof_steps += w.Nx * w.Nz * nf * sum(w.n_slices - k + 1 for k in range(1, kd + 1))
    finally:
        R.rbc_ensemble_destroy(e)
    grids = {}
    for w in runs:
        grids[f"{w.Nx}x{w.Nz}"] = grids.get(f"{w.Nx}x{w.Nz}", 0) + 1
    log(f"ensemble leg: {len(runs)} runs, {n_steps} engine steps in {el:.2f} s")
    return {"runs": len(runs), "grids": grids, "slices_per_run": runs[0].n_slices, "t": [0.0, t_end],
            "iterations": k_max, "engine_steps": n_steps, "s": el, "setup_s": t_setup,
            "fine_dof_steps": dof_steps, "fine_dof_steps_per_s": dof_steps / el,
            "device_bytes_free_at_start": free0}


def serving_leg(n: int = 24, rate: float = 2.0, seed: int = 5000):
    """A Poisson stream of Parareal requests (Ra log-uniform in [1e4, 1e7],
    grids 64x32 .. 512x128, horizons in [0.05, 0.3], tolerance 1e-6 (mixed)
    or 1e-8 (FP64), 16 slices, at most 3 iterations) served with continuous
    batching and admission by free device memory."""
    import torch

    from paper_2001_01609_amd import rbc as R
    from paper_2001_01609_amd import serving as SV
    descs = SV.request_stream(n, rate, seed=seed)
    reqs = [SV.Request(rid=d["rid"], arrival=d["arrival"], params=SV.make_params(R, d), seed=d["seed"],
                       tol=d["tol"], k_max=d["k_max"]) for d in descs]
    eng = SV.GpuEngine()
    free_min = [torch.cuda.mem_get_info()[0]]
    total = torch.cuda.mem_get_info()[1]

    def free():
        f = torch.cuda.mem_get_info()[0]
        free_min[0] = min(free_min[0], f)
        return f

    sched = SV.Scheduler(eng, free_bytes=free, footprint=lambda q: R.rbc_ensemble_footprint(q.params),
                         reserve=8 << 30, max_active=16)
    try:
        wall = SV.serve(reqs, sched)
    finally:
        eng.close()
    rep = SV.latency_report(sched.done, wall)
    dof = 0.0
    for c in sched.done:
        d = descs[c.rid]
        nf = math.ceil(d["t_end"] / d["n_slices"] / d["dt_f"] - 1e-9)
        dof += d["Nx"] * d["Nz"] * nf * sum(d["n_slices"] - k + 1 for k in range(1, c.k_done + 1))
    rep.update({"arrival_rate_per_s": rate, "engine_steps": sched.steps, "peak_active_runs": sched.peak_active,
                "fine_dof_steps_per_s": dof / wall, "peak_device_bytes_used": int(total - free_min[0]),
                "admission_waits": sched.admission_waits,
                "failed": sum(1 for c in sched.done if c.state != 1)})
    log(f"serving leg: {rep['requests']} requests in {wall:.2f} s, p50 {rep['latency_p50_s']:.2f} s, "
        f"p99 {rep['latency_p99_s']:.2f} s")
    return rep


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200, help="timed batched fine steps")
    ap.add_argument("--warmup", type=int, default=20, help="untimed batched fine steps first")
    ap.add_argument("--workload", default=I.C3.name, choices=sorted(I.WORKLOADS))
    ap.add_argument("--cpu-seconds", type=float, default=20.0, help="oracle sample length (0 = skip)")
    ap.add_argument("--no-tts", action="store_true", help="skip the time-to-solution leg")
    ap.add_argument("--no-parareal", action="store_true", help="skip the Parareal throughput leg")
    ap.add_argument("--no-ensemble", action="store_true", help="skip the 24-run ensemble leg")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving leg")
    ap.add_argument("--profile-steps", type=int, default=0, metavar="N",
                    help="counter-collection mode: only N batched fine steps of the headline (same kernels "
                         "and launch shapes), no JSON line")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="also run one plain elementwise copy of MIB MiB (reference for HBM byte counters)")
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
    S, K, W = w.n_slices, args.steps, args.warmup
    p = R.params_from_workload(w, nu_stride=NU_STRIDE, nu_t_start=w.t0, promote_fp64=0)
    h = R.rbc_create(p, stream.cuda_stream)
    try:
        n = R.rbc_state_size(h, 0)
        nf, dtf = R.rbc_steps_per_slice(h, 0)
        U = torch.zeros((S + 1) * n, dtype=torch.float64, device=dev)
        R.rbc_init_state(h, w.seed, w.noise_amp, U)
        if args.profile_steps > 0:
            # counter runs serialise every dispatch: the seeded state in every
            # slice instead of the coarse prediction (the work is the same)
            U.view(S + 1, n)[1:] = U.view(S + 1, n)[0]
        else:
            log(f"{w.name}: coarse prediction for the slice states")
            R.parareal_iterate(h, U, 0, 0.0)
        F = U[: S * n].clone()
        del U
        torch.cuda.synchronize()
        if args.profile_steps > 0:
            R.rbc_fine_step_batch(h, F, F, S, args.profile_steps, None)
            torch.cuda.synchronize()
            if args.calibrate_copy > 0:
                a = torch.empty(args.calibrate_copy * (1 << 20) // 8, dtype=torch.float64, device=dev)
                b = torch.empty_like(a)
                a.fill_(1.0)
                torch.mul(a, 1.0, out=b)
                torch.cuda.synchronize()
                del a, b
            log(f"profile mode: {args.profile_steps} batched fine steps done")
            return 0
        # warmup, the x-pass timed with events in its first half
        R.rbc_kernel_timing_enable(h, 1, 1)
        R.rbc_fine_step_batch(h, F, F, S, max(W // 2, 1), None)
        x_ms, x_cnt, x_batch = R.rbc_kernel_timing(h)
        R.rbc_kernel_timing_enable(h, -1, 0)
        R.rbc_fine_step_batch(h, F, F, S, max(W - W // 2, 1), None)
        nus = torch.zeros(S * (K // NU_STRIDE) * R.RBC_DIAG, dtype=torch.float64, device=dev)
        R.rbc_kernel_timing_enable(h, 0, 1)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record(stream)
        R.rbc_fine_step_batch(h, F, F, S, K, nus)
        e1.record(stream)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        ev_ms = e0.elapsed_time(e1)
        k_ms, k_cnt, k_batch = R.rbc_kernel_timing(h)
        R.rbc_kernel_timing_enable(h, -1, 0)
        finite = bool(torch.isfinite(F).all().item()) and bool(torch.isfinite(nus).all().item())
        rec = nus.view(S, -1, R.RBC_DIAG).cpu().numpy()
        log(f"headline: {K} batched steps of {S} slices in {el:.3f} s")
    finally:
        R.rbc_destroy(h)

    dof = w.Nx * w.Nz
    value = S * dof * K / el
    b_bulk = 4 if w.mixed else 8
    s = w.scheme
    stage_b = stage_bytes_per_dof_launch(s, b_bulk) * dof * k_batch
    achieved = stage_b / (k_ms * 1e-3) / 1e9 if k_ms > 0 else 0.0
    step_b = bytes_per_dof_step(s, b_bulk)
    traffic_state = measured_traffic(w.name)
    x_b = xpass_bytes_per_dof_launch(b_bulk) * dof * x_batch
    out = {
        "metric": "fine-step DOF-steps/s (%HBM roofline); Parareal vs serial time-to-solution",
        "value": value,
        "unit": "DOF-steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": 1e3 * el / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if w.mixed else "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "Ra": w.Ra, "Pr": w.Pr, "grid": [w.Nx, w.Nz],
                   "coarse_grid": [w.Nx_c, w.Nz_c], "slices": S, "t": [w.t0, w.t_end], "dt_f": dtf,
                   "fine_steps_per_slice": nf, "scheme": "ARS443" if s == 4 else "ARS222",
                   "nu_stride": NU_STRIDE,
                   "step": "one batched fine step of every slice (all stages: x-pass, forward transform, "
                           "right-hand side, banded solves, inverse transform), Nusselt records every "
                           f"{NU_STRIDE} steps; slice states from the coarse prediction of the seeded state"},
        "roofline": {"bound": "hbm", "kernel": "per-mode stage (fwd_gemm + stage + inv_gemm kernels of one stage)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic_state * k_batch if traffic_state else None,
                     "bytes_per_launch": stage_b, "bytes_per_dof_launch": stage_bytes_per_dof_launch(s, b_bulk),
                     "mean_launch_ms": k_ms, "timed_launches": k_cnt, "slices_per_launch": k_batch},
        "step_roofline": {"bytes_per_dof_step": step_b, "achieved_gbs": step_b * S * dof * K / el / 1e9,
                          "frac": step_b * S * dof * K / el / 1e9 / HBM_PEAK_GBS,
                          "event_ms_per_step": ev_ms / K},
        "xpass": {"mean_launch_ms": x_ms, "timed_launches": x_cnt,
                  "achieved_gbs": x_b / (x_ms * 1e-3) / 1e9 if x_ms > 0 else 0.0,
                  "frac": x_b / (x_ms * 1e-3) / 1e9 / HBM_PEAK_GBS if x_ms > 0 else 0.0},
        "finite": finite,
        "nusselt_last_sample": {"Nu_V_first_slice": float(rec[0, -1, 0]), "Nu_V_last_slice": float(rec[-1, -1, 0])}
        if rec.shape[1] else None,
    }
    if not args.no_parareal:
        out["parareal_c2"] = parareal_leg(I.C2, 3)
    if not args.no_tts:
        out["time_to_solution"] = time_to_solution(I.C2)
    if not args.no_ensemble:
        out["ensemble"] = ensemble_leg()
    if not args.no_serving:
        out["serving"] = serving_leg()
    if args.cpu_seconds > 0:
        log("timing the CPU oracle")
        out["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
