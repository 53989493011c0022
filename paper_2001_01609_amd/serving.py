"""Serving loop for Parareal requests on one GPU: continuous batching over
the ensemble engine (rbc_ensemble_* in the C library).

Requests arrive over time, each a Parareal run of section 3.1 (Eq. 19) with
its own Rayleigh number, grid, horizon and defect tolerance.  The scheduler
keeps a FIFO queue and admits the request at its head when a run slot is
free and the run's device footprint (rbc_ensemble_footprint) fits in the
free device memory minus a reserve; admitted runs keep their state on the
device and join the engine at the next iteration boundary, where every
active run advances by one Parareal iteration in shared batched launches.
A finished run leaves, freeing its slot and memory for the queue.  Latency
is arrival to completion; the loop reports throughput and the p50 / p99
latencies beside it.

The scheduler is host logic only: the engine, the free-memory probe and the
clock are injected, so it runs on the CPU against a fake engine in tests.
"""
from __future__ import annotations

import dataclasses
import math
import time
from collections import deque
from typing import Callable, Dict, List

import numpy as np


@dataclasses.dataclass
class Request:
    """One Parareal run to serve.  `params` are the run's rbc_params (or any
    object the engine understands); arrival is in seconds of the loop's
    clock."""
    rid: int
    arrival: float
    params: object
    seed: int
    tol: float
    k_max: int
    cost: float = 0.0          # fine DOF-steps the run's iterations compute (reporting)


@dataclasses.dataclass
class Completed:
    rid: int
    arrival: float
    admitted: float
    finished: float
    k_done: int
    stop: int
    state: int
    defects: List[float]
    result: object = None

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


class Scheduler:
    """FIFO admission by free device memory and run slots; one engine
    iteration per step.

    engine: add(request) -> engine run id; step() -> runs still active;
            poll(run_id) -> (state, k_done, stop, defects) with state 0 while
            active; collect(run_id) -> result (or None); release(run_id).
    free_bytes(): free device memory now.  footprint(request): bytes the
    run needs.  reserve: bytes kept free.  max_active: run slots.
    """

    def __init__(self, engine, free_bytes: Callable[[], int], footprint: Callable[[Request], int],
                 reserve: int = 1 << 30, max_active: int = 32, clock: Callable[[], float] = time.monotonic,
                 keep_results: bool = False):
        self.engine = engine
        self.free_bytes = free_bytes
        self.footprint = footprint
        self.reserve = reserve
        self.max_active = max_active
        self.clock = clock
        self.keep_results = keep_results
        self.queue: deque = deque()
        self.active: Dict[int, tuple] = {}     # engine run id -> (request, admitted time)
        self.done: List[Completed] = []
        self.steps = 0
        self.peak_active = 0
        self.admission_waits = 0               # times the head of the queue waited for memory or a slot

    def submit(self, req: Request) -> None:
        self.queue.append(req)

    def admit(self) -> int:
        """Admits queued requests in order while a slot is free and the head's
        footprint fits; returns how many were admitted."""
        n = 0
        while self.queue:
            req = self.queue[0]
            if len(self.active) >= self.max_active or self.footprint(req) + self.reserve > self.free_bytes():
                self.admission_waits += 1
                break
            self.queue.popleft()
            run_id = self.engine.add(req)
            self.active[run_id] = (req, self.clock())
            n += 1
        self.peak_active = max(self.peak_active, len(self.active))
        return n

    def step(self) -> int:
        """Admission, one engine iteration of every active run, retirement of
        the finished ones.  Returns the number of runs completed."""
        self.admit()
        if not self.active:
            return 0
        self.engine.step()
        self.steps += 1
        now = self.clock()
        finished = 0
        for run_id in list(self.active):
            state, k_done, stop, defects = self.engine.poll(run_id)
            if state == 0:
                continue
            req, admitted = self.active.pop(run_id)
            result = self.engine.collect(run_id) if self.keep_results else None
            self.engine.release(run_id)
            self.done.append(Completed(req.rid, req.arrival, admitted, now, k_done, stop, state, list(defects), result))
            finished += 1
        return finished

    def idle(self) -> bool:
        return not self.queue and not self.active


def serve(requests: List[Request], sched: Scheduler, clock: Callable[[], float] = time.monotonic,
          sleep: Callable[[float], None] = time.sleep, max_steps: int = 100000) -> float:
    """Runs the stream: requests are submitted when the clock passes their
    arrival; the loop steps the scheduler until every request completed.
    Returns the wall time from the first arrival to the last completion."""
    pending = deque(sorted(requests, key=lambda r: r.arrival))
    t0 = clock()
    sched.clock = lambda: clock() - t0
    steps = 0
    while pending or not sched.idle():
        now = clock() - t0
        while pending and pending[0].arrival <= now:
            sched.submit(pending.popleft())
        if sched.idle():
            if pending:
                sleep(max(0.0, pending[0].arrival - (clock() - t0)))
            continue
        sched.step()
        steps += 1
        if steps > max_steps:
            raise RuntimeError("serving loop did not drain")
    return clock() - t0


def latency_report(done: List[Completed], wall: float) -> Dict[str, float]:
    lat = np.array([c.latency for c in done]) if done else np.zeros(1)
    return {"requests": len(done), "wall_s": wall, "requests_per_s": len(done) / wall if wall > 0 else 0.0,
            "latency_p50_s": float(np.percentile(lat, 50)), "latency_p99_s": float(np.percentile(lat, 99)),
            "latency_mean_s": float(lat.mean()), "latency_max_s": float(lat.max())}


def poisson_arrivals(n: int, rate: float, seed: int) -> List[float]:
    """Arrival times of a Poisson process of `rate` per second: exponential
    gaps from the seeded generator (inverse transform of 53-bit uniforms)."""
    import rbc_inputs as I
    u = I.uniform53(seed, np.arange(n, dtype=np.uint64))
    gaps = -np.log1p(-u) / rate
    return list(np.cumsum(gaps) - gaps[0])


class GpuEngine:
    """The scheduler's engine interface over the C library's ensemble: adds
    a run from its seeded initial state (device memory), steps, polls,
    returns and frees results."""

    def __init__(self, stream=None, noise_amp: float = 1e-3):
        import torch

        from paper_2001_01609_amd import rbc as R
        self.R, self.torch = R, torch
        self.dev = torch.device("cuda:0")
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.dev).cuda_stream
        self.e = R.rbc_ensemble_create(self.stream)
        self.noise_amp = noise_amp
        self.sizes: Dict[int, int] = {}

    def add(self, req: Request) -> int:
        R, torch = self.R, self.torch
        p = req.params
        n = 4 * (p.Nx // 2) * p.Nz
        U0 = torch.zeros(n, dtype=torch.float64, device=self.dev)
        R.rbc_initial_state(p, req.seed, self.noise_amp, U0, self.stream)
        rid = R.rbc_ensemble_add(self.e, p, U0, req.k_max, req.tol)
        self.sizes[rid] = (p.n_slices + 1) * n
        return rid

    def step(self) -> int:
        return self.R.rbc_ensemble_step(self.e)

    def poll(self, run_id: int):
        return self.R.rbc_ensemble_run_info(self.e, run_id, 64)

    def collect(self, run_id: int):
        U = self.torch.zeros(self.sizes[run_id], dtype=self.torch.float64, device=self.dev)
        self.R.rbc_ensemble_result(self.e, run_id, U)
        self.torch.cuda.synchronize()
        return U.cpu().numpy()

    def release(self, run_id: int) -> None:
        self.R.rbc_ensemble_release(self.e, run_id)

    def close(self) -> None:
        self.R.rbc_ensemble_destroy(self.e)


# Grid ladder of the request stream and the smallest grid that resolves a
# Rayleigh number (at least 256 x 64 above 1e6, 512 x 128 above 1e7 and
# 1024 x 256 above 1e8 would follow the paper's resolution table; the ladder
# is capped to keep a bench leg short).
REQUEST_GRIDS = ((64, 32), (128, 32), (256, 64), (512, 128))


def request_stream(n: int, rate: float, seed: int = 5000, t_range=(0.05, 0.3), ra_range=(1e4, 1e7),
                   n_slices: int = 16, k_max: int = 3) -> List[dict]:
    """Seeded request descriptions: arrival (Poisson at `rate`), Ra
    log-uniform in ra_range, a grid drawn from the ladder rungs that resolve
    it, horizon uniform in t_range, tolerance 1e-6 or 1e-8 with equal
    probability (1e-8 runs in FP64, which reaches it; 1e-6 in mixed
    precision), fine step 1e-4 * 64 / Nz, coarse grid half, coarse step ten
    times the fine one."""
    import rbc_inputs as I
    arr = poisson_arrivals(n, rate, seed)
    out = []
    for j in range(n):
        u = I.uniform53(seed + 1 + j, np.arange(4, dtype=np.uint64))
        Ra = 10.0 ** (math.log10(ra_range[0]) + (math.log10(ra_range[1]) - math.log10(ra_range[0])) * u[0])
        grids = [g for g in REQUEST_GRIDS if (Ra <= 1e6 or g[1] >= 64) and (Ra <= 1e5 or g[1] >= 32)]
        Nx, Nz = grids[min(int(u[1] * len(grids)), len(grids) - 1)]
        t_end = t_range[0] + (t_range[1] - t_range[0]) * u[2]
        tol = 1e-6 if u[3] < 0.5 else 1e-8
        dt = 1e-4 * 64 / Nz
        out.append(dict(rid=j, arrival=float(arr[j]), Ra=Ra, Nx=Nx, Nz=Nz, t_end=t_end, tol=tol, dt_f=dt,
                        dt_c=10 * dt, n_slices=n_slices, k_max=k_max, seed=seed + 1 + j))
    return out


def make_params(R, d: dict):
    """rbc_params of a request description."""
    p = R.rbc_default_params()
    p.Ra, p.Pr, p.Lx, p.Lz = d["Ra"], 1.0, 2.0, 1.0
    p.Nx, p.Nz, p.Nx_c, p.Nz_c = d["Nx"], d["Nz"], d["Nx"] // 2, d["Nz"] // 2
    p.t0, p.t_end, p.n_slices = 0.0, d["t_end"], d["n_slices"]
    p.dt_f, p.dt_c = d["dt_f"], d["dt_c"]
    p.scheme_f = p.scheme_c = R.RBC_ARS443
    p.precision = R.RBC_MIXED if d["tol"] >= 1e-6 else R.RBC_FP64
    p.promote_fp64 = 0
    p.pipelined = 0
    return p
