"""Host logic of the serving loop (no GPU): FIFO admission by free device
memory and run slots, continuous batching at iteration boundaries,
retirement, latency accounting, the seeded arrival process and the request
stream's grid rule; against a fake engine and an injected memory probe."""
import numpy as np

from paper_2001_01609_amd import serving as SV


class FakeEngine:
    """Each run needs `params` iterations; memory is the sum of the active
    runs' footprints; every step advances a simulated clock."""

    def __init__(self, clock, dt=1.0):
        self.clock, self.dt = clock, dt
        self.runs = {}
        self.next = 0
        self.log = []

    def add(self, req):
        rid = self.next
        self.next += 1
        self.runs[rid] = [req, 0]
        self.log.append(("add", req.rid, self.clock.t))
        return rid

    def step(self):
        self.clock.t += self.dt
        for r in self.runs.values():
            r[1] += 1
        self.log.append(("step", sorted(r[0].rid for r in self.runs.values())))
        return sum(1 for r in self.runs.values() if r[1] < r[0].params)

    def poll(self, rid):
        req, k = self.runs[rid]
        return (1 if k >= req.params else 0), k, 2, [0.1] * k

    def collect(self, rid):
        return self.runs[rid][1]

    def release(self, rid):
        del self.runs[rid]


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


def req(rid, arrival, iters, mem=10):
    r = SV.Request(rid=rid, arrival=arrival, params=iters, seed=rid, tol=1e-6, k_max=iters)
    r.mem = mem
    return r


def test_admission_waits_for_memory_and_keeps_fifo_order():
    clock = Clock()
    eng = FakeEngine(clock)
    total = 100
    used = lambda: sum(r[0].mem for r in eng.runs.values())
    s = SV.Scheduler(eng, free_bytes=lambda: total - used(), footprint=lambda r: r.mem, reserve=0,
                     max_active=10, clock=clock)
    s.submit(req(0, 0.0, 3, mem=60))
    s.submit(req(1, 0.0, 1, mem=50))   # does not fit beside run 0
    s.submit(req(2, 0.0, 1, mem=5))    # would fit, but waits behind run 1 (FIFO)
    s.step()
    assert [r[0].rid for r in eng.runs.values()] == [0]
    assert s.admission_waits >= 1
    s.step()
    s.step()                            # run 0 finishes after its third iteration
    assert [c.rid for c in s.done] == [0]
    s.step()                            # now runs 1 and 2 are admitted together
    adds = [e for e in eng.log if e[0] == "add"]
    assert [a[1] for a in adds] == [0, 1, 2] and adds[1][2] == adds[2][2] == 3.0
    assert sorted(c.rid for c in s.done) == [0, 1, 2]
    assert s.idle()


def test_run_slots_limit_concurrency_and_requests_join_between_iterations():
    clock = Clock()
    eng = FakeEngine(clock)
    s = SV.Scheduler(eng, free_bytes=lambda: 1 << 40, footprint=lambda r: 1, reserve=0, max_active=2, clock=clock)
    for i in range(4):
        s.submit(req(i, 0.0, 2))
    while not s.idle():
        s.step()
        assert len(eng.runs) <= 2
    assert s.peak_active == 2
    steps = [e[1] for e in eng.log if e[0] == "step"]
    assert steps[0] == [0, 1] and [2, 3] in steps


def test_serve_drains_a_stream_and_reports_latency():
    clock = Clock()
    eng = FakeEngine(clock, dt=0.5)
    s = SV.Scheduler(eng, free_bytes=lambda: 1 << 40, footprint=lambda r: 1, reserve=0, max_active=8)
    reqs = [req(i, a, 1 + i % 3) for i, a in enumerate([0.0, 0.2, 0.9, 3.0, 3.1])]

    def sleep(dt):
        clock.t += dt

    wall = SV.serve(reqs, s, clock=clock, sleep=sleep)
    assert sorted(c.rid for c in s.done) == list(range(5))
    for c in s.done:
        assert c.finished >= c.arrival and c.latency > 0
        assert c.k_done == 1 + c.rid % 3
    rep = SV.latency_report(s.done, wall)
    lat = sorted(c.latency for c in s.done)
    assert rep["requests"] == 5 and abs(rep["latency_p50_s"] - lat[2]) < 1e-12
    assert lat[3] <= rep["latency_p99_s"] <= lat[4]


def test_poisson_arrivals_have_the_requested_rate():
    a = np.array(SV.poisson_arrivals(20000, 4.0, seed=7))
    gaps = np.diff(a)
    assert a[0] == 0.0 and np.all(gaps >= 0)
    assert abs(gaps.mean() - 0.25) < 0.01 and abs(gaps.std() - 0.25) < 0.01   # exponential: mean = std


def test_request_stream_resolves_each_rayleigh_number():
    reqs = SV.request_stream(200, 5.0, seed=11)
    for d in reqs:
        if d["Ra"] > 1e6:
            assert d["Nz"] >= 64
        assert d["tol"] in (1e-6, 1e-8) and 0.05 <= d["t_end"] <= 0.3
        assert abs(d["dt_f"] - 1e-4 * 64 / d["Nz"]) < 1e-18 and d["dt_c"] == 10 * d["dt_f"]
    assert {d["tol"] for d in reqs} == {1e-6, 1e-8}
    assert len({(d["Nx"], d["Nz"]) for d in reqs}) >= 3
