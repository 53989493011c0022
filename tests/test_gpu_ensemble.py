"""Ensembles of independent Parareal runs (rbc_ensemble_*): runs of
different grids, Rayleigh numbers, steps, horizons and precisions advanced
together, with runs that share a grid shape batched into one launch per
stage.  Every run must equal, bit for bit, the same run on its own handle
(parareal_iterate, sweep-then-batch order, no FP64 switch): iterates,
defects and stop.  A run added after the others have started (continuous
batching) as well.  One FP64 run is checked against the oracle's
Parareal (section 3.1, Eq. 19)."""
import numpy as np
import pytest
import torch

import rbc_inputs as I
from oracle import rbc_oracle as O
from parity_util import assert_blocks

pytestmark = pytest.mark.gpu


def R():
    from paper_2001_01609_amd import rbc
    return rbc


def dev():
    return torch.device("cuda:0")


def case(msg):
    print(f"[case] {msg}", flush=True)


def params(Nx, Nz, Nx_c, Nz_c, Ra, S, t_end, dt, dt_c, mixed, scheme=4):
    r = R()
    p = r.rbc_default_params()
    p.Ra, p.Pr, p.Lx, p.Lz = Ra, 1.0, 2.0, 1.0
    p.Nx, p.Nz, p.Nx_c, p.Nz_c = Nx, Nz, Nx_c, Nz_c
    p.n_slices = S
    p.t0, p.t_end = 0.0, t_end
    p.dt_f, p.dt_c = dt, dt_c
    p.scheme_f = p.scheme_c = scheme
    p.precision = r.RBC_MIXED if mixed else r.RBC_FP64
    p.promote_fp64 = 0
    p.pipelined = 0
    return p


# (params, seed, k_max, tol); runs 1 and 3 share their fine and coarse grid
# shapes (one batch) with different Rayleigh numbers, steps and horizons
RUNS = [
    (dict(Nx=32, Nz=16, Nx_c=16, Nz_c=8, Ra=3e3, S=4, t_end=2.0, dt=0.02, dt_c=0.05, mixed=False), 11, 3, 0.0),
    (dict(Nx=64, Nz=32, Nx_c=32, Nz_c=16, Ra=2e4, S=5, t_end=0.5, dt=4e-3, dt_c=2e-2, mixed=True), 12, 3, 0.0),
    (dict(Nx=128, Nz=64, Nx_c=64, Nz_c=32, Ra=1e5, S=4, t_end=0.08, dt=1e-3, dt_c=4e-3, mixed=True), 13, 2, 0.0),
    (dict(Nx=64, Nz=32, Nx_c=32, Nz_c=16, Ra=7e4, S=5, t_end=0.6, dt=5e-3, dt_c=2.5e-2, mixed=True), 14, 4, 1e-3),
]
LATE = (dict(Nx=64, Nz=32, Nx_c=32, Nz_c=16, Ra=4e4, S=5, t_end=0.4, dt=4e-3, dt_c=2e-2, mixed=True), 15, 3, 0.0)


def initial(p, seed):
    g = O.Grid(p.Ra, p.Pr, p.Lx, p.Lz, p.Nx, p.Nz, p.dt_f)
    return O.initial_state(g, I.gaussian_noise(seed, g.Nx, g.Nz), 0.3).pack()


def alone(p, U0, k_max, tol):
    r = R()
    h = r.rbc_create(p, torch.cuda.current_stream(dev()).cuda_stream)
    try:
        n = r.rbc_state_size(h)
        U = torch.zeros((p.n_slices + 1) * n, dtype=torch.float64, device=dev())
        U[:n] = torch.tensor(U0, dtype=torch.float64, device=dev())
        st, kd, defects, _ = r.parareal_iterate(h, U, k_max, tol)
        return kd, defects, U.cpu().numpy(), r.rbc_stop_reason(h)
    finally:
        r.rbc_destroy(h)


def test_ensemble_runs_equal_runs_alone_bitwise():
    r = R()
    specs = [(params(**pp), sd, km, tol) for pp, sd, km, tol in RUNS]
    late = (params(**LATE[0]), LATE[1], LATE[2], LATE[3])
    e = r.rbc_ensemble_create(torch.cuda.current_stream(dev()).cuda_stream)
    try:
        ids = []
        for p, sd, km, tol in specs:
            U0 = torch.tensor(initial(p, sd), dtype=torch.float64, device=dev())
            ids.append(r.rbc_ensemble_add(e, p, U0, km, tol))
        case("ensemble: first step (predictions)")
        left = r.rbc_ensemble_step(e)
        assert left == len(specs)
        U0 = torch.tensor(initial(late[0], late[1]), dtype=torch.float64, device=dev())
        ids.append(r.rbc_ensemble_add(e, late[0], U0, late[2], late[3]))
        specs.append(late)
        steps = 1
        while left > 0:
            left = r.rbc_ensemble_step(e)
            steps += 1
            assert steps < 20
        got = []
        for rid, (p, sd, km, tol) in zip(ids, specs):
            st, kd, stop, defects = r.rbc_ensemble_run_info(e, rid, km)
            n = (p.n_slices + 1) * 4 * (p.Nx // 2) * p.Nz
            U = torch.zeros(n, dtype=torch.float64, device=dev())
            r.rbc_ensemble_result(e, rid, U)
            torch.cuda.synchronize()
            got.append((st, kd, stop, defects, U.cpu().numpy()))
            r.rbc_ensemble_release(e, rid)
    finally:
        r.rbc_ensemble_destroy(e)
    for i, ((p, sd, km, tol), (st, kd, stop, defects, U)) in enumerate(zip(specs, got)):
        case(f"ensemble run {i}: {p.Nx}x{p.Nz} Ra {p.Ra:g} vs alone")
        kd0, d0, U0, stop0 = alone(p, initial(p, sd), km, tol)
        assert st == R().ENSEMBLE_DONE
        assert kd == kd0 and stop == stop0, (i, kd, kd0, stop, stop0)
        assert np.array_equal(defects, d0[:kd]), (i, defects, d0)
        assert np.array_equal(U, U0), i
    # the tolerance run stopped on its defect
    assert got[3][2] == R().RBC_STOP_DEFECT


def test_ensemble_fp64_run_matches_oracle_parareal():
    r = R()
    pp, sd, km, tol = RUNS[0]
    p = params(**pp)
    U0 = initial(p, sd)
    fine = O.Grid(p.Ra, p.Pr, p.Lx, p.Lz, p.Nx, p.Nz, p.dt_f, scheme=p.scheme_f)
    coarse = O.Grid(p.Ra, p.Pr, p.Lx, p.Lz, p.Nx_c, p.Nz_c, p.dt_c, scheme=p.scheme_c)
    ref = O.RBCParareal(fine, coarse, p.t0, p.t_end, p.n_slices).run(U0, k_max=2)
    e = r.rbc_ensemble_create(torch.cuda.current_stream(dev()).cuda_stream)
    try:
        rid = r.rbc_ensemble_add(e, p, torch.tensor(U0, dtype=torch.float64, device=dev()), 2, 0.0)
        other = params(**RUNS[1][0])
        r.rbc_ensemble_add(e, other, torch.tensor(initial(other, 12), dtype=torch.float64, device=dev()), 3, 0.0)
        case("ensemble FP64 run vs oracle Parareal, k = 2")
        while r.rbc_ensemble_step(e) > 0:
            pass
        n = (p.n_slices + 1) * 4 * (p.Nx // 2) * p.Nz
        U = torch.zeros(n, dtype=torch.float64, device=dev())
        r.rbc_ensemble_result(e, rid, U)
        st, kd, stop, defects = r.rbc_ensemble_run_info(e, rid, 2)
        got = U.cpu().numpy().reshape(p.n_slices + 1, -1)
    finally:
        r.rbc_ensemble_destroy(e)
    assert kd == 2
    for nn in range(p.n_slices + 1):
        assert_blocks(got[nn], ref.U[nn], fine, 1e-11, f"slice {nn}")
    assert np.allclose(defects, ref.defects, rtol=1e-8, atol=1e-14)
