"""The pipelined Parareal iteration (coarse sweep overlapped with the fine
runs on two streams, fine runs of different slices and iterations batched in
one ring) against the sweep-then-batch order of the same library: Eq. 19
fixes every iterate, so the two must agree bit for bit, in the states, the
defects, the Nu histories, the stop iteration and the precision switch.
The sweep-then-batch order itself is checked against the oracle in
test_gpu_parity.py."""
import numpy as np
import pytest
import torch

import rbc_inputs as I
from oracle import rbc_oracle as O

pytestmark = pytest.mark.gpu


def R():
    from paper_2001_01609_amd import rbc
    return rbc


def dev():
    return torch.device("cuda:0")


def case(msg):
    print(f"[case] {msg}", flush=True)


def params(Nx, Nz, Nx_c, Nz_c, S, dt, dt_c, t_end, mixed, Ra=3e3, **kw):
    r = R()
    p = r.rbc_default_params()
    p.Ra, p.Pr, p.Lx, p.Lz = Ra, 1.0, 2.0, 1.0
    p.Nx, p.Nz, p.Nx_c, p.Nz_c = Nx, Nz, Nx_c, Nz_c
    p.n_slices = S
    p.dt_f, p.dt_c = dt, dt_c
    p.t0, p.t_end = 0.0, t_end
    p.scheme_f = p.scheme_c = r.RBC_ARS443
    p.precision = r.RBC_MIXED if mixed else r.RBC_FP64
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def run(p, pipelined, U0, k_max, tol, want_nu):
    p.pipelined = pipelined
    h = R().rbc_create(p, torch.cuda.current_stream(dev()).cuda_stream)
    try:
        n = R().rbc_state_size(h)
        U = torch.zeros((p.n_slices + 1) * n, dtype=torch.float64, device=dev())
        U[:n] = torch.tensor(U0, dtype=torch.float64, device=dev())
        st, kd, defects, nu = R().parareal_iterate(h, U, k_max, tol, want_nu=want_nu)
        kp = R().rbc_fine_fp64_from(h)
        return st, kd, defects, nu, kp, U.cpu().numpy(), R().rbc_stop_reason(h)
    finally:
        R().rbc_destroy(h)


CASES = {
    # FP64 to finite termination: every job of every iteration, ring wrap
    "fp64_to_S": dict(p=dict(Nx=32, Nz=16, Nx_c=16, Nz_c=8, S=5, dt=0.02, dt_c=0.05, t_end=2.5, mixed=False,
                             nu_stride=5, nu_t_start=0.3), k_max=5, tol=0.0),
    # mixed with the FP64 switch (coarse from k+1, fine from k+2): mixed and
    # FP64 jobs in flight together
    "mixed_promote": dict(p=dict(Nx=32, Nz=16, Nx_c=16, Nz_c=8, S=6, dt=0.02, dt_c=0.05, t_end=3.0, mixed=True,
                                 nu_stride=4), k_max=6, tol=1e-14),
    # coarse propagator slower than the fine one (same grid, half the step):
    # the sweep trails the fine runs, the stream waits decide the order
    "slow_coarse": dict(p=dict(Nx=32, Nz=16, Nx_c=32, Nz_c=16, S=7, dt=0.02, dt_c=0.01, t_end=1.4, mixed=False),
                        k_max=4, tol=0.0),
    # stop at a tolerance: the jobs started for the next iteration are
    # abandoned
    "stop_at_tol": dict(p=dict(Nx=32, Nz=16, Nx_c=16, Nz_c=8, S=6, dt=0.02, dt_c=0.05, t_end=3.0, mixed=True,
                               nu_stride=5), k_max=6, tol=1e-3),
    # statistics-based stop
    "stat_stop": dict(p=dict(Nx=32, Nz=16, Nx_c=16, Nz_c=8, S=6, dt=0.02, dt_c=0.05, t_end=3.0, mixed=True,
                             nu_stride=5, stat_tol=0.05), k_max=6, tol=1e-14),
    # split fine path (the transforms as batched GEMMs over the ring's
    # slots, which wrap), mixed with the FP64 switch
    "split_ring": dict(p=dict(Nx=128, Nz=64, Nx_c=32, Nz_c=16, S=5, dt=0.01, dt_c=0.04, t_end=1.0, mixed=True,
                              nu_stride=4), k_max=5, tol=1e-14, env={"RBC_SPLIT": "1"}),
    # prediction only
    "k0": dict(p=dict(Nx=32, Nz=16, Nx_c=16, Nz_c=8, S=4, dt=0.02, dt_c=0.05, t_end=2.0, mixed=False,
                      nu_stride=5), k_max=0, tol=0.0),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_pipelined_equals_sweep_then_batch_bitwise(name, monkeypatch):
    c = CASES[name]
    for k, v in c.get("env", {}).items():
        monkeypatch.setenv(k, v)
    case(f"pipelined vs sweep-then-batch: {name}")
    p = params(**c["p"])
    g = O.Grid(p.Ra, p.Pr, p.Lx, p.Lz, p.Nx, p.Nz, p.dt_f)
    U0 = O.initial_state(g, I.gaussian_noise(31, g.Nx, g.Nz), 0.3).pack()
    want_nu = p.nu_stride > 0
    a = run(params(**c["p"]), 0, U0, c["k_max"], c["tol"], want_nu)
    b = run(params(**c["p"]), 1, U0, c["k_max"], c["tol"], want_nu)
    assert a[0] == b[0] and a[1] == b[1], (a[:2], b[:2])
    assert np.array_equal(a[2], b[2]), (a[2], b[2])
    if want_nu:
        assert np.array_equal(a[3], b[3], equal_nan=True), (a[3], b[3])
    assert a[4] == b[4] and a[6] == b[6]
    assert np.array_equal(a[5], b[5])
    if name == "mixed_promote":
        assert b[4] > 0, "the FP64 switch did not happen"
    if name == "stop_at_tol":
        assert b[1] < p.n_slices and b[2][-1] <= 1e-3


@pytest.mark.parametrize("pipelined", [0, 1])
def test_iterate_history(pipelined):
    """rbc_set_iterate_history: U after the prediction and after every
    iteration; slices 0..k of iterate k equal the serial fine solution bit
    for bit, and the last iterate is the returned state."""
    S = 4
    p = params(32, 16, 16, 8, S, 0.02, 0.05, 2.0, False)
    p.pipelined = pipelined
    case(f"iterate history, pipelined={pipelined}")
    g = O.Grid(p.Ra, p.Pr, p.Lx, p.Lz, p.Nx, p.Nz, p.dt_f)
    U0 = O.initial_state(g, I.gaussian_noise(33, g.Nx, g.Nz), 0.3).pack()
    h = R().rbc_create(p, torch.cuda.current_stream(dev()).cuda_stream)
    try:
        n = R().rbc_state_size(h)
        nf, _ = R().rbc_steps_per_slice(h, 0)
        hist = torch.zeros((S + 1) * (S + 1) * n, dtype=torch.float64, device=dev())
        R().rbc_set_iterate_history(h, hist, S)
        U = torch.zeros((S + 1) * n, dtype=torch.float64, device=dev())
        U[:n] = torch.tensor(U0, dtype=torch.float64, device=dev())
        R().parareal_iterate(h, U, S, 0.0)
        serial = [torch.tensor(U0, dtype=torch.float64, device=dev())]
        for _ in range(S):
            v = serial[-1].clone()
            R().rbc_fine_step_batch(h, v, v, 1, nf)
            serial.append(v)
        H = hist.view(S + 1, S + 1, n).cpu().numpy()
        ser = torch.stack(serial).cpu().numpy()
        u = U.view(S + 1, n).cpu().numpy()
    finally:
        R().rbc_destroy(h)
    for k in range(S + 1):
        for nn in range(k + 1):
            assert np.array_equal(H[k][nn], ser[nn]), (k, nn)
    assert np.array_equal(H[S], u)
    assert not np.array_equal(H[1], H[2])


@pytest.mark.parametrize("env", ["RBC_COARSE_PRIO", "RBC_COARSE_ONE_XCD"])
def test_coarse_launch_placement_changes_no_result(env, monkeypatch):
    """The coarse-grid kernels raise their wave priority and run on one XCD
    (issue order and placement only): the same pipelined run with either
    turned off gives the same states, defects and Nu histories bit for
    bit."""
    c = CASES["mixed_promote"]
    case(f"coarse launch placement: {env} on/off")
    g = O.Grid(3e3, 1.0, 2.0, 1.0, c["p"]["Nx"], c["p"]["Nz"], c["p"]["dt"])
    U0 = O.initial_state(g, I.gaussian_noise(35, g.Nx, g.Nz), 0.3).pack()
    a = run(params(**c["p"]), 1, U0, c["k_max"], c["tol"], True)
    monkeypatch.setenv(env, "0")
    b = run(params(**c["p"]), 1, U0, c["k_max"], c["tol"], True)
    assert a[0] == b[0] and a[1] == b[1] and a[4] == b[4]
    assert np.array_equal(a[2], b[2])
    assert np.array_equal(a[3], b[3], equal_nan=True)
    assert np.array_equal(a[5], b[5])
