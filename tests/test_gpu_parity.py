"""GPU parity: the HIP path through the C ABI against the FP64 oracle on the
same seeded inputs.

Tolerances: the all-FP64 path follows the same arithmetic as the oracle up
to rounding order (banded bordered solves vs dense LU, FFT vs library FFT),
so states agree to ~1e-12 relative; the mixed path (FP32 transforms and
products, FP64 state and solves) must stay within the 1e-6 relative L2 bar
in fields and 1e-4 in Nusselt numbers.
"""
import math
import os

import numpy as np
import pytest

import rbc_inputs as I
from oracle import rbc_oracle as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FP64_TOL = 1e-11
MIXED_TOL = 1e-6


def R():
    from paper_2001_01609_amd import rbc
    return rbc


def dev():
    return torch.device("cuda:0")


def case(msg):
    print(f"[case] {msg}", flush=True)


def params(Nx, Nz, Ra=1e4, dt=1e-3, scheme=4, mixed=False, S=1, Nx_c=None, Nz_c=None, t_end=None,
           dt_c=None, **kw):
    r = R()
    p = r.rbc_default_params()
    p.Ra, p.Pr, p.Lx, p.Lz = Ra, 1.0, 2.0, 1.0
    p.Nx, p.Nz = Nx, Nz
    p.Nx_c, p.Nz_c = Nx_c or Nx, Nz_c or Nz
    p.n_slices = S
    p.dt_f = dt
    p.dt_c = dt_c or dt
    p.t0 = 0.0
    p.t_end = t_end if t_end is not None else dt * S
    p.scheme_f = p.scheme_c = scheme
    p.precision = r.RBC_MIXED if mixed else r.RBC_FP64
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def create(p):
    return R().rbc_create(p, torch.cuda.current_stream(dev()).cuda_stream)


def grid(p, dt=None):
    return O.Grid(p.Ra, p.Pr, p.Lx, p.Lz, p.Nx, p.Nz, dt if dt is not None else p.dt_f, scheme=p.scheme_f)


def oracle_state(g, seed, amp, steps=0):
    X = O.initial_state(g, I.gaussian_noise(seed, g.Nx, g.Nz), amp)
    if steps:
        X = O.Stepper(g).run(X, steps)
    return X


def to_dev(v):
    return torch.tensor(np.asarray(v), dtype=torch.float64, device=dev())


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def band_mask(g):
    """True on the equation rows (the wall-condition rows are zero on the GPU)."""
    m = np.zeros((2, g.Mx, 2, g.Nz), dtype=bool)
    m[0, 0, :, : g.Nz - 2] = True
    m[0, 1:, :, : g.Nz - 4] = True
    m[1, :, :, : g.Nz - 2] = True
    return m.reshape(-1)


# ---------------------------------------------------------------------------

def test_init_state_matches_oracle():
    w = I.C1
    p = R().params_from_workload(w, n_slices=1)
    case(f"init_state {w.Nx}x{w.Nz} seed 0")
    h = create(p)
    try:
        U = torch.zeros(R().rbc_state_size(h), dtype=torch.float64, device=dev())
        R().rbc_init_state(h, 0, 1e-3, U)
        got = U.cpu().numpy()
    finally:
        R().rbc_destroy(h)
    g = grid(p)
    ref = O.initial_state(g, I.gaussian_noise(0, w.Nx, w.Nz), 1e-3).pack()
    assert np.abs(got - ref).max() < 1e-14


@pytest.mark.parametrize("mixed", [False, True])
@pytest.mark.parametrize("Nx,Nz", [(16, 8), (32, 16), (64, 24)])
def test_explicit_terms_match_oracle(Nx, Nz, mixed):
    p = params(Nx, Nz, Ra=1e4, dt=2e-3, mixed=mixed)
    case(f"explicit {Nx}x{Nz} mixed={mixed}")
    g = grid(p)
    X = oracle_state(g, 5, 0.3, steps=10)
    h = create(p)
    try:
        U = to_dev(X.pack())
        E = torch.zeros_like(U)
        R().rbc_explicit_terms(h, U, E)
        torch.cuda.synchronize()
        got = E.cpu().numpy()
    finally:
        R().rbc_destroy(h)
    ref = O.Stepper(g).explicit(X).pack()
    m = band_mask(g)
    err = np.linalg.norm(got[m] - ref[m]) / np.linalg.norm(ref[m])
    assert err < (1e-5 if mixed else 1e-12), err
    assert not got[~m].any()


@pytest.mark.parametrize("scheme", [2, 4])
@pytest.mark.parametrize("Nx,Nz", [(16, 8), (32, 16), (64, 32)])
def test_one_fine_step_fp64(Nx, Nz, scheme):
    p = params(Nx, Nz, Ra=1e5, dt=2e-3, scheme=scheme)
    case(f"one step {Nx}x{Nz} ARS{scheme}")
    g = grid(p)
    X = oracle_state(g, 1, 0.2, steps=5)
    h = create(p)
    try:
        U = to_dev(X.pack())
        R().rbc_fine_step_batch(h, U, U, 1, 1)
        torch.cuda.synchronize()
        got = U.cpu().numpy()
    finally:
        R().rbc_destroy(h)
    ref = O.Stepper(g).step(X).pack()
    assert rel(got, ref) < 1e-13
