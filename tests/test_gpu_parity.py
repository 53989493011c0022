"""GPU parity: the HIP path through the C ABI against the FP64 oracle on the
same seeded inputs.

Tolerances: the all-FP64 path follows the same arithmetic as the oracle up
to rounding order (banded bordered solves vs dense LU, FFT vs library FFT),
so states agree to ~1e-12 relative; the mixed path (FP32 transforms and
products, FP64 state and solves) must stay within the 1e-6 relative L2 bar
in fields and 1e-4 in Nusselt numbers.
"""
import os

import numpy as np
import pytest

import rbc_inputs as I
from oracle import rbc_oracle as O
from parity_util import (NoAdvectionStepper, assert_blocks, assert_sensitive,
                         developed_state)

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
    return O.Grid(p.Ra, p.Pr, p.Lx, p.Lz, p.Nx, p.Nz, dt if dt is not None else p.dt_f, scheme=p.scheme_f,
                  flux=(p.bc_T == R().RBC_BC_FLUX))


def oracle_state(g, seed, amp, steps=0):
    X = O.initial_state(g, I.gaussian_noise(seed, g.Nx, g.Nz), amp)
    if steps:
        X = O.Stepper(g).run(X, steps)
    return X


def to_dev(v):
    return torch.tensor(np.asarray(v), dtype=torch.float64, device=dev())


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


@pytest.mark.parametrize("flux", [False, True])
def test_handle_free_initial_state_equals_handle_initial_state(flux):
    """rbc_initial_state (parameters, seed and stream; no handle, as the
    serving loop uses it) writes the same bits as rbc_init_state on a
    handle of the same parameters."""
    p = params(64, 32, Ra=1e5, dt=1e-3, S=1, bc_T=R().RBC_BC_FLUX if flux else R().RBC_BC_TEMPERATURE)
    case(f"handle-free initial state, {'fixed flux' if flux else 'fixed temperature'}")
    st = torch.cuda.current_stream(dev()).cuda_stream
    h = create(p)
    try:
        n = R().rbc_state_size(h)
        U = torch.zeros(n, dtype=torch.float64, device=dev())
        R().rbc_init_state(h, 77, 0.2, U)
        V = torch.full((n,), float("nan"), dtype=torch.float64, device=dev())
        R().rbc_initial_state(p, 77, 0.2, V, st)
        torch.cuda.synchronize()
        assert np.array_equal(U.cpu().numpy(), V.cpu().numpy())
    finally:
        R().rbc_destroy(h)


@pytest.mark.parametrize("mixed", [False, True])
@pytest.mark.parametrize("Nx,Nz", [(16, 8), (32, 16), (64, 64)])
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
    assert not got[~m].any()
    ref[~m] = 0.0
    assert_blocks(got, ref, g, 1e-5 if mixed else 1e-12, "explicit terms")


@pytest.mark.parametrize("scheme", [2, 4])
@pytest.mark.parametrize("Nx,Nz", [(16, 8), (32, 16), (64, 32), (16, 128), (8, 256)])
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
    assert_blocks(got, ref, g, 1e-13, "one step")


@pytest.mark.parametrize("tile", [None, "6"])
def test_batch_of_slices_many_steps_fp64(tile, monkeypatch):
    """Three slices with different states, 25 steps; a mode tile of 6 gives
    a ragged last tile (Mx = 32)."""
    if tile:
        monkeypatch.setenv("RBC_MODE_TILE", tile)
    p = params(64, 32, Ra=2e4, dt=2e-3, scheme=4, S=3)
    case(f"batch 3 slices 64x32 25 steps tile={tile}")
    g = grid(p)
    Xs = [oracle_state(g, sd, 0.3, steps=3) for sd in (1, 2, 3)]
    h = create(p)
    try:
        U = to_dev(np.concatenate([X.pack() for X in Xs]))
        V = torch.empty_like(U)
        R().rbc_fine_step_batch(h, U, V, 3, 25)
        torch.cuda.synchronize()
        got = V.cpu().numpy().reshape(3, -1)
    finally:
        R().rbc_destroy(h)
    st = O.Stepper(g)
    for i, X in enumerate(Xs):
        assert_blocks(got[i], st.run(X, 25).pack(), g, FP64_TOL, f"slice {i}")


@pytest.mark.parametrize("scheme", [2, 4])
def test_mixed_precision_steps_within_bar(scheme):
    """FP32 transforms/products, FP64 solves: 50 steps within 1e-6 of the
    FP64 oracle, Nusselt numbers within 1e-4."""
    p = params(64, 32, Ra=1e5, dt=2e-3, scheme=scheme, mixed=True, S=2)
    case(f"mixed 64x32 ARS{scheme} 50 steps")
    g = grid(p)
    Xs = [oracle_state(g, sd, 0.3, steps=5) for sd in (7, 8)]
    h = create(p)
    try:
        U = to_dev(np.concatenate([X.pack() for X in Xs]))
        R().rbc_fine_step_batch(h, U, U, 2, 50)
        nu = R().rbc_nusselt(h, U, 2)
        got = U.cpu().numpy().reshape(2, -1)
    finally:
        R().rbc_destroy(h)
    st = O.Stepper(g)
    for i, X in enumerate(Xs):
        Y = st.run(X, 50)
        assert_blocks(got[i], Y.pack(), g, MIXED_TOL, f"slice {i}")
        nref = np.array(O.nusselt(g, Y))
        assert np.all(np.abs(nu[i] - nref) / np.abs(nref) < 1e-4)


def test_nusselt_matches_oracle():
    p = params(32, 16, Ra=1e5, dt=2e-3, S=3)
    case("nusselt 32x16, 3 states")
    g = grid(p)
    Xs = [oracle_state(g, sd, 0.5, steps=20) for sd in (1, 2, 3)]
    Xs[0] = O.conduction_state(g)
    h = create(p)
    try:
        U = to_dev(np.concatenate([X.pack() for X in Xs]))
        nu = R().rbc_nusselt(h, U, 3)
    finally:
        R().rbc_destroy(h)
    for i, X in enumerate(Xs):
        assert np.allclose(nu[i], O.nusselt(g, X), rtol=0, atol=1e-12), (i, nu[i])
    assert np.allclose(nu[0], 1.0, atol=1e-14)


def test_conduction_state_fixed_point_on_gpu():
    for mixed in (False, True):
        p = params(32, 16, Ra=1e6, dt=1e-2, mixed=mixed)
        case(f"conduction fixed point mixed={mixed}")
        g = grid(p)
        X = O.conduction_state(g).pack()
        h = create(p)
        try:
            U = to_dev(X)
            R().rbc_fine_step_batch(h, U, U, 1, 20)
            nu = R().rbc_nusselt(h, U, 1)[0]
            got = U.cpu().numpy()
        finally:
            R().rbc_destroy(h)
        assert np.abs(got - X).max() < 1e-15
        assert np.allclose(nu, 1.0, atol=1e-14)


def test_slice_alone_equals_slice_in_batch_bitwise():
    p = params(32, 16, Ra=1e5, dt=2e-3, S=4, mixed=True)
    case("batch invariance 4 slices")
    g = grid(p)
    Xs = [oracle_state(g, sd, 0.3) for sd in range(4)]
    h = create(p)
    try:
        U = to_dev(np.concatenate([X.pack() for X in Xs]))
        R().rbc_fine_step_batch(h, U, U, 4, 30)
        V = to_dev(Xs[2].pack())
        R().rbc_fine_step_batch(h, V, V, 1, 30)
        torch.cuda.synchronize()
        a = U.cpu().numpy().reshape(4, -1)[2]
        b = V.cpu().numpy()
    finally:
        R().rbc_destroy(h)
    assert np.array_equal(a, b)


# ------------------------------------------------------------ edge cases ---

@pytest.mark.parametrize("mixed", [False, True])
def test_largest_fourier_grid_matches_oracle(mixed):
    """Nx = 2048, the largest grid the library accepts (padded rows of 3072
    points: the x-pass's largest template, one-spectrum rows in FP32), two
    slices of developed flow, three steps, per block against the oracle."""
    p = params(2048, 16, Ra=1e5, dt=1e-3, mixed=mixed, S=2)
    case(f"largest Fourier grid 2048x16, {'mixed' if mixed else 'FP64'}")
    g = grid(p)
    Xs = [developed_state(g, 70 + i) for i in range(2)]
    h = create(p)
    try:
        U = to_dev(np.concatenate([X.pack() for X in Xs]))
        R().rbc_fine_step_batch(h, U, U, 2, 3)
        torch.cuda.synchronize()
        got = U.cpu().numpy().reshape(2, -1)
    finally:
        R().rbc_destroy(h)
    st = O.Stepper(g)
    tol = MIXED_TOL if mixed else FP64_TOL
    for i, X in enumerate(Xs):
        assert_blocks(got[i], st.run(X, 3).pack(), g, tol, f"2048x16 slice {i}", dev_T0=True)


def test_zero_steps_copy_and_batch_bounds():
    """n_steps = 0 copies the input states unchanged; a batch of no slices,
    or of more slices than the handle holds, is rejected before any launch."""
    p = params(32, 16, Ra=1e5, dt=2e-3, S=2)
    case("zero steps, batch bounds")
    g = grid(p)
    X = np.concatenate([oracle_state(g, sd, 0.3).pack() for sd in (1, 2)])
    h = create(p)
    try:
        U = to_dev(X)
        V = torch.zeros_like(U)
        R().rbc_fine_step_batch(h, U, V, 2, 0)
        torch.cuda.synchronize()
        assert np.array_equal(V.cpu().numpy(), X)
        for bad in (0, 3):
            with pytest.raises(R().RbcError) as ei:
                R().rbc_fine_step_batch(h, U, U, bad, 1)
            assert ei.value.status == R().RBC_ERR_ARG
    finally:
        R().rbc_destroy(h)


# ------------------------------------------------------ split fine path ---
# The Chebyshev transforms as batched FP32 MFMA GEMMs around the per-mode
# solve kernel (the default for mixed precision at Nz >= 128; RBC_SPLIT=1
# forces it on smaller eligible grids).

@pytest.mark.parametrize("Nx,Nz", [(128, 64), (128, 128), (128, 256)])
def test_split_explicit_terms_match_oracle(Nx, Nz, monkeypatch):
    monkeypatch.setenv("RBC_SPLIT", "1")
    p = params(Nx, Nz, Ra=1e6, dt=2e-4, mixed=True)
    case(f"split explicit {Nx}x{Nz}")
    g = grid(p)
    X = developed_state(g, 3)
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
    assert not got[~m].any()
    ref[~m] = 0.0
    assert_blocks(got, ref, g, 1e-5, "split explicit terms")


@pytest.mark.parametrize("Nx,Nz,S", [(128, 64, 3), (256, 128, 2)])
def test_split_steps_match_oracle_and_batch_invariance(Nx, Nz, S, monkeypatch):
    """Several slices of developed flow, 8 steps on the split path: each
    slice against the oracle per block (mixed bar), and the last slice
    stepped alone equals itself in the batch, bit for bit."""
    monkeypatch.setenv("RBC_SPLIT", "1")
    p = params(Nx, Nz, Ra=1e6, dt=2e-4, mixed=True, S=S)
    case(f"split steps {Nx}x{Nz} {S} slices")
    g = grid(p)
    Xs = [developed_state(g, 60 + i) for i in range(S)]
    h = create(p)
    try:
        U = to_dev(np.concatenate([X.pack() for X in Xs]))
        R().rbc_fine_step_batch(h, U, U, S, 8)
        V = to_dev(Xs[-1].pack())
        R().rbc_fine_step_batch(h, V, V, 1, 8)
        torch.cuda.synchronize()
        got = U.cpu().numpy().reshape(S, -1)
        alone = V.cpu().numpy()
    finally:
        R().rbc_destroy(h)
    assert np.array_equal(got[-1], alone)
    st = O.Stepper(g)
    for i, X in enumerate(Xs):
        assert_blocks(got[i], st.run(X, 8).pack(), g, MIXED_TOL, f"split slice {i}", dev_T0=True)


def _tiny_parareal_params(mixed=False):
    return params(32, 16, Ra=3e3, dt=0.02, scheme=4, mixed=mixed, S=4, Nx_c=16, Nz_c=8, t_end=2.0,
                  dt_c=0.05)


def test_parareal_matches_oracle_iterates():
    """parareal_iterate vs the oracle's serial Parareal: same iterates (FP64)."""
    p = _tiny_parareal_params()
    case("parareal 32x16 / 16x8, 4 slices vs oracle")
    fine = grid(p)
    coarse = O.Grid(p.Ra, p.Pr, p.Lx, p.Lz, p.Nx_c, p.Nz_c, p.dt_c, scheme=p.scheme_c)
    pp = O.RBCParareal(fine, coarse, p.t0, p.t_end, p.n_slices)
    U0 = O.initial_state(fine, I.gaussian_noise(11, fine.Nx, fine.Nz), 0.3).pack()
    for k_max in (0, 1, 2):
        ref = pp.run(U0, k_max=k_max)
        h = create(p)
        try:
            n = R().rbc_state_size(h)
            U = torch.zeros((p.n_slices + 1) * n, dtype=torch.float64, device=dev())
            U[:n] = to_dev(U0)
            st, kd, defects, _ = R().parareal_iterate(h, U, k_max, 0.0)
            got = U.cpu().numpy().reshape(p.n_slices + 1, -1)
        finally:
            R().rbc_destroy(h)
        assert kd == k_max
        for nn in range(p.n_slices + 1):
            assert_blocks(got[nn], ref.U[nn], fine, FP64_TOL, f"k_max {k_max} slice {nn}")
        assert np.allclose(defects, ref.defects, rtol=1e-8, atol=1e-14)


def test_parareal_exact_on_first_k_slices_bitwise():
    """After k iterations slices 0..k equal the serial fine solve bitwise;
    at k = S the whole trajectory does (finite termination)."""
    p = _tiny_parareal_params(mixed=True)
    p.promote_fp64 = 0          # the serial reference is the mixed propagator itself
    case("parareal finite termination, mixed")
    g = grid(p)
    U0 = O.initial_state(g, I.gaussian_noise(12, g.Nx, g.Nz), 0.3).pack()
    h = create(p)
    try:
        nf, _ = R().rbc_steps_per_slice(h, 0)
        n = R().rbc_state_size(h)
        serial = [to_dev(U0)]
        for s in range(p.n_slices):
            v = serial[-1].clone()
            R().rbc_fine_step_batch(h, v, v, 1, nf)
            serial.append(v)
        ser = torch.stack(serial).cpu().numpy()
        for k in range(0, p.n_slices + 1):
            U = torch.zeros((p.n_slices + 1) * n, dtype=torch.float64, device=dev())
            U[:n] = serial[0]
            st, kd, defects, _ = R().parareal_iterate(h, U, k, 0.0)
            got = U.cpu().numpy().reshape(p.n_slices + 1, -1)
            for nn in range(k + 1):
                assert np.array_equal(got[nn], ser[nn]), (k, nn)
    finally:
        R().rbc_destroy(h)


def test_parareal_reports_nonfinite():
    p = _tiny_parareal_params()
    case("parareal non-finite detection")
    g = grid(p)
    U0 = O.initial_state(g, I.gaussian_noise(13, g.Nx, g.Nz), 0.3).pack()
    U0[5] = np.nan
    h = create(p)
    try:
        n = R().rbc_state_size(h)
        U = torch.zeros((p.n_slices + 1) * n, dtype=torch.float64, device=dev())
        U[:n] = to_dev(U0)
        with pytest.raises(R().RbcError) as ei:
            R().parareal_iterate(h, U, 2, 0.0)
        assert ei.value.status == R().RBC_ERR_NONFINITE
    finally:
        R().rbc_destroy(h)


def test_parareal_stops_at_tolerance_and_tracks_nu():
    p = _tiny_parareal_params()
    p.nu_stride = 5
    p.nu_t_start = 0.5
    case("parareal tolerance stop + Nu history")
    g = grid(p)
    U0 = O.initial_state(g, I.gaussian_noise(14, g.Nx, g.Nz), 0.3).pack()
    h = create(p)
    try:
        n = R().rbc_state_size(h)
        U = torch.zeros((p.n_slices + 1) * n, dtype=torch.float64, device=dev())
        U[:n] = to_dev(U0)
        st, kd, defects, nu = R().parareal_iterate(h, U, 4, 1e-3, want_nu=True)
    finally:
        R().rbc_destroy(h)
    assert st in (R().RBC_OK, R().RBC_NOT_CONVERGED)
    if st == R().RBC_OK and kd < p.n_slices:
        assert defects[-1] <= 1e-3
    assert np.all(np.isfinite(nu[1:]))
    # Nu_V, Nu_b, Nu_t of the fine trajectory are near each other and >= 1
    assert np.all(nu[1:, :3] > 0.99)


# Full workload shapes on developed flow.  Each case runs the kernel
# instantiations of that workload's launches (32 slices of 256x64 at full
# batch: the four-mode per-mode kernel and the four-row x-pass; 64 slices of
# 1024x256; single-slice FP64 runs, the serial FP64 reference stepper) from
# states with O(0.3) rolls, mean shear and mean-temperature bumps, and checks
# the first and last slice block by block.  The oracle with advection
# switched off must differ from the oracle by at least 100x the tolerance in
# every block, so that the comparison can see the nonlinear terms.
FULLSIZE = {
    "ra1e6_256x64_s32_mixed": (I.C2, {}, 4),
    "ra1e6_256x64_s32_fp64": (I.C2_FP64, {}, 4),
    "ra1e6_256x64_serial_fp64": (I.C2_FP64, {"n_slices": 1}, 4),
    "ra1e8_1024x256_s64_mixed": (I.C3, {}, 6),
    "ra1e8_1024x256_serial_fp64": (I.C3, {"n_slices": 1, "precision": 0}, 6),
}
_ORACLE_CACHE = {}


def _oracle_run(g, seed, steps, advect=True):
    """Oracle result of `steps` steps from developed_state(g, seed), cached
    per grid (the 1024x256 stepper is slow to build); BLAS limited to four
    threads (small dense solves run slower on more)."""
    from threadpoolctl import threadpool_limits
    key = (g.Nx, g.Nz, g.dt, g.Ra, seed, steps, advect)
    if key not in _ORACLE_CACHE:
        with threadpool_limits(limits=4):
            skey = (g.Nx, g.Nz, g.dt, g.Ra, advect)
            if skey not in _ORACLE_CACHE:
                _ORACLE_CACHE[skey] = (O.Stepper if advect else NoAdvectionStepper)(g)
            _ORACLE_CACHE[key] = _ORACLE_CACHE[skey].run(developed_state(g, seed), steps).pack()
    return _ORACLE_CACHE[key]


@pytest.mark.parametrize("name", sorted(FULLSIZE))
def test_fullsize_developed_flow_first_and_last_slice(name):
    w, over, steps = FULLSIZE[name]
    p = R().params_from_workload(w, **over)
    mixed = p.precision == R().RBC_MIXED
    S = p.n_slices
    case(f"full size {name}: {S} slices of {p.Nx}x{p.Nz}, {steps} steps, developed flow")
    h = create(p)
    try:
        nf, dt = R().rbc_steps_per_slice(h, 0)
        g = grid(p, dt)
        n = R().rbc_state_size(h)
        seeds = [100 + s for s in range(S)]
        host = np.stack([developed_state(g, sd).pack() for sd in seeds])
        U = to_dev(host.reshape(-1))
        del host
        R().rbc_fine_step_batch(h, U, U, S, steps)
        got = U.view(S, n)[[0, S - 1]].cpu().numpy()
        del U
    finally:
        R().rbc_destroy(h)
    tol = MIXED_TOL if mixed else FP64_TOL
    for i, sd in ((0, seeds[0]), (1, seeds[-1])):
        ref = _oracle_run(g, sd, steps)
        e = assert_blocks(got[i], ref, g, tol, f"{name} slice {'first' if i == 0 else 'last'}", dev_T0=True)
        print(f"[case] {name} seed {sd}: per-block errors {e}", flush=True)
    sens = assert_sensitive(_oracle_run(g, seeds[0], steps), _oracle_run(g, seeds[0], steps, advect=False), g, tol,
                            name)
    print(f"[case] {name}: advection-off differences {sens}", flush=True)


def test_parareal_promotes_stalled_mixed_fine_sweeps_to_fp64():
    """Mixed precision: the defect stalls near the FP32 rounding level; with
    promotion the later fine sweeps run in FP64, the defect reaches a
    tolerance below that floor before finite termination, and the result
    matches the serial all-FP64 fine solve."""
    S, tol = 8, 1e-10
    p = params(32, 16, Ra=5e4, dt=0.01, scheme=4, mixed=True, S=S, t_end=4.0, dt_c=0.04)
    case("parareal FP64 promotion, 8 slices")
    g = grid(p)
    U0 = O.initial_state(g, I.gaussian_noise(21, g.Nx, g.Nz), 0.3).pack()
    h = create(p)
    try:
        n = R().rbc_state_size(h)
        U = torch.zeros((S + 1) * n, dtype=torch.float64, device=dev())
        U[:n] = to_dev(U0)
        st, kd, defects, _ = R().parareal_iterate(h, U, S, tol)
        kp = R().rbc_fine_fp64_from(h)
        got = U.cpu().numpy().reshape(S + 1, -1)[S]
    finally:
        R().rbc_destroy(h)
    assert 2 < kp <= kd, (kp, kd, defects)
    assert kd < S and defects[-1] <= tol, defects
    # serial all-FP64 reference over the whole horizon
    q = params(32, 16, Ra=5e4, dt=0.01, scheme=4, mixed=False, S=S, t_end=4.0, dt_c=0.04)
    h = create(q)
    try:
        nf, _ = R().rbc_steps_per_slice(h, 0)
        V = to_dev(U0)
        for _ in range(S):
            R().rbc_fine_step_batch(h, V, V, 1, nf)
        ref = V.cpu().numpy()
    finally:
        R().rbc_destroy(h)
    # the stop test bounds the change of the whole state vector (1e-10 of a
    # norm the mean temperature dominates); the streamfunction and the
    # temperature rolls are about a hundredth of that norm, so per block the
    # bar is 1e-7 (without the switch the mixed floor leaves them near 1e-5)
    assert_blocks(got, ref, g, 1e-7, "promoted Parareal vs serial FP64")


# ------------------------------------------- consistency checks (section 2.2) ---

@pytest.mark.parametrize("Nx,Nz", [(32, 16), (64, 8), (64, 64), (8, 256)])
def test_diagnostic_records_match_oracle(Nx, Nz):
    """rbc_diagnostics (exact Chebyshev product integrals on the GPU) against
    the oracle's quadratures: Nu_V, Nu_b, Nu_t, KE, epsilon_U, P; one
    partly filled mode chunk (32x16, 64x8) and several chunks (64x64,
    8x256)."""
    p = params(Nx, Nz, Ra=1e5, dt=2e-3, S=3)
    case(f"diagnostics {Nx}x{Nz}, 3 states")
    g = grid(p)
    Xs = [oracle_state(g, sd, 0.5, steps=5) for sd in (4, 5)] + [O.conduction_state(g)]
    h = create(p)
    try:
        U = to_dev(np.concatenate([X.pack() for X in Xs]))
        d = R().rbc_diagnostics(h, U, 3)
    finally:
        R().rbc_destroy(h)
    for i, X in enumerate(Xs):
        ref = O.diagnostics(g, X)
        tol = 1e-11 * np.maximum(np.abs(ref), [1, 1, 1, 0, 0, 0]) + 1e-16
        assert np.all(np.abs(d[i] - ref) <= tol), (i, d[i], ref)
    assert np.allclose(d[2], [1, 1, 1, 0, 0, 0], atol=1e-14)


def test_parareal_time_averages_follow_the_definitions():
    """After finite termination (k = S) the averaged records of the last
    iteration are those of the serial fine run: samples from
    rbc_fine_step_batch, averaged by the oracle's definitions of Re, Nu_int
    and the balance check."""
    p = _tiny_parareal_params()
    p.nu_stride = 5
    S = p.n_slices
    case("parareal time averages vs oracle definitions")
    g = grid(p)
    U0 = O.initial_state(g, I.gaussian_noise(16, g.Nx, g.Nz), 0.3).pack()
    h = create(p)
    try:
        n = R().rbc_state_size(h)
        nf, dt = R().rbc_steps_per_slice(h, 0)
        U = torch.zeros((S + 1) * n, dtype=torch.float64, device=dev())
        U[:n] = to_dev(U0)
        st, kd, defects, avg = R().parareal_iterate(h, U, S, 0.0, want_nu=True)
        assert kd == S and R().rbc_stop_reason(h) == R().RBC_STOP_EXACT
        V = to_dev(U0)
        rec = []
        for _ in range(S):
            smp = torch.zeros((nf // 5) * 6, dtype=torch.float64, device=dev())
            R().rbc_fine_step_batch(h, V, V, 1, nf, smp)
            rec.append(smp.view(-1, 6).cpu().numpy())
    finally:
        R().rbc_destroy(h)
    ref = O.time_averages(grid(p, dt), np.concatenate(rec))
    assert np.allclose(avg[S], ref, rtol=1e-12, atol=1e-15), (avg[S], ref)


def test_parareal_statistics_based_stop():
    """A loose stat_tol stops the iteration once the averaged Nusselt
    numbers settle, before the defect criterion; the reason is reported."""
    p = _tiny_parareal_params()
    p.nu_stride = 5
    p.stat_tol = 0.05
    case("parareal statistics-based stop")
    g = grid(p)
    U0 = O.initial_state(g, I.gaussian_noise(17, g.Nx, g.Nz), 0.3).pack()
    h = create(p)
    try:
        n = R().rbc_state_size(h)
        U = torch.zeros((p.n_slices + 1) * n, dtype=torch.float64, device=dev())
        U[:n] = to_dev(U0)
        st, kd, defects, avg = R().parareal_iterate(h, U, p.n_slices, 1e-14, want_nu=True)
        reason = R().rbc_stop_reason(h)
    finally:
        R().rbc_destroy(h)
    assert st == R().RBC_OK and reason == R().RBC_STOP_STATISTICS, (st, reason, kd, avg[:, :3])
    assert 1 <= kd < p.n_slices
    assert np.all(np.abs(avg[kd, :3] - avg[kd - 1, :3]) <= 0.05 * np.abs(avg[kd, :3]))



# ---------------------------------------------- fixed-flux walls (Eq. 7) ---

def test_init_state_fixed_flux_matches_oracle():
    p = params(32, 16, Ra=1e5, dt=2e-3, bc_T=R().RBC_BC_FLUX)
    case("init_state fixed flux")
    h = create(p)
    try:
        U = torch.zeros(R().rbc_state_size(h), dtype=torch.float64, device=dev())
        R().rbc_init_state(h, 3, 1e-2, U)
        got = U.cpu().numpy()
    finally:
        R().rbc_destroy(h)
    g = grid(p)
    ref = O.initial_state(g, I.gaussian_noise(3, g.Nx, g.Nz), 1e-2).pack()
    assert np.abs(got - ref).max() < 1e-14


@pytest.mark.parametrize("Nx,Nz,mixed", [(16, 8, False), (32, 16, False), (64, 32, False), (32, 16, True)])
def test_steps_fixed_flux_match_oracle(Nx, Nz, mixed):
    """Fixed-flux walls: 5 fine steps and the diagnostic record against the
    oracle (FP64 1e-12, mixed 1e-6)."""
    p = params(Nx, Nz, Ra=2e4, dt=5e-3, mixed=mixed, bc_T=R().RBC_BC_FLUX)
    case(f"fixed flux {Nx}x{Nz} mixed={mixed}")
    g = grid(p)
    X = oracle_state(g, 7, 0.3, steps=3)
    h = create(p)
    try:
        U = to_dev(X.pack())
        R().rbc_fine_step_batch(h, U, U, 1, 5)
        d = R().rbc_diagnostics(h, U, 1)[0]
        got = U.cpu().numpy()
    finally:
        R().rbc_destroy(h)
    Y = O.Stepper(g).run(X, 5)
    assert_blocks(got, Y.pack(), g, 1e-6 if mixed else 1e-12, "fixed flux")
    ref = O.diagnostics(g, Y)
    tol = (1e-5 if mixed else 1e-11) * np.maximum(np.abs(ref), [1, 1, 1, 0, 0, 0]) + 1e-16
    assert np.all(np.abs(d - ref) <= tol), (d, ref)
    # the wall slope stays -1 in the mean profile: Nu_b = Nu_t = 1 / dT
    assert abs(d[1] - d[2]) < 1e-10


def test_conduction_state_fixed_point_fixed_flux_on_gpu():
    for mixed in (False, True):
        p = params(32, 16, Ra=1e5, dt=1e-2, mixed=mixed, bc_T=R().RBC_BC_FLUX)
        case(f"fixed-flux conduction fixed point mixed={mixed}")
        g = grid(p)
        X = O.conduction_state(g).pack()
        h = create(p)
        try:
            U = to_dev(X)
            R().rbc_fine_step_batch(h, U, U, 1, 20)
            nu = R().rbc_nusselt(h, U, 1)[0]
            got = U.cpu().numpy()
        finally:
            R().rbc_destroy(h)
        # the slope wall row weighs coefficients by n^2: rounding, not drift
        assert np.abs(got - X).max() < 1e-13
        assert np.allclose(nu, 1.0, atol=1e-13)


def test_parareal_fixed_flux_matches_oracle_iterates():
    p = params(32, 16, Ra=3e3, dt=0.02, scheme=4, S=4, Nx_c=16, Nz_c=8, t_end=2.0, dt_c=0.05,
               bc_T=R().RBC_BC_FLUX)
    case("parareal fixed flux vs oracle")
    fine = grid(p)
    coarse = O.Grid(p.Ra, p.Pr, p.Lx, p.Lz, p.Nx_c, p.Nz_c, p.dt_c, scheme=p.scheme_c, flux=True)
    pp = O.RBCParareal(fine, coarse, p.t0, p.t_end, p.n_slices)
    U0 = O.initial_state(fine, I.gaussian_noise(19, fine.Nx, fine.Nz), 0.3).pack()
    ref = pp.run(U0, k_max=2)
    h = create(p)
    try:
        n = R().rbc_state_size(h)
        U = torch.zeros((p.n_slices + 1) * n, dtype=torch.float64, device=dev())
        U[:n] = to_dev(U0)
        st, kd, defects, _ = R().parareal_iterate(h, U, 2, 0.0)
        got = U.cpu().numpy().reshape(p.n_slices + 1, -1)
    finally:
        R().rbc_destroy(h)
    for nn in range(p.n_slices + 1):
        assert_blocks(got[nn], ref.U[nn], fine, FP64_TOL, f"slice {nn}")
    assert np.allclose(defects, ref.defects, rtol=1e-8, atol=1e-14)


def test_c1_parareal_to_finite_termination_matches_stored_oracle_samples():
    """The 64x32, 4-slice FP64 workload (Ra 1e4, ARS222, t in [0, 10], the
    coarse propagator on the same grid at ten times the step), Parareal to
    k = 4: the defects, and for every iterate and slice boundary the L2 norm
    and 16 coefficients, against the oracle's (tests/golden/c1_parareal.json,
    written by tests/golden/make_c1_parareal.py from the oracle alone; the
    oracle needs minutes for this run), each block of the state (psi, T for
    m >= 1, T for m = 0) relative to its own norm.  Bound: the FP64 bar of 1e-11 of
    the slice norm; over the four slices the oracle amplifies a
    rounding-level perturbation of the initial state at most ~6 times.  The
    coarse propagator shares the fine grid, so after the first iteration
    (4.5e-10) the defects are rounding noise (~1e-14) on both sides."""
    import json
    with open(os.path.join(os.path.dirname(__file__), "golden", "c1_parareal.json")) as f:
        gold = json.load(f)
    w = I.C1
    p = R().params_from_workload(w)
    S = p.n_slices
    case(f"{w.name}: Parareal to k = {S} vs stored oracle samples")
    g = grid(p)
    U0 = O.initial_state(g, I.gaussian_noise(w.seed, g.Nx, g.Nz), w.noise_amp).pack()
    h = create(p)
    try:
        n = R().rbc_state_size(h)
        hist = torch.zeros((S + 1) * (S + 1) * n, dtype=torch.float64, device=dev())
        R().rbc_set_iterate_history(h, hist, S)
        U = torch.zeros((S + 1) * n, dtype=torch.float64, device=dev())
        U[:n] = to_dev(U0)
        st, kd, defects, _ = R().parareal_iterate(h, U, S, 0.0)
        H = hist.view(S + 1, S + 1, n).cpu().numpy()
    finally:
        R().rbc_destroy(h)
    assert kd == gold["k_done"] == S
    ref_d = np.array(gold["defects"])
    # a difference of two states 4.5e-10 apart: relative accuracy ~1e-15 / 4.5e-10
    assert abs(defects[0] - ref_d[0]) <= 1e-4 * ref_d[0], (defects, ref_d)
    assert np.all(np.asarray(defects[1:]) < 1e-12) and np.all(ref_d[1:] < 1e-12), (defects, ref_d)
    tol = FP64_TOL
    for name, blk in gold["blocks"].items():
        a, b = blk["range"]
        pos = np.array(blk["positions"])
        for k in range(S + 1):
            for nn in range(S + 1):
                ref_norm = blk["norms"][k][nn]
                got = H[k][nn]
                assert abs(np.linalg.norm(got[a:b]) - ref_norm) <= tol * ref_norm, (name, k, nn)
                err = np.max(np.abs(got[pos] - np.array(blk["samples"][k][nn])))
                assert err <= tol * ref_norm, (name, k, nn, err / ref_norm)
