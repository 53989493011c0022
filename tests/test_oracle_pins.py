"""Pins of the FP64 oracle against facts fixed outside it (no GPU needed).

Each test ties one part of the oracle to the mathematics or to a value
printed or cited by the paper, so that a dropped term, a wrong sign or a
transposed operand in the oracle fails at least one of them.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.fft
import scipy.integrate
import scipy.linalg
import scipy.special

import rbc_inputs as I
from oracle import rbc_oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- inputs ---

def test_splitmix64_reference_outputs():
    """Seeded generator = the published SplitMix64 reference outputs."""
    with open(os.path.join(GOLD, "splitmix64.json")) as f:
        cases = json.load(f)["cases"]
    for c in cases:
        got = [int(v) for v in I.splitmix64(c["seed"], np.arange(3))]
        want = [int(s, 0) for s in c["outputs"]]
        assert got == want


def test_gaussian_noise_moments():
    xi = I.gaussian_noise(7, 256, 64)
    assert abs(xi.mean()) < 0.02 and abs(xi.std() - 1.0) < 0.02
    assert np.array_equal(xi, I.gaussian_noise(7, 256, 64))
    assert not np.array_equal(xi, I.gaussian_noise(8, 256, 64))


# ------------------------------------------------------- transforms (P2) ---

def test_chebyshev_transform_matches_scipy_dct():
    """Forward transform on Gauss points = DCT-II, inverse = DCT-III
    (scipy.fft), up to the stated normalisation."""
    rng = np.random.default_rng(0)
    M = 24
    f = rng.standard_normal(M)
    c = O.cheb_forward_matrix(M, M) @ f
    ref = scipy.fft.dct(f, type=2) / M
    ref[0] *= 0.5
    assert np.allclose(c, ref, rtol=0, atol=1e-14)
    back = O.cheb_eval_matrix(M, M) @ c
    assert np.allclose(back, f, rtol=0, atol=1e-13)
    # the Gauss points are the DCT-II nodes, ordered with zeta decreasing
    z = O.gauss_points(M)
    assert np.all(np.diff(z) < 0)


@pytest.mark.parametrize("Nz", [8, 17, 32])
def test_chebyshev_derivative_exact_on_polynomials(Nz):
    """d/dz of a degree < Nz polynomial is exact (z in [0, Lz])."""
    rng = np.random.default_rng(Nz)
    Lz = 1.7
    p = np.polynomial.Polynomial(rng.standard_normal(Nz))   # power basis in z
    z = (O.gauss_points(Nz) + 1) * Lz / 2
    c = O.cheb_forward_matrix(Nz, Nz) @ p(z)
    zt = np.linspace(0, Lz, 11)
    zeta = 2 * zt / Lz - 1
    for order in (1, 2, 3):
        d = c
        for _ in range(order):
            d = O.cheb_deriv(d, 2.0 / Lz)
        got = np.polynomial.chebyshev.chebval(zeta, d)
        want = p.deriv(order)(zt)
        assert np.allclose(got, want, rtol=1e-9, atol=1e-9 * np.abs(want).max())


def test_ultraspherical_operators_against_gegenbauer():
    """D_lam maps T-series to C^(lam)-series of the lam-th derivative and
    S_lam converts C^(lam) to C^(lam+1) (scipy.special Gegenbauer)."""
    rng = np.random.default_rng(1)
    N = 14
    c = np.zeros(N)
    c[: N - 4] = rng.standard_normal(N - 4)      # room for the +2 / +4 shifts
    zeta = np.linspace(-0.95, 0.95, 9)
    n = np.arange(N)

    def tser(a):
        return np.polynomial.chebyshev.chebval(zeta, a)

    def cser(lam, a):
        return sum(a[i] * scipy.special.eval_gegenbauer(i, lam, zeta) for i in range(N))

    for lam in (1, 2, 3, 4):
        d = np.polynomial.chebyshev.chebder(c, lam)
        want = np.polynomial.chebyshev.chebval(zeta, d)
        got = cser(lam, O.op_D(lam, N, 1.0) @ c)
        assert np.allclose(got, want, rtol=1e-10, atol=1e-10 * np.abs(want).max())
    assert np.allclose(cser(1, O.op_S0(N) @ c), tser(c), atol=1e-12)
    a = rng.standard_normal(N)
    a[N - 2:] = 0
    for lam in (1, 2, 3):
        assert np.allclose(cser(lam + 1, O.op_S(lam, N) @ a), cser(lam, a), atol=1e-11)
    # D_lam scales with (2/Lz)^lam
    assert np.allclose(O.op_D(2, N, 2.0), 4.0 * O.op_D(2, N, 1.0))
    del n


def test_fourier_synthesis_matches_direct_sum():
    """to_grid evaluates f_0 + 2 Re sum_m f_m exp(i k_m x) at x_i = i Lx / P."""
    rng = np.random.default_rng(2)
    Mx, N, P, M = 5, 4, 15, 6
    c = rng.standard_normal((Mx, N)) + 1j * rng.standard_normal((Mx, N))
    c[0] = c[0].real
    Lx = 2.0
    g = O.to_grid(c, P, M)
    x = np.arange(P) * Lx / P
    k = 2 * np.pi * np.arange(Mx) / Lx
    zv = c @ O.cheb_eval_matrix(M, N).T            # [Mx, M]
    want = zv[0].real[None, :] + 2 * np.real(np.exp(1j * np.outer(x, k[1:])) @ zv[1:])
    assert np.allclose(g, want, atol=1e-13)
    back = O.from_grid(g, Mx, N)
    assert np.allclose(back, c, atol=1e-13)


# ------------------------------------------------------ dealiasing (P3) ---

def _exact_product_coeffs(a, b, Mx, Nz):
    """Brute-force product of two band-limited (Fourier x Chebyshev) fields:
    full convolution over +-m and numpy's chebmul, then truncation."""
    def full(c):
        d = {0: c[0]}
        for m in range(1, c.shape[0]):
            d[m] = c[m]
            d[-m] = np.conj(c[m])
        return d
    A, B = full(a), full(b)
    out = np.zeros((Mx, Nz), dtype=complex)
    for m in range(Mx):
        acc = np.zeros(2 * Nz, dtype=complex)
        for m1, ca in A.items():
            m2 = m - m1
            if m2 in B:
                pr = (np.polynomial.chebyshev.chebmul(ca.real, B[m2].real)
                      - np.polynomial.chebyshev.chebmul(ca.imag, B[m2].imag)
                      + 1j * (np.polynomial.chebyshev.chebmul(ca.real, B[m2].imag)
                              + np.polynomial.chebyshev.chebmul(ca.imag, B[m2].real)))
                acc[: len(pr)] += pr
        out[m] = acc[:Nz]
    return out


def test_three_halves_dealiasing_is_exact():
    rng = np.random.default_rng(3)
    Nx, Nz = 8, 6
    Mx = Nx // 2
    a = rng.standard_normal((Mx, Nz)) + 1j * rng.standard_normal((Mx, Nz))
    b = rng.standard_normal((Mx, Nz)) + 1j * rng.standard_normal((Mx, Nz))
    a[0] = a[0].real
    b[0] = b[0].real
    P, M = 3 * Nx // 2, 3 * Nz // 2
    prod = O.to_grid(a, P, M) * O.to_grid(b, P, M)
    got = O.from_grid(prod, Mx, Nz)
    assert np.allclose(got, _exact_product_coeffs(a, b, Mx, Nz), atol=1e-12)
    # without padding the same product is aliased
    bad = O.from_grid(O.to_grid(a, Nx, Nz) * O.to_grid(b, Nx, Nz), Mx, Nz)
    assert not np.allclose(bad, got, atol=1e-6)


# ------------------------------------------------------- tau solves (P4) ---

def _cheb_of(poly_z, Lz, N):
    """Chebyshev-T coefficients (in zeta) of a polynomial given in z."""
    z = (O.gauss_points(N) + 1) * Lz / 2
    return O.cheb_forward_matrix(N, N) @ poly_z(z)


@pytest.mark.parametrize("m", [0, 1, 5])
def test_tau_solve_recovers_manufactured_temperature(m):
    """(1 - h kappa (d_zz - k^2)) T = f with T(0)=T_bot, T(Lz)=T_top:
    f built analytically from a polynomial T; the solver returns T."""
    g = O.Grid(1e4, 1.0, 2.0, 1.0, 16, 20, 0.3, scheme=4)
    ops = O.Operators(g)
    h_aii = 0.3 * 0.5
    k = g.k[m]
    Tb, Tt = (g.T_bot, g.T_top) if m == 0 else (0.0, 0.0)
    base = np.polynomial.Polynomial([Tb, Tt - Tb])
    bump = np.polynomial.Polynomial([0, 1, -1]) * np.polynomial.Polynomial([0.3, -1.2, 2.0, 0.7])
    T = base + bump                                       # satisfies both BCs
    f = T - h_aii * g.kappa * (T.deriv(2) - k * k * T)
    Tc = _cheb_of(T, g.Lz, g.Nz)
    rhs = ops.S10 @ _cheb_of(f, g.Lz, g.Nz)
    sol = O.StageSolver(g, ops, h_aii).solve_T(m, rhs.astype(complex))
    assert np.allclose(sol, Tc, atol=1e-12)


@pytest.mark.parametrize("m", [1, 3])
def test_tau_solve_recovers_manufactured_streamfunction(m):
    """(lap - h nu lap^2) psi = f with psi = psi_z = 0 on both walls."""
    g = O.Grid(1e5, 1.0, 2.0, 1.0, 16, 24, 0.05, scheme=4)
    ops = O.Operators(g)
    h_aii = 0.05 * 0.5
    k = g.k[m]
    zz = np.polynomial.Polynomial([0, 1, -1])             # z (1 - z)
    psi = zz * zz * np.polynomial.Polynomial([0.4, -0.5, 1.5])
    lap = psi.deriv(2) - k * k * psi
    lap2 = lap.deriv(2) - k * k * lap
    f = lap - h_aii * g.nu * lap2
    pc = _cheb_of(psi, g.Lz, g.Nz)
    rhs = ops.S3210 @ _cheb_of(f, g.Lz, g.Nz)
    sol = O.StageSolver(g, ops, h_aii).solve_P(m, rhs.astype(complex))
    assert np.allclose(sol, pc, atol=1e-12)


# -------------------------------------------------- time stepper (P1, P5) ---

@pytest.mark.parametrize("scheme", [2, 4])
def test_conduction_state_is_a_fixed_point(scheme):
    """Linear conduction profile, no flow: nothing changes, Nu = 1."""
    g = O.Grid(1e6, 1.0, 2.0, 1.0, 16, 12, 1e-2, scheme=scheme)
    st = O.Stepper(g)
    X = O.conduction_state(g)
    Y = st.run(X, 20)
    assert np.abs(Y.T - X.T).max() < 1e-14 and np.abs(Y.P).max() < 1e-14
    nu = O.nusselt(g, Y)
    assert np.allclose(nu, 1.0, atol=1e-13)


def _decay_error(scheme, dt, t_end, field):
    g = O.Grid(1e4, 1.0, 2.0, 1.0, 8, 24, dt, scheme=scheme)
    st = O.Stepper(g)
    X = O.conduction_state(g)
    a = 0.3
    bump = _cheb_of(lambda z: a * np.sin(np.pi * z), g.Lz, g.Nz)
    if field == "T":
        X.T[0] += bump
        rate = g.kappa
    else:
        X.P[0] += bump
        rate = g.nu
    n = int(round(t_end / dt))
    Y = st.run(X, n)
    exact = bump * math.exp(-rate * np.pi ** 2 * t_end)
    got = (Y.T[0] - O.conduction_state(g).T[0]) if field == "T" else Y.P[0]
    return np.abs(got - exact).max()


@pytest.mark.parametrize("field", ["T", "U"])
@pytest.mark.parametrize("scheme,order", [(2, 2), (4, 3)])
def test_mean_mode_diffusion_closed_form_and_order(scheme, order, field):
    """A horizontally uniform perturbation has no advection; sin(pi z)
    decays as exp(-kappa pi^2 t) (temperature) or exp(-nu pi^2 t) (mean
    flow).  Halving dt divides the error by 2^order."""
    e1 = _decay_error(scheme, 0.8, 16.0, field)
    e2 = _decay_error(scheme, 0.4, 16.0, field)
    assert e2 < 1e-4
    ratio = math.log2(e1 / e2)
    assert abs(ratio - order) < 0.25, ratio


@pytest.mark.parametrize("scheme,order", [(2, 2), (4, 3)])
def test_nonlinear_self_convergence_order(scheme, order):
    """Full IMEX coupling (explicit advection + implicit diffusion and
    buoyancy): errors against a small-step run shrink with the scheme order."""
    def run(dt):
        g = O.Grid(2e3, 1.0, 2.0, 1.0, 16, 12, dt, scheme=scheme)
        X = O.conduction_state(g)
        x, z = O.grid_points(g)
        pert = 0.2 * np.cos(np.pi * x)[:, None] * np.sin(np.pi * z)[None, :]
        X.T += O.from_grid(pert, g.Mx, g.Nz)
        X.P[1] += _cheb_of(lambda zz: 0.3 * (zz * (1 - zz)) ** 2, g.Lz, g.Nz)
        return O.Stepper(g).run(X, int(round(2.0 / dt))).pack()
    ref = run(0.0125)
    e = [np.linalg.norm(run(dt) - ref) for dt in (0.2, 0.1)]
    ratio = math.log2(e[0] / e[1])
    assert abs(ratio - order) < 0.35, ratio


# ---------------------------------------------------- linear onset (P6) ---

def _growth_rate(Ra, k, Nz=24, flux=False):
    """Largest real eigenvalue of the linearised problem built from the
    oracle's operators (conduction background, free-fall units).
    Unknowns (phi, T) with psi = i phi so that the pencil is real.  flux:
    fixed-flux walls (the temperature perturbation has zero wall slope)."""
    Lx = 2 * np.pi / k
    g = O.Grid(Ra, 1.0, Lx, 1.0, 4, Nz, 1.0)
    ops = O.Operators(g)
    N = Nz
    Mp, Lp = ops.P_ops(k)
    Mt, Lt = ops.T_ops(k)
    A = np.zeros((2 * N, 2 * N))
    B = np.zeros((2 * N, 2 * N))
    A[:N, :N] = Lp
    A[:N, N:] = -k * ops.S3210          # buoyancy -i k T, divided by i
    A[N:, :N] = k * ops.S10             # background gradient: +w = -i k psi = k phi
    A[N:, N:] = Lt
    B[:N, :N] = Mp
    B[N:, N:] = Mt
    A[N - 4:N, :] = 0
    A[N - 4:N, :N] = O.bc_rows(N, g.scale, "clamped")
    B[N - 4:N, :] = 0
    A[2 * N - 2:, :] = 0
    A[2 * N - 2:, N:] = O.bc_rows(N, g.scale, "neumann" if flux else "dirichlet")
    B[2 * N - 2:, :] = 0
    w = scipy.linalg.eig(A, B, right=False)
    w = w[np.isfinite(w)]
    return w.real.max()


def test_critical_rayleigh_number_matches_chandrasekhar():
    """Rigid-rigid onset: Ra_c = 1707.76 at a = 3.117 (section 3.3 checks
    against Chandrasekhar to 0.1%; the oracle must do far better)."""
    with open(os.path.join(GOLD, "onset.json")) as f:
        gold = json.load(f)
    a = gold["a_c"]
    Rac = scipy.optimize.brentq(lambda R: _growth_rate(R, a), 1600, 1800, xtol=1e-6)
    assert abs(Rac - gold["Ra_c"]) < 0.02, Rac
    assert abs(Rac / gold["Ra_c"] - 1) < gold["paper_tolerance_rel"]


def _stepped_growth(Ra, t1=40.0, t2=120.0, dt=0.2):
    g = O.Grid(Ra, 1.0, 2.0, 1.0, 8, 24, dt, scheme=4)
    X = O.conduction_state(g)
    x, z = O.grid_points(g)
    X.T += O.from_grid(1e-7 * np.cos(np.pi * x)[:, None] * np.sin(np.pi * z)[None, :], g.Mx, g.Nz)
    st = O.Stepper(g)
    X = st.run(X, int(round(t1 / dt)))
    e1 = O.kinetic_energy(g, X)
    X = st.run(X, int(round((t2 - t1) / dt)))
    e2 = O.kinetic_energy(g, X)
    return 0.5 * math.log(e2 / e1) / (t2 - t1)


def test_time_stepper_onset_between_1700_and_1716():
    """Box of aspect ratio 2 (k = pi): the time-stepped m = 1 disturbance
    decays at Ra = 1700 and grows at Ra = 1716 (Ra_c(pi) ~ 1707.9)."""
    assert _stepped_growth(1700.0) < 0 < _stepped_growth(1716.0)


def test_time_stepper_growth_rate_matches_linear_theory():
    s_step = _stepped_growth(3000.0, t1=30.0, t2=60.0, dt=0.1)
    s_eig = _growth_rate(3000.0, np.pi)
    assert s_eig > 0
    assert abs(s_step / s_eig - 1) < 1e-3, (s_step, s_eig)


# --------------------------------------------------------- Nusselt (D1-D2) ---

def test_nusselt_closed_form():
    """T = 1 - z + a z(1-z) + e cos(kx) sin(pi z), psi = b sin(kx) z^2 (1-z)^2:
    Nu_b = 1 - a, Nu_t = 1 + a (wall gradients of the mean profile), and
    Nu_V = 1 + sqrt(Ra Pr) <w T> with <w T> = -e b k/2 int z^2(1-z)^2 sin(pi z)."""
    Ra, a, e, b = 1e5, 0.2, 0.05, 0.03
    g = O.Grid(Ra, 1.0, 2.0, 1.0, 16, 32, 1.0)
    k = g.k[1]
    x, z = O.grid_points(g)
    T = (1 - z + a * z * (1 - z))[None, :] + e * np.cos(k * x)[:, None] * np.sin(np.pi * z)[None, :]
    psi = b * np.sin(k * x)[:, None] * (z * z * (1 - z) ** 2)[None, :]
    X = O.State(O.from_grid(T, g.Mx, g.Nz), O.from_grid(psi, g.Mx, g.Nz))
    X.P[0] = 0
    nu_v, nu_b, nu_t = O.nusselt(g, X)
    assert abs(nu_b - (1 - a)) < 1e-10 and abs(nu_t - (1 + a)) < 1e-10
    I_, _ = scipy.integrate.quad(lambda s: s * s * (1 - s) ** 2 * np.sin(np.pi * s), 0, 1,
                                 epsabs=1e-15, epsrel=1e-14)
    want = 1 + math.sqrt(Ra) * (-e * b * k / 2) * I_
    assert abs(nu_v - want) < 1e-10, (nu_v, want)


def test_initial_state_profile():
    g = O.Grid(1e4, 1.0, 2.0, 1.0, 16, 8, 1.0)
    X = O.initial_state(g, np.zeros((16, 8)), 1e-3)
    C = O.conduction_state(g)
    assert np.allclose(X.T, C.T, rtol=0, atol=1e-14) and not X.P.any()
    xi = I.gaussian_noise(3, 16, 8)
    Y = O.initial_state(g, xi, 1e-3)
    x, z = O.grid_points(g)
    back = O.to_grid(Y.T, g.Nx, g.Nz)
    want = (1 - z)[None, :] + 1e-3 * xi * (z * (1 - z))[None, :]
    # equal up to the dropped Nyquist mode of the noise
    nyq = (np.cos(np.pi * np.arange(16))[:, None] * np.mean(
        (want - (1 - z)[None, :]) * np.cos(np.pi * np.arange(16))[:, None], axis=0)[None, :])
    assert np.allclose(back, want - nyq, atol=1e-14)


# ------------------------------------------------------- Parareal (P7) ---

def test_parareal_dahlquist_closed_form():
    """Scalar y' = lambda y: iterates equal
    U_n^k = sum_{j<=k} C(n,j) (F - G)^j G^(n-j) U_0  (Gander & Vandewalle)."""
    lam, dT, S = -1.3, 0.4, 7
    Fm = math.exp(lam * dT)
    Gm = 1.0 / (1.0 - lam * dT)
    res = O.parareal(np.array([1.0]), S, lambda u, n: Fm * u, lambda u, n: Gm * u, k_max=S)
    for k, U in enumerate(res.iterates):
        for n in range(S + 1):
            want = sum(math.comb(n, j) * (Fm - Gm) ** j * Gm ** (n - j) for j in range(min(k, n) + 1))
            assert abs(U[n][0] - want) < 1e-14, (k, n)
    assert res.k_done == S


def _tiny_rbc():
    fine = O.Grid(3e3, 1.0, 2.0, 1.0, 16, 12, 0.05, scheme=4)
    coarse = O.Grid(3e3, 1.0, 2.0, 1.0, 8, 8, 0.1, scheme=4)
    return O.RBCParareal(fine, coarse, 0.0, 2.0, 4)


def _tiny_ic(pp):
    g = pp.fine
    X = O.initial_state(g, I.gaussian_noise(11, g.Nx, g.Nz), 0.3)
    return X.pack()


def test_parareal_exact_on_first_k_slices_bitwise():
    pp = _tiny_rbc()
    U0 = _tiny_ic(pp)
    serial = [U0]
    for n in range(pp.S):
        serial.append(pp.F(serial[-1], n))
    res = pp.run(U0, k_max=pp.S)
    for k, U in enumerate(res.iterates):
        for n in range(0, k + 1):
            assert np.array_equal(U[n], serial[n]), (k, n)
    assert res.k_done == pp.S
    # the defect is non-zero before finite termination
    assert res.defects[0] > 1e-8


def test_parareal_with_fine_as_coarse_converges_in_one_iteration():
    pp = _tiny_rbc()
    U0 = _tiny_ic(pp)
    res = O.parareal(U0, pp.S, pp.F, pp.F, k_max=2)
    serial = [U0]
    for n in range(pp.S):
        serial.append(pp.F(serial[-1], n))
    for n in range(pp.S + 1):
        assert np.allclose(res.iterates[1][n], serial[n], rtol=0, atol=1e-13)
    assert res.defects[0] < 1e-13


def test_parareal_iterates_keep_boundary_conditions():
    """Restriction, prolongation and the correction (coefficients 1+1-1)
    preserve T = 1 at z = 0, T = 0 at z = Lz and psi = psi_z = 0."""
    pp = _tiny_rbc()
    res = pp.run(_tiny_ic(pp), k_max=2)
    g = pp.fine
    n = np.arange(g.Nz)
    for U in res.iterates:
        for u in U[1:]:
            X = O.State.unpack(u, g.Mx, g.Nz)
            bot = X.T @ ((-1.0) ** n)
            top = X.T @ np.ones(g.Nz)
            assert abs(bot[0] - 1) < 1e-12 and abs(top[0]) < 1e-12
            assert np.abs(bot[1:]).max() < 1e-12 and np.abs(top[1:]).max() < 1e-12
            P = X.P[1:]
            for row in O.bc_rows(g.Nz, g.scale, "clamped"):
                assert np.abs(P @ row).max() < 1e-10
            assert abs(X.P[0] @ ((-1.0) ** n)) < 1e-12 and abs(X.P[0].sum()) < 1e-12


def test_steps_per_slice_rounding():
    n, dt = O.steps_per_slice(0.0, 50.0, 32, 2e-4)
    assert n == 7813 and abs(dt - 1.5625 / 7813) < 1e-18
    n, dt = O.steps_per_slice(0.0, 10.0, 4, 1e-3)
    assert n == 2500 and dt == 1e-3


def test_kinetic_energy_closed_form():
    """psi = b sin(kx) z^2(1-z)^2 and u_bar = c sin(pi z):
    KE = <(u^2 + w^2)/2> = b^2/4 (int g'^2 + k^2 int g^2) + c^2/4, g = z^2 (1-z)^2."""
    b, c = 0.07, 0.03
    g_ = O.Grid(1e5, 1.0, 2.0, 1.0, 16, 32, 1.0)
    k = g_.k[1]
    x, z = O.grid_points(g_)
    psi = b * np.sin(k * x)[:, None] * (z * z * (1 - z) ** 2)[None, :]
    X = O.State(np.zeros((g_.Mx, g_.Nz), complex), O.from_grid(psi, g_.Mx, g_.Nz))
    X.P[0] = _cheb_of(lambda s: c * np.sin(np.pi * s), g_.Lz, g_.Nz)
    gfun = lambda s: s * s * (1 - s) ** 2
    dg = lambda s: 2 * s * (1 - s) ** 2 - 2 * s * s * (1 - s)
    I1, _ = scipy.integrate.quad(lambda s: dg(s) ** 2, 0, 1, epsabs=1e-15)
    I2, _ = scipy.integrate.quad(lambda s: gfun(s) ** 2, 0, 1, epsabs=1e-15)
    want = b * b / 4 * (I1 + k * k * I2) + c * c / 4
    assert abs(O.kinetic_energy(g_, X) - want) < 1e-13


# ------------------------------------- consistency checks of section 2.2 ---

def test_viscous_dissipation_closed_form():
    """psi = b sin(kx) g(z), g = z^2 (1-z)^2, and u_bar = c sin(pi z):
    <|grad u|^2> = b^2/2 int (g''^2 + 2 k^2 g'^2 + k^4 g^2) + c^2 pi^2 / 2,
    epsilon_U = nu times that."""
    b, c = 0.07, 0.03
    g_ = O.Grid(1e5, 1.0, 2.0, 1.0, 16, 32, 1.0)
    k = g_.k[1]
    x, z = O.grid_points(g_)
    psi = b * np.sin(k * x)[:, None] * (z * z * (1 - z) ** 2)[None, :]
    X = O.State(np.zeros((g_.Mx, g_.Nz), complex), O.from_grid(psi, g_.Mx, g_.Nz))
    X.P[0] = _cheb_of(lambda s: c * np.sin(np.pi * s), g_.Lz, g_.Nz)
    gp = np.polynomial.Polynomial([0, 0, 1, -2, 1])          # z^2 (1-z)^2, integrated exactly
    q = lambda f: (f * f).integ()(1.0)
    want = b * b / 2 * (q(gp.deriv(2)) + 2 * k * k * q(gp.deriv(1)) + k ** 4 * q(gp)) + c * c * np.pi ** 2 / 2
    got = O.viscous_dissipation(g_, X)
    assert abs(got / g_.nu - want) < 1e-12 * want, (got / g_.nu, want)


def test_buoyancy_production_closed_form():
    """T = 1 - z + a z(1-z) + e cos(kx) sin(pi z), psi = b sin(kx) g(z):
    P = <w T> = -(e b k / 2) int g sin(pi z)."""
    a, e, b = 0.2, 0.05, 0.03
    g = O.Grid(1e5, 1.0, 2.0, 1.0, 16, 32, 1.0)
    k = g.k[1]
    x, z = O.grid_points(g)
    T = (1 - z + a * z * (1 - z))[None, :] + e * np.cos(k * x)[:, None] * np.sin(np.pi * z)[None, :]
    psi = b * np.sin(k * x)[:, None] * (z * z * (1 - z) ** 2)[None, :]
    X = O.State(O.from_grid(T, g.Mx, g.Nz), O.from_grid(psi, g.Mx, g.Nz))
    X.P[0] = 0
    I_, _ = scipy.integrate.quad(lambda s: s * s * (1 - s) ** 2 * np.sin(np.pi * s), 0, 1,
                                 epsabs=1e-15, epsrel=1e-14)
    assert abs(O.buoyancy_production(g, X) - (-e * b * k / 2) * I_) < 1e-15


def _convecting_state(steps=300):
    g = O.Grid(3e3, 1.0, 2.0, 1.0, 32, 16, 0.01)
    X = O.initial_state(g, I.gaussian_noise(5, g.Nx, g.Nz), 0.3)
    return g, O.Stepper(g), O.Stepper(g).run(X, steps)


def test_dissipation_equals_enstrophy_for_no_slip_fields():
    """For a divergence-free field vanishing on the walls and periodic in x,
    <|grad u|^2> = <omega^2> (the difference integrates to boundary terms)."""
    g, _, X = _convecting_state()
    u, w, *_ = O.velocity_fields(g, X)
    psi = X.P.copy()
    psi[0] = 0
    om = O.cheb_deriv(O.cheb_deriv(psi, g.scale), g.scale) - (g.k[:, None] ** 2) * psi
    om[0] = O.cheb_deriv(X.P[0].real, g.scale)
    enstrophy = O._volume_mean_sq(g, (om,))
    eps = O.viscous_dissipation(g, X)
    assert abs(eps / g.nu - enstrophy) < 1e-12 * enstrophy


def test_energy_budget_matches_time_derivative():
    """d(KE)/dt = P - epsilon_U along the time-stepped solution (central
    difference over two steps of the fourth-order-in-space, third-order-in-
    time integration; the signs and factors of P and epsilon_U are those of
    the equations actually solved)."""
    g, st, Xm = _convecting_state()
    X0 = st.step(Xm)
    Xp = st.step(X0)
    dke = (O.kinetic_energy(g, Xp) - O.kinetic_energy(g, Xm)) / (2 * g.dt)
    budget = O.buoyancy_production(g, X0) - O.viscous_dissipation(g, X0)
    assert abs(dke - budget) < 1e-4 * abs(budget), (dke, budget)


def test_time_averages_of_the_consistency_checks():
    """Eq. 13 and the balance of Eq. 15 on hand-made records; Re is the mean
    RMS velocity over the viscosity."""
    g = O.Grid(1e6, 1.0, 2.0, 1.0, 16, 8, 1.0)
    s = np.array([[8.0, 7.9, 8.2, 0.02, 0.0070, 0.0071],
                  [8.2, 8.1, 8.0, 0.08, 0.0072, 0.0071]])
    a = O.time_averages(g, s)
    assert np.allclose(a[:3], [8.1, 8.0, 8.1])
    assert abs(a[3] - 0.1 / 8.1) < 1e-15
    assert abs(a[4] - 0.05) < 1e-15
    assert abs(a[5] - (0.2 + 0.4) / 2 / g.nu) < 1e-12 * a[5]
    assert np.allclose(a[6:8], [0.0071, 0.0071]) and a[8] < 1e-12



# ------------------------------------------------ fixed-flux walls (Eq. 7) ---

@pytest.mark.parametrize("m", [0, 1, 5])
def test_tau_solve_recovers_manufactured_temperature_fixed_flux(m):
    """(1 - h kappa (d_zz - k^2)) T = f with dT/dz = -1 (m = 0) or 0 (m >= 1)
    on both walls: f built analytically from a polynomial T; the solver
    returns T."""
    g = O.Grid(1e4, 1.0, 2.0, 1.0, 16, 20, 0.3, scheme=4, flux=True)
    ops = O.Operators(g)
    h_aii = 0.3 * 0.5
    k = g.k[m]
    z2 = np.polynomial.Polynomial([0, 0, 1, -2, 1])       # z^2 (1-z)^2: zero slope at both walls
    T = np.polynomial.Polynomial([0.4, -1.0 if m == 0 else 0.0]) + z2 * np.polynomial.Polynomial([0.3, -1.2, 0.7])
    assert abs(T.deriv()(0.0) - (-1.0 if m == 0 else 0.0)) < 1e-14
    f = T - h_aii * g.kappa * (T.deriv(2) - k * k * T)
    Tc = _cheb_of(T, g.Lz, g.Nz)
    rhs = ops.S10 @ _cheb_of(f, g.Lz, g.Nz)
    sol = O.StageSolver(g, ops, h_aii).solve_T(m, rhs.astype(complex))
    assert np.allclose(sol, Tc, atol=1e-12)


def test_fixed_flux_conduction_state_is_a_fixed_point():
    g = O.Grid(5e3, 1.0, 2.0, 1.0, 16, 16, 0.05, scheme=4, flux=True)
    X = O.conduction_state(g)
    Y = O.Stepper(g).run(X, 20)
    assert np.abs(Y.pack() - X.pack()).max() < 1e-13
    assert np.allclose(O.nusselt(g, Y), 1.0, atol=1e-13)


def test_nusselt_closed_form_fixed_flux():
    """Mean profile 1 - z + a cos(pi z) (slope -1 at both walls, drop
    dT = 1 + 2a) with the flow of test_nusselt_closed_form: Nu_b = Nu_t =
    1/dT and Nu_V = 1 + sqrt(Ra Pr) <w T> / dT (Nu = 1/dT for fixed flux)."""
    Ra, a, e, b = 1e5, 0.15, 0.05, 0.03
    g = O.Grid(Ra, 1.0, 2.0, 1.0, 16, 32, 1.0, flux=True)
    k = g.k[1]
    x, z = O.grid_points(g)
    T = (1 - z + a * np.cos(np.pi * z))[None, :] + e * np.cos(k * x)[:, None] * np.sin(np.pi * z)[None, :]
    psi = b * np.sin(k * x)[:, None] * (z * z * (1 - z) ** 2)[None, :]
    X = O.State(O.from_grid(T, g.Mx, g.Nz), O.from_grid(psi, g.Mx, g.Nz))
    X.P[0] = 0
    nu_v, nu_b, nu_t = O.nusselt(g, X)
    dT = 1 + 2 * a
    assert abs(nu_b - 1 / dT) < 1e-10 and abs(nu_t - 1 / dT) < 1e-10, (nu_b, nu_t)
    I_, _ = scipy.integrate.quad(lambda s: s * s * (1 - s) ** 2 * np.sin(np.pi * s), 0, 1,
                                 epsabs=1e-15, epsrel=1e-14)
    assert abs(nu_v - (1 + math.sqrt(Ra) * (-e * b * k / 2) * I_ / dT)) < 1e-10


def test_fixed_flux_onset_tends_to_720():
    """Rigid, perfectly conducting-flux (insulating) walls: the critical
    Rayleigh number of the long-wave limit is 720 (Hurle, Jakeman & Pike
    1967), approached as Ra_c(k) = 720 + O(k^2)."""
    ra = [scipy.optimize.brentq(lambda R: _growth_rate(R, kk, flux=True), 600, 900, xtol=1e-8)
          for kk in (0.04, 0.02)]
    assert abs(ra[1] - 720.0) < 0.05, ra
    assert ra[0] > ra[1] > 720.0 - 1e-6 and abs((ra[0] - 720) / (ra[1] - 720) - 4) < 0.1, ra


# ------------------------------------ advective terms (section 2.1, Eqs. 3-5) ---
#
# A manufactured, band-limited flow is written as an exact trigonometric
# polynomial in x times ordinary polynomials in z, with a mean shear u_bar(z)
# and tilted rolls (so that <u w> and d u_bar/dz are both nonzero).  The
# advection of momentum and heat is evaluated from the primitive variables
# u, w, T with exact derivatives and exact products, and compared with the
# oracle's pseudo-spectral explicit terms.  Low polynomial degrees keep every
# product inside the retained spectrum, so the comparison is exact to
# rounding.

class _TrigPoly:
    """f(x, z) = sum_m c_m(z) exp(i m k x), c_m numpy Polynomials in z, with
    c_(-m) = conj(c_m) for a real field."""

    def __init__(self, k, coeffs):
        self.k = k
        self.c = {m: p for m, p in coeffs.items()}

    @staticmethod
    def real_field(k, modes):
        """modes: {m >= 0: complex Polynomial c_m}; adds the conjugate modes."""
        c = {}
        for m, p in modes.items():
            c[m] = p
            if m > 0:
                c[-m] = np.polynomial.Polynomial(np.conj(p.coef))
        return _TrigPoly(k, c)

    def __add__(self, o):
        c = dict(self.c)
        for m, p in o.c.items():
            c[m] = c[m] + p if m in c else p
        return _TrigPoly(self.k, c)

    def __sub__(self, o):
        return self + o.scale(-1.0)

    def scale(self, a):
        return _TrigPoly(self.k, {m: p * a for m, p in self.c.items()})

    def __mul__(self, o):
        c = {}
        for m1, p1 in self.c.items():
            for m2, p2 in o.c.items():
                m = m1 + m2
                c[m] = c[m] + p1 * p2 if m in c else p1 * p2
        return _TrigPoly(self.k, c)

    def dx(self):
        return _TrigPoly(self.k, {m: p * (1j * m * self.k) for m, p in self.c.items()})

    def dz(self):
        return _TrigPoly(self.k, {m: p.deriv() for m, p in self.c.items()})

    def mode(self, m):
        return self.c.get(m, np.polynomial.Polynomial([0.0]))


def _cheb_of_complex(p, Lz, N):
    return _cheb_of(lambda z: p(z).real, Lz, N) + 1j * _cheb_of(lambda z: p(z).imag, Lz, N)


def _sheared_rolls(g, b=0.4, c=0.3, e=0.2):
    """Streamfunction with tilted rolls in modes 1 and 2, a no-slip mean
    shear u_bar and a perturbed temperature, as exact trigonometric
    polynomials and as an oracle state."""
    P = np.polynomial.Polynomial
    k = g.k[1]
    zz = P([0, 0, 1, -2, 1])                                  # z^2 (1-z)^2: psi = psi_z = 0 on the walls
    psi = _TrigPoly.real_field(k, {1: zz * P([0.5 * b, -0.6j * b, 0.3j * b]),   # phase varies with z
                                   2: zz * P([0.2 * b + 0.1j * b, 0.25 * b])})
    ubar = P([0, 1, -1]) * P([c, -0.7 * c, 0.9 * c])           # u_bar(0) = u_bar(1) = 0, sheared
    Tf = _TrigPoly.real_field(k, {0: P([1.0, -1.0]) + P([0, 1, -1]) * P([0.1]),
                                  1: P([0, 1, -1]) * P([0.5 * e, 0.3j * e]),
                                  2: P([0, 1, -1]) * P([0.1j * e, -0.2 * e])})
    u = psi.dz() + _TrigPoly(k, {0: ubar})
    w = psi.dx().scale(-1.0)
    X = O.State(np.zeros((g.Mx, g.Nz), complex), np.zeros((g.Mx, g.Nz), complex))
    for m in range(g.Mx):
        X.T[m] = _cheb_of_complex(Tf.mode(m), g.Lz, g.Nz)
        if m > 0:
            X.P[m] = _cheb_of_complex(psi.mode(m), g.Lz, g.Nz)
    X.P[0] = _cheb_of(ubar, g.Lz, g.Nz)
    return u, w, Tf, X


def test_advective_terms_equal_primitive_variable_advection():
    """The explicit terms of the stepper against the advection written in
    primitive variables: the curl of (u.grad)u (vorticity omega = u_z - w_x
    of the streamfunction form), (u.grad)T, and for the mean flow the
    horizontal mean of the x-component of (u.grad)u, each moved to the left
    of the equation (hence the minus sign) and into the equation's basis.
    A flipped sign of the vorticity advection or of the mean-flow forcing,
    or a dropped term, fails here."""
    g = O.Grid(1e5, 1.0, 2.0, 1.0, 16, 32, 1e-3)
    u, w, Tf, X = _sheared_rolls(g)
    ax = u * u.dx() + w * u.dz()                   # x-component of (u.grad)u
    az = u * w.dx() + w * w.dz()                   # z-component
    curl = ax.dz() - az.dx()                       # omega = u_z - w_x
    adv_T = u * Tf.dx() + w * Tf.dz()
    ops = O.Operators(g)
    E = O.Stepper(g).explicit(X)
    def close(got, want):
        return np.abs(got - want).max() <= 1e-12 * max(np.abs(want).max(), 1e-3)

    for m in range(1, g.Mx):
        want = -(ops.S3210 @ _cheb_of_complex(curl.mode(m), g.Lz, g.Nz))
        assert close(E.P[m], want), m
    for m in range(g.Mx):
        want = -(ops.S10 @ _cheb_of_complex(adv_T.mode(m), g.Lz, g.Nz))
        assert close(E.T[m], want), m
    want_u = -(ops.S10 @ _cheb_of_complex(ax.mode(0), g.Lz, g.Nz))
    assert close(E.P[0], want_u)
    # the manufactured flow does exercise every term: mean-flow forcing,
    # vorticity advection in modes 1..4 (products of modes 1 and 2)
    assert np.abs(want_u).max() > 1e-4
    assert min(np.abs(E.P[m]).max() for m in (1, 2, 3, 4)) > 1e-4


def test_mean_flow_forcing_is_minus_the_reynolds_stress_gradient():
    """x-average of (u.grad)u = d<u w>/dz for the divergence-free flow, and
    the oracle's mean-flow term is -S1 D1 of its dealiased <u w>."""
    g = O.Grid(1e5, 1.0, 2.0, 1.0, 16, 32, 1e-3)
    u, w, _, X = _sheared_rolls(g)
    uw = (u * w).mode(0)
    ax = (u * u.dx() + w * u.dz()).mode(0)
    zs = np.linspace(0, 1, 11)
    assert np.allclose(ax(zs), uw.deriv()(zs), atol=1e-13)
    _, _, q_hat = O.nonlinear_terms(g, X)
    assert np.allclose(q_hat, _cheb_of_complex(uw, g.Lz, g.Nz), atol=1e-13)


def test_energy_budget_with_mean_shear_and_tilted_rolls():
    """d(KE)/dt = P - epsilon_U along a time-stepped solution that starts
    from strong mean shear and tilted rolls: the exchange between mean flow
    and rolls (Reynolds stress times shear) enters the mean-flow and the
    roll energy with opposite signs, so a sign error in either advective
    term, or a dropped mean-flow forcing, breaks the budget."""
    g = O.Grid(2e4, 1.0, 2.0, 1.0, 16, 24, 2e-3)
    _, _, _, X = _sheared_rolls(g, b=2.0, c=1.5, e=0.5)
    st = O.Stepper(g)
    Xm = st.step(X)
    X0 = st.step(Xm)
    Xp = st.step(X0)
    dke = (O.kinetic_energy(g, Xp) - O.kinetic_energy(g, Xm)) / (2 * g.dt)
    budget = O.buoyancy_production(g, X0) - O.viscous_dissipation(g, X0)
    assert abs(dke - budget) < 1e-4 * abs(budget), (dke, budget)
