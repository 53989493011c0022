"""FP64 CPU oracle for Parareal applied to 2D Rayleigh-Benard convection.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
baseline leg of the benchmark may import this module.  The GPU library
shares no code with it.

What it computes (each function names the part of the paper it follows):

* the Oberbeck-Boussinesq equations of section 2.1 (Eqs. 3-5) with the
  no-slip walls of fixed temperature (Eq. 6) or fixed flux (Eq. 7, with
  the flux Rayleigh number Ra_f in place of Ra), written in free-fall units on
  z in [0, Lz] (the reading used for the workloads: viscosity sqrt(Pr/Ra),
  diffusivity 1/sqrt(Ra Pr), buoyancy coefficient 1), in the
  streamfunction-vorticity form so that the pressure drops out;
* the Fourier(x) x Chebyshev(z) pseudo-spectral discretisation of
  section 3.2, with products formed on a 3/2-padded grid;
* the implicit-explicit Runge-Kutta schemes of Ascher, Ruuth & Spiteri
  named in sections 3.2 and 3.6 (ARS(2,2,2) and ARS(4,4,3)): diffusion and
  buoyancy implicit, advection explicit; each stage solve is a dense LU
  with partial pivoting of the tau-modified ultraspherical system;
* the Nusselt numbers of section 2.2 (Eqs. 9-11) and the other quantities
  of its consistency checks: the Reynolds number from the RMS velocity, the
  spread Nu_int of the three Nusselt numbers (Eq. 13), and the buoyancy
  production P against the viscous dissipation epsilon_U (Eq. 15);
* the Parareal iteration of section 3.1 (Eq. 19), serially, with a coarse
  propagator built by spatial coarsening and a larger step (section 3.6).

Readings where the paper is silent are listed in the design notes; the
ones that change numbers are restated next to the code that uses them.
Everything is plain and unblocked: dense matrices, numpy FFTs and
matrix products as library steps, no fusion.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, List, Optional, Sequence

import numpy as np
import scipy.linalg

# --------------------------------------------------------------------------
# Butcher tableaux of the IMEX schemes (Ascher, Ruuth & Spiteri 1997), in the
# (s+1)-stage form whose first stage is the old solution.  Index 0 is stage 1.
# --------------------------------------------------------------------------


def ars_tableau(scheme: int):
    """Return (A_explicit, A_implicit) as (s+1)x(s+1) arrays.

    scheme 2: ARS(2,2,2), gamma = 1 - 1/sqrt(2), delta = 1 - 1/(2 gamma)
    ("IMEX RK2" of the small workload).  scheme 4: ARS(4,4,3), the "RK443"
    the paper uses for both propagators (section 3.6).
    """
    if scheme == 2:
        g = 1.0 - 1.0 / math.sqrt(2.0)
        d = 1.0 - 1.0 / (2.0 * g)
        ae = np.array([[0, 0, 0], [g, 0, 0], [d, 1 - d, 0]], dtype=np.float64)
        ai = np.array([[0, 0, 0], [0, g, 0], [0, 1 - g, g]], dtype=np.float64)
    elif scheme == 4:
        ae = np.array([[0, 0, 0, 0, 0],
                       [1 / 2, 0, 0, 0, 0],
                       [11 / 18, 1 / 18, 0, 0, 0],
                       [5 / 6, -5 / 6, 1 / 2, 0, 0],
                       [1 / 4, 7 / 4, 3 / 4, -7 / 4, 0]], dtype=np.float64)
        ai = np.array([[0, 0, 0, 0, 0],
                       [0, 1 / 2, 0, 0, 0],
                       [0, 1 / 6, 1 / 2, 0, 0],
                       [0, -1 / 2, 1 / 2, 1 / 2, 0],
                       [0, 3 / 2, -3 / 2, 1 / 2, 1 / 2]], dtype=np.float64)
    else:
        raise ValueError("scheme must be 2 (ARS222) or 4 (ARS443)")
    return ae, ai


# --------------------------------------------------------------------------
# Chebyshev and ultraspherical building blocks (section 3.2: Chebyshev basis
# in z).  Coefficient vectors are in the Chebyshev-T basis on zeta in [-1,1],
# zeta = 2 z / Lz - 1, so z = 0 (the hot wall) is zeta = -1.
# --------------------------------------------------------------------------


def gauss_points(M: int) -> np.ndarray:
    """Chebyshev-Gauss points zeta_j = cos(pi (j + 1/2) / M), j = 0..M-1."""
    j = np.arange(M, dtype=np.float64)
    return np.cos(np.pi * (j + 0.5) / M)


def cheb_eval_matrix(M: int, N: int) -> np.ndarray:
    """V[j, n] = T_n(zeta_j) at the M Gauss points, n < N."""
    theta = np.pi * (np.arange(M, dtype=np.float64) + 0.5) / M
    return np.cos(np.outer(theta, np.arange(N, dtype=np.float64)))


def cheb_forward_matrix(M: int, N: int) -> np.ndarray:
    """C[n, j] = (2 - delta_n0) / M * T_n(zeta_j): values at M Gauss points
    to the first N Chebyshev coefficients of their interpolant."""
    C = cheb_eval_matrix(M, N).T * (2.0 / M)
    C[0, :] *= 0.5
    return C


def op_D(lam: int, N: int, scale: float) -> np.ndarray:
    """d^lam/dz^lam from the T basis to the C^(lam) basis:
    T_n -> 2^(lam-1) (lam-1)! n C^(lam)_(n-lam), times scale^lam."""
    A = np.zeros((N, N))
    f = 2.0 ** (lam - 1) * math.factorial(lam - 1) * scale ** lam
    for n in range(lam, N):
        A[n - lam, n] = f * n
    return A


def op_S0(N: int) -> np.ndarray:
    """Conversion T -> C^(1): T_0 = C_0, T_1 = C_1/2, T_n = (C_n - C_(n-2))/2."""
    A = np.zeros((N, N))
    A[0, 0] = 1.0
    for n in range(1, N):
        A[n, n] = 0.5
    for n in range(2, N):
        A[n - 2, n] = -0.5
    return A


def op_S(lam: int, N: int) -> np.ndarray:
    """Conversion C^(lam) -> C^(lam+1):
    C^(lam)_n = lam/(n+lam) (C^(lam+1)_n - C^(lam+1)_(n-2))."""
    A = np.zeros((N, N))
    for n in range(N):
        A[n, n] = lam / (n + lam)
        if n >= 2:
            A[n - 2, n] = -lam / (n + lam)
    return A


def cheb_deriv(c: np.ndarray, scale: float) -> np.ndarray:
    """Chebyshev-T coefficients of d/dz along the last axis (library routine
    numpy.polynomial.chebyshev.chebder), times dzeta/dz = scale."""
    N = c.shape[-1]
    d = np.polynomial.chebyshev.chebder(np.moveaxis(c, -1, 0), axis=0) * scale
    out = np.zeros_like(c)
    out[..., : N - 1] = np.moveaxis(d, 0, -1)
    return out


# --------------------------------------------------------------------------
# Problem description
# --------------------------------------------------------------------------


@dataclasses.dataclass
class Grid:
    """Discretisation of one propagator (fine or coarse).

    Ra, Pr: Rayleigh and Prandtl numbers (section 2.1); Lx, Lz: box size
    (aspect ratio 2 in the paper); Nx, Nz: collocation points (section 3.2);
    dt: time step; scheme: 2 or 4 (see ars_tableau).  flux: fixed-flux
    walls dT/dz = -1 (Eq. 7; Ra is then the flux Rayleigh number Ra_f)
    instead of the fixed temperatures T_bot, T_top (Eq. 6).
    """
    Ra: float
    Pr: float
    Lx: float
    Lz: float
    Nx: int
    Nz: int
    dt: float
    scheme: int = 4
    T_bot: float = 1.0   # temperature at z = 0 (Eq. 6)
    T_top: float = 0.0   # temperature at z = Lz (Eq. 6)
    flux: bool = False   # fixed-flux walls (Eq. 7)

    def __post_init__(self):
        if self.Nx % 4 or self.Nz % 2:
            raise ValueError("need Nx % 4 == 0 and Nz % 2 == 0")
        self.Mx = self.Nx // 2           # modes 0..Mx-1; the Nyquist mode is dropped
        self.Px = 3 * self.Nx // 2       # 3/2-padded grid for products
        self.Pz = 3 * self.Nz // 2
        self.nu = math.sqrt(self.Pr / self.Ra)        # free-fall units
        self.kappa = 1.0 / math.sqrt(self.Ra * self.Pr)
        self.k = 2.0 * np.pi * np.arange(self.Mx) / self.Lx
        self.scale = 2.0 / self.Lz


# --------------------------------------------------------------------------
# Transforms (section 3.2).  Fourier: f(x_i) = f_0 + 2 Re sum_{m>=1} f_m
# exp(i k_m x_i) on x_i = i Lx / P; forward f_m = P^-1 sum_i f(x_i)
# exp(-i k_m x_i).  Chebyshev: values at Gauss points, see above.
# --------------------------------------------------------------------------


def to_grid(chat: np.ndarray, P: int, M: int) -> np.ndarray:
    """Spectral [Mx, N] (complex) -> physical values [P, M] on the
    P-point x grid and the M Gauss points in z."""
    Mx, N = chat.shape
    zvals = chat @ cheb_eval_matrix(M, N).T            # [Mx, M]
    H = np.zeros((P // 2 + 1, M), dtype=np.complex128)
    H[:Mx] = zvals * P
    return np.fft.irfft(H, n=P, axis=0)               # [P, M]


def from_grid(f: np.ndarray, Mx: int, N: int) -> np.ndarray:
    """Physical values [P, M] -> spectral [Mx, N], keeping m < Mx, n < N."""
    P, M = f.shape
    F = np.fft.rfft(f, axis=0)[:Mx] / P                # [Mx, M]
    return F @ cheb_forward_matrix(M, N).T


def grid_points(g: Grid, P: Optional[int] = None, M: Optional[int] = None):
    """x_i (length P) and z_j (length M) of the collocation grid."""
    P = g.Nx if P is None else P
    M = g.Nz if M is None else M
    x = np.arange(P) * g.Lx / P
    z = (gauss_points(M) + 1.0) * g.Lz / 2.0
    return x, z


# --------------------------------------------------------------------------
# State.  T[m, n] = Chebyshev coefficients of temperature mode m;
# P[m, n] = streamfunction mode m for m >= 1, and for m = 0 the mean
# horizontal velocity u_bar(z) (the streamfunction's mean is not needed:
# u = d psi/dz, w = -d psi/dx).
# --------------------------------------------------------------------------


@dataclasses.dataclass
class State:
    T: np.ndarray   # complex [Mx, Nz]
    P: np.ndarray   # complex [Mx, Nz]

    def copy(self):
        return State(self.T.copy(), self.P.copy())

    def pack(self) -> np.ndarray:
        """Flat real vector in the library layout [field][m][re, im][n]."""
        def one(a):
            return np.stack([a.real, a.imag], axis=1).reshape(-1)
        return np.concatenate([one(self.P), one(self.T)])

    @staticmethod
    def unpack(v: np.ndarray, Mx: int, Nz: int) -> "State":
        v = np.asarray(v, dtype=np.float64).reshape(2, Mx, 2, Nz)
        P = v[0, :, 0] + 1j * v[0, :, 1]
        T = v[1, :, 0] + 1j * v[1, :, 1]
        return State(T.copy(), P.copy())


def initial_state(g: Grid, xi: np.ndarray, amp: float) -> State:
    """Linear conduction profile plus a small perturbation, u = 0
    (section 2.1): T = T_bot + (T_top - T_bot) z/Lz + amp xi z(Lz - z)/Lz^2
    (fixed flux: T = T_bot - z + the same perturbation) on the Nx x Nz
    collocation grid, transformed; psi = u_bar = 0.
    ``xi`` is the [Nx, Nz] standard-normal noise from the seeded generator."""
    x, z = grid_points(g)
    zz = z[None, :] / g.Lz
    base = g.T_bot - z[None, :] if g.flux else g.T_bot + (g.T_top - g.T_bot) * zz
    Tg = base + amp * xi * zz * (1.0 - zz)
    T = from_grid(Tg, g.Mx, g.Nz)
    T[0] = T[0].real
    return State(T, np.zeros_like(T))


def conduction_state(g: Grid) -> State:
    """T = T_bot + (T_top - T_bot) z / Lz (fixed flux: T_bot - z), no flow."""
    T = np.zeros((g.Mx, g.Nz), dtype=np.complex128)
    if g.flux:
        T[0, 0] = g.T_bot - 0.5 * g.Lz
        T[0, 1] = -0.5 * g.Lz
    else:
        T[0, 0] = 0.5 * (g.T_bot + g.T_top)
        T[0, 1] = 0.5 * (g.T_top - g.T_bot)
    return State(T, np.zeros_like(T))


# --------------------------------------------------------------------------
# Linear operators per Fourier mode (sections 2.1 and 3.2), ultraspherical
# spectral method: rows of the equation are coefficients in C^(2) for the
# temperature and mean-flow equations and C^(4) for the streamfunction one.
# --------------------------------------------------------------------------


class Operators:
    """M (mass), L (implicit linear part) and B (buoyancy coupling) per mode.

    Temperature (Eq. 5):   M = S1 S0,                L = kappa (D2 - k^2 S1 S0)
    Vorticity (curl of Eq. 3), streamfunction psi, m >= 1:
        M = S3 S2 (D2 - k^2 S1 S0)                    (Laplacian of psi)
        L = nu (D4 - 2 k^2 S3 S2 D2 + k^4 S3 S2 S1 S0) (nu times bi-Laplacian)
        B = -i k S3 S2 S1 S0 acting on T               (buoyancy, -dT/dx)
    Mean flow u_bar (m = 0 of the x momentum, no mean pressure gradient):
        M = S1 S0,  L = nu D2.
    """

    def __init__(self, g: Grid):
        N, s = g.Nz, g.scale
        self.S0 = op_S0(N)
        self.S1 = op_S(1, N)
        self.S2 = op_S(2, N)
        self.S3 = op_S(3, N)
        self.D1 = op_D(1, N, s)
        self.D2 = op_D(2, N, s)
        self.D4 = op_D(4, N, s)
        self.S10 = self.S1 @ self.S0
        self.S32 = self.S3 @ self.S2
        self.S3210 = self.S32 @ self.S10
        self.g = g

    def T_ops(self, k):
        return self.S10, self.g.kappa * (self.D2 - k * k * self.S10)

    def P_ops(self, k):
        M = self.S32 @ (self.D2 - k * k * self.S10)
        L = self.g.nu * (self.D4 - 2 * k * k * self.S32 @ self.D2 + k ** 4 * self.S3210)
        return M, L

    def U_ops(self):
        return self.S10, self.g.nu * self.D2


def bc_rows(N: int, scale: float, kind: str) -> np.ndarray:
    """Boundary rows (tau method) on coefficient vectors.

    kind 'dirichlet': value at zeta = -1 (z = 0) and at zeta = +1 (z = Lz),
    T_n(+-1) = (+-1)^n.  kind 'neumann': d/dz at both walls,
    T_n'(1) = n^2, T_n'(-1) = (-1)^(n+1) n^2, times scale.  kind 'clamped':
    the dirichlet rows, then the neumann rows.
    """
    n = np.arange(N, dtype=np.float64)
    value = [(-1.0) ** n, np.ones(N)]
    slope = [(-1.0) ** (n + 1) * n * n * scale, n * n * scale]
    return np.array({"dirichlet": value, "neumann": slope, "clamped": value + slope}[kind])


class StageSolver:
    """Dense LU (partial pivoting) of the tau-modified stage matrices
    M - h a_ii L, factored once per mode and field: the last b equation rows
    (b = 2 for T and u_bar, 4 for psi) are replaced by boundary rows."""

    def __init__(self, g: Grid, ops: Operators, h_aii: float):
        N = g.Nz
        self.g = g
        self.bT = bc_rows(N, g.scale, "neumann" if g.flux else "dirichlet")
        self.bU = bc_rows(N, g.scale, "dirichlet")          # no-slip mean flow
        self.bP = bc_rows(N, g.scale, "clamped")
        self.luT, self.luP = [], []
        for m in range(g.Mx):
            k = g.k[m]
            M, L = ops.T_ops(k)
            A = M - h_aii * L
            A[N - 2:] = self.bT
            self.luT.append(scipy.linalg.lu_factor(A))
            if m == 0:
                M, L = ops.U_ops()
                A = M - h_aii * L
                A[N - 2:] = self.bU
            else:
                M, L = ops.P_ops(k)
                A = M - h_aii * L
                A[N - 4:] = self.bP
            self.luP.append(scipy.linalg.lu_factor(A))

    @staticmethod
    def _solve(lu, rhs):
        return scipy.linalg.lu_solve(lu, rhs.real) + 1j * scipy.linalg.lu_solve(lu, rhs.imag)

    def solve_T(self, m: int, rhs: np.ndarray) -> np.ndarray:
        N = self.g.Nz
        r = rhs.copy()
        if m == 0:
            r[N - 2:] = [-1.0, -1.0] if self.g.flux else [self.g.T_bot, self.g.T_top]
        else:
            r[N - 2:] = 0.0
        return self._solve(self.luT[m], r)

    def solve_P(self, m: int, rhs: np.ndarray) -> np.ndarray:
        N = self.g.Nz
        r = rhs.copy()
        r[N - (2 if m == 0 else 4):] = 0.0
        return self._solve(self.luP[m], r)


# --------------------------------------------------------------------------
# Explicit (advective) terms, formed in grid space on the 3/2-padded grid
# (section 3.2: transforms to grid space, products there, transforms back).
# --------------------------------------------------------------------------


def velocity_fields(g: Grid, X: State):
    """Spectral coefficients of u, w, omega_x, omega_z, T_x, T_z."""
    k = g.k[:, None]
    psi = X.P.copy()
    psi[0] = 0.0
    ubar = X.P[0].real
    u = cheb_deriv(psi, g.scale)
    u[0] = ubar
    w = -1j * k * psi
    om = cheb_deriv(cheb_deriv(psi, g.scale), g.scale) - k * k * psi
    om[0] = cheb_deriv(ubar, g.scale)          # vorticity of the mean flow
    omx = 1j * k * om
    omz = cheb_deriv(om, g.scale)
    Tx = 1j * k * X.T
    Tz = cheb_deriv(X.T, g.scale)
    return u, w, omx, omz, Tx, Tz


def nonlinear_terms(g: Grid, X: State):
    """Dealiased N_omega = u.grad(omega), N_T = u.grad(T) (mode m, Chebyshev
    coefficients n < Nz) and the Chebyshev coefficients of the horizontal
    mean of u w (which drives the mean flow)."""
    u, w, omx, omz, Tx, Tz = velocity_fields(g, X)
    P, M = g.Px, g.Pz
    ug, wg = to_grid(u, P, M), to_grid(w, P, M)
    Nom = ug * to_grid(omx, P, M) + wg * to_grid(omz, P, M)
    NT = ug * to_grid(Tx, P, M) + wg * to_grid(Tz, P, M)
    q = np.mean(ug * wg, axis=0)                      # [M] on Gauss points
    q_hat = cheb_forward_matrix(M, g.Nz) @ q
    return from_grid(Nom, g.Mx, g.Nz), from_grid(NT, g.Mx, g.Nz), q_hat


class Stepper:
    """The fine (or coarse) propagator: IMEX Runge-Kutta steps (section 3.2)
    with implicit diffusion and buoyancy and explicit advection."""

    def __init__(self, g: Grid):
        self.g = g
        self.ops = Operators(g)
        self.ae, self.ai = ars_tableau(g.scheme)
        aii = self.ai[1, 1]
        assert np.all(np.diag(self.ai)[1:] == aii)
        self.solver = StageSolver(g, self.ops, g.dt * aii)
        self.Tops = [self.ops.T_ops(k) for k in g.k]
        self.Pops = [self.ops.U_ops()] + [self.ops.P_ops(k) for k in g.k[1:]]

    def explicit(self, X: State):
        """E_T = -S1 S0 N_T, E_psi = -S3 S2 S1 S0 N_omega (m >= 1),
        E_ubar = -S1 D1 <u w> (m = 0), in the equations' bases."""
        Nom, NT, q_hat = nonlinear_terms(self.g, X)
        o = self.ops
        ET = -(NT @ o.S10.T)
        EP = -(Nom @ o.S3210.T)
        EP[0] = -(o.S1 @ (o.D1 @ q_hat))
        return State(ET, EP)

    def implicit(self, Y: State):
        """L Y per mode, with the buoyancy B T added to the psi equation."""
        g = self.g
        LT = np.stack([self.Tops[m][1] @ Y.T[m] for m in range(g.Mx)])
        LP = np.stack([self.Pops[m][1] @ Y.P[m] for m in range(g.Mx)])
        for m in range(1, g.Mx):
            LP[m] += -1j * g.k[m] * (self.ops.S3210 @ Y.T[m])
        return State(LT, LP)

    def mass(self, X: State):
        g = self.g
        MT = np.stack([self.Tops[m][0] @ X.T[m] for m in range(g.Mx)])
        MP = np.stack([self.Pops[m][0] @ X.P[m] for m in range(g.Mx)])
        return State(MT, MP)

    def step(self, X: State) -> State:
        """One IMEX step in ARS form: Y_1 = X; for each later stage i solve
        (M - h a~_ii L) Y_i = M X + h sum_{j<i} a_ij E(Y_j)
                               + h sum_{1<j<i} a~_ij L Y_j      (temperature first,
        then psi with the buoyancy of the new T on the right); X_new = last Y."""
        g, h = self.g, self.g.dt
        ae, ai = self.ae, self.ai
        ns = ae.shape[0]
        MX = self.mass(X)
        E: List[State] = []
        LY: List[Optional[State]] = [None]
        Y = X
        for i in range(1, ns):
            E.append(self.explicit(Y))
            rT = MX.T.copy()
            rP = MX.P.copy()
            for j in range(i):
                rT += h * ae[i, j] * E[j].T
                rP += h * ae[i, j] * E[j].P
            for j in range(1, i):
                rT += h * ai[i, j] * LY[j].T
                rP += h * ai[i, j] * LY[j].P
            Tn = np.stack([self.solver.solve_T(m, rT[m]) for m in range(g.Mx)])
            Pn = np.empty_like(Tn)
            for m in range(g.Mx):
                r = rP[m]
                if m > 0:
                    r = r + h * ai[i, i] * (-1j * g.k[m]) * (self.ops.S3210 @ Tn[m])
                Pn[m] = self.solver.solve_P(m, r)
            Tn[0] = Tn[0].real
            Pn[0] = Pn[0].real
            Y = State(Tn, Pn)
            if i < ns - 1:
                LY.append(self.implicit(Y))
        return Y

    def run(self, X: State, n_steps: int, callback: Optional[Callable] = None) -> State:
        for s in range(n_steps):
            X = self.step(X)
            if callback is not None:
                callback(s + 1, X)
        return X


# --------------------------------------------------------------------------
# Diagnostics (section 2.2)
# --------------------------------------------------------------------------


def nusselt(g: Grid, X: State):
    """(Nu_V, Nu_b, Nu_t) of Eqs. 9-11, in free-fall units, each divided by
    the conductive flux of the current mean temperature drop, dT / Lz with
    dT = <T>_H(z=0) - <T>_H(z=Lz) (1 for the fixed temperatures of Eq. 6;
    for the fixed flux of Eq. 7 this is the Nu = 1 / dT of that case).

    Nu_b, Nu_t: -dT/dz of the horizontal mean at z = 0 and z = Lz (exact
    endpoint derivatives of the Chebyshev series).
    Nu_V: volume mean of -dT/dz + sqrt(Ra Pr) w T (the advective flux is
    w T / kappa in these units).  The mean of -dT/dz is the endpoint
    difference over Lz; the mean of w T is integrated exactly: an Nx-point
    mean in x (exact for a product of two band-limited fields) and Nz-point
    Gauss-Legendre quadrature in z (exact for degree <= 2 Nz - 1).
    """
    Tm = X.T[0].real
    n = np.arange(g.Nz, dtype=np.float64)
    nu_b = -g.scale * np.sum(Tm * (-1.0) ** (n + 1) * n * n)
    nu_t = -g.scale * np.sum(Tm * n * n)
    T_z0 = np.sum(Tm * (-1.0) ** n)
    T_z1 = np.sum(Tm)
    zl, wl = np.polynomial.legendre.leggauss(g.Nz)
    V = np.cos(np.outer(np.arccos(zl), n))            # T_n at Legendre nodes
    psi = X.P.copy()
    psi[0] = 0.0
    w_hat = -1j * g.k[:, None] * psi

    def phys(c):
        H = np.zeros((g.Nx // 2 + 1, g.Nz), dtype=np.complex128)
        H[: g.Mx] = (c @ V.T) * g.Nx
        return np.fft.irfft(H, n=g.Nx, axis=0)

    wT = np.mean(phys(w_hat) * phys(X.T), axis=0)
    mean_wT = 0.5 * np.sum(wl * wT)
    ref = (T_z0 - T_z1) / g.Lz                         # conductive flux of the drop
    nu_v = ((T_z0 - T_z1) / g.Lz + math.sqrt(g.Ra * g.Pr) * mean_wT) / ref
    return nu_v, nu_b / ref, nu_t / ref


def kinetic_energy(g: Grid, X: State) -> float:
    """Volume mean of (u^2 + w^2)/2 (Nx-point x mean, Gauss-Legendre z)."""
    u, w, *_ = velocity_fields(g, X)
    zl, wl = np.polynomial.legendre.leggauss(g.Nz + 2)
    V = np.cos(np.outer(np.arccos(zl), np.arange(g.Nz)))
    tot = 0.0
    for c in (u, w):
        H = np.zeros((g.Nx // 2 + 1, len(zl)), dtype=np.complex128)
        H[: g.Mx] = (c @ V.T) * g.Nx
        f = np.fft.irfft(H, n=g.Nx, axis=0)
        tot += 0.25 * np.sum(wl * np.mean(f * f, axis=0))
    return tot


def _volume_mean_sq(g: Grid, fields) -> float:
    """Volume mean of the sum of squares of real fields given by their
    spectral coefficients (mode m, Chebyshev n): Nx-point mean in x,
    Gauss-Legendre quadrature in z exact for the squared polynomials."""
    zl, wl = np.polynomial.legendre.leggauss(g.Nz + 2)
    V = np.cos(np.outer(np.arccos(zl), np.arange(g.Nz)))
    tot = 0.0
    for c in fields:
        H = np.zeros((g.Nx // 2 + 1, len(zl)), dtype=np.complex128)
        H[: g.Mx] = (c @ V.T) * g.Nx
        f = np.fft.irfft(H, n=g.Nx, axis=0)
        tot += 0.5 * np.sum(wl * np.mean(f * f, axis=0))
    return tot


def viscous_dissipation(g: Grid, X: State) -> float:
    """epsilon_U of section 2.2 in free-fall units: nu times the volume mean
    of |grad u|^2 = u_x^2 + u_z^2 + w_x^2 + w_z^2 (all four components
    written out).  Dotting the momentum equation with u and averaging gives
    d(KE)/dt = P - epsilon_U for no-slip, periodic boundaries."""
    u, w, *_ = velocity_fields(g, X)
    k = g.k[:, None]
    grads = (1j * k * u, cheb_deriv(u, g.scale), 1j * k * w, cheb_deriv(w, g.scale))
    return g.nu * _volume_mean_sq(g, grads)


def buoyancy_production(g: Grid, X: State) -> float:
    """P of section 2.2 in free-fall units (buoyancy coefficient 1): the
    volume mean of w T."""
    psi = X.P.copy()
    psi[0] = 0.0
    w_hat = -1j * g.k[:, None] * psi
    zl, wl = np.polynomial.legendre.leggauss(g.Nz)
    V = np.cos(np.outer(np.arccos(zl), np.arange(g.Nz)))

    def phys(c):
        H = np.zeros((g.Nx // 2 + 1, g.Nz), dtype=np.complex128)
        H[: g.Mx] = (c @ V.T) * g.Nx
        return np.fft.irfft(H, n=g.Nx, axis=0)

    return 0.5 * np.sum(wl * np.mean(phys(w_hat) * phys(X.T), axis=0))


def diagnostics(g: Grid, X: State) -> np.ndarray:
    """The per-state record (Nu_V, Nu_b, Nu_t, KE, epsilon_U, P)."""
    nu_v, nu_b, nu_t = nusselt(g, X)
    return np.array([nu_v, nu_b, nu_t, kinetic_energy(g, X), viscous_dissipation(g, X),
                     buoyancy_production(g, X)])


def time_averages(g: Grid, samples: np.ndarray) -> np.ndarray:
    """Time averages of section 2.2 over records (Nu_V, Nu_b, Nu_t, KE,
    epsilon_U, P): (Nu_V, Nu_b, Nu_t, Nu_int, KE, Re, epsilon_U, P,
    |P - epsilon_U| / P).  Re is the time average of the RMS velocity
    <u^2 + w^2>^(1/2) over the viscosity (free-fall velocity, height 1);
    Nu_int is Eq. 13 on the averaged Nusselt numbers."""
    s = np.asarray(samples, dtype=np.float64).reshape(-1, 6)
    nv, nb, nt, ke, eps, P = s.mean(axis=0)
    re = np.mean(np.sqrt(2.0 * s[:, 3])) / g.nu
    nu_int = max(abs(nb - nv), abs(nb - nt), abs(nv - nt)) / nv
    return np.array([nv, nb, nt, nu_int, ke, re, eps, P, abs(P - eps) / P])


# --------------------------------------------------------------------------
# Transfer between the fine and the coarse grid (section 3.6: the coarse
# propagator has 1/CF of the points in each direction).  Reading: restrict
# by truncating the spectral coefficients, prolong by zero-padding them.
# --------------------------------------------------------------------------


def restrict(X: State, Mx_c: int, Nz_c: int) -> State:
    return State(X.T[:Mx_c, :Nz_c].copy(), X.P[:Mx_c, :Nz_c].copy())


def prolong(X: State, Mx: int, Nz: int) -> State:
    T = np.zeros((Mx, Nz), dtype=np.complex128)
    P = np.zeros((Mx, Nz), dtype=np.complex128)
    a, b = X.T.shape
    T[:a, :b] = X.T
    P[:a, :b] = X.P
    return State(T, P)


# --------------------------------------------------------------------------
# Parareal (section 3.1, Eq. 19), serial.
# --------------------------------------------------------------------------


def steps_per_slice(t0: float, t_end: float, n_slices: int, dt: float):
    """Steps per slice n = ceil(dT/dt) and the uniform step dT/n actually used
    (reading: the requested step is shrunk so each slice has whole steps)."""
    dT = (t_end - t0) / n_slices
    n = int(math.ceil(dT / dt - 1e-9))
    return n, dT / n


@dataclasses.dataclass
class PararealResult:
    U: List[np.ndarray]                  # U_n^K, n = 0..S (packed vectors)
    iterates: List[List[np.ndarray]]     # iterates[k][n] = U_n^k
    defects: List[float]                 # defect after iteration k = 1..K
    k_done: int


def parareal(U0: np.ndarray, n_slices: int, F: Callable, G: Callable,
             k_max: int, tol: float = 0.0) -> PararealResult:
    """Parareal on packed state vectors.

    k = 0: U_(n+1)^0 = G(U_n^0).  Iteration k >= 1:
        U_(n+1)^k = G(U_n^k) + F(U_n^(k-1)) - G(U_n^(k-1))      (Eq. 19).
    Slices n < k are already exact after k iterations (the fine solution
    has propagated through them), so F is applied from slice k-1 on and
    U_k^k is F(U_(k-1)^(k-1)) itself.  The defect between consecutive
    iterates (section 3.7) is max_n ||U_n^k - U_n^(k-1)|| / ||U_n^k||.
    """
    S = n_slices
    U = [np.array(U0, dtype=np.float64)]
    g = []
    for n in range(S):
        g.append(G(U[n], n))
        U.append(g[n].copy())
    iterates = [[u.copy() for u in U]]
    defects = []
    k = 0
    while k < min(k_max, S):
        k += 1
        f = [None] * S
        for n in range(k - 1, S):
            f[n] = F(U[n], n)
        Unew = [u.copy() for u in U]
        Unew[k] = f[k - 1].copy()
        for n in range(k, S):
            gn = G(Unew[n], n)
            Unew[n + 1] = gn + f[n] - g[n]
            g[n] = gn
        d = 0.0
        for n in range(k, S + 1):
            nrm = np.linalg.norm(Unew[n])
            d = max(d, np.linalg.norm(Unew[n] - U[n]) / (nrm if nrm > 0 else 1.0))
        U = Unew
        iterates.append([u.copy() for u in U])
        defects.append(d)
        if d <= tol:
            break
    return PararealResult(U, iterates, defects, k)


class RBCParareal:
    """F and G for Rayleigh-Benard: F = ``nf`` fine steps on the fine grid;
    G = restrict, ``nc`` coarse steps, prolong."""

    def __init__(self, fine: Grid, coarse: Grid, t0: float, t_end: float, n_slices: int):
        self.nf, dtf = steps_per_slice(t0, t_end, n_slices, fine.dt)
        self.nc, dtc = steps_per_slice(t0, t_end, n_slices, coarse.dt)
        self.fine = dataclasses.replace(fine, dt=dtf)
        self.coarse = dataclasses.replace(coarse, dt=dtc)
        self.Fs = Stepper(self.fine)
        self.Gs = Stepper(self.coarse)
        self.S = n_slices

    def F(self, u: np.ndarray, n: int) -> np.ndarray:
        g = self.fine
        return self.Fs.run(State.unpack(u, g.Mx, g.Nz), self.nf).pack()

    def G(self, u: np.ndarray, n: int) -> np.ndarray:
        g, c = self.fine, self.coarse
        X = restrict(State.unpack(u, g.Mx, g.Nz), c.Mx, c.Nz)
        X = self.Gs.run(X, self.nc)
        return prolong(X, g.Mx, g.Nz).pack()

    def run(self, U0: np.ndarray, k_max: int, tol: float = 0.0) -> PararealResult:
        return parareal(U0, self.S, self.F, self.G, k_max, tol)
