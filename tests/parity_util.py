"""Helpers of the GPU parity tests: per-block relative errors, developed-flow
input states and the advection-off oracle used to show that a comparison
can see the nonlinear terms.

A state vector [field][m][re, im][n] is compared block by block, each block
against its own norm, so that no block hides behind a larger one (the
temperature's conduction profile dominates a whole-state norm):
  psi    field 0: streamfunction modes m >= 1 and the mean flow u_bar (m = 0)
  T'     field 1, modes m >= 1
  T0     field 1, mode 0 (the horizontal mean temperature)
  T0dev  the same minus the conduction profile (developed-flow tests: the
         mean profile's change is small against the profile itself)
"""
import numpy as np

import rbc_inputs as I
from oracle import rbc_oracle as O


def blocks(v, g, dev_T0=False):
    a = np.asarray(v).reshape(2, g.Mx, 2, g.Nz)
    out = {"psi": a[0].ravel(), "T'": a[1, 1:].ravel(), "T0": a[1, 0].ravel()}
    if dev_T0:
        cond = O.conduction_state(g).T[0]
        d = a[1, 0].copy()
        d[0] -= cond.real
        out["T0dev"] = d.ravel()
    return out


def block_errors(got, ref, g, dev_T0=False):
    bg, br = blocks(got, g, dev_T0), blocks(ref, g, dev_T0)
    return {k: float(np.linalg.norm(bg[k] - br[k]) / max(np.linalg.norm(br[k]), 1e-300)) for k in br}


def assert_blocks(got, ref, g, tol, what="", dev_T0=False):
    e = block_errors(got, ref, g, dev_T0)
    bad = {k: v for k, v in e.items() if not v < tol}
    assert not bad, f"{what}: per-block relative L2 above {tol:g}: {e}"
    return e


def developed_state(g, seed, amp=0.3, modes=8):
    """A flow-like state that satisfies the wall conditions: streamfunction
    rolls z^2 (1-z)^2 (1 + c (z - 1/2)) in modes 1..8 with seeded phases and
    amplitudes decaying as exp(-(m-1)/3), temperature rolls z (1-z) (...) in
    phase with the vertical velocity (so that <w T> and the mean-profile
    forcing are nonzero), a mean-temperature bump and a mean shear, all
    O(amp), on the collocation grid, transformed by the oracle."""
    x, z = O.grid_points(g)
    r = I.gaussian_noise(seed, 8, 16)
    k = g.k[1]
    zz = z / g.Lz
    psi = np.zeros((g.Nx, g.Nz))
    T = np.zeros((g.Nx, g.Nz))
    for m in range(1, min(modes, g.Mx // 2) + 1):
        e = np.exp(-(m - 1) / 3.0)
        a, b = r[m % 8, 0], r[m % 8, 1]
        c, s = np.cos(m * k * x)[:, None], np.sin(m * k * x)[:, None]
        psi += e * (a * c + b * s) * (zz ** 2 * (1 - zz) ** 2 * (1 + r[m % 8, 2] * (zz - 0.5)))[None, :]
        T += e * (a * s - b * c + 0.3 * r[m % 8, 3] * c) * (zz * (1 - zz) * (1 + r[m % 8, 5] * (zz - 0.5)))[None, :]
    cond = g.T_bot - z[None, :] if g.flux else (g.T_bot + (g.T_top - g.T_bot) * zz)[None, :]
    Tg = cond + amp * (T + (zz * (1 - zz) * r[0, 6])[None, :])
    X = O.State(O.from_grid(Tg, g.Mx, g.Nz), O.from_grid(amp * 4 * psi, g.Mx, g.Nz))
    X.T[0] = X.T[0].real
    ub = amp * 0.5 * zz * (1 - zz) * (1 + r[0, 7] * (zz - 0.5))
    X.P[0] = O.cheb_forward_matrix(g.Nz, g.Nz) @ ub
    return X


class NoAdvectionStepper(O.Stepper):
    """The oracle's stepper with the explicit (advective) terms switched off:
    the size of the difference it makes is the size of what a parity
    comparison must be able to see."""

    def explicit(self, X):
        E = super().explicit(X)
        return O.State(np.zeros_like(E.T), np.zeros_like(E.P))


def assert_sensitive(ref, ref_noadv, g, tol, what="", factor=100.0):
    """Every block (T0 as its deviation from conduction) moves by at least
    factor x tol when advection is switched off."""
    e = block_errors(ref_noadv, ref, g, dev_T0=True)
    e.pop("T0")
    weak = {k: v for k, v in e.items() if not v >= factor * tol}
    assert not weak, f"{what}: advection changes these blocks by less than {factor:g} x {tol:g}: {e}"
    return e
