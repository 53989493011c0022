"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module holds no arithmetic of the method itself.  It provides

* the counter-based noise generator used for the initial temperature
  perturbation: SplitMix64 (Steele, Lea & Flood, "Fast splittable
  pseudorandom number generators", OOPSLA 2014) turned into 53-bit uniforms
  and then into standard normals by the Box-Muller transform (cosine branch
  only).  The C library re-implements the same published generator on its
  own (``rbc_init_state``); only the definition is shared, never code;
* the workload descriptions (Rayleigh number, grids, time steps, slices)
  of the runs the paper's method is exercised on (section 2.1 of the paper
  fixes Pr = 1 and aspect ratio 2; the rest is the synthetic workload
  recipe documented in the design notes).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, counters: np.ndarray) -> np.ndarray:
    """SplitMix64 output number ``c`` of the stream started at ``seed``.

    The generator state after ``c + 1`` increments is ``seed + (c+1)*golden``;
    the output is that state passed through the SplitMix64 finaliser.
    """
    c = np.asarray(counters, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + (c + np.uint64(1)) * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform53(seed: int, counters: np.ndarray) -> np.ndarray:
    """Uniform doubles in [0, 1): the top 53 bits of SplitMix64 times 2^-53."""
    z = splitmix64(seed, counters)
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def gaussian_noise(seed: int, nx: int, nz: int) -> np.ndarray:
    """Standard normal noise xi[ix, iz] on an nx-by-nz collocation grid.

    Point p = ix*nz + iz uses uniforms u1 = U(2p), u2 = U(2p+1) and
    xi = sqrt(-2 ln(1 - u1)) * cos(2 pi u2)  (Box-Muller, cosine branch).
    """
    p = np.arange(nx * nz, dtype=np.uint64)
    u1 = uniform53(seed, 2 * p)
    u2 = uniform53(seed, 2 * p + 1)
    xi = np.sqrt(-2.0 * np.log(1.0 - u1)) * np.cos(2.0 * math.pi * u2)
    return xi.reshape(nx, nz)


@dataclasses.dataclass(frozen=True)
class Workload:
    """One synthetic run: physical parameters, grids, time steps, slices."""
    name: str
    Ra: float
    Pr: float
    Lx: float
    Lz: float
    Nx: int
    Nz: int
    Nx_c: int
    Nz_c: int
    t0: float
    t_end: float
    n_slices: int
    dt_f: float
    dt_c: float
    scheme: int          # 2 = ARS(2,2,2), 4 = ARS(4,4,3)
    mixed: bool          # False: all-FP64; True: FP32 bulk, FP64 solves
    noise_amp: float = 1e-3
    seed: int = 0
    k_max: int = 4
    tol: float = 0.0


# The small plain FP64 case: Ra 1e4, 64x32, IMEX RK2, dt 1e-3 to t = 10,
# 4 slices, coarse dt 1e-2 on the same grid, at most 4 iterations.
C1 = Workload("ra1e4_64x32_s4_ars222_fp64", 1e4, 1.0, 2.0, 1.0, 64, 32, 64, 32,
              0.0, 10.0, 4, 1e-3, 1e-2, 2, False, k_max=4, tol=0.0)
# Ra 1e6, 256x64, 32 slices over [0, 50], fine dt 2e-4, coarse 128x32 at
# dt 2e-3, ARS(4,4,3); mixed precision; stop at defect <= 1e-8.
C2 = Workload("ra1e6_256x64_s32_ars443_mixed", 1e6, 1.0, 2.0, 1.0, 256, 64, 128, 32,
              0.0, 50.0, 32, 2e-4, 2e-3, 4, True, k_max=32, tol=1e-8)
C2_FP64 = dataclasses.replace(C2, name="ra1e6_256x64_s32_ars443_fp64", mixed=False)
# Ra 1e8, 1024x256, 64 slices over [0, 20], fine dt 2e-5, coarse 256x64 at
# 10x the fine step, mixed precision.
C3 = Workload("ra1e8_1024x256_s64_ars443_mixed", 1e8, 1.0, 2.0, 1.0, 1024, 256, 256, 64,
              0.0, 20.0, 64, 2e-5, 2e-4, 4, True, k_max=10, tol=0.0)

WORKLOADS = {w.name: w for w in (C1, C2, C2_FP64, C3)}


# Ensemble of independent runs: 24 runs, run i with its own seed 4000 + i,
# Ra log-uniform in [1e5, 1e7], fine grid uniform over {128x32, 256x64,
# 512x128} restricted to the grids that resolve Ra (above 1e6: at least
# 256x64), coarse grid half the fine one in each direction, fine step
# 1e-4 * 64 / Nz, coarse step ten times that, 16 slices each, mixed
# precision.  The horizon is a parameter (the runs' length, not their
# shape, sets the cost).
ENSEMBLE_GRIDS = ((128, 32), (256, 64), (512, 128))


def ensemble_runs(n_runs: int = 24, t_end: float = 10.0, n_slices: int = 16, seed0: int = 4000):
    """The runs of the ensemble workload as Workloads (name, Ra, grids,
    steps, slices), drawn from each run's own seed."""
    runs = []
    for i in range(n_runs):
        u = uniform53(seed0 + i, np.arange(2, dtype=np.uint64))
        Ra = 10.0 ** (5.0 + 2.0 * u[0])
        grids = [g for g in ENSEMBLE_GRIDS if Ra <= 1e6 or g[1] >= 64]
        Nx, Nz = grids[min(int(u[1] * len(grids)), len(grids) - 1)]
        dt = 1e-4 * 64 / Nz
        runs.append(Workload(f"ensemble_run{i}", Ra, 1.0, 2.0, 1.0, Nx, Nz, Nx // 2, Nz // 2, 0.0, t_end, n_slices,
                             dt, 10 * dt, 4, True, seed=seed0 + i, k_max=n_slices, tol=1e-8))
    return runs
