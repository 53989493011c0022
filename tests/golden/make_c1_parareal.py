"""Writes c1_parareal.json: the oracle's Parareal (section 3.1, Eq. 19) at the
64x32, 4-slice workload (Ra 1e4, Pr 1, 2x1 box, ARS(2,2,2), FP64, t in
[0, 10], fine step 1e-3, coarse propagator on the same grid at step 1e-2),
from the seeded initial state of section 2.1, run to finite termination
(k = 4).  Stored as sampled outputs, per iteration k = 0..4: the defect
(section 3.7) and, per slice boundary n = 0..4 and per block of the state
(psi / u_bar coefficients; T for m >= 1; T for m = 0), the L2 norm of the
block and 16 coefficients at fixed positions in it.  State layout:
[field psi|u_bar, T][m < Nx/2][re, im][n < Nz].  Calls only oracle/ and the
shared input generator (about five minutes on one core).

    python tests/golden/make_c1_parareal.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import rbc_inputs as I  # noqa: E402
from oracle import rbc_oracle as O  # noqa: E402

N_SAMPLES = 16


def blocks(Mx: int, Nz: int):
    """(name, first, end) of the sampled blocks of a packed state."""
    half = Mx * 2 * Nz
    return [("psi", 0, half), ("T_m_ge_1", half + 2 * Nz, 2 * half), ("T_m0", half, half + 2 * Nz)]


def sample_positions(a: int, b: int):
    return [int(v) for v in np.linspace(a, b - 1, N_SAMPLES + 2)[1:-1].round()]


def main() -> int:
    w = I.C1
    fine = O.Grid(w.Ra, w.Pr, w.Lx, w.Lz, w.Nx, w.Nz, w.dt_f, scheme=w.scheme)
    coarse = O.Grid(w.Ra, w.Pr, w.Lx, w.Lz, w.Nx_c, w.Nz_c, w.dt_c, scheme=w.scheme)
    pp = O.RBCParareal(fine, coarse, w.t0, w.t_end, w.n_slices)
    U0 = O.initial_state(fine, I.gaussian_noise(w.seed, fine.Nx, fine.Nz), w.noise_amp).pack()
    res = pp.run(U0, k_max=w.n_slices)
    out = {
        "description": __doc__.strip().split("\n\n")[0],
        "workload": w.name,
        "k_done": res.k_done,
        "defects": [float(d) for d in res.defects],
        "blocks": {},
    }
    for name, a, b in blocks(fine.Mx, fine.Nz):
        pos = sample_positions(a, b)
        out["blocks"][name] = {
            "range": [a, b],
            "positions": pos,
            "norms": [[float(np.linalg.norm(u[a:b])) for u in it] for it in res.iterates],
            "samples": [[[float(u[i]) for i in pos] for u in it] for it in res.iterates],
        }
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "c1_parareal.json"), "w") as f:
        json.dump(out, f, indent=1)
    print("k_done", res.k_done, "defects", out["defects"])
    return 0


if __name__ == "__main__":
    sys.exit(main())
