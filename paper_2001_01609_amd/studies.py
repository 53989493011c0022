"""Parareal convergence and cost studies of section 4 on one GPU.

Each case runs Parareal to finite termination (k = number of slices) with
the iterate history on: the last iterate is then the serial fine solution
at every slice boundary, so one run gives, for every iteration k,
  - the defect (section 3.7),
  - the L2 error of U_k against the serial fine solution, at the final time
    and the maximum over slice boundaries,
  - the error of the time-averaged Nu_V against the serial fine run's, and
    the internal checks Nu_int (Eq. 13) and |P - epsilon_U|/P (Eq. 15)
    (Figs. 7-9),
  - the kinetic energy at every slice boundary (Fig. 5),
  - the wall time at which iteration k was complete (pipelined schedule),
and, against one serial FP64 fine run over the same window on the same GPU,
the speed-up at the first iteration that meets 1% in the L2 error or in the
Nusselt number (Fig. 10).

Studies: `iterations` (Ra 1e5, 1e6, 1e7, 10 slices, coarsening factor 4),
`cf` (coarsening factors 2, 4, 8 at Ra 1e6, section 3.6), `slices` (4 to 32
slices at Ra 1e6).  All inputs are the seeded conduction profile plus noise.

    python -m paper_2001_01609_amd.studies --study iterations --out studies.json
"""
from __future__ import annotations

import argparse
import json
import sys
import time
from typing import Dict, List

import numpy as np


def _case_params(R, Ra, Nx, Nz, cf, S, t_end, dt_f, dt_c, nu_stride):
    p = R.rbc_default_params()
    p.Ra, p.Pr, p.Lx, p.Lz = Ra, 1.0, 2.0, 1.0
    p.Nx, p.Nz = Nx, Nz
    p.Nx_c, p.Nz_c = Nx // cf, Nz // cf
    p.t0, p.t_end, p.n_slices = 0.0, t_end, S
    p.dt_f, p.dt_c = dt_f, dt_c
    p.scheme_f = p.scheme_c = R.RBC_ARS443
    p.precision = R.RBC_FP64
    p.nu_stride = nu_stride
    p.nu_t_start = 0.0
    p.pipelined = 1
    return p


def run_case(Ra: float, Nx: int, Nz: int, cf: int, S: int, t_end: float, dt_f: float, dt_c: float,
             seed: int = 0, amp: float = 1e-3, nu_stride: int = 20, serial: bool = True) -> Dict:
    import torch

    from paper_2001_01609_amd import rbc as R
    dev = torch.device("cuda:0")
    st = torch.cuda.current_stream(dev).cuda_stream
    p = _case_params(R, Ra, Nx, Nz, cf, S, t_end, dt_f, dt_c, nu_stride)
    out: Dict = {"Ra": Ra, "grid": [Nx, Nz], "coarse_grid": [Nx // cf, Nz // cf], "cf": cf, "slices": S,
                 "t_end": t_end, "dt_f": dt_f, "dt_c": dt_c}
    h = R.rbc_create(p, st)
    try:
        n = R.rbc_state_size(h, 0)
        nf, dtf = R.rbc_steps_per_slice(h, 0)
        nc, dtc = R.rbc_steps_per_slice(h, 1)
        out.update({"fine_steps_per_slice": nf, "coarse_steps_per_slice": nc})
        hist = torch.zeros((S + 1) * (S + 1) * n, dtype=torch.float64, device=dev)
        R.rbc_set_iterate_history(h, hist, S)
        U = torch.zeros((S + 1) * n, dtype=torch.float64, device=dev)
        R.rbc_init_state(h, seed, amp, U)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        try:
            status, kd, defects, avg = R.parareal_iterate(h, U, S, 0.0, want_nu=True)
        except R.RbcError as e:
            out["error"] = str(e)
            return out
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        at = R.rbc_get_pipeline_stats(h)["report_at_s"][: S + 1]
        Hs = hist.view(S + 1, S + 1, n)
        ref = Hs[S]
        ke = np.stack([R.rbc_diagnostics(h, Hs[k].contiguous(), S + 1)[:, 3] for k in range(S + 1)])
        l2_final, l2_max = [], []
        for k in range(S + 1):
            d = torch.linalg.norm(Hs[k][1:] - ref[1:], dim=1) / torch.linalg.norm(ref[1:], dim=1)
            l2_final.append(float(d[-1]))
            l2_max.append(float(d.max()))
    finally:
        R.rbc_destroy(h)
    nuv = avg[:, 0]
    out.update({
        "parareal_wall_s": wall,
        "iteration_done_at_s": [float(v) for v in at],
        "defects": [float(v) for v in defects],
        "l2_final": l2_final, "l2_max": l2_max,
        "nu_v": [float(v) for v in nuv],
        "nu_err": [float(abs(v - nuv[S]) / abs(nuv[S])) for v in nuv],
        "nu_int": [float(v) for v in avg[:, 3]],
        "balance": [float(v) for v in avg[:, 8]],
        "re": [float(v) for v in avg[:, 5]],
        "ke_at_slice_ends": ke.tolist(),
    })
    if serial:
        q = _case_params(R, Ra, Nx, Nz, cf, 1, t_end, dtf, dtf, 0)
        h = R.rbc_create(q, st)
        try:
            V = torch.zeros(n, dtype=torch.float64, device=dev)
            R.rbc_init_state(h, seed, amp, V)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            R.rbc_fine_step_batch(h, V, V, 1, S * nf, None)
            torch.cuda.synchronize()
            t_ser = time.perf_counter() - t0
        finally:
            R.rbc_destroy(h)
        out["serial_fp64_s"] = t_ser
        for name, err in (("l2", l2_final), ("nu", out["nu_err"])):
            k1 = next((k for k in range(1, S + 1) if err[k] <= 1e-2), S)
            out[f"k_{name}_1pct"] = k1
            out[f"speedup_{name}_1pct"] = t_ser / at[k1] if at[k1] > 0 else None
    return out


STUDIES = {
    # Figs. 5, 7-9: per-iteration convergence at three Rayleigh numbers (10
    # slices, CF 4, coarse step twice the fine one)
    "iterations": [
        dict(Ra=1e5, Nx=64, Nz=32, cf=4, S=10, t_end=50.0, dt_f=2e-3, dt_c=4e-3),
        dict(Ra=1e6, Nx=128, Nz=64, cf=4, S=10, t_end=50.0, dt_f=5e-4, dt_c=1e-3),
        dict(Ra=1e7, Nx=128, Nz=64, cf=4, S=10, t_end=30.0, dt_f=2.5e-4, dt_c=5e-4),
    ],
    # section 3.6: coarsening factors 2, 4, 8
    "cf": [dict(Ra=1e6, Nx=128, Nz=64, cf=cf, S=10, t_end=50.0, dt_f=5e-4, dt_c=1e-3) for cf in (2, 4, 8)],
    # Fig. 10: speed-up against the number of slices
    "slices": [dict(Ra=1e6, Nx=128, Nz=64, cf=4, S=S, t_end=50.0, dt_f=5e-4, dt_c=1e-3) for S in (4, 8, 16, 32)],
}


def table(cases: List[Dict]) -> str:
    """Markdown summary: one row per case."""
    rows = ["| Ra | grid / coarse | slices | iterations to 1% L2 | to 1% Nu_V | speed-up (L2 / Nu) | "
            "Nu_V err k=0,1,2 | L2 err k=1,2,3 |", "|---|---|---|---|---|---|---|---|"]
    for c in cases:
        if "error" in c:
            rows.append(f"| {c['Ra']:.0e} | {c['grid'][0]}x{c['grid'][1]} / {c['coarse_grid'][0]}x"
                        f"{c['coarse_grid'][1]} | {c['slices']} | {c['error']} | | | | |")
            continue
        nu = ", ".join(f"{v:.1e}" for v in c["nu_err"][:3])
        l2 = ", ".join(f"{v:.1e}" for v in c["l2_final"][1:4])
        rows.append(f"| {c['Ra']:.0e} | {c['grid'][0]}x{c['grid'][1]} / {c['coarse_grid'][0]}x{c['coarse_grid'][1]} "
                    f"| {c['slices']} | {c.get('k_l2_1pct')} | {c.get('k_nu_1pct')} | "
                    f"{c.get('speedup_l2_1pct', 0):.2f} / {c.get('speedup_nu_1pct', 0):.2f} | {nu} | {l2} |")
    return "\n".join(rows)


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--study", choices=sorted(STUDIES), action="append", required=True)
    ap.add_argument("--out", default=None, help="JSON file for every case's full record")
    args = ap.parse_args()
    res: Dict[str, List[Dict]] = {}
    for name in args.study:
        res[name] = []
        for cfg in STUDIES[name]:
            print(f"[study {name}] {cfg}", file=sys.stderr, flush=True)
            t0 = time.perf_counter()
            res[name].append(run_case(**cfg))
            print(f"[study {name}] done in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
        print(f"\n## {name}\n\n{table(res[name])}\n", flush=True)
    if args.out:
        with open(args.out, "w") as f:
            json.dump(res, f)
    return 0


if __name__ == "__main__":
    sys.exit(main())
