"""Python binding of librbc (include/rbc.h): argument marshalling only.

Every function has the name of the C entry point it calls.  Device arrays
are passed as torch tensors (float64, contiguous, on the GPU) or as raw
integer device addresses; all arithmetic happens in the HIP library.  If
the library has not been built, importing this module raises: there is no
other implementation behind these names.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librbc.so")

RBC_OK = 0
RBC_NOT_CONVERGED = 1
RBC_ERR_ARG = -1
RBC_ERR_OOM = -2
RBC_ERR_HIP = -3
RBC_ERR_NONFINITE = -4
RBC_ERR_STATE = -5
RBC_FP64 = 0
RBC_MIXED = 1
RBC_BC_TEMPERATURE, RBC_BC_FLUX = 0, 1
RBC_DIAG = 6
RBC_DIAG_AVG = 9
DIAG_FIELDS = ("Nu_V", "Nu_b", "Nu_t", "KE", "eps_U", "P")
DIAG_AVG_FIELDS = ("Nu_V", "Nu_b", "Nu_t", "Nu_int", "KE", "Re", "eps_U", "P", "balance")
RBC_STOP_DEFECT, RBC_STOP_STATISTICS, RBC_STOP_KMAX, RBC_STOP_EXACT = 0, 1, 2, 3
RBC_ARS222 = 2
RBC_ARS443 = 4


class RbcError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"rbc status {status}: {msg}")
        self.status = status


class rbc_params(ctypes.Structure):
    _fields_ = [
        ("Ra", ctypes.c_double), ("Pr", ctypes.c_double),
        ("Lx", ctypes.c_double), ("Lz", ctypes.c_double),
        ("Nx", ctypes.c_int32), ("Nz", ctypes.c_int32),
        ("Nx_c", ctypes.c_int32), ("Nz_c", ctypes.c_int32),
        ("t0", ctypes.c_double), ("t_end", ctypes.c_double),
        ("n_slices", ctypes.c_int32),
        ("dt_f", ctypes.c_double), ("dt_c", ctypes.c_double),
        ("scheme_f", ctypes.c_int32), ("scheme_c", ctypes.c_int32),
        ("precision", ctypes.c_int32), ("nu_stride", ctypes.c_int32),
        ("nu_t_start", ctypes.c_double),
        ("T_bot", ctypes.c_double), ("T_top", ctypes.c_double),
        ("promote_fp64", ctypes.c_int32),
        ("pipelined", ctypes.c_int32),
        ("stat_tol", ctypes.c_double),
        ("bc_T", ctypes.c_int32),
    ]


class rbc_pipeline_stats(ctypes.Structure):
    _fields_ = [
        ("wall_s", ctypes.c_double),
        ("host_admit_s", ctypes.c_double), ("host_fine_s", ctypes.c_double),
        ("host_coarse_s", ctypes.c_double), ("host_report_s", ctypes.c_double),
        ("host_wait_s", ctypes.c_double),
        ("fine_steps", ctypes.c_int64), ("coarse_chunks", ctypes.c_int64),
        ("mean_runs_per_step", ctypes.c_double),
        ("report_at_s", ctypes.c_double * 64),
    ]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"librbc.so is not built ({LIB_PATH}); run __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    vp, i32, dbl, st = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double, ctypes.c_int
    sig = {
        "rbc_default_params": (st, [P(rbc_params)]),
        "rbc_query_footprint": (st, [P(rbc_params), P(ctypes.c_size_t)]),
        "rbc_create": (st, [P(rbc_params), vp, P(vp)]),
        "rbc_destroy": (st, [vp]),
        "rbc_last_error": (ctypes.c_char_p, [vp]),
        "rbc_state_size": (st, [vp, i32, P(ctypes.c_size_t)]),
        "rbc_steps_per_slice": (st, [vp, i32, P(i32), P(dbl)]),
        "rbc_init_state": (st, [vp, ctypes.c_uint64, dbl, vp]),
        "rbc_fine_step_batch": (st, [vp, vp, vp, i32, i32, vp]),
        "rbc_coarse_sweep": (st, [vp, i32, i32, vp, vp, vp, P(dbl)]),
        "parareal_iterate": (st, [vp, vp, i32, dbl, P(i32), P(dbl), P(dbl)]),
        "rbc_nusselt": (st, [vp, vp, i32, P(dbl)]),
        "rbc_fine_fp64_from": (st, [vp, P(i32)]),
        "rbc_stop_reason": (st, [vp, P(i32)]),
        "rbc_set_iterate_history": (st, [vp, vp, i32]),
        "rbc_diagnostics": (st, [vp, vp, i32, P(dbl)]),
        "rbc_explicit_terms": (st, [vp, vp, vp]),
        "rbc_kernel_timing_enable": (st, [vp, i32, i32]),
        "rbc_kernel_timing": (st, [vp, P(dbl), P(ctypes.c_int64), P(dbl)]),
        "rbc_synchronize": (st, [vp]),
        "rbc_get_pipeline_stats": (st, [vp, P(rbc_pipeline_stats)]),
        "rbc_diagnostics_noalloc": (st, [vp, vp, i32, vp]),
        "rbc_get_state": (st, [vp, vp, P(ctypes.c_size_t)]),
        "rbc_initial_state": (st, [P(rbc_params), ctypes.c_uint64, dbl, vp, vp]),
        "rbc_tuning_load": (st, [ctypes.c_char_p]),
        "rbc_tuning_entries": (st, [P(i32)]),
        "rbc_ensemble_create": (st, [vp, P(vp)]),
        "rbc_ensemble_destroy": (st, [vp]),
        "rbc_ensemble_last_error": (ctypes.c_char_p, [vp]),
        "rbc_ensemble_footprint": (st, [P(rbc_params), P(ctypes.c_size_t)]),
        "rbc_ensemble_add": (st, [vp, P(rbc_params), vp, i32, dbl, P(i32)]),
        "rbc_ensemble_step": (st, [vp, P(i32)]),
        "rbc_ensemble_run_info": (st, [vp, i32, P(i32), P(i32), P(i32), P(dbl), i32]),
        "rbc_ensemble_result": (st, [vp, i32, vp]),
        "rbc_ensemble_release": (st, [vp, i32]),
        "rbc_ensemble_run_bytes": (st, [vp, i32, P(ctypes.c_size_t)]),
        "rbc_set_state": (st, [vp, vp, ctypes.c_size_t]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_lib = _load()

# launch shapes measured on gfx950 (paper_2001_01609_amd/tune.py writes it)
TUNING_TABLE = os.path.join(_HERE, "tuning_gfx950.txt")


def rbc_tuning_load(path: Optional[str]) -> None:
    _check(_lib.rbc_tuning_load(path.encode() if path else None))


def rbc_tuning_entries() -> int:
    n = ctypes.c_int32()
    _check(_lib.rbc_tuning_entries(ctypes.byref(n)))
    return n.value



def _check(status: int, h=None) -> int:
    if status < 0:
        msg = _lib.rbc_last_error(h)
        raise RbcError(status, msg.decode() if msg else "")
    return status


if os.path.exists(TUNING_TABLE) and not os.environ.get("RBC_NO_TUNING"):
    rbc_tuning_load(TUNING_TABLE)


def _ptr(x) -> Optional[int]:
    if x is None:
        return None
    if hasattr(x, "data_ptr"):
        if not x.is_cuda or str(x.dtype) != "torch.float64" or not x.is_contiguous():
            raise ValueError("device arrays must be contiguous float64 CUDA/HIP tensors")
        return x.data_ptr()
    return int(x)


def rbc_default_params() -> rbc_params:
    p = rbc_params()
    _check(_lib.rbc_default_params(ctypes.byref(p)))
    return p


def rbc_query_footprint(p: rbc_params) -> int:
    n = ctypes.c_size_t()
    _check(_lib.rbc_query_footprint(ctypes.byref(p), ctypes.byref(n)))
    return n.value


def rbc_create(p: rbc_params, stream: Optional[int] = None):
    h = ctypes.c_void_p()
    _check(_lib.rbc_create(ctypes.byref(p), stream, ctypes.byref(h)))
    return h


def rbc_destroy(h) -> None:
    _check(_lib.rbc_destroy(h), h)


def rbc_last_error(h=None) -> str:
    return (_lib.rbc_last_error(h) or b"").decode()


def rbc_state_size(h, coarse: int = 0) -> int:
    n = ctypes.c_size_t()
    _check(_lib.rbc_state_size(h, coarse, ctypes.byref(n)), h)
    return n.value


def rbc_steps_per_slice(h, coarse: int = 0) -> Tuple[int, float]:
    n, dt = ctypes.c_int32(), ctypes.c_double()
    _check(_lib.rbc_steps_per_slice(h, coarse, ctypes.byref(n), ctypes.byref(dt)), h)
    return n.value, dt.value


def rbc_init_state(h, seed: int, noise_amp: float, U0) -> None:
    _check(_lib.rbc_init_state(h, seed, noise_amp, _ptr(U0)), h)


def rbc_initial_state(p: rbc_params, seed: int, noise_amp: float, U0, stream: Optional[int] = None) -> None:
    _check(_lib.rbc_initial_state(ctypes.byref(p), seed, noise_amp, _ptr(U0), stream))


def rbc_fine_step_batch(h, U_in, U_out, n_slices: int, n_steps: int, nu_samples=None) -> None:
    _check(_lib.rbc_fine_step_batch(h, _ptr(U_in), _ptr(U_out), n_slices, n_steps, _ptr(nu_samples)), h)


def rbc_coarse_sweep(h, mode: int, first_slice: int, U, F, G, want_defect: bool = False):
    d = ctypes.c_double()
    _check(_lib.rbc_coarse_sweep(h, mode, first_slice, _ptr(U), _ptr(F), _ptr(G),
                                 ctypes.byref(d) if want_defect else None), h)
    return d.value if want_defect else None


def parareal_iterate(h, U, k_max: int, tol: float, want_nu: bool = False):
    """Returns (status, k_done, defects[k_done], averages[k_done+1, RBC_DIAG_AVG]
    or None); the averages' columns are DIAG_AVG_FIELDS."""
    k = ctypes.c_int32()
    defects = np.zeros(max(k_max, 1))
    nu = np.full((k_max + 1, RBC_DIAG_AVG), np.nan) if want_nu else None
    st = _check(_lib.parareal_iterate(
        h, _ptr(U), k_max, tol, ctypes.byref(k),
        defects.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
        nu.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if want_nu else None), h)
    kd = k.value
    return st, kd, defects[:kd].copy(), (nu[: kd + 1].copy() if want_nu else None)


def rbc_get_state(h) -> bytes:
    """The handle's Parareal checkpoint after the last parareal_iterate."""
    n = ctypes.c_size_t()
    _check(_lib.rbc_get_state(h, None, ctypes.byref(n)), h)
    buf = ctypes.create_string_buffer(n.value)
    _check(_lib.rbc_get_state(h, buf, ctypes.byref(n)), h)
    return buf.raw[: n.value]


def rbc_set_state(h, ckpt: bytes) -> None:
    buf = ctypes.create_string_buffer(bytes(ckpt), len(ckpt))
    _check(_lib.rbc_set_state(h, buf, len(ckpt)), h)


def rbc_set_iterate_history(h, U_hist, k_cap: int) -> None:
    """U_hist: device float64 tensor of (k_cap + 1) (n_slices + 1) states, or None."""
    _check(_lib.rbc_set_iterate_history(h, _ptr(U_hist) if U_hist is not None else None, k_cap), h)


def rbc_stop_reason(h) -> int:
    r = ctypes.c_int32()
    _check(_lib.rbc_stop_reason(h, ctypes.byref(r)), h)
    return r.value


def rbc_diagnostics(h, U, n_states: int) -> np.ndarray:
    """[n_states, RBC_DIAG] records (columns DIAG_FIELDS)."""
    out = np.zeros((max(n_states, 1), RBC_DIAG))
    _check(_lib.rbc_diagnostics(h, _ptr(U), n_states,
                                out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), h)
    return out[:n_states]


def rbc_diagnostics_noalloc(h, U, n_states: int, out) -> None:
    """Records into the device tensor out ([n_states * RBC_DIAG] float64);
    asynchronous, allocates nothing."""
    _check(_lib.rbc_diagnostics_noalloc(h, _ptr(U), n_states, _ptr(out)), h)


def rbc_fine_fp64_from(h) -> int:
    k = ctypes.c_int32()
    _check(_lib.rbc_fine_fp64_from(h, ctypes.byref(k)), h)
    return k.value


def rbc_nusselt(h, U, n_states: int) -> np.ndarray:
    out = np.zeros((max(n_states, 1), 3))
    _check(_lib.rbc_nusselt(h, _ptr(U), n_states,
                            out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), h)
    return out[:n_states]


def rbc_explicit_terms(h, U, E) -> None:
    _check(_lib.rbc_explicit_terms(h, _ptr(U), _ptr(E)), h)


def rbc_kernel_timing_enable(h, kernel: int, every: int) -> None:
    _check(_lib.rbc_kernel_timing_enable(h, kernel, every), h)


def rbc_kernel_timing(h) -> Tuple[float, int, float]:
    """(mean launch ms, timed launches, mean states per timed launch)."""
    ms, n, b = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double()
    _check(_lib.rbc_kernel_timing(h, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(b)), h)
    return ms.value, n.value, b.value


def rbc_synchronize(h) -> None:
    _check(_lib.rbc_synchronize(h), h)


def rbc_get_pipeline_stats(h) -> dict:
    """Scheduler statistics of the last pipelined parareal_iterate."""
    out = rbc_pipeline_stats()
    _check(_lib.rbc_get_pipeline_stats(h, ctypes.byref(out)), h)
    d = {name: getattr(out, name) for name, _ in rbc_pipeline_stats._fields_ if name != "report_at_s"}
    d["report_at_s"] = list(out.report_at_s)
    return d


def params_from_workload(w, **overrides) -> rbc_params:
    """rbc_params for a rbc_inputs.Workload (field-by-field copy)."""
    p = rbc_default_params()
    p.Ra, p.Pr, p.Lx, p.Lz = w.Ra, w.Pr, w.Lx, w.Lz
    p.Nx, p.Nz, p.Nx_c, p.Nz_c = w.Nx, w.Nz, w.Nx_c, w.Nz_c
    p.t0, p.t_end, p.n_slices = w.t0, w.t_end, w.n_slices
    p.dt_f, p.dt_c = w.dt_f, w.dt_c
    p.scheme_f = p.scheme_c = w.scheme
    p.precision = RBC_MIXED if w.mixed else RBC_FP64
    for k, v in overrides.items():
        setattr(p, k, v)
    return p


# ---------------------------------------------------------------- ensembles ---

def _echeck(status: int, e) -> int:
    if status < 0:
        msg = _lib.rbc_ensemble_last_error(e) if e else b""
        raise RbcError(status, msg.decode() if msg else "")
    return status


def rbc_ensemble_create(stream: Optional[int] = None):
    e = ctypes.c_void_p()
    _echeck(_lib.rbc_ensemble_create(stream, ctypes.byref(e)), None)
    return e


def rbc_ensemble_destroy(e) -> None:
    _echeck(_lib.rbc_ensemble_destroy(e), None)


def rbc_ensemble_last_error(e) -> str:
    return (_lib.rbc_ensemble_last_error(e) or b"").decode()


def rbc_ensemble_footprint(p: rbc_params) -> int:
    n = ctypes.c_size_t()
    _echeck(_lib.rbc_ensemble_footprint(ctypes.byref(p), ctypes.byref(n)), None)
    return n.value


def rbc_ensemble_add(e, p: rbc_params, U0, k_max: int, tol: float) -> int:
    rid = ctypes.c_int32()
    _echeck(_lib.rbc_ensemble_add(e, ctypes.byref(p), _ptr(U0), k_max, tol, ctypes.byref(rid)), e)
    return rid.value


def rbc_ensemble_step(e) -> int:
    n = ctypes.c_int32()
    _echeck(_lib.rbc_ensemble_step(e, ctypes.byref(n)), e)
    return n.value


ENSEMBLE_ACTIVE, ENSEMBLE_DONE, ENSEMBLE_FAILED, ENSEMBLE_RELEASED = 0, 1, 2, 3


def rbc_ensemble_run_info(e, run_id: int, hist_len: int = 0):
    """(state, k_done, stop, defects[:min(k_done, hist_len)])."""
    st, k, stop = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    hist = np.zeros(max(hist_len, 1))
    _echeck(_lib.rbc_ensemble_run_info(e, run_id, ctypes.byref(st), ctypes.byref(k), ctypes.byref(stop),
                                       hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), hist_len), e)
    return st.value, k.value, stop.value, hist[: min(k.value, hist_len)].copy()


def rbc_ensemble_result(e, run_id: int, U) -> None:
    _echeck(_lib.rbc_ensemble_result(e, run_id, _ptr(U)), e)


def rbc_ensemble_release(e, run_id: int) -> None:
    _echeck(_lib.rbc_ensemble_release(e, run_id), e)


def rbc_ensemble_run_bytes(e, run_id: int) -> int:
    n = ctypes.c_size_t()
    _echeck(_lib.rbc_ensemble_run_bytes(e, run_id, ctypes.byref(n)), e)
    return n.value
