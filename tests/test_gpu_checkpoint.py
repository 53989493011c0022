"""Checkpoint and resume of the Parareal iteration at an iteration boundary
(section 3.1, Eq. 19): iteration k + 1 reads only U^k, G(U_n^k) and the
decisions of iteration k, so a run stopped after iteration j, saved with
rbc_get_state (plus the caller's U^j), loaded into a fresh handle with
rbc_set_state and continued must give the iterates, defects, averages and
precision switch of the uninterrupted run bit for bit, in either schedule
and across schedules."""
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


def params(S, mixed, nu_stride, **kw):
    r = R()
    p = r.rbc_default_params()
    p.Ra, p.Pr, p.Lx, p.Lz = 5e4, 1.0, 2.0, 1.0
    p.Nx, p.Nz, p.Nx_c, p.Nz_c = 32, 16, 16, 8
    p.n_slices = S
    p.dt_f, p.dt_c = 0.01, 0.04
    p.t0, p.t_end = 0.0, 0.5 * S
    p.scheme_f = p.scheme_c = r.RBC_ARS443
    p.precision = r.RBC_MIXED if mixed else r.RBC_FP64
    p.nu_stride = nu_stride
    p.nu_t_start = 0.2
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def initial(p):
    g = O.Grid(p.Ra, p.Pr, p.Lx, p.Lz, p.Nx, p.Nz, p.dt_f)
    return O.initial_state(g, I.gaussian_noise(21, g.Nx, g.Nz), 0.3).pack()


def iterate(p, pipelined, U, k_max, tol, ckpt=None):
    """One parareal_iterate on a fresh handle, optionally resumed from a
    checkpoint; returns the outputs and the handle's checkpoint after it."""
    p.pipelined = pipelined
    h = R().rbc_create(p, torch.cuda.current_stream(dev()).cuda_stream)
    try:
        if ckpt is not None:
            R().rbc_set_state(h, ckpt)
        st, kd, defects, nu = R().parareal_iterate(h, U, k_max, tol, want_nu=p.nu_stride > 0)
        kp = R().rbc_fine_fp64_from(h)
        return kd, defects, nu, kp, R().rbc_get_state(h)
    finally:
        R().rbc_destroy(h)


CASES = {
    # mixed precision with the FP64 switch: checkpoints before, at and after
    # the switch decision
    "mixed_promote": dict(S=6, mixed=True, nu_stride=4, k_max=6, tol=1e-13, stops=(1, 2, 3, 4)),
    # FP64 to finite termination with diagnostic samples
    "fp64_to_S": dict(S=5, mixed=False, nu_stride=5, k_max=5, tol=0.0, stops=(0, 2, 4)),
}


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("sched", [(1, 1), (0, 0), (1, 0), (0, 1)])
def test_resume_from_checkpoint_is_bitwise(name, sched):
    c = CASES[name]
    save_sched, load_sched = sched
    p = params(c["S"], c["mixed"], c["nu_stride"])
    U0 = initial(p)
    n = U0.size
    S = c["S"]

    def fresh():
        U = torch.zeros((S + 1) * n, dtype=torch.float64, device=dev())
        U[:n] = torch.tensor(U0, dtype=torch.float64, device=dev())
        return U

    case(f"checkpoint {name} uninterrupted, schedule {load_sched}")
    Uref = fresh()
    kd, dref, nuref, kpref, _ = iterate(p, load_sched, Uref, c["k_max"], c["tol"])
    ref = Uref.cpu().numpy()
    for j in c["stops"]:
        if j >= kd:
            continue
        case(f"checkpoint {name}: stop at {j} (schedule {save_sched}), resume (schedule {load_sched})")
        U = fresh()
        kj, _, _, _, ck = iterate(p, save_sched, U, j, c["tol"])
        assert kj == j
        saved = U.clone()
        del U
        k2, d2, nu2, kp2, _ = iterate(p, load_sched, saved, c["k_max"], c["tol"], ckpt=ck)
        assert k2 == kd, (j, k2, kd)
        assert np.array_equal(saved.cpu().numpy(), ref), j
        assert np.array_equal(d2[j:], dref[j:]), (j, d2, dref)
        if nuref is not None:
            assert np.array_equal(nu2[j:], nuref[j:], equal_nan=True), j
        assert kp2 == kpref, (j, kp2, kpref)
    if name == "mixed_promote":
        assert kpref > 0, "the case must exercise the FP64 switch"


def test_checkpoint_rejects_another_configuration():
    p = params(4, False, 0)
    q = params(5, False, 0)
    U0 = initial(p)
    n = U0.size
    U = torch.zeros(5 * n, dtype=torch.float64, device=dev())
    U[:n] = torch.tensor(U0, dtype=torch.float64, device=dev())
    case("checkpoint of another configuration")
    _, _, _, _, ck = iterate(p, 1, U, 1, 0.0)
    h = R().rbc_create(q, torch.cuda.current_stream(dev()).cuda_stream)
    try:
        with pytest.raises(R().RbcError) as ei:
            R().rbc_set_state(h, ck)
        assert ei.value.status == R().RBC_ERR_ARG
        with pytest.raises(R().RbcError) as ei:
            R().rbc_set_state(h, b"not a checkpoint at all, but long enough to read a header from it....." * 4)
        assert ei.value.status == R().RBC_ERR_ARG
    finally:
        R().rbc_destroy(h)
