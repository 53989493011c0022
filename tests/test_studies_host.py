"""Host arithmetic of the Parareal studies (paper_2001_01609_amd/studies.py):
the per-iteration errors, the first iteration within a threshold, the
speed-up and the time averages of section 2.2, on arrays whose answers are
known in closed form.  No GPU."""
import math

import numpy as np

from paper_2001_01609_amd import studies as St


def _iterates(K=4, S=5, n=7, seed=3):
    """ref[j] = (j + 1) v with |v| = 1; H[k][j] = ref[j] + 2^-k w with |w| = 1,
    w orthogonal to v; slice 0 of every iterate set far off (not scored)."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(n)
    v /= np.linalg.norm(v)
    w = rng.standard_normal(n)
    w -= (w @ v) * v
    w /= np.linalg.norm(w)
    ref = np.stack([(j + 1) * v for j in range(S + 1)])
    H = np.stack([ref + 2.0 ** -k * w for k in range(K + 1)])
    H[:, 0] += 1e3
    return H, ref


def test_rel_l2_errors_final_time_and_max_over_slice_boundaries():
    K, S = 4, 5
    H, ref = _iterates(K, S)
    fin, mx = St.rel_l2_errors(H, ref)
    for k in range(K + 1):
        # |2^-k w| / |(j + 1) v| at j = S (final), max over j = 1..S at j = 1
        assert math.isclose(fin[k], 2.0 ** -k / (S + 1), rel_tol=1e-12)
        assert math.isclose(mx[k], 2.0 ** -k / 2, rel_tol=1e-12)


def test_rel_l2_errors_with_a_row_norm_function():
    # the studies pass torch.linalg.norm on device tensors; any norm of a row works
    H, ref = _iterates()
    fin1, _ = St.rel_l2_errors(H, ref, norm=lambda x: float(np.abs(x).max()))
    fin2, _ = St.rel_l2_errors(H, ref)
    assert fin1 != fin2 and all(f > 0 for f in fin1)


def test_first_within_skips_the_prediction():
    assert St.first_within([0.5, 0.2, 0.005, 0.001], 1e-2) == 2
    assert St.first_within([0.0, 0.5, 0.3], 1e-2) is None       # k = 0 never counts
    assert St.first_within([1.0, 1e-2], 1e-2) == 1              # inclusive


def test_speedup_at():
    assert St.speedup_at(10.0, [0.0, 2.0, 5.0], 2) == 2.0
    assert St.speedup_at(10.0, [0.0, 2.0, 5.0], None) is None
    assert St.speedup_at(10.0, [0.0, 0.0], 1) is None


def test_rel_errors():
    assert St.rel_errors([1.0, 1.1, 0.8], 1.0) == [0.0, 0.10000000000000009, 0.19999999999999996]
    assert St.rel_errors([-2.0], -4.0) == [0.5]


def test_time_averages_follow_section_2_2():
    # records (Nu_V, Nu_b, Nu_t, KE, eps_U, P)
    rec = np.array([[2.0, 2.2, 1.8, 0.5, 0.010, 0.012],
                    [4.0, 3.8, 4.2, 2.0, 0.030, 0.028]])
    visc = 1e-3
    out = St.time_averages(rec, visc)
    assert np.allclose(out[:3], [3.0, 3.0, 3.0])
    assert out[3] == 0.0                                   # Nu_int (Eq. 13)
    assert np.isclose(out[4], 1.25)                        # KE
    assert np.isclose(out[5], (1.0 + 2.0) / 2 / visc)      # Re = <sqrt(2 KE)> / nu
    assert np.isclose(out[8], abs(0.020 - 0.020) / 0.020)  # |P - eps_U| / P (Eq. 15)
    # unequal means: Nu_int is the largest pairwise difference over Nu_V
    rec2 = np.array([[2.0, 2.3, 1.9, 0.5, 0.01, 0.02]])
    out2 = St.time_averages(rec2, visc)
    assert np.isclose(out2[3], 0.4 / 2.0)
    assert np.isclose(out2[8], 0.5)


def test_window_table_renders_one_row_per_iteration():
    fields = ("Nu_V", "Nu_b", "Nu_t", "Nu_int", "KE", "Re", "eps_U", "P", "balance")
    avg = [{f: 1.0 + 0.1 * k for f in fields} for k in range(3)]
    c = {"averages_per_iteration": avg, "defects": [1e-2, 1e-4], "speedup_per_iteration": [3.0, 1.5],
         "iteration_done_at_s": [0.5, 1.0, 2.0], "nu_v_err": [0.2, 0.1, 0.0], "nu_b_err": [0.2, 0.1, 0.0],
         "nu_t_err": [0.2, 0.1, 0.0], "l2_final": [1e-1, 1e-3, 1e-5], "l2_max": [1e-1, 1e-3, 1e-5],
         "serial_fp64_s": 3.0, "averages_serial_fp64": {f: 1.2 for f in fields}}
    t = St.window_table(c).splitlines()
    assert len(t) == 2 + 3 + 1
    assert t[3].startswith("| 1 | 1.00 | 1.00e-02 |") and t[3].endswith("| 3.00 |")
    assert t[-1].startswith("| serial FP64 | 3.00 |")


def test_study_definitions_are_complete():
    import inspect
    for name, cases in St.STUDIES.items():
        for cfg in cases:
            cfg = dict(cfg)
            fn = St.window_case if cfg.pop("case", None) == "window" else St.run_case
            params = inspect.signature(fn).parameters
            assert set(cfg) <= set(params), (name, cfg)
            missing = [p for p, v in params.items() if v.default is inspect.Parameter.empty and p not in cfg]
            assert not missing, (name, missing)
