"""Host-side logic of bench.py (no GPU): the byte model behind the roofline
figure, the one-GPU guard and the traffic summary lookup (the time averages
of section 2.2 are tested with the studies' arithmetic)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_byte_model_of_the_three_pass_step():
    # stage data per grid point and step: s state reads, the right-hand-side
    # history 2 + 4 (i - 1) of stage i, 6 writes per stage
    assert bench.stage_data_values(4) == 8 + (2 + 6 + 10 + 14) + 24 == 64
    assert bench.stage_data_values(2) == 4 + (2 + 6) + 12 == 24
    # ARS443: 896 B mixed, 1280 B FP64; ARS222: 384 B and 576 B
    assert bench.bytes_per_dof_step(4, 4) == 96 * 4 + 64 * 8 == 896
    assert bench.bytes_per_dof_step(4, 8) == 1280
    assert bench.bytes_per_dof_step(2, 4) == 384 and bench.bytes_per_dof_step(2, 8) == 576
    # per stage: the per-mode stage's 176 B and the x-pass's 48 B make up the step
    st, xp = bench.stage_bytes_per_dof_launch(4, 4), bench.xpass_bytes_per_dof_launch(4)
    assert st == 176 and xp == 48 and 4 * (st + xp) == 896


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_summary_is_ignored_for_another_workload():
    assert bench.measured_traffic("no_such_workload") is None
