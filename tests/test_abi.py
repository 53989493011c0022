"""Host-side checks of the C ABI (no GPU): the library loads, exports every
function include/rbc.h declares, the Python struct matches the C layout,
and argument validation rejects bad parameters before touching a device."""
import ctypes
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rbc.h")
LIB = os.path.join(ROOT, "paper_2001_01609_amd", "librbc.so")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2001_01609_amd import build
        build.build(verbose=False)
    return ctypes.CDLL(LIB)


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:rbc_status|const char\*)\s+(\w+)\s*\(", src, flags=re.M)
    assert len(names) >= 14
    return names


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_names_match_header():
    from paper_2001_01609_amd import rbc as R
    for name in declared_functions():
        assert callable(getattr(R, name)), name


def test_params_struct_layout_matches_c():
    """Compile a tiny C program against rbc.h and compare sizeof/offsetof."""
    from paper_2001_01609_amd import rbc as R
    fields = [f for f, _ in R.rbc_params._fields_]
    prog = "#include <stdio.h>\n#include <stddef.h>\n#include \"rbc.h\"\nint main(void){\n"
    prog += 'printf("%zu\\n", sizeof(rbc_params));\n'
    for f in fields:
        prog += f'printf("%zu\\n", offsetof(rbc_params, {f}));\n'
    prog += "return 0;}\n"
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        exe = os.path.join(d, "t")
        open(c, "w").write(prog)
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        out = [int(v) for v in subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()]
    assert out[0] == ctypes.sizeof(R.rbc_params)
    for f, off in zip(fields, out[1:]):
        assert getattr(R.rbc_params, f).offset == off, f


def test_argument_validation_without_device():
    from paper_2001_01609_amd import rbc as R
    p = R.rbc_default_params()
    assert R.rbc_query_footprint(p) > 0
    bad = [("Nx", 48), ("Nz", 7), ("Nz", 4), ("Nz", 24), ("Nz", 512), ("Nx", 4096), ("Nx_c", 128), ("n_slices", 0), ("scheme_f", 3),
           ("precision", 7), ("dt_f", 0.0), ("t_end", -1.0)]
    for field, val in bad:
        q = R.rbc_default_params()
        setattr(q, field, val)
        with pytest.raises(R.RbcError) as ei:
            R.rbc_query_footprint(q)
        assert ei.value.status == R.RBC_ERR_ARG
        with pytest.raises(R.RbcError):
            R.rbc_create(q)
        assert R.rbc_last_error(None)


def test_footprint_scales_with_slices():
    from paper_2001_01609_amd import rbc as R
    import rbc_inputs as I
    a = R.rbc_query_footprint(R.params_from_workload(I.C2))
    b = R.rbc_query_footprint(R.params_from_workload(I.C2, n_slices=64, t_end=100.0))
    assert b > 1.8 * a
    # the large workload stays far below one GPU's 288 GB
    c = R.rbc_query_footprint(R.params_from_workload(I.C3))
    assert c < 16e9


def test_tuning_table_parses_and_steers_plans(tmp_path):
    """rbc_tuning_load: a valid table changes the plan the footprint query
    builds (here: the split path for the 256x64 mixed fine grid), a bad line
    is rejected with its line number, NULL clears."""
    import rbc_inputs as I
    from paper_2001_01609_amd import rbc as R
    p = R.params_from_workload(I.C2)
    R.rbc_tuning_load(None)
    assert R.rbc_tuning_entries() == 0
    base = R.rbc_query_footprint(p)
    good = tmp_path / "t.txt"
    good.write_text("# comment\nfine mixed 256 64 32 2 1 0   # split, two-mode tiles\ncoarse fp64 128 32 1 4 0 2\n")
    R.rbc_tuning_load(str(good))
    assert R.rbc_tuning_entries() == 2
    split = R.rbc_query_footprint(p)
    assert split > base          # the split path's by-parity maps and FP32 stage copies
    bad = tmp_path / "b.txt"
    bad.write_text("fine mixed 256 64 32 3 0 0\n")
    with pytest.raises(R.RbcError) as ei:
        R.rbc_tuning_load(str(bad))
    assert ":1:" in str(ei.value)
    assert R.rbc_tuning_entries() == 2     # a failed load keeps the table
    # a "0 0 0" entry keeps the rules for its batch, also beside an entry of
    # another batch that would otherwise be the nearest
    keep = tmp_path / "k.txt"
    keep.write_text("fine mixed 256 64 4 2 1 0\nfine mixed 256 64 32 0 0 0   # measured: rule stays\n")
    R.rbc_tuning_load(str(keep))
    assert R.rbc_tuning_entries() == 2
    assert R.rbc_query_footprint(p) == base
    bad.write_text("fine mixed 256 64 32 0 1 0\n")
    with pytest.raises(R.RbcError):
        R.rbc_tuning_load(str(bad))
    R.rbc_tuning_load(None)
    assert R.rbc_query_footprint(p) == base
    if os.path.exists(R.TUNING_TABLE):
        R.rbc_tuning_load(R.TUNING_TABLE)


def test_shipped_tuning_table_covers_every_tuned_plan():
    """The gfx950 table holds one entry (a measured shape or "0 0 0", keep
    the rules) for every plan the autotuner measures, so that no plan takes,
    by nearest-batch lookup, a shape measured for another batch."""
    from paper_2001_01609_amd import rbc as R
    from paper_2001_01609_amd import tune
    keys = set()
    for line in open(R.TUNING_TABLE):
        line = line.split("#", 1)[0].split()
        if line:
            keys.add((line[0], line[1], int(line[2]), int(line[3]), int(line[4])))
    want = {(t[0], t[1], t[2], t[3], t[4]) for t in tune.TARGETS}
    assert want <= keys
    R.rbc_tuning_load(R.TUNING_TABLE)
    assert R.rbc_tuning_entries() == len(keys)
