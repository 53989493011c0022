"""The autotuner's choice logic (paper_2001_01609_amd/tune.py choose) with
a timing function injected: candidate sets, the two-step search, the 3%
margin and the keep-the-rule entries, and that every line it writes is one
the library's table parser accepts.  No GPU."""
from paper_2001_01609_amd import tune as T

FINE = ("fine", "mixed", 1024, 256, 64, 64, 1e8, 2e-5, (256, 64), "test fine")
COARSE = ("coarse", "mixed", 128, 32, 1, 1, 1e6, 2e-3, None, "test coarse")


def timer(table, default=10.0):
    """timed(env) from a dict keyed by (MT, split, xrows); the rule is ()."""
    seen = []

    def timed(env):
        key = () if not env else (env["RBC_MODE_TILE"], env["RBC_SPLIT"], env.get("RBC_XPASS_ROWS", 0))
        seen.append(key)
        return table.get(key, default)
    return timed, seen


def test_a_clear_winner_enters_the_table():
    timed, seen = timer({(): 10.0, (4, 1, 0): 8.0, (4, 1, 2): 7.5})
    line = T.choose(FINE, timed, log=lambda m: None)
    assert line.split("#")[0].split() == ["fine", "mixed", "1024", "256", "64", "4", "1", "2"]
    # split candidates are timed for the mixed fine grid, then x-pass rows with the best
    assert (2, 1, 0) in seen and (4, 1, 0) in seen
    assert [k for k in seen if len(k) == 3 and k[2]] == [(4, 1, 1), (4, 1, 2), (4, 1, 4)]


def test_within_the_margin_the_rule_stays():
    timed, _ = timer({(): 10.0, (4, 0, 0): 9.8})
    line = T.choose(FINE, timed, log=lambda m: None)
    assert line.split("#")[0].split() == ["fine", "mixed", "1024", "256", "64", "0", "0", "0"]
    assert "the rule stays" in line


def test_coarse_plans_never_try_the_split_path():
    timed, seen = timer({(): 10.0})
    T.choose(COARSE, timed, log=lambda m: None)
    assert all(k == () or k[1] == 0 for k in seen)


def test_a_failing_candidate_is_skipped():
    class Fail(Exception):
        pass

    def timed(env):
        if env.get("RBC_MODE_TILE") == 8:
            raise Fail("no plan")
        return 5.0 if env.get("RBC_MODE_TILE") == 2 and env.get("RBC_SPLIT") == 0 else 10.0
    logs = []
    line = T.choose(FINE, timed, log=logs.append, errors=(Fail,))
    assert line.split()[5] == "2"
    assert any("failed" in m for m in logs)


def test_written_lines_parse_in_the_library(tmp_path):
    from paper_2001_01609_amd import rbc as R
    timed1, _ = timer({(): 10.0, (8, 0, 4): 5.0})
    timed2, _ = timer({(): 10.0})
    lines = list(T.HEADER) + [T.choose(FINE, timed1, log=lambda m: None), T.choose(COARSE, timed2, log=lambda m: None)]
    path = tmp_path / "t.txt"
    path.write_text("\n".join(lines) + "\n")
    try:
        R.rbc_tuning_load(str(path))
        assert R.rbc_tuning_entries() == 2
    finally:
        R.rbc_tuning_load(R.TUNING_TABLE)
