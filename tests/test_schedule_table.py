"""The per-width schedule table written by the autotuner is read by libqe at
first use (QE_TUNE_TABLE), and QE_SCHEDULE overrides single widths.  Runs in
subprocesses because the table is loaded once per process; no GPU needed."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROBE = ("import sys; sys.path.insert(0, %r); from paper_1809_11134_amd import qe; "
         "print(' '.join(str(qe.get_schedule(n)) for n in range(1, 7)))" % ROOT)


def schedule_with(env_extra):
    env = dict(os.environ)
    env.pop("QE_SCHEDULE", None)
    env.pop("QE_TUNE_TABLE", None)
    env.update(env_extra)
    out = subprocess.run([sys.executable, "-c", PROBE], env=env, capture_output=True, text=True,
                         check=True)
    return [int(x) for x in out.stdout.split()]


def test_table_and_override(tmp_path):
    table = tmp_path / "tune.txt"
    table.write_text("# test table\n4 0   # register\n5 1\n6 0 # comment\n")
    assert schedule_with({"QE_TUNE_TABLE": str(table)})[3:] == [0, 1, 0]
    assert schedule_with({"QE_TUNE_TABLE": str(table), "QE_SCHEDULE": "6:1,4:1"})[3:] == [1, 1, 1]


def test_missing_table_keeps_defaults(tmp_path):
    got = schedule_with({"QE_TUNE_TABLE": str(tmp_path / "absent.txt")})
    assert got[:3] == [0, 0, 0] and all(x in (0, 1) for x in got)
