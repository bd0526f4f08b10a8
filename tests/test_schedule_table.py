"""The schedule table written by the autotuner is read by libqe at first use
(QE_TUNE_TABLE), in its full form ("n lclass lds waves cpb") and the short
one ("n lds"); QE_SCHEDULE overrides single widths; impossible schedules are
ignored.  Runs in subprocesses because the table is loaded once per process;
no GPU needed."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROBE = ("import sys; sys.path.insert(0, %r); from paper_1809_11134_amd import qe; "
         "print(' '.join(str(qe.get_schedule(n)) for n in range(1, 7))); "
         "print(' '.join(','.join(str(x) for x in qe.get_schedule_ex(n, c)) for n in range(1, 7) for c in (0, 1))); "
         "print(' '.join(','.join(str(x) for x in qe.get_schedule_lib(n, c, k)) "
         "for n in range(1, 7) for c in (0, 1) for k in (0, 1, 2))); "
         "print(' '.join(str(qe.get_mfma_min_block(n, c)) for n in range(1, 7) for c in (0, 1)))"
         % ROOT)


def schedule_with(env_extra):
    env = dict(os.environ)
    env.pop("QE_SCHEDULE", None)
    env.pop("QE_TUNE_TABLE", None)
    env.update(env_extra)
    out = subprocess.run([sys.executable, "-c", PROBE], env=env, capture_output=True, text=True,
                         check=True)
    a, b, c3, c4 = out.stdout.split("\n")[:4]
    mm = [int(x) for x in c4.split()]
    schedule_with.mfma = {(n, c): mm[2 * (n - 1) + c] for n in range(1, 7) for c in (0, 1)}
    full = [tuple(int(x) for x in t.split(",")) for t in b.split()]
    by_lib = [tuple(int(x) for x in t.split(",")) for t in c3.split()]
    schedule_with.by_lib = {(n, c, k): by_lib[6 * (n - 1) + 3 * c + k]
                            for n in range(1, 7) for c in (0, 1) for k in (0, 1, 2)}
    return [int(x) for x in a.split()], {(n, c): full[2 * (n - 1) + c] for n in range(1, 7) for c in (0, 1)}


def test_table_and_override(tmp_path):
    table = tmp_path / "tune.txt"
    table.write_text("# test table\n4 0   # register\n5 1\n6 0 # comment\n")
    assert schedule_with({"QE_TUNE_TABLE": str(table)})[0][3:] == [0, 1, 0]
    assert schedule_with({"QE_TUNE_TABLE": str(table), "QE_SCHEDULE": "6:1,4:1"})[0][3:] == [1, 1, 1]


def test_full_table_lines(tmp_path):
    table = tmp_path / "tune.txt"
    table.write_text("5 0 1 2 1   # short circuits: two wavefronts\n"
                     "5 1 1 1 1\n"
                     "4 1 1 1 1\n"
                     "6 0 1 2 1   # impossible (n = 6 takes four wavefronts): ignored\n"
                     "5 1 1 3 4   # impossible: ignored\n")
    short, full = schedule_with({"QE_TUNE_TABLE": str(table)})
    assert full[(5, 0)] == (1, 2, 1) and full[(5, 1)] == (1, 1, 1)
    assert full[(4, 1)] == (1, 1, 1) and full[(4, 0)] == (1, 1, 4)
    assert full[(6, 0)] == (1, 4, 1)
    _, full = schedule_with({"QE_TUNE_TABLE": str(table), "QE_SCHEDULE": "5:1:2,4:1:1:4"})
    assert full[(5, 0)] == (1, 2, 1) and full[(5, 1)] == (1, 2, 1)
    assert full[(4, 0)] == (1, 1, 4) and full[(4, 1)] == (1, 1, 4)


def test_missing_table_keeps_defaults(tmp_path):
    got, full = schedule_with({"QE_TUNE_TABLE": str(tmp_path / "absent.txt")})
    assert got[:3] == [0, 0, 0] and all(x in (0, 1) for x in got)
    assert full[(5, 1)][1] in (1, 2) and full[(6, 1)][1] == 4


def test_set_schedule_ex_validates():
    import pytest
    from paper_1809_11134_amd import qe
    with pytest.raises(qe.QeError):
        qe.set_schedule_ex(6, 1, 1, 2, 1)
    with pytest.raises(qe.QeError):
        qe.set_schedule_ex(5, 2, 1, 1, 4)
    with pytest.raises(qe.QeError):
        qe.set_schedule_ex(4, 0, 1, 1, 3)


def test_library_class_lines(tmp_path):
    """"n lclass lib lds waves cpb" sets one library class; the five-field
    form sets all three; later lines win."""
    table = tmp_path / "tune.txt"
    table.write_text("5 1 1 1 1\n"
                     "5 1 1 1 2 1   # sampled, long: two wavefronts\n"
                     "5 0 2 1 2 1   # Ising, short\n"
                     "4 0 1 1 4\n"
                     "4 0 2 1 1 1\n"
                     "5 1 3 1 1 1   # no such class: ignored\n")
    schedule_with({"QE_TUNE_TABLE": str(table)})
    got = schedule_with.by_lib
    assert got[(5, 1, 1)] == (1, 2, 1) and got[(5, 1, 0)] == (1, 1, 1) and got[(5, 1, 2)] == (1, 1, 1)
    assert got[(5, 0, 2)] == (1, 2, 1) and got[(5, 0, 0)][1] == 1
    assert got[(4, 0, 0)] == (1, 1, 4) and got[(4, 0, 1)] == (1, 1, 4) and got[(4, 0, 2)] == (1, 1, 1)
    # QE_SCHEDULE overrides every class of a width
    schedule_with({"QE_TUNE_TABLE": str(table), "QE_SCHEDULE": "5:1:1:4"})
    got = schedule_with.by_lib
    assert all(got[(5, c, k)] == (1, 1, 4) for c in (0, 1) for k in (0, 1, 2))


def test_set_schedule_lib_validates():
    import pytest
    from paper_1809_11134_amd import qe
    saved = qe.get_schedule_lib(5, 1, qe.SCHED_ISING)
    try:
        qe.set_schedule_lib(5, 1, qe.SCHED_ISING, 1, 2, 1)
        assert qe.get_schedule_lib(5, 1, qe.SCHED_ISING) == (1, 2, 1)
        with pytest.raises(qe.QeError):
            qe.set_schedule_lib(5, 1, 3, 1, 1, 1)
        with pytest.raises(qe.QeError):
            qe.set_schedule_lib(6, 0, qe.SCHED_SAMPLED, 1, 1, 1)
        with pytest.raises(qe.QeError):
            qe.get_schedule_lib(5, 2, 0)
    finally:
        qe.set_schedule_lib(5, 1, qe.SCHED_ISING, *saved)


def test_mfma_min_block_lines(tmp_path):
    """"mfma n lclass min_block" lines set the MFMA block threshold; values
    outside 1..65 are ignored; the default fuses every group."""
    table = tmp_path / "tune.txt"
    table.write_text("mfma 6 1 4   # long circuits at n = 6\n"
                     "mfma 5 0 3\n"
                     "mfma 5 1 0   # out of range: ignored\n"
                     "mfma 5 1 66  # out of range: ignored\n"
                     "5 1 1 1 1\n")
    schedule_with({"QE_TUNE_TABLE": str(table)})
    got = schedule_with.mfma
    assert got[(6, 1)] == 4 and got[(5, 0)] == 3 and got[(5, 1)] == 1 and got[(6, 0)] == 1
    schedule_with({"QE_TUNE_TABLE": str(tmp_path / "absent.txt")})
    assert all(v == 1 for v in schedule_with.mfma.values())


def test_set_mfma_min_block_validates():
    import pytest
    from paper_1809_11134_amd import qe
    saved = qe.get_mfma_min_block(6, 0)
    try:
        qe.set_mfma_min_block(6, 0, 65)
        assert qe.get_mfma_min_block(6, 0) == 65
        for bad in ((6, 0, 0), (6, 0, 66), (7, 0, 3), (6, 2, 3)):
            with pytest.raises(qe.QeError):
                qe.set_mfma_min_block(*bad)
    finally:
        qe.set_mfma_min_block(6, 0, saved)
