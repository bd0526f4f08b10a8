"""The named targets of the convergence runs (textbook reversible gates,
wire 0 = most significant bit, target bit on wire 0) and a short run."""
import numpy as np
import pytest
import torch

from paper_1809_11134_amd import experiments, qe


def truth(n, fn):
    return [fn(i) for i in range(1 << n)]


def test_targets_are_the_textbook_gates():
    def tof(i):
        c, a, b = (i >> 2) & 1, (i >> 1) & 1, i & 1
        return ((c ^ (a & b)) << 2) | (a << 1) | b

    def per(i):
        c, a, b = (i >> 2) & 1, (i >> 1) & 1, i & 1
        return ((c ^ (a & b)) << 2) | (a << 1) | (b ^ a)
    expect = {"cnot": (2, [0, 3, 2, 1]), "toffoli": (3, truth(3, tof)), "peres": (3, truth(3, per)),
              "cccnot": (4, [i ^ 8 if (i & 7) == 7 else i for i in range(16)])}
    for name, (n, table) in expect.items():
        m, U = experiments.target_unitary(name)
        assert m == n
        assert np.array_equal(U, np.eye(1 << n)[table].T.astype(complex)), name


@pytest.mark.gpu
def test_short_run_solves_cnot():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    qe.load()
    r = experiments.run("cnot", qe.ALG_QEQEA, L=8, P=64, generations=400, chunk=20)
    assert r["best_f_fp64"] == pytest.approx(1.0, abs=1e-12)
    assert r["first_generation_reaching"]["1.0"] <= 400
    assert r["curve"] and all(0 <= f <= 1 for _, f in r["curve"])


@pytest.mark.gpu
def test_short_ising_run_reports_angled_best_circuit():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    qe.load()
    r = experiments.run("cnot", qe.ALG_QEQEA, L=3, P=16, generations=200, chunk=50,
                        library=qe.LIB_ISING)
    assert r["library"] == "ising" and len(r["best_circuit"]) == 3
    for kind, a, b, theta in r["best_circuit"]:
        assert kind in (7, 8, 9, 10) and 0 <= theta < 2 * np.pi + 1e-6
    assert abs(r["best_f_fp32"] - r["best_f_fp64"]) <= 1e-5
    fs = [f for _, f in r["curve"]]
    assert fs == sorted(fs)                          # the best so far never decreases

