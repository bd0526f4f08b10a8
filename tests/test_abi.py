"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function include/qe.h declares, validates arguments before touching the
device, and shares the gate-library enumeration with the oracle."""
import ctypes

import pytest

from paper_1809_11134_amd import qe


@pytest.fixture(scope="module")
def lib():
    return qe.load()


def test_exports_every_declared_symbol(lib):
    names = qe.header_functions()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_version_and_last_error(lib):
    assert b"gfx950" in lib.qe_version()
    assert isinstance(lib.qe_last_error(), bytes)


def test_lib_tables_match_oracle(oracle):
    for library in (0, 1):
        for n in range(1, 7):
            assert qe.load().qe_lib_size(library, n) == oracle.lib_size(library, n)
            assert qe.lib_table(library, n) == [int(x) for x in oracle.lib_table(library, n)]
    assert qe.load().qe_lib_size(2, 3) == -1
    assert qe.load().qe_lib_size(0, 7) == -1


def _problem(**kw):
    base = dict(n_qubits=3, library=0, algorithm=0, size_of_individual=10,
                size_of_population=8, n_instances=1, prob_mutation=0.1,
                mutation_range=0.78, ga_crossover_prob=0.9, ga_gene_mutation_prob=0.1, seed=1,
                fitness_mode=0)
    base.update(kw)
    return qe.Problem(*[base[f] for f, _ in qe.Problem._fields_])


@pytest.mark.parametrize("kw,status", [
    (dict(n_qubits=0), qe.QE_ERR_INVALID),
    (dict(n_qubits=7), qe.QE_ERR_INVALID),
    (dict(n_qubits=1), qe.QE_ERR_INVALID),                  # QEQEA needs a wire pair
    (dict(library=1), qe.QE_ERR_UNSUPPORTED),               # QEQEA decodes to library 0 or 2
    (dict(library=2, algorithm=1), qe.QE_ERR_UNSUPPORTED),  # the GA genome holds no angles
    (dict(library=5), qe.QE_ERR_INVALID),
    (dict(algorithm=3), qe.QE_ERR_INVALID),
    (dict(size_of_individual=0), qe.QE_ERR_INVALID),
    (dict(size_of_individual=2000), qe.QE_ERR_INVALID),
    (dict(size_of_population=0), qe.QE_ERR_INVALID),
    (dict(algorithm=1, size_of_population=5000), qe.QE_ERR_INVALID),
    (dict(n_instances=0), qe.QE_ERR_INVALID),
    (dict(prob_mutation=1.5), qe.QE_ERR_INVALID),
    (dict(prob_mutation=float("nan")), qe.QE_ERR_INVALID),
    (dict(mutation_range=7.0), qe.QE_ERR_INVALID),
    (dict(ga_crossover_prob=-0.1), qe.QE_ERR_INVALID),
    (dict(fitness_mode=5), qe.QE_ERR_INVALID),
    (dict(fitness_mode=-1), qe.QE_ERR_INVALID),
])
def test_create_rejects_bad_problems(lib, kw, status):
    h = ctypes.c_void_p(0)
    p = _problem(**kw)
    assert lib.qe_create(ctypes.byref(p), ctypes.byref(h)) == status
    assert not h.value
    assert lib.qe_last_error()


def test_null_arguments_rejected(lib):
    assert lib.qe_create(None, None) == qe.QE_ERR_INVALID
    assert lib.qe_eval_fitness(None, None, 0, None, None, None, None) == qe.QE_ERR_INVALID
    assert lib.qe_destroy(None) == qe.QE_ERR_INVALID
    assert lib.qe_device_errors(None) == qe.QE_ERR_INVALID
    assert lib.qe_set_schedule(0, 1) == qe.QE_ERR_INVALID
    b = qe.Batch()
    b.num_circuits = -1
    assert lib.qe_eval_fitness(None, ctypes.byref(b), 0, None, None, None, None) == qe.QE_ERR_INVALID
    b.num_circuits = 4
    b.uniform_n = 9
    assert lib.qe_eval_fitness(None, ctypes.byref(b), 0, None, None, None, None) == qe.QE_ERR_INVALID
    b.uniform_n = 3
    b.uniform_L = 5
    b.num_gates = 10                      # 4 circuits x 5 gates do not fit
    assert lib.qe_eval_fitness(None, ctypes.byref(b), 0, None, None, None, None) == qe.QE_ERR_INVALID


def test_schedule_roundtrip(lib):
    old = qe.get_schedule(5)
    qe.set_schedule(5, 1 - old)
    assert qe.get_schedule(5) == 1 - old
    qe.set_schedule(5, old)
    assert qe.get_schedule(5) == old


def test_probes_validate_arguments(lib):
    """The measurement probes refuse bad modes, NULL buffers and sizes out of
    range before launching anything."""
    dummy = ctypes.c_void_p(16)           # never dereferenced: rejected first
    assert lib.qe_probe_lds(3, 1, 1, dummy, None, None) == qe.QE_ERR_INVALID
    assert lib.qe_probe_lds(0, 0, 1, dummy, None, None) == qe.QE_ERR_INVALID
    assert lib.qe_probe_lds(0, 1, 1, None, None, None) == qe.QE_ERR_INVALID
    assert lib.qe_probe_records(2, dummy, 10, 10, 0, dummy, None) == qe.QE_ERR_INVALID
    assert lib.qe_probe_records(0, None, 10, 10, 0, dummy, None) == qe.QE_ERR_INVALID
    assert lib.qe_probe_records(0, dummy, 10, 10, 0, None, None) == qe.QE_ERR_INVALID
    assert lib.qe_probe_records(0, dummy, 0, 10, 0, dummy, None) == qe.QE_ERR_INVALID
    assert lib.qe_probe_records(0, dummy, 1 << 32, 10, 0, dummy, None) == qe.QE_ERR_INVALID
    assert lib.qe_probe_records(1, dummy, 10, -1, 0, dummy, None) == qe.QE_ERR_INVALID
    assert lib.qe_probe_records(1, dummy, 10, 0, 0, dummy, None) == qe.QE_OK   # nothing to launch
