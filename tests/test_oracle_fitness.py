"""Pins of the oracle's circuit unitary and Eq. 11 fitness against facts fixed
outside the oracle: closed forms, textbook gate identities, the known NCV
costs of Toffoli (5) and Peres (4), the register convention of Eqs. 1-2, an
independent Kronecker-product construction, and brute force on 3 wires."""
import itertools
import math

import numpy as np
import pytest

from conftest import read_golden

NOT, CNOT, CV, CVDG, H, TG = 1, 2, 3, 4, 5, 6


def d(kind, t=0, c=0):
    return kind | (t << 4) | (c << 8)


def perm_matrix(n, fn):
    N = 1 << n
    M = np.zeros((N, N), complex)
    for i in range(N):
        M[fn(i), i] = 1
    return M


def toffoli_fn(i):
    # wire 0 (most significant bit) is the target, wires 1 and 2 the controls
    c, a, b = (i >> 2) & 1, (i >> 1) & 1, i & 1
    return ((c ^ (a & b)) << 2) | (a << 1) | b


def peres_fn(i):
    c, a, b = (i >> 2) & 1, (i >> 1) & 1, i & 1
    return ((c ^ (a & b)) << 2) | (a << 1) | (b ^ a)


def test_eq2_not_on_first_qubit_swaps_halves(oracle):
    # Eq. 2: X on the first qubit reorders the coefficients as
    # |00>,|01>,|10>,|11> <- |10>,|11>,|00>,|01>.
    U = oracle.unitary(2, [d(NOT, 0)])
    psi = np.array([1, 2, 3, 4], complex)        # a_a a_b, a_a b_b, b_a a_b, b_a b_b
    assert np.allclose(U @ psi, [3, 4, 1, 2])


def test_first_gate_acts_first(oracle):
    # U = G1 G0 for the list [G0, G1]: CNOT(0->1) then NOT(0) differs from
    # the reverse order; check against explicit matrices.
    g0, g1 = d(CNOT, 1, 0), d(NOT, 0)
    U = oracle.unitary(2, [g0, g1])
    assert np.allclose(U, oracle.unitary(2, [g1]) @ oracle.unitary(2, [g0]))
    assert not np.allclose(U, oracle.unitary(2, [g0]) @ oracle.unitary(2, [g1]))


@pytest.mark.parametrize("row", read_golden("closed_forms.txt"))
def test_closed_forms(oracle, row):
    n, kind, t, c = (int(x) for x in row[:4])
    expr = row[4]
    value = {"1-sqrt(1/2)": 1 - math.sqrt(0.5),
             "1-sqrt(1-sqrt(10)/4)": 1 - math.sqrt(1 - math.sqrt(10) / 4),
             "1-sqrt(1-cos(pi/8))": 1 - math.sqrt(1 - math.cos(math.pi / 8)),
             "0": 0.0}[expr]
    assert abs(value - float(row[5])) < 1e-15
    f, g, delta, ftr = oracle.fitness(n, [d(kind, t, c)], np.eye(1 << n))
    assert abs(f - value) < 1e-12
    assert abs(ftr - value) < 1e-12


def test_fitness_identity_and_global_phase(oracle):
    rng = np.random.default_rng(0)
    for n in (2, 3, 4):
        tab = oracle.lib_table(1, n)
        g = tab[rng.integers(0, len(tab), 20)]
        U = oracle.unitary(n, g)
        for alpha in (0.0, 0.3, -2.0, math.pi):
            f, gg, delta, ftr = oracle.fitness(n, g, np.exp(1j * alpha) * U)
            assert abs(f - 1) < 1e-12 and abs(gg - 1) < 1e-12 and abs(delta) < 1e-12


def test_fitness_zero_for_traceless(oracle):
    # |tr| = 0 gives fitness 0 (size - 0 over size = 1 under the root).
    for n in (1, 2, 3):
        f, g, delta, _ = oracle.fitness(n, [d(NOT, 0)], np.eye(1 << n))
        assert abs(f) < 1e-15 and abs(g) < 1e-15 and abs(delta - (1 << n)) < 1e-12


def test_trace_and_residual_forms_agree(oracle):
    # size - |tr(S^dagger T)| = (1/2) min_phi ||S - e^{i phi} T||^2 for unitaries.
    rng = np.random.default_rng(1)
    for n in (1, 2, 3, 4, 5):
        for lib in (0, 1):
            tab = oracle.lib_table(lib, n)
            for _ in range(10):
                g = tab[rng.integers(0, len(tab), rng.integers(1, 30))]
                tg = tab[rng.integers(0, len(tab), rng.integers(1, 30))]
                T = oracle.unitary(n, tg)
                f, gg, delta, ftr = oracle.fitness(n, g, T)
                tr = np.trace(oracle.unitary(n, g).conj().T @ T)
                assert abs(delta - ((1 << n) - abs(tr))) < 1e-10
                assert abs(f - ftr) < 1e-6 or abs(delta) < 1e-12
                assert abs(gg - abs(tr) / (1 << n)) < 1e-12
                assert 0 <= f <= 1


def test_unitarity(oracle):
    rng = np.random.default_rng(2)
    for n in range(1, 7):
        tab = oracle.lib_table(1, n)
        U = oracle.unitary(n, tab[rng.integers(0, len(tab), 40)])
        assert np.abs(U.conj().T @ U - np.eye(1 << n)).max() < 1e-12


def test_gate_identities(oracle):
    # V^2 = X, V V+ = I, H^2 = I, T^8 = I, CNOT^2 = I, each as a circuit
    # against the expected target.
    I4 = np.eye(4)
    cnot = oracle.unitary(2, [d(CNOT, 1, 0)])
    assert oracle.fitness(2, [d(CV, 1, 0)] * 2, cnot)[0] == pytest.approx(1, abs=1e-12)
    assert oracle.fitness(2, [d(CV, 1, 0), d(CVDG, 1, 0)], I4)[0] == pytest.approx(1, abs=1e-12)
    assert oracle.fitness(2, [d(H, 0)] * 2, I4)[0] == pytest.approx(1, abs=1e-12)
    assert oracle.fitness(2, [d(TG, 1)] * 8, I4)[0] == pytest.approx(1, abs=1e-12)
    assert oracle.fitness(2, [d(CNOT, 0, 1)] * 2, I4)[0] == pytest.approx(1, abs=1e-12)
    # and a few that must not be the identity
    assert oracle.fitness(2, [d(TG, 1)] * 4, I4)[0] < 0.5
    assert np.allclose(cnot, perm_matrix(2, lambda i: i ^ (1 if i & 2 else 0)))


def test_textbook_ncv_realizations(oracle):
    # Toffoli = CV(b->c) CNOT(a->b) CV+(b->c) CNOT(a->b) CV(a->c), Peres with
    # four gates (Barenco et al. 1995; the NCV costs 5 and 4).
    tof = [d(CV, 0, 2), d(CNOT, 2, 1), d(CVDG, 0, 2), d(CNOT, 2, 1), d(CV, 0, 1)]
    per = [d(CV, 0, 2), d(CV, 0, 1), d(CNOT, 2, 1), d(CVDG, 0, 2)]
    assert oracle.fitness(3, tof, perm_matrix(3, toffoli_fn))[0] == pytest.approx(1, abs=1e-12)
    assert oracle.fitness(3, per, perm_matrix(3, peres_fn))[0] == pytest.approx(1, abs=1e-12)


def test_dense_kronecker_definition(oracle):
    from oracle import dense
    rng = np.random.default_rng(3)
    for n in range(1, 5):
        tab = np.concatenate([oracle.lib_table(0, n), oracle.lib_table(1, n)])
        for _ in range(40):
            g = tab[rng.integers(0, len(tab), rng.integers(0, 16))]
            assert np.abs(oracle.unitary(n, g) - dense.unitary(n, g)).max() < 1e-12
            T = dense.unitary(n, tab[rng.integers(0, len(tab), 6)])
            # compare the radicands of Eq. 11 (the square root amplifies
            # rounding near fitness 1)
            rad_o = (1 - oracle.fitness(n, g, T)[3]) ** 2
            rad_d = (1 - dense.fitness_eq11(n, dense.unitary(n, g), T)) ** 2
            assert abs(rad_o - rad_d) < 1e-12


def test_brute_force_n3_all_length3(oracle):
    # Every length-3 sequence of the 22 instances of {I,NOT,CNOT,CV,CV+} on 3
    # wires: the per-gate oracle equals the Kronecker definition.
    from oracle import dense
    tab = oracle.lib_table(0, 3)
    assert len(tab) == 22
    seqs = np.array(list(itertools.product(range(22), repeat=3)))
    assert len(seqs) == 10648
    for s in seqs:
        g = tab[s]
        assert np.abs(oracle.unitary(3, g) - dense.unitary(3, g)).max() < 1e-12


def _best_over_sequences(oracle, T, length):
    tab = oracle.lib_table(0, 3)
    seqs = np.array(list(itertools.product(range(len(tab)), repeat=length)), np.int64)
    gates = tab[seqs].reshape(-1)
    B = len(seqs)
    out = oracle.eval_batch(np.full(B, 3, np.int8), np.arange(B + 1, dtype=np.int32) * length,
                            gates, np.zeros(B, np.int64), T)
    return out[:, 0]


def _argmax_count(f, m):
    return int((f >= m - 1e-9).sum())


def test_brute_force_ncv_costs(oracle):
    # Exhaustive search over <= 3 and <= 4 gates of the 22 NCV instances on 3
    # wires (I pads shorter circuits).  Toffoli (NCV cost 5) is not reached:
    # the best circuits score exactly the closed form of a CV gate against
    # the identity, 1 - sqrt(1 - sqrt(10)/4) (the best partial realisation
    # agrees with Toffoli on the 6 basis states whose controls are not both
    # set and applies a CV-like block to the other two), reached by 36
    # sequences of length 3 and 544 of length 4.  Peres (NCV cost 4) is
    # reached by exactly 8 sequences of 4 gates and not within 3 (best: the
    # same CV value, 14 sequences).  Among the 10 648 length-3 sequences the
    # fitness against Toffoli takes 52 distinct values.
    best_cv = 1 - math.sqrt(1 - math.sqrt(10) / 4)
    assert abs(best_cv - 0.542364) < 5e-7
    f_tof3 = _best_over_sequences(oracle, perm_matrix(3, toffoli_fn), 3)
    f_tof4 = _best_over_sequences(oracle, perm_matrix(3, toffoli_fn), 4)
    f_per3 = _best_over_sequences(oracle, perm_matrix(3, peres_fn), 3)
    f_per4 = _best_over_sequences(oracle, perm_matrix(3, peres_fn), 4)
    for f, m, cnt in ((f_tof3, best_cv, 36), (f_tof4, best_cv, 544), (f_per3, best_cv, 14),
                      (f_per4, 1.0, 8)):
        assert abs(f.max() - m) < 1e-12
        assert _argmax_count(f, f.max()) == cnt
    assert len(np.unique(np.round(f_tof3, 9))) == 52
    assert np.all(f_tof4 >= 0) and np.all(f_tof4 <= 1)


def test_brute_force_distinct_unitaries(oracle):
    # The 10 648 length-3 NCV sequences on 3 wires realise 3 806 distinct
    # unitaries, also 3 806 up to a global phase.
    tab = oracle.lib_table(0, 3)
    exact, upto_phase = set(), set()
    for s in itertools.product(range(len(tab)), repeat=3):
        U = oracle.unitary(3, tab[list(s)]).ravel()
        exact.add((np.round(U, 9) + 0.0).tobytes())
        k = int(np.argmax(np.abs(U) > 1e-9))
        upto_phase.add((np.round(U * (abs(U[k]) / U[k]), 9) + 0.0).tobytes())
    assert len(exact) == 3806 and len(upto_phase) == 3806


def test_batch_matches_single(oracle):
    rng = np.random.default_rng(5)
    nq, goff, gates, toff, targets = [], [0], [], [], []
    singles = []
    off = 0
    for b in range(30):
        n = int(rng.integers(1, 6))
        tab = oracle.lib_table(1, n)
        L = int(rng.integers(0, 20))
        g = tab[rng.integers(0, len(tab), L)]
        T = oracle.unitary(n, tab[rng.integers(0, len(tab), 5)])
        nq.append(n); goff.append(goff[-1] + L); gates.append(g); toff.append(off)
        targets.append(T.ravel()); off += T.size
        singles.append(oracle.fitness(n, g, T))
    out = oracle.eval_batch(nq, goff, np.concatenate(gates), toff, np.concatenate(targets))
    assert np.allclose(out, np.array(singles), atol=0, rtol=0)


def test_bad_descriptor_rejected(oracle):
    assert not oracle.check_desc(3, d(CNOT, 1, 1))     # control == target
    assert not oracle.check_desc(3, d(CV, 3, 0))       # wire out of range
    assert not oracle.check_desc(3, 9)                 # unknown kind
    assert oracle.check_desc(3, 0)
    with pytest.raises(ValueError):
        oracle.unitary(3, [d(CNOT, 1, 1)])


def test_table2_reproduces_only_phase_insensitively():
    # Reading of Eq. 11 (documented): the printed Toffoli matrix holds
    # |S_ij|^2 (rows/columns sum to 1), its mean error per term against
    # Toffoli is the ~0.02 quoted in the text, and the Table III accuracy
    # 0.7047 is reproduced by 1 - sqrt(1 - sum |S_ij|^2 |T_ij|^2 / size),
    # a phase-insensitive fitness; Eq. 11 as printed is the primary fitness.
    A = np.array([[float(x) for x in r] for r in read_golden("table2_toffoli.txt")])
    assert np.allclose(A.sum(0), 1, atol=2e-3) and np.allclose(A.sum(1), 1, atol=2e-3)
    Tm = perm_matrix(3, toffoli_fn)
    assert abs(np.abs(A - Tm).mean() - 0.02) < 0.005
    fP = 1 - math.sqrt(1 - (A * np.abs(Tm) ** 2).sum() / 8)
    assert abs(fP - 0.7047) < 1e-3


# ------------------------------------------ phase-insensitive fitness (oracle)
def test_phase_insensitive_closed_form(oracle):
    # CV against CNOT on (control 0, target 1): |U|^2 is 1 on the identity
    # block and 1/2 on the V block, so gP = (1 + 1 + 1/2 + 1/2) / 4 = 3/4 and
    # fP = 1 - sqrt(1/4) = 1/2, where Eq. 11 gives 1 - sqrt(1 - sqrt(10)/4)
    T = oracle.unitary(2, [d(CNOT, 1, 0)])
    fP, gP, rad = oracle.fitness_pi(2, [d(CV, 1, 0)], T)
    assert abs(gP - 0.75) < 1e-15 and abs(fP - 0.5) < 1e-15 and abs(rad - 0.25) < 1e-15
    f = oracle.fitness(2, [d(CV, 1, 0)], T)[0]
    assert abs(f - (1 - math.sqrt(1 - math.sqrt(10) / 4))) < 1e-12
    # exact synthesis scores 1, a circuit with no overlap 0
    assert oracle.fitness_pi(2, [d(CNOT, 1, 0)], T)[0] == 1.0
    assert abs(oracle.fitness_pi(1, [d(NOT, 0)], np.eye(2))[0]) < 1e-15


def test_phase_insensitive_ignores_diagonal_phases(oracle):
    # T gates (diagonal phases) before or after a circuit leave |U_ij| and so
    # fP unchanged, while the phase-sensitive Eq. 11 value moves
    rng = np.random.default_rng(11)
    lib1 = oracle.lib_table(1, 3)
    tgt = perm_matrix(3, peres_fn)
    moved = 0
    for _ in range(40):
        c = [int(x) for x in rng.choice(lib1, 6)]
        ph = [d(TG, int(w)) for w in rng.integers(0, 3, 3)]
        a = oracle.fitness_pi(3, c, tgt)
        for v in (ph + c, c + ph, ph + c + ph):
            b = oracle.fitness_pi(3, v, tgt)
            assert abs(a[0] - b[0]) < 1e-12 and abs(a[1] - b[1]) < 1e-12
        moved += abs(oracle.fitness(3, c + ph, tgt)[0] - oracle.fitness(3, c, tgt)[0]) > 1e-9
    assert moved > 0


def test_phase_insensitive_forms_agree(oracle):
    # rad + gP = 1 for any target (unitarity of U); for a permutation target
    # rad is the energy off the diagonal of U T^dagger / size
    rng = np.random.default_rng(12)
    for n in (1, 2, 3, 4):
        lib = oracle.lib_table(1, n)
        for _ in range(20):
            c = [int(x) for x in rng.choice(lib, 9)]
            U = oracle.unitary(n, c)
            Tg = oracle.unitary(n, [int(x) for x in rng.choice(lib, 5)])
            fP, gP, rad = oracle.fitness_pi(n, c, Tg)
            assert abs(rad + gP - 1) < 1e-12
            assert abs(gP - (np.abs(U) ** 2 * np.abs(Tg) ** 2).sum() / (1 << n)) < 1e-12
            perm = rng.permutation(1 << n)
            P = perm_matrix(n, lambda i: int(perm[i]))
            fP, gP, rad = oracle.fitness_pi(n, c, P)
            M = U @ P.conj().T
            off = (np.abs(M) ** 2).sum() - (np.abs(np.diag(M)) ** 2).sum()
            assert abs(rad - off / (1 << n)) < 1e-12
            assert abs(fP - (1 - math.sqrt(max(0.0, min(1.0, off / (1 << n)))))) < 1e-12


def cccnot_fn(i):
    b = [(i >> (3 - w)) & 1 for w in range(4)]
    b[0] ^= b[1] & b[2] & b[3]
    return (b[0] << 3) | (b[1] << 2) | (b[2] << 1) | b[3]


def test_table3_cccnot_value_is_the_identity_plateau(oracle):
    # Table III prints 0.6464 for the QEQEA on CCCNOT (stopped at the
    # generation limit).  Under the phase-insensitive reading that is exactly
    # the fitness of a circuit agreeing with CCCNOT on 14 of its 16 basis
    # states -- the identity, for one: 1 - sqrt(2/16) = 0.64645
    T = perm_matrix(4, cccnot_fn)
    fP, gP, rad = oracle.fitness_pi(4, [0, 0, 0], T)
    assert abs(gP - 14 / 16) < 1e-15 and abs(rad - 2 / 16) < 1e-15
    assert abs(fP - (1 - math.sqrt(2 / 16))) < 1e-15
    assert round(fP, 4) == 0.6464
    # (for the identity the trace is 14 as well, so Eq. 11 as printed agrees;
    # the readings differ on circuits with relative phases)
    assert abs(oracle.fitness(4, [0, 0, 0], T)[0] - (1 - math.sqrt(2 / 16))) < 1e-12
