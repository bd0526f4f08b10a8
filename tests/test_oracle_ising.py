"""Pins of the oracle's Ising gate model (Eqs. 3-6 of Sec. III) and of the
QEQEA encoding for the Ising library (Secs. IV-A to IV-D), against facts
fixed outside the oracle: the Table I CNOT circuit, textbook identities that
tie each rotation and the interaction to the already pinned discrete gates
(T, H, CNOT), an independent Kronecker/template construction, and counting
arguments for the encoding."""
import math

import numpy as np
import pytest

from conftest import read_golden

NOT, CNOT, H, TG = 1, 2, 5, 6
RX, RY, RZ, ZZ = 7, 8, 9, 10
QUARTER = 1 << 30          # a quarter turn as a u32 angle: theta = pi / 2


def d(kind, t=0, c=0):
    return kind | (t << 4) | (c << 8)


def theta_of(u):
    return 2 * math.pi * int(u) / 2.0 ** 32


def cnot_target0(n=2):
    """CNOT with the target on wire 0 (most significant bit), control wire 1."""
    N = 1 << n
    M = np.zeros((N, N), complex)
    for i in range(N):
        b0, b1 = (i >> (n - 1)) & 1, (i >> (n - 2)) & 1
        M[i ^ ((b1) << (n - 1)), i] = 1
    return M


def test_per_gate_matches_kronecker_templates(oracle):
    # random circuits mixing the discrete and Ising kinds, against the dense
    # construction (Kronecker products, exponentiated +-1 template diagonals)
    from oracle import dense
    rng = np.random.default_rng(1809)
    for n in (1, 2, 3, 4):
        for _ in range(12):
            L = int(rng.integers(1, 14))
            gates, angles = [], []
            for _ in range(L):
                kind = int(rng.choice([RX, RY, RZ, ZZ, NOT, H, TG, CNOT] if n > 1 else [RX, RY, RZ, NOT, H, TG]))
                t = int(rng.integers(n))
                c = int(rng.choice([w for w in range(n) if w != t])) if n > 1 else 0
                gates.append(d(kind, t, c if kind in (ZZ, CNOT) else 0))
                angles.append(int(rng.integers(0, 1 << 32, dtype=np.uint64)))
            U = oracle.unitary(n, gates, angles)
            W = dense.unitary(n, gates, [theta_of(a) for a in angles])
            assert np.abs(U - W).max() < 1e-12
            assert np.abs(U.conj().T @ U - np.eye(1 << n)).max() < 1e-12


@pytest.mark.parametrize("n,w", [(1, 0), (2, 1), (3, 0), (3, 2)])
def test_rz_eighth_turn_is_t_up_to_global_phase(oracle, n, w):
    # T = diag(1, e^{i pi/4}) = e^{i pi/8} R_z(pi/4): pins the sign of Eq. 5
    # and the turn-fraction encoding of the angle (pi/4 = 2^29)
    Urz = oracle.unitary(n, [d(RZ, w)], [1 << 29])
    Ut = oracle.unitary(n, [d(TG, w)])
    assert np.abs(Ut - np.exp(1j * math.pi / 8) * Urz).max() < 1e-14
    f, g, delta, _ = oracle.fitness(n, [d(RZ, w)], Ut, angles=[1 << 29])
    assert abs(g - 1.0) < 1e-14 and delta < 1e-12
    # the opposite sign would give T^dagger, which is not T up to phase
    f2, g2, _, _ = oracle.fitness(n, [d(RZ, w)], Ut, angles=[(1 << 32) - (1 << 29)])
    assert g2 < 0.93


@pytest.mark.parametrize("u", [0, 1 << 29, 0x5A5A5A5A, 3 * QUARTER + 12345])
def test_rx_is_h_rz_h_and_ry_is_s_rx_sdg(oracle, u):
    # H Z H = X and S X S^dagger = Y (S = T^2, S^dagger = T^6) carry over to
    # the exponentials, exactly: pins Eq. 3 against Eq. 5 and Eq. 4 against 3
    for n, w in ((1, 0), (3, 1)):
        assert np.abs(oracle.unitary(n, [d(H, w), d(RZ, w), d(H, w)], [0, u, 0])
                      - oracle.unitary(n, [d(RX, w)], [u])).max() < 1e-14
        gates = [d(TG, w)] * 6 + [d(RX, w)] + [d(TG, w)] * 2
        angles = [0] * 6 + [u] + [0] * 2
        assert np.abs(oracle.unitary(n, gates, angles)
                      - oracle.unitary(n, [d(RY, w)], [u])).max() < 1e-13


@pytest.mark.parametrize("n,a,b", [(2, 0, 1), (3, 0, 2), (3, 2, 1), (4, 1, 3)])
def test_interaction_is_cnot_rz_cnot(oracle, n, a, b):
    # exp(-i theta/2 Z_a Z_b) = CNOT_{a->b} R_z,b(theta) CNOT_{a->b}; the
    # interaction is symmetric in its two wires
    for u in (QUARTER, 3 * QUARTER, 0x12345678):
        J = oracle.unitary(n, [d(ZZ, a, b)], [u])
        C = oracle.unitary(n, [d(CNOT, b, a), d(RZ, b), d(CNOT, b, a)], [0, u, 0])
        assert np.abs(J - C).max() < 1e-14
        assert np.abs(J - oracle.unitary(n, [d(ZZ, b, a)], [u])).max() < 1e-15
        assert np.abs(J - np.diag(np.diag(J))).max() == 0.0


def test_half_turns_reach_not_and_hadamard(oracle):
    # R_x(pi) = -iX and H = i R_x(pi) R_y(pi/2): Eq. 11 is 1 for both
    half = 1 << 31
    X = oracle.unitary(1, [d(NOT)])
    f, g, _, _ = oracle.fitness(1, [d(RX)], X, angles=[half])
    assert abs(g - 1) < 1e-15 and f > 1 - 1e-7
    Hm = oracle.unitary(2, [d(H, 1)])
    f, g, _, _ = oracle.fitness(2, [d(RY, 1), d(RX, 1)], Hm, angles=[QUARTER, half])
    assert abs(g - 1) < 1e-15 and f > 1 - 1e-7


def test_table1_decodes_to_the_printed_cnot_circuit(oracle):
    # Table I: memory indices 0, 7, 2 with L=3, P=1, n=2 and the printed
    # angles and axes decode to R_1y(pi/2) J_12(3pi/2) R_1x(3pi/2), which
    # is CNOT up to phases applied after it: the phase-insensitive fitness
    # is 1, while Eq. 11 as printed gives |tr| = 2, i.e. 1 - sqrt(1/2).
    n, L, P = 2, 3, 1
    R = oracle.regions(n, oracle.LIB_ISING)
    assert R == 3
    theta = np.zeros(R * L * P, np.uint32)
    qutrit = np.zeros(n * L * P * 6, np.float32)
    want = []
    for pos, index, pis, gate, *wires in read_golden("table1_cnot_ising.txt"):
        s = int(index)
        theta[s] = oracle.turns(float(pis) * math.pi)
        if gate in ("rx", "ry", "rz"):
            axis = "xyz".index(gate[1])
            qutrit[6 * s + 2 * axis] = 1.0        # a qutrit that measures this axis surely
            want.append(d(RX + axis, int(wires[0])))
        else:
            want.append(d(ZZ, int(wires[0]), int(wires[1])))
    gates, angles = [], []
    for pos, index, *_ in read_golden("table1_cnot_ising.txt"):
        g, a = oracle.decode_slot(n, oracle.LIB_ISING, L, P, 7, 0, 0, int(index), theta, qutrit)
        gates.append(g)
        angles.append(a)
    assert gates == want
    assert [round(theta_of(a), 6) for a in angles] == [1.570796, 4.712389, 4.712389]
    T = cnot_target0()
    fP, gP, rad = oracle.fitness_pi(n, gates, T, angles=angles)
    assert abs(fP - 1.0) < 1e-7 and abs(gP - 1.0) < 1e-15
    f, g, delta, _ = oracle.fitness(n, gates, T, angles=angles)
    assert abs(g - 0.5) < 1e-15
    assert abs(f - (1 - math.sqrt(0.5))) < 1e-14


@pytest.mark.parametrize("n", [2, 3, 4, 5, 6])
def test_ising_regions_cover_each_unordered_pair_once(oracle, n):
    L, P = 2, 3
    R = oracle.regions(n, oracle.LIB_ISING)
    assert R == n + n * (n - 1) // 2
    assert oracle.regions(n, 0) == n * n
    theta = np.full(R * L * P, 0x1234, np.uint32)
    qutrit = np.zeros(n * L * P * 6, np.float32)
    qutrit[2::6] = 1.0                                # every rotation measures y
    pairs = []
    for r in range(R):
        s = oracle.segment_index(L, P, r, 1, 1)
        g, a = oracle.decode_slot(n, oracle.LIB_ISING, L, P, 3, 0, 0, s, theta, qutrit)
        assert a == 0x1234
        if r < n:
            assert g == d(RY, r)
        else:
            assert g & 15 == ZZ
            pairs.append(((g >> 4) & 15, (g >> 8) & 15))
    assert pairs == [(a, b) for a in range(n) for b in range(a + 1, n)]


def test_ising_sampling_takes_slot_angles_and_born_axes(oracle):
    n, L, P, I = 3, 9, 40, 2
    st = oracle.QeqeaState(n, L, P, I, seed=77, library=oracle.LIB_ISING)
    R = n + n * (n - 1) // 2
    S = R * L * P
    slots, gates, angles = st.sample(5, with_angles=True)
    axes = np.zeros(3, int)
    for row in range(I * P):
        i = row // P
        for pos in range(L):
            s, g, a = int(slots[row, pos]), int(gates[row, pos]), int(angles[row, pos])
            assert s % L == pos and s < S
            assert a == st.theta[i * S + s]
            r = s // (L * P)
            if r < n:
                assert g & 15 in (RX, RY, RZ) and (g >> 4) & 15 == r
                axes[(g & 15) - RX] += 1
            else:
                assert g & 15 == ZZ
    # qutrits start in (1,1,1)/sqrt(3): every axis is equally likely
    frac = axes / axes.sum()
    assert np.abs(frac - 1 / 3).max() < 0.06


def test_ising_update_moves_every_region(oracle):
    # with pm = 1 every individual mutates; in qubit mode all R*L of its
    # angles move (no slot used yet, so segFit = 0 and the step is the full
    # range), in qutrit mode none of them do and only qutrits move (each by
    # one SU(3) step, three of the eight parameters of which are no-ops)
    n, L, P, I = 3, 4, 16, 1
    st = oracle.QeqeaState(n, L, P, I, seed=9, library=oracle.LIB_ISING)
    R = n + n * (n - 1) // 2
    th0, q0 = st.theta.copy(), st.qutrit.copy()
    slots = np.full((P, L), 0xFFFFFFFF, np.uint32)     # no slot used this generation
    st.update(0, 1.0, math.pi / 4, slots, np.full(P, -1.0, np.float32))
    moved = (st.theta != th0).reshape(R, P, L)
    qmoved = (st.qutrit != q0).reshape(n, P, L, 6).any(axis=3)
    modes = set()
    for ind in range(P):
        if moved[:, ind, :].any():
            assert moved[:, ind, :].all() and not qmoved[:, ind, :].any()
            modes.add("qubit")
        else:
            assert qmoved[:, ind, :].any()
            modes.add("qutrit")
    assert modes == {"qubit", "qutrit"}


def test_check_desc_ising(oracle):
    assert oracle.check_desc(3, d(ZZ, 0, 2), ising=True)
    assert not oracle.check_desc(3, d(ZZ, 1, 1), ising=True)     # one wire twice
    assert not oracle.check_desc(3, d(ZZ, 0, 3), ising=True)     # wire out of range
    assert not oracle.check_desc(3, d(RX, 3), ising=True)
    assert not oracle.check_desc(3, 11, ising=True)               # unknown kind
    assert oracle.check_desc(3, d(CNOT, 0, 1), ising=True)
    assert not oracle.check_desc(3, d(RX, 0))                     # discrete-only check
    with pytest.raises(ValueError):
        oracle.unitary(2, [d(RX, 0)])                             # angles required


def test_batch_with_angles_matches_single_circuits(oracle):
    rng = np.random.default_rng(5)
    nq, goff, gates, angles, toff, targets = [], [0], [], [], [], []
    singles = []
    for b in range(7):
        n = int(rng.integers(1, 5))
        L = int(rng.integers(0, 9))
        g = [d(RX + int(rng.integers(3)), int(rng.integers(n))) for _ in range(L)]
        a = [int(x) for x in rng.integers(0, 1 << 32, size=L, dtype=np.uint64)]
        T = oracle.unitary(n, [d(RY, 0), d(H, n - 1)], [12345, 0])
        nq.append(n); gates += g; angles += a; goff.append(len(gates))
        toff.append(sum(t.size for t in targets)); targets.append(T)
        singles.append((n, g, a, T))
    flat = np.concatenate([t.ravel() for t in targets])
    out0 = oracle.eval_batch_ang(nq, goff, gates, angles, toff, flat, mode=0)
    out1 = oracle.eval_batch_ang(nq, goff, gates, angles, toff, flat, mode=1)
    for b, (n, g, a, T) in enumerate(singles):
        assert np.allclose(out0[b], oracle.fitness(n, g, T, angles=a), atol=0, rtol=0)
        assert np.allclose(out1[b, :3], oracle.fitness_pi(n, g, T, angles=a), atol=0, rtol=0)
