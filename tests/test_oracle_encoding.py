"""Pins of the oracle's random numbers, circuit construction (Eq. 10),
qutrit measurement, SU(3) mutation (Eq. 12), elitism, adaptive mutation and
GA operators, against published vectors, the paper's worked example and
invariants of the definitions."""
import math

import numpy as np
import pytest

from conftest import read_golden


def test_philox_known_answers(oracle):
    for row in read_golden("philox_kat.txt"):
        vals = [int(x, 16) for x in row if x != "|"]
        ctr, key, want = vals[:4], vals[4:6], vals[6:10]
        assert list(oracle.philox(ctr, key)) == want


def test_eq10_table1_indices(oracle):
    # Table I: L=3, P=1, n=2 with one template -> memory indices 0, 7, 2.
    for pos, region, ind, index, *_ in read_golden("table1_cnot.txt"):
        assert oracle.segment_index(3, 1, int(region), int(ind), int(pos)) == int(index)


def _count_axis(oracle, q, axis_max):
    """Number of grid points u = m * 2^-24 whose measured axis is <= axis_max
    (the axis is non-decreasing in u, so binary search finds the edge)."""
    lo, hi = 0, 1 << 24                       # find first m with axis > axis_max
    while lo < hi:
        mid = (lo + hi) // 2
        if oracle.measure(q, mid << 8) <= axis_max:
            lo = mid + 1
        else:
            hi = mid
    return lo


def test_measurement_born_rule_table1(oracle):
    # Table I qutrit states: the printed axis is the most probable Born
    # outcome, and the measurement maps the uniform grid onto the outcomes in
    # proportion to |amplitude|^2 (no normalisation needed).
    for row in read_golden("table1_cnot.txt"):
        if row[4] == "-":
            continue
        q = np.array([float(x) for x in row[5:11]], np.float32)
        p = np.array([q[0] ** 2 + q[1] ** 2, q[2] ** 2 + q[3] ** 2, q[4] ** 2 + q[5] ** 2], float)
        axis = "xyz"[int(np.argmax(p))]
        assert axis == row[4]
        c0 = _count_axis(oracle, q, 0)
        c1 = _count_axis(oracle, q, 1)
        freq = np.array([c0, c1 - c0, (1 << 24) - c1]) / float(1 << 24)
        assert np.abs(freq - p / p.sum()).max() < 1e-6


def test_measurement_unnormalised_and_degenerate(oracle):
    q = np.array([0, 0, 3, 0, 0, 4], np.float32)       # p = (0, 9, 16)
    assert _count_axis(oracle, q, 0) == 0
    c1 = _count_axis(oracle, q, 1)
    assert abs(c1 / float(1 << 24) - 9 / 25) < 1e-6
    for w in (0, 1 << 31, 0xFFFFFFFF):
        assert oracle.measure(np.array([1, 0, 0, 0, 0, 0], np.float32), w) == 0


def test_sampling_indices_and_uniformity(oracle):
    n, L, P = 3, 7, 5
    st = oracle.QeqeaState(n, L, P, 2, seed=11)
    slots, gates = st.sample(3)
    R = n * n
    assert slots.shape == (2 * P, L)
    r = slots // (L * P)
    ind = (slots % (L * P)) // L
    pos = slots % L
    assert np.all(r < R) and np.all(ind < P)
    assert np.all(pos == np.arange(L)[None, :])          # Eq. 10: position is the thread index
    big = oracle.QeqeaState(n, 16, 64, 1, seed=12)
    s2, _ = big.sample(0)
    reg = (s2 // (16 * 64)).ravel()
    counts = np.bincount(reg, minlength=R)
    exp = len(reg) / R
    chi2 = ((counts - exp) ** 2 / exp).sum()
    assert chi2 < 30                                    # 8 dof, p ~ 2e-4
    s3, _ = big.sample(1)
    assert not np.array_equal(s2, s3)                   # generations draw afresh


def _unitary(oracle, n, g):
    return oracle.unitary(n, [g])


def test_decode_quarter_turns(oracle):
    # Template slots decode to the controlled V^q (q = angle in quarter
    # turns): I, CV, CNOT, CV+.  Since V^2 = X these satisfy
    # decode(q)^2 = decode(2q mod 4); a rotation slot decodes to NOT only at
    # a half turn with measured axis x (R_x(pi) ~ X), else to I.
    n, L, P = 3, 4, 3
    for q in range(4):
        st = oracle.QeqeaState(n, L, P, 1, seed=5)
        st.theta[:] = np.uint32(q << 30)
        st.qutrit[:] = 0
        st.qutrit[0::6] = 1.0                          # axis x with certainty
        slots, gates = st.sample(0)
        for s, gte in zip(slots.ravel(), gates.ravel()):
            r = s // (L * P)
            kind, t, c = gte & 15, (gte >> 4) & 15, (gte >> 8) & 15
            if r < n:
                assert (kind, t) == ((1, r) if q == 2 else (0, 0))
            else:
                p = r - n
                cc = p // (n - 1)
                tt = p % (n - 1)
                tt = tt if tt < cc else tt + 1
                assert kind == [0, 3, 2, 4][q]
                if q:
                    assert (t, c) == (tt, cc)
        # V^q algebra on one template
        dq = [0, 3 | (1 << 4), 2 | (1 << 4), 4 | (1 << 4)]
        Uq = _unitary(oracle, 2, dq[q])
        assert np.allclose(Uq @ Uq, _unitary(oracle, 2, dq[(2 * q) % 4]))


def test_su3_unitary_det1(oracle):
    rng = np.random.default_rng(7)
    assert np.allclose(oracle.su3(np.zeros(8)), np.eye(3))
    for _ in range(500):
        p = np.concatenate([rng.uniform(0, np.pi / 2, 3), rng.uniform(0, 2 * np.pi, 5)])
        U = oracle.su3(p)
        assert np.abs(U.conj().T @ U - np.eye(3)).max() < 1e-12
        assert abs(np.linalg.det(U) - 1) < 1e-12


def test_su3_single_parameter_steps(oracle):
    # The mutation step is Eq. 12 with one parameter non-zero.
    rng = np.random.default_rng(8)
    for j in range(8):
        for a in (0, 1, 1000, 2048, 4095):
            q = rng.normal(size=6).astype(np.float32)
            p = np.zeros(8)
            p[j] = a * (np.pi / 2 if j < 3 else 2 * np.pi) / 4096
            U = oracle.su3(p)
            z = q[0::2].astype(float) + 1j * q[1::2].astype(float)
            want = U @ z
            got = oracle.su3_step(q, j, a)
            gz = got[0::2].astype(float) + 1j * got[1::2].astype(float)
            assert np.abs(gz - want).max() < 2e-6 * max(1.0, np.abs(z).max())
            if j >= 5 or a == 0:
                assert np.array_equal(got, q)


def _used_slots(slots, I, S):
    used = [set() for _ in range(I)]
    P_L = slots.shape[0] // I
    for i in range(I):
        used[i] = set(int(s) for s in slots[i * P_L:(i + 1) * P_L].ravel())
    return used


def test_update_elitism_and_invariants(oracle):
    n, L, P, I = 3, 6, 8, 2
    st = oracle.QeqeaState(n, L, P, I, seed=21)
    S, Q = n * n * L * P, n * L * P
    rng = np.random.default_rng(9)
    pm, mrange = 0.0, float(np.pi / 4)
    for gen in range(6):
        before = st.copy()
        slots, gates = st.sample(gen)
        f = rng.uniform(0, 1, I * P).astype(np.float32)
        st.update(gen, pm, mrange, slots, f)
        used = _used_slots(slots, I, S)
        for i in range(I):
            seg = np.full(S, -1.0, np.float32)
            for k in range(P):
                for s in slots[i * P + k]:
                    seg[s] = max(seg[s], f[i * P + k])
            for s in range(S):
                o = i * S + s
                if s not in used[i]:                       # unused: untouched
                    assert st.theta[o] == before.theta[o]
                    assert st.best_f[o] == before.best_f[o]
                    continue
                assert st.best_f[o] == max(before.best_f[o], seg[s])   # best non-decreasing
                if seg[s] > before.best_f[o]:
                    assert st.best_theta[o] == before.theta[o]
                    assert st.theta[o] == before.theta[o]
                else:
                    assert st.theta[o] == before.best_theta[o]        # reverted


def test_mutation_magnitude_bound(oracle):
    n, L, P, I = 3, 5, 16, 1
    st = oracle.QeqeaState(n, L, P, I, seed=31)
    S = n * n * L * P
    mrange = float(np.pi / 4)
    rng = np.random.default_rng(10)
    changed = 0
    for gen in range(4):
        slots, gates = st.sample(gen)
        f = rng.uniform(0, 1, P).astype(np.float32)
        st.update(gen, 0.0, mrange, slots, f)           # elitism only
        after_elit = st.copy()
        # the same generation again with pm = 1: elitism is idempotent on the
        # reverted state, then every individual mutates
        st2 = after_elit.copy()
        st2.update(gen, 1.0, mrange, np.zeros_like(slots), np.full(P, -1, np.float32))
        d = (st2.theta.astype(np.int64) - after_elit.theta.astype(np.int64)) % (1 << 32)
        d = np.minimum(d, (1 << 32) - d)
        seg = np.maximum(after_elit.best_f, 0).astype(np.float64)
        # (1 - segFit) * range in turn units, with the float32 rounding of the
        # step (a few units of 2^-24 relative) as slack
        bound = (1 - seg) * mrange / (2 * np.pi) * 2 ** 32 * (1 + 2 ** -21) + 1
        assert np.all(d <= bound)
        changed += int((d > 0).sum())
        assert np.all(d[after_elit.best_f >= 1] == 0)
        st = after_elit
    assert changed > 0


def test_ga_sus_counts(oracle):
    rng = np.random.default_rng(11)
    for P in (2, 7, 64, 100):
        for _ in range(20):
            f = rng.uniform(0, 1, P).astype(np.float32)
            f[rng.random(P) < 0.2] = 0
            w = np.floor(f.astype(np.float32) * np.float32(2 ** 24)).astype(np.int64)
            if w.sum() == 0:
                w[:] = 1
            sel = oracle.ga_sus(f, int(rng.integers(0, 2 ** 32)))
            counts = np.bincount(sel, minlength=P)
            e = P * w / w.sum()
            assert np.all(counts >= np.floor(e) - 1e-9) and np.all(counts <= np.ceil(e) + 1e-9)
            assert np.all(np.diff(sel) >= 0)


def test_ga_update_invariants(oracle):
    n, lib, L, P, I = 3, 0, 10, 64, 2
    g0 = oracle.ga_init(n, lib, L, P, I, seed=41)
    tab = set(int(x) for x in oracle.lib_table(lib, n))
    assert set(int(x) for x in g0.ravel()) <= tab
    rng = np.random.default_rng(12)
    f = rng.uniform(0, 1, I * P).astype(np.float32)
    # no crossover, no mutation: children are copies of selected parents,
    # slot 0 is the best individual
    g1 = oracle.ga_update(n, lib, L, P, I, 41, 0, 0.0, 0.0, f, g0)
    for i in range(I):
        par = {tuple(x) for x in g0[i * P:(i + 1) * P]}
        assert all(tuple(x) in par for x in g1[i * P:(i + 1) * P])
        assert np.array_equal(g1[i * P], g0[i * P + int(np.argmax(f[i * P:(i + 1) * P]))])
    # crossover only: per position, the multiset of genes over the pair is kept
    g2 = oracle.ga_update(n, lib, L, P, I, 41, 0, 1.0, 0.0, f, g0)
    sel_src = oracle.ga_update(n, lib, L, P, I, 41, 0, 0.0, 0.0, f, g0)
    for i in range(I):
        half = P // 2
        for j in range(1, half):
            x, y = g2[i * P + j], g2[i * P + j + half]
            u, v = sel_src[i * P + j], sel_src[i * P + j + half]
            for pos in range(L):
                assert sorted((x[pos], y[pos])) == sorted((u[pos], v[pos]))
    # mutation only: genes stay in the library
    g3 = oracle.ga_update(n, lib, L, P, I, 41, 0, 0.0, 1.0, f, g0)
    assert set(int(x) for x in g3.ravel()) <= tab
    assert not np.array_equal(g3, sel_src)
