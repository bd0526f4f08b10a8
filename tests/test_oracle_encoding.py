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


# ------------------------------------------------ adaptive mutation (Sec. IV-F)
# With pm = 1 every individual mutates, in qubit or qutrit mode (equiprobably).
# A state with no used slot (every circuit fitness negative) leaves elitism
# out, so the change from the call is the mutation alone.  Qutrits start as
# (1, 1, 1) (real), so that every one-parameter step of Eq. 12 that is not
# the identity changes a component, and both the parameter j and the step
# index a can be read back from the result.
def _mutate_once(oracle, seg, n=3, L=16, P=256, gen=0, seed=77, mrange=math.pi / 4):
    st = oracle.QeqeaState(n, L, P, 1, seed=seed)
    st.best_f[:] = np.float32(seg)
    st.qutrit[:] = np.tile(np.array([1, 0, 1, 0, 1, 0], np.float32), n * L * P)
    st.best_qutrit[:] = st.qutrit
    before = st.copy()
    st.update(gen, 1.0, mrange, np.zeros((P, L), np.uint32), np.full(P, -1, np.float32))
    return before, st


def _individual_slots(n, L, P, ind, R):
    return np.array([r * L * P + ind * L + pos for r in range(R) for pos in range(L)])


def _read_su3_step(q):
    """(j, a) of a one-parameter step applied to (1, 1, 1), or (None, 0)
    when the qutrit is unchanged (j >= 5, or a = 0)."""
    one = np.array([1, 0, 1, 0, 1, 0], np.float32)
    if np.array_equal(q, one):
        return None, 0
    z = q[0::2].astype(float) + 1j * q[1::2].astype(float)
    same = [z[k] == 1 for k in range(3)]
    if np.any(q[1::2] != 0):                       # a phase step
        j = 3 if not same[0] else 4
        c, s = (z[0].real, z[0].imag) if j == 3 else (z[1].real, z[1].imag)
        return j, int(round((math.atan2(s, c) % (2 * math.pi)) / (2 * math.pi) * 4096)) % 4096
    if same[2]:
        j, A, B = 0, z[0].real, z[1].real          # (c + s, c - s)
    elif same[1]:
        j, A, B = 1, z[0].real, z[2].real
    else:
        j, A, B = 2, z[2].real, z[1].real
    c, s = (A + B) / 2, (A - B) / 2
    return j, int(round(math.atan2(s, c) / (math.pi / 2) * 4096))


def test_mutation_full_fitness_changes_nothing(oracle):
    # Sec. IV-F: the mutation is proportional to the error; a slot whose
    # segment fitness is 1 does not move, in either mode
    before, after = _mutate_once(oracle, 1.0)
    assert np.array_equal(after.theta, before.theta)
    assert np.array_equal(after.qutrit, before.qutrit)
    assert np.array_equal(after.best_f, before.best_f)


@pytest.mark.parametrize("seg", [-1.0, 0.0, 0.25, 0.9])
def test_qutrit_step_scales_with_error(oracle, seg):
    # Eq. 12 with one parameter j (of 8) set to a * domain / 4096, with the
    # step index a uniform on [0, (1 - segFit) * 4096] (segFit of an unused
    # slot is 0).  The qutrit-mode individuals are the ones whose angles did
    # not move.
    n, L, P = 3, 16, 256
    R = n * n
    before, after = _mutate_once(oracle, seg, n, L, P)
    om = 1.0 - max(seg, 0.0)
    amax = math.floor(float(np.float32(om)) * 4096)
    qmode, js, avals = 0, [], []
    for ind in range(P):
        sl = _individual_slots(n, L, P, ind, R)
        if np.any(after.theta[sl] != before.theta[sl]):
            continue
        qmode += 1
        for s in sl[sl < n * L * P]:
            j, a = _read_su3_step(after.qutrit[6 * s:6 * s + 6])
            js.append(-1 if j is None else j)
            if j is not None:
                avals.append(a)
    # the mode is a fair coin per individual
    assert abs(qmode - P / 2) <= 5 * math.sqrt(P / 4)
    js = np.array(js)
    N = len(js)
    # j uniform over the 8 parameters: each of j = 0..4 one eighth, the three
    # phases that only multiply sine terms (identity) three eighths
    counts = np.array([(js == j).sum() for j in range(5)] + [(js == -1).sum()], float)
    exp = N * np.array([1, 1, 1, 1, 1, 3]) / 8.0
    assert ((counts - exp) ** 2 / exp).sum() < 30          # 5 dof, p ~ 1e-5
    av = np.array(avals, float)
    assert av.min() >= 0 and av.max() <= amax
    assert av.max() >= 0.95 * amax                          # the range is filled
    # uniform on [0, amax]: eight equal bins
    h = np.bincount(np.minimum((av / (amax + 1) * 8).astype(int), 7), minlength=8)
    e = len(av) / 8.0
    assert ((h - e) ** 2 / e).sum() < 35                    # 7 dof, p ~ 1e-5


@pytest.mark.parametrize("seg", [-1.0, 0.0, 0.25, 0.9])
def test_qubit_step_is_error_times_range(oracle, seg):
    # Qubit mode: every slot of the individual moves by +-(1 - segFit) *
    # mutationRange (angles as u32 turn fractions), the sign a fair coin
    n, L, P = 3, 16, 256
    R = n * n
    mrange = math.pi / 4
    before, after = _mutate_once(oracle, seg, n, L, P, mrange=mrange)
    om = 1.0 - max(seg, 0.0)
    step = om * mrange / (2 * math.pi) * 2 ** 32
    plus = minus = 0
    for ind in range(P):
        sl = _individual_slots(n, L, P, ind, R)
        dth = (after.theta[sl].astype(np.int64) - before.theta[sl].astype(np.int64)) % (1 << 32)
        if not np.any(dth):
            continue                                         # qutrit mode
        up = dth < (1 << 31)
        mag = np.where(up, dth, (1 << 32) - dth)
        assert np.all(np.abs(mag - step) <= step * 2 ** -20 + 1)
        plus += int(up.sum())
        minus += int((~up).sum())
    tot = plus + minus
    assert tot > 0 and abs(plus - tot / 2) <= 5 * math.sqrt(tot / 4)


# ------------------------------------------------------- GA rates (Sec. V-B)
def _distinct_population(oracle, I, P, L, n=6, lib=1):
    # every parent has a different gene at every position (n = 6, library
    # {H, T, CNOT, CV, CV+}: 102 instances >= P), so any exchange of genes
    # between two children is visible
    tab = oracle.lib_table(lib, n)
    assert P <= len(tab)
    g = np.zeros((I * P, L), np.uint16)
    for i in range(I):
        for k in range(P):
            for pos in range(L):
                g[i * P + k, pos] = tab[(k + 7 * pos + 3 * i) % len(tab)]
    return g, len(tab)


def test_ga_equal_fitness_selects_every_parent_once(oracle):
    I, P, L = 4, 64, 10
    g0, _ = _distinct_population(oracle, I, P, L)
    f = np.full(I * P, 0.5, np.float32)
    g1 = oracle.ga_update(6, 1, L, P, I, 5, 0, 0.0, 0.0, f, g0)
    assert np.array_equal(g1, g0)


def test_ga_two_point_crossover_rate(oracle):
    # pc = 0.9: a pair is crossed with probability pc; the exchanged genes of
    # a crossed pair are one contiguous run [lo, hi) between two cut points
    # drawn uniformly from 0..L (equal cuts exchange nothing)
    I, P, L, pc = 32, 64, 10, 0.9
    g0, _ = _distinct_population(oracle, I, P, L)
    f = np.full(I * P, 0.5, np.float32)
    half = P // 2
    visible, lengths, pairs = 0, [], 0
    for gen in range(4):
        g2 = oracle.ga_update(6, 1, L, P, I, 9, gen, pc, 0.0, f, g0)
        for i in range(I):
            for j in range(1, half):
                a, b = i * P + j, i * P + j + half
                diff = np.nonzero(g2[a] != g0[a])[0]
                assert np.array_equal(diff, np.nonzero(g2[b] != g0[b])[0])
                assert np.array_equal(g2[a][diff], g0[b][diff])
                assert np.array_equal(g2[b][diff], g0[a][diff])
                pairs += 1
                if len(diff):
                    assert diff[-1] - diff[0] + 1 == len(diff)   # one contiguous run
                    visible += 1
                    lengths.append(len(diff))
    p_vis = pc * (1 - 1 / (L + 1))
    assert abs(visible - pairs * p_vis) <= 5 * math.sqrt(pairs * p_vis * (1 - p_vis))
    # |a - b| for two uniform cuts in 0..L, given a != b: mean (L + 2) / 3
    d = np.arange(1, L + 1)
    pd = 2.0 * (L + 1 - d) / (L + 1) ** 2
    pd /= pd.sum()
    mean, var = (d * pd).sum(), ((d - (d * pd).sum()) ** 2 * pd).sum()
    assert abs(np.mean(lengths) - mean) <= 5 * math.sqrt(var / len(lengths))
    assert abs(mean - (L + 2) / 3) < 1e-12


def test_ga_gene_mutation_rate(oracle):
    # pg = 1/L: each gene is redrawn with probability pg, uniformly from the
    # library (so it stays the same with probability 1/|library|); child 0
    # is the best parent, unchanged
    I, P, L = 32, 64, 10
    pg = 1.0 / L
    g0, nl = _distinct_population(oracle, I, P, L)
    tab = set(int(x) for x in oracle.lib_table(1, 6))
    f = np.full(I * P, 0.5, np.float32)
    changed, genes = 0, 0
    for gen in range(4):
        g3 = oracle.ga_update(6, 1, L, P, I, 13, gen, 0.0, pg, f, g0)
        assert set(int(x) for x in g3.ravel()) <= tab
        for i in range(I):
            assert np.array_equal(g3[i * P], g0[i * P])
            blk = slice(i * P + 1, (i + 1) * P)
            changed += int((g3[blk] != g0[blk]).sum())
            genes += (P - 1) * L
    p = pg * (1 - 1 / nl)
    assert abs(changed - genes * p) <= 5 * math.sqrt(genes * p * (1 - p))
