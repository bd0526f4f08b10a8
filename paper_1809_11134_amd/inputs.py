"""Seeded synthetic inputs for the circuit-fitness path (both the HIP path and
the CPU oracle consume them).

This module holds none of the method's arithmetic: it only draws gate lists
(16-bit descriptors) with numpy's PCG64 generator.  Target unitaries are
built from the drawn gate lists by whichever side consumes them.

Descriptor layout: kind in bits 0-3, target wire in bits 4-7, control wire in
bits 8-11.  Kinds: 0 I, 1 NOT, 2 CNOT, 3 CV, 4 CV+, 5 H, 6 T; the Ising kinds
7 R_x, 8 R_y, 9 R_z, 10 J (second wire in the control field) carry an angle,
a u32 fraction of a full turn, drawn here as raw 32-bit integers.

The paper's own workloads are small reversible targets (CNOT, Toffoli,
Peres, CCCNOT; Sec. V, Tables I-III) reached by short circuits of library
gates.  The workloads here keep that structure -- targets are products of a
few library gates, permutation targets are products of NOT/CNOT -- at the
batch sizes of the throughput study.
"""
import numpy as np

I_, NOT, CNOT, CV, CVDG, H, T = range(7)
RX, RY, RZ, ZZ = 7, 8, 9, 10
LIB_NCV = 0      # {I, NOT, CNOT, CV, CV+}
LIB_HT_NCV = 1   # {H, T, CNOT, CV, CV+}
LIB_ISING = 2    # {R_x, R_y, R_z, J} with angles

# angles that sit on the quarter-turn boundaries of the half-angle reduction
EDGE_ANGLES = np.array([0, 1, (1 << 30) - 1, 1 << 30, (1 << 31) - 1, 1 << 31, 3 << 30,
                        (3 << 30) - 1, 0xFFFFFFFF], np.uint32)

SEED_BASE = 1809111340


def desc(kind, tgt=0, ctl=0):
    return (kind & 15) | ((tgt & 15) << 4) | ((ctl & 15) << 8)


def _pairs(n):
    return [(c, t) for c in range(n) for t in range(n) if t != c]


def library(lib, n):
    """All gate instances of a library on n wires, as descriptors."""
    out = []
    if lib == LIB_NCV:
        out.append(desc(I_))
        out += [desc(NOT, w) for w in range(n)]
    else:
        out += [desc(H, w) for w in range(n)]
        out += [desc(T, w) for w in range(n)]
    for c, t in _pairs(n):
        out += [desc(CNOT, t, c), desc(CV, t, c), desc(CVDG, t, c)]
    return np.array(out, np.uint16)


def permutation_gates(n):
    """NOT and CNOT instances: their products are permutation matrices."""
    return np.array([desc(NOT, w) for w in range(n)] +
                    [desc(CNOT, t, c) for c, t in _pairs(n)], np.uint16)


def random_circuits(rng, count, n, L, lib):
    tab = library(lib, n)
    return tab[rng.integers(0, len(tab), size=(count, L))].astype(np.uint16)


def random_target_gates(rng, n, length, lib=None, permutation=False):
    tab = permutation_gates(n) if permutation else library(lib, n)
    if lib == LIB_NCV and not permutation:
        tab = tab[1:]            # a target is a product of non-identity gates
    return tab[rng.integers(0, len(tab), size=length)].astype(np.uint16)


def planted_population(rng, target_gates, count, n, L, lib, max_edits=8):
    """Circuits near the target: the target's own gate list with 0..max_edits
    random substitutions, insertions or deletions, padded with I or
    truncated to L gates."""
    tab = library(lib, n)
    out = np.zeros((count, L), np.uint16)
    for k in range(count):
        g = list(int(x) for x in target_gates)
        for _ in range(int(rng.integers(0, max_edits + 1))):
            op = int(rng.integers(0, 3))
            if op == 0 and g:
                g[int(rng.integers(0, len(g)))] = int(tab[rng.integers(0, len(tab))])
            elif op == 1:
                g.insert(int(rng.integers(0, len(g) + 1)), int(tab[rng.integers(0, len(tab))]))
            elif g:
                del g[int(rng.integers(0, len(g)))]
        g = (g + [desc(I_)] * L)[:L]
        out[k] = g
    return out


def random_ising_circuits(rng, count, n, L, discrete_frac=0.0, edge_frac=0.1):
    """(gates [count, L] uint16, angles [count, L] uint32): each gate is a
    rotation about x, y or z on a random wire or (n >= 2) an interaction on
    a random unordered wire pair, with a uniform 32-bit angle (a fraction
    edge_frac of them taken from EDGE_ANGLES); a fraction discrete_frac of
    the gates are drawn from {H, T, CNOT, CV, CV+} instead (angle 0)."""
    kinds = [RX, RY, RZ] + ([ZZ] if n >= 2 else [])
    disc = library(LIB_HT_NCV, n)
    gates = np.zeros((count, L), np.uint16)
    angles = rng.integers(0, 1 << 32, size=(count, L), dtype=np.uint64).astype(np.uint32)
    edge = rng.random((count, L)) < edge_frac
    angles[edge] = EDGE_ANGLES[rng.integers(0, len(EDGE_ANGLES), size=int(edge.sum()))]
    for c in range(count):
        for p in range(L):
            if rng.random() < discrete_frac:
                gates[c, p] = disc[rng.integers(0, len(disc))]
                angles[c, p] = 0
                continue
            k = int(kinds[rng.integers(0, len(kinds))])
            a = int(rng.integers(0, n))
            b = int(rng.integers(0, n - 1)) if n >= 2 else 0
            b = b + 1 if b >= a else b
            gates[c, p] = desc(k, a, b if k == ZZ else 0)
    return gates, angles


# ----------------------------------------------------------------- workloads
def workload_ga_n3(scale=1):
    """n=3, library {I,NOT,CNOT,CV,CV+}, target = product of 5 random library
    gates, classical GA with 64 circuits x 10 gates, 20 generations."""
    rng = np.random.default_rng(SEED_BASE + 1)
    return dict(name="ga_n3_p64_l10", n=3, lib=LIB_NCV, algorithm="ga", P=64, L=10,
                instances=1, generations=20,
                target_gates=[random_target_gates(rng, 3, 5, LIB_NCV)],
                seed=SEED_BASE + 1)


def workload_qeqea_n4(P=4096, instances=1):
    """n=4, library {I,NOT,CNOT,CV,CV+}, target = product of 12 random
    NOT/CNOT gates (a reversible permutation), QEQEA with P=4096 circuits of
    30 gates sampled per generation, 100 generations."""
    rng = np.random.default_rng(SEED_BASE + 2)
    return dict(name="qeqea_n4_p4096_l30", n=4, lib=LIB_NCV, algorithm="qeqea", P=P, L=30,
                instances=instances, generations=100,
                target_gates=[random_target_gates(rng, 4, 12, permutation=True)
                              for _ in range(instances)],
                seed=SEED_BASE + 2)


def workload_uneven(count=16384, per_population=64, seed_offset=3):
    """Uneven eval-only batch: populations of `per_population` circuits share
    a width n ~ U{3..6} and a target (product of U[8,40] gates of
    {H,T,CNOT,CV,CV+}); each circuit has its own length L ~ U[8,64]."""
    rng = np.random.default_rng(SEED_BASE + seed_offset)
    pops = (count + per_population - 1) // per_population
    nq, goff, gates, tgt_gates, tidx = [], [0], [], [], []
    for p in range(pops):
        n = int(rng.integers(3, 7))
        tgt_gates.append((n, random_target_gates(rng, n, int(rng.integers(8, 41)), LIB_HT_NCV)))
        for _ in range(min(per_population, count - p * per_population)):
            L = int(rng.integers(8, 65))
            gates.append(random_circuits(rng, 1, n, L, LIB_HT_NCV)[0])
            goff.append(goff[-1] + L)
            nq.append(n)
            tidx.append(p)
    return dict(name=f"uneven_{count}", nq=np.array(nq, np.int8), goff=np.array(goff, np.int32),
                gates=np.concatenate(gates).astype(np.uint16), target_gates=tgt_gates,
                target_index=np.array(tidx, np.int64))


def workload_mixed_ga(populations=256, P=64, seed_offset=8):
    """Mixed GA search: `populations` independent GA populations of P
    circuits, population i on n_i ~ U{3..6} wires with genomes of
    L_i ~ U[8,64] gates of {H,T,CNOT,CV,CV+}, its target a product of
    U[8,40] gates of the same library (16384 evaluations per generation at
    the defaults), 50 generations."""
    rng = np.random.default_rng(SEED_BASE + seed_offset)
    widths, lengths, tgt = [], [], []
    for _ in range(populations):
        n = int(rng.integers(3, 7))
        widths.append(n)
        lengths.append(int(rng.integers(8, 65)))
        tgt.append(random_target_gates(rng, n, int(rng.integers(8, 41)), LIB_HT_NCV))
    return dict(name=f"mixed_ga_i{populations}_p{P}", lib=LIB_HT_NCV, algorithm="ga", P=P,
                instances=populations, generations=50, widths=widths, lengths=lengths,
                target_gates=tgt, seed=SEED_BASE + seed_offset)


def workload_precision_n6(P=8192, L=48):
    """n=6, library {H,T,CNOT,CV,CV+}, P=8192 circuits x 48 gates, target =
    product of 40 library gates.  A quarter of the circuits are uniform
    random, three quarters are the target's gate list with 0..8 random
    edits, so that fitness values spread over (0, 1]."""
    rng = np.random.default_rng(SEED_BASE + 4)
    n, lib = 6, LIB_HT_NCV
    tg = random_target_gates(rng, n, 40, lib)
    nr = P // 4
    pop = np.concatenate([random_circuits(rng, nr, n, L, lib),
                          planted_population(rng, tg, P - nr, n, L, lib)])
    return dict(name="precision_n6_p8192_l48", n=n, lib=lib, P=P, L=L, target_gates=tg,
                gates=pop)


def workload_qeqea_n5(instances=1024, P=64, L=40):
    """n=5, library {I,NOT,CNOT,CV,CV+}, 1024 QEQEA populations x 64 circuits
    of 40 gates (65536 evaluations per generation), 200 generations; each
    population's target is a product of 16 random NOT/CNOT gates."""
    rng = np.random.default_rng(SEED_BASE + 5)
    return dict(name="qeqea_n5_i1024_p64_l40", n=5, lib=LIB_NCV, algorithm="qeqea", P=P, L=L,
                instances=instances, generations=200,
                target_gates=[random_target_gates(rng, 5, 16, permutation=True)
                              for _ in range(instances)],
                seed=SEED_BASE + 5)


def workload_qeqea_ising_n4(P=4096, L=30, instances=1):
    """n=4, the Ising library of Sec. III (rotations about x, y, z and the
    interaction on each of the 6 wire pairs), QEQEA with P=4096 circuits of
    30 gates per generation; target = product of 12 random NOT/CNOT gates
    (a reversible permutation, as the paper's targets are)."""
    rng = np.random.default_rng(SEED_BASE + 6)
    return dict(name="qeqea_ising_n4_p4096_l30", n=4, lib=LIB_ISING, algorithm="qeqea", P=P, L=L,
                instances=instances, generations=100,
                target_gates=[random_target_gates(rng, 4, 12, permutation=True)
                              for _ in range(instances)],
                seed=SEED_BASE + 6)
