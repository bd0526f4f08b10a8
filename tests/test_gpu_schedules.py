"""Every schedule the autotuner can choose for the LDS-staged kernels --
wavefronts per circuit (width 5: one or two), circuits per workgroup of the
one-wavefront population kernels (one or four), either length class, each
library class on its own -- gives
the same fitness bit for bit (the reduction runs in an order fixed by the
width), in every kernel family: qe_eval_fitness on uniform and mixed-width
batches, the population evaluation, the fused QEQEA kernel (discrete and
Ising libraries, whose whole encoding then evolves identically) and the
mixed-population GA; the register-resident kernel agrees with them within the
FP32 tolerance, and all of them with the oracle."""
import math

import numpy as np
import pytest
import torch

from paper_1809_11134_amd import inputs, qe

pytestmark = pytest.mark.gpu
TOL32 = 1e-5
LDS_SCHEDULES = {4: [(1, 1, 4), (1, 1, 1)], 5: [(1, 1, 4), (1, 1, 1), (1, 2, 1)], 6: [(1, 4, 1)]}


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    qe.load()
    return torch.device("cuda", 0)


@pytest.fixture()
def restore_schedules():
    saved = {(n, c, k): qe.get_schedule_lib(n, c, k) for n in range(1, 7) for c in (0, 1) for k in (0, 1, 2)}
    yield
    for (n, c, k), v in saved.items():
        qe.set_schedule_lib(n, c, k, *v)


def set_all(n, sched):
    for c in (0, 1):
        qe.set_schedule_ex(n, c, *sched)


def t16(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int16)).to(dev)


@pytest.mark.parametrize("n", [4, 5, 6])
@pytest.mark.parametrize("L", [20, 48])
def test_eval_fitness_same_bits_every_schedule(dev, oracle, restore_schedules, n, L):
    rng = np.random.default_rng(70 + 10 * n + L)
    B = 96
    gates = inputs.random_circuits(rng, B, n, L, inputs.LIB_HT_NCV)
    T = oracle.unitary(n, inputs.random_target_gates(rng, n, 10, inputs.LIB_HT_NCV))
    Td = torch.from_numpy(T).to(dev)
    ref = oracle.eval_batch(np.full(B, n, np.int8), np.arange(B + 1, dtype=np.int32) * L,
                            gates.ravel(), np.zeros(B, np.int64), T)
    outs = []
    for sched in LDS_SCHEDULES[n]:
        set_all(n, sched)
        f, g, d = qe.eval_fitness(t16(gates, dev), Td, n=n, L=L, target_stride=0, want_g=True, want_delta=True)
        outs.append((sched, f, g, d))
    for sched, f, g, d in outs[1:]:
        assert torch.equal(f, outs[0][1]) and torch.equal(g, outs[0][2]) and torch.equal(d, outs[0][3]), sched
    assert np.abs(outs[0][1].cpu().numpy() - ref[:, 0]).max() <= TOL32
    fr, _, _ = qe.eval_fitness(t16(gates, dev), Td, n=n, L=L, target_stride=0, path=qe.PATH_FP32_REG)
    assert np.abs(fr.cpu().numpy() - outs[0][1].cpu().numpy()).max() <= TOL32
    assert qe.device_errors() == 0


def test_mixed_batch_same_bits_every_width5_schedule(dev, oracle, restore_schedules):
    rng = np.random.default_rng(5150)
    B = 300
    nq = rng.integers(3, 7, size=B).astype(np.int8)
    lens = rng.integers(1, 70, size=B)
    goff = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    gates = np.concatenate([inputs.random_circuits(rng, 1, int(n), int(L), 1)[0] for n, L in zip(nq, lens)])
    mats = [oracle.unitary(int(n), inputs.random_target_gates(rng, int(n), 6, 1)) for n in nq]
    toff = np.cumsum([0] + [m.size for m in mats])[:-1].astype(np.int64)
    flat = np.concatenate([m.ravel() for m in mats])
    args = dict(nq=torch.from_numpy(nq).to(dev), goff=torch.from_numpy(goff).to(dev),
                toff=torch.from_numpy(toff).to(dev), target_stride=None)
    outs = []
    for sched in LDS_SCHEDULES[5]:
        set_all(5, sched)
        for ws in (True, False):      # the sorted single launch, one launch per width
            f, _, _ = qe.eval_fitness(t16(gates, dev), torch.from_numpy(flat).to(dev), workspace=ws, **args)
            outs.append(f)
    for f in outs[1:]:
        assert torch.equal(f, outs[0])
    ref = oracle.eval_batch(nq, goff, gates, toff, flat)
    assert np.abs(outs[0].cpu().numpy() - ref[:, 0]).max() <= TOL32


@pytest.mark.parametrize("n,lib", [(4, qe.LIB_NCV), (5, qe.LIB_NCV), (4, qe.LIB_ISING), (5, qe.LIB_ISING)])
def test_qeqea_loop_same_bits_every_schedule(dev, oracle, restore_schedules, n, lib):
    L, P, I, seed = 40, 48, 3, 4000 + n + 10 * lib
    rng = np.random.default_rng(seed)
    T = np.stack([oracle.unitary(n, inputs.random_target_gates(rng, n, 10, permutation=True)) for _ in range(I)])
    runs = []
    for sched in LDS_SCHEDULES[n]:
        set_all(n, sched)
        ctx = qe.Context(n, lib, qe.ALG_QEQEA, L, P, I, prob_mutation=0.3, mutation_range=math.pi / 4,
                         seed=seed)
        ctx.set_targets(torch.from_numpy(T).to(dev))
        fs = [ctx.generation(gen).clone() for gen in range(3)]
        out = ctx.sample_eval(3)
        fe = ctx.eval_population(out[1], angles=out[2] if lib == qe.LIB_ISING else None)
        torch.cuda.synchronize()
        state = {k: ctx.state(k).cpu().numpy() for k in ("theta", "qutrit", "best_f")}
        runs.append((sched, fs, out, fe, state))
        ctx.close()
    base = runs[0]
    for sched, fs, out, fe, state in runs[1:]:
        for a, b in zip(fs, base[1]):
            assert torch.equal(a, b), sched
        for a, b in zip(out, base[2]):
            assert torch.equal(a, b), sched
        assert torch.equal(fe, base[3]) and torch.equal(fe, out[-1]), sched
        for k in state:
            assert np.array_equal(state[k].view(np.uint32), base[4][k].view(np.uint32)), (sched, k)
    assert qe.device_errors() == 0


def test_mixed_ga_same_bits_every_width5_schedule(dev, oracle, restore_schedules):
    widths, lengths, P, seed = [5, 4, 6, 5, 3], [30, 12, 20, 45, 9], 32, 61
    rng = np.random.default_rng(seed)
    T = np.concatenate([oracle.unitary(n, inputs.random_target_gates(rng, n, 8, 1)).ravel() for n in widths])
    runs = []
    for sched in LDS_SCHEDULES[5]:
        set_all(5, sched)
        ctx = qe.Context(0, qe.LIB_HT_NCV, qe.ALG_GA, 0, P, seed=seed, widths=widths, lengths=lengths)
        ctx.set_targets(torch.from_numpy(T).to(dev))
        runs.append([ctx.generation(gen).clone() for gen in range(3)])
        ctx.close()
    for r in runs[1:]:
        for a, b in zip(r, runs[0]):
            assert torch.equal(a, b)


@pytest.mark.parametrize("lib", [qe.LIB_NCV, qe.LIB_ISING])
def test_library_classes_take_own_schedules_same_bits(dev, oracle, restore_schedules, lib):
    """The sampled, discrete and Ising classes each under a schedule of their
    own (width 5): the QEQEA loop, its population re-evaluation and a batch
    evaluation keep the bits of one common schedule."""
    n, L, P, I, seed = 5, 40, 48, 2, 4321 + lib
    rng = np.random.default_rng(seed)
    T = np.stack([oracle.unitary(n, inputs.random_target_gates(rng, n, 10, permutation=True)) for _ in range(I)])
    own = {qe.SCHED_SAMPLED: (1, 2, 1), qe.SCHED_DISCRETE: (1, 1, 1), qe.SCHED_ISING: (1, 2, 1)}
    runs = []
    for per_class in (False, True):
        for c in (0, 1):
            for k in (0, 1, 2):
                qe.set_schedule_lib(n, c, k, *(own[k] if per_class else (1, 1, 4)))
        ctx = qe.Context(n, lib, qe.ALG_QEQEA, L, P, I, prob_mutation=0.3, mutation_range=math.pi / 4,
                         seed=seed)
        ctx.set_targets(torch.from_numpy(T).to(dev))
        fs = [ctx.generation(gen).clone() for gen in range(3)]
        out = ctx.sample_eval(3)
        fe = ctx.eval_population(out[1], angles=out[2] if lib == qe.LIB_ISING else None)
        torch.cuda.synchronize()
        runs.append((fs, out, fe))
        ctx.close()
    for a, b in zip(runs[0][0], runs[1][0]):
        assert torch.equal(a, b)
    for a, b in zip(runs[0][1], runs[1][1]):
        assert torch.equal(a, b)
    assert torch.equal(runs[0][2], runs[1][2]) and torch.equal(runs[1][2], runs[1][1][-1])
    assert qe.device_errors() == 0
