"""The FP64 re-check kernel of widths 4 and 5 (one or two wavefronts per
circuit over column blocks, the row map for NOT / CNOT, each chunk's gate
program read across lanes) against the oracle: both discrete libraries
(QEQEA-sampled {I, NOT, CNOT, CV, CV+} and GA genomes over {H, T, CNOT, CV,
CV+}), circuits of one, two and three chunks of 64 gates, both fitness
modes, populations whose elites do not fill the last workgroup, and a
malformed descriptor (NaN and the descriptor error flag)."""
import math

import numpy as np
import pytest
import torch

from paper_1809_11134_amd import inputs, qe

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    qe.load()
    return torch.device("cuda", 0)


def check(oracle, n, gates, f, idx, f64, T, P, k, mode=0):
    fh = f.cpu().numpy()
    gh = gates.cpu().numpy().view(np.uint16).reshape(-1, gates.shape[-1])
    idx, f64 = idx.cpu().numpy(), f64.cpu().numpy()
    for i in range(idx.shape[0]):
        fi = fh[i * P:(i + 1) * P]
        assert list(idx[i]) == sorted(range(P), key=lambda c: (-fi[c], c))[:k]
        for e in range(k):
            g = gh[i * P + idx[i, e]]
            ref = (oracle.fitness_pi if mode else oracle.fitness)(n, g, T[i])[0]
            # compare 1 - f squared: f = 1 - sqrt(q) loses digits near f = 1
            assert abs((1 - f64[i, e]) ** 2 - (1 - ref) ** 2) <= 1e-12, (i, e)
            assert abs(f64[i, e] - fi[idx[i, e]]) <= 1e-5


@pytest.mark.parametrize("n", [4, 5])
@pytest.mark.parametrize("L", [16, 70, 130])
def test_qeqea_elites(dev, oracle, n, L):
    P, I, k, seed = 24, 3, 7, 300 + 10 * n + L            # 21 elites: the last workgroup part-filled
    rng = np.random.default_rng(seed)
    T = np.stack([oracle.unitary(n, inputs.random_target_gates(rng, n, 10, permutation=True))
                  for _ in range(I)])
    ctx = qe.Context(n, qe.LIB_NCV, qe.ALG_QEQEA, L, P, I, prob_mutation=0.3,
                     mutation_range=math.pi / 4, seed=seed)
    ctx.set_targets(torch.from_numpy(T).to(dev))
    for gen in range(2):
        ctx.generation(gen)
    _, gates = ctx.sample(2)
    f = ctx.eval_population(gates)
    idx, f64 = ctx.elite_recheck(gates, f, k)
    check(oracle, n, gates, f, idx, f64, T, P, k)
    assert qe.device_errors() == 0
    ctx.close()


@pytest.mark.parametrize("n", [4, 5])
@pytest.mark.parametrize("mode", [qe.FIT_EQ11, qe.FIT_PHASE_INSENSITIVE])
def test_ga_elites_with_h_and_t(dev, oracle, n, mode):
    L, P, I, k, seed = 90, 32, 2, 9, 71 + n
    rng = np.random.default_rng(seed)
    T = np.stack([oracle.unitary(n, inputs.random_target_gates(rng, n, 8, permutation=True))
                  for _ in range(I)])
    ctx = qe.Context(n, qe.LIB_HT_NCV, qe.ALG_GA, L, P, I, seed=seed, fitness_mode=mode)
    ctx.set_targets(torch.from_numpy(T).to(dev))
    _, gates = ctx.sample(0)
    g = gates.cpu().numpy().view(np.uint16)
    assert np.isin(g & 15, [5, 6]).any()                  # H and T do occur
    f = ctx.eval_population(gates)
    idx, f64 = ctx.elite_recheck(gates, f, k)
    check(oracle, n, gates, f, idx, f64, T, P, k, mode)
    assert qe.device_errors() == 0
    ctx.close()


def test_malformed_descriptor_gives_nan(dev, oracle):
    n, L, P, I, k, seed = 5, 20, 16, 1, 16, 5
    rng = np.random.default_rng(seed)
    T = oracle.unitary(n, inputs.random_target_gates(rng, n, 6, permutation=True))[None]
    ctx = qe.Context(n, qe.LIB_NCV, qe.ALG_QEQEA, L, P, I, seed=seed)
    ctx.set_targets(torch.from_numpy(T).to(dev))
    _, gates = ctx.sample(0)
    f = torch.linspace(1.0, 0.0, P, device=dev)            # circuit c ranks c-th
    g = gates.clone()
    g[3, 5] = 0x0F3                                        # kind 3 (CV) on target 15 of 5 wires
    qe.device_errors()                                   # (reads and clears the flags)
    idx, f64 = ctx.elite_recheck(g, f, k)
    f64 = f64.cpu().numpy()[0]
    assert list(idx.cpu().numpy()[0]) == list(range(P))
    assert np.isnan(f64[3]) and not np.isnan(np.delete(f64, 3)).any()
    assert qe.device_errors() & qe.DEVERR_DESC
    ctx.close()
