"""The MFMA path (fused 4-wire gate blocks, bf16/fp16 hi+lo, FP32
accumulation) against the CPU oracle.  Its error is stated rather than
bounded by the FP32 tolerance of 1e-5; the bounds here are about ten times
the largest error measured on MI355X over these cases and the n=6 benchmark
batch (|df|: bf16 1.3e-6, bf16 without renormalisation 1.7e-6, fp16 1.1e-7,
fp16 without renormalisation 2.0e-7), so a regression in the split products
or the renormalisation shows, and the fp16 variant must be the more
accurate one."""
import numpy as np
import pytest
import torch

from paper_1809_11134_amd import inputs, qe

pytestmark = pytest.mark.gpu
MFMA_PATHS = [qe.PATH_MFMA_BF16, qe.PATH_MFMA_FP16, qe.PATH_MFMA_BF16_RAW, qe.PATH_MFMA_FP16_RAW]
# (bound on |df|, bound on |dg|) per path
BOUNDS = {qe.PATH_MFMA_BF16: (2e-5, 1e-5), qe.PATH_MFMA_BF16_RAW: (2e-5, 1e-5),
          qe.PATH_MFMA_FP16: (3e-6, 2e-6), qe.PATH_MFMA_FP16_RAW: (3e-6, 2e-6)}


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    qe.load()
    return torch.device("cuda", 0)


def run(oracle, dev, n, gates, T, path):
    B, L = gates.shape
    f, g, _ = qe.eval_fitness(torch.from_numpy(gates.astype(np.int16)).to(dev),
                              torch.from_numpy(T).to(dev), n=n, L=L, target_stride=0, path=path,
                              want_g=True)
    ref = oracle.eval_batch(np.full(B, n, np.int8), np.arange(B + 1, dtype=np.int32) * L,
                            gates.ravel(), np.zeros(B, np.int64), T)
    return f.cpu().numpy().astype(np.float64), g.cpu().numpy().astype(np.float64), ref


@pytest.mark.parametrize("n", [5, 6])
@pytest.mark.parametrize("L", [1, 7, 48, 70])
def test_mfma_close_to_oracle(dev, oracle, n, L):
    rng = np.random.default_rng(40 + n + L)
    B = 40
    tg = inputs.random_target_gates(rng, n, 24, 1)
    gates = np.concatenate([inputs.random_circuits(rng, B // 2, n, L, 1),
                            inputs.planted_population(rng, tg, B // 2, n, L, 1, max_edits=3)])
    T = oracle.unitary(n, tg)
    print(f"n={n} L={L}", flush=True)
    errs = {}
    for path in MFMA_PATHS:
        f, g, ref = run(oracle, dev, n, gates, T, path)
        errs[path] = (np.abs(f - ref[:, 0]).max(), np.abs(g - ref[:, 1]).max())
        assert np.all(np.isfinite(f))
        assert errs[path][0] <= BOUNDS[path][0], (path, errs[path])
        assert errs[path][1] <= BOUNDS[path][1], (path, errs[path])
    assert errs[qe.PATH_MFMA_FP16][1] <= errs[qe.PATH_MFMA_BF16][1] + 1e-6
    assert qe.device_errors() == 0


def test_mfma_single_block_exact_permutations(dev, oracle):
    # NOT/CNOT circuits on the first 4 wires are permutation blocks: every
    # hi+lo product is exact, so the MFMA result matches the oracle closely
    rng = np.random.default_rng(3)
    n, L, B = 6, 12, 16
    perm = np.array([d for d in inputs.permutation_gates(n)
                     if ((d >> 4) & 15) < 4 and (((d & 15) == 1) or ((d >> 8) & 15) < 4)], np.uint16)
    gates = perm[rng.integers(0, len(perm), (B, L))]
    T = oracle.unitary(n, gates[0])
    for path in MFMA_PATHS:
        f, g, ref = run(oracle, dev, n, gates, T, path)
        assert np.abs(f - ref[:, 0]).max() <= 1e-5
        assert f[0] == pytest.approx(1.0, abs=1e-6)


def test_mfma_rejects_other_widths(dev):
    T = torch.eye(16, dtype=torch.complex64, device=dev)
    g = torch.zeros((2, 3), dtype=torch.int16, device=dev)
    with pytest.raises(qe.QeError) as e:
        qe.eval_fitness(g, T, n=4, L=3, path=qe.PATH_MFMA_BF16)
    assert e.value.status == qe.QE_ERR_UNSUPPORTED


@pytest.mark.parametrize("n", [5, 6])
@pytest.mark.parametrize("min_block", [1, 3, 65])
def test_mfma_block_threshold(dev, oracle, n, min_block):
    """Groups of fewer than min_block gates go gate by gate in FP32 (65: every
    group, 1: none); the results stay within the path's bounds, circuits of
    two descriptor chunks included."""
    saved = {c: qe.get_mfma_min_block(n, c) for c in (0, 1)}
    try:
        for c in (0, 1):
            qe.set_mfma_min_block(n, c, min_block)
        for L in (7, 70):
            rng = np.random.default_rng(900 + 10 * n + L + min_block)
            B = 24
            tg = inputs.random_target_gates(rng, n, 24, 1)
            gates = np.concatenate([inputs.random_circuits(rng, B // 2, n, L, 1),
                                    inputs.planted_population(rng, tg, B // 2, n, L, 1, max_edits=3)])
            T = oracle.unitary(n, tg)
            for path in (qe.PATH_MFMA_BF16, qe.PATH_MFMA_FP16):
                f, g, ref = run(oracle, dev, n, gates, T, path)
                assert np.all(np.isfinite(f))
                assert np.abs(f - ref[:, 0]).max() <= BOUNDS[path][0], (L, path)
                assert np.abs(g - ref[:, 1]).max() <= BOUNDS[path][1], (L, path)
                if min_block == 65:        # no block at all: the FP32 per-gate error
                    assert np.abs(f - ref[:, 0]).max() <= 1e-5
        assert qe.device_errors() == 0
    finally:
        for c, v in saved.items():
            qe.set_mfma_min_block(n, c, v)
