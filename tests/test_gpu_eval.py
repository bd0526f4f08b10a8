"""Parity of the HIP fitness kernels (Eq. 11) with the CPU oracle, element by
element, through the C ABI.  Tolerance: |df| <= 1e-5 and |dg| <= 1e-5 on the
FP32 paths, 1e-12 on the FP64 path."""
import itertools

import numpy as np
import pytest
import torch

from paper_1809_11134_amd import inputs, qe

pytestmark = pytest.mark.gpu

TOL32 = 1e-5
TOL64 = 1e-12
FP32_PATHS = [qe.PATH_FP32, qe.PATH_FP32_REG, qe.PATH_FP32_LDS]


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    qe.load()
    return torch.device("cuda", 0)


def oracle_batch(oracle, n, gates, T):
    B, L = gates.shape
    return oracle.eval_batch(np.full(B, n, np.int8), np.arange(B + 1, dtype=np.int32) * L,
                             gates.ravel(), np.zeros(B, np.int64), T)


def t16(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a).astype(np.int16)).to(dev)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6])
@pytest.mark.parametrize("lib", [0, 1])
@pytest.mark.parametrize("L", [1, 17, 64, 65, 150])
def test_fp32_paths_match_oracle(dev, oracle, n, lib, L):
    rng = np.random.default_rng(1000 * n + 10 * lib + L)
    B = 70                                     # 17 workgroups of 4 circuits + a ragged tail
    gates = inputs.random_circuits(rng, B, n, L, lib)
    T = oracle.unitary(n, inputs.random_target_gates(rng, n, 10, lib))
    ref = oracle_batch(oracle, n, gates, T)
    print(f"n={n} lib={lib} L={L} B={B}", flush=True)
    for path in FP32_PATHS:
        f, g, d = qe.eval_fitness(t16(gates, dev), torch.from_numpy(T).to(dev), n=n, L=L,
                                  target_stride=0, path=path, want_g=True, want_delta=True)
        f, g, d = (x.cpu().numpy().astype(np.float64) for x in (f, g, d))
        assert np.abs(f - ref[:, 0]).max() <= TOL32, (path, np.abs(f - ref[:, 0]).max())
        assert np.abs(g - ref[:, 1]).max() <= TOL32, path
        assert np.abs(d - ref[:, 2]).max() <= TOL32 * (1 << n), path
    assert qe.device_errors() == 0


@pytest.mark.parametrize("n", [2, 3, 4, 5, 6])
def test_near_solutions(dev, oracle, n):
    # planted circuits: the target's own gates with a few edits, so f spans
    # (0, 1] including exact solutions where the square root is steepest
    rng = np.random.default_rng(77 + n)
    L = 40
    tg = inputs.random_target_gates(rng, n, 30, 1)
    T = oracle.unitary(n, tg)
    gates = inputs.planted_population(rng, tg, 96, n, L, 1, max_edits=3)
    ref = oracle_batch(oracle, n, gates, T)
    assert (ref[:, 0] > 1 - 1e-9).sum() > 3
    for path in FP32_PATHS:
        f, g, _ = qe.eval_fitness(t16(gates, dev), torch.from_numpy(T).to(dev), n=n, L=L,
                                  target_stride=0, path=path, want_g=True)
        f = f.cpu().numpy().astype(np.float64)
        assert np.abs(f - ref[:, 0]).max() <= TOL32, (path, np.abs(f - ref[:, 0]).max())
        assert np.all((f >= 0) & (f <= 1))


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6])
def test_fp64_matches_oracle(dev, oracle, n):
    rng = np.random.default_rng(500 + n)
    L, B = 50, 20
    gates = inputs.random_circuits(rng, B, n, L, 1)
    gates[:5] = inputs.planted_population(rng, gates[5], 5, n, L, 1, max_edits=1)
    T = oracle.unitary(n, gates[5])
    ref = oracle_batch(oracle, n, gates, T)
    f, g, d = qe.eval_fitness_fp64(t16(gates, dev), torch.from_numpy(T).to(dev), n=n, L=L,
                                   target_stride=0, want_g=True, want_delta=True)
    f, g, d = (x.cpu().numpy() for x in (f, g, d))
    rad = (1 - f) ** 2
    assert np.abs(rad - (1 - ref[:, 0]) ** 2).max() <= TOL64
    assert np.abs(g - ref[:, 1]).max() <= TOL64
    assert np.abs(d - ref[:, 2]).max() <= TOL64 * (1 << n)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6])
@pytest.mark.parametrize("precision", [0, 1])
def test_build_unitary(dev, oracle, n, precision):
    rng = np.random.default_rng(900 + n)
    L, B = 33, 9
    gates = inputs.random_circuits(rng, B, n, L, 1)
    U = qe.build_unitary(t16(gates, dev), n, L, precision=precision).cpu().numpy()
    tol = 1e-5 if precision == 0 else 1e-12
    for b in range(B):
        assert np.abs(U[b] - oracle.unitary(n, gates[b])).max() <= tol


def test_uneven_batch_per_circuit_targets(dev, oracle):
    w = inputs.workload_uneven(count=300, per_population=7, seed_offset=40)
    nq, goff, gates = w["nq"], w["goff"], w["gates"]
    tmats = [oracle.unitary(n, tg) for n, tg in w["target_gates"]]
    toff_pop = np.cumsum([0] + [m.size for m in tmats])[:-1]
    toff = toff_pop[w["target_index"]].astype(np.int64)
    flat = np.concatenate([m.ravel() for m in tmats])
    ref = oracle.eval_batch(nq, goff, gates, toff, flat)
    print(f"uneven: {len(nq)} circuits, widths {sorted(set(nq.tolist()))}", flush=True)
    for path in FP32_PATHS:
        f, g, _ = qe.eval_fitness(t16(gates, dev), torch.from_numpy(flat).to(dev),
                                  nq=torch.from_numpy(nq).to(dev), goff=torch.from_numpy(goff).to(dev),
                                  toff=torch.from_numpy(toff).to(dev), target_stride=None,
                                  path=path, want_g=True)
        assert np.abs(f.cpu().numpy() - ref[:, 0]).max() <= TOL32, path
        assert np.abs(g.cpu().numpy() - ref[:, 1]).max() <= TOL32, path
    assert qe.device_errors() == 0


def test_per_circuit_target_stride(dev, oracle):
    rng = np.random.default_rng(31)
    n, L, B = 5, 24, 40
    gates = inputs.random_circuits(rng, B, n, L, 0)
    Ts = np.stack([oracle.unitary(n, inputs.random_target_gates(rng, n, 6, permutation=True))
                   for _ in range(B)])
    ref = np.array([oracle.fitness(n, gates[b], Ts[b]) for b in range(B)])
    f, _, _ = qe.eval_fitness(t16(gates, dev), torch.from_numpy(Ts).to(dev), n=n, L=L,
                              target_stride=(1 << n) ** 2)
    assert np.abs(f.cpu().numpy() - ref[:, 0]).max() <= TOL32


def test_brute_force_n3_batch(dev, oracle):
    # all 22^3 length-3 circuits of {I,NOT,CNOT,CV,CV+} on 3 wires vs Toffoli
    tab = oracle.lib_table(0, 3)
    seqs = np.array(list(itertools.product(range(22), repeat=3)))
    gates = tab[seqs]
    T = np.zeros((8, 8), complex)
    for i in range(8):
        c, a, b = (i >> 2) & 1, (i >> 1) & 1, i & 1
        T[((c ^ (a & b)) << 2) | (a << 1) | b, i] = 1
    ref = oracle_batch(oracle, 3, gates, T)
    f, _, _ = qe.eval_fitness(t16(gates, dev), torch.from_numpy(T).to(dev), n=3, L=3, target_stride=0)
    f = f.cpu().numpy()
    assert np.abs(f - ref[:, 0]).max() <= TOL32
    assert int(np.argmax(f)) == int(np.argmax(ref[:, 0]))


def test_edge_cases(dev, oracle):
    T = torch.eye(8, dtype=torch.complex64, device=dev)
    # empty batch
    f, _, _ = qe.eval_fitness(torch.zeros((0, 4), dtype=torch.int16, device=dev), T, n=3, L=4)
    assert f.numel() == 0
    # identity circuit (all I) and zero-length circuits through offsets
    f, _, _ = qe.eval_fitness(torch.zeros((3, 5), dtype=torch.int16, device=dev), T, n=3, L=5)
    assert torch.allclose(f.cpu(), torch.ones(3))
    goff = torch.tensor([0, 0, 2, 2], dtype=torch.int32, device=dev)
    g = torch.tensor([1 | (1 << 4), 1 | (1 << 4)], dtype=torch.int16, device=dev)   # NOT NOT
    f, _, _ = qe.eval_fitness(g, T, n=3, goff=goff)
    assert torch.allclose(f.cpu(), torch.ones(3))
    assert qe.device_errors() == 0


def test_malformed_device_data_flags(dev):
    T = torch.eye(16, dtype=torch.complex64, device=dev)
    bad = torch.tensor([[2 | (1 << 4) | (1 << 8)], [0]], dtype=torch.int16, device=dev)  # control == target
    for path in FP32_PATHS:
        f, _, _ = qe.eval_fitness(bad, T, n=4, L=1, path=path)
        f = f.cpu()
        assert torch.isnan(f[0]) and f[1] == 1
        assert qe.device_errors() & qe.DEVERR_DESC
    # width out of range in a mixed batch, and offsets beyond the buffers
    nq = torch.tensor([4, 9], dtype=torch.int8, device=dev)
    goff = torch.tensor([0, 1, 1], dtype=torch.int32, device=dev)
    toff = torch.tensor([0, 0], dtype=torch.int64, device=dev)
    f, _, _ = qe.eval_fitness(bad[1], T, nq=nq, goff=goff, toff=toff, target_stride=None)
    f = f.cpu()
    assert f[0] == 1 and torch.isnan(f[1])
    assert qe.device_errors() & qe.DEVERR_WIDTH
    goff = torch.tensor([0, 5], dtype=torch.int32, device=dev)
    f, _, _ = qe.eval_fitness(bad[1], T, n=4, goff=goff)
    assert torch.isnan(f.cpu()[0])
    assert qe.device_errors() & qe.DEVERR_RANGE
    toff = torch.tensor([10], dtype=torch.int64, device=dev)
    f, _, _ = qe.eval_fitness(bad[1:], T, n=4, L=1, toff=toff, target_stride=None)
    assert torch.isnan(f.cpu()[0])
    assert qe.device_errors() & qe.DEVERR_RANGE
    assert qe.device_errors() == 0


def test_deterministic(dev, oracle):
    rng = np.random.default_rng(5)
    gates = inputs.random_circuits(rng, 256, 6, 48, 1)
    T = torch.from_numpy(oracle.unitary(6, gates[0])).to(dev)
    g = t16(gates, dev)
    for path in FP32_PATHS:
        a = qe.eval_fitness(g, T, n=6, L=48, path=path)[0]
        b = qe.eval_fitness(g, T, n=6, L=48, path=path)[0]
        assert torch.equal(a, b)
