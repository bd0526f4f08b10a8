"""Parity of the phase-insensitive fitness mode (QE_FIT_PHASE_INSENSITIVE)
with the oracle's phase-insensitive fitness, element by element through the
C ABI, on permutation targets (the paper's kind of target) and on every path;
then the QEQEA and GA loops run in that mode, teacher-forced against the
oracle."""
import numpy as np
import pytest
import torch

from paper_1809_11134_amd import inputs, qe

pytestmark = pytest.mark.gpu

TOL32 = 1e-5
TOL64 = 1e-12
PI = qe.FIT_PHASE_INSENSITIVE
FP32_PATHS = [qe.PATH_FP32, qe.PATH_FP32_REG, qe.PATH_FP32_LDS]


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    qe.load()
    return torch.device("cuda", 0)


def t16(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a).astype(np.int16)).to(dev)


def perm_gates(rng, n, count=12):
    return inputs.random_target_gates(rng, n, count, lib=0, permutation=True)


def oracle_pi(oracle, n, gates, T):
    return np.array([oracle.fitness_pi(n, g, T) for g in gates])


def population(rng, n, lib, B, L, tg):
    """Half uniform circuits, half the target's gate list with a few edits
    (so that f reaches 1 exactly and spans the range near it)."""
    a = inputs.random_circuits(rng, B // 2, n, L, lib)
    b = inputs.planted_population(rng, tg, B - B // 2, n, L, lib, max_edits=2)
    return np.concatenate([a, b])


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6])
@pytest.mark.parametrize("lib", [0, 1])
@pytest.mark.parametrize("L", [17, 65])
def test_fp32_paths_match_oracle(dev, oracle, n, lib, L):
    rng = np.random.default_rng(600 + 100 * n + 10 * lib + L)
    B = 70
    tg = perm_gates(rng, n)
    T = oracle.unitary(n, tg)
    gates = population(rng, n, lib, B, L, tg)
    ref = oracle_pi(oracle, n, gates, T)
    print(f"n={n} lib={lib} L={L}", flush=True)
    for path in FP32_PATHS:
        f, g, d = qe.eval_fitness(t16(gates, dev), torch.from_numpy(T).to(dev), n=n, L=L,
                                  target_stride=0, path=path, want_g=True, want_delta=True,
                                  fitness_mode=PI)
        f, g, d = (x.cpu().numpy().astype(np.float64) for x in (f, g, d))
        assert np.abs(f - ref[:, 0]).max() <= TOL32, (path, np.abs(f - ref[:, 0]).max())
        assert np.abs(g - ref[:, 1]).max() <= TOL32, path
        assert np.abs(d - ref[:, 2] * (1 << n)).max() <= TOL32 * (1 << n), path
    assert qe.device_errors() == 0


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6])
def test_fp64_matches_oracle(dev, oracle, n):
    rng = np.random.default_rng(700 + n)
    L = 30
    tg = perm_gates(rng, n)
    T = oracle.unitary(n, tg)
    gates = population(rng, n, 1, 40, L, tg)
    ref = oracle_pi(oracle, n, gates, T)
    f, g, _ = qe.eval_fitness_fp64(t16(gates, dev), torch.from_numpy(T).to(dev), n=n, L=L,
                                   target_stride=0, want_g=True, fitness_mode=PI)
    assert np.abs(f.cpu().numpy() - ref[:, 0]).max() <= TOL64
    assert np.abs(g.cpu().numpy() - ref[:, 1]).max() <= TOL64


def test_mixed_widths_one_launch(dev, oracle):
    rng = np.random.default_rng(801)
    nq, goff, gates, toff, mats = [], [0], [], [], []
    off = 0
    for p in range(24):
        n = int(rng.integers(1, 7))
        T = oracle.unitary(n, perm_gates(rng, n))
        mats.append(T.ravel())
        for _ in range(5):
            L = int(rng.integers(4, 70))
            gates.append(inputs.random_circuits(rng, 1, n, L, 1)[0])
            goff.append(goff[-1] + L)
            nq.append(n)
            toff.append(off)
        off += T.size
    nq, goff, toff = np.array(nq, np.int8), np.array(goff, np.int32), np.array(toff, np.int64)
    flat = np.concatenate(mats)
    gl = np.concatenate(gates).astype(np.uint16)
    ref = np.array([oracle.fitness_pi(int(nq[b]), gl[goff[b]:goff[b + 1]],
                                      flat[toff[b]:toff[b] + (1 << (2 * int(nq[b])))].reshape(
                                          1 << int(nq[b]), 1 << int(nq[b])))
                    for b in range(len(nq))])
    for path in FP32_PATHS:
        f, _, _ = qe.eval_fitness(t16(gl, dev), torch.from_numpy(flat).to(dev),
                                  nq=torch.from_numpy(nq).to(dev), goff=torch.from_numpy(goff).to(dev),
                                  toff=torch.from_numpy(toff).to(dev), target_stride=None, path=path,
                                  fitness_mode=PI)
        assert np.abs(f.cpu().numpy() - ref[:, 0]).max() <= TOL32, path
    assert qe.device_errors() == 0


@pytest.mark.parametrize("n", [5, 6])
def test_mfma_paths(dev, oracle, n):
    # the fused-block paths in this mode: error stated (printed), bounded
    # loosely (BF16 / FP16 operands with hi+lo splitting)
    rng = np.random.default_rng(900 + n)
    L = 48
    tg = perm_gates(rng, n)
    T = oracle.unitary(n, tg)
    gates = population(rng, n, 1, 64, L, tg)
    ref = oracle_pi(oracle, n, gates, T)
    for path in (qe.PATH_MFMA_BF16, qe.PATH_MFMA_FP16, qe.PATH_MFMA_BF16_RAW, qe.PATH_MFMA_FP16_RAW):
        f, _, _ = qe.eval_fitness(t16(gates, dev), torch.from_numpy(T).to(dev), n=n, L=L,
                                  target_stride=0, path=path, fitness_mode=PI)
        err = np.abs(f.cpu().numpy() - ref[:, 0]).max()
        print(f"n={n} path={path} max |df| = {err:.3g}", flush=True)
        assert err <= 1e-4, (path, err)


@pytest.mark.parametrize("n", [3, 4, 5])
def test_qeqea_teacher_forced(dev, oracle, n):
    L, P, I, seed, pm = 14, 36, 2, 2020 + n, 0.4
    rng = np.random.default_rng(seed)
    T = np.stack([oracle.unitary(n, perm_gates(rng, n)) for _ in range(I)])
    ctx = qe.Context(n, qe.LIB_NCV, qe.ALG_QEQEA, L, P, I, prob_mutation=pm,
                     mutation_range=float(np.pi / 4), seed=seed, fitness_mode=PI)
    ctx.set_targets(torch.from_numpy(T).to(dev))
    keys = ("theta", "qutrit", "best_f", "best_theta", "best_qutrit")
    for gen in range(4):
        torch.cuda.synchronize()
        st = {k: ctx.state(k).cpu().numpy() for k in keys}
        o = oracle.QeqeaState(n, L, P, I, seed)
        o.theta[:] = st["theta"].view(np.uint32)
        o.qutrit[:] = st["qutrit"]
        o.best_f[:] = st["best_f"]
        o.best_theta[:] = st["best_theta"].view(np.uint32)
        o.best_qutrit[:] = st["best_qutrit"]
        rs, rg = o.sample(gen)
        f = ctx.generation(gen)
        fh = f.cpu().numpy()
        ref = np.array([oracle.fitness_pi(n, rg[c], T[c // P])[0] for c in range(I * P)])
        assert np.abs(fh - ref).max() <= TOL32, gen
        o.update(gen, pm, float(np.pi / 4), rs, fh)
        torch.cuda.synchronize()
        assert np.array_equal(o.theta, ctx.state("theta").cpu().numpy().view(np.uint32))
        assert np.array_equal(o.best_f.view(np.uint32), ctx.state("best_f").cpu().numpy().view(np.uint32))
    gates, f32, f64 = ctx.get_best(0)
    assert abs(f64 - oracle.fitness_pi(n, gates, T[0])[0]) <= TOL64
    ctx.close()


def test_ga_eval_population(dev, oracle):
    n, L, P, seed = 3, 10, 64, 55
    rng = np.random.default_rng(seed)
    T = oracle.unitary(n, perm_gates(rng, n, 5))
    ctx = qe.Context(n, qe.LIB_NCV, qe.ALG_GA, L, P, 1, seed=seed, fitness_mode=PI)
    ctx.set_targets(torch.from_numpy(T[None]).to(dev))
    _, gates = ctx.sample(0)
    f = ctx.eval_population(gates).cpu().numpy()
    g = gates.cpu().numpy().view(np.uint16)
    ref = oracle_pi(oracle, n, g, T)
    assert np.abs(f - ref[:, 0]).max() <= TOL32
    ctx.close()


def test_unknown_mode_rejected(dev):
    g = torch.zeros((2, 3), dtype=torch.int16, device=dev)
    T = torch.eye(4, dtype=torch.complex64, device=dev)
    with pytest.raises(qe.QeError):
        qe.eval_fitness(g, T, n=2, L=3, fitness_mode=2)
    with pytest.raises(qe.QeError):
        qe.Context(3, qe.LIB_NCV, qe.ALG_QEQEA, 4, 8, 1, fitness_mode=7)


@pytest.mark.parametrize("n", [2, 4, 5])
def test_monomial_targets_with_phases(dev, oracle, n):
    """Targets that are permutations with phases (CNOT, NOT and T gates: every
    entry of modulus 0 or 1) are where the kernels' diagonal overlap equals
    the oracle's sum |U_ij|^2 |T_ij|^2: parity on every FP32 path and FP64."""
    rng = np.random.default_rng(900 + n)
    tab = np.concatenate([inputs.permutation_gates(n),
                          np.array([inputs.desc(inputs.T, w) for w in range(n)], np.uint16)])
    tg = tab[rng.integers(0, len(tab), 14)]
    T = oracle.unitary(n, tg)
    B, L = 40, 24
    gates = population(rng, n, 1, B, L, tg)
    ref = oracle_pi(oracle, n, gates, T)[:, 0]
    for path in FP32_PATHS:
        f, _, _ = qe.eval_fitness(t16(gates, dev), torch.from_numpy(T).to(dev), n=n, L=L,
                                  target_stride=0, path=path, fitness_mode=PI)
        assert np.abs(f.cpu().numpy().astype(np.float64) - ref).max() <= TOL32, path
    f64, _, _ = qe.eval_fitness_fp64(t16(gates, dev), torch.from_numpy(T).to(dev), n=n, L=L,
                                     target_stride=0, fitness_mode=PI)
    assert np.abs(f64.cpu().numpy() - ref).max() <= TOL64
    assert qe.device_errors() == 0


def test_other_targets_are_refused(dev, oracle):
    """A target with entries of modulus strictly between 0 and 1 (library
    {H,T,CNOT,CV,CV+}): the phase-insensitive evaluation gives NaN and
    QE_DEVERR_TARGET for its circuits (FP32 and FP64 calls), only for them;
    a context in that mode refuses such targets."""
    rng = np.random.default_rng(77)
    n, L, B = 4, 12, 8
    good = oracle.unitary(n, perm_gates(rng, n))
    bad = oracle.unitary(n, inputs.random_target_gates(rng, n, 10, lib=1))
    assert np.any((np.abs(bad) ** 2 > 1e-3) & (np.abs(bad) ** 2 < 1 - 1e-3))
    gates = inputs.random_circuits(rng, B, n, L, 1)
    targets = np.stack([good, bad])
    toff = torch.tensor([0 if b % 2 == 0 else 256 for b in range(B)], dtype=torch.int64, device=dev)
    nq = torch.full((B,), n, dtype=torch.int8, device=dev)
    goff = torch.arange(B + 1, dtype=torch.int32, device=dev) * L
    for fp64 in (False, True):
        fn = qe.eval_fitness_fp64 if fp64 else qe.eval_fitness
        f, g, d = fn(t16(gates, dev), torch.from_numpy(targets).to(dev), nq=nq, goff=goff, toff=toff,
                     target_stride=None, fitness_mode=PI, want_g=True, want_delta=True)
        fh = f.cpu().numpy()
        assert np.all(np.isnan(fh[1::2])) and np.all(np.isnan(g.cpu().numpy()[1::2]))
        assert np.all(np.isfinite(fh[0::2]))
        assert qe.device_errors() == qe.DEVERR_TARGET
    # one shared target
    f, _, _ = qe.eval_fitness(t16(gates, dev), torch.from_numpy(bad).to(dev), n=n, L=L,
                              target_stride=0, fitness_mode=PI)
    assert np.all(np.isnan(f.cpu().numpy()))
    assert qe.device_errors() == qe.DEVERR_TARGET
    # Eq. 11 takes any target
    f, _, _ = qe.eval_fitness(t16(gates, dev), torch.from_numpy(bad).to(dev), n=n, L=L, target_stride=0)
    assert np.all(np.isfinite(f.cpu().numpy()))
    assert qe.device_errors() == 0
    ctx = qe.Context(n, 0, qe.ALG_GA, L, 16, 2, seed=3, fitness_mode=PI)
    with pytest.raises(qe.QeError) as e:
        ctx.set_targets(torch.from_numpy(targets).to(dev))
    assert e.value.status == qe.QE_ERR_UNSUPPORTED
    ctx.set_targets(torch.from_numpy(np.stack([good, good])).to(dev))
    ctx.generation(0)
    torch.cuda.synchronize()
    assert qe.device_errors() == 0
    ctx.close()
