"""The Ising gate model (Sec. III, Eqs. 3-6) on the GPU: fitness of angled
circuits on every path that takes them (FP32 one-element-per-lane and
LDS-staged, FP64, unitary builder, mixed widths) against the oracle, the
Table I CNOT circuit, and the QEQEA loop with the Ising library (Secs.
IV-A to IV-F) bit-exact against the oracle, teacher-forced as in the
discrete-library tests."""
import math

import numpy as np
import pytest
import torch

from paper_1809_11134_amd import inputs, qe

pytestmark = pytest.mark.gpu

RX, RY, RZ, ZZ = 7, 8, 9, 10
PI4 = float(np.pi / 4)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    qe.load()
    return torch.device("cuda", 0)


def d(kind, t=0, c=0):
    return kind | (t << 4) | (c << 8)


def perm_target(oracle, n, rng):
    return oracle.unitary(n, inputs.random_target_gates(rng, n, 12, permutation=True))


def dense_target(oracle, n, rng):
    g, a = inputs.random_ising_circuits(rng, 1, n, 10, discrete_frac=0.3)
    return oracle.unitary(n, g[0], a[0])


def angles_dev(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int32)).to(dev)


def gates_dev(g, dev):
    return torch.from_numpy(np.ascontiguousarray(g).view(np.int16)).to(dev)


# ------------------------------------------------------------------ batches
@pytest.mark.parametrize("mode", [qe.FIT_EQ11, qe.FIT_PHASE_INSENSITIVE])
@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6])
def test_angled_batch_fp32_and_fp64_match_oracle(dev, oracle, n, mode):
    rng = np.random.default_rng(700 + 10 * n + mode)
    print(f"angled batch n={n} mode={mode}", flush=True)
    for L in (1, 37, 64, 65, 150):
        B = 24
        g, a = inputs.random_ising_circuits(rng, B, n, L, discrete_frac=0.15)
        # the phase-insensitive mode is defined for permutation targets
        T = perm_target(oracle, n, rng) if mode == qe.FIT_PHASE_INSENSITIVE else dense_target(oracle, n, rng)
        ref = np.array([(oracle.fitness_pi(n, g[b], T, angles=a[b]) if mode else
                         oracle.fitness(n, g[b], T, angles=a[b]))[:2] for b in range(B)])
        for path in (qe.PATH_FP32, qe.PATH_FP32_LDS):
            f, gg, _ = qe.eval_fitness(gates_dev(g, dev), torch.from_numpy(T).to(dev), n=n, L=L,
                                       path=path, want_g=True, fitness_mode=mode,
                                       angles=angles_dev(a, dev))
            assert np.abs(f.cpu().numpy() - ref[:, 0]).max() <= 1e-5, (L, path)
            assert np.abs(gg.cpu().numpy() - ref[:, 1]).max() <= 1e-5, (L, path)
        f64, g64, _ = qe.eval_fitness_fp64(gates_dev(g, dev), torch.from_numpy(T).to(dev), n=n, L=L,
                                           want_g=True, fitness_mode=mode, angles=angles_dev(a, dev))
        assert np.abs(f64.cpu().numpy() - ref[:, 0]).max() <= 1e-12, L
        assert np.abs(g64.cpu().numpy() - ref[:, 1]).max() <= 1e-12, L
    assert qe.device_errors() == 0


@pytest.mark.parametrize("n", [2, 4, 5, 6])
def test_angled_unitaries_match_oracle(dev, oracle, n):
    rng = np.random.default_rng(910 + n)
    B, L = 6, 70
    g, a = inputs.random_ising_circuits(rng, B, n, L, discrete_frac=0.2)
    for precision, tol in ((1, 1e-12), (0, 1e-5)):
        U = qe.build_unitary(gates_dev(g, dev), n, L, precision=precision,
                             angles=angles_dev(a, dev)).cpu().numpy()
        for b in range(B):
            assert np.abs(U[b] - oracle.unitary(n, g[b], a[b])).max() <= tol, (precision, b)


def test_angled_mixed_widths_and_lengths(dev, oracle):
    rng = np.random.default_rng(77)
    nq, goff, gl, al, toff, tl, singles = [], [0], [], [], [], [], []
    off = 0
    for b in range(40):
        n = int(rng.integers(1, 7))
        L = int(rng.choice([0, 1, 5, 63, 64, 65, 130]))
        g, a = inputs.random_ising_circuits(rng, 1, n, L, discrete_frac=0.2)
        T = dense_target(oracle, n, rng)
        nq.append(n); gl.append(g[0]); al.append(a[0]); goff.append(goff[-1] + L)
        toff.append(off); tl.append(T.ravel()); off += T.size
        singles.append((n, g[0], a[0], T))
    G = np.concatenate(gl).astype(np.uint16)
    A = np.concatenate(al).astype(np.uint32)
    Tf = torch.from_numpy(np.concatenate(tl)).to(dev)
    f, _, _ = qe.eval_fitness(gates_dev(G, dev), Tf, nq=torch.tensor(nq, dtype=torch.int8, device=dev),
                              goff=torch.tensor(goff, dtype=torch.int32, device=dev),
                              toff=torch.tensor(toff, dtype=torch.int64, device=dev), target_stride=None,
                              angles=angles_dev(A, dev))
    ref = np.array([oracle.fitness(n, g, T, angles=a)[0] for n, g, a, T in singles])
    assert np.abs(f.cpu().numpy() - ref).max() <= 1e-5
    assert qe.device_errors() == 0


def test_angled_batches_rejected_where_unsupported(dev, oracle):
    n, L = 5, 8
    g, a = inputs.random_ising_circuits(np.random.default_rng(3), 4, n, L)
    T = torch.from_numpy(perm_target(oracle, n, np.random.default_rng(4))).to(dev)
    for path in (qe.PATH_FP32_REG, qe.PATH_MFMA_BF16, qe.PATH_MFMA_FP16):
        with pytest.raises(qe.QeError) as e:
            qe.eval_fitness(gates_dev(g, dev), T, n=n, L=L, path=path, angles=angles_dev(a, dev))
        assert e.value.status == qe.QE_ERR_UNSUPPORTED
    # Ising kinds without angles are malformed descriptors: NaN and the flag
    qe.device_errors()
    f, _, _ = qe.eval_fitness(gates_dev(g, dev), T, n=n, L=L)
    assert torch.isnan(f).all()
    assert qe.device_errors() & qe.DEVERR_DESC


def test_table1_circuit_on_the_gpu(dev, oracle):
    # R_1y(pi/2) J_12(3 pi/2) R_1x(3 pi/2) against CNOT (target wire 0):
    # phase-insensitive fitness 1, Eq. 11 1 - sqrt(1/2) (|tr| = 2)
    g = np.array([[d(RY, 0), d(ZZ, 0, 1), d(RX, 0)]], np.uint16)
    a = np.array([[1 << 30, 3 << 30, 3 << 30]], np.uint32)
    T = np.zeros((4, 4), complex)
    for i in range(4):
        T[i ^ ((i & 1) << 1), i] = 1
    Td = torch.from_numpy(T).to(dev)
    f, gg, _ = qe.eval_fitness(gates_dev(g, dev), Td, n=2, L=3, want_g=True,
                               fitness_mode=qe.FIT_PHASE_INSENSITIVE, angles=angles_dev(a, dev))
    assert abs(float(f[0]) - 1.0) <= 1e-5 and abs(float(gg[0]) - 1.0) <= 1e-5
    f, gg, _ = qe.eval_fitness(gates_dev(g, dev), Td, n=2, L=3, want_g=True, angles=angles_dev(a, dev))
    assert abs(float(f[0]) - (1 - math.sqrt(0.5))) <= 1e-5 and abs(float(gg[0]) - 0.5) <= 1e-6


# -------------------------------------------------------------------- QEQEA
def ising_ctx(dev, oracle, n, L, P, I, seed, pm=0.3, mode=qe.FIT_EQ11):
    ctx = qe.Context(n, qe.LIB_ISING, qe.ALG_QEQEA, L, P, I, prob_mutation=pm,
                     mutation_range=PI4, seed=seed, fitness_mode=mode)
    rng = np.random.default_rng(seed)
    T = np.stack([perm_target(oracle, n, rng) for _ in range(I)])
    ctx.set_targets(torch.from_numpy(T).to(dev))
    return ctx, T


def gpu_state(ctx):
    torch.cuda.synchronize()
    return {k: ctx.state(k).cpu().numpy() for k in ("theta", "qutrit", "best_f", "best_theta",
                                                    "best_qutrit")}


def to_oracle(oracle, ctx, st):
    o = oracle.QeqeaState(ctx.n, ctx.L, ctx.P, ctx.I, ctx.problem.seed, library=oracle.LIB_ISING)
    o.theta[:] = st["theta"].view(np.uint32)
    o.qutrit[:] = st["qutrit"]
    o.best_f[:] = st["best_f"]
    o.best_theta[:] = st["best_theta"].view(np.uint32)
    o.best_qutrit[:] = st["best_qutrit"]
    return o


def assert_same_state(o, st):
    assert np.array_equal(o.theta, st["theta"].view(np.uint32))
    assert np.array_equal(o.best_theta, st["best_theta"].view(np.uint32))
    assert np.array_equal(o.best_f.view(np.uint32), st["best_f"].view(np.uint32))
    assert np.array_equal(o.qutrit.view(np.uint32), st["qutrit"].view(np.uint32))
    assert np.array_equal(o.best_qutrit.view(np.uint32), st["best_qutrit"].view(np.uint32))


def oracle_f(oracle, n, P, T, rg, ra, mode):
    fn = oracle.fitness_pi if mode == qe.FIT_PHASE_INSENSITIVE else oracle.fitness
    return np.array([fn(n, rg[c], T[c // P], angles=ra[c])[0] for c in range(len(rg))])


@pytest.mark.parametrize("n", [2, 3, 4, 5, 6])
def test_ising_init_and_sampling_bitexact(dev, oracle, n):
    L, P, I, seed = 13, 24, 3, 5151 + n
    ctx, _ = ising_ctx(dev, oracle, n, L, P, I, seed)
    o = oracle.QeqeaState(n, L, P, I, seed, library=oracle.LIB_ISING)
    R = n + n * (n - 1) // 2
    assert ctx.state("theta").numel() == I * R * L * P
    assert_same_state(o, gpu_state(ctx))
    for gen in (0, 1, 7, 2 ** 31 + 5):
        slots, gates, angles = ctx.sample(gen)
        rs, rg, ra = o.sample(gen, with_angles=True)
        assert np.array_equal(slots.cpu().numpy().view(np.uint32), rs)
        assert np.array_equal(gates.cpu().numpy().view(np.uint16), rg)
        assert np.array_equal(angles.cpu().numpy().view(np.uint32), ra)


@pytest.mark.parametrize("n", [2, 3, 4, 5, 6])
def test_ising_update_teacher_forced(dev, oracle, n):
    L, P, I, seed, pm = 11, 16, 2, 8080 + n, 0.45
    ctx, T = ising_ctx(dev, oracle, n, L, P, I, seed, pm=pm)
    for gen in range(5):
        o = to_oracle(oracle, ctx, gpu_state(ctx))
        slots, gates, angles = ctx.sample(gen)
        rs, rg, ra = o.sample(gen, with_angles=True)
        assert np.array_equal(angles.cpu().numpy().view(np.uint32), ra)
        f = ctx.eval_population(gates, angles)
        fh = f.cpu().numpy()
        assert np.abs(fh - oracle_f(oracle, n, P, T, rg, ra, 0)).max() <= 1e-5
        ctx.update(gen, slots, gates, f, angles=angles)
        o.update(gen, pm, PI4, rs, fh)
        assert_same_state(o, gpu_state(ctx))


@pytest.mark.parametrize("n,L,P,mode", [(2, 3, 1, qe.FIT_PHASE_INSENSITIVE), (3, 16, 40, 0),
                                        (4, 30, 64, 0), (4, 70, 20, qe.FIT_PHASE_INSENSITIVE),
                                        (5, 40, 33, 0), (6, 129, 9, 0)])
def test_ising_fused_generation_teacher_forced(dev, oracle, n, L, P, mode):
    I, seed, pm = 2, 6262 + n + L, 0.4
    print(f"ising fused n={n} L={L} P={P} mode={mode}", flush=True)
    qe.device_errors()
    ctx, T = ising_ctx(dev, oracle, n, L, P, I, seed, pm=pm, mode=mode)
    for gen in (0, 1, 2, 2, 5, 3):
        o = to_oracle(oracle, ctx, gpu_state(ctx))
        rs, rg, ra = o.sample(gen, with_angles=True)
        fh = ctx.generation(gen).cpu().numpy()
        assert np.abs(fh - oracle_f(oracle, n, P, T, rg, ra, mode)).max() <= 1e-5, gen
        o.update(gen, pm, PI4, rs, fh)
        assert_same_state(o, gpu_state(ctx))
    assert qe.device_errors() == 0


@pytest.mark.parametrize("n", [3, 5])
def test_ising_sample_eval_graph_and_best(dev, oracle, n):
    L, P, I, seed, G = 14, 32, 3, 7373 + n, 4
    a, T = ising_ctx(dev, oracle, n, L, P, I, seed)
    b, _ = ising_ctx(dev, oracle, n, L, P, I, seed)
    c, _ = ising_ctx(dev, oracle, n, L, P, I, seed)
    for gen in range(G):
        rs, rg, ra = a.sample(gen)                 # (before qe_sample_eval, which commits)
        slots, gates, angles, f = a.sample_eval(gen)
        assert torch.equal(slots, rs) and torch.equal(gates, rg) and torch.equal(angles, ra)
        a.update(gen, slots, gates, f, angles=angles)
        assert torch.equal(f, b.generation(gen))
    hist = torch.empty((G, I * P), dtype=torch.float32, device=dev)
    c.run_graph(0, G, hist)
    torch.cuda.synchronize()
    sa, sb, sc = gpu_state(a), gpu_state(b), gpu_state(c)
    for k in sa:
        assert np.array_equal(sa[k], sb[k]) and np.array_equal(sa[k], sc[k]), k
    # best circuit ever: its gates and angles reproduce its fitness
    for inst in range(I):
        gates, f32, f64, angles = b.get_best(inst, with_angles=True)
        ref = oracle.fitness(n, gates, T[inst], angles=angles)[0]
        assert abs(f32 - ref) <= 1e-5 and abs(f64 - ref) <= 1e-12
    # FP64 elite re-check of the last generation, internal and explicit
    fl = b.generation(G)
    idx, f64 = b.elite_recheck(None, fl, 4)
    o = to_oracle(oracle, a, sa)
    _, rg, ra = o.sample(G, with_angles=True)
    for inst in range(I):
        for e in range(4):
            k = int(idx[inst, e])
            ref = oracle.fitness(n, rg[inst * P + k], T[inst], angles=ra[inst * P + k])[0]
            assert abs(float(f64[inst, e]) - ref) <= 1e-12
    slots, gates, angles = a.sample(G)
    fa = a.eval_population(gates, angles)
    idx2, f64b = a.elite_recheck(gates, fa, 4, angles=angles)
    for inst in range(I):
        for e in range(4):
            k = int(idx2[inst, e])
            ref = oracle.fitness(n, rg[inst * P + k], T[inst], angles=ra[inst * P + k])[0]
            assert abs(float(f64b[inst, e]) - ref) <= 1e-12


def test_ising_checkpoint_resume_and_argument_checks(dev, oracle):
    n, L, P, I, seed = 3, 9, 16, 2, 99
    a, _ = ising_ctx(dev, oracle, n, L, P, I, seed)
    for gen in range(3):
        a.generation(gen)
    blob = a.checkpoint()
    b, _ = ising_ctx(dev, oracle, n, L, P, I, seed)
    b.restore(blob)
    for gen in range(3, 6):
        assert torch.equal(a.generation(gen), b.generation(gen))
    assert a.get_best(1, with_angles=True) == b.get_best(1, with_angles=True)
    # the Ising library needs its angle buffers; the GA has no angles
    slots, gates, angles = a.sample(6)
    for fn, args in (("qe_sample", (a.handle, 6, qe._ptr(slots), qe._ptr(gates), None, None)),
                     ("qe_eval_population", (a.handle, qe._ptr(gates), None, qe._ptr(slots), None))):
        with pytest.raises(qe.QeError) as e:
            qe._call(fn, *args)
        assert e.value.status == qe.QE_ERR_INVALID
    with pytest.raises(qe.QeError) as e:
        qe.Context(n, qe.LIB_ISING, qe.ALG_GA, L, P, 1)
    assert e.value.status == qe.QE_ERR_UNSUPPORTED
