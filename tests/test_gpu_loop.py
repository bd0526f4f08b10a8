"""Bit-exact parity of the HIP circuit construction and update kernels with the
CPU oracle (teacher-forced: the oracle update is given the GPU's pre-update
state and the GPU's fitness values), plus the equivalence of the fused,
step-by-step and graph-captured generation loops, elite FP64 re-check,
best-circuit tracking and checkpoint / resume."""
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


def targets_for(oracle, n, I, seed, permutation=True):
    rng = np.random.default_rng(seed)
    return np.stack([oracle.unitary(n, inputs.random_target_gates(rng, n, 12, lib=0,
                                                                    permutation=permutation))
                     for _ in range(I)])


def qeqea_ctx(dev, oracle, n, L, P, I, seed, pm=0.3):
    ctx = qe.Context(n, qe.LIB_NCV, qe.ALG_QEQEA, L, P, I, prob_mutation=pm,
                     mutation_range=float(np.pi / 4), seed=seed)
    T = targets_for(oracle, n, I, seed)
    ctx.set_targets(torch.from_numpy(T).to(dev))
    return ctx, T


def gpu_state(ctx):
    torch.cuda.synchronize()
    return {k: ctx.state(k).cpu().numpy() for k in ("theta", "qutrit", "best_f", "best_theta",
                                                    "best_qutrit")}


def to_oracle(oracle, ctx, st):
    o = oracle.QeqeaState(ctx.n, ctx.L, ctx.P, ctx.I, ctx.problem.seed)
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


@pytest.mark.parametrize("n", [2, 3, 4, 5, 6])
def test_qeqea_init_and_sampling_bitexact(dev, oracle, n):
    L, P, I, seed = 13, 24, 3, 4242 + n
    ctx, _ = qeqea_ctx(dev, oracle, n, L, P, I, seed)
    o = oracle.QeqeaState(n, L, P, I, seed)
    assert_same_state(o, gpu_state(ctx))
    for gen in (0, 1, 7, 2 ** 31 + 5):
        slots, gates = ctx.sample(gen)
        rs, rg = o.sample(gen)
        assert np.array_equal(slots.cpu().numpy().view(np.uint32), rs)
        assert np.array_equal(gates.cpu().numpy().view(np.uint16), rg)


@pytest.mark.parametrize("n", [2, 3, 4, 5, 6])
def test_qeqea_update_teacher_forced(dev, oracle, n):
    L, P, I, seed = 11, 16, 2, 777 + n
    pm = 0.45
    ctx, T = qeqea_ctx(dev, oracle, n, L, P, I, seed, pm=pm)
    modes = set()
    for gen in range(6):
        st = gpu_state(ctx)
        o = to_oracle(oracle, ctx, st)
        slots, gates = ctx.sample(gen)
        rs, rg = o.sample(gen)
        assert np.array_equal(slots.cpu().numpy().view(np.uint32), rs)
        assert np.array_equal(gates.cpu().numpy().view(np.uint16), rg)
        f = ctx.eval_population(gates)
        fh = f.cpu().numpy()
        ref = np.array([oracle.fitness(n, rg[c], T[c // P])[0] for c in range(I * P)])
        assert np.abs(fh - ref).max() <= 1e-5
        ctx.update(gen, slots, gates, f)
        o.update(gen, pm, float(np.pi / 4), rs, fh)
        assert_same_state(o, gpu_state(ctx))
        # record which mutation modes this generation exercised
        for i in range(I):
            for ind in range(P):
                w = oracle.philox([3, gen, i, ind], [seed & 0xFFFFFFFF, seed >> 32])
                if w[0] < int(pm * 2 ** 32):
                    modes.add(int(w[1] & 1))
    assert modes == {0, 1}


@pytest.mark.parametrize("n", [3, 4, 5])
def test_fused_generation_teacher_forced_any_order(dev, oracle, n):
    # the internal generation path (fused kernel + update) against the oracle,
    # over generation numbers that jump back and forth and repeat: the
    # decision masks must be cleared whenever a generation does not follow
    # the previous one
    L, P, I, seed = 12, 40, 2, 1313 + n
    pm = 0.4
    ctx, T = qeqea_ctx(dev, oracle, n, L, P, I, seed, pm=pm)
    for gen in (0, 1, 5, 5, 2, 3, 3, 4, 2 ** 31 + 1, 0):
        o = to_oracle(oracle, ctx, gpu_state(ctx))
        rs, rg = o.sample(gen)
        f = ctx.generation(gen)
        fh = f.cpu().numpy()
        ref = np.array([oracle.fitness(n, rg[c], T[c // P])[0] for c in range(I * P)])
        assert np.abs(fh - ref).max() <= 1e-5, gen
        o.update(gen, pm, float(np.pi / 4), rs, fh)
        assert_same_state(o, gpu_state(ctx))


@pytest.mark.parametrize("n,L,P", [(4, 64, 20), (5, 70, 33), (3, 300, 12), (4, 31, 8), (6, 129, 9)])
def test_fused_generation_long_circuits(dev, oracle, n, L, P):
    # circuit lengths at and beyond one wavefront of positions (L = 64 leaves
    # no spare lane for the mutation decision; L > 256 exceeds the slots a
    # wavefront keeps for the key updates), populations that are not a
    # multiple of the 32-bit decision words
    I, seed, pm = 2, 5150 + L, 0.5
    qe.device_errors()                      # start from a clear error word
    ctx, T = qeqea_ctx(dev, oracle, n, L, P, I, seed, pm=pm)
    for gen in range(3):
        o = to_oracle(oracle, ctx, gpu_state(ctx))
        rs, rg = o.sample(gen)
        f = ctx.generation(gen)
        fh = f.cpu().numpy()
        ref = np.array([oracle.fitness(n, rg[c], T[c // P])[0] for c in range(I * P)])
        assert np.abs(fh - ref).max() <= 1e-5, gen
        o.update(gen, pm, float(np.pi / 4), rs, fh)
        assert_same_state(o, gpu_state(ctx))
    assert qe.device_errors() == 0


@pytest.mark.parametrize("n,L,I", [(3, 64, 96), (5, 40, 72), (2, 64, 16)])
def test_many_populations_update_bitexact(dev, oracle, n, L, I):
    # enough mutating individuals per launch that the update serves four
    # slots per lane in part B (the layout of the n = 5 benchmark), with the
    # qutrit-mode split between parts A and B; state bit-exact with the oracle
    # (n = 2: four regions, so each population shares hundreds of entries and
    # part A's workgroup walks its list several times over)
    P, seed, pm = 64, 8080 + n, 0.5
    qe.device_errors()
    ctx, T = qeqea_ctx(dev, oracle, n, L, P, I, seed, pm=pm)
    for gen in range(3):
        o = to_oracle(oracle, ctx, gpu_state(ctx))
        rs, rg = o.sample(gen)
        f = ctx.generation(gen)
        fh = f.cpu().numpy()
        ref = np.concatenate([oracle.eval_batch(np.full(P, n, np.int8), np.arange(P + 1, dtype=np.int32) * L,
                                                rg[i * P:(i + 1) * P].ravel(), np.zeros(P, np.int64), T[i])[:, 0]
                              for i in range(I)])
        assert np.abs(fh - ref).max() <= 1e-5, gen
        o.update(gen, pm, float(np.pi / 4), rs, fh)
        assert_same_state(o, gpu_state(ctx))
    assert qe.device_errors() == 0


@pytest.mark.parametrize("n", [4, 6])
def test_sample_eval_then_update_equals_generation(dev, oracle, n):
    L, P, I, seed = 17, 48, 3, 4040 + n
    a, _ = qeqea_ctx(dev, oracle, n, L, P, I, seed)
    b, _ = qeqea_ctx(dev, oracle, n, L, P, I, seed)
    for gen in range(4):
        # (qe_sample before qe_sample_eval: the latter already commits the
        # elitism of the slots one circuit alone used)
        rs, rg = a.sample(gen)
        slots, gates, f = a.sample_eval(gen)
        assert torch.equal(slots, rs) and torch.equal(gates, rg)
        a.update(gen, slots, gates, f)
        fb = b.generation(gen)
        assert torch.equal(f, fb)
    sa, sb = gpu_state(a), gpu_state(b)
    for k in sa:
        assert np.array_equal(sa[k], sb[k]), k


@pytest.mark.parametrize("L", [20, 64, 65, 150])
def test_fused_fitness_equals_eval_bitwise(dev, oracle, L):
    # n = 4 circuits in the fused kernel take a CV/CV+-only body (per-row-
    # group offsets from the gate table, CV+ as CV with a sign): its fitness
    # must round exactly as the evaluation kernel's does, over one, two and
    # three chunks of 64 positions, and match the oracle
    n, P, I, seed = 4, 40, 2, 6060 + L
    a, T = qeqea_ctx(dev, oracle, n, L, P, I, seed)
    for gen in range(3):
        slots, gates, f = a.sample_eval(gen)
        fe = a.eval_population(gates)
        assert torch.equal(f, fe), gen
        g = gates.cpu().numpy().view(np.uint16)
        ref = np.array([oracle.fitness(n, g[c], T[c // P])[0] for c in range(I * P)])
        assert np.abs(f.cpu().numpy() - ref).max() <= 1e-5, gen
        a.update(gen, slots, gates, f)
    # many data-moving gates per chunk (the largest scale factors)
    kinds = (g & 15)
    assert ((kinds == inputs.CV) | (kinds == inputs.CVDG)).sum(1).max() >= min(L, 64) // 3
    assert qe.device_errors() == 0


def test_state_read_fields(dev, oracle):
    n, L, P, I, seed = 3, 5, 8, 2, 31
    ctx, _ = qeqea_ctx(dev, oracle, n, L, P, I, seed)
    S, Q = n * n * L * P, n * L * P
    sizes = {"theta": I * S, "best_f": I * S, "best_theta": I * S, "qutrit": I * Q * 6,
             "best_qutrit": I * Q * 6, "genomes0": 0, "genomes1": 0,
             "mutation_masks": 2 * I * ((P + 31) // 32)}
    for name, size in sizes.items():
        assert ctx.state(name).numel() == size, name
    assert np.all(ctx.state("best_f").cpu().numpy() == -1.0)
    with pytest.raises(qe.QeError):
        qe._call("qe_state_read", ctx.handle, 8, None, qe.ctypes.byref(qe.ctypes.c_int64(0)), None)


def test_mutation_masks_hold_the_decisions(dev, oracle):
    """After qe_sample_eval of generation gen, the decision bitmaps (state
    field 7) mark exactly the individuals whose MUT_IND draw falls below the
    mutation threshold, and qe_update without slots (the generation's second
    kernel alone) leaves the state the oracle's update gives."""
    n, L, P, I, seed, pm = 3, 6, 40, 3, 57, 0.3
    ctx, T = qeqea_ctx(dev, oracle, n, L, P, I, seed, pm=pm)
    thr = int(np.floor(pm * 2 ** 32))
    for gen in range(4):
        o = to_oracle(oracle, ctx, gpu_state(ctx))
        slots, gates, f = ctx.sample_eval(gen)
        masks = ctx.state("mutation_masks").cpu().numpy().view(np.uint32).reshape(2, I, -1)[gen & 1]
        bits = np.unpackbits(masks.view(np.uint8), bitorder="little").reshape(I, -1)[:, :P]
        want = np.array([[oracle.philox([3, gen, i, ind], [seed & 0xFFFFFFFF, seed >> 32])[0] < thr
                          for ind in range(P)] for i in range(I)])
        assert np.array_equal(bits.astype(bool), want), gen
        ctx.update(gen, None, gates, f)
        o.update(gen, pm, float(np.pi / 4), slots.cpu().numpy().view(np.uint32), f.cpu().numpy())
        assert_same_state(o, gpu_state(ctx))
    with pytest.raises(qe.QeError):      # no qe_sample_eval of that generation just before
        ctx.update(9, None, gates, f)


def run_steps(ctx, gens):
    fs = []
    for gen in gens:
        slots, gates = ctx.sample(gen)
        f = ctx.eval_population(gates)
        ctx.update(gen, slots, gates, f)
        fs.append(f.clone())
    return fs


@pytest.mark.parametrize("n", [3, 4, 5])
def test_generation_and_graph_equal_steps(dev, oracle, n):
    L, P, I, seed, G = 20, 32, 4, 99 + n, 5
    a, _ = qeqea_ctx(dev, oracle, n, L, P, I, seed)
    b, _ = qeqea_ctx(dev, oracle, n, L, P, I, seed)
    c, _ = qeqea_ctx(dev, oracle, n, L, P, I, seed)
    fa = run_steps(a, range(2 * G))
    fb = [b.generation(gen).clone() for gen in range(2 * G)]
    hist = torch.empty((G, I * P), dtype=torch.float32, device=dev)
    fc = []
    for rep in range(2):
        c.run_graph(rep * G, G, hist)
        torch.cuda.synchronize()
        fc += [hist[j].clone() for j in range(G)]
    sa, sb, sc = gpu_state(a), gpu_state(b), gpu_state(c)
    for k in sa:
        assert np.array_equal(sa[k], sb[k]) and np.array_equal(sa[k], sc[k]), k
    for x, y, z in zip(fa, fb, fc):
        assert torch.equal(x, y) and torch.equal(x, z)
    ga = a.get_best(0, with_fp64=False)
    assert ga[:2] == c.get_best(0, with_fp64=False)[:2]


def test_graph_many_populations_equal_generations(dev, oracle):
    # the layout of the n = 5 benchmark (P * L within the shared-slot search):
    # in a graph each update runs the next generation's search, and a replay
    # or generation that follows on reuses it; replays of two and of one
    # generation (one after a skipped generation, whose words are then
    # searched again) against single generations, state bit for bit
    n, L, P, I, seed = 5, 40, 64, 72, 6060
    a, _ = qeqea_ctx(dev, oracle, n, L, P, I, seed, pm=0.3)
    b, _ = qeqea_ctx(dev, oracle, n, L, P, I, seed, pm=0.3)
    ha = torch.empty((2, I * P), dtype=torch.float32, device=dev)
    fa = []
    for first, G in ((0, 2), (2, 2), (4, 1), (6, 2)):
        a.run_graph(first, G, ha)
        torch.cuda.synchronize()
        fa += [ha[j].clone() for j in range(G)]
    fb = [b.generation(gen).clone() for gen in (0, 1, 2, 3, 4, 6, 7)]
    for x, y in zip(fa, fb):
        assert torch.equal(x, y)
    sa, sb = gpu_state(a), gpu_state(b)
    for k in sa:
        assert np.array_equal(sa[k], sb[k]), k


def test_mixed_calls_reuse_slot_words(dev, oracle):
    # graph replays, qe_generation and qe_sample_eval + qe_update in one
    # sequence, with a skipped generation: each call reuses the slot words the
    # update before it wrote, or searches them when they are missing; the
    # fitness and the state match single generations bit for bit
    n, L, P, I, seed = 4, 24, 32, 6, 6161
    a, _ = qeqea_ctx(dev, oracle, n, L, P, I, seed, pm=0.4)
    b, _ = qeqea_ctx(dev, oracle, n, L, P, I, seed, pm=0.4)
    hist = torch.empty((2, I * P), dtype=torch.float32, device=dev)
    fa = []
    a.run_graph(0, 2, hist)
    torch.cuda.synchronize()
    fa += [hist[0].clone(), hist[1].clone()]
    _, gates, f = a.sample_eval(2, keep_slots=False)
    a.update(2, None, gates, f)
    fa.append(f.clone())
    fa.append(a.generation(3).clone())
    _, gates, f = a.sample_eval(5, keep_slots=False)
    a.update(5, None, gates, f)
    fa.append(f.clone())
    a.run_graph(6, 2, hist)
    torch.cuda.synchronize()
    fa += [hist[0].clone(), hist[1].clone()]
    fb = [b.generation(gen).clone() for gen in (0, 1, 2, 3, 5, 6, 7)]
    for j, (x, y) in enumerate(zip(fa, fb)):
        assert torch.equal(x, y), j
    sa, sb = gpu_state(a), gpu_state(b)
    for k in sa:
        assert np.array_equal(sa[k], sb[k]), k


def test_graph_replays_are_stable(dev, oracle):
    # several replays with eager work and synchronisation between them
    n, L, P, I, seed = 4, 16, 64, 2, 5
    a, _ = qeqea_ctx(dev, oracle, n, L, P, I, seed)
    b, _ = qeqea_ctx(dev, oracle, n, L, P, I, seed)
    for rep in range(4):
        a.run_graph(3 * rep, 3)
        torch.cuda.synchronize()
        _ = torch.ones(1000, device=dev).sum().item()
        for gen in range(3 * rep, 3 * rep + 3):
            b.generation(gen)
        sa, sb = gpu_state(a), gpu_state(b)
        for k in sa:
            assert np.array_equal(sa[k], sb[k]), (rep, k)


def test_ga_teacher_forced(dev, oracle):
    w = inputs.workload_ga_n3()
    n, L, P = w["n"], w["L"], w["P"]
    seed = w["seed"]
    ctx = qe.Context(n, w["lib"], qe.ALG_GA, L, P, 1, seed=seed, ga_crossover_prob=0.9,
                     ga_gene_mutation_prob=1.0 / L)
    T = oracle.unitary(n, w["target_gates"][0])[None]
    ctx.set_targets(torch.from_numpy(T).to(dev))
    genomes = oracle.ga_init(n, w["lib"], L, P, 1, seed)
    assert np.array_equal(ctx.state("genomes0").cpu().numpy().view(np.uint16).reshape(P, L), genomes)
    best = -1.0
    for gen in range(w["generations"]):
        _, gates = ctx.sample(gen)
        assert np.array_equal(gates.cpu().numpy().view(np.uint16), genomes)
        f = ctx.eval_population(gates)
        fh = f.cpu().numpy()
        ref = np.array([oracle.fitness(n, genomes[k], T[0])[0] for k in range(P)])
        assert np.abs(fh - ref).max() <= 1e-5
        best = max(best, float(fh.max()))
        ctx.update(gen, None, gates, f)
        genomes = oracle.ga_update(n, w["lib"], L, P, 1, seed, gen, 0.9, 1.0 / L, fh, genomes)
        torch.cuda.synchronize()
        got = ctx.state("genomes1" if gen % 2 == 0 else "genomes0").cpu().numpy().view(np.uint16)
        assert np.array_equal(got.reshape(P, L), genomes), gen
    g, f32, f64 = ctx.get_best(0)
    assert f32 == pytest.approx(best, abs=0)
    assert abs(f64 - oracle.fitness(n, g, T[0])[0]) <= 1e-12
    assert abs(f64 - f32) <= 1e-5


def test_ga_graph_equals_generations(dev, oracle):
    n, L, P, I, seed = 4, 12, 48, 3, 31
    T = torch.from_numpy(targets_for(oracle, n, I, seed, permutation=False)).to(dev)
    a = qe.Context(n, 0, qe.ALG_GA, L, P, I, seed=seed)
    b = qe.Context(n, 0, qe.ALG_GA, L, P, I, seed=seed)
    a.set_targets(T)
    b.set_targets(T)
    fa = [a.generation(gen).clone() for gen in range(6)]
    hist = torch.empty((6, I * P), dtype=torch.float32, device=dev)
    b.run_graph(0, 6, hist)
    torch.cuda.synchronize()
    for j in range(6):
        assert torch.equal(fa[j], hist[j])
    assert torch.equal(a.state("genomes0"), b.state("genomes0"))


@pytest.mark.parametrize("n", [3, 5])
def test_elite_recheck(dev, oracle, n):
    L, P, I, seed, k = 16, 64, 3, 12 + n, 8
    ctx, T = qeqea_ctx(dev, oracle, n, L, P, I, seed)
    slots, gates = ctx.sample(0)
    f = ctx.eval_population(gates)
    idx, f64 = ctx.elite_recheck(gates, f, k)
    fh, gh = f.cpu().numpy(), gates.cpu().numpy().view(np.uint16)
    idx, f64 = idx.cpu().numpy(), f64.cpu().numpy()
    for i in range(I):
        fi = fh[i * P:(i + 1) * P]
        want = sorted(range(P), key=lambda c: (-fi[c], c))[:k]
        assert list(idx[i]) == want
        for e in range(k):
            ref = oracle.fitness(n, gh[i * P + idx[i, e]], T[i])[0]
            assert abs((1 - f64[i, e]) ** 2 - (1 - ref) ** 2) <= 1e-12
            assert abs(f64[i, e] - fi[idx[i, e]]) <= 1e-5


@pytest.mark.parametrize("P,k", [(4096, 4096), (3000, 1000), (1, 1), (4096, 32), (4096, 64),
                                 (257, 64), (300, 7), (256, 256), (512, 65)])
def test_elite_selection_orders_whole_populations(dev, oracle, P, k):
    # the selection sorts (f desc, index asc) over every stage of its network:
    # in-register, in-wavefront and through LDS; ties are frequent here.  One
    # tile of 256 circuits, tiles whose top k (<= 64) are merged (a partial
    # last tile included), and the whole-population sort for larger k
    n, L, I = 3, 6, 2
    ctx, T = qeqea_ctx(dev, oracle, n, L, P, I, 77 + P)
    slots, gates = ctx.sample(0)
    f = ctx.eval_population(gates)
    f[::7] = float("nan")                      # NaN sorts last
    idx, _ = ctx.elite_recheck(gates, f, k)
    fh, idx = f.cpu().numpy(), idx.cpu().numpy()
    for i in range(I):
        fi = fh[i * P:(i + 1) * P]
        key = lambda c: (1, 0.0, c) if np.isnan(fi[c]) else (0, -fi[c], c)
        assert list(idx[i]) == sorted(range(P), key=key)[:k]


def test_checkpoint_resume(dev, oracle):
    n, L, P, I, seed = 4, 10, 32, 2, 2024
    a, T = qeqea_ctx(dev, oracle, n, L, P, I, seed, pm=0.5)
    for gen in range(3):
        a.generation(gen)
    blob = a.checkpoint()
    fa = [a.generation(gen).clone() for gen in range(3, 7)]
    sa = gpu_state(a)
    b, _ = qeqea_ctx(dev, oracle, n, L, P, I, seed, pm=0.5)
    b.restore(blob)
    fb = [b.generation(gen).clone() for gen in range(3, 7)]
    sb = gpu_state(b)
    for k in sa:
        assert np.array_equal(sa[k], sb[k]), k
    for x, y in zip(fa, fb):
        assert torch.equal(x, y)
    assert a.get_best(1, with_fp64=False)[:2] == b.get_best(1, with_fp64=False)[:2]
    other = qe.Context(n, 0, qe.ALG_QEQEA, L, P, I, prob_mutation=0.5, seed=seed + 1)
    with pytest.raises(qe.QeError):
        other.restore(blob)
    with pytest.raises(qe.QeError):
        a.restore(blob[:100])


def test_get_best_tracks_maximum(dev, oracle):
    n, L, P, I, seed = 3, 8, 64, 2, 606
    ctx, T = qeqea_ctx(dev, oracle, n, L, P, I, seed, pm=0.2)
    best = [-1.0] * I
    best_gates = [None] * I
    for gen in range(8):
        slots, gates = ctx.sample(gen)
        f = ctx.eval_population(gates)
        ctx.update(gen, slots, gates, f)
        fh, gh = f.cpu().numpy(), gates.cpu().numpy().view(np.uint16)
        for i in range(I):
            fi = fh[i * P:(i + 1) * P]
            k = int(np.argmax(fi))
            if fi[k] > best[i]:
                best[i], best_gates[i] = float(fi[k]), list(gh[i * P + k])
    for i in range(I):
        g, f32, f64 = ctx.get_best(i)
        assert f32 == best[i] and g == best_gates[i]
        assert abs(f64 - oracle.fitness(n, g, T[i])[0]) <= 1e-12


def test_state_requires_targets(dev):
    ctx = qe.Context(3, 0, qe.ALG_QEQEA, 4, 4, 1, seed=1)
    with pytest.raises(qe.QeError) as e:
        ctx.generation(0)
    assert e.value.status == qe.QE_ERR_STATE
