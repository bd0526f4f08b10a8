"""Mixed widths and lengths: the GA over populations of their own width and
genome length (Sec. V-B with the uneven batches of Sec. IV-D), evaluated in
one cost-sorted launch per generation, against the CPU oracle (teacher-forced:
the oracle's GA update gets the GPU's fitness values), its graph against
step-by-step generations, and the mixed-width evaluation with a workspace
(one sorted launch) against the one without (one launch per width) and the
oracle."""
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


def mixed_setup(oracle, widths, lengths, seed, lib=inputs.LIB_HT_NCV):
    rng = np.random.default_rng(seed)
    tg = [inputs.random_target_gates(rng, n, int(rng.integers(4, 12)), lib) for n in widths]
    T = [oracle.unitary(n, g) for n, g in zip(widths, tg)]
    packed = np.concatenate([t.ravel() for t in T])
    return T, packed


def split_genomes(flat, P, lengths):
    out, o = [], 0
    for L in lengths:
        out.append(flat[o:o + P * L].reshape(P, L))
        o += P * L
    return out


def mixed_ctx(dev, oracle, widths, lengths, P, seed, pc=0.9, pg=0.05, lib=inputs.LIB_HT_NCV):
    ctx = qe.Context(0, lib, qe.ALG_GA, 0, P, seed=seed, ga_crossover_prob=pc,
                     ga_gene_mutation_prob=pg, widths=widths, lengths=lengths)
    T, packed = mixed_setup(oracle, widths, lengths, seed, lib)
    ctx.set_targets(torch.from_numpy(packed).to(dev))
    return ctx, T


WIDTHS = [3, 4, 5, 6, 3, 4, 2, 5]
LENGTHS = [8, 20, 13, 40, 64, 9, 17, 33]


def test_mixed_ga_teacher_forced(dev, oracle):
    P, seed, pc, pg = 16, 91, 0.9, 0.05
    ctx, T = mixed_ctx(dev, oracle, WIDTHS, LENGTHS, P, seed, pc, pg)
    lib = inputs.LIB_HT_NCV
    genomes = [oracle.ga_init_at(n, lib, L, P, i, seed) for i, (n, L) in enumerate(zip(WIDTHS, LENGTHS))]
    got = split_genomes(ctx.state("genomes0").cpu().numpy().view(np.uint16), P, LENGTHS)
    for i in range(len(WIDTHS)):
        assert np.array_equal(got[i], genomes[i]), i
    for gen in range(4):
        f = ctx.generation(gen)
        torch.cuda.synchronize()
        fh = f.cpu().numpy().reshape(len(WIDTHS), P)
        for i, (n, L) in enumerate(zip(WIDTHS, LENGTHS)):
            ref = np.array([oracle.fitness(n, genomes[i][k], T[i])[0] for k in range(P)])
            assert np.abs(fh[i] - ref).max() <= 1e-5, (gen, i)
            genomes[i] = oracle.ga_update_at(n, lib, L, P, i, seed, gen, pc, pg, fh[i], genomes[i])
        got = split_genomes(ctx.state("genomes1" if gen % 2 == 0 else "genomes0").cpu().numpy()
                            .view(np.uint16), P, LENGTHS)
        for i in range(len(WIDTHS)):
            assert np.array_equal(got[i], genomes[i]), (gen, i)
    for i, (n, L) in enumerate(zip(WIDTHS, LENGTHS)):
        g, f32, f64 = ctx.get_best(i)
        assert len(g) == L
        assert abs(f64 - oracle.fitness(n, np.array(g, np.uint16), T[i])[0]) <= 1e-12
        assert abs(f64 - f32) <= 1e-5
    ctx.close()


def test_mixed_graph_equals_generations(dev, oracle):
    P, seed, G = 32, 17, 5
    a, _ = mixed_ctx(dev, oracle, WIDTHS, LENGTHS, P, seed)
    b, _ = mixed_ctx(dev, oracle, WIDTHS, LENGTHS, P, seed)
    fa = [a.generation(gen).clone() for gen in range(G)]
    hist = torch.empty((G, len(WIDTHS) * P), dtype=torch.float32, device=dev)
    b.run_graph(0, G, hist)
    torch.cuda.synchronize()
    for j in range(G):
        assert torch.equal(fa[j], hist[j]), j
    assert torch.equal(a.state("genomes1"), b.state("genomes1"))
    # the graph replays: the next G generations continue both searches alike
    fa = [a.generation(G + gen).clone() for gen in range(G)]
    b.run_graph(G, G, hist)
    torch.cuda.synchronize()
    for j in range(G):
        assert torch.equal(fa[j], hist[j]), G + j
    a.close()
    b.close()


def test_mixed_elite_recheck_and_checkpoint(dev, oracle):
    P, seed, k = 64, 23, 8
    ctx, T = mixed_ctx(dev, oracle, WIDTHS, LENGTHS, P, seed)
    for gen in range(3):
        f = ctx.generation(gen)
    _, gates = ctx.sample(3)
    f = ctx.eval_population(gates)
    idx, f64 = ctx.elite_recheck(gates, f, k)
    torch.cuda.synchronize()
    fh = f.cpu().numpy().reshape(len(WIDTHS), P)
    flat = gates.cpu().numpy().view(np.uint16).ravel()
    genomes = split_genomes(flat, P, LENGTHS)
    idx, f64 = idx.cpu().numpy(), f64.cpu().numpy()
    for i, n in enumerate(WIDTHS):
        want = sorted(range(P), key=lambda c: (-fh[i][c], c))[:k]
        assert list(idx[i]) == want
        for e in range(k):
            assert abs(f64[i, e] - oracle.fitness(n, genomes[i][idx[i, e]], T[i])[0]) <= 1e-12
    blob = ctx.checkpoint()
    fa = [ctx.generation(4 + j).clone() for j in range(3)]
    ctx.restore(blob)
    fb = [ctx.generation(4 + j).clone() for j in range(3)]
    torch.cuda.synchronize()
    for x, y in zip(fa, fb):
        assert torch.equal(x, y)
    # a context with other widths or lengths refuses the checkpoint
    other, _ = mixed_ctx(dev, oracle, WIDTHS[::-1], LENGTHS[::-1], P, seed)
    with pytest.raises(qe.QeError):
        other.restore(blob)
    other.close()
    ctx.close()


def random_mixed_batch(rng, oracle, B, lib=inputs.LIB_HT_NCV):
    nq = rng.integers(1, 7, size=B).astype(np.int8)
    lens = rng.integers(0, 70, size=B)
    goff = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    gates = np.concatenate([inputs.random_circuits(rng, 1, int(n), int(L), lib)[0]
                            for n, L in zip(nq, lens)] + [np.zeros(0, np.uint16)]).astype(np.uint16)
    mats, toff, o = [], [], 0
    for n in nq:
        T = oracle.unitary(int(n), inputs.random_target_gates(rng, int(n), 6, lib))
        mats.append(T.ravel())
        toff.append(o)
        o += T.size
    return nq, goff, gates, np.concatenate(mats), np.array(toff, np.int64)


@pytest.mark.parametrize("B", [1, 37, 300])
def test_mixed_eval_workspace_equals_per_width(dev, oracle, B):
    rng = np.random.default_rng(1000 + B)
    nq, goff, gates, T, toff = random_mixed_batch(rng, oracle, B)
    args = dict(nq=torch.from_numpy(nq).to(dev), goff=torch.from_numpy(goff).to(dev),
                toff=torch.from_numpy(toff).to(dev), target_stride=None, want_g=True, want_delta=True)
    g = torch.from_numpy(gates.view(np.int16)).to(dev)
    Td = torch.from_numpy(T).to(dev).to(torch.complex64)
    fw, gw, dw = qe.eval_fitness(g, Td, workspace=True, **args)
    fp, gp, dp = qe.eval_fitness(g, Td, workspace=False, **args)
    torch.cuda.synchronize()
    # the two schedules give the same bits
    assert torch.equal(fw, fp) and torch.equal(gw, gp) and torch.equal(dw, dp)
    ref = oracle.eval_batch(nq, goff, gates, toff, T)
    assert np.abs(fw.cpu().numpy().astype(np.float64) - ref[:, 0]).max() <= 1e-5
    assert qe.device_errors() == 0


def test_mixed_eval_two_streams(dev, oracle):
    """Two mixed batches of different sizes on two streams, each with its own
    workspace, overlap without interfering."""
    rng = np.random.default_rng(77)
    batches = [random_mixed_batch(rng, oracle, B) for B in (900, 130)]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    outs = []
    torch.cuda.synchronize()
    prepared = []
    for (nq, goff, gates, T, toff) in batches:
        prepared.append((torch.from_numpy(nq).to(dev), torch.from_numpy(goff).to(dev),
                         torch.from_numpy(gates.view(np.int16)).to(dev),
                         torch.from_numpy(T).to(dev).to(torch.complex64), torch.from_numpy(toff).to(dev),
                         qe.eval_workspace(len(nq), dev)))
    torch.cuda.synchronize()
    for rep in range(3):
        outs = []
        for (nqd, goffd, gd, Td, toffd, ws), st in zip(prepared, streams):
            with torch.cuda.stream(st):
                f, _, _ = qe.eval_fitness(gd, Td, nq=nqd, goff=goffd, toff=toffd, target_stride=None,
                                          workspace=ws, stream=st)
            outs.append(f)
        torch.cuda.synchronize()
        for (nq, goff, gates, T, toff), f in zip(batches, outs):
            ref = oracle.eval_batch(nq, goff, gates, toff, T)
            assert np.abs(f.cpu().numpy().astype(np.float64) - ref[:, 0]).max() <= 1e-5, rep
    assert qe.device_errors() == 0


def test_mixed_context_lends_its_workspace(dev, oracle):
    """qe_eval_fitness with a mixed context uses the context's own
    workspace (one sorted launch) and leaves the context's generation order
    intact."""
    P, seed = 16, 5
    ctx, _ = mixed_ctx(dev, oracle, WIDTHS, LENGTHS, P, seed)
    ref_ctx, _ = mixed_ctx(dev, oracle, WIDTHS, LENGTHS, P, seed)
    rng = np.random.default_rng(3)
    nq, goff, gates, T, toff = random_mixed_batch(rng, oracle, 50)
    f, _, _ = qe.eval_fitness(torch.from_numpy(gates.view(np.int16)).to(dev),
                              torch.from_numpy(T).to(dev).to(torch.complex64),
                              nq=torch.from_numpy(nq).to(dev), goff=torch.from_numpy(goff).to(dev),
                              toff=torch.from_numpy(toff).to(dev), target_stride=None, workspace=False,
                              ctx=ctx)
    a = ctx.generation(0)
    b = ref_ctx.generation(0)
    torch.cuda.synchronize()
    ref = oracle.eval_batch(nq, goff, gates, toff, T)
    assert np.abs(f.cpu().numpy().astype(np.float64) - ref[:, 0]).max() <= 1e-5
    assert torch.equal(a, b)
    ctx.close()
    ref_ctx.close()


def test_mixed_create_rejects_bad_tables(dev):
    with pytest.raises(qe.QeError):
        qe.Context(0, inputs.LIB_HT_NCV, qe.ALG_GA, 0, 16, widths=[3, 7], lengths=[4, 4])
    with pytest.raises(qe.QeError):
        qe.Context(0, inputs.LIB_HT_NCV, qe.ALG_GA, 0, 16, widths=[3, 4], lengths=[4, 0])
    with pytest.raises(qe.QeError):
        qe.Context(0, inputs.LIB_NCV, qe.ALG_QEQEA, 0, 16, widths=[3, 4], lengths=[4, 4])
