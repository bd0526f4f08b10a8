#!/usr/bin/env python3
"""Throughput of the QEQEA circuit-fitness hot path on one MI355X.

Headline workload (seeded, synthetic): n = 5 wires, library {I, NOT, CNOT,
CV, CV+}, 1024 independent QEQEA populations, each sampled into P = 64
circuits of L = 40 gates per generation (65536 circuit evaluations per
generation); each population's target is a random reversible permutation
built from 16 NOT/CNOT gates (the paper's targets are small reversible
gates).  A step is one generation of the whole hot path: circuit
construction by sampling the encoding (Sec. IV-D, Eq. 10, qutrit
measurement), Eq. 11 fitness of every circuit (FP32 per-gate path), segment
fitness, elitism and adaptive mutation (Secs. IV-E.1, IV-F, Eq. 12).  K
generations run as one HIP graph followed by the FP64 re-check of each
population's 32 best circuits of the last generation; after W warm-up
generations the same graph and re-check run once untimed, then three timed
replays (each exactly K generations plus the re-check, bracketed by device
synchronisations and HIP events) give the median.

Prints one JSON line (the metric is circuit-fitness evaluations per second)
with a roofline entry for the dominant kernel (the fused sampling + fitness
kernel, against the LDS bandwidth measured by a probe kernel in the same
run) and one for the update kernel (against HBM), each timed launch by launch
with HIP events on the launch stream, and the CPU oracle's rate on a bounded
sample of the same workload on one host core and on all of them.  The
"secondary" object adds the other workloads of the study: the n=6 precision
study (FP32 against the bf16/fp16 hi+lo MFMA paths, with their fitness error
against the FP64 path, elite top-32 agreement and Kendall tau), one n=4
population of 4096 circuits, a mixed-width GA batch, and the Ising,
phase-insensitive and dense-ablation variants.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "circuit-fitness evals/sec (n=4..6), FP32 vs BF16-MFMA at stated fitness error"
FP32_VECTOR_PEAK_TFLOPS = 157.3   # MI355X, 256 CUs x 4 SIMD x 16 lanes x 2 x 2 (packed) x 2.4 GHz
LDS_SPEC_GBPS = 256 * 128 * 2.4   # MI355X LDS from unit counts: 256 CUs x 128 B/clock x 2.4 GHz
HBM_PEAK_GBPS = 8000.0            # MI355X HBM3E, published
# The LDS peak the rooflines divide by: the best rate of the LDS probe kernel
# measured in this run (set by main), the unit-count figure until then.
LDS_PEAK_GBPS = LDS_SPEC_GBPS


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def source_hash():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1809_11134_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as fh:
            h.update(name.encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def algorithmic_flops(gates, n):
    """Real floating-point operations the method needs for these circuits
    (N = 2^n): a CV or CV+ gate updates the N^2/2 controlled entries of
    U T^dagger at 6 flops each, H all N^2 entries at 4, T N^2/2 at 4; NOT,
    CNOT and I only permute rows (0); an Ising gate (R_x, R_y, R_z, J)
    updates all N^2 entries at 6 (two real outputs of two products and a
    sum); the fitness reduction reads every entry once (|m|^2 accumulated:
    4 flops)."""
    import numpy as np
    NN = float(1 << (2 * n))
    kinds = np.asarray(gates).astype(np.int64) & 15
    per_kind = np.zeros(16)
    per_kind[3] = per_kind[4] = 3.0 * NN
    per_kind[5] = 4.0 * NN
    per_kind[6] = 2.0 * NN
    per_kind[7:11] = 6.0 * NN
    return float(per_kind[kinds].sum() + kinds.shape[0] * 4.0 * NN)


def algorithmic_lds_bytes(gates, n):
    """LDS bytes the per-gate method must move for these circuits (N = 2^n):
    every complex64 entry a gate changes is read and written once (16 B);
    CV, CV+ and T change N^2/2 entries, H and the Ising gates (R_x, R_y, R_z,
    J) all N^2, NOT / CNOT / I none (a row relabelling); plus one pass
    writing T^dagger and one reading the result for the fitness (8 B per
    entry each)."""
    import numpy as np
    NN = float(1 << (2 * n))
    kinds = np.asarray(gates).astype(np.int64) & 15
    per_kind = np.zeros(16)
    per_kind[3] = per_kind[4] = per_kind[6] = 8.0 * NN
    per_kind[5] = 16.0 * NN
    per_kind[7:11] = 16.0 * NN
    circuits = kinds.shape[0] if kinds.ndim > 1 else 1
    return float(per_kind[kinds].sum() + circuits * 16.0 * NN)


def traffic_from_profiles(kernel_key, src_hash):
    path = os.path.join(ROOT, "profiles", f"pmc_{kernel_key}_traffic.txt")   # JSON text
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("source_hash") != src_hash:
        return None
    return d.get("hbm_bytes_per_launch")


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, seconds, instances=16):
    """The oracle (test infrastructure) on a bounded sample of the workload:
    whole QEQEA generations of the first `instances` populations -- sampling,
    FP64 fitness of their circuits (OpenMP over circuits), update -- for
    about seconds / 2 on one thread, then on all the threads OpenMP gives
    it.  The populations are independent and their encodings do not depend
    on how many are run, so the sample is part of the same search."""
    import numpy as np
    from oracle import oracle as O
    n, L, P, seed = w["n"], w["L"], w["P"], w["seed"]
    I = min(instances, w["instances"])
    N = 1 << n
    T = np.concatenate([O.unitary(n, np.asarray(tg, np.uint16)).reshape(1, N, N)
                        for tg in w["target_gates"][:I]])
    nq = np.full(I * P, n, np.int8)
    goff = np.arange(I * P + 1, dtype=np.int32) * L
    toff = (np.arange(I * P, dtype=np.int64) // P) * (N * N)
    all_threads = O.num_threads()

    def run(threads, budget):
        O.set_num_threads(threads)
        st = O.QeqeaState(n, L, P, I, seed)
        gens = 0
        t0 = time.perf_counter()
        while True:
            slots, gates = st.sample(gens)
            out = O.eval_batch(nq, goff, gates.ravel(), toff, T)
            st.update(gens, 0.1, math.pi / 4, slots, out[:, 0].astype(np.float32))
            gens += 1
            el = time.perf_counter() - t0
            if el >= budget:
                return gens, el

    g1, e1 = run(1, seconds / 2)
    ga, ea = run(all_threads, seconds / 2)
    O.set_num_threads(all_threads)
    return dict(value=ga * I * P / ea, unit="evals/s", cores=all_threads, kind="oracle",
                value_1core=g1 * I * P / e1, cpu_model=cpu_model(), host_cpus=os.cpu_count(),
                sample=f"whole QEQEA generations of {I} of the {w['instances']} populations of "
                       f"{w['name']} ({I * P} circuits per generation; FP64 fitness over OpenMP "
                       f"threads, sampling and update single-threaded): {g1} generations in "
                       f"{e1:.1f} s on 1 thread, {ga} in {ea:.1f} s on {all_threads} threads")


def _timed_eval(batch, path, B, reps, dev):
    """Median duration of one evaluation launch (preallocated output and
    workspace, launched through the C ABI: qe_eval_fitness_ws, so that a
    mixed-width batch takes the cost-sorted single launch), and the
    output."""
    import ctypes

    import torch
    from paper_1809_11134_amd import qe
    f = torch.empty(B, dtype=torch.float32, device=dev)
    ws = qe.eval_workspace(B, dev)
    launch = lambda: qe._call("qe_eval_fitness_ws", ctypes.byref(batch), path, qe._ptr(f), None,
                              None, qe._ptr(ws), ws.numel() * 4, qe._stream(None))
    return _events_us(launch, reps), f


def _events_us(fn, reps):
    import torch
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(reps)]
    fn()
    torch.cuda.synchronize()
    for a, b in evs:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    t = sorted(a.elapsed_time(b) * 1e3 for a, b in evs)
    return t[len(t) // 2]


def secondary_precision(dev, reps=5):
    """n=6, library {H,T,CNOT,CV,CV+}, 8192 circuits x 48 gates (3/4 planted
    near the target): evaluations/s of each path and its fitness error against
    the FP64 path, elite top-32 agreement (tie-aware) and Kendall tau."""
    import numpy as np
    import torch
    from scipy.stats import kendalltau
    from paper_1809_11134_amd import inputs, qe
    w = inputs.workload_precision_n6()
    n, L, P = w["n"], w["L"], w["P"]
    g = torch.from_numpy(w["gates"].astype(np.int16)).to(dev)
    tg = torch.from_numpy(w["target_gates"].astype(np.int16)[None]).to(dev)
    T64 = qe.build_unitary(tg, n, tg.shape[1], precision=1)[0]
    T32 = T64.to(torch.complex64)
    f64 = qe.eval_fitness_fp64(g, T64, n=n, L=L)[0].cpu().numpy()
    order64 = np.lexsort((np.arange(P), -f64))
    cut = f64[order64[31]]
    out = {"workload": w["name"], "reference": "FP64 path on the GPU", "paths": {}}
    batch, keep, _ = qe.make_batch(g, T32, n=n, L=L, target_stride=0)
    lds = algorithmic_lds_bytes(w["gates"], n)
    lc = 1 if L >= 32 else 0
    tuned_mb = qe.get_mfma_min_block(n, lc)
    out["mfma_min_block"] = tuned_mb
    for name, path, mb in (("fp32", qe.PATH_FP32, tuned_mb), ("bf16_mfma", qe.PATH_MFMA_BF16, tuned_mb),
                           ("fp16_mfma", qe.PATH_MFMA_FP16, tuned_mb),
                           ("bf16_mfma_no_renorm", qe.PATH_MFMA_BF16_RAW, tuned_mb),
                           ("fp16_mfma_no_renorm", qe.PATH_MFMA_FP16_RAW, tuned_mb),
                           ("bf16_mfma_every_block", qe.PATH_MFMA_BF16, 1)):
        # (the tuned threshold: groups of fewer gates go gate by gate in FP32;
        # every_block fuses every group)
        qe.set_mfma_min_block(n, lc, mb)
        us, fd = _timed_eval(batch, path, P, reps, dev)
        f = fd.cpu().numpy().astype(np.float64)
        err = np.abs(f - f64)
        top = np.lexsort((np.arange(P), -f))[:32]
        agree = int((f64[top] >= cut - 1e-6).sum())
        out["paths"][name] = {"evals_per_s": P / (us * 1e-6), "kernel_us": us,
                              "max_abs_df": float(err.max()), "p99_abs_df": float(np.quantile(err, 0.99)),
                              "elite32_agreement": agree, "kendall_tau": float(kendalltau(f, f64)[0])}
        if path == qe.PATH_FP32:
            # the per-gate model's LDS bytes for these circuits against the LDS peak
            out["paths"][name]["algorithmic_lds_bytes"] = lds
            out["paths"][name]["lds_frac"] = lds / (us * 1e-6) / 1e9 / LDS_PEAK_GBPS
    qe.set_mfma_min_block(n, lc, tuned_mb)
    return out


def secondary_phase_insensitive(dev, gens=100):
    """The bench workload (n=4, P=4096, L=30) with the search maximising the
    phase-insensitive fitness (QE_FIT_PHASE_INSENSITIVE): a graph of `gens`
    whole generations."""
    import numpy as np
    import torch
    from paper_1809_11134_amd import inputs, qe
    w = inputs.workload_qeqea_n4()
    n, L, P, I = w["n"], w["L"], w["P"], w["instances"]
    tg = torch.from_numpy(np.stack(w["target_gates"]).astype(np.int16)).to(dev)
    T = qe.build_unitary(tg, n, tg.shape[1], precision=1)
    ctx = qe.Context(n, w["lib"], qe.ALG_QEQEA, L, P, I, prob_mutation=0.1,
                     mutation_range=math.pi / 4, seed=w["seed"], fitness_mode=qe.FIT_PHASE_INSENSITIVE)
    ctx.set_targets(T)
    hist = torch.empty((gens, I * P), dtype=torch.float32, device=dev)
    ctx.graph_prepare(gens, hist)
    ctx.run_graph(0, gens, hist)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    ctx.run_graph(gens, gens, hist)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    best = ctx.get_best(0)
    ctx.close()
    return {"workload": w["name"] + "_phase_insensitive", "generations": gens,
            "evals_per_s": gens * I * P / (ms * 1e-3), "ms_per_generation": ms / gens,
            "best_f_fp32": best[1], "best_f_fp64": best[2]}


def secondary_qeqea_ising(dev, gens=100, reps=50):
    """The bench shape (n=4, P=4096, L=30) with the Ising library of Sec. III
    (rotations about the measured axis and interactions, continuous angles):
    a graph of `gens` whole generations, and the fused sampling + fitness
    kernel timed over `reps` back-to-back launches with its LDS roofline."""
    import numpy as np
    import torch
    from paper_1809_11134_amd import inputs, qe
    w = inputs.workload_qeqea_ising_n4()
    n, L, P, I = w["n"], w["L"], w["P"], w["instances"]
    tg = torch.from_numpy(np.stack(w["target_gates"]).astype(np.int16)).to(dev)
    T = qe.build_unitary(tg, n, tg.shape[1], precision=1)
    ctx = qe.Context(n, w["lib"], qe.ALG_QEQEA, L, P, I, prob_mutation=0.1,
                     mutation_range=math.pi / 4, seed=w["seed"])
    ctx.set_targets(T)
    hist = torch.empty((gens, I * P), dtype=torch.float32, device=dev)
    ctx.graph_prepare(gens, hist)
    ctx.run_graph(0, gens, hist)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    ctx.run_graph(gens, gens, hist)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    slots, gates, angles, fk = ctx.sample_eval(2 * gens)
    torch.cuda.synchronize()
    e0.record()
    for r in range(reps):
        ctx.sample_eval(2 * gens + 1 + r, slots, gates, fk, angles=angles)
    e1.record()
    torch.cuda.synchronize()
    kern_ms = e0.elapsed_time(e1) / reps
    gh = gates.cpu().numpy()
    lds = algorithmic_lds_bytes(gh, n)
    flops = algorithmic_flops(gh, n)
    achieved = lds / (kern_ms / 1e3) / 1e9
    best = ctx.get_best(0)
    ctx.close()
    return {"workload": w["name"], "generations": gens,
            "evals_per_s": gens * I * P / (ms * 1e-3), "ms_per_generation": ms / gens,
            "kernel": "population_kernel<4,1,true,true> (sampling + Ising decode + Eq. 11 fitness "
                      "+ segment max, LDS-staged)",
            "kernel_us": kern_ms * 1e3, "algorithmic_lds_bytes_per_launch": lds,
            "lds_gbps": achieved, "lds_frac": achieved / LDS_PEAK_GBPS,
            "alu_tflops": flops / (kern_ms / 1e3) / 1e12,
            "best_f_fp32": best[1], "best_f_fp64": best[2]}


def dense_flops(gates, n):
    """FP32 work of the dense segment-matrix scheme (Sec. IV-C, steps 3-5) for
    these circuits: each non-identity gate is one N x N by N x N complex
    product, 8 N^3 real operations (4 multiply-add pairs per complex
    multiply-add); the Kronecker expansion and the fitness reduction are
    lower order and not counted."""
    import numpy as np
    kinds = np.asarray(gates).astype(np.int64) & 15
    return float(np.count_nonzero(kinds) * 8.0 * float(1 << (3 * n)))


def secondary_dense(dev, reps=5):
    """Ablation: the paper's dense segment matrices against the per-gate row
    updates on the same circuits -- the bench shape (4096 circuits of 30
    gates, n=4, library {I,NOT,CNOT,CV,CV+}) and 1024 circuits of the n=6
    precision workload (48 gates, library {H,T,CNOT,CV,CV+})."""
    import ctypes

    import numpy as np
    import torch
    from paper_1809_11134_amd import inputs, qe
    out = {}
    rng = np.random.default_rng(inputs.SEED_BASE + 7)
    pw = inputs.workload_precision_n6()
    for name, n, gates, tgates in (
            ("n4_p4096_l30", 4, inputs.random_circuits(rng, 4096, 4, 30, inputs.LIB_NCV),
             inputs.random_target_gates(rng, 4, 12, permutation=True)),
            ("n6_p1024_l48", 6, pw["gates"][:1024], pw["target_gates"])):
        L = gates.shape[1]
        gd = torch.from_numpy(np.ascontiguousarray(gates).view(np.int16)).to(dev)
        T = qe.build_unitary(torch.from_numpy(np.asarray(tgates, np.uint16).view(np.int16)[None]).to(dev),
                             n, len(tgates), precision=0)[0]
        batch, keep, B = qe.make_batch(gd, T, n=n, L=L, target_stride=0)
        res = {}
        for path, key in ((qe.PATH_FP32, "per_gate"), (qe.PATH_DENSE, "dense")):
            f = torch.empty(B, dtype=torch.float32, device=dev)
            launch = lambda: qe._call("qe_eval_fitness", None, ctypes.byref(batch), path, qe._ptr(f),
                                      None, None, qe._stream(None))
            us = _events_us(launch, reps)
            res[key] = {"us_per_launch": us, "evals_per_s": B / (us * 1e-6), "f": f}
        fl = dense_flops(gates, n)
        d_us = res["dense"]["us_per_launch"]
        out[name] = {"per_gate_us": res["per_gate"]["us_per_launch"], "dense_us": d_us,
                     "per_gate_evals_per_s": res["per_gate"]["evals_per_s"],
                     "dense_evals_per_s": res["dense"]["evals_per_s"],
                     "per_gate_speedup": d_us / res["per_gate"]["us_per_launch"],
                     "dense_flops_per_launch": fl, "dense_tflops": fl / (d_us * 1e-6) / 1e12,
                     "dense_alu_frac": fl / (d_us * 1e-6) / 1e12 / FP32_VECTOR_PEAK_TFLOPS,
                     "max_abs_df_dense_vs_per_gate":
                         float((res["dense"]["f"] - res["per_gate"]["f"]).abs().max())}
    return out


def measure_lds_peak(dev, reps=5):
    """LDS bandwidth of the probe kernel (16-byte accesses, no bank
    conflicts, five 32 KB workgroups per compute unit): reads, writes, and a
    copy within LDS; GB/s of each (median of `reps` launches)."""
    import torch
    from paper_1809_11134_amd import qe
    wg, iters = 256 * 5 * 4, 256
    sink = torch.empty(wg * 256, dtype=torch.int32, device=dev)
    out = {}
    for mode, name in ((0, "read_b128"), (1, "write_b128"), (2, "copy_b128")):
        nbytes = qe.probe_lds(mode, wg, iters, sink)
        us = _events_us(lambda: qe.probe_lds(mode, wg, iters, sink), reps)
        out[name] = round(nbytes / (us * 1e-6) / 1e9, 1)
    return out


def measure_record_floor(dev, records, accesses, reps=5):
    """Random 16-byte record accesses in HBM (the record probe): `accesses`
    uniform random records of a buffer of `records` records (the size of the
    workload's slot encoding), read, and read then written back; microseconds
    per launch (median of `reps`)."""
    import torch
    from paper_1809_11134_amd import qe
    buf = torch.zeros((records, 4), dtype=torch.int32, device=dev)
    sink = torch.zeros(1, dtype=torch.int32, device=dev)
    out = {}
    for mode, name in ((0, "read_us"), (1, "read_write_us")):
        out[name] = round(_events_us(lambda: qe.probe_records(mode, buf, accesses, sink, salt=mode), reps), 2)
    del buf
    torch.cuda.empty_cache()
    return out


def qeqea_context(w, dev, fitness_mode=0):
    import numpy as np
    import torch
    from paper_1809_11134_amd import qe
    n, L, P, I = w["n"], w["L"], w["P"], w["instances"]
    tg = torch.from_numpy(np.stack(w["target_gates"]).astype(np.int16)).to(dev)
    T = qe.build_unitary(tg, n, tg.shape[1], precision=1)          # [I, N, N] complex128
    ctx = qe.Context(n, w["lib"], qe.ALG_QEQEA, L, P, I, prob_mutation=0.1,
                     mutation_range=math.pi / 4, seed=w["seed"], fitness_mode=fitness_mode)
    ctx.set_targets(T)
    return ctx


def qeqea_graph_run(ctx, K, W, dev, reps=3, elite_k=32):
    """W warm-up generations (their own graph), then the K-generation graph
    and the FP64 re-check of each population's elite_k best once untimed,
    then `reps` timed replays of both (generations continue where the last
    run stopped).  Returns (median ms per replay, all replay times in ms,
    the next generation index, FP32 vs FP64 error of the last re-check)."""
    import torch
    IP = ctx.I * ctx.P
    f_warm = torch.empty((W, IP), dtype=torch.float32, device=dev)
    f_hist = torch.empty((K, IP), dtype=torch.float32, device=dev)
    ctx.graph_prepare(W, f_warm)
    ctx.graph_prepare(K, f_hist)
    ctx.run_graph(0, W, f_warm)
    gen = W
    ctx.run_graph(gen, K, f_hist)
    ctx.elite_recheck(None, f_hist[K - 1], elite_k)
    gen += K
    torch.cuda.synchronize()
    times = []
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    for _ in range(reps):
        torch.cuda.synchronize()
        e0.record()
        ctx.run_graph(gen, K, f_hist)
        idx, f64 = ctx.elite_recheck(None, f_hist[K - 1], elite_k)
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
        gen += K
    f32 = f_hist[K - 1].view(ctx.I, ctx.P).gather(1, idx.long()).double()
    err = float((f32 - f64).abs().max().item())
    return sorted(times)[len(times) // 2], times, gen, err


def time_generation_kernels(ctx, gen0, R, dev):
    """The two kernels of a generation as the graph launches them, timed
    with HIP events on the launch stream.  Populations small enough for the
    shared-slot search: R generations run as qe_sample_eval (without slot
    output) then qe_update, each launch between its own two events; after the
    first generation qe_sample_eval is the fused sampling + fitness kernel
    alone (the update before it ran the generation's search) and qe_update
    is the update kernel with the next generation's search, as in the graph.
    Other populations: R fused launches back to back between two events,
    then R generations with each update between its own two events.
    Returns (fused us, update us, the last generation's gates, next
    generation index)."""
    import torch
    IP = ctx.I * ctx.P
    gates = torch.empty((IP, ctx.L), dtype=torch.int16, device=dev)
    f = torch.empty(IP, dtype=torch.float32, device=dev)
    gen = gen0
    for _ in range(2):
        ctx.sample_eval(gen, None, gates, f, keep_slots=False)
        ctx.update(gen, None, gates, f)
        gen += 1
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(R)]
    if ctx.P * ctx.L <= 4096 and ctx.L <= 256:
        torch.cuda.synchronize()
        for r in range(R):
            ev[r][0].record()
            ctx.sample_eval(gen + r, None, gates, f, keep_slots=False)
            ev[r][1].record()
            ev[r][2].record()
            ctx.update(gen + r, None, gates, f)
            ev[r][3].record()
        torch.cuda.synchronize()
        fused = sum(e[0].elapsed_time(e[1]) for e in ev) / R * 1e3
    else:
        torch.cuda.synchronize()
        ev[0][0].record()
        for r in range(R):
            ctx.sample_eval(gen + r, None, gates, f, keep_slots=False)
        ev[0][1].record()
        torch.cuda.synchronize()
        fused = ev[0][0].elapsed_time(ev[0][1]) / R * 1e3
        ctx.update(gen + R - 1, None, gates, f)
        gen += R
        torch.cuda.synchronize()
        for r in range(R):
            ctx.sample_eval(gen + r, None, gates, f, keep_slots=False)
            ev[r][2].record()
            ctx.update(gen + r, None, gates, f)
            ev[r][3].record()
        torch.cuda.synchronize()
    upd = sum(e[2].elapsed_time(e[3]) for e in ev) / R * 1e3
    return fused, upd, gates, gen + R


def update_algorithmic_bytes(ctx, gen, dev):
    """HBM bytes the update of generation `gen` must move (the per-unit
    figures are those of the design notes): for every distinct used slot,
    elitism reads its segment fitness, angle, best angle and best fitness
    and writes two of them (24 B), a rotation slot also reads its qutrit and
    best qutrit and writes one (72 B); every slot of a mutating individual in
    qubit mode reads its angle and best fitness and writes the angle (12 B,
    R*L slots), every rotation slot of one in qutrit mode reads its qutrit and
    best fitness and writes the qutrit (52 B, n*L slots), the two modes
    equiprobable; the generation's best circuit reads the P fitness values
    (4 B each); with the shared-slot search, the update writes the next
    generation's slot words (4 B per entry) and reads this generation's list
    of shared entries and writes the next one's (8 + 8 B per shared entry,
    this generation's count standing for both).
    Counts come from the generation's own slots and decision bitmaps (it is
    sampled here, then updated).  Returns the update kernel's bytes (the
    elitism of the shared slots, the mutation, the best circuit, the words),
    the bytes of the elitism the fused kernel commits (the slots one circuit
    alone used) and the counts."""
    import numpy as np
    import torch
    IP = ctx.I * ctx.P
    slots = torch.empty((IP, ctx.L), dtype=torch.int32, device=dev)
    gates = torch.empty((IP, ctx.L), dtype=torch.int16, device=dev)
    f = torch.empty(IP, dtype=torch.float32, device=dev)
    ctx.sample_eval(gen, slots, gates, f)
    masks = ctx.state("mutation_masks")
    ctx.update(gen, None, gates, f)
    torch.cuda.synchronize()
    sl = slots.cpu().numpy().view(np.uint32).reshape(ctx.I, ctx.P * ctx.L).astype(np.int64)
    Q = ctx.n * ctx.L * ctx.P
    R = ctx.n + ctx.n * (ctx.n - 1)
    inst = np.arange(ctx.I, dtype=np.int64)[:, None] * (R * ctx.L * ctx.P)
    used, uses = np.unique((sl + inst).ravel(), return_counts=True)
    rot = (used % (R * ctx.L * ctx.P)) < Q
    used_rot = int(np.count_nonzero(rot))
    # slots one circuit alone used: their elitism is committed by the fused
    # kernel (populations small enough for the shared-slot search)
    dedup = ctx.P * ctx.L <= 4096 and ctx.L <= 256
    alone = (uses == 1) if dedup else np.zeros(used.size, bool)
    alone_n, alone_rot = int(alone.sum()), int((alone & rot).sum())
    mw = (ctx.P + 31) // 32
    m = masks.cpu().numpy().view(np.uint32).reshape(2, ctx.I, mw)[gen & 1]
    bits = np.unpackbits(m.view(np.uint8), bitorder="little").reshape(ctx.I, mw * 32)[:, :ctx.P]
    mutated = int(bits.sum())
    per_mut = 0.5 * (R * ctx.L * 12.0) + 0.5 * (ctx.n * ctx.L * 52.0)
    shared_entries = int(uses[uses > 1].sum()) if dedup else 0
    update_bytes = ((used.size - alone_n) * 24.0 + (used_rot - alone_rot) * 72.0 + mutated * per_mut
                    + IP * 4.0 + ((IP * ctx.L * 4.0 + shared_entries * 16.0) if dedup else 0.0))
    commit_bytes = alone_n * 24.0 + alone_rot * 72.0
    return update_bytes, commit_bytes, {"used_slots": int(used.size), "used_rotation_slots": used_rot,
                                        "committed_by_fused_kernel": alone_n,
                                        "committed_rotation_slots": alone_rot,
                                        "shared_entries": shared_entries,
                                        "mutated_individuals": mutated}


def sampled_schedule(n, L):
    """(wavefronts per circuit, circuits per workgroup) of the fused QEQEA
    kernel for width n and length L (the sampled library class)."""
    from paper_1809_11134_amd import qe
    _, waves, cpb = qe.get_schedule_lib(n, 1 if L >= 32 else 0, qe.SCHED_SAMPLED)
    return waves, (cpb if waves == 1 else 1)


def secondary_qeqea_n4(dev, K, W):
    """n=4, library {I,NOT,CNOT,CV,CV+}, one QEQEA population of 4096
    circuits x 30 gates: the graph of K generations + the FP64 re-check
    (timed as the headline), and its fused kernel against the LDS peak."""
    from paper_1809_11134_amd import inputs
    w = inputs.workload_qeqea_n4()
    ctx = qeqea_context(w, dev)
    ms, times, gen, err = qeqea_graph_run(ctx, K, W, dev)
    fused_us, upd_us, gates, _ = time_generation_kernels(ctx, gen, 50, dev)
    lds = algorithmic_lds_bytes(gates.cpu().numpy(), w["n"])
    ctx.close()
    return {"workload": w["name"], "generations": K, "evals_per_s": K * w["P"] / (ms * 1e-3),
            "ms_per_generation": ms / K, "replay_ms": times, "elite_fp32_vs_fp64_max_abs_df": err,
            "fused_kernel": "population_kernel<4,{},true,false,{}>".format(*sampled_schedule(4, w["L"])),
            "fused_kernel_us": fused_us,
            "update_kernel_us": upd_us, "algorithmic_lds_bytes_per_launch": lds,
            "lds_frac": lds / (fused_us * 1e-6) / 1e9 / LDS_PEAK_GBPS,
            "traffic": traffic_from_profiles("qeqea_fused_n4", source_hash())}


def secondary_mixed_ga(dev, gens=50, reps=10):
    """256 GA populations of 64 circuits, population i on n_i ~ U{3..6}
    wires with genomes of L_i ~ U[8,64] gates of {H,T,CNOT,CV,CV+} and its
    own target (16384 evaluations per generation): the graph of `gens`
    generations (genome copy, one cost-sorted evaluation launch, the GA
    update of every population), and the evaluation launch alone against the
    LDS peak."""
    import numpy as np
    import torch
    from paper_1809_11134_amd import inputs, qe
    w = inputs.workload_mixed_ga()
    P, I = w["P"], w["instances"]
    mats = [qe.build_unitary(torch.from_numpy(tg.astype(np.int16)[None]).to(dev), n, len(tg),
                             precision=1)[0].reshape(-1)
            for n, tg in zip(w["widths"], w["target_gates"])]
    ctx = qe.Context(0, w["lib"], qe.ALG_GA, 0, P, seed=w["seed"], widths=w["widths"],
                     lengths=w["lengths"])
    ctx.set_targets(torch.cat(mats))
    hist = torch.empty((gens, I * P), dtype=torch.float32, device=dev)
    ctx.graph_prepare(gens, hist)
    ctx.run_graph(0, gens, hist)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    ctx.run_graph(gens, gens, hist)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    _, gates = ctx.sample(2 * gens)
    f = ctx.eval_population(gates)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        ctx.eval_population(gates)
    e1.record()
    torch.cuda.synchronize()
    eval_us = e0.elapsed_time(e1) / reps * 1e3
    flat = gates.cpu().numpy().view(np.uint16)
    lds, o = 0.0, 0
    for n, L in zip(w["widths"], w["lengths"]):
        lds += algorithmic_lds_bytes(flat[o:o + P * L].reshape(P, L), n)
        o += P * L
    best = max(ctx.get_best(i, with_fp64=False)[1] for i in range(I))
    ctx.close()
    return {"workload": w["name"], "generations": gens, "evals_per_s": gens * I * P / (ms * 1e-3),
            "ms_per_generation": ms / gens, "eval_kernel": "mix_kernel (cost order fixed at creation)",
            "eval_kernel_us": eval_us, "algorithmic_lds_bytes_per_launch": lds,
            "lds_frac": lds / (eval_us * 1e-6) / 1e9 / LDS_PEAK_GBPS, "best_f": best}


def secondary_uneven(dev, reps=7):
    """16384 circuits, width n ~ U{3..6} per population of 64, length
    L ~ U[8,64] per circuit, per-population targets of library
    {H,T,CNOT,CV,CV+}: one mixed-width launch."""
    import numpy as np
    import torch
    from paper_1809_11134_amd import inputs, qe
    w = inputs.workload_uneven()
    nq, goff, gates = w["nq"], w["goff"], w["gates"]
    mats, offs, off = [], [], 0
    for n, tg in w["target_gates"]:
        U = qe.build_unitary(torch.from_numpy(tg.astype(np.int16)[None]).to(dev), n, len(tg), precision=0)[0]
        mats.append(U.reshape(-1))
        offs.append(off)
        off += U.numel()
    flat = torch.cat(mats)
    toff = torch.tensor(np.array(offs)[w["target_index"]], dtype=torch.int64, device=dev)
    g = torch.from_numpy(gates.astype(np.int16)).to(dev)
    nqd, goffd = torch.from_numpy(nq).to(dev), torch.from_numpy(goff).to(dev)
    batch, keep, B = qe.make_batch(g, flat, nq=nqd, goff=goffd, toff=toff, target_stride=None)
    us, _ = _timed_eval(batch, qe.PATH_FP32, B, reps, dev)
    # the per-gate model's LDS bytes, width by width
    lds = 0.0
    for n in range(1, 7):
        rows = np.nonzero(nq == n)[0]
        if len(rows) == 0:
            continue
        flat_g = np.concatenate([gates[goff[b]:goff[b + 1]] for b in rows])
        lds += algorithmic_lds_bytes(flat_g, n) + (len(rows) - 1) * 16.0 * float(1 << (2 * n))
    return {"workload": w["name"], "circuits": len(nq), "evals_per_s": len(nq) / (us * 1e-6),
            "kernel_us": us, "algorithmic_lds_bytes": lds,
            "lds_frac": lds / (us * 1e-6) / 1e9 / LDS_PEAK_GBPS}


def main():
    global LDS_PEAK_GBPS
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--timed-replays", type=int, default=5,
                    help="timed replays of the K-generation graph (the median is reported)")
    ap.add_argument("--cpu-seconds", type=float, default=16.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel-reps", type=int, default=10)
    ap.add_argument("--pmc-calibration-mb", type=int, default=0,
                    help="after the run, copy a buffer of this many MiB (a plain copy kernel "
                         "of known traffic that scales the FETCH_SIZE / WRITE_SIZE counters)")
    ap.add_argument("--no-secondary", action="store_true",
                    help="skip the secondary workloads")
    ap.add_argument("--secondary", default="precision,qeqea_n4,uneven,mixed_ga,phase_insensitive,ising,dense",
                    help="comma list of the secondary workloads to run (precision, qeqea_n4, "
                         "uneven, mixed_ga, phase_insensitive, ising, dense)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the hot path runs on a single MI355X (independent "
              "populations would shard across GPUs with no exchange).  Run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)
    K, W = args.steps, args.warmup
    if K < 1 or W < 1:
        ap.error("--steps and --warmup must be >= 1")

    import torch
    from paper_1809_11134_amd import inputs, qe

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    qe.load()
    src = source_hash()

    # the per-gate kernels read and write every element they touch once, so
    # their LDS ceiling is the probe's copy rate (equal reads and writes)
    lds_probe = measure_lds_peak(dev)
    LDS_PEAK_GBPS = lds_probe["copy_b128"]
    log(f"LDS probe: {lds_probe} GB/s -> peak {LDS_PEAK_GBPS:.0f} GB/s for equal reads and writes "
        f"({LDS_PEAK_GBPS / LDS_SPEC_GBPS:.3f} of the unit-count figure)")

    w = inputs.workload_qeqea_n5()
    n, L, P, I = w["n"], w["L"], w["P"], w["instances"]
    log(f"workload {w['name']}: n={n} L={L} P={P} instances={I}; steps={K} warmup={W}")
    ctx = qeqea_context(w, dev)
    t0 = time.perf_counter()
    ms, times, gen, fit_err = qeqea_graph_run(ctx, K, W, dev, reps=max(1, args.timed_replays))
    wall = time.perf_counter() - t0
    assert qe.device_errors() == 0, "device error flags raised"
    value = K * I * P / (ms / 1e3)
    log(f"timed: {K} generations + elite re-check, replays {['%.3f' % t for t in times]} ms "
        f"(median {ms:.3f} ms) -> {value:.4g} evals/s")

    # the generation's two kernels, launch by launch
    R = max(1, args.kernel_reps)
    fused_us, upd_us, gates, gen = time_generation_kernels(ctx, gen, R, dev)
    gh = gates.cpu().numpy()
    flops = algorithmic_flops(gh, n)
    lds_bytes = algorithmic_lds_bytes(gh, n)
    achieved = lds_bytes / (fused_us * 1e-6) / 1e9
    alu = flops / (fused_us * 1e-6) / 1e12
    waves, cpb = sampled_schedule(n, L)
    roofline = {"bound": "lds", "achieved": round(achieved, 2), "peak": round(LDS_PEAK_GBPS, 1),
                "unit": "GB/s", "frac": round(achieved / LDS_PEAK_GBPS, 6),
                "traffic": traffic_from_profiles("qeqea_fused_n5", src),
                "kernel": f"population_kernel<5,{waves},true,false,{cpb}> (circuit construction from the "
                          f"slot words + Eq. 11 fitness + elitism of the slots a circuit alone used + "
                          f"segment max of the shared ones + mutation decisions, LDS-staged, {waves} "
                          f"wavefront(s) per circuit, {cpb} circuit(s) per workgroup)",
                "kernel_us": round(fused_us, 3), "algorithmic_lds_bytes_per_launch": lds_bytes,
                "peak_source": "LDS probe kernel in this run, copy mode (each 16-byte word read and "
                               "written once, the mix of the per-gate updates)",
                "lds_probe_gbps": lds_probe,
                "frac_of_read_peak": round(achieved / lds_probe["read_b128"], 6),
                "frac_of_unit_count_peak": round(achieved / LDS_SPEC_GBPS, 6),
                "algorithmic_flops_per_launch": flops, "alu_tflops": round(alu, 4),
                "alu_frac": round(alu / FP32_VECTOR_PEAK_TFLOPS, 6)}
    log(f"fused kernel: {fused_us:.2f} us/launch, {achieved:.1f} GB/s algorithmic LDS "
        f"({achieved / LDS_PEAK_GBPS:.3f} of the measured peak)")
    upd_bytes, commit_bytes, upd_counts = update_algorithmic_bytes(ctx, gen, dev)
    roofline["commit_hbm_bytes_per_launch"] = commit_bytes
    roofline["commit_note"] = ("elitism of the slots one circuit alone used, committed by this kernel "
                               "(24 B per slot, 72 B more per rotation slot)")
    gen += 1
    upd_ach = upd_bytes / (upd_us * 1e-6) / 1e9
    roofline_update = {"bound": "hbm", "achieved": round(upd_ach, 2), "peak": HBM_PEAK_GBPS,
                       "unit": "GB/s", "frac": round(upd_ach / HBM_PEAK_GBPS, 6),
                       "traffic": traffic_from_profiles("qeqea_update_n5", src),
                       "kernel": "qeqea_update_kernel (elitism of the slots several circuits used, mutation, "
                                 "best circuit, the next generation's shared-slot search)",
                       "kernel_us": round(upd_us, 3), "algorithmic_hbm_bytes_per_launch": upd_bytes,
                       "units": upd_counts}
    # the elitism's record work at random places (each used slot's record, and
    # a used rotation slot's qutrit record, read and written back), timed on a
    # buffer the size of the encoding; the fused kernel does most of it now,
    # on records it has just gathered
    S = n * n * L * P                # slots per population (n^2 regions of L x P, discrete library)
    acc = upd_counts["used_slots"] + upd_counts["used_rotation_slots"]
    probe = measure_record_floor(dev, I * S, acc)
    roofline_update["record_probe"] = dict(probe, accesses=acc, records=I * S)
    log(f"record probe: {probe} for {acc} records; update kernel {upd_us:.1f} us")
    for r, us in ((roofline, fused_us), (roofline_update, upd_us)):
        if r["traffic"] is not None:    # the counted HBM bytes at the measured duration
            r["traffic_gbps"] = round(r["traffic"] / (us * 1e-6) / 1e9, 2)
            r["traffic_frac_of_hbm_peak"] = round(r["traffic_gbps"] / HBM_PEAK_GBPS, 6)
    log(f"update kernel: {upd_us:.2f} us/launch, {upd_ach:.1f} GB/s algorithmic HBM "
        f"({upd_ach / HBM_PEAK_GBPS:.3f} of peak)")
    ctx.close()

    if args.pmc_calibration_mb > 0:
        nb = args.pmc_calibration_mb << 20
        src_buf = torch.ones(nb // 4, dtype=torch.float32, device=dev)
        dst_buf = torch.empty_like(src_buf)
        dst_buf.copy_(src_buf)
        torch.cuda.synchronize()
        log(f"calibration copy: {args.pmc_calibration_mb} MiB read + {args.pmc_calibration_mb} MiB written")

    secondary = None
    known = {"precision", "qeqea_n4", "uneven", "mixed_ga", "phase_insensitive", "ising", "dense"}
    which = set() if args.no_secondary else {s.strip() for s in args.secondary.split(",") if s.strip()}
    if which - known:
        ap.error(f"unknown secondary workloads: {sorted(which - known)}")
    if which:
        secondary = {}
        if "precision" in which:
            log("secondary: n=6 precision study (FP32 vs bf16/fp16 MFMA)")
            secondary["precision_n6"] = secondary_precision(dev)
        if "qeqea_n4" in which:
            log("secondary: n=4 QEQEA, one population of 4096")
            secondary["qeqea_n4"] = secondary_qeqea_n4(dev, K, W)
        if "uneven" in which:
            log("secondary: uneven batch")
            secondary["uneven"] = secondary_uneven(dev)
        if "mixed_ga" in which:
            log("secondary: mixed-width GA populations, 50-generation graph")
            secondary["mixed_ga"] = secondary_mixed_ga(dev)
        if "phase_insensitive" in which:
            log("secondary: n=4 workload with the phase-insensitive fitness")
            secondary["phase_insensitive"] = secondary_phase_insensitive(dev)
        if "ising" in which:
            log("secondary: n=4 shape with the Ising library")
            secondary["qeqea_ising_n4"] = secondary_qeqea_ising(dev)
        if "dense" in which:
            log("secondary: dense segment-matrix ablation")
            secondary["dense_ablation"] = secondary_dense(dev)
        assert qe.device_errors() == 0, "device error flags raised"

    cpu = None
    if not args.no_cpu_baseline:
        log(f"cpu baseline: oracle for ~{args.cpu_seconds:.0f} s")
        cpu = cpu_baseline(w, args.cpu_seconds)
        log(f"cpu baseline: {cpu['value']:.4g} evals/s on {cpu['cores']} threads, "
            f"{cpu['value_1core']:.4g} on one ({cpu['cpu_model']})")

    out = {
        "metric": METRIC, "value": value, "unit": "evals/s", "n_gpus": 1, "steps": K,
        "warmup": W, "ms_per_step": ms / K, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": w["name"], "n_qubits": n, "library": "I,NOT,CNOT,CV,CV+",
                   "algorithm": "QEQEA", "instances": I, "population": P, "layers": L,
                   "evals_per_generation": I * P, "path": "fp32", "graph": True,
                   "elite_fp64_recheck": 32, "timed_replays_ms": times,
                   "parallelism": "single GPU"},
        "fitness_error_fp32_vs_fp64": fit_err,
        "roofline": roofline,
        "roofline_update": roofline_update,
        "cpu_baseline": cpu,
        "secondary": secondary,
        "source_hash": src,
        "wall_s_timed_phase": round(wall, 3),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
