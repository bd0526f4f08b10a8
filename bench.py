#!/usr/bin/env python3
"""Throughput of the QEQEA circuit-fitness hot path on one MI355X.

Workload (seeded, synthetic): n = 4 wires, library {I, NOT, CNOT, CV, CV+},
one QEQEA population whose encoding is sampled into P = 4096 circuits of
L = 30 gates per generation; target = a random reversible permutation built
from 12 NOT/CNOT gates (the paper's targets are small reversible gates).
A step is one generation of the whole hot path: circuit construction by
sampling (Sec. IV-D), Eq. 11 fitness of all P circuits (FP32), segment
fitness / elitism / adaptive mutation (Secs. IV-E.1, IV-F).  The K timed
generations run as one HIP graph; the final FP64 re-check of the last
generation's 32 best circuits is inside the timed region.

Prints one JSON line (the metric is circuit-fitness evaluations per second)
with a roofline entry for the dominant kernel (the fused sampling + fitness
kernel, timed per launch with HIP events) and the CPU oracle's rate on a
bounded sample of the same workload.  The "secondary" object adds the other
workloads of the study: the n=6 precision study (FP32 against the bf16/fp16
hi+lo MFMA paths, with their fitness error against the FP64 path, elite
top-32 agreement and Kendall tau), 1024 QEQEA populations at n=5, and an
uneven batch of widths 3..6 in one launch.
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
LDS_PEAK_GBPS = 256 * 128 * 2.4   # MI355X LDS: 256 CUs x 128 B/clock x 2.4 GHz = 78643 GB/s


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


def cpu_baseline(w, T, seconds):
    """The oracle (test infrastructure) on a bounded sample of the workload:
    whole generations -- sampling, FP64 fitness of all P circuits (OpenMP
    over circuits), update -- until `seconds` of wall time have passed."""
    import numpy as np
    from oracle import oracle as O
    n, L, P = w["n"], w["L"], w["P"]
    st = O.QeqeaState(n, L, P, 1, w["seed"])
    nq = np.full(P, n, np.int8)
    goff = np.arange(P + 1, dtype=np.int32) * L
    toff = np.zeros(P, np.int64)
    gens = 0
    t0 = time.perf_counter()
    while True:
        slots, gates = st.sample(gens)
        out = O.eval_batch(nq, goff, gates.ravel(), toff, T)
        st.update(gens, 0.1, math.pi / 4, slots, out[:, 0].astype(np.float32))
        gens += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    return dict(value=gens * P / el, unit="evals/s", cores=O.num_threads(), kind="oracle",
                sample=f"{gens} whole QEQEA generations of the n=4, P={P}, L={L} workload "
                       f"({gens * P} circuit evaluations in FP64 over OpenMP threads, sampling "
                       f"and update single-threaded), {el:.1f} s")


def _timed_eval(batch, path, B, reps, dev):
    """Median duration of one qe_eval_fitness launch (preallocated output,
    launched through the C ABI), and the output."""
    import ctypes

    import torch
    from paper_1809_11134_amd import qe
    f = torch.empty(B, dtype=torch.float32, device=dev)
    launch = lambda: qe._call("qe_eval_fitness", None, ctypes.byref(batch), path, qe._ptr(f), None,
                              None, qe._stream(None))
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
    for name, path in (("fp32", qe.PATH_FP32), ("bf16_mfma", qe.PATH_MFMA_BF16),
                       ("fp16_mfma", qe.PATH_MFMA_FP16), ("bf16_mfma_no_renorm", qe.PATH_MFMA_BF16_RAW),
                       ("fp16_mfma_no_renorm", qe.PATH_MFMA_FP16_RAW)):
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


def secondary_qeqea_n5(dev, gens=20):
    """n=5, library {I,NOT,CNOT,CV,CV+}, 1024 QEQEA populations x 64 circuits x
    40 gates (65536 evaluations per generation): a graph of `gens` whole
    generations plus the FP64 re-check of each population's 32 best."""
    import numpy as np
    import torch
    from paper_1809_11134_amd import inputs, qe
    w = inputs.workload_qeqea_n5()
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
    idx, f64 = ctx.elite_recheck(None, hist[gens - 1], 32)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    f32 = hist[gens - 1].view(I, P).gather(1, idx.long()).double()
    best = [ctx.get_best(i, with_fp64=False)[1] for i in range(4)]
    # the fused sampling + fitness kernel alone, against the LDS peak
    slots, gates, fk = ctx.sample_eval(2 * gens)
    torch.cuda.synchronize()
    reps = 10
    e0.record()
    for r in range(reps):
        ctx.sample_eval(2 * gens + 1 + r, slots, gates, fk)
    e1.record()
    torch.cuda.synchronize()
    kern_ms = e0.elapsed_time(e1) / reps
    lds = algorithmic_lds_bytes(gates.cpu().numpy(), n)
    ctx.close()
    return {"workload": w["name"], "generations": gens, "evals_per_s": gens * I * P / (ms * 1e-3),
            "ms_per_generation": ms / gens, "elite_fp32_vs_fp64_max_abs_df": float((f32 - f64).abs().max()),
            "best_f_first_populations": best,
            "fused_kernel": "population_kernel<5,2,true,false>", "fused_kernel_us": kern_ms * 1e3,
            "algorithmic_lds_bytes_per_launch": lds,
            "lds_frac": lds / (kern_ms * 1e-3) / 1e9 / LDS_PEAK_GBPS}


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
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel-reps", type=int, default=50)
    ap.add_argument("--pmc-calibration-mb", type=int, default=0,
                    help="after the run, copy a buffer of this many MiB (a plain copy kernel "
                         "of known traffic that scales the FETCH_SIZE / WRITE_SIZE counters)")
    ap.add_argument("--no-secondary", action="store_true",
                    help="skip the secondary workloads")
    ap.add_argument("--secondary", default="precision,qeqea_n5,uneven,phase_insensitive,ising,dense",
                    help="comma list of the secondary workloads to run (precision, qeqea_n5, "
                         "uneven, phase_insensitive, ising, dense)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the hot path runs on a single MI355X (independent "
              "populations would shard across GPUs with no exchange).  Run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)
    K, W = args.steps, args.warmup
    if K < 1 or W < 1:
        ap.error("--steps and --warmup must be >= 1")

    import numpy as np
    import torch
    from paper_1809_11134_amd import inputs, qe

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    qe.load()
    w = inputs.workload_qeqea_n4()
    n, L, P, I = w["n"], w["L"], w["P"], w["instances"]
    log(f"workload {w['name']}: n={n} L={L} P={P} instances={I}; steps={K} warmup={W}")

    tg = torch.from_numpy(np.stack(w["target_gates"]).astype(np.int16)).to(dev)
    T = qe.build_unitary(tg, n, tg.shape[1], precision=1)          # [I, N, N] complex128
    ctx = qe.Context(n, w["lib"], qe.ALG_QEQEA, L, P, I, prob_mutation=0.1,
                     mutation_range=math.pi / 4, seed=w["seed"])
    ctx.set_targets(T)
    f_warm = torch.empty((W, I * P), dtype=torch.float32, device=dev)
    f_hist = torch.empty((K, I * P), dtype=torch.float32, device=dev)
    ctx.graph_prepare(W, f_warm)
    ctx.graph_prepare(K, f_hist)
    ctx.run_graph(0, W, f_warm)
    torch.cuda.synchronize()
    log("warmup done")

    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record()
    ctx.run_graph(W, K, f_hist)
    idx, f64 = ctx.elite_recheck(None, f_hist[K - 1], 32)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    assert qe.device_errors() == 0, "device error flags raised"
    value = K * I * P / (ms / 1e3)
    log(f"timed: {K} generations in {ms:.3f} ms (wall {wall * 1e3:.3f} ms) -> {value:.4g} evals/s")

    # FP32 vs FP64 fitness error on the re-checked elites of the last generation
    f32_el = f_hist[K - 1].view(I, P).gather(1, idx.long()).double()
    fit_err = float((f32_el - f64).abs().max().item())

    # dominant kernel: fused sampling + fitness, timed launch by launch
    R = max(1, args.kernel_reps)
    slots = torch.empty((I * P, L), dtype=torch.int32, device=dev)
    gates = torch.empty((I * P, L), dtype=torch.int16, device=dev)
    fk = torch.empty(I * P, dtype=torch.float32, device=dev)
    # R launches back to back on the current stream between two events: the
    # average duration per launch, as a kernel trace reports it
    k0 = torch.cuda.Event(enable_timing=True)
    k1 = torch.cuda.Event(enable_timing=True)
    ctx.sample_eval(W + K, slots, gates, fk)
    torch.cuda.synchronize()
    k0.record()
    for r in range(R):
        ctx.sample_eval(W + K + r, slots, gates, fk)
    k1.record()
    torch.cuda.synchronize()
    kern_ms = k0.elapsed_time(k1) / R
    gh = gates.cpu().numpy()
    flops = algorithmic_flops(gh, n)
    lds_bytes = algorithmic_lds_bytes(gh, n)
    achieved = lds_bytes / (kern_ms / 1e3) / 1e9
    alu = flops / (kern_ms / 1e3) / 1e12
    src = source_hash()
    roofline = {"bound": "lds", "achieved": round(achieved, 2), "peak": round(LDS_PEAK_GBPS, 1),
                "unit": "GB/s", "frac": round(achieved / LDS_PEAK_GBPS, 6),
                "traffic": traffic_from_profiles("qeqea_fused_n4", src),
                "kernel": "population_kernel<4,1,true,false> (sampling + Eq. 11 fitness + segment max, LDS-staged)",
                "kernel_ms": round(kern_ms, 6), "algorithmic_lds_bytes_per_launch": lds_bytes,
                "algorithmic_flops_per_launch": flops, "alu_tflops": round(alu, 4),
                "alu_frac": round(alu / FP32_VECTOR_PEAK_TFLOPS, 6)}
    log(f"dominant kernel: {kern_ms * 1e3:.2f} us/launch, {achieved:.1f} GB/s algorithmic LDS "
        f"({achieved / LDS_PEAK_GBPS:.3f} of peak), {alu:.3f} TFLOP/s")

    if args.pmc_calibration_mb > 0:
        nb = args.pmc_calibration_mb << 20
        src_buf = torch.ones(nb // 4, dtype=torch.float32, device=dev)
        dst_buf = torch.empty_like(src_buf)
        dst_buf.copy_(src_buf)
        torch.cuda.synchronize()
        log(f"calibration copy: {args.pmc_calibration_mb} MiB read + {args.pmc_calibration_mb} MiB written")

    secondary = None
    which = set() if args.no_secondary else {s.strip() for s in args.secondary.split(",") if s.strip()}
    unknown = which - {"precision", "qeqea_n5", "uneven", "phase_insensitive", "ising", "dense"}
    if unknown:
        ap.error(f"unknown secondary workloads: {sorted(unknown)}")
    if which:
        secondary = {}
        if "precision" in which:
            log("secondary: n=6 precision study (FP32 vs bf16/fp16 MFMA)")
            secondary["precision_n6"] = secondary_precision(dev)
        if "qeqea_n5" in which:
            log("secondary: n=5 QEQEA, 1024 populations")
            secondary["qeqea_n5"] = secondary_qeqea_n5(dev)
        if "uneven" in which:
            log("secondary: uneven batch")
            secondary["uneven"] = secondary_uneven(dev)
        if "phase_insensitive" in which:
            log("secondary: bench workload with the phase-insensitive fitness")
            secondary["phase_insensitive"] = secondary_phase_insensitive(dev)
        if "ising" in which:
            log("secondary: bench shape with the Ising library")
            secondary["qeqea_ising_n4"] = secondary_qeqea_ising(dev)
        if "dense" in which:
            log("secondary: dense segment-matrix ablation")
            secondary["dense_ablation"] = secondary_dense(dev)
        assert qe.device_errors() == 0, "device error flags raised"

    cpu = None
    if not args.no_cpu_baseline:
        log(f"cpu baseline: oracle for ~{args.cpu_seconds:.0f} s")
        Th = T[0].cpu().numpy()
        cpu = cpu_baseline(w, Th, args.cpu_seconds)
        log(f"cpu baseline: {cpu['value']:.4g} evals/s on {cpu['cores']} threads")

    out = {
        "metric": METRIC, "value": value, "unit": "evals/s", "n_gpus": 1, "steps": K,
        "warmup": W, "ms_per_step": ms / K, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": w["name"], "n_qubits": n, "library": "I,NOT,CNOT,CV,CV+",
                   "algorithm": "QEQEA", "population": P, "layers": L, "instances": I,
                   "path": "fp32", "graph": True, "elite_fp64_recheck": 32,
                   "parallelism": "single GPU"},
        "fitness_error_fp32_vs_fp64": fit_err,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "secondary": secondary,
        "source_hash": src,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
