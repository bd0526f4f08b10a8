"""Autotuner for the schedule of the FP32 fitness path.

The schedule is chosen per width n in 4..6, length class (circuits of 20
gates stand for L < 32, of 48 gates for L >= 32) and library class:

* discrete (qe.SCHED_DISCRETE): circuits given in a discrete library, timed
  as qe_eval_fitness of uniform-random {H, T, CNOT, CV, CV+} circuits plus
  the population evaluation of a GA context over that library;
* sampled (qe.SCHED_SAMPLED): circuits the QEQEA sampler decodes, timed as
  the fused sampling + fitness kernel of a QEQEA generation over
  {I, NOT, CNOT, CV, CV+};
* Ising (qe.SCHED_ISING): circuits of the Ising library with angled gates,
  timed as qe_eval_fitness of random Ising circuits plus the fused kernel of
  a QEQEA generation over the Ising library.

Every schedule libqe can run for the class is timed -- the register-resident
kernel (not for angled circuits, which always take the LDS-staged kernels),
and the LDS-staged kernels with each allowed number of wavefronts per circuit
and circuits per workgroup; timings are medians of repeated launches between
HIP events, and the schedule with the smallest sum wins (libqe's default
when it is within 2 %, the run-to-run noise).  The table (lines
"n lclass lib lds waves cpb", then "mfma n lclass min_block": the
fewest gates a fused MFMA block needs, smaller groups going gate by gate
in FP32) goes to tune_mi355x.txt, which libqe reads at
first use (QE_TUNE_TABLE points elsewhere, QE_SCHEDULE overrides single
widths).  Widths 1..3 always use the one-entry-per-lane kernel.  Every
LDS-staged schedule gives the same bits, so the choice changes only speed.

    python -m paper_1809_11134_amd.tune [--out PATH]
"""
import argparse
import math
import os
import sys

import numpy as np
import torch

from . import inputs, qe

HERE = os.path.dirname(os.path.abspath(__file__))

# (lds, waves, cpb) per width: the register kernel, then the LDS schedules
CANDIDATES = {4: [(0, 1, 4), (1, 1, 4), (1, 1, 1)],
              5: [(0, 1, 4), (1, 1, 4), (1, 1, 1), (1, 2, 1)],
              6: [(0, 4, 1), (1, 4, 1)]}
LENGTHS = {0: 20, 1: 48}
DEFAULT = {4: (1, 1, 4), 5: (1, 1, 4), 6: (1, 4, 1)}    # libqe's built-in schedule
TIE = 0.02
CLASSES = {qe.SCHED_DISCRETE: "discrete", qe.SCHED_SAMPLED: "sampled", qe.SCHED_ISING: "ising"}


def _median_us(fn, reps):
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


def _qeqea_fused_us(n, L, P, library, reps, rng, dev):
    tg = torch.from_numpy(inputs.random_target_gates(rng, n, 12, permutation=True).astype(np.int16)[None]).to(dev)
    ctx = qe.Context(n, library, qe.ALG_QEQEA, L, P, 1, prob_mutation=0.1, mutation_range=math.pi / 4,
                     seed=inputs.SEED_BASE)
    ctx.set_targets(qe.build_unitary(tg, n, tg.shape[1], precision=1))
    out = ctx.sample_eval(0)
    if library == qe.LIB_ISING:
        s, gq, a, f = out
        t = _median_us(lambda: ctx.sample_eval(1, s, gq, f, angles=a), reps)
    else:
        s, gq, f = out
        t = _median_us(lambda: ctx.sample_eval(1, s, gq, f), reps)
    ctx.close()
    return t


def time_schedule(n, L, cls, sched, reps, rng, dev, log):
    """Summed median time (us) of the class's kernels under one schedule."""
    for c in (0, 1):
        qe.set_schedule_lib(n, c, cls, *sched)
    P = 4096 if n < 6 else 1024
    parts = {}
    if cls == qe.SCHED_DISCRETE:
        B = {4: 4096, 5: 16384, 6: 8192}[n]
        g = torch.from_numpy(inputs.random_circuits(rng, B, n, L, 1).astype(np.int16)).to(dev)
        T = qe.build_unitary(g[:1], n, L, precision=0)[0]
        parts["eval"] = _median_us(lambda: qe.eval_fitness(g, T, n=n, L=L), reps)
        ga = qe.Context(n, 1, qe.ALG_GA, L, P, 1, seed=inputs.SEED_BASE)
        ga.set_targets(qe.build_unitary(g[:1], n, L, precision=1))
        _, gg = ga.sample(0)
        parts["population"] = _median_us(lambda: ga.eval_population(gg), reps)
        ga.close()
    elif cls == qe.SCHED_SAMPLED:
        parts["fused"] = _qeqea_fused_us(n, L, P, qe.LIB_NCV, reps, rng, dev)
    else:
        B = {4: 4096, 5: 8192, 6: 2048}[n]
        g, a = inputs.random_ising_circuits(rng, B, n, L, discrete_frac=0.0)
        gd = torch.from_numpy(np.ascontiguousarray(g).view(np.int16)).to(dev)
        ad = torch.from_numpy(np.ascontiguousarray(a).view(np.int32)).to(dev)
        T = qe.build_unitary(gd[:1], n, L, precision=0, angles=ad[:1])[0]
        parts["eval"] = _median_us(lambda: qe.eval_fitness(gd, T, n=n, L=L, angles=ad), reps)
        parts["fused"] = _qeqea_fused_us(n, L, P, qe.LIB_ISING, reps, rng, dev)
    log(f"n={n} L={L} {CLASSES[cls]} schedule lds={sched[0]} waves={sched[1]} cpb={sched[2]}: " +
        ", ".join(f"{k} {v:.1f} us" for k, v in parts.items()))
    return sum(parts.values())


def candidates(n, cls):
    c = CANDIDATES[n]
    return [s for s in c if s[0] == 1] if cls == qe.SCHED_ISING else c


def sweep(reps=7, log=print, widths=(4, 5, 6)):
    dev = torch.device("cuda", 0)
    saved = {(n, c, k): qe.get_schedule_lib(n, c, k) for n in widths for c in (0, 1) for k in CLASSES}
    table = {}
    try:
        for n in widths:
            for lclass, L in LENGTHS.items():
                for cls in CLASSES:
                    times = {}
                    for sched in candidates(n, cls):
                        rng = np.random.default_rng(inputs.SEED_BASE + 77 + 10 * n + lclass)
                        times[sched] = time_schedule(n, L, cls, sched, reps, rng, dev, log)
                    best = min(times, key=times.get)
                    # within TIE of the best, the default schedule is kept (the
                    # differences are run-to-run noise)
                    if times.get(DEFAULT[n], math.inf) <= (1.0 + TIE) * times[best]:
                        best = DEFAULT[n]
                    table[(n, lclass, cls)] = (best, times)
    finally:
        for (n, c, k), v in saved.items():
            qe.set_schedule_lib(n, c, k, *v)
    return table


MFMA_MIN_BLOCK = (1, 2, 3, 4, 5, 6, 8)


def sweep_mfma(reps=7, log=print, widths=(5, 6)):
    """Fewest gates of a fused MFMA block (smaller groups go gate by gate in
    FP32), per width and length class: qe_eval_fitness of uniform-random
    {H, T, CNOT, CV, CV+} circuits on the BF16 MFMA path."""
    dev = torch.device("cuda", 0)
    saved = {(n, c): qe.get_mfma_min_block(n, c) for n in widths for c in (0, 1)}
    table = {}
    try:
        for n in widths:
            for lclass, L in LENGTHS.items():
                rng = np.random.default_rng(inputs.SEED_BASE + 91 + 10 * n + lclass)
                B = {5: 16384, 6: 8192}[n]
                g = torch.from_numpy(inputs.random_circuits(rng, B, n, L, 1).astype(np.int16)).to(dev)
                T = qe.build_unitary(g[:1], n, L, precision=0)[0]
                times = {}
                for mb in MFMA_MIN_BLOCK:
                    qe.set_mfma_min_block(n, lclass, mb)
                    times[mb] = _median_us(lambda: qe.eval_fitness(g, T, n=n, L=L, path=qe.PATH_MFMA_BF16), reps)
                    log(f"n={n} L={L} mfma min_block={mb}: {times[mb]:.1f} us")
                table[(n, lclass)] = (min(times, key=times.get), times)
    finally:
        for (n, c), v in saved.items():
            qe.set_mfma_min_block(n, c, v)
    return table


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(HERE, "tune_mi355x.txt"))
    ap.add_argument("--reps", type=int, default=7)
    args = ap.parse_args()
    qe.load()
    table = sweep(args.reps, log=lambda m: print(m, flush=True))
    lines = ["# libqe FP32 schedule: n lclass lib lds waves cpb",
             "#   lclass 0: L < 32, 1: L >= 32; lib 0: discrete library, 1: QEQEA-sampled, 2: Ising;",
             "#   lds 1 = LDS-staged, 0 = register-resident; waves = wavefronts per circuit;",
             "#   cpb = circuits per workgroup (one-wavefront population kernels)",
             "# written by paper_1809_11134_amd/tune.py on " + torch.cuda.get_device_name(0) +
             " (sum of the class's kernel medians per schedule, us)"]
    for (n, lclass, cls), (best, times) in sorted(table.items()):
        alt = ", ".join(f"{s[0]}/{s[1]}/{s[2]}: {t:.1f}" for s, t in times.items())
        lines.append(f"{n} {lclass} {cls} {best[0]} {best[1]} {best[2]}   # {CLASSES[cls]}: {alt}")
    mt = sweep_mfma(args.reps, log=lambda m: print(m, flush=True))
    lines.append("# MFMA paths: mfma n lclass min_block (groups of fewer gates go gate by gate in FP32)")
    for (n, lclass), (best, times) in sorted(mt.items()):
        alt = ", ".join(f"{mb}: {t:.1f}" for mb, t in times.items())
        lines.append(f"mfma {n} {lclass} {best}   # bf16 eval us: {alt}")
    with open(args.out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


if __name__ == "__main__":
    sys.exit(main())
