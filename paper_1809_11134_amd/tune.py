"""Autotuner for the schedule of the FP32 fitness path.

For each width n in 4..6 and each length class (circuits of 20 gates for
L < 32, 48 gates for L >= 32) it times every schedule libqe can run -- the
register-resident kernel, and the LDS-staged kernels with each allowed number
of wavefronts per circuit and circuits per workgroup -- on three kernel
families: qe_eval_fitness of a batch of uniform-random library circuits, the
population evaluation of a GA context, and the fused sampling + fitness
kernel of a QEQEA generation.  Timings are medians of repeated launches
between HIP events; the schedule with the smallest sum wins.  The table
(lines "n lclass lds waves cpb") goes to tune_mi355x.txt, which libqe reads
at first use (the environment variable QE_TUNE_TABLE points elsewhere,
QE_SCHEDULE overrides single widths).  Widths 1..3 always use the
one-entry-per-lane kernel.  Every LDS-staged schedule gives the same bits,
so the choice changes only speed.

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


def time_schedule(n, L, sched, reps, rng, dev, log):
    for c in (0, 1):
        qe.set_schedule_ex(n, c, *sched)
    B = {4: 4096, 5: 16384, 6: 8192}[n]
    g = torch.from_numpy(inputs.random_circuits(rng, B, n, L, 1).astype(np.int16)).to(dev)
    T = qe.build_unitary(g[:1], n, L, precision=0)[0]
    t_eval = _median_us(lambda: qe.eval_fitness(g, T, n=n, L=L), reps)
    # population evaluation of a GA context (library {H,T,CNOT,CV,CV+})
    P = 4096 if n < 6 else 1024
    ga = qe.Context(n, 1, qe.ALG_GA, L, P, 1, seed=inputs.SEED_BASE)
    ga.set_targets(qe.build_unitary(g[:1], n, L, precision=1))
    _, gg = ga.sample(0)
    t_pop = _median_us(lambda: ga.eval_population(gg), reps)
    ga.close()
    # the fused kernel of a QEQEA generation (library {I,NOT,CNOT,CV,CV+})
    tg = torch.from_numpy(inputs.random_target_gates(rng, n, 12, permutation=True).astype(np.int16)[None]).to(dev)
    ctx = qe.Context(n, 0, qe.ALG_QEQEA, L, P, 1, prob_mutation=0.1, mutation_range=math.pi / 4,
                     seed=inputs.SEED_BASE)
    ctx.set_targets(qe.build_unitary(tg, n, tg.shape[1], precision=1))
    s, gq, f = ctx.sample_eval(0)
    t_fused = _median_us(lambda: ctx.sample_eval(1, s, gq, f), reps)
    ctx.close()
    log(f"n={n} L={L} schedule lds={sched[0]} waves={sched[1]} cpb={sched[2]}: eval {t_eval:.1f} us, "
        f"population {t_pop:.1f} us, fused {t_fused:.1f} us")
    return t_eval + t_pop + t_fused


def sweep(reps=7, log=print):
    dev = torch.device("cuda", 0)
    table = {}
    for n in (4, 5, 6):
        for lclass, L in LENGTHS.items():
            times = {}
            for sched in CANDIDATES[n]:
                rng = np.random.default_rng(inputs.SEED_BASE + 77 + 10 * n + lclass)
                times[sched] = time_schedule(n, L, sched, reps, rng, dev, log)
            best = min(times, key=times.get)
            table[(n, lclass)] = (best, times)
    return table


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(HERE, "tune_mi355x.txt"))
    ap.add_argument("--reps", type=int, default=7)
    args = ap.parse_args()
    qe.load()
    table = sweep(args.reps, log=lambda m: print(m, flush=True))
    lines = ["# libqe FP32 schedule: n lclass lds waves cpb",
             "#   lclass 0: L < 32, 1: L >= 32; lds 1 = LDS-staged, 0 = register-resident;",
             "#   waves = wavefronts per circuit; cpb = circuits per workgroup (one-wavefront kernels)",
             "# written by paper_1809_11134_amd/tune.py on " + torch.cuda.get_device_name(0) +
             " (sum of the eval, population and fused-kernel medians per schedule, us)"]
    for (n, lclass), (best, times) in sorted(table.items()):
        alt = ", ".join(f"{s[0]}/{s[1]}/{s[2]}: {t:.1f}" for s, t in times.items())
        lines.append(f"{n} {lclass} {best[0]} {best[1]} {best[2]}   # {alt}")
    with open(args.out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


if __name__ == "__main__":
    sys.exit(main())
