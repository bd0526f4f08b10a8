"""Autotuner for the per-width schedule of the FP32 fitness path.

For each width n in 4..6 it times qe_eval_fitness with the register-resident
and the LDS-staged kernels (HIP events, median of repeated launches) on
representative batches -- uniform-random library circuits of 20 and 48 gates
-- and the fused QEQEA generation kernel for library 0, and writes the faster
choice per width to tune_mi355x.txt (read by libqe at first use; the
environment variable QE_TUNE_TABLE points elsewhere, QE_SCHEDULE overrides
single entries).  Widths 1..3 always use the one-entry-per-lane kernel.

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


def sweep(reps=9, log=print):
    dev = torch.device("cuda", 0)
    rng = np.random.default_rng(inputs.SEED_BASE + 77)
    table = {}
    for n in (4, 5, 6):
        B = {4: 4096, 5: 16384, 6: 8192}[n]
        totals = {0: 0.0, 1: 0.0}
        for L, lib in ((20, 0), (48, 1)):
            g = torch.from_numpy(inputs.random_circuits(rng, B, n, L, lib).astype(np.int16)).to(dev)
            T = qe.build_unitary(g[:1], n, L, precision=0)[0]
            for lds, path in ((0, qe.PATH_FP32_REG), (1, qe.PATH_FP32_LDS)):
                t = _median_us(lambda: qe.eval_fitness(g, T, n=n, L=L, path=path), reps)
                totals[lds] += t
                log(f"n={n} B={B} L={L} lib={lib} {'lds' if lds else 'reg'}: {t:.2f} us")
        # the fused sampling + fitness kernel of a QEQEA generation
        P, L = 1024 if n == 6 else 4096, 30
        tg = torch.from_numpy(inputs.random_target_gates(rng, n, 12, permutation=True).astype(np.int16)[None]).to(dev)
        Tq = qe.build_unitary(tg, n, tg.shape[1], precision=1)
        for lds in (0, 1):
            qe.set_schedule(n, lds)
            ctx = qe.Context(n, 0, qe.ALG_QEQEA, L, P, 1, prob_mutation=0.1,
                             mutation_range=math.pi / 4, seed=inputs.SEED_BASE)
            ctx.set_targets(Tq)
            s, gg, f = ctx.sample_eval(0)
            t = _median_us(lambda: ctx.sample_eval(1, s, gg, f), reps)
            totals[lds] += t
            log(f"n={n} fused QEQEA P={P} L={L} {'lds' if lds else 'reg'}: {t:.2f} us")
            ctx.close()
        table[n] = (1 if totals[1] <= totals[0] else 0, totals)
    return table


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(HERE, "tune_mi355x.txt"))
    ap.add_argument("--reps", type=int, default=9)
    args = ap.parse_args()
    qe.load()
    table = sweep(args.reps, log=lambda m: print(m, flush=True))
    lines = ["# libqe FP32 schedule per width: n lds (1 = LDS-staged, 0 = register-resident)",
             "# written by paper_1809_11134_amd/tune.py on " + torch.cuda.get_device_name(0)]
    for n in range(1, 7):
        if n in table:
            lds, tot = table[n]
            lines.append(f"{n} {lds}   # summed medians: register {tot[0]:.1f} us, LDS {tot[1]:.1f} us")
        else:
            lines.append(f"{n} 0   # one entry per lane")
    with open(args.out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


if __name__ == "__main__":
    sys.exit(main())
