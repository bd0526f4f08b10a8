"""Named-target convergence runs (the shape of the paper's experiments,
Sec. VI and Table III): the QEQEA and the classical GA search a circuit of
the gate library equal to a textbook reversible gate, and the best fitness
is reported against the generation count.

Targets (wire 0 = most significant bit of a basis index, as in Eqs. 1-2; the
paper's named targets put the target bit on wire 0):
  cnot   (n=2): wire 0 ^= wire 1
  toffoli(n=3): wire 0 ^= wire 1 & wire 2
  peres  (n=3): wire 0 ^= wire 1 & wire 2, then wire 2 ^= wire 1
  cccnot (n=4): wire 0 ^= wire 1 & wire 2 & wire 3

Every generation runs on the GPU through libqe (HIP graphs of whole
generations); this module only builds the targets and records the results.

    python -m paper_1809_11134_amd.experiments --targets cnot,toffoli,peres

With --library ising the QEQEA searches the Ising gate model of Sec. III
(rotations about x, y, z and the interaction J, continuous angles), the
model of the paper's own runs; Table I's configuration is

    python -m paper_1809_11134_amd.experiments --targets cnot --algorithms qeqea \
        --library ising --L 3 --P 1
"""
import argparse
import json
import math
import sys
import time

import numpy as np
import torch

from . import qe


def _perm_unitary(n, fn):
    N = 1 << n
    U = np.zeros((N, N), np.complex128)
    for i in range(N):
        U[fn(i), i] = 1.0
    return U


def _bits(i, n):
    return [(i >> (n - 1 - w)) & 1 for w in range(n)]     # wire 0 first


def _from_bits(b):
    v = 0
    for x in b:
        v = (v << 1) | x
    return v


def _cnot(i):
    b = _bits(i, 2)
    b[0] ^= b[1]
    return _from_bits(b)


def _toffoli(i):
    b = _bits(i, 3)
    b[0] ^= b[1] & b[2]
    return _from_bits(b)


def _peres(i):
    b = _bits(i, 3)
    b[0] ^= b[1] & b[2]
    b[2] ^= b[1]
    return _from_bits(b)


def _cccnot(i):
    b = _bits(i, 4)
    b[0] ^= b[1] & b[2] & b[3]
    return _from_bits(b)


TARGETS = {"cnot": (2, _cnot), "toffoli": (3, _toffoli), "peres": (3, _peres), "cccnot": (4, _cccnot)}


def target_unitary(name):
    n, fn = TARGETS[name]
    return n, _perm_unitary(n, fn)


def run(name, algorithm, L, P, generations, chunk=50, fitness_mode=qe.FIT_PHASE_INSENSITIVE,
        seed=1809111340, pm=0.1, mutation_range=math.pi / 4, thresholds=(0.9, 0.99, 1.0),
        dev=None, library=qe.LIB_NCV):
    """One search; returns a dict with the best fitness after every chunk of
    generations and the first generation (upper bound, in chunks) at which
    the best fitness reached each threshold.  library: qe.LIB_NCV or (QEQEA
    only) qe.LIB_ISING, the gate model of the paper's own runs."""
    dev = dev or torch.device("cuda", torch.cuda.current_device())
    n, T = target_unitary(name)
    ctx = qe.Context(n, library, algorithm, L, P, 1, prob_mutation=pm,
                     mutation_range=mutation_range, seed=seed, fitness_mode=fitness_mode)
    ctx.set_targets(torch.from_numpy(T[None]).to(dev))
    curve, reached = [], {}
    gen = 0
    t0 = time.perf_counter()
    while gen < generations:
        g = min(chunk, generations - gen)
        ctx.run_graph(gen, g)
        gen += g
        gates, f32, _ = ctx.get_best(0, with_fp64=False)
        curve.append((gen, f32))
        for th in thresholds:
            if th not in reached and f32 >= th - 1e-6:
                reached[th] = gen
        if f32 >= 1.0 - 1e-6:
            break
    seconds = time.perf_counter() - t0
    gates, f32, f64, angles = ctx.get_best(0, with_angles=True)
    ctx.close()
    if library == qe.LIB_ISING:
        # (kind, wire, second wire, theta in radians) per gate
        best = [(g & 15, (g >> 4) & 15, (g >> 8) & 15, round(a * 2 * math.pi / 2 ** 32, 6))
                for g, a in zip(gates, angles)]
    else:
        best = [g for g in gates if g & 15]
    return {"target": name, "n": n, "algorithm": "QEQEA" if algorithm == qe.ALG_QEQEA else "GA",
            "library": "ising" if library == qe.LIB_ISING else "ncv",
            "fitness": "phase_insensitive" if fitness_mode == qe.FIT_PHASE_INSENSITIVE else "eq11",
            "L": L, "P": P, "generations": gen, "seconds": seconds, "best_f_fp32": f32,
            "best_f_fp64": f64, "best_circuit": best,
            "first_generation_reaching": {str(k): v for k, v in sorted(reached.items())},
            "curve": curve}


def main(argv=None):
    ap = argparse.ArgumentParser(description="named-target convergence runs (QEQEA vs GA)")
    ap.add_argument("--targets", default="cnot,toffoli,peres,cccnot")
    ap.add_argument("--algorithms", default="qeqea,ga")
    ap.add_argument("--generations", type=int, default=2000)
    ap.add_argument("--P", type=int, default=256)
    ap.add_argument("--L", type=int, default=0, help="circuit length (0: 4 + 4 n)")
    ap.add_argument("--fitness", choices=("phase_insensitive", "eq11"), default="phase_insensitive")
    ap.add_argument("--library", choices=("ncv", "ising"), default="ncv",
                    help="gate library of the QEQEA (the GA runs on ncv only)")
    ap.add_argument("--chunk", type=int, default=50, help="generations between best-fitness reads")
    ap.add_argument("--seed", type=int, default=1809111340)
    args = ap.parse_args(argv)
    if not torch.cuda.is_available():
        print("the convergence runs need a GPU", file=sys.stderr)
        return 2
    qe.load()
    mode = qe.FIT_PHASE_INSENSITIVE if args.fitness == "phase_insensitive" else qe.FIT_EQ11
    for name in [t for t in args.targets.split(",") if t]:
        n = TARGETS[name][0]
        L = args.L or 4 + 4 * n
        lib = qe.LIB_ISING if args.library == "ising" else qe.LIB_NCV
        for alg in [a for a in args.algorithms.split(",") if a]:
            if alg == "ga" and lib == qe.LIB_ISING:
                continue
            r = run(name, qe.ALG_QEQEA if alg == "qeqea" else qe.ALG_GA, L, args.P,
                    args.generations, chunk=args.chunk, fitness_mode=mode, seed=args.seed,
                    library=lib)
            print(json.dumps(r), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
