"""Builds libqe.so (the HIP kernels and the C ABI) for gfx950 with hipcc.

Flags:
  -ffp-contract=off
      one rounding per floating-point operation: the encoding updates and the
      measurement must reproduce the oracle bit for bit;
  -Xclang -target-feature -Xclang -packed-fp32-ops
      no packed FP32 instructions are generated;
  -mllvm -simplifycfg-sink-common=false
      keeps the per-gate dispatch of the register-resident kernels from being
      merged into pointer phis (which would demote the matrix to scratch).
"""
import concurrent.futures
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libqe.so")
SOURCES = ["qe_api.hip", "qe_eval.hip", "qe_loop.hip", "qe_mfma.hip", "qe_dense.hip", "qe_probe.hip"]
ARCH = os.environ.get("QE_OFFLOAD_ARCH", "gfx950")

FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-mllvm", "-simplifycfg-sink-common=false",
         "-I", os.path.join(ROOT, "include"), "-Wall"]


# host code under AddressSanitizer and UndefinedBehaviorSanitizer (the device
# code is built as usual): libqe_san.so, for the sanitizer test on the CPU
SAN_LIB = os.path.join(HERE, "libqe_san.so")
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]


def _compile(src, obj, verbose, extra=()):
    cmd = ["hipcc", *FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    msgs = [l for l in (r.stderr or "").splitlines() if "packed-fp32-ops" not in l]
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n" + "\n".join(msgs))
    return obj


def build(verbose: bool = False, sanitize: bool = False) -> str:
    objdir = os.path.join(HERE, "_build_san" if sanitize else "_build")
    out = SAN_LIB if sanitize else LIB
    extra = SAN_FLAGS if sanitize else ()
    os.makedirs(objdir, exist_ok=True)
    objs = [os.path.join(objdir, s.replace(".hip", ".o")) for s in SOURCES]
    with concurrent.futures.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        list(ex.map(lambda so: _compile(so[0], so[1], verbose, extra), zip(SOURCES, objs)))
    tmp = out + ".tmp"
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", *extra, *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
