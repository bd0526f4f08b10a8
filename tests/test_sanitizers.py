"""CPU sanitizer runs: the C oracle built with AddressSanitizer and
UndefinedBehaviorSanitizer (gcc) under the oracle's own pin tests, and the
host side of libqe built with them (clang, device code unchanged) under the
C-ABI tests that need no GPU (argument validation, exports, library tables).
Every finding aborts the child process, which fails the test."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _stale(lib, sources):
    return not os.path.exists(lib) or any(os.path.getmtime(s) > os.path.getmtime(lib) for s in sources)


def _run(env_extra, preload, tests):
    env = dict(os.environ)
    env.update(env_extra)
    env["LD_PRELOAD"] = preload
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    cmd = [sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu", *tests]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    return out


def test_oracle_under_asan_ubsan():
    from oracle import build as ob
    if _stale(ob.SAN_LIB, [ob.SRC]):
        ob.build_oracle(sanitize=True)
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(asan):
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    out = _run({"QE_ORACLE_LIB": ob.SAN_LIB}, asan,
               ["tests/test_oracle_fitness.py", "tests/test_oracle_encoding.py", "tests/test_oracle_ising.py"])
    assert " passed" in out


def test_abi_host_code_under_asan_ubsan():
    from paper_1809_11134_amd import build as qb
    srcs = [os.path.join(qb.CSRC, s) for s in os.listdir(qb.CSRC)] + [os.path.join(ROOT, "include", "qe.h")]
    if _stale(qb.SAN_LIB, srcs):
        qb.build(sanitize=True)
    clang = "/opt/rocm/lib/llvm/bin/clang"
    rt = subprocess.run([clang, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True,
                        text=True).stdout.strip() if os.path.exists(clang) else ""
    if not os.path.isabs(rt) or not os.path.exists(rt):
        pytest.skip("clang's AddressSanitizer runtime is not installed")
    out = _run({"QE_LIB": qb.SAN_LIB}, rt, ["tests/test_abi.py"])
    assert " passed" in out
