"""Host AddressSanitizer + UndefinedBehaviorSanitizer run of the CPU tests.

Builds the C ABI library with the sanitizers on its host code only (the
device code is compiled as usual: GPU sanitizers are not used) and the
oracle with the same sanitizers, both with the ROCm clang so that one
sanitizer runtime serves the process, then runs the CPU test suite
(``-m "not gpu"``) against these builds:

    python -m paper_2509_14726_amd.sanitize [pytest args...]

The builds go to a temporary directory; the in-tree libraries are not
touched.  The run loads them through MPPI_LIBRARY and ORACLE_LIBRARY and
preloads the clang sanitizer runtime (Python itself is not instrumented).
Leak checking is off: the interpreter keeps its own allocations until exit.
Any sanitizer report ends the run with a non-zero status.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys
import tempfile

from . import build as B

ROOT = os.path.dirname(B.HERE)
LLVM = "/opt/rocm/llvm"

# -Xarch_host before each sanitizer option: the host half of every HIP
# source (and the host link) is instrumented, the gfx950 half is not.
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
            "-Xarch_host", "-shared-libsan"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"{' '.join(cmd[:3])} ... failed:\n{r.stderr}")


def asan_runtime() -> str:
    libs = sorted(glob.glob(os.path.join(LLVM, "lib", "clang", "*", "lib", "linux",
                                         "libclang_rt.asan-x86_64.so")))
    if not libs:
        raise RuntimeError("clang's AddressSanitizer runtime not found under " + LLVM)
    return libs[-1]


def build_sanitized(out_dir: str) -> tuple[str, str]:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objs = []
    for src in B.SOURCES:
        obj = os.path.join(out_dir, src.replace(".hip", ".o"))
        _run([hipcc, *B.FLAGS, "-g", *HOST_SAN, "-c", os.path.join(B.CSRC, src), "-o", obj])
        objs.append(obj)
    lib = os.path.join(out_dir, "libmppi_san.so")
    _run([hipcc, f"--offload-arch={B.ARCH}", "-shared", "-fPIC", *HOST_SAN, "-o", lib, *objs])
    orc = os.path.join(out_dir, "liborc_san.so")
    clang = os.path.join(LLVM, "bin", "clang")
    _run([clang, "-O1", "-g", "-std=c99", "-Wall", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
          "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
          "-shared-libsan", "-o", orc, os.path.join(ROOT, "oracle", "mppi_oracle.c"), "-lm"])
    return lib, orc


def main(argv: list[str]) -> int:
    with tempfile.TemporaryDirectory(prefix="mppi_san_") as tmp:
        lib, orc = build_sanitized(tmp)
        # reports go to files (the test runner captures stderr)
        log = os.path.join(tmp, "report")
        env = dict(os.environ)
        env.update(MPPI_LIBRARY=lib, ORACLE_LIBRARY=orc, LD_PRELOAD=asan_runtime(),
                   ASAN_OPTIONS=f"detect_leaks=0:abort_on_error=1:detect_odr_violation=0:log_path={log}",
                   UBSAN_OPTIONS=f"print_stacktrace=1:halt_on_error=1:log_path={log}")
        cmd = [sys.executable, "-m", "pytest", os.path.join(ROOT, "tests"), "-m", "not gpu", "-x", "-q",
               "-p", "no:cacheprovider", *argv]
        print("sanitized builds:", lib, orc, flush=True)
        rc = subprocess.call(cmd, env=env, cwd=ROOT)
        reports = sorted(glob.glob(log + ".*"))
        for f in reports:
            print(f"--- sanitizer report {os.path.basename(f)}")
            print(open(f).read())
        print(f"sanitizer reports: {len(reports)}, test status {rc}", flush=True)
        return rc if rc != 0 else (1 if reports else 0)


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
