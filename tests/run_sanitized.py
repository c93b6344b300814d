"""Run the CPU test suite against AddressSanitizer / UndefinedBehaviorSanitizer builds.

    python tests/run_sanitized.py [extra pytest arguments]

Copies the sources into a temporary tree, builds there
  * the library with its host code (program compiler, frame schedule, C ABI)
    instrumented (`-Xarch_host -fsanitize=...`: the gfx950 device code is
    built as usual and never runs on the CPU), and
  * the C oracle with clang and the same sanitizers,
then runs `pytest -m "not gpu"` in that tree with the clang sanitizer runtime
preloaded into Python.  Any sanitizer report stops the run with a non-zero
status.  Leak checking is off: the interpreter itself keeps allocations alive
at exit.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang"
COPY = ["paper_2607_28600_amd", "include", "oracle", "tests", "workloads", "pytest.ini", "conftest.py", "setup.cfg"]
SAN = ["address", "undefined"]


def _run(cmd, **kw):
    print("+", " ".join(cmd), flush=True)
    subprocess.check_call(cmd, **kw)


def build_library(tree: str) -> None:
    csrc = os.path.join(tree, "paper_2607_28600_amd", "csrc")
    build = os.path.join(tree, "_build_san")
    os.makedirs(build, exist_ok=True)
    host_san = []
    for s in SAN:
        host_san += ["-Xarch_host", f"-fsanitize={s}"]
    flags = ["-x", "hip", "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all"] + host_san
    sys.path.insert(0, os.path.join(tree, "paper_2607_28600_amd"))
    from build import SOURCES  # the library's own source list
    sys.path.pop(0)
    objs = []
    for src in SOURCES:
        obj = os.path.join(build, os.path.splitext(src)[0] + ".o")
        _run([HIPCC] + flags + ["-c", os.path.join(csrc, src), "-o", obj])
        objs.append(obj)
    lib = os.path.join(tree, "paper_2607_28600_amd", "libsymft.so")
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-shared-libsan"] +
         [f"-fsanitize={s}" for s in SAN] + ["-o", lib] + objs)


def build_oracle(tree: str) -> None:
    src = os.path.join(tree, "oracle", "symft_oracle.c")
    lib = os.path.join(tree, "oracle", "libsymft_oracle.so")
    _run([CLANG, "-O1", "-g", "-std=gnu11", "-fPIC", "-shared", "-shared-libsan", "-fno-omit-frame-pointer",
          "-fno-sanitize-recover=all", "-fopenmp"] + [f"-fsanitize={s}" for s in SAN] +
         [src, "-o", lib, "-lm"])


def main() -> int:
    runtime = subprocess.check_output([CLANG, "-print-file-name=libclang_rt.asan-x86_64.so"], text=True).strip()
    with tempfile.TemporaryDirectory(prefix="symft_san_") as tree:
        for name in COPY:
            p = os.path.join(ROOT, name)
            if os.path.isdir(p):
                shutil.copytree(p, os.path.join(tree, name),
                                ignore=shutil.ignore_patterns("*.so", "__pycache__", "_build*"))
            elif os.path.exists(p):
                shutil.copy(p, os.path.join(tree, name))
        build_library(tree)
        build_oracle(tree)
        env = dict(os.environ)
        env["LD_PRELOAD"] = runtime
        env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1:abort_on_error=1:alloc_dealloc_mismatch=0"
        env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
        env["LD_LIBRARY_PATH"] = "/opt/rocm/llvm/lib:" + env.get("LD_LIBRARY_PATH", "")
        # -s: a sanitizer report goes to the terminal before the process aborts
        cmd = [sys.executable, "-m", "pytest", "tests", "-x", "-q", "-s", "-m", "not gpu", "-p", "no:cacheprovider"]
        cmd += sys.argv[1:]
        print("+", " ".join(cmd), flush=True)
        return subprocess.call(cmd, cwd=tree, env=env)


if __name__ == "__main__":
    sys.exit(main())
