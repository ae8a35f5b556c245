"""Host-side AddressSanitizer / UndefinedBehaviorSanitizer run (CPU only).

    python -m paper_2005_13679_amd.sanitize

Builds libmc.so with its host code instrumented (device code as usual) and
the C oracle with the same sanitizers, both with clang and the shared
sanitizer runtime, into paper_2005_13679_amd/_build/asan and
oracle/_build/asan, then runs the CPU test suite (pytest -m "not gpu") with
those libraries (MC_LIBRARY, MC_ORACLE_LIBRARY) and the runtime preloaded.
The host code covered: argument and size checks of every entry point, the
hash and table-size arithmetic, the batch and graph plans, the tridiagonal
eigen-solvers, and the whole oracle.  Exit status: pytest's.
"""

from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

from . import build as B

ROOT = B.ROOT
ASAN_DIR = os.path.join(B.HERE, "_build", "asan")
ORACLE_SRC = os.path.join(ROOT, "oracle", "mc_oracle.c")
ORACLE_DIR = os.path.join(ROOT, "oracle", "_build", "asan")
CLANG = "/opt/rocm/llvm/bin/clang"
CLANGXX = "/opt/rocm/llvm/bin/clang++"
SAN = ["address", "undefined"]


def _host_flags():
    f = []
    for x in SAN:
        f += ["-Xarch_host", f"-fsanitize={x}"]
    return f + ["-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host",
                "-fno-sanitize-recover=undefined", "-Xarch_host", "-shared-libsan"]


def _compile(src: str) -> str:
    obj = os.path.join(ASAN_DIR, os.path.splitext(src)[0] + ".o")
    cmd = [B.HIPCC, *B.FLAGS, *_host_flags(), "-g", "-c", os.path.join(B.CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build_sanitized() -> tuple[str, str]:
    os.makedirs(ASAN_DIR, exist_ok=True)
    os.makedirs(ORACLE_DIR, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=len(B.SOURCES)) as ex:
        objs = list(ex.map(_compile, B.SOURCES))
    lib = os.path.join(ASAN_DIR, "libmc.so")
    san = ",".join(SAN)
    # host link with clang++ (the objects carry their device code)
    subprocess.check_call([CLANGXX, "-shared", f"-fsanitize={san}", "-shared-libsan", "-o", lib,
                           *objs, "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"])
    olib = os.path.join(ORACLE_DIR, "libmc_oracle.so")
    subprocess.check_call([CLANG, "-O1", "-g", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                           f"-fsanitize={san}", "-fno-sanitize-recover=undefined",
                           "-shared-libsan", "-fno-omit-frame-pointer", "-Wall", "-o", olib,
                           ORACLE_SRC, "-lm"])
    return lib, olib


def main() -> int:
    lib, olib = build_sanitized()
    rt = subprocess.check_output([CLANG, "-print-file-name=libclang_rt.asan-x86_64.so"],
                                 text=True).strip()
    env = dict(os.environ)
    env.update({
        "MC_LIBRARY": lib,
        "MC_ORACLE_LIBRARY": olib,
        "LD_PRELOAD": rt,
        # the interpreter and the HIP runtime are not instrumented: their
        # allocations are not reported as leaks
        "ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1:abort_on_error=1",
        "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1",
    })
    print(f"[sanitize] {lib}\n[sanitize] {olib}\n[sanitize] runtime {rt}", flush=True)
    return subprocess.call([sys.executable, "-m", "pytest", os.path.join(ROOT, "tests"), "-q",
                            "-m", "not gpu", "-p", "no:cacheprovider"], env=env, cwd=ROOT)


if __name__ == "__main__":
    sys.exit(main())
