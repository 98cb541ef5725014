"""Build the HIP library libagf2.so for gfx950 with hipcc (in-tree).

Every translation unit under csrc/ is compiled to an object file on its own
(in parallel), then the objects are linked into libagf2.so."""
from __future__ import annotations

import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libagf2.so")
OBJ = os.path.join(HERE, "_build")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = os.path.join(ROCM, "bin", "hipcc")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # keep the compiler from emitting packed-FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def sources():
    return sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    msgs = [ln for ln in (r.stdout + r.stderr).splitlines()
            if "packed-fp32-ops" not in ln and ln.strip()]
    return r.returncode, "\n".join(msgs)


def build(verbose: bool = True, jobs: int | None = None) -> str:
    srcs = sources()
    os.makedirs(OBJ, exist_ok=True)
    inc = ["-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(ROCM, "include")]
    objs = [os.path.join(OBJ, os.path.basename(s)[:-4] + ".o") for s in srcs]
    cmds = [[HIPCC] + HIPCC_FLAGS + inc + ["-c", s, "-o", o] for s, o in zip(srcs, objs)]
    jobs = jobs or min(len(cmds), max(1, min(8, os.cpu_count() or 1)))
    if verbose:
        print(f"hipcc {' '.join(HIPCC_FLAGS)} -c <{len(srcs)} sources> ({jobs} jobs)",
              flush=True)
    with ThreadPoolExecutor(jobs) as ex:
        results = list(ex.map(_run, cmds))
    failed = False
    for s, (rc, msg) in zip(srcs, results):
        if msg and (verbose or rc != 0):
            print(f"--- {os.path.basename(s)}\n{msg}", file=sys.stderr if rc else sys.stdout)
        failed |= rc != 0
    if failed:
        raise RuntimeError("hipcc failed to compile libagf2.so")
    tmp = LIB + ".tmp"
    link = ([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC"] + objs +
            ["-o", tmp, "-L" + os.path.join(ROCM, "lib"), "-lrocsolver", "-lrocblas",
             "-Wl,-rpath," + os.path.join(ROCM, "lib")])
    rc, msg = _run(link)
    if rc != 0:
        sys.stderr.write(msg + "\n")
        raise RuntimeError("hipcc failed to link libagf2.so")
    os.replace(tmp, LIB)
    return LIB


ASAN_EXE = os.path.join(HERE, "agf2_asan_check")
# host code only: each sanitizer flag applies to the host compilation
SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer"]


def build_asan_check(verbose: bool = True, jobs: int | None = None) -> str:
    """The library's sources and tests/asan_driver.cpp with the host code
    built under AddressSanitizer and UndefinedBehaviorSanitizer, linked into
    one executable (a check of the host paths of the C ABI; run on a GPU)."""
    srcs = sources() + [os.path.join(ROOT, "tests", "asan_driver.cpp")]
    odir = os.path.join(OBJ, "asan")
    os.makedirs(odir, exist_ok=True)
    inc = ["-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(ROCM, "include")]
    flags = [f for f in HIPCC_FLAGS if f != "-O3"] + ["-O1", "-g"] + SANITIZE
    objs = [os.path.join(odir, os.path.basename(s).rsplit(".", 1)[0] + ".o") for s in srcs]
    cmds = []
    for s, o in zip(srcs, objs):
        lang = ["-x", "hip"] if s.endswith(".cpp") else []
        cmds.append([HIPCC] + flags + inc + ["-c"] + lang + [s, "-o", o])
    jobs = jobs or min(len(cmds), max(1, min(8, os.cpu_count() or 1)))
    with ThreadPoolExecutor(jobs) as ex:
        results = list(ex.map(_run, cmds))
    for s, (rc, msg) in zip(srcs, results):
        if rc != 0:
            sys.stderr.write(f"--- {os.path.basename(s)}\n{msg}\n")
            raise RuntimeError("hipcc failed to compile the sanitizer check")
    tmp = ASAN_EXE + ".tmp"
    link = ([HIPCC, "--offload-arch=gfx950"] + SANITIZE + objs +
            ["-o", tmp, "-L" + os.path.join(ROCM, "lib"), "-lrocsolver", "-lrocblas",
             "-Wl,-rpath," + os.path.join(ROCM, "lib")])
    rc, msg = _run(link)
    if rc != 0:
        sys.stderr.write(msg + "\n")
        raise RuntimeError("hipcc failed to link the sanitizer check")
    os.replace(tmp, ASAN_EXE)
    if verbose:
        print(f"built {ASAN_EXE}", flush=True)
    return ASAN_EXE


if __name__ == "__main__":
    build()
    build_asan_check()
