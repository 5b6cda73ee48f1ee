"""Build libmam.so (HIP, gfx950) in place next to this file.

    python -m paper_2309_05315_amd.build [--host-sanitizers]

Every translation unit under csrc/ is compiled for gfx950 in parallel and
linked into one shared library.  Packed FP32 instructions are disabled
(-packed-fp32-ops target feature) and no fast-math flag is used: the
kernels' FP64 row sums, thresholds and the cost helper's operation order
rely on IEEE rounding.

With --host-sanitizers (build(sanitize=True)) the host side of every
translation unit is instrumented with AddressSanitizer and
UndefinedBehaviorSanitizer (the device code is compiled as usual) into
_build/hostsan/libmam_hostsan.so, for the CPU tests of the C ABI.  The
library is linked without the sanitizer runtime: a process loads it after
preloading the runtime (asan_runtime()), which also holds UBSan's handlers.
"""
from __future__ import annotations

import glob
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libmam.so")
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")

FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-result",
         "-I", os.path.join(ROOT, "include"), "-I", CSRC]


HOSTSAN_DIR = os.path.join(BUILD, "hostsan")
HOSTSAN_LIB = os.path.join(HOSTSAN_DIR, "libmam_hostsan.so")
# host-only instrumentation: every sanitizer flag is scoped to the host pass
HOSTSAN_FLAGS = ("-Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined "
                 "-Xarch_host -fno-omit-frame-pointer -Xarch_host -O1 -g").split()


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    return cmd, res


def sources() -> list:
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def build(verbose: bool = False, jobs: int = 0, sanitize: bool = False) -> str:
    """Compile every source into libmam.so (or, with sanitize, the host-
    instrumented libmam_hostsan.so); always recompiles."""
    objdir = HOSTSAN_DIR if sanitize else BUILD
    out = HOSTSAN_LIB if sanitize else LIB
    os.makedirs(objdir, exist_ok=True)
    flags = FLAGS + (HOSTSAN_FLAGS if sanitize else [])
    objs, cmds = [], []
    for src in sources():
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        objs.append(obj)
        cmds.append([hipcc(), *flags, "-c", src, "-o", obj])
    jobs = jobs or min(len(cmds), max(1, (os.cpu_count() or 4)))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        for cmd, res in ex.map(_run, cmds):
            if verbose:
                print(" ".join(cmd), flush=True)
            if res.returncode != 0:
                sys.stderr.write(res.stdout + res.stderr)
                raise RuntimeError(f"hipcc failed on {cmd[-3]}")
    tmp = out + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", "--offload-arch=gfx950", *objs, "-o", tmp]
    cmd, res = _run(cmd)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"linking {os.path.basename(out)} failed")
    os.replace(tmp, out)
    return out


def hostsan_library() -> str:
    """The host-instrumented library, rebuilt when a source or header is newer."""
    deps = sources() + glob.glob(os.path.join(CSRC, "*.hpp")) + glob.glob(os.path.join(ROOT, "include", "*.h"))
    if not os.path.exists(HOSTSAN_LIB) or os.path.getmtime(HOSTSAN_LIB) < max(os.path.getmtime(d) for d in deps):
        build(sanitize=True)
    return HOSTSAN_LIB


def asan_runtime() -> str:
    """Path of the compiler's shared ASan runtime (to preload)."""
    clang = os.path.join(os.path.dirname(os.path.realpath(hipcc())), "..", "llvm", "bin", "clang")
    for cand in (clang, "/opt/rocm/llvm/bin/clang", shutil.which("clang") or ""):
        if cand and os.path.exists(cand):
            res = subprocess.run([cand, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
            path = res.stdout.strip()
            if res.returncode == 0 and os.path.isabs(path) and os.path.exists(path):
                return path
    raise RuntimeError("the ASan runtime of the HIP compiler was not found")


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, sanitize="--host-sanitizers" in sys.argv))
