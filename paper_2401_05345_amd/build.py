"""Build libgsr.so for gfx950 in-tree (hipcc, one object per translation unit).

    python -m paper_2401_05345_amd.build [--verbose]

Flags that matter:
  --offload-arch=gfx950           CDNA4 code objects only
  -packed-fp32-ops disabled        no packed FP32 VALU forms are generated
  -munsafe-fp-atomics              fp32 atomic add is the hardware global_atomic_add_f32
  -amdgpu-atomic-optimizer-strategy=None
                                   keeps every atomic the source writes: the compiler
                                   would otherwise turn uniform-address atomics into
                                   its own wave reduction, which would silently change
                                   the plain-atomic backward into a reduced one
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIBDIR = os.path.join(HERE, "_lib")
LIB = os.path.join(LIBDIR, "libgsr.so")
SOURCES = ["runtime.hip", "k_preprocess.hip", "k_sort.hip", "k_composite.hip", "k_composite_compiler_reduce.hip",
           "k_train.hip", "k_loss.hip", "k_micro.hip", "server.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics",
    "-mllvm", "-amdgpu-atomic-optimizer-strategy=None",
    "-I", INCLUDE, "-I", CSRC,
]


# The compiler-reduced ablation of the plain-atomic backward is the one source built with LLVM's
# atomic optimizer on (everything else keeps atomics as written, so the plain baseline stays plain).
OPTIMIZED_ATOMICS = {"k_composite_compiler_reduce.hip"}


def flags_for(src: str):
    if src not in OPTIMIZED_ATOMICS:
        return list(HIPCC_FLAGS)
    return [("-amdgpu-atomic-optimizer-strategy=DPP" if f == "-amdgpu-atomic-optimizer-strategy=None" else f)
            for f in HIPCC_FLAGS]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found; libgsr needs ROCm's hipcc to build")


def _compile(src: str, obj: str, extra, verbose: bool):
    cmd = [hipcc(), *flags_for(src), *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{out}")
    if out.strip() and verbose:
        print(out, flush=True)
    return obj


def build(verbose: bool = False, extra=()) -> str:
    """Compile every source and link libgsr.so (always rebuilds)."""
    objdir = os.path.join(LIBDIR, "obj")
    os.makedirs(objdir, exist_ok=True)
    jobs = min(len(SOURCES), max(1, (os.cpu_count() or 2)))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, os.path.join(objdir, s.replace(".hip", ".o")), extra, verbose),
                           SOURCES))
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="--verbose" in sys.argv))
