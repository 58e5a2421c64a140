"""Build libcmhd.so (gfx950) in-tree with hipcc.

    python -m paper_1908_08557_amd.build [--verbose]

Every HIP translation unit under csrc/ is compiled for gfx950 and linked
into one shared library next to this file.  Packed FP32 instructions are
disabled (-packed-fp32-ops) for all device code.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libcmhd.so")
BUILD = os.path.join(HERE, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-mcode-object-version=5",
    f"-I{INCLUDE}", f"-I{CSRC}",
]


# per-source extra flags.  The fused substage kernel runs 16 waves per CU at
# 128 registers each: machine loop-invariant code motion would hoist the
# float64 constants of exp() and other loop-invariant values out of the plane
# loop into registers, which this register budget cannot hold.
SOURCE_FLAGS = {
    "substage.hip": ["-mllvm", "-disable-machine-licm"],
}


# Kernels that must run without scratch memory: their register budget is
# exact (16 waves per CU at 128 registers), and builds of the fused substage
# kernel that spilled to scratch gave wrong Runge-Kutta substages 2-3.  The
# build fails if the compiler places any scratch access in them.
NO_SCRATCH = {"substage.hip": "k_substage"}


def scratch_report(src: str, kernel_substr: str, extra_flags=()) -> dict:
    """Scratch load/store instruction count of every kernel of `src` whose
    name contains `kernel_substr`, from the device assembly of this build."""
    import re
    import tempfile
    with tempfile.TemporaryDirectory() as tmp:
        out = os.path.join(tmp, "k.s")
        cmd = [HIPCC, *FLAGS, *SOURCE_FLAGS.get(os.path.basename(src), []), *extra_flags,
               "--cuda-device-only", "-S", src, "-o", out]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc -S failed for {src}:\n{r.stderr}")
        text = open(out).read()
    counts = {}
    for m in re.finditer(r"^(\S*" + re.escape(kernel_substr) + r"\S*):", text, re.M):
        end = text.index("s_endpgm", m.end())
        counts[m.group(1)] = len(re.findall(r"\bscratch_(?:load|store)", text[m.end():end]))
    return counts


def check_no_scratch(extra_flags=()) -> None:
    for name, kern in NO_SCRATCH.items():
        counts = scratch_report(os.path.join(CSRC, name), kern, extra_flags)
        if not counts:
            raise RuntimeError(f"no {kern} kernel found in {name}")
        bad = {k: n for k, n in counts.items() if n}
        if bad:
            raise RuntimeError(f"{name}: kernels with scratch accesses: {bad}")


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def build(verbose: bool = False, extra_flags=()) -> str:
    os.makedirs(BUILD, exist_ok=True)
    objs = []

    def compile_one(src):
        obj = os.path.join(BUILD, os.path.basename(src) + ".o")
        cmd = [HIPCC, *FLAGS, *SOURCE_FLAGS.get(os.path.basename(src), []), *extra_flags, "-c", src,
               "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
        if verbose and r.stderr:
            print(r.stderr, flush=True)
        return obj

    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(compile_one, sources()))
        guard = ex.submit(check_no_scratch, extra_flags)
        guard.result()
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    extra = []
    if "--resource-usage" in sys.argv:
        extra = ["-Rpass-analysis=kernel-resource-usage"]
    print(build(verbose="--verbose" in sys.argv or bool(extra), extra_flags=extra))
