"""Builds libclaw.so (HIP, gfx950) in-tree from csrc/.

hipcc compiles each translation unit for gfx950 only; packed FP32 VALU
instructions are disabled for the whole library.  Floating-point contraction
is decided per source expression (-ffp-contract=on), so a formula compiles to
the same operations wherever it is inlined: results do not depend on tile
shapes or on which kernel computes an interface.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libclaw.so")
# debug build: the same sources with CLAW_DEBUG (range checks on every buffer
# access and on the boundary index map, counted per kernel file and read with
# claw_debug_take)
OUT_DEBUG = os.path.join(HERE, "libclaw_debug.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SOURCES = ["sweeps.hip", "fused.hip", "batch.hip", "control.hip", "learned.hip", "runtime.hip", "stream.hip"]
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-result",
         "-ffp-contract=on",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(HERE, "..", "include")]
# per file: the learned network's matrix products accumulate in ordinary VGPRs
# (gfx950 allows it), which saves a v_accvgpr_read per result element
FILE_FLAGS = {"learned.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"]}


def build(verbose=False, jobs=4, debug=False):
    objdir = os.path.join(HERE, "_build_debug" if debug else "_build")
    out = OUT_DEBUG if debug else OUT
    os.makedirs(objdir, exist_ok=True)

    def compile_one(src):
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        cmd = [HIPCC] + FLAGS + FILE_FLAGS.get(src, []) + (["-DCLAW_DEBUG"] if debug else []) + \
            ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
        if verbose and r.stderr.strip():
            print(r.stderr, flush=True)
        return obj

    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    tmp = out + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    build(verbose="-v" in sys.argv, debug="--debug" in sys.argv)
