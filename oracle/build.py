"""Builds the CPU oracle libraries (test infrastructure only).

liboracle.so      FP64 oracle, gcc -O2 -ffp-contract=off, OpenMP over lines.
liboracle_f32.so  the same source with real = float, used only to measure the
                  rounding floor of single precision against the FP64 oracle.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "claw_oracle.c")
FLAGS = ["-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
         "-fopenmp", "-Wall", "-Wno-unknown-pragmas"]


def build(verbose=False):
    outs = []
    for name, extra in (("liboracle.so", []), ("liboracle_f32.so", ["-DORACLE_REAL=float"])):
        out = os.path.join(HERE, name)
        tmp = out + ".tmp"
        cmd = ["gcc"] + FLAGS + extra + ["-o", tmp, SRC, "-lm"]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(tmp, out)
        outs.append(out)
    return outs


def ensure_built():
    """Builds the oracle if it is missing or older than its source."""
    src_m = max(os.path.getmtime(SRC), os.path.getmtime(os.path.join(HERE, "claw_oracle.h")))
    for name in ("liboracle.so", "liboracle_f32.so"):
        p = os.path.join(HERE, name)
        if not os.path.exists(p) or os.path.getmtime(p) < src_m:
            build()
            return


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
