"""Build the oracle's C library in its two precisions (test infrastructure).

    python oracle/build.py

writes oracle/liboracle_f32.so and oracle/liboracle_f64.so with plain gcc:
-O2, no FP contraction, no fast-math (IEEE infinities carry meaning).
"""

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "bp_oracle.c")


def build(verbose=False):
    outs = {}
    for tag, real in (("f32", "float"), ("f64", "double")):
        out = os.path.join(HERE, f"liboracle_{tag}.so")
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared", f"-DREAL={real}", "-Wall", "-Wextra",
               "-o", out, SRC, "-lm"]
        if verbose:
            print(" ".join(cmd))
        subprocess.run(cmd, check=True)
        outs[tag] = out
    return outs


if __name__ == "__main__":
    build(verbose="-q" not in sys.argv)
