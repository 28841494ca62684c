"""Build libpbp.so (HIP, gfx950) in-tree.

    python -m paper_1505_04979_amd.build

Flags that carry meaning:
  -ffp-contract=off   no fused multiply-add: every product of eq. (1) rounds
                      once, before the sum, as in the FP32 operation order.
  (no fast-math)      IEEE infinities are the frozen messages of Section III.
  -packed-fp32-ops    disabled: packed FP32 instructions are not used.
  -mno-amdgpu-ieee    device code only: no message is ever NaN (LLRs are
                      finite, infinities only meet finite values), so min()
                      needs no signalling-NaN quieting of its operands.
"""

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libpbp.so")
SOURCES = ["pbp_host.cpp", "pbp_decode.hip", "pbp_r10.hip", "pbp_unrolled.hip"]

HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("PBP_OFFLOAD_ARCH", "gfx950")

FLAGS = ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-shared",
         "-ffp-contract=off", "-fno-fast-math",
         # device code: messages are never NaN, so the min of eq. (1) needs no
         # signalling-NaN quieting (IEEE mode off)
         "-Xarch_device", "-mno-amdgpu-ieee", "-Xarch_device", "-fno-honor-nans",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-result"]


def build(verbose=False):
    srcs = []
    for s in SOURCES:
        p = os.path.join(CSRC, s)
        srcs += (["-x", "hip", p] if s.endswith(".cpp") else [p])
    tmp = LIB + ".tmp"
    cmd = [HIPCC] + FLAGS + ["-I", INCLUDE, "-I", CSRC] + srcs + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-q" not in sys.argv)
