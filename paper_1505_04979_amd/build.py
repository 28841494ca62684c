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
SOURCES = ["pbp_host.cpp", "pbp_decode.hip", "pbp_r10.hip", "pbp_unrolled.hip",
           "pbp_roundtrip.hip", "pbp_mixed.hip", "pbp_sc.hip",
           "pbp_quant.hip"]

HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("PBP_OFFLOAD_ARCH", "gfx950")

FLAGS = ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC",
         "-ffp-contract=off", "-fno-fast-math",
         # device code: messages are never NaN, so the min of eq. (1) needs no
         # signalling-NaN quieting (IEEE mode off)
         "-Xarch_device", "-mno-amdgpu-ieee", "-Xarch_device", "-fno-honor-nans",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-result"]


def _compile(src, obj, verbose):
    cmd = [HIPCC] + FLAGS + ["-c", "-I", INCLUDE, "-I", CSRC]
    cmd += (["-x", "hip", src] if src.endswith(".cpp") else [src])
    cmd += ["-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose=False):
    """Compile every source to an object (in parallel), then link."""
    from concurrent.futures import ThreadPoolExecutor
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = [os.path.join(objdir, os.path.splitext(s)[0] + ".o")
            for s in SOURCES]
    jobs = max(1, min(len(SOURCES), os.cpu_count() or 1, 16))
    with ThreadPoolExecutor(jobs) as ex:
        for f in [ex.submit(_compile, os.path.join(CSRC, s), o, verbose)
                  for s, o in zip(SOURCES, objs)]:
            f.result()
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC"] + objs + \
        ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-q" not in sys.argv)
