"""Build libgrmhd.so for gfx950 with hipcc (cross-compiles without a GPU)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libgrmhd.so")
SOURCES = [os.path.join(HERE, "csrc", "grmhd.hip"), os.path.join(HERE, "csrc", "learned.hip"),
           os.path.join(HERE, "csrc", "amr.hip")]
HEADERS = [os.path.join(HERE, "csrc", "physics.hpp"), os.path.join(HERE, "csrc", "mlp.hpp"),
           os.path.join(ROOT, "include", "grmhd.h")]

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
    # no packed-FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # every product and sum rounded on its own, as written (no contraction to
    # fused multiply-adds; explicit fma() calls stay): mirror-image states
    # then give mirror-image results bit for bit (with contraction only the
    # Riemann flux kept from fusing, the blast wave's y mirror still broke),
    # and the rounding follows the oracle's operation by operation where the
    # two write an expression alike.  About 3% of the step time on the star.
    "-ffp-contract=off",
    "-I", os.path.join(ROOT, "include"),
]


def build(verbose=False):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp"
    cmd = [hipcc] + HIPCC_FLAGS + SOURCES + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
