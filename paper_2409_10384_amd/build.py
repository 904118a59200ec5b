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
    # contraction to fused multiply-adds only within one expression (FP_CONTRACT
    # on; HIP's default "fast" mode fuses across statements and ignores the
    # pragma below).  Where mirrored states exchange the roles of two terms --
    # the Riemann flux of the two sides, the corner EMFs, the CT face update --
    # the code switches contraction off with `#pragma clang fp contract(off)`,
    # so a mirror-image state still gives mirror-image results bit for bit;
    # everywhere else a fused product is one instruction instead of two
    # (learned.hip opts out as a whole; its header says why).
    "-ffp-contract=on",
    # matrix-core results in ordinary VGPRs: the network's activations then
    # read them directly instead of one v_accvgpr_read per value (only
    # learned.hip has MFMA code)
    "-mllvm", "-amdgpu-mfma-vgpr-form",
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
