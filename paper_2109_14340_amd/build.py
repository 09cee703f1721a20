"""Build libtenoaa.so (HIP, gfx950) in-tree next to this file."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libtenoaa.so")
SOURCES = ["tenoaa_kernels.hip", "tenoaa_adjoint.hip", "tenoaa_capi.hip"]
HEADERS = ["tenoaa_internal.h", "tenoaa_sos.h", "tenoaa_device.h"]

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # one fixed order of IEEE operations: no contraction anywhere
    "-ffp-contract=off",
    # keep the compiler from emitting packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def build(verbose=False, out=None, defines=()):
    """Compile the library; `out`/`defines` build a variant elsewhere (tuning)."""
    target = out or LIB
    cmd = ["hipcc"] + FLAGS + ["-D%s" % d for d in defines] + ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    cmd += [os.path.join(CSRC, s) for s in SOURCES] + ["-o", target + ".tmp"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(target + ".tmp", target)
    return target


def sources():
    return [os.path.join(CSRC, s) for s in SOURCES + HEADERS] + [os.path.join(ROOT, "include", "tenoaa.h")]


if __name__ == "__main__":
    build(verbose=True)
