"""Build libtenoaa.so (HIP, gfx950) in-tree next to this file."""
import os
import subprocess
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libtenoaa.so")
SOURCES = ["tenoaa_kernels.hip", "tenoaa_tail.hip", "tenoaa_audit.hip", "tenoaa_adjoint.hip",
           "tenoaa_adjoint_general.hip", "tenoaa_adjoint_tail.hip", "tenoaa_batch.hip", "tenoaa_advect.hip",
           "tenoaa_capi.hip"]
HEADERS = ["tenoaa_internal.h", "tenoaa_sos.h", "tenoaa_device.h", "tenoaa_stencil.h", "tenoaa_vjp.h"]

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # one fixed order of IEEE operations: no contraction anywhere
    "-ffp-contract=off",
    # keep the compiler from emitting packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def build(verbose=False, out=None, defines=()):
    """Compile the library (one process per source, then link);
    `out`/`defines` build a variant elsewhere (tuning)."""
    target = out or LIB
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    dflags = ["-D%s" % d for d in defines]
    with tempfile.TemporaryDirectory(prefix="tenoaa_build_") as tmp:
        objs, procs = [], []
        for s in SOURCES:
            o = os.path.join(tmp, s.replace(".hip", ".o"))
            cmd = ["hipcc"] + FLAGS + dflags + inc + ["-c", os.path.join(CSRC, s), "-o", o]
            if verbose:
                print(" ".join(cmd))
            procs.append((s, subprocess.Popen(cmd)))
            objs.append(o)
        failed = [s for s, p in procs if p.wait() != 0]
        if failed:
            raise RuntimeError("compilation failed: %s" % ", ".join(failed))
        link = ["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + ["-o", target + ".tmp"]
        if verbose:
            print(" ".join(link))
        subprocess.run(link, check=True)
    os.replace(target + ".tmp", target)
    return target


def sources():
    return [os.path.join(CSRC, s) for s in SOURCES + HEADERS] + [os.path.join(ROOT, "include", "tenoaa.h")]


if __name__ == "__main__":
    build(verbose=True)
