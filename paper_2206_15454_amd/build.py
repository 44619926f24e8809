"""Build the HIP library ``liblbmx.so`` for gfx950 with hipcc (in-tree).

Packed FP32 instructions are disabled (``-packed-fp32-ops``): every FP32
operation is issued unpacked.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblbmx.so")
SOURCES = ["lbm_kernels.hip", "mlp_kernels.hip", "lbm_api.hip", "mlp_train.hip",
           "closure_data.hip", "forest.hip"]
ARCH = os.environ.get("LBMX_ARCH", "gfx950")


def hipcc_flags(extra=()):
    return ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-result", *extra]


def build(verbose=False, extra=(), out=None, jobs=4):
    """Compile each source to an object in parallel, then link the library."""
    out = out or LIB
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    procs = []
    objs = []
    for src in SOURCES:
        obj = os.path.join(objdir, src.replace(".hip", ".o"))
        objs.append(obj)
        cmd = ["hipcc", *hipcc_flags(extra), "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((cmd, subprocess.Popen(cmd)))
    for cmd, p in procs:
        if p.wait() != 0:
            raise RuntimeError("hipcc failed: " + " ".join(cmd))
    link = ["hipcc", "--offload-arch=" + ARCH, "-shared", "-fPIC", *objs, "-o", out + ".tmp"]
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.run(link, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
