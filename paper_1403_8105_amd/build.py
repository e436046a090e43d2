"""Build libfld.so (HIP, gfx950) in-tree with hipcc.

Every HIP source is compiled with -ffp-contract=off (no multiply-add
contraction: FP64 results follow the plain evaluation order) and with the
packed-FP32 instructions disabled.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libfld.so")
SOURCES = ["csrc/fld_kernels.hip", "csrc/fld_engine.cpp", "csrc/fld_render.hip",
           "csrc/fld_noalloc.hip"]
ARCH = os.environ.get("FLD_OFFLOAD_ARCH", "gfx950")

HIPFLAGS = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", f"--offload-arch={ARCH}",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-function", "-Wno-unused-variable", "-Wno-unused-value",
            "-Wno-unused-result",
            "-I", os.path.join(ROOT, "include")]


def build(verbose: bool = False) -> str:
    objs = []
    for src in SOURCES:
        path = os.path.join(HERE, src)
        obj = os.path.join(HERE, "csrc", os.path.basename(src) + ".o")
        cmd = ["hipcc", *HIPFLAGS, "-x", "hip", "-c", path, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        msgs = [l for l in (r.stderr or "").splitlines() if "packed-fp32-ops" not in l]
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {src}:\n" + "\n".join(msgs))
        if verbose and msgs:
            print("\n".join(msgs))
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
