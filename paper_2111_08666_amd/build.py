"""Build the HIP library liblbm.so (gfx950) in-tree with hipcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liblbm.so")
SOURCES = [os.path.join(HERE, "csrc", s) for s in ("lbm_kernels.hip", "lbm_step_srt.hip", "lbm_step_mrt.hip",
                                                    "lbm_step_trt.hip", "lbm_api.cpp", "unet_kernels.hip")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # keep FP32 arithmetic off the packed-math path
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # fuse a*b + c only inside one source expression: kernels that share the
    # node arithmetic then round alike, whatever else surrounds it
    "-ffp-contract=on",
    "-Wno-unused-command-line-argument",
]


def kernel_source_hash() -> str:
    """Hash of the step kernels' sources and of the host code that lays out
    their data (the node numbering sets the memory traffic): counter
    measurements are tied to it."""
    import hashlib
    h = hashlib.sha256()
    for f in ("lbm_kernels.hip", "lbm_step.h", "lattice.h", "lbm_device.h", "lbm_api.cpp"):
        with open(os.path.join(HERE, "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def build(verbose: bool = False, extra=()) -> str:
    """Compile the sources to objects in parallel, then link the library."""
    obj_dir = os.path.join(os.path.dirname(HERE), "_build")
    os.makedirs(obj_dir, exist_ok=True)
    compile_flags = [f for f in FLAGS if f != "-shared"]
    procs, objs = [], []
    for src in SOURCES:
        obj = os.path.join(obj_dir, os.path.basename(src) + ".o")
        cmd = [HIPCC, *compile_flags, *extra, "-x", "hip", "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd))
        objs.append(obj)
    codes = [p.wait() for p in procs]
    if any(codes):
        raise subprocess.CalledProcessError(max(codes), "hipcc")
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True, extra=sys.argv[1:]))
