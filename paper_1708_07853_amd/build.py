"""Builds libdwt2.so (HIP for gfx950) in place, next to this file.

    python -m paper_1708_07853_amd.build

Every translation unit compiles to an object file of its own, in parallel
(the strip kernels of each direction are separate units), and the objects are
linked into one shared library.  Objects go to a scratch folder under the
package's `_build/`, which the repository does not track.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
LIB = os.path.join(HERE, "libdwt2.so")
OBJDIR = os.path.join(HERE, "_build")
SOURCES = ["strip_fwd.hip", "strip_inv.hip", "strip_bwd.hip", "job_fwd.hip", "job_inv.hip", "job_bwd.hip",
           "fused_fwd.hip", "fused_inv.hip", "fused_bwd.hip",
           "tail_kernels.hip", "lds_kernels.hip", "separable.hip", "cdf97.hip", "noalloc.hip", "api.cpp",
           "batched.cpp"]
ARCH = os.environ.get("DWT2_ARCH", "gfx950")

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-ffp-contract=off",
    # No packed FP32 instructions (v_pk_fma_f32 and friends) in the device
    # code.  The device compiler honours this feature switch; the host pass
    # prints that it does not know it, which is harmless.
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def _compile(hipcc, src, verbose):
    obj = os.path.join(OBJDIR, os.path.basename(src) + ".o")
    cmd = [hipcc, *FLAGS, f"-I{INCLUDE}", "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    # drop the host pass's notice about the device-only feature switch
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l)
    if out.strip():
        print(out, flush=True)
    if r.returncode != 0:
        raise subprocess.CalledProcessError(r.returncode, cmd)
    return obj


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJDIR, exist_ok=True)
    jobs = max(1, min(len(SOURCES), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4))))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(hipcc, s, verbose), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    print(LIB)
    sys.exit(0)
