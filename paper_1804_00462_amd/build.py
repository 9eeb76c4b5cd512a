"""Build libsorsvd.so (gfx950) in-tree with hipcc.

    python -m paper_1804_00462_amd.build      # or build() from Python

Each HIP source is compiled to an object for gfx950 only, then linked into
``paper_1804_00462_amd/libsorsvd.so``. Packed FP32 instructions are disabled
for every device compile. The Gaussian generator is compiled without
floating-point contraction so that its operation sequence is exactly the
documented one.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libsorsvd.so")

SOURCES = {
    "gemm_bf16.hip": [],
    "gemm_f16.hip": [],
    "batched.hip": [],
    "small.hip": [],
    "wide.hip": [],
    "philox.hip": ["-ffp-contract=off"],
    "gemm.hip": [],
    "sorsvd.hip": [],
    "pack.hip": [],
    "noalloc.hip": [],
    "residual.hip": [],
    "mlp.hip": [],
    "rpca.hip": [],
}

COMMON = [
    "--offload-arch=gfx950",
    "-O3",
    "-fPIC",
    "-std=c++17",
    "-Wall",
    "-Wno-unused-result",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", INCLUDE,
]


def hipcc():
    for cand in ("/opt/rocm/bin/hipcc", "hipcc"):
        if os.path.sep not in cand or os.path.exists(cand):
            return cand
    return "hipcc"


def _compile(src, extra, verbose):
    obj = os.path.join(BUILD, src.replace(".hip", ".o"))
    cmd = [hipcc(), *COMMON, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed on {src}")
    return obj


def build(verbose=False, jobs=None):
    """Compiles the sources in parallel (jobs: worker count, default
    min(8, CPUs)) and links the library."""
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or max(1, min(8, os.cpu_count() or 1))
    with ThreadPoolExecutor(max_workers=jobs) as ex:  # SOURCES lists the slowest units first
        futs = {src: ex.submit(_compile, src, SOURCES[src], verbose) for src in SOURCES}
        objs = [futs[src].result() for src in SOURCES]
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("link of libsorsvd.so failed")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
