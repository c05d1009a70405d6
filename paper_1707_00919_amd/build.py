"""Build libmuca.so (the C-ABI library of include/muca.h) for gfx950 in-tree.

    python -m paper_1707_00919_amd.build

Compiles the HIP kernels and the host runtime with hipcc and links them into
``paper_1707_00919_amd/libmuca.so``.  No fast-math and no floating-point
contraction: the host threshold table and the weight update must round
exactly as written.
"""
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libmuca.so")
ARCH = "gfx950"

SOURCES = ["muca_kernels.hip", "muca_sweep_fast.hip", "muca_sweep_split.hip", "muca_sweep_wide.hip", "muca_runtime.cpp",
           "muca_host_math.cpp", "muca_batch.cpp", "muca_server.cpp", "muca_analysis.cpp", "muca_probe.hip", "muca_static.hip",
           "muca_order.hip"]
COMMON = [
    "-O3", "-std=c++17", "-fPIC", "-Wall",
    "-ffp-contract=off", "-fno-fast-math",
    "-I" + INCLUDE, "-I" + CSRC,
]
DEVICE = [
    "--offload-arch=" + ARCH,
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc():
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def _compile(src, obj_dir):
    path = os.path.join(CSRC, src)
    obj = os.path.join(obj_dir, src + ".o")
    # host-only sources are still HIP translation units (they include the HIP
    # runtime); they hold no kernels, but are built for the same target
    cmd = [hipcc()] + COMMON + DEVICE + ["-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, " ".join(cmd), r.stderr))
    return obj


def build(verbose=False):
    """Compile and link libmuca.so; returns its path."""
    obj_dir = os.path.join(HERE, "_build")
    os.makedirs(obj_dir, exist_ok=True)
    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(lambda s: _compile(s, obj_dir), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (" ".join(cmd), r.stderr))
    os.replace(tmp, LIB)
    if verbose:
        print(LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
