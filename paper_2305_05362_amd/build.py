"""Build step for the RAM HIP library (libram.so, in-tree, for gfx950).

    python -m paper_2305_05362_amd.build

compiles csrc/*.hip and csrc/ram_api.cpp with hipcc into
paper_2305_05362_amd/libram.so.  Cross-compiles on a machine without a GPU.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB_PATH = os.path.join(HERE, "libram.so")
ARCH = os.environ.get("RAM_OFFLOAD_ARCH", "gfx950")

SOURCES = ["ram_kernels.hip", "ram_step_shared.hip", "ram_step_fast.hip", "ram_step_fast64.hip", "ram_adjoint.hip",
           "ram_adjoint_shared.hip", "ram_adjoint_fast.hip", "ram_limited.hip", "ram_reduce.hip", "ram_radial.hip",
           "ram_average4.hip", "ram_noalloc.hip", "ram_api.cpp"]

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # keep the compiler from emitting packed FP32 arithmetic
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # hardware FP atomics for the adjoint's boundary accumulation
    "-munsafe-fp-atomics",
    "-Wall", "-Wno-unused-function",
]


# sources of the shared-mesh step kernel (the one the traffic counters cover)
STEP_KERNEL_SOURCES = ["ram_step_shared.hip", "ram_device.h", "ram_internal.h"]
# sources of each kernel family whose counters are committed
FAST_SOURCES = ["ram_step_fast.hip", "ram_wave.h", "ram_device.h", "ram_internal.h"]
ADJ_FAST_SOURCES = ["ram_adjoint_fast.hip", "ram_adjoint_dev.h", "ram_wave.h", "ram_device.h",
                    "ram_internal.h"]
KERNEL_SOURCES = {"k_step_sh": STEP_KERNEL_SOURCES,
                  "k_step_uni": FAST_SOURCES,
                  "k_step_gen": FAST_SOURCES,
                  "k_step_rag": FAST_SOURCES,
                  "k_step_uni_lim": FAST_SOURCES,
                  "k_step_gen_lim": FAST_SOURCES,
                  "k_step64": ["ram_step_fast64.hip", "ram_kernels.hip", "ram_wave.h", "ram_device.h",
                               "ram_internal.h"],
                  "k_adjf_uni": ADJ_FAST_SOURCES,
                  "k_adjf_gen": ADJ_FAST_SOURCES,
                  "k_ladj": ADJ_FAST_SOURCES,
                  "k_radial": ["ram_radial.hip", "ram_device.h", "ram_internal.h"],
                  "k_average4": ["ram_average4.hip", "ram_device.h", "ram_internal.h"],
                  "k_adj_sh": ["ram_adjoint_shared.hip", "ram_adjoint_dev.h", "ram_device.h",
                               "ram_internal.h"],
                  "k_shift_lim_adj": ["ram_adjoint.hip", "ram_device.h", "ram_internal.h"]}


def kernel_digest(kernel: str = "k_step_sh") -> str:
    """Digest of one kernel family's sources and the compile flags (`kernel`
    names the family, e.g. "k_step_sh" or "k_radial<float, 16>")."""
    import hashlib
    fam = kernel.split("<")[0].split("::")[-1]
    h = hashlib.sha256(" ".join(HIPCC_FLAGS).encode())
    for name in KERNEL_SOURCES[fam]:
        with open(os.path.join(CSRC, name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def hipcc() -> str:
    path = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(path):
        raise RuntimeError("hipcc not found; the RAM library needs ROCm")
    return path


def build_library(verbose: bool = False) -> str:
    objs = []
    build_dir = os.path.join(HERE, "_build")
    os.makedirs(build_dir, exist_ok=True)
    for src in SOURCES:
        obj = os.path.join(build_dir, os.path.splitext(src)[0] + ".o")
        cmd = [hipcc(), *HIPCC_FLAGS, "-I", INCLUDE, "-I", CSRC, "-c",
               os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = LIB_PATH + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp,
           *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


if __name__ == "__main__":
    print(build_library(verbose="-v" in sys.argv))
