"""Build liblbm.so: HIP kernels for gfx950 with hipcc, host code (grid
builder, C-ABI, scheduler) with g++ and OpenMP, linked by hipcc."""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "liblbm.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")

HIP_SOURCES = ["k_d2q9.hip", "k_d3q27.hip", "k_d2q13.hip", "k_d2q21.hip", "k_d2q37.hip", "k_d2q37_newton64.hip",
               "k_d2q37_newton32.hip", "mlp.hip", "k_remesh.hip", "sums.hip",
               "grid_device.hip"]
CXX_SOURCES = ["grid_builder.cpp", "layout.cpp", "remesh.cpp", "lbm_api.cpp"]
HIPCC_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]
# per-unit flags: the surrogate's matrix products accumulate in ordinary
# VGPRs (not AGPRs), so that the collide holding the Newton state next to
# them keeps two wavefronts per SIMD
UNIT_FLAGS = {"k_d2q21.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form=1"],
              "mlp.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form=1"]}
CXX_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-fopenmp", "-D__HIP_PLATFORM_AMD__",
             "-I" + os.path.join(ROOT, "include"), "-I" + CSRC, "-I" + os.path.join(ROCM, "include")]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError("build failed: " + " ".join(cmd) + "\n" + out)
    return out


def torch_lib_dir() -> str:
    """PyTorch's bundled HIP runtime: the library must share it with torch,
    so that one HIP runtime owns the device in the process."""
    import torch
    return os.path.join(os.path.dirname(torch.__file__), "lib")


def _stale(obj: str, src: str) -> bool:
    """an object is stale when it is older than its source or any header"""
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    deps = [src] + [os.path.join(d, h) for d in (CSRC, os.path.join(ROOT, "include"))
                    for h in os.listdir(d) if h.endswith((".h", ".cuh"))]
    return any(os.path.getmtime(p) > t for p in deps)


def build(verbose: bool = False, jobs: int = 8, incremental: bool = False) -> str:
    """compile every source (or, with incremental=True, only the objects
    older than their source or a header) and link liblbm.so"""
    os.makedirs(BUILD, exist_ok=True)
    cmds = []
    objs = []
    for s in HIP_SOURCES:
        o = os.path.join(BUILD, s.replace(".hip", ".o"))
        if not incremental or _stale(o, os.path.join(CSRC, s)):
            cmds.append([os.path.join(ROCM, "bin", "hipcc")] + HIPCC_FLAGS + UNIT_FLAGS.get(s, [])
                        + ["-c", os.path.join(CSRC, s), "-o", o])
        objs.append(o)
    for s in CXX_SOURCES:
        o = os.path.join(BUILD, s.replace(".cpp", ".o"))
        if not incremental or _stale(o, os.path.join(CSRC, s)):
            cmds.append(["g++"] + CXX_FLAGS + ["-c", os.path.join(CSRC, s), "-o", o])
        objs.append(o)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        for out in ex.map(_run, cmds):
            if verbose and out.strip():
                print(out)
    tmp = LIB + ".tmp"
    tdir = torch_lib_dir()
    _run(["g++", "-shared", "-fPIC", "-o", tmp] + objs
         + ["-L" + tdir, "-l:libamdhip64.so", "-lgomp", "-Wl,-rpath," + tdir, "-Wl,--no-undefined"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, incremental="-i" in sys.argv))
