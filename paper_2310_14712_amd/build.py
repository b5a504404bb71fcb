"""Build libimex.so (host setup + HIP kernels for gfx950) in the package
directory with hipcc.  Run as ``python -m paper_2310_14712_amd.build``."""
from __future__ import annotations

import concurrent.futures
import os
import subprocess
import sys
import time

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libimex.so")
OBJ = os.path.join(PKG, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("IMEX_OFFLOAD_ARCH", "gfx950")
COMMON = ["-O3", "-std=c++17", "-fPIC", "-I", os.path.join(ROOT, "include"), "-I", CSRC]
DEVICE_FLAGS = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
SOURCES = [
    ("basis.cpp", False),
    ("setup.cpp", False),
    ("nd_factor.cpp", False),
    ("capi.cpp", True),
    ("explicit.hip", True),
    ("implicit.hip", True),
    ("util.hip", True),
    ("setup_gpu.hip", True),
    ("learned.hip", True),
    ("learned_host.cpp", "host+hip"),
]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout)
        raise RuntimeError("build step failed: " + " ".join(cmd))
    return r.stdout


def build(verbose: bool = True) -> str:
    """Compile every source (always) and link libimex.so; returns its path."""
    os.makedirs(OBJ, exist_ok=True)
    objs, cmds = [], []
    t0 = time.time()
    for src, is_hip in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(OBJ, src + ".o")
        if is_hip == "host+hip":  # host code that calls the HIP runtime, with OpenMP
            cmd = [HIPCC, "-x", "c++", "-fopenmp", "-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include", *COMMON,
                   "-c", path, "-o", obj]
        elif is_hip:
            cmd = [HIPCC, "-x", "hip", *DEVICE_FLAGS, *COMMON, "-c", path, "-o", obj]
        else:
            cmd = [HIPCC, "-x", "c++", "-fopenmp", *COMMON, "-c", path, "-o", obj]
        cmds.append(cmd)
        objs.append(obj)
    # the translation units are independent: compile them side by side
    jobs = max(1, min(len(cmds), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    with concurrent.futures.ThreadPoolExecutor(max_workers=jobs) as ex:
        list(ex.map(_run, cmds))
    tmp = LIB + ".tmp"
    _run([HIPCC, *DEVICE_FLAGS, "-shared", "-fopenmp", "-o", tmp, *objs,
          "-Wl,-rpath,/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/llvm/lib"])
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB} in {time.time() - t0:.1f} s")
    return LIB


if __name__ == "__main__":
    build()
