"""Builds libfastpfp.so (HIP device code for gfx950 + C++ host API).

    python -m paper_1207_1114_amd.build

The library lands next to this file so that it travels with the source tree.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libfastpfp.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
ARCH = "gfx950"

# (source, object name, extra defines).  The solver kernel source is compiled
# once per inner projection so that each kernel sits alone in its code object
# (sharing one, the out-of-line helpers are register-allocated for both
# callers and the alternating kernel spills more).
HIP_SOURCES = [("fastpfp_kernels.hip", "fastpfp_kernels", []),
               ("fastpfp_kernels.hip", "fastpfp_kernels_dykstra",
                ["-DFPFP_DYKSTRA_BUILD=1"]),
               ("warmstart.hip", "warmstart", []),
               ("discretize_device.hip", "discretize_device", []),
               ("project_stream.hip", "project_stream", []),
               ("noalloc.hip", "noalloc", [])]
CXX_SOURCES = ["fastpfp_api.cpp", "warmstart_api.cpp", "discretize.cpp",
               "discretize_device_api.cpp", "project_stream_api.cpp"]

# Packed FP32 VALU instructions stay off: ordinary float code only.
HIPCC_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-munsafe-fp-atomics", "-Wno-unused-command-line-argument"]
CXX_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-Wall", "-D__HIP_PLATFORM_AMD__",
             f"-I{ROCM}/include"]


def _run(cmd: list[str]) -> None:
    r = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                    if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"build step failed: {' '.join(cmd)}\n{out}")
    if out.strip():
        print(out, file=sys.stderr)


def build(verbose: bool = False, jobs: int = 4) -> str:
    """Compiles every source (independent compiles in parallel) and links
    the library; always rebuilds."""
    from concurrent.futures import ThreadPoolExecutor
    os.makedirs(BUILD, exist_ok=True)
    hipcc = os.path.join(ROCM, "bin", "hipcc")
    cmds, objs = [], []
    for src, name, defs in HIP_SOURCES:
        obj = os.path.join(BUILD, name + ".hip.o")
        cmds.append([hipcc, *HIPCC_FLAGS, *defs, f"-I{INCLUDE}", f"-I{CSRC}",
                     "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    for src in CXX_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        cmds.append(["g++", *CXX_FLAGS, f"-I{INCLUDE}", f"-I{CSRC}", "-c",
                     os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    with ThreadPoolExecutor(max_workers=max(1, jobs)) as pool:
        for f in [pool.submit(_run, c) for c in cmds]:
            f.result()
    tmp = LIB + ".tmp"
    _run([hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o",
          tmp])
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
