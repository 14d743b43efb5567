"""Builds libgsmap.so (the HIP kernels behind the C ABI) for gfx950.

Every translation unit is compiled by hipcc for gfx950 only.  Packed FP32
instructions are disabled for device code.  The projection, view-dependent
colour and compositing units are compiled without FMA contraction: the
projection so its FP64 front end rounds exactly in source order, the others
so their forward and backward kernels take bit-identical decisions (they
place FMAs explicitly).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
LIB = os.path.join(HERE, "libgsmap.so")
OBJ = os.path.join(HERE, "_build")

ARCH = "gfx950"
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
          "-munsafe-fp-atomics", "-Xclang", "-target-feature", "-Xclang",
          "-packed-fp32-ops", "-fvisibility=hidden", "-I", INCLUDE,
          "-Wall", "-Wno-unused-result"]
NO_CONTRACT = ["-ffp-contract=off"]
# The backward adds row partial sums into LDS from a few lanes per wave; the
# compiler's atomic optimizer would turn each such add into a serial
# cross-lane loop.
NO_ATOMIC_OPT = ["-mllvm", "-amdgpu-atomic-optimizer-strategy=None"]

# (source, extra flags)
UNITS = [
    ("api.hip", []),
    ("project.hip", NO_CONTRACT),
    ("sh.hip", NO_CONTRACT),
    ("bin.hip", []),
    ("sort.hip", []),
    ("render_fwd.hip", NO_CONTRACT),
    ("render_bwd.hip", NO_CONTRACT + NO_ATOMIC_OPT),
    ("optim.hip", []),
    ("ssim.hip", []),
    ("densify.hip", []),
    ("mlp.hip", NO_CONTRACT),
    ("window.hip", []),
    ("noalloc.hip", []),
]


def hipcc() -> str:
    path = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    return path


def _compile(src, extra, verbose):
    obj = os.path.join(OBJ, src.replace(".hip", ".o"))
    cmd = [hipcc(), *COMMON, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    msgs = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                     if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{msgs}")
    if verbose and msgs.strip():
        print(msgs)
    return obj


def build(verbose: bool = False, jobs: int = 8) -> str:
    os.makedirs(OBJ, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda u: _compile(u[0], u[1], verbose), UNITS))
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o",
           LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
