"""Build the HIP library libocp_admm.so in-tree for gfx950 with hipcc.

The kernels of each compiled stage shape and iteration precision sit in
their own translation unit (csrc/inst.hip compiled with -D flags), the host
code in csrc/ocp.hip; the units compile in parallel and link into one
shared library.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB_NAME = "libocp_admm.so"
LIB_PATH = os.path.join(HERE, LIB_NAME)

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # packed FP32 instructions are kept off for all device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]

# (nx, nu, ng) of the table in csrc/ocp.hip; each in FP64 and FP32 iterations
SHAPES = ((4, 2, 4), (12, 4, 16), (4, 2, 3))


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the ROCm toolchain is required to build the library")


def units():
    """(object name, source, extra flags) of every translation unit."""
    out = [("ocp", "ocp.hip", [])]
    for nx, nu, ng in SHAPES:
        for prec in ("f64", "f32"):
            flags = [f"-DOCP_NX={nx}", f"-DOCP_NU={nu}", f"-DOCP_NG={ng}"] + (["-DOCP_F32"] if prec == "f32" else [])
            out.append((f"inst_{nx}_{nu}_{ng}_{prec}", "inst.hip", flags))
    return out


def build(verbose: bool = False, jobs: int | None = None) -> str:
    """Compile every unit and link paper_2606_24039_amd/libocp_admm.so (always rebuilds)."""
    cc = hipcc()
    jobs = jobs or max(1, min(len(units()), len(os.sched_getaffinity(0)), 16))
    with tempfile.TemporaryDirectory(prefix="ocp_build_") as tmpdir:
        def compile_one(u):
            name, src, flags = u
            obj = os.path.join(tmpdir, name + ".o")
            cmd = [cc, *HIPCC_FLAGS, *flags, f"-I{INCLUDE}", f"-I{CSRC}", "-c", os.path.join(CSRC, src), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            res = subprocess.run(cmd, capture_output=True, text=True)
            if res.returncode != 0:
                raise RuntimeError(f"hipcc failed on {name} ({res.returncode}):\n{res.stderr}")
            return obj

        with ThreadPoolExecutor(jobs) as ex:
            objs = list(ex.map(compile_one, units()))
        tmp = LIB_PATH + ".tmp"
        cmd = [cc, "--offload-arch=gfx950", "-fPIC", "-shared", *objs, "-o", tmp]
        if verbose:
            print(" ".join(cmd), flush=True)
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            raise RuntimeError(f"link failed ({res.returncode}):\n{res.stderr}")
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
