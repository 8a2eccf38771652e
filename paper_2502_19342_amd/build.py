"""Build the HIP library ``libdgfv.so`` in-tree for gfx950 with hipcc.

Usage: ``python -m paper_2502_19342_amd.build`` (or ``build()`` from Python).
The per-degree kernels are compiled as seven objects in parallel.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libdgfv.so")
ARCH = os.environ.get("DGFV_OFFLOAD_ARCH", "gfx950")

COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Wall", "-Wno-unused-function"]
# packed FP32 instructions stay off in every HIP translation unit
DEVICE_ONLY = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _jobs():
    jobs = []
    for n in range(1, 8):
        jobs.append((["-x", "hip", os.path.join(CSRC, "dgfv_degree.hip"), f"-DDGFV_N={n}"] + DEVICE_ONLY,
                     os.path.join(OUT_DIR, f"dgfv_degree_{n}.o")))
        jobs.append((["-x", "hip", os.path.join(CSRC, "dgfv_viscous.hip"), f"-DDGFV_N={n}"] + DEVICE_ONLY,
                     os.path.join(OUT_DIR, f"dgfv_viscous_{n}.o")))
    for name in ("dgfv_faces", "dgfv_lists", "dgfv_state", "dgfv_fvstored"):
        jobs.append((["-x", "hip", os.path.join(CSRC, name + ".hip")] + DEVICE_ONLY,
                     os.path.join(OUT_DIR, name + ".o")))
    for name in ("dgfv_host.cpp", "dgfv_ops1d.cpp"):
        jobs.append(([os.path.join(CSRC, name)], os.path.join(OUT_DIR, name.replace(".cpp", ".o"))))
    return jobs


def build(verbose: bool = False) -> str:
    """Compile every source (always) and link ``libdgfv.so``; return its path."""
    hipcc = _hipcc()
    os.makedirs(OUT_DIR, exist_ok=True)

    def run(job):
        args, obj = job
        cmd = [hipcc] + COMMON + ["-c"] + args + ["-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
        return obj

    workers = max(1, min(10, os.cpu_count() or 1))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        objs = list(ex.map(run, _jobs()))
    tmp = LIB + ".tmp"
    cmd = [hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
