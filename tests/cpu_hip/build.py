"""Build the library's sources for the CPU (test infrastructure).

The HIP sources of ``paper_2502_19342_amd/csrc`` are compiled as C++ against
the CPU stand-in ``tests/cpu_hip/hip/hip_runtime.h`` with AddressSanitizer and
UndefinedBehaviorSanitizer, into ``tests/cpu_hip/_build/libdgfv_cpu.so``, which
exports the same C ABI as the GPU library.  A process that loads it needs
libasan preloaded (``asan_env()``).
"""
from __future__ import annotations

import fcntl
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_2502_19342_amd", "csrc")
OUT = os.path.join(HERE, "_build")
LIB = os.path.join(OUT, "libdgfv_cpu.so")
FLAGS = ["-std=c++17", "-O1", "-g", "-fPIC", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
         "-fno-sanitize-recover=undefined", "-Wno-unused-function", "-I", HERE,
         # the adjoint paths that stay off on the GPU run here
         "-DDGFV_CPU_ADJOINT_ALL_PATHS"]


def _jobs():
    jobs = [(["-x", "c++", os.path.join(CSRC, "dgfv_degree.hip"), f"-DDGFV_N={n}"],
             os.path.join(OUT, f"degree_{n}.o")) for n in range(1, 8)]
    jobs += [(["-x", "c++", os.path.join(CSRC, "dgfv_viscous.hip"), f"-DDGFV_N={n}"],
              os.path.join(OUT, f"viscous_{n}.o")) for n in range(1, 8)]
    for name in ("dgfv_faces.hip", "dgfv_lists.hip", "dgfv_state.hip", "dgfv_fvstored.hip"):
        jobs.append((["-x", "c++", os.path.join(CSRC, name)], os.path.join(OUT, name.replace(".hip", ".o"))))
    for name in ("dgfv_host.cpp", "dgfv_ops1d.cpp"):
        jobs.append(([os.path.join(CSRC, name)], os.path.join(OUT, name.replace(".cpp", ".o"))))
    jobs.append(([os.path.join(HERE, "cpu_hip_runtime.cpp")], os.path.join(OUT, "cpu_hip_runtime.o")))
    return jobs


def _sources():
    srcs = [os.path.join(CSRC, f) for f in os.listdir(CSRC)]
    srcs += [os.path.join(HERE, "cpu_hip_runtime.cpp"), os.path.join(HERE, "hip", "hip_runtime.h"), __file__]
    return srcs


def _fresh() -> bool:
    if not os.path.exists(LIB):
        return False
    t = os.path.getmtime(LIB)
    return all(os.path.getmtime(s) <= t for s in _sources())


def build(force: bool = False) -> str:
    """Compile (when a source is newer than the library) and return the library path.

    Test processes running side by side take turns through a lock file."""
    if not force and _fresh():
        return LIB
    os.makedirs(OUT, exist_ok=True)
    with open(os.path.join(OUT, ".lock"), "w") as lk:
        fcntl.flock(lk, fcntl.LOCK_EX)
        if not force and _fresh():
            return LIB
        return _compile()


def _compile() -> str:

    def run(job):
        args, obj = job
        cmd = ["g++"] + FLAGS + ["-c"] + args + ["-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stderr[-6000:]}")
        return obj

    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(run, _jobs()))
    tmp = LIB + ".tmp"
    r = subprocess.run(["g++", "-shared", "-fsanitize=address,undefined", "-o", tmp] + objs + ["-lpthread"],
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed\n{r.stderr[-4000:]}")
    os.replace(tmp, LIB)
    return LIB


def asan_env() -> dict:
    """Environment for a child process that loads the CPU library."""
    lib = subprocess.run(["g++", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    env = dict(os.environ)
    env["LD_PRELOAD"] = lib
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1:allocator_may_return_null=0"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    return env


if __name__ == "__main__":
    print(build(force="-f" in sys.argv))
