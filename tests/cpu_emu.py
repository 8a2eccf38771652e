"""Runs C-ABI calls of the CPU (AddressSanitizer) build of the library in a child process."""
import os
import subprocess
import sys
import tempfile

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def _builder():
    import importlib.util
    spec = importlib.util.spec_from_file_location("cpu_hip_build", os.path.join(HERE, "cpu_hip", "build.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def run(wl, u, calls, alpha=None, w=None, dt=None, launch_mode=None, timeout=900, guard="end", **extra):
    """Mesh of workload ``wl``; ``calls`` in rhs, vjp, rk_step, stage_vjp, prim_to_cons,
    indicator, coords (``extra`` arrays, e.g. stage, ubar, kbar, go to the child as they are)."""
    cpu_build = _builder()
    cpu_build.build()
    m = wl.mesh
    z = dict(degree=np.asarray(m.degree), corners=np.asarray(m.corners), faces=np.asarray(m.faces),
             n_var=wl.n_var, n_fv=wl.n_fv, metric_degree=wl.metric_degree, gamma=wl.gamma,
             kappa=np.asarray(wl.kappa, dtype=np.float64), R=np.asarray(wl.R, dtype=np.float64),
             params=np.array([wl.volume_flux, wl.face_flux_dg, wl.face_flux_fv, wl.ind_vars, wl.ind_T,
                              wl.ind_dT], dtype=np.float64),
             u=np.asarray(u, dtype=np.float64), calls=np.array(calls))
    if len(getattr(m, "mortars", [])):
        z["mortars"] = np.asarray(m.mortars, dtype=np.int32)
    if getattr(wl, "viscous", False):
        z["transport"] = np.asarray(tuple(wl.mu) + tuple(wl.Pr) + tuple(wl.D), dtype=np.float64)
    if alpha is not None:
        z["alpha"] = np.asarray(alpha, dtype=np.float64)
    if w is not None:
        z["w"] = np.asarray(w, dtype=np.float64)
    if dt is not None:
        z["dt"] = float(dt)
    if launch_mode is not None:
        z["launch_mode"] = int(launch_mode)
    for key, val in extra.items():
        z[key] = np.asarray(val)
    with tempfile.TemporaryDirectory() as td:
        src, dst = os.path.join(td, "in.npz"), os.path.join(td, "out.npz")
        np.savez(src, **z)
        env = cpu_build.asan_env()
        env["CPU_HIP_GUARD"] = guard
        r = subprocess.run([sys.executable, os.path.join(HERE, "cpu_hip", "drive.py"), src, dst],
                           capture_output=True, text=True, env=env, timeout=timeout)
        if r.returncode != 0:
            raise RuntimeError(f"CPU build run failed ({r.returncode}):\n{r.stdout[-3000:]}\n{r.stderr[-12000:]}")
        return dict(np.load(dst))
