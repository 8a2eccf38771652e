"""Expected values of two long runs at full workload size, computed by the oracle alone.

* ``c2_100_steps.json``: the 16^3, N = 5 blast workload after 100 Runge-Kutta
  steps at CFL 0.5, the blending factors recomputed from the modal indicator
  at the start of every step (Section 3.4 drives the blend; Section 3.3
  steps) and the positivity limiter of Section 3.5 applied to the initial
  state and after every stage.
* ``c4_adjoint_50_steps.json``: the 16^3, N = 4 isentropic-vortex workload (with
  its additive N(0, 1e-3) perturbation): the cotangent of the initial state of
  <w, u_50> after 50 steps, reversed stage by stage through autograd of the
  oracle's stage.

Both store sampled entries, per-variable max norms and, for the adjoint,
full-field dot products with seeded directions.  Run from the repository root:
``python tests/golden/make_fullsize_rollouts.py [c2|c4]`` (about half an hour
each on 8 cores).
"""
import json
import os
import sys
import time

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import indicator, limiter, lsrk, problem  # noqa: E402
from paper_2502_19342_amd import workloads as W  # noqa: E402

T = torch.float64


def sample_positions(n_node, n_var, count, seed):
    rng = np.random.default_rng(seed)
    nodes = np.sort(rng.choice(n_node, size=count, replace=False))
    return nodes.tolist()


def c2():
    wl = W.make_workload("C2")
    mesh, gas, f = problem.build(wl)
    u = problem.initial_state(mesh, gas, wl.prim)
    _, a0 = indicator.indicator(mesh, gas, u, wl.ind_T, wl.ind_dT, wl.ind_vars)
    u = limiter.limit(mesh, gas, u, a0)[0]                 # the jump's sub-cell means, once
    dt = float(lsrk.timestep(mesh, gas, u, 0.5, a0))
    t0 = time.time()
    blended, limited = [], 0
    k = torch.zeros_like(u)
    for s in range(100):
        _, alpha = indicator.indicator(mesh, gas, u, wl.ind_T, wl.ind_dT, wl.ind_vars)
        blended.append(float((alpha > 0).double().mean()))
        for st in range(5):
            u, k = lsrk.stage(lambda v: f(v, alpha), u, k, st, dt)
            u, n_lim, n_bad = limiter.limit(mesh, gas, u, alpha)
            limited += n_lim
            assert n_bad == 0
        print(f"c2 step {s + 1}/100 ({time.time() - t0:.0f} s, blended {blended[-1]:.3f}, "
              f"limited element-stages {limited})", flush=True)
    nodes = sample_positions(mesh.n_node, wl.n_var, 2000, 2002)
    rec = {"workload": "C2 16^3 N=5 blast (the jump), 100 steps, CFL 0.5, alpha from the indicator each step, "
                       "positivity limiter on the initial state and after every stage",
           "limited_element_stages": limited,
           "dt": dt, "steps": 100, "sample_nodes": nodes,
           "u_sample": u[:, nodes].tolist(), "linf": u.abs().amax(1).tolist(),
           "blended_fraction_per_step": blended}
    with open(os.path.join(HERE, "c2_100_steps.json"), "w") as fh:
        json.dump(rec, fh)


def c4():
    wl = W.make_workload("C4")
    mesh, gas, f = problem.build(wl)
    u0 = problem.initial_state(mesh, gas, wl.prim)
    u0 = u0 + torch.as_tensor(W.noise(wl.seed, tuple(u0.shape), wl.noise), dtype=T)
    alpha = torch.zeros(mesh.K, dtype=T)
    w = torch.as_tensor(W.cotangents(4040, tuple(u0.shape)), dtype=T)
    dt = float(lsrk.timestep(mesh, gas, u0, 0.5))
    steps = 50
    A, B = lsrk.A_F64, lsrk.B_F64
    t0 = time.time()
    checkpoints = []
    u = u0
    for s in range(steps):
        checkpoints.append(u)
        u = lsrk.step(lambda v: f(v, alpha), u, dt)
    print(f"c4 forward done ({time.time() - t0:.0f} s)", flush=True)
    ub = w.clone()
    for s in reversed(range(steps)):
        # stage inputs of step s
        us, ks = [checkpoints[s]], [torch.zeros_like(u0)]
        for st in range(4):
            k = A[st] * ks[-1] + dt * f(us[-1], alpha)
            ks.append(k)
            us.append(us[-1] + B[st] * k)
        kb = torch.zeros_like(ub)
        for st in range(4, -1, -1):
            uu = us[st].clone().requires_grad_(True)
            kk = ks[st].clone().requires_grad_(True)
            k = A[st] * kk + dt * f(uu, alpha)
            un = uu + B[st] * k
            gu, gk = torch.autograd.grad((un * ub).sum() + (k * kb).sum(), (uu, kk))
            ub, kb = gu, gk
        print(f"c4 reverse step {s} ({time.time() - t0:.0f} s)", flush=True)
    g = ub
    nodes = sample_positions(mesh.n_node, wl.n_var, 2000, 4004)
    dirs = [torch.as_tensor(W.cotangents(4041 + i, tuple(u0.shape)), dtype=T) for i in range(3)]
    rec = {"workload": "C4 16^3 N=4 vortex + additive N(0,1e-3), 50 steps at CFL 0.5, pure DG, "
                       "cotangent of <w, u_50> with w = cotangents(4040)",
           "dt": dt, "steps": steps, "w_seed": 4040, "dir_seeds": [4041, 4042, 4043],
           "sample_nodes": nodes, "g_sample": g[:, nodes].tolist(), "g_linf": g.abs().amax(1).tolist(),
           "g_dot_dirs": [float((g * v).sum()) for v in dirs],
           "u_end_linf": u.abs().amax(1).tolist()}
    with open(os.path.join(HERE, "c4_adjoint_50_steps.json"), "w") as fh:
        json.dump(rec, fh)


if __name__ == "__main__":
    which = sys.argv[1:] or ["c2", "c4"]
    for name in which:
        {"c2": c2, "c4": c4}[name]()
