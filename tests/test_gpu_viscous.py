"""Viscous multi-species terms on the GPU against the oracle (Sections 2, 3.1.1 and 3.2.2).

The BR1-lifted gradient, the rate with the viscous terms on curved scrambled
meshes with degree jumps and blended elements (one and two species), RK steps
under graph replay, the switch back to the inviscid rate, and the viscous
Taylor-Green workload at full size (64^3 elements, N = 7) against the exact
viscous rate of its initial state at sampled nodes.
"""
import dataclasses

import numpy as np
import pytest
import torch

from oracle import lsrk, viscous
from paper_2502_19342_amd import workloads as W

from gpu_common import Case, announce, rel_err, rhs_tol
from oracle_cases import curved_mixed, seeded_alpha, smooth_state

pytestmark = pytest.mark.gpu
T = torch.float64


def _wl(n_var=5, n=3, nmin=1, nmax=4, scramble=19, n_fv=5, metric_degree=0):
    flux = {} if n_var == 5 else dict(volume_flux=W.VOL_PIROZZOLI, face_dg=W.RIEMANN_LLF)
    wl = curved_mixed(n=n, nmin=nmin, nmax=nmax, n_var=n_var, scramble=scramble, metric_degree=metric_degree,
                      n_fv=n_fv, **flux)
    return dataclasses.replace(wl, mu=(0.02, 0.03), Pr=(0.7, 0.9), D=(0.01, 0.04))


@pytest.mark.parametrize("n_var", [5, 6])
def test_lift_on_gpu(n_var):
    announce(f"viscous lift n_var={n_var}")
    from paper_2502_19342_amd import dgfv
    c = Case(_wl(n_var), prim=smooth_state(61, n_var), noise=1e-3, seed=2)
    g = dgfv.lift(c.gmesh, c.gpu(c.u))
    torch.cuda.synchronize()
    want = viscous.lift(c.mesh, c.u)
    assert rel_err(g.cpu().reshape(3 * n_var, -1), want.reshape(3 * n_var, -1)) <= 1e-12


@pytest.mark.parametrize("n_var", [5, 6])
def test_viscous_rhs_on_gpu(n_var):
    announce(f"viscous rhs blended n_var={n_var}")
    c = Case(_wl(n_var), prim=smooth_state(63, n_var), noise=1e-3, seed=3)
    c.alpha = seeded_alpha(c.mesh.K, 64, values=(0.0, 0.0, 0.4, 1.0))
    err = rel_err(c.gpu_rhs(), c.oracle_rhs())
    print(f"[viscous] rhs rel err {err:.3e}", flush=True)
    assert err <= rhs_tol(c)


def test_viscous_rk_steps_with_graphs():
    announce("viscous 10 RK steps, graph replays")
    from paper_2502_19342_amd import dgfv
    c = Case(_wl(5, nmin=2, nmax=5, scramble=23, n_fv=6), prim=smooth_state(65), noise=1e-3, seed=4)
    dt = 0.3 * lsrk.timestep(c.mesh, c.gas, c.u, 0.5)
    c.gmesh.graphs(True)
    ug = c.gpu(c.u)
    k = torch.zeros_like(ug)
    uo = c.u.clone()
    for _ in range(10):
        dgfv.rk_step(c.gmesh, c.params, dt, ug, k, None)
        uo = lsrk.step(lambda v: c.f(v, c.alpha), uo, dt)
    torch.cuda.synchronize()
    err = rel_err(ug.cpu(), uo)
    print(f"[viscous] 10 steps rel err {err:.3e}", flush=True)
    assert err <= 1e-10


def test_viscous_step_with_traces_equals_stages():
    # degrees 6 and 7: between the stages of dg_rk_step the lift kernel reads the
    # neighbours' xi_1 sides from the traces; five dg_rk_stage calls read them from u
    announce("viscous step with traces, N=6,7")
    from paper_2502_19342_amd import dgfv
    c = Case(_wl(5, n=3, nmin=6, nmax=7, scramble=31, n_fv=8), prim=smooth_state(71), noise=1e-3, seed=8)
    dt = 0.3 * lsrk.timestep(c.mesh, c.gas, c.u, 0.5)
    a, b = c.gpu(c.u), c.gpu(c.u)
    ka, kb = torch.zeros_like(a), torch.zeros_like(b)
    dgfv.rk_step(c.gmesh, c.params, dt, a, ka, None)
    for st in range(1, 6):
        dgfv.rk_stage(c.gmesh, c.params, st, dt, b, kb, None)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    uo = lsrk.step(lambda v: c.f(v, c.alpha), c.u, dt)
    assert rel_err(a.cpu(), uo) <= 1e-11


def test_viscous_switch_and_unsupported_calls():
    announce("viscous on/off, unsupported calls")
    from paper_2502_19342_amd import dgfv
    c = Case(_wl(5), prim=smooth_state(67), noise=1e-3, seed=5)
    u = c.gpu(c.u)
    r_visc = dgfv.rhs(c.gmesh, c.params, u)
    c.gmesh.transport((0.0, 0.0), (0.7, 0.7), (0.0, 0.0))     # no viscosity: the inviscid rate exactly
    r_zero = dgfv.rhs(c.gmesh, c.params, u)
    c.gmesh.transport(None)
    r_off = dgfv.rhs(c.gmesh, c.params, u)
    torch.cuda.synchronize()
    assert torch.equal(r_zero, r_off)
    assert not torch.equal(r_visc, r_off)
    c.gmesh.transport(c.wl.mu, c.wl.Pr, c.wl.D)
    K, nf = c.mesh.K, c.wl.n_fv
    with pytest.raises(dgfv.DgfvError):
        dgfv.rhs_fv(c.gmesh, c.params, u, torch.zeros(K, 5, nf ** 3, dtype=T, device="cuda"),
                    torch.zeros(K, dtype=T, device="cuda"))
    with pytest.raises(dgfv.DgfvError):
        dgfv.rhs_vjp(c.gmesh, c.params, u, None, torch.ones_like(u))
    r_again = dgfv.rhs(c.gmesh, c.params, u)
    torch.cuda.synchronize()
    assert torch.equal(r_again, r_visc)


@pytest.mark.parametrize("n_var,viscous", [(5, True), (6, True), (6, False)])
def test_timestep_on_gpu(n_var, viscous):
    announce(f"time step n_var={n_var} viscous={viscous}")
    from oracle import problem
    from paper_2502_19342_amd import dgfv
    wl = _wl(n_var, scramble=29)
    if not viscous:
        wl = dataclasses.replace(wl, mu=(0.0, 0.0), D=(0.0, 0.0))
    c = Case(wl, prim=smooth_state(69, n_var), noise=1e-3, seed=7)
    c.alpha = seeded_alpha(c.mesh.K, 70, values=(0.0, 0.0, 0.4, 1.0))
    got = dgfv.timestep(c.gmesh, c.gpu(c.u), c.gpu(c.alpha), 0.6, 0.3)
    want = lsrk.timestep(c.mesh, c.gas, c.u, 0.6, c.alpha, problem.transport_of(wl) if viscous else None, 0.3)
    assert abs(got - want) <= 1e-13 * want
    bad = c.u.clone()
    bad[0, 7] = -1.0                                           # negative density: no time step
    with pytest.raises(dgfv.DgfvError):
        dgfv.timestep(c.gmesh, c.gpu(bad), None, 0.6, 0.3)


def _exact_viscous_rate(wl, x: np.ndarray, gas) -> torch.Tensor:
    """-div F^v of the exact initial state at points x [P, 3] (autograd, float64)."""
    xt = torch.as_tensor(x, dtype=T).requires_grad_(True)
    k = 2 * np.pi
    gam = wl.gamma
    s = [torch.sin(k * xt[:, d]) for d in range(3)]
    cs = [torch.cos(k * xt[:, d]) for d in range(3)]
    p = 1.0 / (gam * 0.01) + (torch.cos(2 * k * xt[:, 0]) + torch.cos(2 * k * xt[:, 1])) * \
        (torch.cos(2 * k * xt[:, 2]) + 2.0) / 16.0
    v = torch.stack([s[0] * cs[1] * cs[2], -cs[0] * s[1] * cs[2], torch.zeros_like(p)])
    rho = torch.ones_like(p)
    u = torch.stack([rho, rho * v[0], rho * v[1], rho * v[2], p / (gam - 1.0) + 0.5 * rho * (v * v).sum(0)])
    g = torch.stack([torch.stack([torch.autograd.grad(u[c].sum(), xt, create_graph=True)[0][:, d]
                                  for c in range(5)]) for d in range(3)])          # [3, 5, P]
    F = viscous.viscous_flux(u, g, gas, viscous.Transport(mu=tuple(wl.mu), Pr=tuple(wl.Pr), D=tuple(wl.D)))
    div = torch.zeros(5, x.shape[0], dtype=T)
    for c in range(1, 5):
        for d in range(3):
            div[c] += torch.autograd.grad(F[d, c].sum(), xt, retain_graph=True)[0][:, d]
    return -div.detach()


def test_tgv_full_size_viscous_rate():
    # 64^3 elements at N = 7: the GPU's viscous rate (with minus without the
    # viscous terms) at 4096 sampled nodes against the exact rate of the
    # initial state; spectral accuracy leaves ~1e-8 of the rate's scale
    announce("TGV 64^3 N=7 viscous rate, sampled")
    from paper_2502_19342_amd import dgfv
    from oracle import problem
    wl = W.make_workload("TGV")
    gm = dgfv.Mesh.from_workload(wl)
    prm = dgfv.params_of(wl)
    xyz = gm.node_coords()
    w = torch.as_tensor(np.asarray(wl.prim(xyz.T))).to("cuda").contiguous()
    u = dgfv.prim_to_cons(gm, w)
    r_v = dgfv.rhs(gm, prm, u)
    gm.transport(None)
    r_c = dgfv.rhs(gm, prm, u)
    torch.cuda.synchronize()
    idx = torch.as_tensor(np.random.default_rng(7).choice(gm.n_node, 4096, replace=False))
    got = (r_v - r_c)[:, idx.cuda()].cpu()
    want = _exact_viscous_rate(wl, xyz[:, idx.numpy()].T, problem.gas_of(wl))
    diff = (got - want).abs().amax(dim=1)
    e_mom = float(diff[1:4].max() / want[1:4].abs().max())      # the rate of rho v3 is zero
    e_en = float(diff[4] / want[4].abs().max())
    print(f"[viscous] TGV sampled rel err: momentum {e_mom:.3e}, energy {e_en:.3e}", flush=True)
    assert e_mom <= 1e-6 and e_en <= 1e-6
    assert float(got[0].abs().max()) == 0.0
