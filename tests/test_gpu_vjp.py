"""Parity of the HIP adjoint (dg_rhs_vjp) with the oracle's reference VJP and with finite differences.

Reference: autograd through the CPU oracle (itself pinned against central
differences on the CPU).  Bars: <= 1e-12 of the max norm of the oracle VJP per
variable (or four times the oracle's own 1-ulp spread on FV-blended cases,
as for the forward); GPU VJP against central differences of the GPU RHS
(h = 1e-6): <= 1e-6 relative.
"""
import numpy as np
import pytest
import torch

from oracle import lsrk
from paper_2502_19342_amd import workloads as W

from gpu_common import Case, announce, rel_err
from oracle_cases import curved_mixed, seeded_alpha, smooth_state

pytestmark = pytest.mark.gpu
T = torch.float64


def oracle_vjp(c, w, u=None):
    uu = (c.u if u is None else u).clone().requires_grad_(True)
    r = c.f(uu, c.alpha)
    (g,) = torch.autograd.grad((r * w).sum(), uu)
    return g


def vjp_tol(c, w, g_ref, base=1e-12):
    if not bool((c.alpha > 0).any()):
        return base
    gen = torch.Generator().manual_seed(1)
    worst = 0.0
    for _ in range(2):
        up = c.u * (1.0 + 2.0 ** -52 * torch.randn(tuple(c.u.shape), generator=gen, dtype=T))
        worst = max(worst, rel_err(oracle_vjp(c, w, up), g_ref))
    return max(base, 4.0 * worst)


def gpu_vjp(c, w, alpha="case"):
    from paper_2502_19342_amd import dgfv
    a = c.gpu(c.alpha) if alpha == "case" else alpha
    g = dgfv.rhs_vjp(c.gmesh, c.params, c.gpu(c.u), a, c.gpu(w))
    torch.cuda.synchronize()
    return g.cpu()


def cot(c, seed):
    return torch.as_tensor(W.cotangents(seed, tuple(c.u.shape)), dtype=T)


@pytest.mark.parametrize("vol,face", [(W.VOL_RANOCHA, W.RIEMANN_ROE_HH), (W.VOL_PIROZZOLI, W.RIEMANN_LLF),
                                      (W.VOL_CENTRAL, W.RIEMANN_EC)])
def test_vjp_dg_uniform(vol, face):
    announce(f"vjp dg uniform {vol} {face}")
    wl = curved_mixed(n=3, nmin=3, nmax=3, scramble=21, volume_flux=vol, face_dg=face)
    c = Case(wl, prim=smooth_state(81), noise=1e-3, seed=6)
    w = cot(c, 82)
    g_ref = oracle_vjp(c, w)
    assert rel_err(gpu_vjp(c, w, alpha=None), g_ref) <= 1e-12


FAULT_SKIP = pytest.mark.skip(reason="the adjoint of FV-blended elements and degree jumps faulted the GPU "
                               "once; the path is switched off (DGFV_ERR_UNSUPPORTED) until the cause is found")


@FAULT_SKIP
def test_vjp_mixed_degree_blended():
    announce("vjp mixed blended")
    wl = curved_mixed(n=3, nmin=1, nmax=4, scramble=23, metric_degree=1, n_fv=5)
    c = Case(wl, prim=smooth_state(83), noise=1e-3, seed=7)
    c.alpha = seeded_alpha(c.mesh.K, 24, values=(0.0, 0.0, 0.4, 1.0))
    w = cot(c, 84)
    g_ref = oracle_vjp(c, w)
    assert rel_err(gpu_vjp(c, w), g_ref) <= vjp_tol(c, w, g_ref)


@FAULT_SKIP
def test_vjp_two_species_blended():
    announce("vjp two species blended")
    wl = curved_mixed(n=3, nmin=2, nmax=4, n_var=6, scramble=25, volume_flux=W.VOL_PIROZZOLI,
                      face_dg=W.RIEMANN_LLF, n_fv=6)
    c = Case(wl, prim=smooth_state(85, n_var=6), noise=1e-3, seed=8)
    c.alpha = seeded_alpha(c.mesh.K, 26, values=(0.0, 0.5, 1.0))
    w = cot(c, 86)
    g_ref = oracle_vjp(c, w)
    assert rel_err(gpu_vjp(c, w), g_ref) <= vjp_tol(c, w, g_ref)


def test_vjp_batch_equals_single_calls():
    announce("vjp batch")
    from paper_2502_19342_amd import dgfv
    wl = curved_mixed(n=2, nmin=3, nmax=3, scramble=27)
    c = Case(wl, prim=smooth_state(87), noise=1e-3, seed=9)
    ws = torch.stack([cot(c, 90 + b) for b in range(3)]).to("cuda")
    gb = dgfv.rhs_vjp(c.gmesh, c.params, c.gpu(c.u), None, ws)
    for b in range(3):
        g1 = dgfv.rhs_vjp(c.gmesh, c.params, c.gpu(c.u), None, ws[b].contiguous())
        assert torch.equal(gb[b], g1)
    out = torch.empty_like(ws[0])                     # a single cotangent into a given output
    assert dgfv.rhs_vjp(c.gmesh, c.params, c.gpu(c.u), None, ws[0].contiguous(), out=out) is out
    assert torch.equal(out, gb[0])


def test_vjp_against_central_differences_c4():
    # C4: 16^3, N = 4, isentropic vortex + N(0, 1e-3) on each value, 20 random directions, h = 1e-6
    announce("vjp FD C4")
    from paper_2502_19342_amd import dgfv
    wl = W.make_workload("C4")
    gm = dgfv.Mesh.from_workload(wl)
    prm = dgfv.params_of(wl)
    xyz = gm.node_coords()
    wp = torch.as_tensor(np.asarray(wl.prim(xyz.T))[:5]).to("cuda").contiguous()
    u = dgfv.prim_to_cons(gm, wp)
    u = (u + torch.as_tensor(W.noise(wl.seed, tuple(u.shape), wl.noise)).to("cuda")).contiguous()
    w = torch.as_tensor(W.cotangents(41, tuple(u.shape))).to("cuda").contiguous()
    g = dgfv.rhs_vjp(gm, prm, u, None, w)
    rng = np.random.default_rng(42)
    scale = u.abs().mean(dim=1, keepdim=True)
    worst = 0.0
    for _ in range(20):
        v = torch.as_tensor(rng.standard_normal(tuple(u.shape))).to("cuda") * scale
        h = 1e-6
        rp = dgfv.rhs(gm, prm, (u + h * v).contiguous())
        rm = dgfv.rhs(gm, prm, (u - h * v).contiguous())
        fd = float(((rp - rm) * w).sum()) / (2 * h)
        ad = float((g * v).sum())
        worst = max(worst, abs(fd - ad) / abs(ad))
    assert worst <= 1e-6, worst


def test_checkpointed_rollout_matches_oracle():
    announce("rollout adjoint")
    from paper_2502_19342_amd import dgfv
    wl = curved_mixed(n=2, nmin=3, nmax=3, scramble=29)
    c = Case(wl, prim=smooth_state(89), noise=1e-3, seed=10)
    dt = lsrk.timestep(c.mesh, c.gas, c.u, 0.5)
    nst = 5
    w = cot(c, 91)
    # oracle: autograd through the LSRK steps
    uu = c.u.clone().requires_grad_(True)
    x = uu
    for _ in range(nst):
        x = lsrk.step(lambda v: c.f(v, c.alpha), x, dt)
    (g_ref,) = torch.autograd.grad((x * w).sum(), uu)
    # GPU: checkpointed rollout through torch.autograd
    ug = c.gpu(c.u).requires_grad_(True)
    out = dgfv.checkpointed_rollout(ug, c.gmesh, c.params, nst, dt, None)
    (out * c.gpu(w)).sum().backward()
    assert rel_err(out.detach().cpu(), x.detach()) <= 1e-10
    assert rel_err(ug.grad.cpu(), g_ref) <= 1e-10


@pytest.mark.parametrize("stage", [1, 2, 3, 4, 5])
def test_rk_stage_vjp_matches_oracle(stage):
    # reverse of k_s = A_s k + dt R(u), u_s = u + B_s k_s: autograd through one oracle stage
    announce(f"rk stage vjp s={stage}")
    from paper_2502_19342_amd import dgfv
    wl = curved_mixed(n=2, nmin=3, nmax=3, scramble=35)
    c = Case(wl, prim=smooth_state(97), noise=1e-3, seed=12)
    dt = lsrk.timestep(c.mesh, c.gas, c.u, 0.5)
    k0 = 0.1 * cot(c, 98)
    ubar, kbar = cot(c, 99), cot(c, 100)
    uu = c.u.clone().requires_grad_(True)
    kk = k0.clone().requires_grad_(True)
    ks = lsrk.A_F64[stage - 1] * kk + dt * c.f(uu, c.alpha)
    us = uu + lsrk.B_F64[stage - 1] * ks
    gu, gk = torch.autograd.grad((us * ubar).sum() + (ks * kbar).sum(), (uu, kk))
    ub, kb = c.gpu(ubar), c.gpu(kbar)
    dgfv.rk_stage_vjp(c.gmesh, c.params, stage, dt, c.gpu(c.u), ub, kb, None)
    torch.cuda.synchronize()
    assert rel_err(ub.cpu(), gu) <= 1e-12
    if stage == 1:
        assert bool((kb == 0).all())
    else:
        assert rel_err(kb.cpu(), gk) <= 1e-14


@pytest.mark.parametrize("n_var", [5, 6])
def test_prim_to_cons_on_device(n_var):
    announce(f"prim_to_cons n_var={n_var}")
    from oracle.physics import prim_to_cons
    from paper_2502_19342_amd import dgfv
    wl = curved_mixed(n=2, nmin=2, nmax=3, n_var=n_var)
    c = Case(wl, prim=smooth_state(101, n_var))
    w = torch.as_tensor(np.asarray(smooth_state(102, n_var)(c.mesh.node_coords().numpy().T)), dtype=T)
    u = dgfv.prim_to_cons(c.gmesh, c.gpu(w)).cpu()
    assert rel_err(u, prim_to_cons(w, c.gas)) <= 1e-15


def test_rhs_function_autograd():
    announce("RHSFunction")
    from paper_2502_19342_amd import dgfv
    wl = curved_mixed(n=2, nmin=3, nmax=3, scramble=31)
    c = Case(wl, prim=smooth_state(93), noise=1e-3, seed=11)
    ug = c.gpu(c.u).requires_grad_(True)
    r = dgfv.RHSFunction.apply(ug, c.gmesh, c.params, None)
    w = cot(c, 94)
    (r * c.gpu(w)).sum().backward()
    assert rel_err(ug.grad.cpu(), oracle_vjp(c, w)) <= 1e-12


def test_disabled_adjoint_paths_raise():
    announce("vjp disabled paths")
    from paper_2502_19342_amd import dgfv
    wl = curved_mixed(n=2, nmin=2, nmax=3, scramble=33, n_fv=4)
    c = Case(wl, prim=smooth_state(95))
    w = cot(c, 96)
    with pytest.raises(dgfv.DgfvError) as e:
        dgfv.rhs_vjp(c.gmesh, c.params, c.gpu(c.u), None, c.gpu(w))
    assert e.value.status == dgfv.ERR_UNSUPPORTED
