"""Non-conforming (mortar) faces on the GPU against the oracle (Section 3.2.3).

Mortar meshes of types 1/2 (refinement in y) and 3 (in y and z), scrambled
element frames, degree jumps across the mortars, curved watertight elements,
one and two species, pure DG and blended (the FV variants), with and without
the viscous terms: the RHS, the lifted gradient, free-stream preservation,
RK steps under graph replay, FV-stored elements at the mortars, the adjoint
(pure DG, one degree), and the calls that reject mortar meshes.
"""
import dataclasses

import numpy as np
import pytest
import torch

from oracle import lsrk
from paper_2502_19342_amd import workloads as W

from gpu_common import Case, announce, rel_err, rhs_tol
from oracle_cases import seeded_alpha, smooth_state

pytestmark = pytest.mark.gpu
T = torch.float64


def _wl(refine, degree, scramble, amp, n_var=5, n=4):
    mesh = W.mortar_mesh(n, refine, degree, scramble_seed=scramble, amp=amp)
    kw = {} if n_var == 5 else dict(kappa=W.GAS_AIR_H2["kappa"], R=W.GAS_AIR_H2["R"])
    flux = (W.VOL_RANOCHA, W.RIEMANN_ROE_HH) if n_var == 5 else (W.VOL_PIROZZOLI, W.RIEMANN_LLF)
    return W.Workload("mortar", mesh, n_var, W.density_wave, flux[0], flux[1], W.RIEMANN_LLF, n_fv=8,
                      metric_degree=2 if amp else 1, **kw)


CASES = [("y", (4, 2), 7, 0.05, 5), ("y", 3, None, 0.0, 5), ("yz", (2, 4), 5, 0.0, 5), ("yz", (3, 3), 9, 0.05, 6),
         ("yz", (7, 6), 11, 0.05, 5)]


@pytest.mark.parametrize("refine,degree,scramble,amp,n_var", CASES)
def test_mortar_rhs_on_gpu(refine, degree, scramble, amp, n_var):
    announce(f"mortar rhs {refine} {degree} {scramble} {amp} {n_var}")
    c = Case(_wl(refine, degree, scramble, amp, n_var), prim=smooth_state(57, n_var), noise=1e-3, seed=9)
    err = rel_err(c.gpu_rhs(alpha=None), c.oracle_rhs())
    print(f"[mortar] rhs rel err {err:.3e}", flush=True)
    assert err <= 1e-12


@pytest.mark.parametrize("refine,amp", [("y", 0.05), ("yz", 0.05)])
def test_mortar_freestream_on_gpu(refine, amp):
    announce(f"mortar free-stream {refine}")
    c = Case(_wl(refine, (4, 3), 13, amp), prim=lambda x: W.freestream(x, 5))
    ref = Case(_wl(refine, (4, 3), 13, amp), prim=smooth_state(3))
    scale = float(ref.oracle_rhs().abs().max())
    # metric degree 2 (curved) carries rounding of about 5e-13 of the rate's scale
    assert float(c.gpu_rhs(alpha=None).abs().max()) <= 1e-11 * scale


def test_mortar_rk_steps_with_graphs():
    announce("mortar 10 RK steps, graph replays")
    from paper_2502_19342_amd import dgfv
    c = Case(_wl("yz", (3, 4), 15, 0.05), prim=smooth_state(59), noise=1e-3, seed=10)
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
    print(f"[mortar] 10 steps rel err {err:.3e}", flush=True)
    assert err <= 1e-10


def test_mortar_unsupported_calls():
    announce("mortar: unsupported calls")
    from paper_2502_19342_amd import dgfv
    c = Case(_wl("y", 3, None, 0.0), prim=smooth_state(61), noise=1e-3, seed=11)
    u = c.gpu(c.u)
    K = c.mesh.K
    with pytest.raises(dgfv.DgfvError):
        c.gmesh.face_fusion(True)
    with pytest.raises(dgfv.DgfvError):                 # the adjoint: pure DG only
        dgfv.rhs_vjp(c.gmesh, c.params, u, torch.zeros(K, dtype=T, device="cuda"), torch.ones_like(u))
    cj = Case(_wl("y", (3, 2), None, 0.0), prim=smooth_state(61), noise=1e-3, seed=11)
    with pytest.raises(dgfv.DgfvError):                 # ... and no degree jump across a mortar
        dgfv.rhs_vjp(cj.gmesh, cj.params, cj.gpu(cj.u), None, torch.ones_like(cj.gpu(cj.u)))
    r = dgfv.rhs(c.gmesh, c.params, u)                # the mesh still works
    torch.cuda.synchronize()
    assert rel_err(r.cpu(), c.oracle_rhs()) <= 1e-12


@pytest.mark.parametrize("refine,degree,scramble,amp,n_fv,n_var", [("y", (4, 3), 7, 0.05, 8, 5),
                                                                   ("yz", (3, 2), 5, 0.0, 5, 5),
                                                                   ("yz", (7, 6), 11, 0.05, 8, 6)])
def test_mortar_blended_rhs_on_gpu(refine, degree, scramble, amp, n_fv, n_var):
    # the FV variants: blending factors 0, 0.4 and 1 on both sides of the mortars
    announce(f"mortar blended rhs {refine} {degree} {scramble} {amp} {n_fv} {n_var}")
    wl = dataclasses.replace(_wl(refine, degree, scramble, amp, n_var), n_fv=n_fv)
    c = Case(wl, prim=smooth_state(73, n_var), noise=1e-3, seed=12)
    c.alpha = seeded_alpha(c.mesh.K, scramble, values=(0.0, 0.4, 1.0))
    err = rel_err(c.gpu_rhs(), c.oracle_rhs())
    print(f"[mortar] blended rhs rel err {err:.3e}", flush=True)
    assert err <= rhs_tol(c)


def test_mortar_blended_rk_steps_with_graphs():
    announce("mortar blended 10 RK steps, graph replays")
    from paper_2502_19342_amd import dgfv
    c = Case(_wl("yz", (3, 4), 15, 0.05), prim=smooth_state(75), noise=1e-3, seed=13)
    c.alpha = seeded_alpha(c.mesh.K, 76, values=(0.0, 0.0, 0.4, 1.0))
    dt = 0.3 * lsrk.timestep(c.mesh, c.gas, c.u, 0.5, c.alpha)
    c.gmesh.graphs(True)
    ug = c.gpu(c.u)
    k = torch.zeros_like(ug)
    a = c.gpu(c.alpha)
    uo = c.u.clone()
    for _ in range(10):
        dgfv.rk_step(c.gmesh, c.params, dt, ug, k, a)
        uo = lsrk.step(lambda v: c.f(v, c.alpha), uo, dt)
    torch.cuda.synchronize()
    err = rel_err(ug.cpu(), uo)
    print(f"[mortar] blended 10 steps rel err {err:.3e}", flush=True)
    assert err <= 1e-10


def _vwl(refine, degree, scramble, amp, n_var=5):
    return dataclasses.replace(_wl(refine, degree, scramble, amp, n_var), mu=(0.02, 0.03), Pr=(0.7, 0.9),
                               D=(0.01, 0.04))


@pytest.mark.parametrize("refine,degree,scramble,amp,n_var", [("y", (4, 2), 7, 0.05, 5), ("yz", (2, 4), 5, 0.0, 6),
                                                              ("yz", (7, 6), 11, 0.05, 5)])
def test_mortar_viscous_on_gpu(refine, degree, scramble, amp, n_var):
    announce(f"mortar viscous {refine} {degree} {scramble} {amp} {n_var}")
    from oracle import viscous
    from paper_2502_19342_amd import dgfv
    c = Case(_vwl(refine, degree, scramble, amp, n_var), prim=smooth_state(79, n_var), noise=1e-3, seed=15)
    g = dgfv.lift(c.gmesh, c.gpu(c.u))
    torch.cuda.synchronize()
    want = viscous.lift(c.mesh, c.u)
    eg = rel_err(g.cpu().reshape(3 * n_var, -1), want.reshape(3 * n_var, -1))
    er = rel_err(c.gpu_rhs(alpha=None), c.oracle_rhs())
    print(f"[mortar] viscous lift rel err {eg:.3e}, rhs rel err {er:.3e}", flush=True)
    assert eg <= 1e-12 and er <= 1e-12


def test_mortar_viscous_blended_rk_steps_with_graphs():
    announce("mortar viscous blended 10 RK steps, graph replays")
    from paper_2502_19342_amd import dgfv
    c = Case(_vwl("yz", (3, 4), 15, 0.05), prim=smooth_state(81), noise=1e-3, seed=16)
    c.alpha = seeded_alpha(c.mesh.K, 82, values=(0.0, 0.0, 0.4, 1.0))
    dt = 0.3 * lsrk.timestep(c.mesh, c.gas, c.u, 0.5, c.alpha)
    c.gmesh.graphs(True)
    ug = c.gpu(c.u)
    k = torch.zeros_like(ug)
    a = c.gpu(c.alpha)
    uo = c.u.clone()
    for _ in range(10):
        dgfv.rk_step(c.gmesh, c.params, dt, ug, k, a)
        uo = lsrk.step(lambda v: c.f(v, c.alpha), uo, dt)
    torch.cuda.synchronize()
    err = rel_err(ug.cpu(), uo)
    print(f"[mortar] viscous blended 10 steps rel err {err:.3e}", flush=True)
    assert err <= 1e-10


@pytest.mark.parametrize("refine,degree,scramble,amp,n_var", [("y", 3, 7, 0.05, 5), ("yz", 4, 5, 0.0, 6),
                                                              ("yz", 7, 11, 0.05, 5)])
def test_mortar_vjp_on_gpu(refine, degree, scramble, amp, n_var):
    announce(f"mortar vjp {refine} {degree} {scramble} {amp} {n_var}")
    from paper_2502_19342_amd import dgfv
    c = Case(_wl(refine, degree, scramble, amp, n_var), prim=smooth_state(87, n_var), noise=1e-3, seed=17)
    w = torch.as_tensor(W.cotangents(88, tuple(c.u.shape)), dtype=T)
    uu = c.u.clone().requires_grad_(True)
    (g_ref,) = torch.autograd.grad((c.f(uu, c.alpha) * w).sum(), uu)
    g = dgfv.rhs_vjp(c.gmesh, c.params, c.gpu(c.u), None, c.gpu(w))
    torch.cuda.synchronize()
    err = rel_err(g.cpu(), g_ref)
    print(f"[mortar] vjp rel err {err:.3e}", flush=True)
    assert err <= 1e-12


def _fvs_case(refine, degree, scramble, amp, n_fv, seed, n_var=5):
    from oracle import native_fv
    wl = dataclasses.replace(_wl(refine, degree, scramble, amp, n_var), n_fv=n_fv)
    c = Case(wl, prim=smooth_state(91, n_var), noise=1e-3, seed=seed)
    K = c.mesh.K
    rng = np.random.default_rng(seed)
    flag = rng.random(K) < 0.4
    ufv = torch.zeros(K, n_var, n_fv, n_fv, n_fv, dtype=T)
    fvel = np.nonzero(flag)[0]
    ufv[torch.as_tensor(fvel)] = native_fv.dg_to_fv(c.mesh, c.u, fvel)
    ufv = ufv * (1.0 + 2e-2 * torch.as_tensor(rng.standard_normal(tuple(ufv.shape))))
    dg = torch.as_tensor(np.repeat(~flag, [int(c.mesh.offset[e + 1] - c.mesh.offset[e]) for e in range(K)]))
    return c, flag, ufv, dg


@pytest.mark.parametrize("refine,degree,scramble,amp,n_fv,n_var", [("y", (4, 3), 7, 0.05, 8, 5),
                                                                   ("yz", (3, 2), 5, 0.0, 5, 5),
                                                                   ("yz", (7, 6), 11, 0.05, 8, 5),
                                                                   ("yz", (3, 4), 17, 0.05, 6, 6)])
def test_mortar_fv_stored_rhs_on_gpu(refine, degree, scramble, amp, n_fv, n_var):
    announce(f"mortar FV-stored rhs {refine} {degree} {scramble} {amp} {n_fv} {n_var}")
    from oracle import native_fv, problem
    from paper_2502_19342_amd import dgfv
    c, flag, ufv, dg = _fvs_case(refine, degree, scramble, amp, n_fv, 19, n_var)
    K = c.mesh.K
    R, Rfv = native_fv.NativeRhs(c.mesh, c.gas, problem.params_of(c.wl))(c.u, ufv, flag)
    r, rf = dgfv.rhs_fv(c.gmesh, c.params, c.gpu(c.u), c.gpu(ufv.reshape(K, n_var, -1)),
                        c.gpu(torch.as_tensor(flag, dtype=T)))
    torch.cuda.synchronize()
    sel = torch.as_tensor(flag)
    e1 = rel_err(r.cpu()[:, dg], R[:, dg])
    e2 = rel_err(rf.cpu().reshape(K, n_var, -1)[sel].transpose(0, 1).reshape(n_var, -1),
                 Rfv[sel].transpose(0, 1).reshape(n_var, -1))
    print(f"[mortar] FV-stored rhs rel err DG {e1:.3e}, FV {e2:.3e}", flush=True)
    assert e1 <= 1e-12 and e2 <= 1e-12                # measured up to 6e-14


@pytest.mark.parametrize("graphs", [False, True])
def test_mortar_fv_stored_rk_steps(graphs):
    announce(f"mortar FV-stored 10 RK steps, graphs={graphs}")
    from oracle import native_fv, problem
    from paper_2502_19342_amd import dgfv
    c, flag, ufv, dg = _fvs_case("yz", (3, 4), 15, 0.05, 8, 20)
    c.gmesh.graphs(graphs)
    K = c.mesh.K
    native = native_fv.NativeRhs(c.mesh, c.gas, problem.params_of(c.wl))
    dt = 0.2 * lsrk.timestep(c.mesh, c.gas, c.u, 0.5, torch.as_tensor(flag, dtype=T))
    fv = c.gpu(torch.as_tensor(flag, dtype=T))
    ug, ufg = c.gpu(c.u), c.gpu(ufv.reshape(K, 5, -1))
    k, kf = torch.zeros_like(ug), torch.zeros_like(ufg)
    uo, ufo = c.u.clone(), ufv.clone()
    for _ in range(10):
        dgfv.rk_step_fv(c.gmesh, c.params, dt, ug, k, ufg, kf, fv)
        ko, kfo = torch.zeros_like(uo), torch.zeros_like(ufo)
        for s in range(5):
            uo, ufo, ko, kfo = native_fv.stage(lambda a, b: native(a, b, flag), uo, ufo, ko, kfo, s, dt,
                                               lsrk.A_F64, lsrk.B_F64)
    torch.cuda.synchronize()
    sel = torch.as_tensor(flag)
    e1 = rel_err(ug.cpu()[:, dg], uo[:, dg])
    e2 = rel_err(ufg.cpu().reshape(K, 5, -1)[sel].transpose(0, 1).reshape(5, -1),
                 ufo[sel].transpose(0, 1).reshape(5, -1))
    print(f"[mortar] FV-stored 10 steps: DG {e1:.3e}, FV {e2:.3e}", flush=True)
    assert e1 <= 1e-10 and e2 <= 1e-10


@pytest.mark.parametrize("stage", [1, 3, 5])
def test_mortar_rk_stage_vjp_on_gpu(stage):
    # the reverse of one RK stage through the mortars: autograd through the oracle's stage
    announce(f"mortar rk stage vjp s={stage}")
    from paper_2502_19342_amd import dgfv
    c = Case(_wl("yz", 3, 13, 0.05), prim=smooth_state(93), noise=1e-3, seed=21)
    dt = lsrk.timestep(c.mesh, c.gas, c.u, 0.5)
    cot = lambda s: torch.as_tensor(W.cotangents(s, tuple(c.u.shape)), dtype=T)
    k0, ubar, kbar = 0.1 * cot(94), cot(95), cot(96)
    uu = c.u.clone().requires_grad_(True)
    kk = k0.clone().requires_grad_(True)
    ks = lsrk.A_F64[stage - 1] * kk + dt * c.f(uu, c.alpha)
    us = uu + lsrk.B_F64[stage - 1] * ks
    gu, gk = torch.autograd.grad((us * ubar).sum() + (ks * kbar).sum(), (uu, kk))
    ub, kb = c.gpu(ubar), c.gpu(kbar)
    dgfv.rk_stage_vjp(c.gmesh, c.params, stage, dt, c.gpu(c.u), ub, kb, None)
    torch.cuda.synchronize()
    assert rel_err(ub.cpu(), gu) <= 1e-12
    if stage > 1:
        assert rel_err(kb.cpu(), gk) <= 1e-14


def test_m3_full_size_rate_is_the_exact_divergence():
    # the M3 workload at full size (34,560 elements at N = 7, 1,152 type-3 mortars), pure DG:
    # the density wave is an exact solution, so the rate at every node is the exact
    # -div F = rho_t (1, 1, 1, 1, 3/2) with rho_t = -3 (0.2 pi) cos 2 pi (x + y + z);
    # spectral accuracy leaves ~4e-11 of its scale, at the nodes next to the mortars too
    announce("M3 full size, exact rate")
    from paper_2502_19342_amd import dgfv
    wl = W.make_workload("M3")
    gm = dgfv.Mesh.from_workload(wl)
    prm = dgfv.params_of(wl)
    xyz = torch.as_tensor(gm.node_coords(), device="cuda")
    w = torch.as_tensor(np.asarray(wl.prim(gm.node_coords().T)), device="cuda").contiguous()
    u = dgfv.prim_to_cons(gm, w)
    r = dgfv.rhs(gm, prm, u)
    rho_t = -3.0 * 0.2 * np.pi * torch.cos(2 * np.pi * xyz.sum(0))
    want = torch.stack([rho_t, rho_t, rho_t, rho_t, 1.5 * rho_t])
    err = float((r - want).abs().max() / want.abs().max())
    big = torch.as_tensor(np.unique(np.concatenate([np.arange(gm.elem_offset[e], gm.elem_offset[e + 1])
                                                    for e in wl.mesh.mortars[:, 0]])), device="cuda")
    err_m = float((r[:, big] - want[:, big]).abs().max() / want.abs().max())
    print(f"[mortar] M3 full size: rate rel err {err:.3e} (big sides of mortars {err_m:.3e})", flush=True)
    assert err <= 1e-9 and err_m <= 1e-9


def test_m3v_full_size_viscous_rate():
    # M3 with the viscous terms at full size: the viscous rate (with minus without
    # the transport coefficients) at 4096 sampled nodes and at every node of the
    # mortars' big sides against the exact viscous rate of the density wave (the
    # heat flux of its temperature field; autograd through the oracle's flux on the
    # analytic fields)
    announce("M3V full size, exact viscous rate")
    from oracle import problem, viscous
    from paper_2502_19342_amd import dgfv
    wl = W.make_workload("M3V")
    gm = dgfv.Mesh.from_workload(wl)
    prm = dgfv.params_of(wl)
    xyz = gm.node_coords()
    w = torch.as_tensor(np.asarray(wl.prim(xyz.T)), device="cuda").contiguous()
    u = dgfv.prim_to_cons(gm, w)
    r_v = dgfv.rhs(gm, prm, u)
    gm.transport(None)
    r_c = dgfv.rhs(gm, prm, u)
    torch.cuda.synchronize()
    big = np.unique(np.concatenate([np.arange(gm.elem_offset[e], gm.elem_offset[e + 1])
                                    for e in wl.mesh.mortars[:, 0]]))
    idx = np.unique(np.concatenate([np.random.default_rng(8).choice(gm.n_node, 4096, replace=False),
                                    big[np.random.default_rng(9).choice(len(big), 4096, replace=False)]]))
    got = (r_v - r_c)[:, torch.as_tensor(idx, device="cuda")].cpu()
    gas = problem.gas_of(wl)
    xt = torch.as_tensor(xyz[:, idx].T, dtype=T).requires_grad_(True)
    rho = 1.0 + 0.1 * torch.sin(2 * np.pi * xt.sum(1))
    one = torch.ones_like(rho)
    from oracle.physics import prim_to_cons
    uu = prim_to_cons(torch.stack([rho, one, one, one, one]), gas)
    g = torch.stack([torch.stack([torch.autograd.grad(uu[c].sum(), xt, create_graph=True)[0][:, d]
                                  for c in range(5)]) for d in range(3)])
    F = viscous.viscous_flux(uu, g, gas, problem.transport_of(wl))
    want = torch.zeros(5, len(idx), dtype=T)
    for c in range(1, 5):
        for d in range(3):
            want[c] -= torch.autograd.grad(F[d, c].sum(), xt, retain_graph=True)[0][:, d].detach()
    err = float((got - want).abs().max() / want.abs().max())
    print(f"[mortar] M3V full size: viscous rate rel err {err:.3e}", flush=True)
    assert err <= 1e-8                      # measured 8.7e-10


def test_mortar_p_adaptation():
    # p-adaptation on a curved mortar mesh: the degree decision from I(rho), the mesh of
    # the new degrees (degree jumps across the mortars), the state transfer and the rate
    # on the new mesh, each against the oracle doing the same
    announce("mortar p-adaptation")
    from oracle import p_adapt, problem
    from paper_2502_19342_amd import dgfv
    c = Case(_wl("yz", 4, 23, 0.05), prim=smooth_state(97), noise=1e-3, seed=22)
    from oracle.indicator import indicator
    I, _ = indicator(c.mesh, c.gas, c.u, 0.0, 1.0, ind_vars=2)               # I(rho), the p-adaptation indicator
    t_ref, t_coa = float(np.quantile(I.numpy(), 0.3)), float(np.quantile(I.numpy(), 0.7))
    want_deg = p_adapt.degrees(c.mesh, c.gas, c.u, t_ref, t_coa, 2, 5)
    ug = c.gpu(c.u)
    got_deg = dgfv.p_degrees(c.gmesh, c.params, ug, t_ref, t_coa, 2, 5)
    assert np.array_equal(np.asarray(got_deg), np.asarray(want_deg))
    assert len(set(np.asarray(got_deg).tolist())) > 1
    new = c.gmesh.redegree(np.asarray(got_deg))
    u2 = dgfv.transfer_degree(c.gmesh, new, ug)
    wl2 = dataclasses.replace(c.wl, mesh=dataclasses.replace(c.wl.mesh, degree=np.asarray(got_deg)))
    om2, gas2, f2 = problem.build(wl2)
    uo2 = p_adapt.transfer(c.mesh, om2, c.u)
    assert rel_err(u2.cpu(), uo2) <= 1e-13
    r2 = dgfv.rhs(new, c.params, u2)
    torch.cuda.synchronize()
    assert rel_err(r2.cpu(), f2(uo2, torch.zeros(om2.K, dtype=T))) <= 1e-12
