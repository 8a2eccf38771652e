"""The library's kernels and host code run on the CPU, against the oracle.

The HIP sources are built with g++ against a CPU stand-in of the HIP runtime
(``tests/cpu_hip``): every GPU thread is a fiber, wavefront operations act on
64-lane wavefronts and stop the run when a shuffle reads a thread that has
returned or the lanes of one wavefront split between a wavefront operation and
a workgroup barrier; device allocations sit flush against inaccessible guard
regions (after the end, then before the start) and start as NaN; everything
runs under AddressSanitizer and UndefinedBehaviorSanitizer.  This is where new
kernels and host code are checked before a GPU run, and where the adjoint of
FV-blended elements and degree jumps, which stays off on the GPU (it faulted
the GPU once, with no cause shown), is exercised.
"""
import types

import numpy as np
import pytest
import torch

import cpu_emu
from gpu_common import oracle_spread, rel_err
from oracle import lsrk, problem
from paper_2502_19342_amd import workloads as W

from oracle_cases import curved_mixed, seeded_alpha, smooth_state

T = torch.float64


def _case(wl, prim, noise=0.0, seed=0):
    mesh, gas, f = problem.build(wl)
    u = problem.initial_state(mesh, gas, prim)
    if noise:
        rng = np.random.default_rng(seed)
        u = u * (1.0 + noise * torch.as_tensor(rng.standard_normal(tuple(u.shape))))
    c = types.SimpleNamespace(wl=wl, mesh=mesh, gas=gas, f=f, u=u, alpha=torch.zeros(mesh.K, dtype=T))
    c.oracle_rhs = lambda: c.f(c.u, c.alpha)
    return c


def _tol(c, base=1e-12):
    return base if not bool((c.alpha > 0).any()) else max(base, 4.0 * oracle_spread(c))


def test_cpu_build_c1_rhs_and_rk_step():
    wl = W.make_workload("C1")
    c = _case(wl, wl.prim)
    dt = lsrk.timestep(c.mesh, c.gas, c.u, 0.5)
    out = cpu_emu.run(wl, c.u.numpy(), ["rhs", "rk_step", "coords"], alpha=c.alpha.numpy(), dt=dt)
    assert rel_err(torch.as_tensor(out["rhs"]), c.f(c.u, c.alpha)) <= 1e-12
    ref = lsrk.step(lambda v: c.f(v, c.alpha), c.u, dt)
    assert rel_err(torch.as_tensor(out["rk_step"]), ref) <= 1e-12
    assert np.abs(out["coords"] - c.mesh.node_coords().numpy()).max() <= 1e-14


@pytest.mark.parametrize("n_var", [5, 6])
def test_cpu_build_per_element_metrics(n_var):
    # metric_degree 0 on a curved, scrambled mesh with degrees 1..7 side by side
    flux = {} if n_var == 5 else dict(volume_flux=W.VOL_PIROZZOLI, face_dg=W.RIEMANN_LLF)
    wl = curved_mixed(n=3, nmin=1, nmax=7, n_var=n_var, scramble=5, metric_degree=0, n_fv=8, **flux)
    c = _case(wl, smooth_state(73, n_var), noise=1e-3, seed=2)
    c.alpha = seeded_alpha(c.mesh.K, 11, values=(0.0, 0.0, 0.35, 1.0))
    fs = _case(wl, lambda x: W.freestream(x, n_var))
    out = cpu_emu.run(wl, c.u.numpy(), ["rhs"], alpha=c.alpha.numpy())
    assert rel_err(torch.as_tensor(out["rhs"]), c.f(c.u, c.alpha)) <= _tol(c)
    out = cpu_emu.run(wl, fs.u.numpy(), ["rhs"], alpha=np.zeros(c.mesh.K))
    from test_oracle_rhs import term_scale
    assert np.abs(out["rhs"]).max() <= 1e-13 * term_scale(fs.mesh, fs.gas, fs.f.params, fs.u)


@pytest.mark.parametrize("n_var", [5, 6])
def test_cpu_build_fused_faces(n_var):
    # degrees 5..7 side by side, curved and scrambled, blended elements: the
    # element kernels of degree 6 and 7 evaluate their conforming DG faces
    # themselves (dg_rhs; dg_rk_step over two state buffers), with results
    # equal bit for bit to the separate face kernels' and close to the oracle's
    flux = {} if n_var == 5 else dict(volume_flux=W.VOL_PIROZZOLI, face_dg=W.RIEMANN_LLF)
    wl = curved_mixed(n=3, nmin=5, nmax=7, n_var=n_var, scramble=7, metric_degree=0, n_fv=8, **flux)
    c = _case(wl, smooth_state(41, n_var), noise=1e-3, seed=5)
    c.alpha = seeded_alpha(c.mesh.K, 13, values=(0.0, 0.0, 0.0, 0.4, 1.0))
    dt = lsrk.timestep(c.mesh, c.gas, c.u, 0.3)
    out = cpu_emu.run(wl, c.u.numpy(), ["fusion_on", "rhs", "rk_step", "rhs_unfused", "rk_step_unfused"],
                      alpha=c.alpha.numpy(), dt=dt)
    assert np.array_equal(out["rhs"], out["rhs_unfused"])
    assert np.array_equal(out["rk_step"], out["rk_step_unfused"])
    assert rel_err(torch.as_tensor(out["rhs"]), c.f(c.u, c.alpha)) <= _tol(c)
    ref = lsrk.step(lambda v: c.f(v, c.alpha), c.u, dt)
    assert rel_err(torch.as_tensor(out["rk_step"]), ref) <= _tol(c)


def _oracle_vjp(c, w):
    uu = c.u.clone().requires_grad_(True)
    (g,) = torch.autograd.grad((c.f(uu, c.alpha) * w).sum(), uu)
    return g


def _vjp_tol(c, w, g_ref):
    gen = torch.Generator().manual_seed(1)
    worst = 0.0
    for _ in range(2):
        up = c.u * (1.0 + 2.0 ** -52 * torch.randn(tuple(c.u.shape), generator=gen, dtype=T))
        worst = max(worst, rel_err(_oracle_vjp(types.SimpleNamespace(u=up, f=c.f, alpha=c.alpha), w), g_ref))
    return max(1e-12, 4.0 * worst)


@pytest.mark.parametrize("guard", ["end", "start"])
def test_cpu_build_adjoint_blended_mixed_degree(guard):
    # the case that faulted the GPU: 3^3, degrees 1..4, N_FV = 5, scrambled frames,
    # alpha in {0, 0.4, 1}
    wl = curved_mixed(n=3, nmin=1, nmax=4, scramble=23, metric_degree=1, n_fv=5)
    c = _case(wl, smooth_state(83), noise=1e-3, seed=7)
    c.alpha = seeded_alpha(c.mesh.K, 24, values=(0.0, 0.0, 0.4, 1.0))
    w = torch.as_tensor(W.cotangents(84, tuple(c.u.shape)), dtype=T)
    ws = torch.stack([w, torch.as_tensor(W.cotangents(85, tuple(c.u.shape)), dtype=T)])
    out = cpu_emu.run(wl, c.u.numpy(), ["vjp"], alpha=c.alpha.numpy(), w=ws.numpy(), guard=guard)
    for b in range(2):
        g_ref = _oracle_vjp(c, ws[b])
        assert rel_err(torch.as_tensor(out["vjp"][b]), g_ref) <= _vjp_tol(c, ws[b], g_ref)


def test_cpu_build_adjoint_two_species_blended():
    wl = curved_mixed(n=3, nmin=2, nmax=4, n_var=6, scramble=25, volume_flux=W.VOL_PIROZZOLI,
                      face_dg=W.RIEMANN_LLF, n_fv=6)
    c = _case(wl, smooth_state(85, n_var=6), noise=1e-3, seed=8)
    c.alpha = seeded_alpha(c.mesh.K, 26, values=(0.0, 0.5, 1.0))
    w = torch.as_tensor(W.cotangents(86, tuple(c.u.shape)), dtype=T)
    out = cpu_emu.run(wl, c.u.numpy(), ["vjp"], alpha=c.alpha.numpy(), w=w.numpy()[None])
    g_ref = _oracle_vjp(c, w)
    assert rel_err(torch.as_tensor(out["vjp"][0]), g_ref) <= _vjp_tol(c, w, g_ref)


def test_cpu_build_rk_stage_vjp_and_prim_to_cons():
    # reverse of one RK stage on a blended mixed-degree mesh, against autograd
    # through the oracle's stage; and the device primitive -> conservative map
    wl = curved_mixed(n=3, nmin=2, nmax=4, scramble=37, n_fv=5)
    c = _case(wl, smooth_state(103), noise=1e-3, seed=13)
    c.alpha = seeded_alpha(c.mesh.K, 27, values=(0.0, 0.0, 0.5, 1.0))
    dt = lsrk.timestep(c.mesh, c.gas, c.u, 0.5, c.alpha)
    stage = 3
    k0 = 0.1 * torch.as_tensor(W.cotangents(104, tuple(c.u.shape)), dtype=T)
    ubar = torch.as_tensor(W.cotangents(105, tuple(c.u.shape)), dtype=T)
    kbar = torch.as_tensor(W.cotangents(106, tuple(c.u.shape)), dtype=T)
    uu = c.u.clone().requires_grad_(True)
    kk = k0.clone().requires_grad_(True)
    ks = lsrk.A_F64[stage - 1] * kk + dt * c.f(uu, c.alpha)
    us = uu + lsrk.B_F64[stage - 1] * ks
    gu, gk = torch.autograd.grad((us * ubar).sum() + (ks * kbar).sum(), (uu, kk))
    out = cpu_emu.run(wl, c.u.numpy(), ["stage_vjp"], alpha=c.alpha.numpy(), dt=dt, stage=stage,
                      ubar=ubar.numpy(), kbar=kbar.numpy())
    tol = _vjp_tol(c, kbar + lsrk.B_F64[stage - 1] * ubar, gu)
    assert rel_err(torch.as_tensor(out["ubar"]), gu) <= tol
    assert rel_err(torch.as_tensor(out["kbar"]), gk) <= 1e-14
    from oracle.physics import prim_to_cons
    w = torch.as_tensor(np.asarray(smooth_state(107)(c.mesh.node_coords().numpy().T)), dtype=T)
    out = cpu_emu.run(wl, w.numpy(), ["prim_to_cons"])
    assert rel_err(torch.as_tensor(out["cons"]), prim_to_cons(w, c.gas)) <= 1e-15


def test_cpu_build_positivity_limiter():
    # the HIP limiter kernel (wave-shuffle reductions) against the oracle's limiter
    from oracle import limiter
    from test_oracle_limiter import _spoil
    wl = curved_mixed(n=3, nmin=2, nmax=5, scramble=9, metric_degree=0, n_fv=6)
    c = _case(wl, smooth_state(3))
    u = _spoil(c.mesh, c.u, 11)
    alpha = seeded_alpha(c.mesh.K, 5, values=(0.0, 1.0))
    ref, n_lim, _ = limiter.limit(c.mesh, c.gas, u, alpha)
    out = cpu_emu.run(wl, u.numpy(), ["limiter"], alpha=alpha.numpy())
    assert rel_err(torch.as_tensor(out["limited"]), ref) <= 1e-12
    changed = [e for e in range(c.mesh.K) if not torch.equal(u[:, c.mesh.offset[e]:c.mesh.offset[e + 1]],
                                                             ref[:, c.mesh.offset[e]:c.mesh.offset[e + 1]])]
    assert sorted(np.nonzero(out["theta"] < 1.0)[0].tolist()) == changed and len(changed) == n_lim


def _fv_stored_case(n_var, seed=7):
    from oracle import native_fv
    flux = {} if n_var == 5 else dict(volume_flux=W.VOL_PIROZZOLI, face_dg=W.RIEMANN_LLF)
    wl = curved_mixed(n=3, nmin=2, nmax=4, n_var=n_var, scramble=19, metric_degree=0, n_fv=5, **flux)
    c = _case(wl, smooth_state(83, n_var), noise=1e-3, seed=seed)
    rng = np.random.default_rng(seed)
    flag = rng.random(c.mesh.K) < 0.4
    nf = wl.n_fv
    ufv = torch.zeros(c.mesh.K, n_var, nf, nf, nf, dtype=T)
    fvel = np.nonzero(flag)[0]
    ufv[torch.as_tensor(fvel)] = native_fv.dg_to_fv(c.mesh, c.u, fvel)
    ufv = ufv * (1.0 + 2e-2 * torch.as_tensor(rng.standard_normal(tuple(ufv.shape))))
    return wl, c, flag, ufv


@pytest.mark.parametrize("n_var", [5, 6])
def test_cpu_build_fv_stored_elements(n_var):
    # FV-stored elements (N_FV = 5 = 2N + 1 at N = 2) beside DG elements of degrees 2..4:
    # rates, five RK stages and the switch against the oracle
    from oracle import lsrk, native_fv, problem
    wl, c, flag, ufv = _fv_stored_case(n_var)
    K, nf = c.mesh.K, wl.n_fv
    native = native_fv.NativeRhs(c.mesh, c.gas, problem.params_of(wl))
    R, Rfv = native(c.u, ufv, flag)
    fv = flag.astype(np.float64)
    fv_new = (np.random.default_rng(5).random(K) < 0.5).astype(np.float64)
    dt = 0.2 * lsrk.timestep(c.mesh, c.gas, c.u, 0.5, torch.as_tensor(fv))
    out = cpu_emu.run(wl, c.u.numpy(), ["rhs_fv", "rk_step_fv", "switch_fv"], dt=dt,
                      ufv=ufv.reshape(K, n_var, -1).numpy(), fv=fv, fv_new=fv_new)
    dg = np.repeat(~flag, [int(c.mesh.offset[e + 1] - c.mesh.offset[e]) for e in range(K)])
    got_dg = torch.as_tensor(out["rhs_fv_dg"])[:, torch.as_tensor(dg)]
    assert rel_err(got_dg, R[:, torch.as_tensor(dg)]) <= 1e-11
    sel = torch.as_tensor(flag)
    got_fv = torch.as_tensor(out["rhs_fv_fv"]).reshape(K, n_var, -1)[sel].transpose(0, 1).reshape(n_var, -1)
    assert rel_err(got_fv, Rfv[sel].transpose(0, 1).reshape(n_var, -1)) <= 1e-11
    # five stages
    u, uf = c.u.clone(), ufv.clone()
    k, kf = torch.zeros_like(u), torch.zeros_like(uf)
    for s in range(5):
        u, uf, k, kf = native_fv.stage(lambda a, b: native(a, b, flag), u, uf, k, kf, s, dt,
                                       lsrk.A_F64, lsrk.B_F64)
    got = torch.as_tensor(out["step_fv_dg"])[:, torch.as_tensor(dg)]
    assert rel_err(got, u[:, torch.as_tensor(dg)]) <= 1e-11
    got = torch.as_tensor(out["step_fv_fv"]).reshape(K, n_var, -1)[sel].transpose(0, 1).reshape(n_var, -1)
    assert rel_err(got, uf[sel].transpose(0, 1).reshape(n_var, -1)) <= 1e-11
    # switch
    su, sf = native_fv.switch(c.mesh, c.u, ufv, flag, fv_new > 0)
    new = fv_new > 0
    dgn = np.repeat(~new, [int(c.mesh.offset[e + 1] - c.mesh.offset[e]) for e in range(K)])
    assert rel_err(torch.as_tensor(out["switch_dg"])[:, torch.as_tensor(dgn)], su[:, torch.as_tensor(dgn)]) <= 1e-12
    seln = torch.as_tensor(new)
    got = torch.as_tensor(out["switch_fv"]).reshape(K, n_var, -1)[seln].transpose(0, 1).reshape(n_var, -1)
    assert rel_err(got, sf[seln].transpose(0, 1).reshape(n_var, -1)) <= 1e-12


def test_cpu_build_fv_stored_step_with_traces():
    # degrees 6 and 7 (their DG faces read the xi_1 sides from traces between the
    # stages of dg_rk_step_fv): the one-call step equals five stage calls bit for bit
    from oracle import lsrk
    wl = curved_mixed(n=2, nmin=6, nmax=7, n_var=5, scramble=3, metric_degree=0, n_fv=8)
    c = _case(wl, smooth_state(29, 5), noise=1e-3, seed=4)
    rng = np.random.default_rng(4)
    flag = rng.random(c.mesh.K) < 0.3
    flag[0] = True
    from oracle import native_fv
    nf = wl.n_fv
    ufv = torch.zeros(c.mesh.K, 5, nf, nf, nf, dtype=T)
    fvel = np.nonzero(flag)[0]
    ufv[torch.as_tensor(fvel)] = native_fv.dg_to_fv(c.mesh, c.u, fvel)
    dt = 0.2 * lsrk.timestep(c.mesh, c.gas, c.u, 0.5, torch.as_tensor(flag, dtype=T))
    out = cpu_emu.run(wl, c.u.numpy(), ["rk_step_fv", "rk_step_fv_one_call"], dt=dt,
                      ufv=ufv.reshape(c.mesh.K, 5, -1).numpy(), fv=flag.astype(np.float64))
    dg = np.repeat(~flag, np.diff(c.mesh.offset))
    assert np.array_equal(out["step1_fv_dg"][:, dg], out["step_fv_dg"][:, dg])
    assert np.array_equal(out["step1_fv_fv"][flag], out["step_fv_fv"][flag])


def test_cpu_build_p_adaptation():
    # the degree decision from I(rho) and the transfer to the new degrees, against the oracle
    import dataclasses
    from oracle import p_adapt
    from oracle.geometry import OracleMesh
    wl = curved_mixed(n=3, nmin=2, nmax=5, scramble=7, metric_degree=0, n_fv=8)
    c = _case(wl, smooth_state(31, 5), noise=1e-2, seed=6)
    from oracle.indicator import indicator
    I, _ = indicator(c.mesh, c.gas, c.u, 0.0, 1.0, ind_vars=2)
    t_ref, t_coarse = float(np.quantile(I.numpy(), 0.3)), float(np.quantile(I.numpy(), 0.7))
    want = p_adapt.degrees(c.mesh, c.gas, c.u, t_ref, t_coarse, 1, 7)
    assert (want > c.mesh.degree).any() and (want < c.mesh.degree).any()
    m2 = OracleMesh(dataclasses.replace(c.mesh.spec, degree=want.astype(np.int8)), c.mesh.n_fv, 0)
    u2 = p_adapt.transfer(c.mesh, m2, c.u)
    out = cpu_emu.run(wl, c.u.numpy(), ["p_degrees", "transfer"], p_thresholds=np.array([t_ref, t_coarse, 1, 7]),
                      degree_to=want, metric_degree_to=0)
    assert np.array_equal(out["p_degrees"].astype(np.int64), want)
    assert rel_err(torch.as_tensor(out["transfer"]), u2) <= 1e-13


@pytest.mark.parametrize("n_var", [5, 6])
def test_cpu_build_viscous(n_var):
    # BR1 lifting, viscous rates with degree jumps and blended elements, one RK step
    import dataclasses
    from oracle import viscous
    flux = {} if n_var == 5 else dict(volume_flux=W.VOL_PIROZZOLI, face_dg=W.RIEMANN_LLF)
    wl = curved_mixed(n=3, nmin=1, nmax=4, n_var=n_var, scramble=17, metric_degree=0, n_fv=5, **flux)
    wl = dataclasses.replace(wl, mu=(0.02, 0.03), Pr=(0.7, 0.9), D=(0.01, 0.04))
    c = _case(wl, smooth_state(47, n_var), noise=1e-3, seed=5)
    c.alpha = seeded_alpha(c.mesh.K, 48, values=(0.0, 0.0, 0.4, 1.0))
    dt = 0.2 * lsrk.timestep(c.mesh, c.gas, c.u, 0.5, c.alpha)
    out = cpu_emu.run(wl, c.u.numpy(), ["lift", "rhs", "rk_step"], alpha=c.alpha.numpy(), dt=dt)
    g = viscous.lift(c.mesh, c.u)
    assert rel_err(torch.as_tensor(out["lift"]).reshape(3 * n_var, -1), g.reshape(3 * n_var, -1)) <= 1e-12
    assert rel_err(torch.as_tensor(out["rhs"]), c.oracle_rhs()) <= _tol(c)
    want = lsrk.step(lambda v: c.f(v, c.alpha), c.u, dt)
    assert rel_err(torch.as_tensor(out["rk_step"]), want) <= 1e-11


@pytest.mark.parametrize("n_var,viscous", [(5, True), (6, True), (5, False)])
def test_cpu_build_timestep(n_var, viscous):
    # the convective and parabolic time steps over degrees 1..4 with blended elements
    import dataclasses
    from oracle import problem as P
    wl = curved_mixed(n=3, nmin=1, nmax=4, n_var=n_var, scramble=29, metric_degree=0, n_fv=5)
    if viscous:
        wl = dataclasses.replace(wl, mu=(0.02, 0.05), Pr=(0.7, 0.6), D=(0.01, 0.2))
    c = _case(wl, smooth_state(53, n_var), noise=1e-3, seed=6)
    c.alpha = seeded_alpha(c.mesh.K, 54, values=(0.0, 0.0, 0.4, 1.0))
    out = cpu_emu.run(wl, c.u.numpy(), ["timestep"], alpha=c.alpha.numpy(), cfl=np.array([0.6, 0.3]))
    want = lsrk.timestep(c.mesh, c.gas, c.u, 0.6, c.alpha, P.transport_of(wl) if viscous else None, 0.3)
    assert abs(float(out["timestep"][0]) - want) <= 1e-13 * want


def test_cpu_build_viscous_step_with_traces():
    # degrees 6 and 7: dg_rk_step's lift reads the neighbours' xi_1 sides from the
    # stage traces; five dg_rk_stage calls read u; both equal, and match the oracle
    import dataclasses
    wl = curved_mixed(n=2, nmin=6, nmax=7, scramble=31, metric_degree=0, n_fv=8)
    wl = dataclasses.replace(wl, mu=(0.02, 0.03), Pr=(0.7, 0.9))
    c = _case(wl, smooth_state(71, 5), noise=1e-3, seed=8)
    dt = 0.3 * lsrk.timestep(c.mesh, c.gas, c.u, 0.5)
    out = cpu_emu.run(wl, c.u.numpy(), ["rk_step", "rk_stages"], dt=dt)
    assert np.array_equal(out["rk_step"], out["rk_stages"])
    want = lsrk.step(lambda v: c.f(v, c.alpha), c.u, dt)
    assert rel_err(torch.as_tensor(out["rk_step"]), want) <= 1e-11


@pytest.mark.parametrize("refine,degree,scramble,amp,n_var", [("y", (4, 2), 7, 0.05, 5), ("yz", (2, 4), 5, 0.0, 5),
                                                              ("yz", (3, 3), 9, 0.05, 6)])
def test_cpu_build_mortars(refine, degree, scramble, amp, n_var):
    # non-conforming faces of types 1/2 and 3 with degree jumps across them, scrambled frames,
    # curved watertight elements: the RHS and one RK step against the oracle
    mesh = W.mortar_mesh(4, refine, degree, scramble_seed=scramble, amp=amp)
    kw = {} if n_var == 5 else dict(kappa=W.GAS_AIR_H2["kappa"], R=W.GAS_AIR_H2["R"])
    flux = (W.VOL_RANOCHA, W.RIEMANN_ROE_HH) if n_var == 5 else (W.VOL_PIROZZOLI, W.RIEMANN_LLF)
    wl = W.Workload("mortar", mesh, n_var, W.density_wave, flux[0], flux[1], W.RIEMANN_LLF, n_fv=8,
                    metric_degree=2 if amp else 1, **kw)
    c = _case(wl, smooth_state(57, n_var), noise=1e-3, seed=9)
    dt = 0.3 * lsrk.timestep(c.mesh, c.gas, c.u, 0.5)
    out = cpu_emu.run(wl, c.u.numpy(), ["rhs", "rk_step"], dt=dt)
    assert rel_err(torch.as_tensor(out["rhs"]), c.oracle_rhs()) <= 1e-12
    want = lsrk.step(lambda v: c.f(v, c.alpha), c.u, dt)
    assert rel_err(torch.as_tensor(out["rk_step"]), want) <= 1e-11


@pytest.mark.parametrize("refine,degree,scramble,amp,n_fv", [("y", (4, 3), 7, 0.05, 8), ("yz", (3, 2), 5, 0.0, 5)])
def test_cpu_build_mortars_blended(refine, degree, scramble, amp, n_fv):
    # the FV variants of the mortars: blending factors 0, 0.4 and 1 on both sides
    mesh = W.mortar_mesh(4, refine, degree, scramble_seed=scramble, amp=amp)
    wl = W.Workload("mortar", mesh, 5, W.density_wave, W.VOL_RANOCHA, W.RIEMANN_ROE_HH, W.RIEMANN_LLF,
                    n_fv=n_fv, metric_degree=2 if amp else 1)
    c = _case(wl, smooth_state(73), noise=1e-3, seed=12)
    c.alpha = seeded_alpha(c.mesh.K, scramble, values=(0.0, 0.4, 1.0))
    out = cpu_emu.run(wl, c.u.numpy(), ["rhs"], alpha=c.alpha.numpy())
    assert rel_err(torch.as_tensor(out["rhs"]), c.oracle_rhs()) <= 1e-12


@pytest.mark.parametrize("refine,degree,scramble,amp,n_var", [("y", (3, 2), 7, 0.05, 5), ("yz", (2, 3), 5, 0.0, 6)])
def test_cpu_build_viscous_mortars(refine, degree, scramble, amp, n_var):
    # viscous terms at mortars: the lifted gradient and the rate against the oracle
    from oracle import viscous
    mesh = W.mortar_mesh(4, refine, degree, scramble_seed=scramble, amp=amp)
    kw = {} if n_var == 5 else dict(kappa=W.GAS_AIR_H2["kappa"], R=W.GAS_AIR_H2["R"])
    flux = (W.VOL_RANOCHA, W.RIEMANN_ROE_HH) if n_var == 5 else (W.VOL_PIROZZOLI, W.RIEMANN_LLF)
    wl = W.Workload("mortar", mesh, n_var, W.density_wave, flux[0], flux[1], W.RIEMANN_LLF, n_fv=8,
                    metric_degree=2 if amp else 1, mu=(0.02, 0.03), Pr=(0.7, 0.9), D=(0.01, 0.04), **kw)
    c = _case(wl, smooth_state(77, n_var), noise=1e-3, seed=14)
    out = cpu_emu.run(wl, c.u.numpy(), ["lift", "rhs"])
    want_g = viscous.lift(c.mesh, c.u)
    assert rel_err(torch.as_tensor(out["lift"]).reshape(3 * n_var, -1), want_g.reshape(3 * n_var, -1)) <= 1e-12
    assert rel_err(torch.as_tensor(out["rhs"]), c.oracle_rhs()) <= 1e-12


@pytest.mark.parametrize("refine,degree,scramble,amp,flux", [("y", 3, 7, 0.05, 0), ("yz", 2, 5, 0.0, 1)])
def test_cpu_build_mortar_vjp(refine, degree, scramble, amp, flux):
    # the adjoint through the mortar fluxes (pure DG, one degree): two cotangents
    # against autograd through the oracle
    mesh = W.mortar_mesh(4, refine, degree, scramble_seed=scramble, amp=amp)
    pair = [(W.VOL_RANOCHA, W.RIEMANN_ROE_HH), (W.VOL_PIROZZOLI, W.RIEMANN_LLF)][flux]
    wl = W.Workload("mortar", mesh, 5, W.density_wave, pair[0], pair[1], W.RIEMANN_LLF, n_fv=8,
                    metric_degree=2 if amp else 1)
    c = _case(wl, smooth_state(87), noise=1e-3, seed=17)
    ws = torch.stack([torch.as_tensor(W.cotangents(s, tuple(c.u.shape)), dtype=T) for s in (88, 89)])
    out = cpu_emu.run(wl, c.u.numpy(), ["vjp"], w=ws.numpy())
    for b in range(2):
        assert rel_err(torch.as_tensor(out["vjp"][b]), _oracle_vjp(c, ws[b])) <= 1e-12


@pytest.mark.parametrize("refine,degree,scramble,amp,n_fv", [("y", (4, 3), 7, 0.05, 8), ("yz", (3, 2), 5, 0.0, 5)])
def test_cpu_build_fv_stored_mortars(refine, degree, scramble, amp, n_fv):
    # FV-stored elements on both sides of mortars: the rates against the oracle
    from oracle import native_fv, problem
    mesh = W.mortar_mesh(4, refine, degree, scramble_seed=scramble, amp=amp)
    wl = W.Workload("mortar", mesh, 5, W.density_wave, W.VOL_RANOCHA, W.RIEMANN_ROE_HH, W.RIEMANN_LLF,
                    n_fv=n_fv, metric_degree=2 if amp else 1)
    c = _case(wl, smooth_state(91), noise=1e-3, seed=18)
    K = c.mesh.K
    rng = np.random.default_rng(scramble)
    flag = rng.random(K) < 0.4
    ufv = torch.zeros(K, 5, n_fv, n_fv, n_fv, dtype=T)
    fvel = np.nonzero(flag)[0]
    ufv[torch.as_tensor(fvel)] = native_fv.dg_to_fv(c.mesh, c.u, fvel)
    ufv = ufv * (1.0 + 2e-2 * torch.as_tensor(rng.standard_normal(tuple(ufv.shape))))
    R, Rfv = native_fv.NativeRhs(c.mesh, c.gas, problem.params_of(wl))(c.u, ufv, flag)
    out = cpu_emu.run(wl, c.u.numpy(), ["rhs_fv"], ufv=ufv.reshape(K, 5, -1).numpy(), fv=flag.astype(np.float64))
    dg = torch.as_tensor(np.repeat(~flag, [int(c.mesh.offset[e + 1] - c.mesh.offset[e]) for e in range(K)]))
    assert rel_err(torch.as_tensor(out["rhs_fv_dg"])[:, dg], R[:, dg]) <= 1e-11
    sel = torch.as_tensor(flag)
    got_fv = torch.as_tensor(out["rhs_fv_fv"]).reshape(K, 5, -1)[sel].transpose(0, 1).reshape(5, -1)
    assert rel_err(got_fv, Rfv[sel].transpose(0, 1).reshape(5, -1)) <= 1e-11
