"""Pins of the oracle's FV-stored elements at mortars (Sections 3.1.2, 3.2 and 3.2.3).

* free-stream and discrete conservation on mortar meshes of types 1/2 and 3
  (curved, degree jumps, scrambled frames) with FV-stored elements on both
  sides of the mortars;
* with the slopes forced to zero, the FV-stored path equals the blended
  first-order path at the mortars (alpha = 1 on the same elements, the FV
  variants of the mortar maps) mapped to sub-cell means;
* the rates at each physical node (FV elements' rates taken to nodes) are
  unchanged when every element's frame is rotated.
"""
import numpy as np
import pytest
import torch

from oracle import native_fv, problem
from paper_2502_19342_amd import workloads as W

from oracle_cases import smooth_state

T = torch.float64


def _case(refine, degree, scramble, amp, n_fv, seed=3, flag_seed=None, noise=1e-2):
    mesh = W.mortar_mesh(4, refine, degree, scramble_seed=scramble, amp=amp)
    wl = W.Workload("mortar", mesh, 5, W.density_wave, W.VOL_RANOCHA, W.RIEMANN_ROE_HH, W.RIEMANN_LLF,
                    n_fv=n_fv, metric_degree=2 if amp else 1)
    om, gas, f = problem.build(wl)
    u = problem.initial_state(om, gas, smooth_state(seed))
    rng = np.random.default_rng(seed)
    u = u * (1.0 + noise * torch.as_tensor(rng.standard_normal(tuple(u.shape))))
    flag = np.random.default_rng(flag_seed if flag_seed is not None else seed).random(om.K) < 0.4
    touched = set(mesh.mortars[:, 0].tolist()) | set(mesh.mortars[:, 3:7].reshape(-1).tolist())
    assert any(flag[e] for e in touched if e >= 0) and any(not flag[e] for e in touched if e >= 0)
    return wl, om, gas, f, u, flag


def _means(om, u, flag):
    nfv = om.n_fv
    ufv = torch.zeros(om.K, u.shape[0], nfv, nfv, nfv, dtype=T)
    fvel = np.nonzero(flag)[0]
    ufv[torch.as_tensor(fvel)] = native_fv.dg_to_fv(om, u, fvel)
    return ufv


CASES = [("y", (4, 3), 7, 0.05, 8), ("yz", (3, 2), 5, 0.0, 5), ("yz", (2, 4), 9, 0.05, 6)]


@pytest.mark.parametrize("refine,degree,scramble,amp,n_fv", CASES)
def test_fv_stored_mortars_freestream_and_conservation(refine, degree, scramble, amp, n_fv):
    wl, om, gas, f, u, flag = _case(refine, degree, scramble, amp, n_fv)
    native = native_fv.NativeRhs(om, gas, problem.params_of(wl))
    u0 = problem.initial_state(om, gas, lambda x: W.freestream(x, 5))
    R0, Rfv0 = native(u0, _means(om, u0, flag), flag)
    ref, _ = native(u, _means(om, u, flag), flag)
    scale = float(ref.abs().max())
    assert float(R0.abs().max()) <= (1e-12 if amp == 0 else 1e-11) * scale
    assert float(Rfv0.abs().max()) <= (1e-12 if amp == 0 else 1e-11) * scale
    ufv = _means(om, u, flag)
    ufv = ufv * (1.0 + 1e-2 * torch.randn(ufv.shape, generator=torch.Generator().manual_seed(1), dtype=T))
    R, Rfv = native(u, ufv, flag)
    wJ = om.weights_flat() * om.jacobian_flat()
    total = (R * wJ[None]).sum(1)
    h = 2.0 / om.n_fv
    for N in om.groups:
        jb = native.jbar(N)
        for s, e in enumerate(om.groups[N].elems.tolist()):
            if flag[e]:
                total = total + (h ** 3 * jb[s][None] * Rfv[e]).sum(dim=(1, 2, 3))
    assert float((total.abs() / ((R.abs() * wJ[None]).sum(1) + 1.0)).max()) <= 1e-13


@pytest.mark.parametrize("refine,degree,scramble,amp,n_fv", CASES)
def test_fv_stored_mortars_with_zero_slopes_equal_the_blended_path(monkeypatch, refine, degree, scramble, amp,
                                                                    n_fv):
    wl, om, gas, f, u, flag = _case(refine, degree, scramble, amp, n_fv)
    ufv = _means(om, u, flag)
    monkeypatch.setattr(native_fv, "minmod", lambda a, b: torch.zeros_like(a))
    R, Rfv = native_fv.NativeRhs(om, gas, problem.params_of(wl))(u, ufv, flag)
    Rb = f(u, torch.as_tensor(flag, dtype=T))
    for e in range(om.K):
        a, b = int(om.offset[e]), int(om.offset[e + 1])
        scale = float(Rb.abs().max())
        if not flag[e]:
            assert torch.allclose(R[:, a:b], Rb[:, a:b], rtol=1e-12, atol=1e-12 * scale), e
        else:
            nodal = native_fv.fv_to_dg(om, Rfv, [e])[e].reshape(Rb.shape[0], -1)
            assert torch.allclose(nodal, Rb[:, a:b], rtol=1e-10, atol=1e-10 * scale), e


@pytest.mark.parametrize("refine,degree,amp,n_fv,seed", [("y", (4, 3), 0.05, 8, 7), ("yz", (3, 2), 0.0, 5, 5)])
def test_fv_stored_mortar_rates_are_frame_invariant(refine, degree, amp, n_fv, seed):
    rates, coords = [], []
    for scramble in (None, seed):
        # no noise: it is drawn per node index, which the frames reorder
        wl, om, gas, f, u, flag = _case(refine, degree, scramble, amp, n_fv, seed=11, flag_seed=seed, noise=0.0)
        R, Rfv = native_fv.NativeRhs(om, gas, problem.params_of(wl))(u, _means(om, u, flag), flag)
        fvel = np.nonzero(flag)[0].tolist()
        nodal = native_fv.fv_to_dg(om, Rfv, fvel)
        for e in fvel:
            R[:, int(om.offset[e]):int(om.offset[e + 1])] = nodal[e].reshape(R.shape[0], -1)
        rates.append(R)
        coords.append((om.node_coords().numpy(), om.offset))
    scale = rates[0].abs().amax(1, keepdim=True)
    worst = 0.0
    for e in range(len(coords[0][1]) - 1):
        cols = [off[e] + np.lexsort(np.round(x[:, off[e]:off[e + 1]], 9)[::-1]) for (x, off) in coords]
        worst = max(worst, float(((rates[0][:, cols[0]] - rates[1][:, cols[1]]).abs() / scale).max()))
    assert worst <= 1e-11, worst


@pytest.mark.parametrize("refine,n_fv", [("y", 4), ("yz", 5)])
def test_fv_stored_mortars_reduce_to_1d_minmod_fv(refine, n_fv):
    # every element FV-stored, means that vary with x only (frames unscrambled, so
    # the first sub-cell index runs along x): the mortar ghosts are the means of the
    # small sides' boundary data, so the scheme is the 1D second-order FV scheme
    # (minmod on the primitives, the FV Riemann flux) on the periodic row of
    # 4 N_FV sub-cells in x, written out here
    from oracle.physics import prim_to_cons, riemann
    wl, om, gas, f, u, _ = _case(refine, 3, None, 0.0, n_fv, noise=0.0)
    flag = np.ones(om.K, dtype=bool)
    C = 4 * n_fv
    xc = (np.arange(C) + 0.5) / C
    k = 2 * np.pi
    w1 = torch.as_tensor(np.stack([1 + 0.2 * np.sin(k * xc) + 0.1 * np.cos(2 * k * xc), 0.3 + 0.1 * np.sin(k * xc),
                                   0.2 + 0 * xc, -0.1 + 0 * xc, 1 + 0.1 * np.cos(k * xc)]))
    c1 = prim_to_cons(w1, gas)                                         # [5, C]
    ufv = torch.zeros(om.K, 5, n_fv, n_fv, n_fv, dtype=T)
    cell0 = {}
    for N, g in om.groups.items():
        xmin = g.X[:, 0].amin(dim=(1, 2, 3))
        for s, e in enumerate(g.elems.tolist()):
            i0 = int(round(float(xmin[s]) * 4)) * n_fv
            cell0[e] = i0
            ufv[e] = c1[:, i0:i0 + n_fv][:, None, None, :].expand(-1, n_fv, n_fv, -1)
    _, Rfv = native_fv.NativeRhs(om, gas, problem.params_of(wl))(u, ufv, flag)
    # the 1D scheme
    wp = native_fv.to_w(c1, gas)
    ext = torch.cat([wp[:, -1:], wp, wp[:, :1]], dim=1)
    sig = native_fv.minmod(ext[:, 1:-1] - ext[:, :-2], ext[:, 2:] - ext[:, 1:-1])
    wl_ = wp + 0.5 * sig                                              # left state of face i + 1/2
    wr_ = torch.roll(wp - 0.5 * sig, -1, dims=1)                      # right state of face i + 1/2
    nx = torch.zeros(3, C, dtype=T)
    nx[0] = 1.0
    F = riemann(wl.face_flux_fv, prim_to_cons(wl_, gas), prim_to_cons(wr_, gas), nx, gas, wl.volume_flux)
    R1 = -(F - torch.roll(F, 1, dims=1)) * C                          # dC/dt / volume, dx = 1 / C
    worst = 0.0
    for e, i0 in cell0.items():
        want = R1[:, i0:i0 + n_fv][:, None, None, :]
        worst = max(worst, float((Rfv[e] - want).abs().max()))
    assert worst <= 1e-12 * float(R1.abs().max()), worst
