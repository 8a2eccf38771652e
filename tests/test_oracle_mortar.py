"""Pins of the oracle's non-conforming (mortar) faces (Section 3.2.3).

* the 1D maps: projecting the interpolations to both halves returns a
  big-side polynomial (half their sum is the identity); the projection keeps the
  quadrature sum of the flux (conservation); interpolation to a half is exact
  for polynomials of the big side's degree;
* the mesh generator: every element side is covered exactly once, by a
  conforming face or by a mortar, with the expected mortar types;
* the operator: free-stream preservation and conservation on mortar meshes of
  types 1, 2 and 3, scrambled frames, degree jumps across the mortar, affine
  and curved (watertight) elements; the rate of a smooth state converges
  spectrally to the exact divergence of the Euler flux, the nodes next to the
  mortars included.
"""
import numpy as np
import pytest
import torch

from oracle import ops1d, physics, problem
from paper_2502_19342_amd import workloads as W

from oracle_cases import smooth_state

T = torch.float64


@pytest.mark.parametrize("N", range(1, 8))
def test_mortar_maps(N):
    I = 0.5 * sum(ops1d.mortar_project(N, k) @ ops1d.mortar_interp(N, k) for k in (0, 1))
    assert np.abs(I - np.eye(N + 1)).max() <= 1e-13
    _, w = ops1d.lgl(N)
    for k in (0, 1):
        assert np.abs(w @ ops1d.mortar_project(N, k) - w).max() <= 1e-14
        # a degree-N polynomial, restricted to half k and read in the half's coordinate
        x, _ = ops1d.lgl(N)
        c = np.random.default_rng(N + 10 * k).standard_normal(N + 1)
        p = lambda t: np.polynomial.polynomial.polyval(t, c)
        assert np.abs(ops1d.mortar_interp(N, k) @ p(x) - p((x + 2 * k - 1) / 2)).max() <= 1e-13


def _wl(refine, degree, scramble=None, amp=0.0, n=4, nvar=5):
    # curved faces: the face-normal polynomials are exact (so that a small side's
    # normal is the restriction of the big side's) from metric degree 2 on
    mesh = W.mortar_mesh(n, refine, degree, scramble_seed=scramble, amp=amp)
    kw = {} if nvar == 5 else dict(kappa=W.GAS_AIR_H2["kappa"], R=W.GAS_AIR_H2["R"])
    flux = (W.VOL_RANOCHA, W.RIEMANN_ROE_HH) if nvar == 5 else (W.VOL_PIROZZOLI, W.RIEMANN_LLF)
    return W.Workload("mortar", mesh, nvar, W.density_wave, flux[0], flux[1], W.RIEMANN_LLF, n_fv=8,
                      metric_degree=2 if amp else 1, **kw)


@pytest.mark.parametrize("refine,scramble", [("y", None), ("y", 3), ("yz", None), ("yz", 5)])
def test_mortar_mesh_covers_every_side_once(refine, scramble):
    m = W.mortar_mesh(4, refine, 3, scramble_seed=scramble)
    cnt = {}

    def add(e, s):
        cnt[(int(e), int(s))] = cnt.get((int(e), int(s)), 0) + 1
    for f in m.faces:
        add(f[0], f[1])
        add(f[2], f[3])
    for row in m.mortars:
        add(row[0], row[1])
        for k in range(4):
            if row[3 + k] >= 0:
                add(row[3 + k], row[7 + k])
    assert len(cnt) == 6 * m.n_elem and set(cnt.values()) == {1}
    types = set(m.mortars[:, 2].tolist())
    assert types == ({3} if refine == "yz" else ({1} if scramble is None else {1, 2}))
    # the coarse half meets the fine half across x = 1/2 and x = 0: one mortar per coarse face there
    assert len(m.mortars) == 2 * 4 * 4


CASES = [("y", 3, 3, 0.0), ("y", (4, 2), 7, 0.05), ("yz", 3, None, 0.0), ("yz", (2, 4), 5, 0.0),
         ("yz", (3, 3), 5, 0.05)]


@pytest.mark.parametrize("refine,degree,scramble,amp", CASES)
def test_mortar_freestream_and_conservation(refine, degree, scramble, amp):
    wl = _wl(refine, degree, scramble, amp)
    mesh, gas, f = problem.build(wl)
    zero = torch.zeros(mesh.K, dtype=T)
    u = problem.initial_state(mesh, gas, lambda x: W.freestream(x, 5))
    scale = float(f(problem.initial_state(mesh, gas, smooth_state(3)), zero).abs().max())
    # metric degree 2 (curved) carries rounding of about 5e-13 of the rate's scale
    # on conforming curved meshes as well
    assert float(f(u, zero).abs().max()) <= (1e-13 if amp == 0 else 1e-11) * scale
    u2 = problem.initial_state(mesh, gas, smooth_state(5))
    R = f(u2, zero)
    wJ = mesh.weights_flat() * mesh.jacobian_flat()
    assert float(((R * wJ).sum(1).abs() / (R.abs() * wJ).sum(1))[1:].max()) <= 1e-14


def _exact_rate(x: np.ndarray, gas, prim_fn) -> torch.Tensor:
    """-div F^c of the primitive field at points x [P, 3], by automatic differentiation."""
    xt = torch.as_tensor(x, dtype=T).requires_grad_(True)
    k = 2 * np.pi
    rho = 1.0 + 0.1 * torch.sin(k * (xt[:, 0] + xt[:, 1] + xt[:, 2])) + 0.05 * torch.cos(k * xt[:, 1])
    v = torch.stack([1.0 + 0.1 * torch.sin(k * xt[:, 2]), 0.5 + 0 * xt[:, 0], -0.3 + 0.1 * torch.cos(k * xt[:, 0])])
    p = 1.0 + 0.1 * torch.cos(k * (xt[:, 1] - xt[:, 2]))
    u = physics.prim_to_cons(torch.stack([rho, v[0], v[1], v[2], p]), gas)
    q = physics.to_prim(u, gas)
    div = torch.zeros(5, x.shape[0], dtype=T)
    for d in range(3):
        a = torch.zeros(3, x.shape[0], dtype=T)
        a[d] = 1.0
        F = physics.euler_flux(q, a)
        for c in range(5):
            div[c] += torch.autograd.grad(F[c].sum(), xt, retain_graph=True)[0][:, d]
    return -div.detach()


def _prim(x):
    k = 2 * np.pi
    rho = 1.0 + 0.1 * np.sin(k * (x[..., 0] + x[..., 1] + x[..., 2])) + 0.05 * np.cos(k * x[..., 1])
    v = [1.0 + 0.1 * np.sin(k * x[..., 2]), 0.5 + 0 * x[..., 0], -0.3 + 0.1 * np.cos(k * x[..., 0])]
    p = 1.0 + 0.1 * np.cos(k * (x[..., 1] - x[..., 2]))
    return np.stack([rho, v[0], v[1], v[2], p])


@pytest.mark.parametrize("refine,scramble", [("y", 3), ("yz", 5)])
def test_mortar_rate_converges_to_the_exact_divergence(refine, scramble):
    errs = []
    for N in (3, 6):
        wl = _wl(refine, N, scramble, 0.0)
        mesh, gas, f = problem.build(wl)
        u = problem.initial_state(mesh, gas, _prim)
        R = f(u, torch.zeros(mesh.K, dtype=T))
        want = _exact_rate(mesh.node_coords().numpy().T, gas, _prim)
        errs.append(float(((R - want).abs().amax(1) / want.abs().amax(1)).max()))
    assert errs[1] < 2e-3 and errs[1] < errs[0] / 20, errs


@pytest.mark.parametrize("NFV", [5, 6, 8])
def test_mortar_fv_maps(NFV):
    # the half's sub-faces copy (or, for odd N_FV, average) the big side's; the big side's
    # sub-faces sum the halves' fluxes by overlap: columns of M^FV_k0 sum to one, and
    # projecting the copies of both halves gives twice the big side's data
    S = sum(ops1d.mortar_fv_project(NFV, k) @ ops1d.mortar_fv_interp(NFV, k) for k in (0, 1))
    assert np.abs(S - 2 * np.eye(NFV)).max() <= 1e-15 or NFV % 2
    for k in (0, 1):
        assert np.abs(ops1d.mortar_fv_project(NFV, k).sum(0) - 1).max() <= 1e-15
        assert np.abs(ops1d.mortar_fv_interp(NFV, k).sum(1) - 1).max() <= 1e-15


@pytest.mark.parametrize("refine,degree,scramble,amp,n_fv", [("y", (4, 3), 7, 0.05, 8), ("yz", (3, 2), 5, 0.0, 5),
                                                             ("yz", (2, 4), 9, 0.05, 6)])
def test_mortar_blended_freestream_and_conservation(refine, degree, scramble, amp, n_fv):
    # FV-blended elements at mortars (the FV variants): a constant state stays, every variable is
    # conserved, with blending factors 0, 0.4 and 1 on both sides of the mortars
    mesh = W.mortar_mesh(4, refine, degree, scramble_seed=scramble, amp=amp)
    wl = W.Workload("mortar", mesh, 5, W.density_wave, W.VOL_RANOCHA, W.RIEMANN_ROE_HH, W.RIEMANN_LLF,
                    n_fv=n_fv, metric_degree=2 if amp else 1)
    om, gas, f = problem.build(wl)
    alpha = torch.as_tensor(np.random.default_rng(scramble).choice([0.0, 0.4, 1.0], size=om.K), dtype=T)
    touched = set(mesh.mortars[:, 0].tolist()) | set(mesh.mortars[:, 3:7].reshape(-1).tolist())
    assert any(alpha[e] > 0 for e in touched if e >= 0)
    u = problem.initial_state(om, gas, lambda x: W.freestream(x, 5))
    scale = float(f(problem.initial_state(om, gas, smooth_state(3)), alpha).abs().max())
    assert float(f(u, alpha).abs().max()) <= (1e-12 if amp == 0 else 1e-11) * scale
    R = f(problem.initial_state(om, gas, smooth_state(5)), alpha)
    wJ = om.weights_flat() * om.jacobian_flat()
    assert float(((R * wJ).sum(1).abs() / (R.abs() * wJ).sum(1))[1:].max()) <= 1e-13


@pytest.mark.parametrize("refine,degree,amp,n_fv,seed", [("y", (4, 3), 0.05, 8, 7), ("yz", (3, 2), 0.0, 5, 5)])
def test_mortar_rate_is_frame_invariant(refine, degree, amp, n_fv, seed):
    # the same physical mesh, state and blending with every element's local frame rotated:
    # the rate at each physical node is the same (the orientation maps of the DG and FV
    # variants, the sub-face grids of both sides, the reversed normals)
    rates, coords = [], []
    alpha = None
    for scramble in (None, seed):
        mesh = W.mortar_mesh(4, refine, degree, scramble_seed=scramble, amp=amp)
        wl = W.Workload("mortar", mesh, 5, W.density_wave, W.VOL_RANOCHA, W.RIEMANN_ROE_HH, W.RIEMANN_LLF,
                        n_fv=n_fv, metric_degree=2 if amp else 1)
        om, gas, f = problem.build(wl)
        if alpha is None:
            alpha = torch.as_tensor(np.random.default_rng(seed).choice([0.0, 0.4, 1.0], size=om.K), dtype=T)
        rates.append(f(problem.initial_state(om, gas, smooth_state(9)), alpha))
        coords.append((om.node_coords().numpy(), om.offset))
    scale = rates[0].abs().amax(1, keepdim=True)
    worst = 0.0
    for e in range(len(coords[0][1]) - 1):
        cols = []
        for (x, off) in coords:
            xe = np.round(x[:, off[e]:off[e + 1]], 9)
            cols.append(off[e] + np.lexsort(xe[::-1]))
        a, b = rates[0][:, cols[0]], rates[1][:, cols[1]]
        assert np.allclose(coords[0][0][:, cols[0]], coords[1][0][:, cols[1]], atol=1e-12)
        worst = max(worst, float(((a - b).abs() / scale).max()))
    assert worst <= 1e-12, worst
