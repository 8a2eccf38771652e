"""Pins of the oracle's viscous terms on meshes with mortars (Sections 3.1.1, 3.2.2 and 3.2.3).

* lifting: the gradient of a continuous field that is linear inside every
  element is exact on affine mortar meshes of types 1/2 and 3, with degree
  jumps across the mortars and scrambled frames; the quadrature sum of J g
  vanishes for any (discontinuous) state on affine mortar meshes, the
  discrete divergence theorem that the big side's projected face values keep;
* the operator: a constant state has zero gradient and zero viscous rate on
  curved mortar meshes; every variable is conserved (affine and curved); the
  rate of two shear waves across the mortars, varying along them in both
  face directions, converges to the analytic one; one constant state on the
  coarse half and another on the fine half reduce the operator to the 1D BR1
  DGSEM, written out here on a periodic row of cells (the face values and
  fluxes the averages of both sides); the rate at each physical node is
  unchanged when every element's frame is rotated.
"""
import dataclasses

import numpy as np
import pytest
import torch

from oracle import physics, problem, viscous
from paper_2502_19342_amd import workloads as W

from oracle_cases import smooth_state

T = torch.float64


def _vwl(refine, degree, scramble=None, amp=0.0, n_var=5, n=4):
    mesh = W.mortar_mesh(n, refine, degree, scramble_seed=scramble, amp=amp)
    kw = {} if n_var == 5 else dict(kappa=W.GAS_AIR_H2["kappa"], R=W.GAS_AIR_H2["R"])
    flux = (W.VOL_RANOCHA, W.RIEMANN_ROE_HH) if n_var == 5 else (W.VOL_PIROZZOLI, W.RIEMANN_LLF)
    wl = W.Workload("mortar", mesh, n_var, W.density_wave, flux[0], flux[1], W.RIEMANN_LLF, n_fv=8,
                    metric_degree=2 if amp else 1, **kw)
    return dataclasses.replace(wl, mu=(0.02, 0.03), Pr=(0.7, 0.9), D=(0.01, 0.04))


def _tent(x):
    """Periodic, continuous, linear on [0, 1/2] and [1/2, 1]: kinks only on element faces."""
    y = np.mod(x, 1.0)
    return np.where(y < 0.5, y, 1.0 - y), np.where(y < 0.5, 1.0, -1.0)


CASES = [("y", (2, 3), 3), ("y", (3, 1), None), ("yz", (3, 2), 5), ("yz", (2, 4), 9)]


@pytest.mark.parametrize("refine,degree,scramble", CASES)
def test_mortar_lift_exact_on_piecewise_linear_fields(refine, degree, scramble):
    wl = _vwl(refine, degree, scramble)
    mesh, gas, _ = problem.build(wl)
    x = mesh.node_coords().numpy()
    # element centres decide the slope at the kinks' nodes (shared by two elements)
    cen = np.zeros_like(x)
    for N, g in mesh.groups.items():
        ctr = g.X.mean(dim=(2, 3, 4)).numpy()
        for s, e in enumerate(g.elems.tolist()):
            cen[:, mesh.offset[e]:mesh.offset[e + 1]] = ctr[s][:, None]
    coef = np.random.default_rng(1).standard_normal((5, 3))
    u = np.zeros((5, x.shape[1]))
    want = np.zeros((3, 5, x.shape[1]))
    for d in range(3):
        val, _ = _tent(x[d])
        _, slope = _tent(cen[d])
        for v in range(5):
            u[v] += coef[v, d] * val
            want[d, v] = coef[v, d] * slope
    u[0] += 2.0
    g = viscous.lift(mesh, torch.as_tensor(u))
    assert float((g - torch.as_tensor(want)).abs().max()) <= 1e-11


@pytest.mark.parametrize("refine,degree,scramble", CASES)
def test_mortar_lift_quadrature_sum_vanishes(refine, degree, scramble):
    wl = _vwl(refine, degree, scramble)
    mesh, gas, _ = problem.build(wl)
    u = problem.initial_state(mesh, gas, smooth_state(3))
    u = u + 0.05 * torch.as_tensor(np.random.default_rng(2).standard_normal(u.shape))   # jumps at every face
    g = viscous.lift(mesh, u)
    wJ = mesh.weights_flat() * mesh.jacobian_flat()
    total = (g * wJ).sum(-1)                                   # [3, nvar]
    scale = (g.abs() * wJ).sum(-1)
    assert float((total.abs() / scale).max()) <= 1e-13


@pytest.mark.parametrize("refine,degree,n_var", [("y", (4, 3), 5), ("yz", (3, 3), 6)])
def test_mortar_constant_state_has_no_viscous_terms(refine, degree, n_var):
    wl = _vwl(refine, degree, 11, amp=0.05, n_var=n_var)
    mesh, gas, _ = problem.build(wl)
    u = problem.initial_state(mesh, gas, lambda x: W.freestream(x, n_var))
    g = viscous.lift(mesh, u)
    R = viscous.viscous_rhs(mesh, gas, problem.transport_of(wl), u)
    ref = viscous.viscous_rhs(mesh, gas, problem.transport_of(wl),
                              problem.initial_state(mesh, gas, smooth_state(4, n_var)))
    assert float(g.abs().max()) <= 1e-10
    assert float(R.abs().max()) <= 1e-11 * float(ref.abs().max())


@pytest.mark.parametrize("refine,degree,scramble,amp,n_var", [("y", (4, 2), 7, 0.0, 5), ("yz", (2, 4), 5, 0.05, 5),
                                                              ("yz", (3, 3), 9, 0.05, 6)])
def test_mortar_viscous_rate_conserves(refine, degree, scramble, amp, n_var):
    wl = _vwl(refine, degree, scramble, amp, n_var)
    mesh, gas, _ = problem.build(wl)
    u = problem.initial_state(mesh, gas, smooth_state(5, n_var))
    u = u + 1e-3 * torch.as_tensor(np.random.default_rng(3).standard_normal(u.shape))
    R = viscous.viscous_rhs(mesh, gas, problem.transport_of(wl), u)
    wJ = mesh.weights_flat() * mesh.jacobian_flat()
    assert float(((R * wJ).sum(1).abs() / (R.abs() * wJ).sum(1))[1:].max()) <= 1e-13


@pytest.mark.parametrize("refine,scramble", [("y", 3), ("yz", 5)])
def test_mortar_shear_waves_converge(refine, scramble):
    # v = eps (0, sin k(x1 + x3), sin k(x1 + x2)): divergence-free, the stresses
    # cross the mortars at x1 = 0 and 1/2 and vary along them in both face
    # directions; d(rho v2)/dt = -2 mu k^2 eps sin k(x1 + x3), d(rho v3)/dt =
    # -2 mu k^2 eps sin k(x1 + x2), d(rho v1)/dt = mu d1(div v) = 0
    mu, eps, k = 0.05, 0.1, 2 * np.pi
    errs = []
    for N in (4, 7):
        wl = dataclasses.replace(_vwl(refine, N, scramble), mu=(mu, 0.0), Pr=(0.7, 0.7), D=(0.0, 0.0))
        mesh, gas, _ = problem.build(wl)
        x = mesh.node_coords()
        one = torch.ones_like(x[0])
        a2, a3 = k * (x[0] + x[2]), k * (x[0] + x[1])
        u = physics.prim_to_cons(torch.stack([one, 0 * one, eps * torch.sin(a2), eps * torch.sin(a3), one]), gas)
        R = viscous.viscous_rhs(mesh, gas, problem.transport_of(wl), u)
        sc = 2 * mu * k ** 2 * eps
        e = max(float((R[2] + sc * torch.sin(a2)).abs().max()), float((R[3] + sc * torch.sin(a3)).abs().max()),
                float(R[1].abs().max())) / sc
        errs.append((e, float(R[0].abs().max()) / sc))
    (e4, r4), (e7, r7) = errs
    assert e7 < 1e-3 and e7 < e4 / 10, errs
    assert max(r4, r7) <= 1e-9, errs


def _br1_1d(N, h, cells, gas, tr):
    """The 1D BR1 DGSEM (strong form on LGL nodes) on a periodic row of cells of width h with
    constant states ``cells[c]`` [nvar]: lifted gradient and viscous rate per cell, [C, nvar, N+1]."""
    from oracle import ops1d
    D = torch.as_tensor(ops1d.dmat(N))
    _, w = ops1d.lgl(N)
    w0 = float(w[0])
    C = len(cells)
    jac = h / 2
    U = torch.stack([c[:, None].expand(-1, N + 1) for c in cells])       # [C, nvar, n]
    ust = [0.5 * (U[c - 1, :, -1] + U[c, :, 0]) for c in range(C)]     # value at the left end of cell c
    G = torch.zeros_like(U)
    for c in range(C):
        G[c] = U[c] @ D.T
        G[c, :, -1] += (ust[(c + 1) % C] - U[c, :, -1]) / w0
        G[c, :, 0] -= (ust[c] - U[c, :, 0]) / w0
        G[c] /= jac
    def fx(uu, gx):                                                    # x component of F^v
        g3 = torch.stack([gx, torch.zeros_like(gx), torch.zeros_like(gx)])
        return viscous.viscous_flux(uu, g3, gas, tr)[0]
    F = torch.stack([fx(U[c], G[c]) for c in range(C)])                 # [C, nvar, n]
    fst = [0.5 * (F[c - 1, :, -1] + F[c, :, 0]) for c in range(C)]
    R = torch.zeros_like(U)
    for c in range(C):
        acc = F[c] @ D.T
        acc[:, -1] += (fst[(c + 1) % C] - F[c, :, -1]) / w0
        acc[:, 0] -= (fst[c] - F[c, :, 0]) / w0
        R[c] = -acc / jac
    return G, R


@pytest.mark.parametrize("refine,degree", [("y", (3, 3)), ("yz", (4, 4))])
def test_mortar_two_constant_states_reduce_to_1d_br1(refine, degree):
    # one constant state on the coarse half (x < 1/2), another on the fine half: a 1D
    # problem in x whose BR1 face values and fluxes are the averages of the two sides,
    # so the mortar operator must give the 1D BR1 DGSEM on a periodic row of 4 cells
    wl = _vwl(refine, degree, None)
    mesh, gas, _ = problem.build(wl)
    tr = problem.transport_of(wl)
    c0 = physics.prim_to_cons(torch.tensor([1.0, 0.3, -0.2, 0.1, 1.0], dtype=T), gas)
    c1 = physics.prim_to_cons(torch.tensor([0.7, -0.1, 0.4, 0.2, 0.6], dtype=T), gas)
    x = mesh.node_coords()
    u = torch.empty(5, x.shape[1], dtype=T)
    N = degree[0]
    # the nodes of each element take the state of its centre
    for Ng, g in mesh.groups.items():
        ctr = g.X.mean(dim=(2, 3, 4))
        for s, e in enumerate(g.elems.tolist()):
            u[:, mesh.offset[e]:mesh.offset[e + 1]] = (c0 if ctr[s, 0] < 0.5 else c1)[:, None]
    G1, R1 = _br1_1d(N, 0.25, [c0, c0, c1, c1], gas, tr)
    g3 = viscous.lift(mesh, u)
    R3 = viscous.viscous_rhs(mesh, gas, tr, u)
    from oracle import ops1d
    xi, _ = ops1d.lgl(N)
    worst_g = worst_r = 0.0
    for Ng, g in mesh.groups.items():
        ctr = g.X.mean(dim=(2, 3, 4))
        for s, e in enumerate(g.elems.tolist()):
            cell = int(ctr[s, 0] // 0.25)
            sl = slice(mesh.offset[e], mesh.offset[e + 1])
            xl = (x[0, sl] - (cell * 0.25 + 0.125)) / 0.125              # reference coordinate in x
            i = torch.as_tensor(np.abs(xl.numpy()[:, None] - xi[None, :]).argmin(1))
            worst_g = max(worst_g, float((g3[0, :, sl] - G1[cell][:, i]).abs().max()),
                          float(g3[1:, :, sl].abs().max()))
            worst_r = max(worst_r, float((R3[:, sl] - R1[cell][:, i]).abs().max()))
    assert worst_g <= 1e-11 * float(G1.abs().max()), worst_g
    assert worst_r <= 1e-11 * float(R1.abs().max()), worst_r


@pytest.mark.parametrize("refine,degree,amp,n_var,seed", [("y", (4, 3), 0.05, 5, 7), ("yz", (3, 2), 0.0, 6, 5)])
def test_mortar_viscous_rate_is_frame_invariant(refine, degree, amp, n_var, seed):
    rates, coords = [], []
    for scramble in (None, seed):
        wl = _vwl(refine, degree, scramble, amp, n_var)
        mesh, gas, _ = problem.build(wl)
        u = problem.initial_state(mesh, gas, smooth_state(9, n_var))
        rates.append(viscous.viscous_rhs(mesh, gas, problem.transport_of(wl), u))
        coords.append((mesh.node_coords().numpy(), mesh.offset))
    scale = rates[0].abs().amax(1, keepdim=True)
    worst = 0.0
    for e in range(len(coords[0][1]) - 1):
        cols = [off[e] + np.lexsort(np.round(x[:, off[e]:off[e + 1]], 9)[::-1]) for (x, off) in coords]
        worst = max(worst, float(((rates[0][:, cols[0]] - rates[1][:, cols[1]]).abs() / scale).max()))
    assert worst <= 1e-12, worst
