"""Pins of the oracle's FV-stored elements (Sections 3.1.2 and 3.2).

* minmod and the reconstructed face values: a table of cases, and no new
  extrema (a face value lies between its cell's mean and the neighbour's);
* on an affine periodic mesh of FV elements only, with scrambled element
  frames, the rates equal those of a brute-force second-order finite-volume
  scheme (minmod on the primitives, LLF) on the global fine grid of
  (n N_FV)^3 cells, written here from scratch;
* with the slopes forced to zero, the FV-stored path equals the first-order
  blended path (alpha = 1 on the same elements) mapped to sub-cell means;
* free-stream and discrete conservation on curved, scrambled, mixed-degree
  meshes with FV and DG elements side by side;
* switching: DG -> FV -> DG returns the DG state, FV -> DG -> FV returns the
  means when N_FV = N + 1, and both directions keep every element's content.
"""
import numpy as np
import pytest
import torch

from oracle import geometry, native_fv, ops1d, problem
from oracle.physics import prim_to_cons
from paper_2502_19342_amd import workloads as W

from oracle_cases import curved_mixed, smooth_state

T = torch.float64


def test_minmod_table_and_face_values():
    a = torch.tensor([1.0, -1.0, 2.0, -3.0, 0.0, 1.0, -2.0, 0.5])
    b = torch.tensor([2.0, -0.5, -1.0, 4.0, 1.0, 0.0, -2.0, 0.25])
    want = torch.tensor([1.0, -0.5, 0.0, 0.0, 0.0, 0.0, -2.0, 0.25])
    assert torch.equal(native_fv.minmod(a, b), want)
    rng = np.random.default_rng(3)
    wb, wi, wg = (torch.as_tensor(rng.standard_normal(10000)) for _ in range(3))
    fv = native_fv.face_value(wb, wi, wg)
    lo, hi = torch.minimum(wb, wg), torch.maximum(wb, wg)
    assert bool(((fv >= lo - 1e-15) & (fv <= hi + 1e-15)).all())       # between the cell and its neighbour
    # linear data: the face value is exact
    assert torch.allclose(native_fv.face_value(torch.tensor(1.0), torch.tensor(0.0), torch.tensor(2.0)),
                          torch.tensor(1.5))


def _llf(wl_, wr_, d, gamma):
    """LLF flux in direction d (unit normal) from primitive arrays [5, ...]."""
    def cons(w):
        rho, v, p = w[0], w[1:4], w[4]
        return np.stack([rho, rho * v[0], rho * v[1], rho * v[2], p / (gamma - 1) + 0.5 * rho * (v * v).sum(0)])

    def flux(w):
        rho, v, p = w[0], w[1:4], w[4]
        u = cons(w)
        vn = v[d]
        f = vn * u
        f[1 + d] = f[1 + d] + p
        f[4] = f[4] + p * vn
        return f
    lam = np.maximum(np.abs(wl_[1 + d]) + np.sqrt(gamma * wl_[4] / wl_[0]),
                     np.abs(wr_[1 + d]) + np.sqrt(gamma * wr_[4] / wr_[0]))
    return 0.5 * (flux(wl_) + flux(wr_)) - 0.5 * lam * (cons(wr_) - cons(wl_))


def _brute_force_rate(Wg, dx, gamma):
    """Rates of the cell means on a periodic uniform grid: MUSCL, minmod on primitives, LLF."""
    rate = np.zeros_like(Wg)
    for d in range(3):
        ax = 3 - d                                      # arrays are [var, z, y, x]
        fwd = np.roll(Wg, -1, axis=ax) - Wg
        bwd = Wg - np.roll(Wg, 1, axis=ax)
        sig = np.where(fwd * bwd > 0, np.sign(fwd) * np.minimum(np.abs(fwd), np.abs(bwd)), 0.0)
        left = Wg + 0.5 * sig                           # state at the cell's + face
        right = np.roll(Wg - 0.5 * sig, -1, axis=ax)    # the next cell's state at that face
        F = _llf(left, right, d, gamma)                 # flux through the + face of each cell
        rate -= (F - np.roll(F, 1, axis=ax)) / dx
    return rate


@pytest.mark.parametrize("N,n_fv,scramble", [(2, 5, None), (2, 5, 11), (3, 7, 5), (3, 4, 9)])
def test_all_fv_mesh_equals_fine_grid_muscl(N, n_fv, scramble):
    n = 3
    spec = W.structured_mesh(n, (0, 0, 0), (1, 1, 1), N, scramble_seed=scramble)
    wl = W.Workload("fv", spec, 5, W.density_wave, W.VOL_RANOCHA, W.RIEMANN_LLF, W.RIEMANN_LLF,
                    n_fv=n_fv, metric_degree=1)
    mesh, gas, _ = problem.build(wl)
    G = n * n_fv
    dx = 1.0 / G
    rng = np.random.default_rng(17)
    c = (np.arange(G) + 0.5) * dx
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    Wg = np.stack([1.0 + 0.2 * np.sin(2 * np.pi * (x + 2 * y)) + 0.05 * rng.random(x.shape),
                   0.3 * np.cos(2 * np.pi * z) + 0.05 * rng.standard_normal(x.shape),
                   -0.2 + 0.05 * rng.standard_normal(x.shape),
                   0.1 * np.sin(2 * np.pi * y) + 0.05 * rng.standard_normal(x.shape),
                   1.0 + 0.3 * np.cos(2 * np.pi * (x - z)) + 0.05 * rng.random(x.shape)])
    want = _brute_force_rate(Wg, dx, gas.gamma)
    Ug = prim_to_cons(torch.as_tensor(Wg), gas)
    # each element's sub-cells take the fine-grid cell that holds their centre
    K = mesh.K
    ufv = torch.zeros(K, 5, n_fv, n_fv, n_fv, dtype=T)
    where = np.zeros((K, 3, n_fv, n_fv, n_fv), dtype=np.int64)
    xi = torch.as_tensor(-1.0 + (np.arange(n_fv) + 0.5) * (2.0 / n_fv))
    centres = geometry.trilinear(torch.as_tensor(spec.corners), xi).numpy()      # [K, 3, s3, s2, s1]
    cell = np.floor(np.mod(centres, 1.0) / dx).astype(np.int64)
    for e in range(K):
        ix, iy, iz = cell[e, 0], cell[e, 1], cell[e, 2]
        ufv[e] = Ug[:, iz, iy, ix]
        where[e] = cell[e]
    flag = np.ones(K, dtype=bool)
    u = torch.zeros(5, mesh.n_node, dtype=T)
    R, Rfv = native_fv.NativeRhs(mesh, gas, problem.params_of(wl))(u, ufv, flag)
    assert float(R.abs().max()) == 0.0
    got = np.zeros_like(want)
    seen = np.zeros(want.shape[1:], dtype=np.int64)
    for e in range(K):
        ix, iy, iz = where[e, 0], where[e, 1], where[e, 2]
        got[:, iz, iy, ix] = Rfv[e].numpy()
        seen[iz, iy, ix] += 1
    assert np.all(seen == 1)                           # the sub-cells tile the fine grid once
    scale = np.abs(want).reshape(5, -1).max(axis=1)[:, None]
    err = (np.abs(got - want).reshape(5, -1) / scale).max()
    assert err <= 1e-12, err


def _mixed_case(n_var=5, seed=3, N_range=(2, 4), n_fv=None):
    flux = {} if n_var == 5 else dict(volume_flux=W.VOL_PIROZZOLI, face_dg=W.RIEMANN_LLF)
    wl = curved_mixed(n=3, nmin=N_range[0], nmax=N_range[1], n_var=n_var, scramble=13, metric_degree=0,
                      n_fv=n_fv or N_range[1] + 1, **flux)
    mesh, gas, f = problem.build(wl)
    u = problem.initial_state(mesh, gas, smooth_state(seed, n_var))
    rng = np.random.default_rng(seed)
    u = u * (1.0 + 1e-2 * torch.as_tensor(rng.standard_normal(tuple(u.shape))))
    flag = rng.random(mesh.K) < 0.4
    return wl, mesh, gas, f, u, flag


def test_zero_slopes_equal_the_blended_first_order_path(monkeypatch):
    wl, mesh, gas, f, u, flag = _mixed_case()
    fvel = np.nonzero(flag)[0]
    ufv = torch.zeros(mesh.K, 5, mesh.n_fv, mesh.n_fv, mesh.n_fv, dtype=T)
    ufv[torch.as_tensor(fvel)] = native_fv.dg_to_fv(mesh, u, fvel)
    monkeypatch.setattr(native_fv, "minmod", lambda a, b: torch.zeros_like(a))
    R, Rfv = native_fv.NativeRhs(mesh, gas, problem.params_of(wl))(u, ufv, flag)
    Rb = f(u, torch.as_tensor(flag, dtype=T))
    dg = ~flag
    for e in range(mesh.K):
        a, b = int(mesh.offset[e]), int(mesh.offset[e + 1])
        if dg[e]:
            assert torch.allclose(R[:, a:b], Rb[:, a:b], rtol=1e-12, atol=1e-12 * float(Rb.abs().max()))
        else:
            # the blended path's nodal FV rate is V3^+(dC/dt) / (h^3 J): the means' rate taken to DG
            nodal = native_fv.fv_to_dg(mesh, Rfv, [e])[e].reshape(Rb.shape[0], -1)
            scale = float(Rb[:, a:b].abs().max())
            assert torch.allclose(nodal, Rb[:, a:b], rtol=1e-10, atol=1e-10 * scale)


@pytest.mark.parametrize("n_var", [5, 6])
def test_freestream_and_conservation_mixed(n_var):
    wl, mesh, gas, f, u, flag = _mixed_case(n_var=n_var)
    nfv = mesh.n_fv
    native = native_fv.NativeRhs(mesh, gas, problem.params_of(wl))
    # free-stream: a constant state has zero rates everywhere
    u0 = problem.initial_state(mesh, gas, lambda x: W.freestream(x, n_var))
    ufv0 = torch.zeros(mesh.K, n_var, nfv, nfv, nfv, dtype=T)
    fvel = np.nonzero(flag)[0]
    ufv0[torch.as_tensor(fvel)] = native_fv.dg_to_fv(mesh, u0, fvel)
    R0, Rfv0 = native(u0, ufv0, flag)
    from test_oracle_rhs import term_scale
    scale = term_scale(mesh, gas, problem.params_of(wl), u0)      # the largest single DG term
    assert float(R0.abs().max()) <= 1e-13 * scale
    assert float(Rfv0.abs().max()) <= 1e-13 * scale
    # conservation: DG contents sum_w J R plus FV contents h^3 Jbar Rfv add to zero
    ufv = torch.zeros_like(ufv0)
    ufv[torch.as_tensor(fvel)] = native_fv.dg_to_fv(mesh, u, fvel)
    ufv = ufv * (1.0 + 1e-2 * torch.randn(ufv.shape, generator=torch.Generator().manual_seed(1), dtype=T))
    R, Rfv = native(u, ufv, flag)
    wJ = mesh.weights_flat() * mesh.jacobian_flat()
    total = (R * wJ[None]).sum(1)
    h = 2.0 / nfv
    for N in mesh.groups:
        jb = native.jbar(N)
        for s, e in enumerate(mesh.groups[N].elems.tolist()):
            if flag[e]:
                total = total + (h ** 3 * jb[s][None] * Rfv[e]).sum(dim=(1, 2, 3))
    scale = (R.abs() * wJ[None]).sum(1) + 1.0
    assert float((total.abs() / scale).max()) <= 1e-13


@pytest.mark.parametrize("N_range,n_fv", [((2, 4), 5), ((3, 3), 7), ((2, 2), 3)])
def test_switch_round_trips_and_contents(N_range, n_fv):
    wl, mesh, gas, f, u, flag = _mixed_case(N_range=N_range, n_fv=n_fv)
    K = mesh.K
    ufv = torch.zeros(K, 5, n_fv, n_fv, n_fv, dtype=T)
    none, all_ = np.zeros(K, bool), np.ones(K, bool)
    u1, ufv1 = native_fv.switch(mesh, u, ufv, none, all_)          # every element to FV
    u2, _ = native_fv.switch(mesh, u1, ufv1, all_, none)           # and back
    assert torch.allclose(u2, u, rtol=1e-12, atol=1e-12)
    h = 2.0 / n_fv
    wJ = mesh.weights_flat() * mesh.jacobian_flat()
    native = native_fv.NativeRhs(mesh, gas, problem.params_of(wl))
    for N, g in mesh.groups.items():
        jb = native.jbar(N)
        for s, e in enumerate(g.elems.tolist()):
            a, b = int(mesh.offset[e]), int(mesh.offset[e + 1])
            dg_content = (u[:, a:b] * wJ[a:b]).sum(1)
            fv_content = (h ** 3 * jb[s][None] * ufv1[e]).sum(dim=(1, 2, 3))
            assert torch.allclose(dg_content, fv_content, rtol=1e-13, atol=1e-15)
            if n_fv == N + 1:                                        # square maps: FV -> DG -> FV too
                back = native_fv.dg_to_fv(mesh, u2, [e])[0]
                assert torch.allclose(back, ufv1[e], rtol=1e-11, atol=1e-12)
