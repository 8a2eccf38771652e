"""Pins of the oracle's viscous terms and BR1 lifting (Sections 2, 3.1.1 and 3.2.2).

* lifting: the gradient of a continuous field that is linear, or quadratic,
  inside every element is exact on affine meshes of mixed degree with
  scrambled element frames; a constant state lifts to zero on curved meshes;
  the lifted gradient of a smooth periodic field converges spectrally to the
  analytic one on a curved mesh;
* physics: a plane Couette flow and pure heat conduction against their closed
  forms; frame invariance under a rotation; the Stokes hypothesis (no bulk
  stress); the species diffusion fluxes sum to zero, and equal diffusivities
  reduce them to ``-rho D grad Y``;
* the operator: conservation of every variable on curved mixed-degree meshes
  (mortar-free periodic boxes); a shear wave, a temperature wave and a species
  wave against the analytic viscous rates.
"""
import numpy as np
import pytest
import torch

from oracle import physics, problem, viscous
from paper_2502_19342_amd import workloads as W

from oracle_cases import curved_mixed, smooth_state

T = torch.float64


def _mesh(n, nmin, nmax, amp=0.0, scramble=5, n_var=5, metric_degree=None, seed=7):
    wl = curved_mixed(n=n, nmin=nmin, nmax=nmax, amp=amp, scramble=scramble, n_var=n_var,
                      metric_degree=metric_degree, seed=seed)
    mesh, gas, _ = problem.build(wl)
    return wl, mesh, gas


def _element_centres(mesh):
    """Centre of the element that owns each node, ``[n_node, 3]``."""
    c = np.zeros((mesh.n_node, 3))
    for N, g in mesh.groups.items():
        ctr = g.X.mean(dim=(2, 3, 4)).numpy()                 # [E, 3]
        for s, e in enumerate(g.elems.tolist()):
            a, b = int(mesh.offset[e]), int(mesh.offset[e + 1])
            c[a:b] = ctr[s]
    return c


def _piecewise_field(mesh, n, quadratic):
    """Continuous periodic fields, linear (or quadratic) inside each element; values and exact gradients."""
    x = mesh.node_coords().numpy().T                           # [n_node, 3]
    xc = _element_centres(mesh)
    rng = np.random.default_rng(4)
    a = rng.uniform(-1, 1, size=(5, 3))
    b = rng.uniform(-1, 1, size=(5, 3)) if quadratic else np.zeros((5, 3))
    cell = np.floor(xc * n)                                    # element index along each axis
    s = x * n - cell                                           # local coordinate in [0, 1]
    sgn = np.where(cell % 2 == 0, 1.0, -1.0)
    tent = np.where(cell % 2 == 0, s, 1.0 - s)                 # distance of x n to the nearest even integer
    dtent = n * sgn
    quad = s * (1.0 - s)
    dquad = n * (1.0 - 2.0 * s)
    val = np.zeros((5, len(x)))
    grad = np.zeros((3, 5, len(x)))
    for v in range(5):
        base = 2.0 if v in (0, 4) else 0.0                     # keep rho and rho e away from zero
        val[v] = base + (a[v] * tent + b[v] * quad).sum(1)
        for d in range(3):
            grad[d, v] = a[v, d] * dtent[:, d] + b[v, d] * dquad[:, d]
    return torch.as_tensor(val), torch.as_tensor(grad)


@pytest.mark.parametrize("quadratic,nmin", [(False, 1), (True, 2)])
def test_lift_exact_on_piecewise_polynomials(quadratic, nmin):
    n = 4
    wl, mesh, gas = _mesh(n, nmin, 4)
    u, gx = _piecewise_field(mesh, n, quadratic)
    g = viscous.lift(mesh, u)
    assert torch.allclose(g, gx, rtol=0, atol=1e-11 * n), float((g - gx).abs().max())


@pytest.mark.parametrize("metric_degree", [0, 1])
def test_lift_of_constant_is_zero_on_curved_meshes(metric_degree):
    wl, mesh, gas = _mesh(3, 1, 4, amp=0.05, scramble=11, metric_degree=metric_degree)
    u = torch.tensor([1.3, 0.2, -0.4, 0.1, 2.5], dtype=T)[:, None].expand(5, mesh.n_node).contiguous()
    g = viscous.lift(mesh, u)
    assert float(g.abs().max()) <= 1e-11


def test_lift_converges_spectrally_on_curved_meshes():
    errs = []
    for N in (3, 5, 7):
        wl, mesh, gas = _mesh(2, N, N, amp=0.05, scramble=3, metric_degree=0)
        x = mesh.node_coords()                                 # [3, n_node]
        k = 2 * np.pi
        u = torch.stack([torch.sin(k * x[0]) * torch.cos(k * x[1]) + 2.0 + torch.sin(k * x[2])] * 5)
        gx = torch.stack([k * torch.cos(k * x[0]) * torch.cos(k * x[1]),
                          -k * torch.sin(k * x[0]) * torch.sin(k * x[1]),
                          k * torch.cos(k * x[2])])[:, None].expand(3, 5, mesh.n_node)
        errs.append(float((viscous.lift(mesh, u) - gx).abs().max()) / k)
    assert errs[2] < 2e-3 and errs[1] < errs[0] / 5 and errs[2] < errs[1] / 5, errs


def test_lift_of_piecewise_constants():
    # u = f(centre) in every element of an affine box: the volume part vanishes
    # and each node on a side of physical normal e_d gets, from that side,
    # (u* - u) n_d s / (J w_0) = +-2 (f_nbr - f_e) / (2 h w_0) in component d
    n = 4
    h = 1.0 / n
    wl, mesh, gas = _mesh(n, 1, 4, scramble=21)
    f = lambda c: np.stack([1.0 + np.sin(6 * c[..., 0] + 2 * c[..., 1]) + c[..., 2] ** 2 * (v + 1)
                            for v in range(5)])
    xc = _element_centres(mesh)
    x = mesh.node_coords().numpy().T
    u = torch.as_tensor(f(xc))
    deg = np.repeat(mesh.degree, np.diff(mesh.offset))
    w0 = 2.0 / (deg * (deg + 1.0))
    want = np.zeros((3, 5, mesh.n_node))
    for d in range(3):
        for sgn in (1.0, -1.0):
            on = np.abs((x[:, d] - xc[:, d]) - sgn * h / 2) < 1e-9
            nb = xc.copy()
            nb[:, d] = (nb[:, d] + sgn * h) % 1.0
            jump = 0.5 * (f(nb) - f(xc))
            want[d] += np.where(on, sgn * 2.0 * jump / (h * w0), 0.0)
    g = viscous.lift(mesh, u)
    assert torch.allclose(g, torch.as_tensor(want), rtol=0, atol=1e-11 * float(np.abs(want).max()))


def _mirror_map(mesh):
    """Node permutation of the reflection x_1 -> 1 - x_1 on a uniform affine box."""
    x = mesh.node_coords().numpy().T
    xc = _element_centres(mesh)
    key = lambda c, y: tuple(np.round(np.concatenate([c, y]) * 1e6).astype(np.int64).tolist())
    where = {key(xc[i], x[i]): i for i in range(len(x))}
    perm = np.empty(len(x), dtype=np.int64)
    for i in range(len(x)):
        c, y = xc[i].copy(), x[i].copy()
        c[0] = 1.0 - c[0]
        y[0] = 1.0 - y[0]
        perm[i] = where[key(c, y)]
    return torch.as_tensor(perm)


@pytest.mark.parametrize("n_var", [5, 6])
def test_mirror_symmetry(n_var):
    # the viscous rate of the mirrored state is the mirrored rate: the face
    # fluxes treat both sides alike and the element frames do not matter
    wl, mesh, gas = _mesh(3, 3, 3, scramble=31, n_var=n_var)
    tr = viscous.Transport(mu=(0.05, 0.03), Pr=(0.7, 0.9), D=(0.02, 0.05))
    u = problem.initial_state(mesh, gas, smooth_state(23, n_var))
    perm = _mirror_map(mesh)
    flip = torch.ones(n_var, 1, dtype=T)
    flip[1] = -1.0
    um = flip * u[:, perm]
    R = viscous.viscous_rhs(mesh, gas, tr, u)
    Rm = viscous.viscous_rhs(mesh, gas, tr, um)
    assert torch.allclose(Rm, flip * R[:, perm], rtol=0, atol=1e-11 * float(R.abs().max()))


# ---------------------------------------------------------------------------
# physics
# ---------------------------------------------------------------------------
def _state_and_grad(gas, rho, v, p, grho, gv, gp, Y=None, gY=None):
    """Conservative state and its gradient from primitives and their gradients (product rule)."""
    w = torch.stack([rho, v[0], v[1], v[2], p] + ([Y] if Y is not None else []))
    u = physics.prim_to_cons(w, gas)
    kap = gas.kappa_mix(Y) if Y is not None else torch.full_like(rho, gas.gamma)
    g = torch.zeros(3, gas.nvar, *rho.shape, dtype=T)
    for x in range(3):
        g[x, 0] = grho[x]
        g[x, 1:4] = grho[x] * v + rho * gv[x]
        dkap = 0.0
        if Y is not None:
            cv = [gas.R[j] / (gas.kappa[j] - 1.0) for j in range(2)]
            cp = [gas.kappa[j] * cv[j] for j in range(2)]
            cvm = Y * cv[0] + (1 - Y) * cv[1]
            cpm = Y * cp[0] + (1 - Y) * cp[1]
            dkap = ((cp[0] - cp[1]) * cvm - cpm * (cv[0] - cv[1])) / cvm ** 2 * gY[x]
            g[x, 5] = grho[x] * Y + rho * gY[x]
        g[x, 4] = gp[x] / (kap - 1.0) - p * dkap / (kap - 1.0) ** 2 \
            + 0.5 * grho[x] * (v * v).sum(0) + rho * (v * gv[x]).sum(0)
    return u, g


def test_couette_flow():
    gas = physics.Gas()
    tr = viscous.Transport(mu=(0.03, 0.0))
    a, y = 2.0, torch.tensor([0.3], dtype=T)
    one, zero = torch.ones(1, dtype=T), torch.zeros(1, dtype=T)
    v = torch.stack([a * y, zero, zero])
    gv = torch.zeros(3, 3, 1, dtype=T)
    gv[1, 0] = a                                              # d v_1 / d x_2
    u, g = _state_and_grad(gas, one, v, one, torch.zeros(3, 1, dtype=T), gv, torch.zeros(3, 1, dtype=T))
    F = viscous.viscous_flux(u, g, gas, tr)
    want = torch.zeros(3, 5, 1, dtype=T)
    want[1, 1] = -0.03 * a                                     # x_2-flux of rho v_1: -tau_21
    want[0, 2] = -0.03 * a                                     # x_1-flux of rho v_2: -tau_12
    want[1, 4] = -0.03 * a * (a * y)                           # x_2-flux of energy: -tau_21 v_1
    assert torch.allclose(F, want, rtol=1e-14, atol=1e-15)


def test_heat_conduction():
    gas = physics.Gas(R=(287.0, 287.0))
    mu, Pr = 0.02, 0.7
    tr = viscous.Transport(mu=(mu, 0.0), Pr=(Pr, 0.72))
    p = torch.tensor([1e5], dtype=T)
    Tm, dT = 300.0, torch.tensor([4.0, -1.0, 2.5], dtype=T)[:, None]
    rho = p / (287.0 * Tm)
    grho = -p / (287.0 * Tm ** 2) * dT
    zero3 = torch.zeros(3, 1, dtype=T)
    u, g = _state_and_grad(gas, rho, zero3, p, grho, torch.zeros(3, 3, 1, dtype=T), zero3)
    F = viscous.viscous_flux(u, g, gas, tr)
    lam = mu * 1.4 * 287.0 / 0.4 / Pr
    assert torch.allclose(F[:, 4], -lam * dT, rtol=1e-12)
    assert float(F[:, :4].abs().max()) <= 1e-12 * float(lam * dT.abs().max())


def _random_state(gas, shape, seed):
    r = np.random.default_rng(seed)
    rho = torch.as_tensor(r.uniform(0.5, 2.0, shape))
    v = torch.as_tensor(r.uniform(-1, 1, (3,) + shape))
    p = torch.as_tensor(r.uniform(0.5, 2.0, shape))
    Y = torch.as_tensor(r.uniform(0.1, 0.9, shape)) if gas.nvar == 6 else None
    u = physics.prim_to_cons(torch.stack([rho, *v, p] + ([Y] if Y is not None else [])), gas)
    g = torch.as_tensor(r.standard_normal((3, gas.nvar) + shape))
    return u, g


@pytest.mark.parametrize("n_var", [5, 6])
def test_frame_invariance_and_no_bulk_stress(n_var):
    gas = physics.Gas(nvar=n_var, kappa=W.GAS_AIR_H2["kappa"], R=W.GAS_AIR_H2["R"])
    tr = viscous.Transport(mu=(0.03, 0.05), Pr=(0.7, 0.8), D=(0.01, 0.04))
    u, g = _random_state(gas, (7,), 3)
    F = viscous.viscous_flux(u, g, gas, tr)                    # [3(x), nvar, 7]
    assert float((F[0, 1] + F[1, 2] + F[2, 3]).abs().max()) <= 1e-13   # trace of tau
    Q, _ = np.linalg.qr(np.random.default_rng(5).standard_normal((3, 3)))
    Q = torch.as_tensor(Q)
    ur = u.clone()
    ur[1:4] = Q @ u[1:4]
    gr = torch.einsum("xy,yv...->xv...", Q, g).clone()        # grad in the rotated frame
    gr[:, 1:4] = torch.einsum("ij,xj...->xi...", Q, gr[:, 1:4])
    Fr = viscous.viscous_flux(ur, gr, gas, tr)
    # scalar rows transform as vectors, the momentum rows as a tensor
    want = torch.einsum("xy,yv...->xv...", Q, F).clone()
    want[:, 1:4] = torch.einsum("ij,xj...->xi...", Q, want[:, 1:4])
    assert torch.allclose(Fr, want, rtol=1e-12, atol=1e-13)


def test_species_fluxes_sum_to_zero_and_reduce_for_equal_diffusivities():
    gas = physics.Gas(nvar=6, kappa=W.GAS_AIR_H2["kappa"], R=W.GAS_AIR_H2["R"])
    u, g = _random_state(gas, (9,), 8)
    J1, J2 = viscous.species_fluxes(u, g, gas, viscous.Transport(D=(0.01, 0.07)))
    assert float((J1 + J2).abs().max()) <= 1e-15
    D = 0.03
    J1, _ = viscous.species_fluxes(u, g, gas, viscous.Transport(D=(D, D)))
    rho = u[0]
    gY = (g[:, 5] - u[5] / rho * g[:, 0]) / rho
    assert torch.allclose(J1, -rho * D * gY, rtol=1e-13, atol=1e-15)


def test_interspecies_enthalpy_flux():
    # uniform temperature, a mass-fraction gradient and different species: the
    # energy flux is q_d = sum_j c_p,j T J_j, with grad T = 0 only if the
    # mixture's c_v enters the temperature gradient correctly
    gas = physics.Gas(nvar=6, kappa=W.GAS_AIR_H2["kappa"], R=W.GAS_AIR_H2["R"])
    D, Tm = 0.02, 2.0
    Y = torch.tensor([0.3], dtype=T)
    gY = torch.tensor([0.5, -1.0, 0.25], dtype=T)[:, None]
    Rm = Y * gas.R[0] + (1 - Y) * gas.R[1]
    rho = torch.ones(1, dtype=T)
    p = rho * Rm * Tm
    gp = rho * (gas.R[0] - gas.R[1]) * Tm * gY
    zero3 = torch.zeros(3, 1, dtype=T)
    u, g = _state_and_grad(gas, rho, zero3, p, zero3, torch.zeros(3, 3, 1, dtype=T), gp, Y=Y, gY=gY)
    F = viscous.viscous_flux(u, g, gas, viscous.Transport(mu=(0.01, 0.02), D=(D, D)))
    cp = [gas.kappa[j] * gas.R[j] / (gas.kappa[j] - 1.0) for j in range(2)]
    J1 = -rho * D * gY
    assert torch.allclose(F[:, 5], J1, rtol=1e-13)
    assert torch.allclose(F[:, 4], (cp[0] - cp[1]) * Tm * J1, rtol=1e-11)
    assert float(F[:, 1:4].abs().max()) == 0.0


# ---------------------------------------------------------------------------
# the operator
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n_var", [5, 6])
def test_conservation_on_curved_mixed_meshes(n_var):
    wl, mesh, gas = _mesh(3, 1, 4, amp=0.05, scramble=9, n_var=n_var, metric_degree=0)
    tr = viscous.Transport(mu=(0.05, 0.03), Pr=(0.7, 0.9), D=(0.02, 0.05))
    u = problem.initial_state(mesh, gas, smooth_state(17, n_var))
    R = viscous.viscous_rhs(mesh, gas, tr, u)
    wJ = mesh.weights_flat() * mesh.jacobian_flat()
    tot = (R * wJ).sum(1)
    scale = (R.abs() * wJ).sum(1)
    assert float((tot.abs() / scale.clamp_min(1e-300))[1:].max()) <= 1e-12
    assert float(R[0].abs().max()) == 0.0                      # no viscous mass flux


def _wave_case(N, n_var=5):
    wl, mesh, gas = _mesh(3, N, N, amp=0.0, scramble=13, n_var=n_var)
    return mesh, gas, mesh.node_coords()


def _errors(rate, scale):
    """Relative max errors of one rate at N = 5 and N = 7, and the largest other rate."""
    out = []
    for N in (5, 7):
        R, target, rest = rate(N)
        out.append((float((R - target).abs().max()) / scale, float(rest.abs().max())))
    return out


def _converges(errs, bound):
    (e5, r5), (e7, r7) = errs
    assert e7 < bound and e7 < e5 / 10, errs
    assert max(r5, r7) <= 1e-9, errs


def test_shear_wave_rate():
    mu, eps, k = 0.05, 0.1, 2 * np.pi

    def run(N, var):
        mesh, gas, x = _wave_case(N)
        one = torch.ones_like(x[0])
        u = physics.prim_to_cons(torch.stack([one, eps * torch.sin(k * x[1]), 0 * one, 0 * one, one]), gas)
        R = viscous.viscous_rhs(mesh, gas, viscous.Transport(mu=(mu, 0.0)), u)
        if var == 1:                                           # d(rho v1)/dt = mu v1''
            return R[1], -mu * k ** 2 * eps * torch.sin(k * x[1]), R[2:4]
        # d(rho e)/dt = d(tau_21 v1)/dx2 (uniform temperature: no heat flux)
        return R[4], mu * eps ** 2 * k ** 2 * torch.cos(2 * k * x[1]), R[2:4]
    _converges(_errors(lambda N: run(N, 1), mu * k ** 2 * eps), 5e-4)
    _converges(_errors(lambda N: run(N, 4), mu * eps ** 2 * k ** 2), 5e-2)


def test_temperature_wave_rate():
    mu, Pr, eps, k, T0 = 0.05, 0.7, 0.05, 2 * np.pi, 1.0
    lam = mu * (1.4 / 0.4) / Pr

    def run(N):
        mesh, _, x = _wave_case(N)
        gas = physics.Gas(R=(1.0, 1.0))
        Tm = T0 * (1 + eps * torch.sin(k * x[0]))
        p = torch.ones_like(Tm)
        z = torch.zeros_like(Tm)
        u = physics.prim_to_cons(torch.stack([p / Tm, z, z, z, p]), gas)
        R = viscous.viscous_rhs(mesh, gas, viscous.Transport(mu=(mu, 0.0), Pr=(Pr, Pr)), u)
        return R[4], -lam * T0 * eps * k ** 2 * torch.sin(k * x[0]), R[:4]   # d(rho e)/dt = lambda T''
    _converges(_errors(run, lam * T0 * eps * k ** 2), 3e-3)


def test_species_wave_rate():
    D, eps, k = 0.04, 0.2, 2 * np.pi

    def run(N):
        mesh, _, x = _wave_case(N, n_var=6)
        gas = physics.Gas(nvar=6, kappa=(1.4, 1.4), R=(1.0, 1.0))   # equal species: rho, p, T stay uniform
        one = torch.ones_like(x[0])
        z = 0 * one
        Y = 0.5 + eps * torch.sin(k * x[2])
        u = physics.prim_to_cons(torch.stack([one, z, z, z, one, Y]), gas)
        R = viscous.viscous_rhs(mesh, gas, viscous.Transport(mu=(0.0, 0.0), D=(D, D)), u)
        return R[5], -D * eps * k ** 2 * torch.sin(k * x[2]), R[:5]          # d(rho Y1)/dt = rho D Y1''
    _converges(_errors(run, D * eps * k ** 2), 5e-4)


# ---------------------------------------------------------------------------
# the time step
# ---------------------------------------------------------------------------
def test_parabolic_time_step_on_an_affine_box():
    # uniform state at rest on n^3 cubes of side h: |Ja^d|^2 / J^2 sums to 12 / h^2,
    # so dt^v = h^2 / (3 (2N + 1) delta) with delta = max(4/3, gamma / Pr) mu / rho
    from oracle import lsrk
    n, N = 4, 3
    wl, mesh, gas = _mesh(n, N, N, scramble=3)
    h = 1.0 / n
    rho, p = 1.3, 0.9
    u = physics.prim_to_cons(torch.tensor([rho, 0.0, 0.0, 0.0, p], dtype=T)[:, None].expand(5, mesh.n_node), gas)
    c = float(np.sqrt(1.4 * p / rho))
    dtc = 2.0 / ((2 * N + 1) * 3 * c * 2.0 / h)            # |Ja^d| / J = 2 / h per direction
    assert abs(lsrk.timestep(mesh, gas, u, 0.7) - 0.7 * dtc) <= 1e-13 * dtc
    for mu, Pr in ((0.01, 0.72), (0.3, 2.0)):
        delta = max(4.0 / 3.0, 1.4 / Pr) * mu / rho
        dtv = h * h / (3 * (2 * N + 1) * delta)
        got = lsrk.timestep(mesh, gas, u, 0.7, transport=viscous.Transport(mu=(mu, 0.0), Pr=(Pr, Pr)), cfl_v=0.4)
        want = 1.0 / (1.0 / (0.7 * dtc) + 1.0 / (0.4 * dtv))
        assert abs(got - want) <= 1e-13 * want
    # vanishing viscosity leaves the convective step; blended elements take the sub-cell spacing
    got = lsrk.timestep(mesh, gas, u, 0.7, transport=viscous.Transport(mu=(1e-300, 0.0)))
    assert abs(got - 0.7 * dtc) <= 1e-13 * dtc
    alpha = torch.zeros(mesh.K, dtype=T)
    alpha[5] = 0.5
    mu = 0.05
    delta = max(4.0 / 3.0, 1.4 / 0.72) * mu / rho
    dtv_fv = (2.0 / mesh.n_fv) ** 2 / (delta * 12 / h ** 2)
    dtc_fv = (2.0 / mesh.n_fv) / (3 * c * 2.0 / h)
    got = lsrk.timestep(mesh, gas, u, 0.7, alpha=alpha, transport=viscous.Transport(mu=(mu, 0.0)), cfl_v=0.4)
    want = 1.0 / (1.0 / (0.7 * min(dtc, dtc_fv)) + 1.0 / (0.4 * min(h * h / (3 * (2 * N + 1) * delta), dtv_fv)))
    assert abs(got - want) <= 1e-13 * want


def test_parabolic_time_step_uses_the_largest_diffusivity():
    from oracle import lsrk
    wl, mesh, gas = _mesh(3, 2, 2, scramble=None, n_var=6)
    gas = physics.Gas(nvar=6, kappa=(1.4, 1.4), R=(1.0, 1.0))
    w = torch.tensor([1.0, 0.0, 0.0, 0.0, 1.0, 0.5], dtype=T)[:, None].expand(6, mesh.n_node)
    u = physics.prim_to_cons(w, gas)
    small = lsrk.timestep(mesh, gas, u, 1.0, transport=viscous.Transport(mu=(1e-3, 1e-3), D=(0.0, 0.0)))
    big = lsrk.timestep(mesh, gas, u, 1.0, transport=viscous.Transport(mu=(1e-3, 1e-3), D=(0.0, 5.0)))
    h, N = 1.0 / 3, 2
    dtc = 2.0 / ((2 * N + 1) * 3 * np.sqrt(1.4) * 2.0 / h)
    dtv = h * h / (3 * (2 * N + 1) * 5.0)
    assert big < small
    assert abs(big - 1.0 / (1.0 / dtc + 1.0 / dtv)) <= 1e-13 * big
