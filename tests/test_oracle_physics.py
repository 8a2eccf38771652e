"""Pins of the oracle's EOS, two-point fluxes and Riemann solvers."""
import mpmath as mp
import numpy as np
import pytest
import torch

from oracle.physics import (Gas, entropy_vars, euler_flux, log_mean, prim_to_cons, riemann,
                            to_prim, two_point)

T = torch.float64
G1 = Gas(nvar=5, gamma=1.4)
G2 = Gas(nvar=6, gamma=1.4, kappa=(1.4, 1.41), R=(287.0, 4124.0))


def random_states(n, gas, seed, spread=0.3):
    rng = np.random.default_rng(seed)
    rho = 1 + spread * rng.uniform(-1, 1, n)
    v = rng.uniform(-1, 1, (3, n))
    p = 1 + spread * rng.uniform(-1, 1, n)
    comps = [rho, *v, p]
    if gas.nvar == 6:
        comps.append(rng.uniform(0.05, 0.95, n))
    w = torch.as_tensor(np.stack(comps), dtype=T)
    return prim_to_cons(w, gas)


def test_log_mean_matches_high_precision():
    rng = np.random.default_rng(0)
    a = rng.uniform(0.1, 3, 200)
    b = a * np.exp(rng.uniform(-1e-1, 1e-1, 200) * rng.choice([1e-6, 1e-3, 1e-1, 1.0], 200))
    got = log_mean(torch.tensor(a), torch.tensor(b)).numpy()
    for ai, bi, gi in zip(a, b, got):
        with mp.workdps(40):
            A, B = mp.mpf(ai), mp.mpf(bi)
            ref = A if A == B else (A - B) / (mp.log(A) - mp.log(B))
        # ln(a/b) loses ~eps/|ln(a/b)| relative accuracy; the switch keeps |ln(a/b)| > 0.02
        assert abs(gi - float(ref)) <= 2e-14 * float(ref)
    # equal arguments
    assert log_mean(torch.tensor([2.0]), torch.tensor([2.0])).item() == 2.0


def test_kappa_mix():
    # identical species -> the common ratio; pure species -> its own ratio
    g = Gas(nvar=6, kappa=(1.4, 1.4), R=(287.0, 4124.0))
    assert torch.allclose(g.kappa_mix(torch.tensor([0.0, 0.3, 1.0], dtype=T)), torch.tensor(1.4, dtype=T))
    assert abs(G2.kappa_mix(torch.tensor(1.0, dtype=T)).item() - 1.4) < 1e-15
    assert abs(G2.kappa_mix(torch.tensor(0.0, dtype=T)).item() - 1.41) < 1e-15
    # cp_mix / cv_mix by hand for Y1 = 0.25
    cv = [287 / 0.4, 4124 / 0.41]
    cp = [1.4 * cv[0], 1.41 * cv[1]]
    ref = (0.25 * cp[0] + 0.75 * cp[1]) / (0.25 * cv[0] + 0.75 * cv[1])
    assert abs(G2.kappa_mix(torch.tensor(0.25, dtype=T)).item() - ref) < 1e-15


@pytest.mark.parametrize("gas,kinds", [(G1, (0, 1, 2)), (G2, (1, 2))])
def test_two_point_consistency_and_symmetry(gas, kinds):
    uL = random_states(64, gas, 1)
    uR = random_states(64, gas, 2)
    a = torch.as_tensor(np.random.default_rng(3).standard_normal((3, 64)), dtype=T)
    qL, qR = to_prim(uL, gas), to_prim(uR, gas)
    for k in kinds:
        f_same = two_point(k, qL, qL, a, gas)
        assert torch.allclose(f_same, euler_flux(qL, a), rtol=1e-14, atol=1e-14)
        assert torch.allclose(two_point(k, qL, qR, a, gas), two_point(k, qR, qL, a, gas),
                              rtol=1e-14, atol=1e-14)


def test_ranocha_tadmor_entropy_condition():
    # (w_R - w_L) . f#(uL, uR) = (psi_R - psi_L) . a with psi = rho v (entropy U = -rho s/(gamma-1))
    uL = random_states(256, G1, 4, spread=0.5)
    uR = random_states(256, G1, 5, spread=0.5)
    # include nearly equal states (series branch of the log mean)
    uR[:, :64] = uL[:, :64] * (1 + 1e-5 * torch.randn(5, 64, dtype=T, generator=torch.Generator().manual_seed(0)))
    a = torch.as_tensor(np.random.default_rng(6).standard_normal((3, 256)), dtype=T)
    qL, qR = to_prim(uL, G1), to_prim(uR, G1)
    f = two_point(0, qL, qR, a, G1)
    wL, wR = entropy_vars(uL, G1), entropy_vars(uR, G1)
    dw = wR - wL
    lhs = (dw * f).sum(0)
    rhs = ((qR.rho * qR.v - qL.rho * qL.v) * a).sum(0)
    # the differences dw themselves carry ~eps |w| of rounding
    scale = (f.abs() * (dw.abs() + 1e-3 * (wL.abs() + wR.abs()))).sum(0)
    assert torch.max((lhs - rhs).abs() / scale) < 1e-13


def test_pirozzoli_kinetic_energy_form():
    # momentum flux is f_rho {v} + {p} a and energy flux f_rho {H}
    uL = random_states(16, G2, 7)
    uR = random_states(16, G2, 8)
    a = torch.ones(3, 16, dtype=T)
    qL, qR = to_prim(uL, G2), to_prim(uR, G2)
    f = two_point(1, qL, qR, a, G2)
    frho = 0.25 * (qL.rho + qR.rho) * ((qL.v + qR.v) * a).sum(0)
    assert torch.allclose(f[0], frho, rtol=1e-15)
    HL = (qL.E + qL.p) / qL.rho
    HR = (qR.E + qR.p) / qR.rho
    assert torch.allclose(f[4], frho * 0.5 * (HL + HR), rtol=1e-14)
    assert torch.allclose(f[5], frho * 0.5 * (qL.Y + qR.Y), rtol=1e-14)


@pytest.mark.parametrize("gas,kind", [(G1, 0), (G1, 1), (G2, 1), (G1, 2)])
def test_riemann_consistency_and_antisymmetry(gas, kind):
    uL = random_states(128, gas, 9)
    uR = random_states(128, gas, 10)
    n = torch.as_tensor(np.random.default_rng(11).standard_normal((3, 128)), dtype=T)
    s = torch.sqrt((n * n).sum(0))
    F = riemann(kind, uL, uL, n, gas)
    assert torch.allclose(F, euler_flux(to_prim(uL, gas), n), rtol=1e-13, atol=1e-13)
    F1 = riemann(kind, uL, uR, n, gas)
    F2 = riemann(kind, uR, uL, -n, gas)
    assert torch.allclose(F1, -F2, rtol=1e-13, atol=1e-13)
    # scaling with the area element
    F3 = riemann(kind, uL, uR, 3.0 * n, gas)
    assert torch.allclose(F3, 3.0 * F1, rtol=1e-13, atol=1e-13)
    del s


def test_roe_resolves_stationary_contact():
    # equal pressure, zero velocity, density jump: Roe flux = (0, p n, 0)
    w = torch.tensor([[1.0, 0.3], [0, 0], [0, 0], [0, 0], [2.0, 2.0]], dtype=T)
    u = prim_to_cons(w, G1)
    n = torch.tensor([[0.6], [0.0], [0.8]], dtype=T)
    F = riemann(0, u[:, :1], u[:, 1:], n, G1)
    ref = torch.tensor([[0.0], [1.2], [0.0], [1.6], [0.0]], dtype=T)
    assert torch.allclose(F, ref, atol=1e-15)
    # LLF smears it (dissipation proportional to the density jump)
    F_llf = riemann(1, u[:, :1], u[:, 1:], n, G1)
    assert abs(F_llf[0].item()) > 1e-3


def test_roe_entropy_fix_only_near_sonic_points():
    # supersonic states: no fix active, Roe equals the upwind flux f(uL)
    w = torch.tensor([[1.0, 1.1], [3.0, 3.05], [0, 0], [0, 0], [1.0, 1.05]], dtype=T)
    u = prim_to_cons(w, G1)
    n = torch.tensor([[1.0], [0.0], [0.0]], dtype=T)
    F = riemann(0, u[:, :1], u[:, 1:], n, G1)
    assert torch.allclose(F, euler_flux(to_prim(u[:, :1], G1), n), rtol=1e-12)
