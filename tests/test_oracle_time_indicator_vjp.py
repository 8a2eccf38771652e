"""Pins of the oracle's time integrator, indicator, convergence order and reference VJP."""
import math
from fractions import Fraction

import numpy as np
import pytest
import torch

from oracle import lsrk, ops1d
from oracle.indicator import modal_indicator, ramp, indicator
from paper_2502_19342_amd import workloads as W

from oracle_cases import curved_mixed, oracle_of, seeded_alpha, smooth_state, state

T = torch.float64


def test_lsrk_order_conditions():
    a, b, c = lsrk.butcher()
    S = len(b)
    Fr = Fraction

    def dot(x, y):
        return sum((xi * yi for xi, yi in zip(x, y)), Fr(0))

    def matvec(m, x):
        return [dot(row, x) for row in m]
    ac = matvec(a, c)
    conds = [
        (sum(b, Fr(0)), Fr(1)),
        (dot(b, c), Fr(1, 2)),
        (dot(b, [ci ** 2 for ci in c]), Fr(1, 3)),
        (dot(b, ac), Fr(1, 6)),
        (dot(b, [ci ** 3 for ci in c]), Fr(1, 4)),
        (dot(b, [ci * aci for ci, aci in zip(c, ac)]), Fr(1, 8)),
        (dot(b, matvec(a, [ci ** 2 for ci in c])), Fr(1, 12)),
        (dot(b, matvec(a, ac)), Fr(1, 24)),
    ]
    for got, want in conds:
        assert abs(float(got - want)) < 1e-15
    assert c[0] == 0 and S == 5


def test_lsrk_fourth_order_on_linear_ode():
    lam = -1.3 + 0.7j
    errs = []
    for n in (20, 40, 80):
        dt = 1.0 / n
        y = torch.tensor([1.0, 0.0], dtype=T)        # complex as 2-vector
        M = torch.tensor([[lam.real, -lam.imag], [lam.imag, lam.real]], dtype=T)
        for _ in range(n):
            y = lsrk.step(lambda v: M @ v, y, dt)
        ex = np.exp(lam)
        errs.append(math.hypot(y[0].item() - ex.real, y[1].item() - ex.imag))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(3.8 < r < 4.3 for r in rates), rates


def test_indicator_recovers_exact_decay_rate():
    # q_hat_ijk = a_i a_j a_k with a_m^2 = exp(-sigma m): every direction has w_m = c exp(-sigma m)
    N = 5
    sigma = 1.7
    am = torch.tensor([math.exp(-0.5 * sigma * m) for m in range(N + 1)], dtype=T)
    qh = am[:, None, None] * am[None, :, None] * am[None, None, :]
    V = torch.as_tensor(ops1d.vleg(N), dtype=T)
    q = qh
    for ax in range(3):
        q = torch.movedim(torch.movedim(q, 2 - ax, -1) @ V.T, -1, 2 - ax)
    ind = modal_indicator(q[None], N)
    assert abs(ind.item() - sigma) < 1e-12


def test_indicator_smooth_vs_jump_and_ramp():
    N = 4
    x, _ = ops1d.lgl(N)
    X = torch.as_tensor(x, dtype=T)
    lin = 2.0 + 0.1 * X[None, None, :] + 0.05 * X[None, :, None] + 0 * X[:, None, None]
    jump = torch.where(X[None, None, :] > 0.1, 10.0, 0.1) + 0 * X[:, None, None] + 0 * X[None, :, None]
    ind = modal_indicator(torch.stack([lin, jump]), N)
    assert ind[0] > 10.0 and ind[1] < 1.0
    a = ramp(torch.tensor([-1.0, 0.5, 1.0, 1.5, 4.0, math.inf], dtype=T), 1.0, 0.5)
    assert a[0] == 1 and a[1] == 1 and abs(a[2] - 0.5) < 1e-15 and a[4] == 0 and a[5] == 0
    assert abs(a[3] - 0.5 * (1 - math.sin(math.pi / 2))) < 1e-15
    # zero energy -> +inf
    assert torch.isinf(modal_indicator(torch.zeros(1, N + 1, N + 1, N + 1, dtype=T), N)).all()


def test_indicator_blast_marks_the_front():
    wl = W.make_workload("C2", n=8)
    mesh, gas, f = oracle_of(wl)
    u = state(mesh, gas, wl.prim)
    I, alpha = indicator(mesh, gas, u, wl.ind_T, wl.ind_dT, wl.ind_vars)
    # the constant-pressure elements away from the sphere are smooth, the front is not
    assert float(alpha.max()) > 0.0
    assert float((alpha == 0).float().mean()) > 0.3


@pytest.mark.slow
def test_eoc_density_wave():
    # Section 4.2: order N+1 for a smooth density wave; split form on LGL nodes, N = 3
    from oracle.problem import build, initial_state
    errs = []
    t_end = 0.1
    for n in (4, 8):
        wl = W.make_workload("C1", n=n)
        mesh, gas, f = build(wl)
        u = initial_state(mesh, gas, W.density_wave)
        alpha = torch.zeros(mesh.K, dtype=T)
        dt0 = lsrk.timestep(mesh, gas, u, 0.5)
        nst = int(math.ceil(t_end / dt0))
        dt = t_end / nst
        for _ in range(nst):
            u = lsrk.step(lambda v: f(v, alpha), u, dt)
        x = mesh.node_coords().numpy().T
        ex = initial_state(mesh, gas, lambda y: W.density_wave_exact(y, t_end))
        w = mesh.weights_flat() * mesh.jacobian_flat()
        errs.append(float(torch.sqrt(((u[0] - ex[0]) ** 2 * w).sum())))
        del x
    eoc = math.log(errs[0] / errs[1]) / math.log(2.0)
    assert 3.5 < eoc < 5.0, (errs, eoc)


def test_reference_vjp_against_finite_differences():
    # autograd through the oracle is its reference VJP; pin it with central differences
    wl = curved_mixed(n=2, nmin=2, nmax=3, scramble=3, seed=5)
    mesh, gas, f = oracle_of(wl)
    u = state(mesh, gas, smooth_state(61))
    alpha = seeded_alpha(mesh.K, 8, values=(0.0, 0.5))
    rng = np.random.default_rng(62)
    w = torch.as_tensor(rng.standard_normal(tuple(u.shape)), dtype=T)
    uu = u.clone().requires_grad_(True)
    r = f(uu, alpha)
    (g,) = torch.autograd.grad((r * w).sum(), uu)
    h = 1e-6
    for k in range(3):
        v = torch.as_tensor(rng.standard_normal(tuple(u.shape)), dtype=T) * u.abs().mean(1, keepdim=True)
        fd = ((f(u + h * v, alpha) - f(u - h * v, alpha)) * w).sum() / (2 * h)
        ad = (g * v).sum()
        assert abs(float(fd - ad)) <= 1e-6 * abs(float(ad)), (float(fd), float(ad))
