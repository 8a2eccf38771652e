"""How far two correct evaluation orders of the FV sub-cell path lie apart (oracle, CPU).

On blended elements the GPU parity bar is four times the oracle's own spread
under 1-ulp input perturbations, because V^{FV->DG} (a pseudo-inverse,
Section 3.2) amplifies rounding by up to ||V^+||^3.  This checks that bar
against a second, equally valid evaluation order of the same arithmetic: the
three one-dimensional factors of the sub-cell maps V3 and V3^+ applied along
xi3, xi2, xi1 instead of xi1, xi2, xi3.  The two orders differ by more than
1e-12 at N = 5 and N = 7, by as much as the largest GPU error measured on
blended data (8.2e-12, the 64^3 N = 7 patches), and by at least half the 1-ulp
spread; on pure DG data they agree exactly (the order change touches only
the sub-cell path).
"""
import types

import numpy as np
import pytest
import torch

from oracle import geometry, problem
from oracle import rhs as oracle_rhs

from gpu_common import oracle_spread, rel_err
from oracle_cases import curved_mixed, seeded_alpha, smooth_state

T = torch.float64


def _reversed_apply3(A, f):
    for ax in (2, 1, 0):
        f = geometry.apply_axis(A, f, ax)
    return f


def _case(nmin, nmax, n_fv, alpha_values):
    wl = curved_mixed(n=3, nmin=nmin, nmax=nmax, scramble=5, metric_degree=0, n_fv=n_fv)
    mesh, gas, f = problem.build(wl)
    u = problem.initial_state(mesh, gas, smooth_state(73))
    rng = np.random.default_rng(2)
    u = u * (1.0 + 1e-3 * torch.as_tensor(rng.standard_normal(tuple(u.shape))))
    alpha = seeded_alpha(mesh.K, 11, values=alpha_values)
    return mesh, f, u, alpha


def _order_difference(f, u, alpha, monkeypatch):
    r1 = f(u, alpha)
    with monkeypatch.context() as mp:
        mp.setattr(oracle_rhs, "apply3", _reversed_apply3)
        r2 = f(u, alpha)
    return rel_err(r2, r1)


@pytest.mark.parametrize("nmin,nmax,n_fv,floor", [(5, 5, 6, 1e-12), (7, 7, 8, 8.2e-12), (1, 7, 8, 1e-12)])
def test_two_fv_evaluation_orders_differ_at_the_bar(nmin, nmax, n_fv, floor, monkeypatch):
    mesh, f, u, alpha = _case(nmin, nmax, n_fv, (0.0, 0.0, 0.5, 1.0))
    diff = _order_difference(f, u, alpha, monkeypatch)
    c = types.SimpleNamespace(f=f, u=u, alpha=alpha)
    c.oracle_rhs = lambda: f(u, alpha)
    spread = oracle_spread(c)
    assert diff > floor
    assert diff >= 0.5 * spread


def test_two_fv_evaluation_orders_agree_on_dg_data(monkeypatch):
    mesh, f, u, _ = _case(1, 7, 8, (0.0,))
    assert _order_difference(f, u, torch.zeros(mesh.K, dtype=T), monkeypatch) == 0.0
