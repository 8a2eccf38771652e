"""Pins of the oracle's positivity-preserving limiter (Zhang and Shu; Section 3.5).

* an admissible state is returned bit for bit;
* after limiting, density and pressure are positive at every node and, on
  blended elements, at every sub-cell mean, and the element means (w J
  weighted) are kept;
* theta is the largest admissible one: at the critical point the density or the
  pressure sits at eps (the scaling goes no further than needed);
* the pressure root of the quadratic matches a 50-digit bisection of
  p(ubar + t d) = eps.
"""
import mpmath as mp
import numpy as np
import torch

from oracle import limiter, ops1d, problem
from oracle.geometry import apply3, _t
from oracle.physics import to_prim
from paper_2502_19342_amd import workloads as W

from oracle_cases import curved_mixed, seeded_alpha, smooth_state, state

T = torch.float64


def _case(seed=3):
    wl = curved_mixed(n=3, nmin=2, nmax=5, scramble=9, metric_degree=0, n_fv=6)
    mesh, gas, f = problem.build(wl)
    u = state(mesh, gas, smooth_state(seed))
    return wl, mesh, gas, u


def _element_means(mesh, u):
    w = mesh.weights_flat() * mesh.jacobian_flat()
    out = []
    for e in range(mesh.K):
        a, b = mesh.offset[e], mesh.offset[e + 1]
        out.append((u[:, a:b] * w[a:b]).sum(1) / w[a:b].sum())
    return torch.stack(out)


def _spoil(mesh, u, seed):
    """Push density and internal energy below zero at a few nodes, keeping every element mean admissible."""
    rng = np.random.default_rng(seed)
    u = u.clone()
    for e in rng.choice(mesh.K, size=8, replace=False):
        a, b = int(mesh.offset[e]), int(mesh.offset[e + 1])
        nodes = rng.choice(np.arange(a, b), size=2, replace=False)
        u[0, nodes[0]] = -0.05                                 # negative density
        u[4, nodes[1]] = 0.3 * u[4, nodes[1]] - 0.5 * float((u[1:4, nodes[1]] ** 2).sum() / u[0, nodes[1]])
    return u


def _subcell_means(mesh, u, N, slots):
    g = mesh.groups[N]
    U = mesh.gather(u, N)[slots]
    V = _t(ops1d.dg2fv(N, mesh.n_fv))
    return apply3(V, U * g.J[slots][:, None]) / apply3(V, g.J[slots])[:, None]


def test_admissible_state_is_unchanged():
    wl, mesh, gas, u = _case()
    alpha = seeded_alpha(mesh.K, 5)
    v, n_lim, n_bad = limiter.limit(mesh, gas, u, alpha)
    assert n_lim == 0 and n_bad == 0
    assert torch.equal(v, u)


def test_bounds_means_and_optimality():
    wl, mesh, gas, u = _case()
    u = _spoil(mesh, u, 11)
    alpha = seeded_alpha(mesh.K, 5, values=(0.0, 1.0))
    v, n_lim, n_bad = limiter.limit(mesh, gas, u, alpha)
    assert n_lim >= 8 and n_bad == 0
    q = to_prim(v, gas)
    assert float(q.rho.min()) > 0.0 and float(q.p.min()) > 0.0
    assert torch.allclose(_element_means(mesh, v), _element_means(mesh, u), rtol=1e-13, atol=1e-15)
    # blended elements: the sub-cell means are admissible too
    for N, g in mesh.groups.items():
        slots = torch.nonzero(alpha[g.elems] > 0).reshape(-1)
        if len(slots):
            sm = to_prim(_subcell_means(mesh, v, N, slots).transpose(0, 1), gas)
            assert float(sm.rho.min()) > 0.0 and float(sm.p.min()) > 0.0
    # changed elements: some node sits at eps = 1e-10 x the element mean, in density or
    # pressure (no more scaling than needed)
    means = _element_means(mesh, u)
    changed = [e for e in range(mesh.K) if not torch.equal(u[:, mesh.offset[e]:mesh.offset[e + 1]],
                                                           v[:, mesh.offset[e]:mesh.offset[e + 1]])]
    assert len(changed) == n_lim
    for e in changed:
        a, b = mesh.offset[e], mesh.offset[e + 1]
        if float(alpha[e]) > 0:
            continue                                          # the critical point may be a sub-cell mean
        qe = to_prim(v[:, a:b], gas)
        qm = to_prim(means[e][:, None], gas)
        r_rel = float(qe.rho.min() / qm.rho[0]) / 1e-10
        p_rel = float(qe.p.min() / qm.p[0]) / 1e-10
        # (eps_p is 1e-10 p: the 1e-13 rounding of E - |m|^2/2rho is 1e-3 of it)
        assert min(abs(r_rel - 1.0), abs(p_rel - 1.0)) <= 1e-2, (r_rel, p_rel)


def test_pressure_root_against_high_precision_bisection():
    rng = np.random.default_rng(7)
    g = 1.4
    for _ in range(40):
        ubar = np.array([1 + rng.random(), *(rng.uniform(-1, 1, 3)), 0.0])
        ubar[4] = 1.0 / (g - 1) + 0.5 * (ubar[1:4] ** 2).sum() / ubar[0]          # p(ubar) = 1
        target = np.array([0.5 + rng.random(), *(rng.uniform(-2, 2, 3)), 0.0])
        target[4] = -0.2 / (g - 1) + 0.5 * (target[1:4] ** 2).sum() / target[0]  # p(target) = -0.2
        d = target - ubar
        eps = 1e-10
        t = float(limiter._root_in_unit_interval(torch.as_tensor(ubar)[:, None], torch.as_tensor(d)[:, None],
                                                 torch.tensor([eps], dtype=T), g)[0])
        with mp.workdps(50):
            ub = [mp.mpf(float(x)) for x in ubar]
            dd = [mp.mpf(float(x)) for x in d]

            def p(s):
                w = [ub[i] + s * dd[i] for i in range(5)]
                return (mp.mpf(g) - 1) * (w[4] - (w[1] ** 2 + w[2] ** 2 + w[3] ** 2) / (2 * w[0])) - mp.mpf(eps)
            lo, hi = mp.mpf(0), mp.mpf(1)
            for _ in range(200):
                mid = (lo + hi) / 2
                lo, hi = (mid, hi) if p(mid) > 0 else (lo, mid)
            ref = float(lo)
        assert abs(t - ref) <= 1e-13 * max(ref, 1e-3)
