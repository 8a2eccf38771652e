"""Positivity-preserving limiter of Zhang and Shu (oracle).

Test infrastructure: a plain, slow reference.  Only the tests, the smoke check
and the benchmark's CPU-baseline leg use it.

Section 3.5 applies the limiter of Zhang and Shu to keep density and pressure
positive.  Per element, with the element mean ``ubar = sum w J u / sum w J``
(the quantity the scheme conserves), every point value ``u_P`` is replaced by
``ubar + theta (u_P - ubar)`` with one ``theta`` in [0, 1] per element, taken
in two steps as Zhang and Shu do:

1. density: ``theta_rho = min(1, min_P (rhobar - eps_rho) / (rhobar - rho_P))``
   over the points with ``rho_P < eps_rho``; only the density is scaled;
2. pressure: for every point whose pressure, after step 1, is below ``eps_p``,
   ``t_P`` solves ``p(ubar + t (u~_P - ubar)) = eps_p`` on (0, 1): with
   ``p = (gamma - 1)(E - |m|^2 / (2 rho))`` the product ``rho p / (gamma - 1)``
   is a quadratic in ``t``, positive at 0 and negative at 1, so it has one
   root there; ``theta_p = min_P t_P`` scales every variable.

The bounds are a small fraction of the element's own mean,
``eps_rho = 1e-10 rhobar`` and ``eps_p = 1e-10 p(ubar)`` (the paper leaves them
open): an absolute 1e-13 lies below the rounding of ``E - |m|^2 / (2 rho)``
when ``E`` is of order one, so the limited pressure could still come out
negative.  The
points are the LGL nodes and, on elements with ``alpha > 0``, the
J-weighted sub-cell means (``V3(J u) / V3(J)``, Section 3.2), which the FV
operator evaluates: a sub-cell mean of ``ubar + theta d`` is ``ubar + theta
d_s``, so the same formulas apply to them.  An element whose mean has
``rhobar <= 0`` or ``p(ubar) <= 0`` cannot be repaired and is left as it is
(reported).  One species only.
"""
from __future__ import annotations

import numpy as np
import torch

from . import ops1d
from .geometry import OracleMesh, apply3, _t
from .physics import Gas

T = torch.float64
EPS_REL = 1e-10


def _pressure(u: torch.Tensor, gamma: float) -> torch.Tensor:
    return (gamma - 1.0) * (u[4] - 0.5 * (u[1] ** 2 + u[2] ** 2 + u[3] ** 2) / u[0])


def _root_in_unit_interval(ubar, d, eps_p, gamma):
    """t in (0, 1) with p(ubar + t d) = eps_p, for points with p(ubar + d) < eps_p (ubar admissible).

    f(t) = rho(t) E(t) - |m(t)|^2 / 2 - eps_p rho(t) / (gamma - 1) = a t^2 + b t + c, c > 0 > f(1).
    """
    g1 = 1.0 / (gamma - 1.0)
    rb, mb, Eb = ubar[0], ubar[1:4], ubar[4]
    dr, dm, dE = d[0], d[1:4], d[4]
    a = dr * dE - 0.5 * (dm * dm).sum(0)
    b = rb * dE + Eb * dr - (mb * dm).sum(0) - eps_p * g1 * dr
    c = rb * Eb - 0.5 * (mb * mb).sum(0) - eps_p * g1 * rb
    disc = torch.clamp(b * b - 4.0 * a * c, min=0.0)
    # the root where f changes sign from + to - on (0, 1): stable forms of the two roots
    q = -0.5 * (b + torch.where(b >= 0, 1.0, -1.0) * torch.sqrt(disc))
    r1 = torch.where(a != 0, q / torch.where(a != 0, a, torch.ones_like(a)), torch.full_like(a, 2.0))
    r2 = torch.where(q != 0, c / torch.where(q != 0, q, torch.ones_like(q)), torch.full_like(q, 2.0))
    lin = -c / b                                               # a = 0: one linear root
    inside1 = (r1 >= 0) & (r1 <= 1)
    inside2 = (r2 >= 0) & (r2 <= 1)
    t = torch.where(inside2, r2, torch.where(inside1, r1, torch.zeros_like(r1)))
    return torch.where(a == 0, torch.clamp(lin, 0.0, 1.0), t)


def limit(mesh: OracleMesh, gas: Gas, u: torch.Tensor, alpha: torch.Tensor):
    """Limited state and the number of elements changed (``alpha`` selects the sub-cell points).

    Returns ``(u_new, n_limited, n_bad_mean)``.
    """
    if gas.nvar != 5:
        raise ValueError("the positivity limiter is single-species only")
    g = gas.gamma
    out = {}
    n_lim = 0
    n_bad = 0
    alpha = torch.as_tensor(alpha, dtype=T)
    for N, grp in mesh.groups.items():
        U = mesh.gather(u, N)                                    # [E, 5, n, n, n]
        w1 = grp.w
        w3 = w1[:, None, None] * w1[None, :, None] * w1[None, None, :]
        wJ = w3[None] * grp.J                                    # [E, n, n, n]
        ubar = (U * wJ[:, None]).sum(dim=(2, 3, 4)) / wJ.sum(dim=(1, 2, 3))[:, None]   # [E, 5]
        E = U.shape[0]
        pts = U.reshape(E, 5, -1)                                # nodes
        blended = alpha[grp.elems] > 0
        if bool(blended.any()):
            V = _t(ops1d.dg2fv(N, mesh.n_fv))
            sub = apply3(V, U * grp.J[:, None]) / apply3(V, grp.J)[:, None]
            sub = sub.reshape(E, 5, -1)
            # elements without blending repeat a node as their sub-cell points (no effect)
            sub = torch.where(blended[:, None, None], sub, pts[:, :, :1].expand_as(sub))
            pts = torch.cat([pts, sub], dim=2)
        rb = ubar[:, 0]
        pb = _pressure(ubar.T, g)
        good = (rb > 0) & (pb > 0)
        n_bad += int((~good).sum())
        eps_r = EPS_REL * rb
        eps_p = EPS_REL * pb
        # step 1: density
        rho = pts[:, 0]
        low = rho < eps_r[:, None]
        ratio = (rb[:, None] - eps_r[:, None]) / torch.where(low, rb[:, None] - rho, torch.ones_like(rho))
        th_r = torch.where(low, ratio, torch.ones_like(rho)).amin(1).clamp(max=1.0)
        th_r = torch.where(good, th_r, torch.ones_like(th_r))
        pts_t = pts.clone()
        pts_t[:, 0] = rb[:, None] + th_r[:, None] * (rho - rb[:, None])
        # step 2: pressure
        d = pts_t - ubar[:, :, None]                             # [E, 5, P]
        p_t = _pressure(pts_t.transpose(0, 1), g)                # [E, P]
        lowp = p_t < eps_p[:, None]
        t = _root_in_unit_interval(ubar.T[:, :, None].expand(5, E, d.shape[2]), d.transpose(0, 1),
                                   eps_p[:, None], g)
        th_p = torch.where(lowp, t, torch.ones_like(t)).amin(1).clamp(max=1.0)
        th_p = torch.where(good, th_p, torch.ones_like(th_p))
        changed = (th_r < 1.0) | (th_p < 1.0)
        n_lim += int(changed.sum())
        Ut = U.clone()
        Ut[:, 0] = rb[:, None, None, None] + th_r[:, None, None, None] * (U[:, 0] - rb[:, None, None, None])
        Un = ubar[:, :, None, None, None] + th_p[:, None, None, None, None] * (Ut - ubar[:, :, None, None, None])
        out[N] = torch.where(changed[:, None, None, None, None], Un, U)
    return mesh.scatter(out, 5), n_lim, n_bad
