"""Modal decay indicator and blending factor (oracle).

Test infrastructure: a plain, slow reference.  Only the tests, the smoke check
and the benchmark's CPU-baseline leg use it.

Section 3.4: the nodal values of an indicator variable ``q`` are transformed
to the orthonormal Legendre basis, ``q_hat = (V_Leg^{-1})^{(x)3} q``.  The
share of mode ``m`` in direction ``d`` is the energy of the coefficients whose
index ``d`` equals ``m`` over the total energy (eq. modal_contribution).  A
least-squares line through ``(m, ln w_m)``, m = 0..N, gives the decay rate
``sigma_d = -slope`` (eq. modal_fit) and the indicator is
``I = min_d |sigma_d|`` (eq. modal_indicator).  The h-refinement indicator
takes the minimum of ``I(p)`` and ``I(Y)`` (two species).

The blending factor follows a sine ramp of half-width ``dT`` around ``T``:
``alpha = 1`` for ``I <= T - dT``, ``0`` for ``I >= T + dT`` and
``(1 - sin(pi (I - T) / (2 dT))) / 2`` between.  Energies below 1e-300 give
``I = +inf``; shares are floored at 1e-30 before the logarithm.
"""
from __future__ import annotations

import math

import torch

from . import ops1d
from .geometry import OracleMesh, apply3, _t
from .physics import Gas, to_prim

T = torch.float64


def modal_indicator(q: torch.Tensor, N: int) -> torch.Tensor:
    """``I`` for nodal fields ``q[E, n, n, n]`` of degree N."""
    qh = apply3(_t(ops1d.vleg_inv(N)), q)
    e2 = qh * qh
    tot = e2.sum(dim=(1, 2, 3))
    m = torch.arange(N + 1, dtype=T)
    mbar = m.mean()
    sigmas = []
    for d in range(3):
        dim = 3 - d                      # axis d of [E, k, j, i]
        other = tuple(x for x in (1, 2, 3) if x != dim)
        Em = e2.sum(dim=other)           # [E, n] ordered by the index along d
        w = Em / tot[:, None]
        y = torch.log(torch.clamp(w, min=1e-30))
        slope = ((m - mbar) * (y - y.mean(dim=1, keepdim=True))).sum(1) / ((m - mbar) ** 2).sum()
        sigmas.append((-slope).abs())
    ind = torch.minimum(torch.minimum(sigmas[0], sigmas[1]), sigmas[2])
    return torch.where(tot < 1e-300, torch.full_like(ind, math.inf), ind)


def ramp(ind: torch.Tensor, T0: float, dT: float) -> torch.Tensor:
    x = (ind - T0) / dT
    mid = 0.5 * (1.0 - torch.sin(0.5 * math.pi * torch.clamp(x, -1.0, 1.0)))
    return torch.where(x <= -1.0, torch.ones_like(ind), torch.where(x >= 1.0, torch.zeros_like(ind), mid))


def indicator(mesh: OracleMesh, gas: Gas, u: torch.Tensor, T0: float, dT: float,
              ind_vars: int = 1):
    """Per-element ``(I, alpha)``; ``ind_vars`` bit 0 pressure, bit 1 density, bit 2 Y1."""
    K = mesh.K
    I = torch.full((K,), math.inf, dtype=T)
    for N, g in mesh.groups.items():
        U = mesh.gather(u, N).transpose(0, 1)                  # [nvar, E, n, n, n]
        q = to_prim(U, gas)
        vals = []
        if ind_vars & 1:
            vals.append(modal_indicator(q.p, N))
        if ind_vars & 2:
            vals.append(modal_indicator(q.rho, N))
        if (ind_vars & 4) and q.Y is not None:
            vals.append(modal_indicator(q.Y, N))
        Ig = vals[0]
        for v in vals[1:]:
            Ig = torch.minimum(Ig, v)
        I[g.elems] = Ig
    return I, ramp(I, T0, dT)
