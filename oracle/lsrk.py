"""Explicit low-storage Runge-Kutta time stepping and the CFL time step (oracle).

Test infrastructure: a plain, slow reference.  Only the tests, the smoke check
and the benchmark's CPU-baseline leg use it.

Section 3.3 integrates with a fourth-order low-storage explicit RK scheme of
Kennedy and Carpenter; the coefficients are not printed there.  This is the
five-stage, fourth-order, two-register (2N) scheme of Carpenter and Kennedy
(NASA TM-109112, 1994):

    k <- A_s k + dt R(u),   u <- u + B_s k,   s = 1..5,  A_1 = 0.

The convective time step of Section 3.3 is taken with ``alpha_RK = 1`` and the
element signal speed ``lambda_e = max_nodes sum_d (|v . Ja^d| + c |Ja^d|) / J``,
``dt = CFL min_e 2 / ((2 N_e + 1) lambda_e)``; blended elements also limit it by
``CFL h_FV / lambda_e`` with ``h_FV = 2 / N_FV``.

With viscous terms the parabolic step of Section 3.3 joins it,
``dt = 1 / (1 / (CFL dt^c) + 1 / (CFL^v dt^v))``, with ``beta_RK = 1``, the
element's parabolic rate ``lambda^v_e = max_nodes delta^v sum_d |Ja^d|^2 / J^2``
(the reference length 2 squared stands for ``dx^2``) and
``dt^v = min_e 4 / ((2 N_e + 1) lambda^v_e)``, blended elements also limiting
it by ``h_FV^2 / lambda^v_e``.  Readings: ``(2N + 1)`` to the first power, as
printed; ``delta^v = max(4/3 mu / rho, kappa mu / (Pr rho), D_1, D_2)`` at each
node, the largest of the momentum, heat and species diffusivities.
"""
from __future__ import annotations

from fractions import Fraction

import torch

from .geometry import OracleMesh
from .physics import Gas, sound_speed, to_prim

A = [Fraction(0), Fraction(-567301805773, 1357537059087), Fraction(-2404267990393, 2016746695238),
     Fraction(-3550918686646, 2091501179385), Fraction(-1275806237668, 842570457699)]
B = [Fraction(1432997174477, 9575080441755), Fraction(5161836677717, 13612068292357),
     Fraction(1720146321549, 2090206949498), Fraction(3134564353537, 4481467310338),
     Fraction(2277821191437, 14882151754819)]
A_F64 = [float(a) for a in A]
B_F64 = [float(b) for b in B]


def butcher():
    """The equivalent Butcher tableau (exact rationals) of the 2N scheme.

    Stage ``s`` evaluates R at ``u + sum_j a_sj dt R_j``; with
    ``k_s = A_s k_{s-1} + dt R_s`` and ``u_s = u_{s-1} + B_s k_s`` the weight of
    ``R_j`` inside ``k_s`` is ``prod_{r=j+1..s} A_r``.
    """
    S = len(A)

    def kw(s, j):                       # weight of dt R_j in k_s (0-based, j <= s)
        w = Fraction(1)
        for r in range(j + 1, s + 1):
            w *= A[r]
        return w

    a = [[Fraction(0)] * S for _ in range(S)]
    for s in range(1, S):
        for j in range(s):
            a[s][j] = sum((B[r] * kw(r, j) for r in range(j, s)), Fraction(0))
    b = [sum((B[r] * kw(r, j) for r in range(j, S)), Fraction(0)) for j in range(S)]
    c = [sum(row, Fraction(0)) for row in a]
    return a, b, c


def stage(rhs_fn, u: torch.Tensor, k: torch.Tensor, s: int, dt: float):
    """One stage (s = 0..4): returns the new ``(u, k)``; stage 0 writes ``k = dt R``."""
    R = rhs_fn(u)
    k = dt * R if s == 0 else A_F64[s] * k + dt * R
    return u + B_F64[s] * k, k


def step(rhs_fn, u: torch.Tensor, dt: float):
    k = torch.zeros_like(u)
    for s in range(5):
        u, k = stage(rhs_fn, u, k, s, dt)
    return u


def timestep(mesh: OracleMesh, gas: Gas, u: torch.Tensor, cfl: float, alpha=None, transport=None,
             cfl_v: float = 1.0) -> float:
    """The time step (module docstring); ``transport`` (an ``oracle.viscous.Transport``) adds the parabolic one."""
    best, best_v = float("inf"), float("inf")
    for N, g in mesh.groups.items():
        U = mesh.gather(u, N).transpose(0, 1)
        q = to_prim(U, gas)
        c = sound_speed(q)
        lam = torch.zeros_like(q.rho)
        metric2 = torch.zeros_like(q.rho)
        for d in range(3):
            a = g.Ja[:, d].transpose(0, 1)                     # [3, E, ...]
            lam = lam + ((q.v * a).sum(0).abs() + c * torch.sqrt((a * a).sum(0)))
            metric2 = metric2 + (a * a).sum(0)
        lam = (lam / g.J).amax(dim=(1, 2, 3))                  # [E]
        dtg = 2.0 / ((2 * N + 1) * lam)
        al = torch.as_tensor(alpha)[g.elems] if alpha is not None else None
        if al is not None:
            dfv = (2.0 / mesh.n_fv) / lam
            dtg = torch.where(al > 0, torch.minimum(dtg, dfv), dtg)
        best = min(best, float(dtg.min()))
        if transport is not None:
            if gas.nvar == 6:
                Y = q.Y
                mu = Y * transport.mu[0] + (1.0 - Y) * transport.mu[1]
                Pr = Y * transport.Pr[0] + (1.0 - Y) * transport.Pr[1]
                dmax = max(transport.D[0], transport.D[1])
            else:
                mu, Pr, dmax = transport.mu[0], transport.Pr[0], 0.0
            delta = torch.maximum(torch.maximum((4.0 / 3.0) * mu / q.rho, q.kappa * mu / (Pr * q.rho)),
                                  torch.full_like(q.rho, dmax))
            lam_v = (delta * metric2 / (g.J * g.J)).amax(dim=(1, 2, 3))
            dtv = 4.0 / ((2 * N + 1) * lam_v)
            if al is not None:
                dtv = torch.where(al > 0, torch.minimum(dtv, (2.0 / mesh.n_fv) ** 2 / lam_v), dtv)
            best_v = min(best_v, float(dtv.min()))
    if transport is None:
        return cfl * best
    return 1.0 / (1.0 / (cfl * best) + 1.0 / (cfl_v * best_v))
