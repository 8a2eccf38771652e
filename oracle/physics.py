"""Equation of state, physical fluxes, two-point fluxes and Riemann solvers (oracle).

Test infrastructure: a plain, slow reference.  Only the tests, the smoke check
and the benchmark's CPU-baseline leg use it.

States are tensors ``[nvar, ...]`` of conservative variables
``(rho, rho v1, rho v2, rho v3, rho e, [rho Y1])`` (Section 2, eq. ns_equation
without the viscous terms; with two species only ``Y1`` is transported and
``Y2 = 1 - Y1``, eq. species_closure).  Directions are unnormalised vectors
``a[3, ...]``; every flux returned is already contracted with ``a``.
"""
from __future__ import annotations

from dataclasses import dataclass

import torch


@dataclass(frozen=True)
class Gas:
    """Single species (``nvar = 5``, ratio ``gamma``) or two ideal-gas species."""

    nvar: int = 5
    gamma: float = 1.4
    kappa: tuple = (1.4, 1.4)
    R: tuple = (287.0, 287.0)

    def kappa_mix(self, Y1: torch.Tensor) -> torch.Tensor:
        """Mixture heat-capacity ratio from linear mixing rules (eq. mix_R_kappa, eq. mix_cp_cv)."""
        cv = [self.R[j] / (self.kappa[j] - 1.0) for j in range(2)]
        cp = [self.kappa[j] * cv[j] for j in range(2)]
        Y2 = 1.0 - Y1
        return (Y1 * cp[0] + Y2 * cp[1]) / (Y1 * cv[0] + Y2 * cv[1])


@dataclass
class Prim:
    rho: torch.Tensor
    v: torch.Tensor          # [3, ...]
    p: torch.Tensor
    E: torch.Tensor          # rho e, total energy per volume
    kappa: torch.Tensor      # heat-capacity ratio (constant or mixture)
    Y: torch.Tensor | None   # Y1 for two species


def to_prim(u: torch.Tensor, gas: Gas) -> Prim:
    """Conservative -> primitive; ``p = (kappa - 1)(rho e - |rho v|^2 / (2 rho))`` (eq. eos, eq. energy)."""
    rho = u[0]
    v = u[1:4] / rho
    E = u[4]
    if gas.nvar == 6:
        Y = u[5] / rho
        kap = gas.kappa_mix(Y)
    else:
        Y = None
        kap = torch.full_like(rho, gas.gamma)
    p = (kap - 1.0) * (E - 0.5 * rho * (v * v).sum(0))
    return Prim(rho, v, p, E, kap, Y)


def prim_to_cons(w: torch.Tensor, gas: Gas) -> torch.Tensor:
    """Primitive ``(rho, v1, v2, v3, p[, Y1])`` -> conservative."""
    rho, v, p = w[0], w[1:4], w[4]
    if gas.nvar == 6:
        Y = w[5]
        kap = gas.kappa_mix(Y)
    else:
        kap = torch.full_like(rho, gas.gamma)
    E = p / (kap - 1.0) + 0.5 * rho * (v * v).sum(0)
    comps = [rho, rho * v[0], rho * v[1], rho * v[2], E]
    if gas.nvar == 6:
        comps.append(rho * w[5])
    return torch.stack(comps)


def sound_speed(q: Prim) -> torch.Tensor:
    return torch.sqrt(q.kappa * q.p / q.rho)


def euler_flux(q: Prim, a: torch.Tensor) -> torch.Tensor:
    """Convective flux ``F^c(u) . a`` (inviscid part of eq. ns_flux_notation)."""
    vn = (q.v * a).sum(0)
    comps = [q.rho * vn]
    comps += [q.rho * q.v[d] * vn + q.p * a[d] for d in range(3)]
    comps.append((q.E + q.p) * vn)
    if q.Y is not None:
        comps.append(q.rho * q.Y * vn)
    return torch.stack(comps)


def _safe_where(cond, a_fn, b_fn, *args):
    return torch.where(cond, a_fn(*args), b_fn(*args))


def log_mean(a: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
    """Logarithmic mean ``(a - b) / (ln a - ln b)`` (Ismail & Roe 2009 evaluation).

    With ``zeta = a/b``, ``f = (zeta-1)/(zeta+1)``, ``u = f^2``: for ``u < 1e-4``
    the series ``F = 1 + u/3 + u^2/5 + u^3/7`` replaces ``ln(zeta)/(2f)``; the mean
    is ``(a+b)/(2F)``.
    """
    f = (a - b) / (a + b)
    u = f * f
    small = u < 1e-4
    F_series = 1.0 + u / 3.0 + u * u / 5.0 + u * u * u / 7.0
    f_safe = torch.where(small, torch.ones_like(f), f)
    zeta_safe = torch.where(small, torch.full_like(f, 2.0), a / b)
    F_log = torch.log(zeta_safe) / (2.0 * f_safe)
    F = torch.where(small, F_series, F_log)
    return (a + b) / (2.0 * F)


def flux_ranocha(qL: Prim, qR: Prim, a: torch.Tensor, gamma: float) -> torch.Tensor:
    """Entropy-conserving and kinetic-energy-preserving two-point flux (Ranocha 2018).

    Single species only.  ``a`` is the averaged contravariant direction.
    """
    rho_ln = log_mean(qL.rho, qR.rho)
    beta_ln = log_mean(qL.rho / qL.p, qR.rho / qR.p)        # mean of rho/p
    vbar = 0.5 * (qL.v + qR.v)
    pbar = 0.5 * (qL.p + qR.p)
    vn = (vbar * a).sum(0)
    f_rho = rho_ln * vn
    comps = [f_rho] + [f_rho * vbar[d] + pbar * a[d] for d in range(3)]
    vLvR = 0.5 * (qL.v * qR.v).sum(0)
    pv = 0.5 * (qL.p * (qR.v * a).sum(0) + qR.p * (qL.v * a).sum(0))
    comps.append(f_rho * (1.0 / ((gamma - 1.0) * beta_ln) + vLvR) + pv)
    return torch.stack(comps)


def flux_pirozzoli(qL: Prim, qR: Prim, a: torch.Tensor) -> torch.Tensor:
    """Kinetic-energy-preserving two-point flux of Pirozzoli (Section 3.5).

    Mass flux ``{rho}{v}.a``, momentum ``f_rho {v} + {p} a``, energy
    ``f_rho {H}`` with ``H = (rho e + p)/rho``; a transported mass fraction
    gets ``f_rho {Y}``.
    """
    rho_bar = 0.5 * (qL.rho + qR.rho)
    vbar = 0.5 * (qL.v + qR.v)
    pbar = 0.5 * (qL.p + qR.p)
    Hbar = 0.5 * ((qL.E + qL.p) / qL.rho + (qR.E + qR.p) / qR.rho)
    f_rho = rho_bar * (vbar * a).sum(0)
    comps = [f_rho] + [f_rho * vbar[d] + pbar * a[d] for d in range(3)] + [f_rho * Hbar]
    if qL.Y is not None:
        comps.append(f_rho * 0.5 * (qL.Y + qR.Y))
    return torch.stack(comps)


def flux_central(qL: Prim, qR: Prim, a: torch.Tensor) -> torch.Tensor:
    """Arithmetic mean of the physical fluxes, ``(f(uL) + f(uR))/2 . a``."""
    return 0.5 * (euler_flux(qL, a) + euler_flux(qR, a))


def two_point(kind: int, qL: Prim, qR: Prim, a: torch.Tensor, gas: Gas) -> torch.Tensor:
    if kind == 0:
        if gas.nvar != 5:
            raise ValueError("the entropy-conserving flux is single-species only")
        return flux_ranocha(qL, qR, a, gas.gamma)
    if kind == 1:
        return flux_pirozzoli(qL, qR, a)
    if kind == 2:
        return flux_central(qL, qR, a)
    raise ValueError(kind)


def riemann_llf(uL, uR, qL: Prim, qR: Prim, nvec: torch.Tensor) -> torch.Tensor:
    """Local Lax-Friedrichs flux times the face area (Section 5.1 uses it at FV faces).

    ``nvec = n s``: unit normal times area element.
    """
    s = torch.sqrt((nvec * nvec).sum(0))
    n = nvec / s
    lam = torch.maximum((qL.v * n).sum(0).abs() + sound_speed(qL),
                        (qR.v * n).sum(0).abs() + sound_speed(qR))
    F = 0.5 * (euler_flux(qL, n) + euler_flux(qR, n)) - 0.5 * lam * (uR - uL)
    return F * s


def riemann_roe_hh(uL, uR, qL: Prim, qR: Prim, nvec: torch.Tensor, gamma: float) -> torch.Tensor:
    """Roe flux with the Harten-Hyman entropy fix, times the face area (Section 3.1.1).

    Single species.  Acoustic waves ``k = 1, 5`` get the fix
    ``delta = max(0, lam~ - lam(uL), lam(uR) - lam~)``; if ``|lam~| < delta``,
    ``|lam~|`` is replaced by ``(lam~^2/delta + delta)/2``.
    """
    s = torch.sqrt((nvec * nvec).sum(0))
    n = nvec / s
    sL, sR = torch.sqrt(qL.rho), torch.sqrt(qR.rho)
    wsum = sL + sR
    v = (sL * qL.v + sR * qR.v) / wsum
    HL = (qL.E + qL.p) / qL.rho
    HR = (qR.E + qR.p) / qR.rho
    H = (sL * HL + sR * HR) / wsum
    v2 = (v * v).sum(0)
    c2 = (gamma - 1.0) * (H - 0.5 * v2)
    c = torch.sqrt(c2)
    rho_t = sL * sR
    vn = (v * n).sum(0)

    drho = qR.rho - qL.rho
    dp = qR.p - qL.p
    dv = qR.v - qL.v
    dvn = (dv * n).sum(0)

    a1 = (dp - rho_t * c * dvn) / (2.0 * c2)
    a5 = (dp + rho_t * c * dvn) / (2.0 * c2)
    a2 = drho - dp / c2
    dvt = dv - dvn * n                                       # tangential velocity jump

    cL, cR = sound_speed(qL), sound_speed(qR)
    vnL, vnR = (qL.v * n).sum(0), (qR.v * n).sum(0)

    def fixed(lam, lamL, lamR):
        delta = torch.clamp(torch.maximum(lam - lamL, lamR - lam), min=0.0)
        alam = lam.abs()
        use = alam < delta
        delta_safe = torch.where(use, delta, torch.ones_like(delta))
        return torch.where(use, 0.5 * (lam * lam / delta_safe + delta_safe), alam)

    l1 = fixed(vn - c, vnL - cL, vnR - cR)
    l5 = fixed(vn + c, vnL + cL, vnR + cR)
    l2 = vn.abs()

    r1 = [torch.ones_like(vn)] + [v[d] - c * n[d] for d in range(3)] + [H - c * vn]
    r5 = [torch.ones_like(vn)] + [v[d] + c * n[d] for d in range(3)] + [H + c * vn]
    r2 = [torch.ones_like(vn)] + [v[d] for d in range(3)] + [0.5 * v2]
    rt = [torch.zeros_like(vn)] + [dvt[d] for d in range(3)] + [(v * dvt).sum(0)]

    diss = torch.stack([l1 * a1 * r1[k] + l5 * a5 * r5[k] + l2 * (a2 * r2[k] + rho_t * rt[k])
                        for k in range(5)])
    F = 0.5 * (euler_flux(qL, n) + euler_flux(qR, n)) - 0.5 * diss
    return F * s


def riemann(kind: int, uL, uR, nvec, gas: Gas, vol_kind: int = 0) -> torch.Tensor:
    """Numerical flux ``F* s`` for the selector ``kind`` (0 Roe-HH, 1 LLF, 2 EC two-point)."""
    qL, qR = to_prim(uL, gas), to_prim(uR, gas)
    if kind == 0:
        if gas.nvar != 5:
            raise ValueError("the Roe solver is single-species only")
        return riemann_roe_hh(uL, uR, qL, qR, nvec, gas.gamma)
    if kind == 1:
        return riemann_llf(uL, uR, qL, qR, nvec)
    if kind == 2:
        return two_point(vol_kind, qL, qR, nvec, gas)
    raise ValueError(kind)


def entropy_vars(u: torch.Tensor, gas: Gas) -> torch.Tensor:
    """Entropy variables of the single-species Euler equations, ``U = -rho s/(gamma-1)``."""
    q = to_prim(u, gas)
    g = gas.gamma
    s = torch.log(q.p) - g * torch.log(q.rho)
    v2 = (q.v * q.v).sum(0)
    w0 = (g - s) / (g - 1.0) - 0.5 * q.rho * v2 / q.p
    return torch.stack([w0, q.rho * q.v[0] / q.p, q.rho * q.v[1] / q.p, q.rho * q.v[2] / q.p,
                        -q.rho / q.p])
