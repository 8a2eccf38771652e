"""Viscous terms of the multi-species Navier-Stokes equations with BR1 lifting (oracle).

Test infrastructure: a plain, slow reference.  Only the tests, the smoke check
and the benchmark's CPU-baseline leg use it.

Physics (Section 2, eq. ns_equation, eq. visc_stress, eq. fourier_law,
eq. enthalpy_flux, eq. fickian_law, eq. mix_lambda_mu).  With the viscous flux
written on the left-hand side, ``u_t + div F^c + div F^v = 0``, the flux in
physical direction ``x`` is

    F^v_x = -(0, tau_x1, tau_x2, tau_x3, (tau v)_x - q_h,x - q_d,x, -J_1,x)

with ``tau = mu (grad v + grad v^T - 2/3 div v I)``, ``q_h = -lambda grad T``,
``q_d = sum_j h_j J_j`` and ``J_k = -rho D_k grad Y_k + rho Y_k sum_j D_j grad Y_j``.

Discretisation (Section 3.1.1, eq. lift_weak and eq. semidiscrete_lift; the
viscous part of eq. semidiscrete; Section 3.2.2 for mixed interfaces), on
LGL nodes in the strong form, which equals the printed weak form by the
summation-by-parts property of the collocated operators:

* lifting: ``g_x = (1/J) sum_d [ sum_m D_im (Ja^d_x u)_m
  + (u* - u) Ja^d_x / w_N  at the +xi_d end  - (u* - u) Ja^d_x / w_0 at the - end ]``,
  the BR1 face value ``u* = (u^- + u^+) / 2`` (eq. lift_flux); at a degree
  jump it is formed on the lower degree (the higher side's trace projected
  down) and interpolated up to the higher side (fig. p_coupling_lift);
* viscous rate: ``R^v = -(1/J) sum_d [ sum_m D_im Ft^d_m + (F^v* - Ft^d) / w
  at the ends, with outward sign ]`` with ``Ft^d = sum_x Ja^d_x F^v_x`` and
  the face flux ``F^v* = (F^v(u^-, g^-) + F^v(u^+, g^+)) / 2 . n s``
  (eq. visc_flux), formed as the convective flux: both sides' traces of
  ``u`` and ``g`` interpolated to the higher degree of the face, the fluxes
  evaluated there with the left side's outward normal, the lower side
  receiving the projection;
* mortars (Section 3.2.3): both face terms go through the mortar's virtual
  small sides as the convective flux does.  On half (quarter) k the big
  side's traces of ``u`` (and ``g``) are interpolated with ``M_0k``; the BR1
  value is formed there as at a conforming face (on the lower of the two
  degrees, interpolated up), the small side takes it, and the big side takes
  the L2 projection of the piecewise values, ``(1/2)^s sum_k M_k0 u*_k`` for
  ``s`` split directions (``M_k0`` projects twice the half's data per split
  direction); the viscous flux is the mean of both sides' fluxes on the
  common degree with the small side's outward normal reversed, the small
  side receiving it reversed and the big side ``sum_k M_k0`` of it.

Readings where the paper is silent or garbled:

* the lifted quantity is the conservative state ``u`` (the contravariant
  solution of the lifting equation); ``grad v``, ``grad T`` and ``grad Y`` follow
  from ``g = grad u`` by the chain rule at each node;
* the correction term of Fick's law carries the sign and the range (all
  species) that give ``sum_k J_k = 0``, its stated purpose;
* species enthalpies ``h_j = c_p,j T``; mixture ``mu``, ``Pr`` and ``c_p`` from
  linear mixing in ``Y`` and ``lambda = mu c_p / Pr``; one species: ``T = p /
  (rho R)``, ``c_p = gamma R / (gamma - 1)``, so ``R`` cancels in ``q_h``;
* the lifting surface term uses the element's own contravariant vectors at
  its boundary nodes, so that a constant state lifts to zero wherever the
  discrete metric identities hold;
* FV sub-cell blending acts on the convective operator only: the viscous
  rate of every element is this DG operator, ``R = (1 - alpha) R^c_DG +
  alpha R^c_FV + R^v``.  In the blended DG storage the FV side's polynomial
  representation (``V^{FV->DG} V^{DG->FV} u = u``) is the nodal state itself,
  so the lifting flux at DG/FV faces (fig. h_coupling_lift) is the DG one.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

from . import ops1d
from .geometry import OracleMesh, apply_axis, face_slice, _t
from .physics import Gas
from .rhs import apply2, mortar_halves, split_apply, to_left, to_right

T = torch.float64


@dataclass(frozen=True)
class Transport:
    """Constant species transport coefficients (species 1 first; one species uses index 0)."""

    mu: tuple = (0.0, 0.0)
    Pr: tuple = (0.72, 0.72)
    D: tuple = (0.0, 0.0)


# ---------------------------------------------------------------------------
# physics
# ---------------------------------------------------------------------------
def _species_heat(gas: Gas):
    """(c_p, c_v) per species; one species: gas constant R[0]."""
    if gas.nvar == 5:
        cv = gas.R[0] / (gas.gamma - 1.0)
        return (gas.gamma * cv,), (cv,)
    cv = tuple(gas.R[j] / (gas.kappa[j] - 1.0) for j in range(2))
    cp = tuple(gas.kappa[j] * cv[j] for j in range(2))
    return cp, cv


def primitive_gradients(u: torch.Tensor, g: torch.Tensor, gas: Gas):
    """Velocity, temperature and mass-fraction gradients from ``u [nvar, ...]`` and ``g = grad u [3, nvar, ...]``.

    Returns ``(v [3], T, Y or None, gv [3(x), 3(i)] = d v_i / d x, gT [3], gY [3] or None)``.
    """
    rho = u[0]
    v = u[1:4] / rho
    grho = g[:, 0]
    gv = (g[:, 1:4] - v[None] * grho[:, None]) / rho
    cp, cv = _species_heat(gas)
    if gas.nvar == 6:
        Y = u[5] / rho
        gY = (g[:, 5] - Y * grho) / rho
        cvm = Y * cv[0] + (1.0 - Y) * cv[1]
        gcv = (cv[0] - cv[1]) * gY
    else:
        Y, gY = None, None
        cvm = torch.full_like(rho, cv[0])
        gcv = torch.zeros_like(g[:, 0])
    Es = u[4] / rho                                            # specific total energy
    eps = Es - 0.5 * (v * v).sum(0)                            # specific internal energy
    geps = (g[:, 4] - Es * grho) / rho - (gv * v[None]).sum(1)
    Tm = eps / cvm
    gT = (geps - Tm * gcv) / cvm
    return v, Tm, Y, gv, gT, gY


def viscous_flux(u: torch.Tensor, g: torch.Tensor, gas: Gas, tr: Transport) -> torch.Tensor:
    """``F^v_x`` for x = 1..3 as ``[3(x), nvar, ...]`` (module docstring)."""
    rho = u[0]
    v, Tm, Y, gv, gT, gY = primitive_gradients(u, g, gas)
    cp, _ = _species_heat(gas)
    if gas.nvar == 6:
        Ys = [Y, 1.0 - Y]
        gYs = [gY, -gY]
        mu = Ys[0] * tr.mu[0] + Ys[1] * tr.mu[1]
        Pr = Ys[0] * tr.Pr[0] + Ys[1] * tr.Pr[1]
        cpm = Ys[0] * cp[0] + Ys[1] * cp[1]
    else:
        mu = torch.full_like(rho, tr.mu[0])
        Pr = torch.full_like(rho, tr.Pr[0])
        cpm = torch.full_like(rho, cp[0])
    lam = mu * cpm / Pr
    div = gv[0, 0] + gv[1, 1] + gv[2, 2]
    tau = torch.stack([torch.stack([mu * (gv[x, i] + gv[i, x] - (2.0 / 3.0) * div * (1.0 if x == i else 0.0))
                                    for i in range(3)]) for x in range(3)])   # [3(x), 3(i), ...]
    qh = -lam * gT                                             # [3, ...]
    if gas.nvar == 6:
        corr = sum(tr.D[j] * gYs[j] for j in range(2))         # sum_j D_j grad Y_j
        Jk = [-rho * tr.D[k] * gYs[k] + rho * Ys[k] * corr for k in range(2)]
        qd = sum(cp[j] * Tm * Jk[j] for j in range(2))
    else:
        Jk, qd = None, torch.zeros_like(qh)
    out = []
    for x in range(3):
        comps = [torch.zeros_like(rho), -tau[x, 0], -tau[x, 1], -tau[x, 2],
                 -(tau[x] * v).sum(0) + qh[x] + qd[x]]
        if gas.nvar == 6:
            comps.append(Jk[0][x])
        out.append(torch.stack(comps))
    return torch.stack(out)


def species_fluxes(u: torch.Tensor, g: torch.Tensor, gas: Gas, tr: Transport):
    """The diffusion fluxes ``J_1, J_2`` of both species, ``[3, ...]`` each (two species)."""
    rho = u[0]
    _, _, Y, _, _, gY = primitive_gradients(u, g, gas)
    Ys, gYs = [Y, 1.0 - Y], [gY, -gY]
    corr = sum(tr.D[j] * gYs[j] for j in range(2))
    return [-rho * tr.D[k] * gYs[k] + rho * Ys[k] * corr for k in range(2)]


# ---------------------------------------------------------------------------
# discretisation
# ---------------------------------------------------------------------------
def _add_on_side(L: torch.Tensor, side: int, val: torch.Tensor) -> None:
    """``L[..., k, j, i]`` += ``val[..., q, p]`` on the nodes of ``side``."""
    d, last = side // 2, side % 2
    idx = -1 if last else 0
    if d == 0:
        L[..., :, :, idx] += val
    elif d == 1:
        L[..., :, idx, :] += val
    else:
        L[..., idx, :, :] += val


def _face_groups(mesh: OracleMesh):
    faces = mesh.faces
    deg = mesh.degree
    keys = np.stack([deg[faces[:, 0]], deg[faces[:, 2]], faces[:, 1], faces[:, 3], faces[:, 4]], axis=1)
    uniq, inv = np.unique(keys, axis=0, return_inverse=True)
    inv = inv.reshape(-1)
    for gi, key in enumerate(uniq.tolist()):
        fsel = np.nonzero(inv == gi)[0]
        yield key, faces[fsel, 0], faces[fsel, 2]


def lift_face_values(mesh: OracleMesh, U: dict) -> dict:
    """BR1 face values ``u*`` per element side at the element's degree: ``{N: [[E][6] -> [nvar, n, n]]}``."""
    out = {N: [[None] * 6 for _ in range(len(g.elems))] for N, g in mesh.groups.items()}
    for (NL, NR, sL, sR, o), eL, eR in _face_groups(mesh):
        slL = torch.as_tensor(mesh.slot[eL], dtype=torch.long)
        slR = torch.as_tensor(mesh.slot[eR], dtype=torch.long)
        tL = face_slice(U[NL][slL], sL)                        # [F, nvar, nL, nL]
        tR = to_left(face_slice(U[NR][slR], sR), o)            # on the left grid
        lo = min(NL, NR)
        if NL > lo:
            tL = apply2(_t(ops1d.project(NL, lo)), tL)
        if NR > lo:
            tR = apply2(_t(ops1d.project(NR, lo)), tR)
        us = 0.5 * (tL + tR)                                   # at the lower degree
        usL = apply2(_t(ops1d.interp(lo, NL)), us) if NL > lo else us
        usR = apply2(_t(ops1d.interp(lo, NR)), us) if NR > lo else us
        usR = to_right(usR, o)
        for r, (a, b) in enumerate(zip(slL.tolist(), slR.tolist())):
            out[NL][a][sL] = usL[r]
            out[NR][b][sR] = usR[r]
    if len(mesh.mortars):
        _mortar_lift_values(mesh, U, out)
    return out


def _mortar_lift_values(mesh: OracleMesh, U: dict, out: dict) -> None:
    """BR1 values of the mortar sides into ``out`` (module docstring, mortars)."""
    deg = mesh.degree
    for row in mesh.mortars.tolist():
        e0, s0 = row[0], row[1]
        N0 = int(deg[e0])
        sl0 = int(mesh.slot[e0])
        u0 = face_slice(U[N0][sl0:sl0 + 1], s0)[0]            # [nvar, n0, n0], big side's grid
        big = torch.zeros_like(u0)
        for ek, sk, ok, kp, kq in mortar_halves(row):
            Nk = int(deg[ek])
            slk = int(mesh.slot[ek])
            uv = split_apply(lambda k: ops1d.mortar_interp(N0, k), u0, kp, kq)
            tk = to_left(face_slice(U[Nk][slk:slk + 1], sk), ok)[0]
            lo = min(N0, Nk)
            a = apply2(_t(ops1d.project(N0, lo)), uv) if N0 > lo else uv
            b = apply2(_t(ops1d.project(Nk, lo)), tk) if Nk > lo else tk
            us = 0.5 * (a + b)
            usk = apply2(_t(ops1d.interp(lo, Nk)), us) if Nk > lo else us
            out[Nk][slk][sk] = to_right(usk[None], ok)[0]
            us0 = apply2(_t(ops1d.interp(lo, N0)), us) if N0 > lo else us
            share = 0.5 ** ((kp is not None) + (kq is not None))
            big = big + share * split_apply(lambda k: ops1d.mortar_project(N0, k), us0, kp, kq)
        out[N0][sl0][s0] = big


def lift(mesh: OracleMesh, u: torch.Tensor) -> torch.Tensor:
    """Lifted gradient ``g = grad u`` at every node, flat ``[3, nvar, n_node]``."""
    nvar = u.shape[0]
    U = {N: mesh.gather(u, N) for N in mesh.groups}
    ustar = lift_face_values(mesh, U)
    parts = {}
    for N, g in mesh.groups.items():
        E = len(g.elems)
        w_end = float(g.w[0])
        G = torch.zeros(E, 3, nvar, N + 1, N + 1, N + 1, dtype=T)
        for d in range(3):
            for x in range(3):
                Ut = g.Ja[:, d, x][:, None] * U[N]             # (Ja^d_x u), [E, nvar, n, n, n]
                G[:, x] += apply_axis(g.D, Ut, d)
        for s in range(6):
            d = s // 2
            sign = 1.0 if s % 2 else -1.0
            us = torch.stack([ustar[N][e][s] for e in range(E)])    # [E, nvar, n, n]
            jump = us - face_slice(U[N], s)
            for x in range(3):
                nx = face_slice(g.Ja[:, d, x], s)[:, None]     # [E, 1, n, n]
                _add_on_side(G[:, x], s, sign * nx * jump / w_end)
        parts[N] = (G / g.J[:, None, None]).reshape(E, 3 * nvar, N + 1, N + 1, N + 1)
    return mesh.scatter(parts, 3 * nvar).reshape(3, nvar, -1)


def viscous_rhs(mesh: OracleMesh, gas: Gas, tr: Transport, u: torch.Tensor,
                g: torch.Tensor | None = None) -> torch.Tensor:
    """Viscous rate ``R^v`` at every node, flat ``[nvar, n_node]`` (``g`` lifted here when not given)."""
    nvar = u.shape[0]
    if g is None:
        g = lift(mesh, u)
    U = {N: mesh.gather(u, N) for N in mesh.groups}
    Gd = {N: mesh.gather(g.reshape(3 * nvar, -1), N) for N in mesh.groups}   # [E, 3 nvar, n, n, n]
    Fv = {}
    for N, grp in mesh.groups.items():
        E = len(grp.elems)
        Uv = U[N].transpose(0, 1)                              # [nvar, E, ...]
        Gv = Gd[N].reshape(E, 3, nvar, N + 1, N + 1, N + 1).permute(1, 2, 0, 3, 4, 5)
        Fv[N] = viscous_flux(Uv, Gv, gas, tr).transpose(1, 2)  # [3(x), E, nvar, n, n, n]

    side = {N: [[None] * 6 for _ in range(len(g_.elems))] for N, g_ in mesh.groups.items()}
    G5 = {N: Gd[N].reshape(len(grp.elems), 3, nvar, N + 1, N + 1, N + 1) for N, grp in mesh.groups.items()}
    for (NL, NR, sL, sR, o), eL, eR in _face_groups(mesh):
        slL = torch.as_tensor(mesh.slot[eL], dtype=torch.long)
        slR = torch.as_tensor(mesh.slot[eR], dtype=torch.long)
        uL = face_slice(U[NL][slL], sL)                        # [F, nvar, n, n]
        uR = to_left(face_slice(U[NR][slR], sR), o)
        gL = face_slice(G5[NL][slL], sL)                       # [F, 3, nvar, n, n]
        gR = to_left(face_slice(G5[NR][slR], sR), o)
        nvec = mesh.groups[NL].outward_normal(sL)[slL]         # [F, 3, nL, nL]
        M = max(NL, NR)
        # as for the convective flux: both sides' traces (state and gradient)
        # on degree M, the fluxes evaluated there
        if NL < M:
            VL = _t(ops1d.interp(NL, M))
            uL, gL, nvec = apply2(VL, uL), apply2(VL, gL), apply2(VL, nvec)
        if NR < M:
            VR = _t(ops1d.interp(NR, M))
            uR, gR = apply2(VR, uR), apply2(VR, gR)
        fL = viscous_flux(uL.transpose(0, 1), gL.permute(1, 2, 0, 3, 4), gas, tr)   # [3, nvar, F, M+1, M+1]
        fR = viscous_flux(uR.transpose(0, 1), gR.permute(1, 2, 0, 3, 4), gas, tr)
        Fs = sum(0.5 * (fL[x] + fR[x]) * nvec[:, x] for x in range(3)).transpose(0, 1)   # [F, nvar, M+1, M+1]
        FL = apply2(_t(ops1d.project(M, NL)), Fs) if NL < M else Fs
        FR = apply2(_t(ops1d.project(M, NR)), Fs) if NR < M else Fs
        FR = -to_right(FR, o)
        for r, (a, b) in enumerate(zip(slL.tolist(), slR.tolist())):
            side[NL][a][sL] = FL[r]
            side[NR][b][sR] = FR[r]
    if len(mesh.mortars):
        _mortar_viscous_fluxes(mesh, gas, tr, U, G5, side)

    parts = {}
    for N, grp in mesh.groups.items():
        E = len(grp.elems)
        w_end = float(grp.w[0])
        acc = torch.zeros(E, nvar, N + 1, N + 1, N + 1, dtype=T)
        for d in range(3):
            Ft = sum(grp.Ja[:, d, x][:, None] * Fv[N][x] for x in range(3))   # contravariant, [E, nvar, ...]
            acc += apply_axis(grp.D, Ft, d)
            for s in (2 * d, 2 * d + 1):
                sign = 1.0 if s % 2 else -1.0
                Fs = torch.stack([side[N][e][s] for e in range(E)])
                _add_on_side(acc, s, (Fs - sign * face_slice(Ft, s)) / w_end)
        parts[N] = -acc / grp.J[:, None]
    return mesh.scatter(parts, nvar)


def _mortar_viscous_fluxes(mesh: OracleMesh, gas: Gas, tr: Transport, U: dict, G5: dict, side: dict) -> None:
    """Outward viscous fluxes of the mortar sides into ``side`` (module docstring, mortars)."""
    deg = mesh.degree

    def flux_n(uu, gg, nvec):                                  # F^v(u, g) . n on a face grid
        f = viscous_flux(uu, gg, gas, tr)                      # [3, nvar, n, n]
        return sum(f[x] * nvec[x] for x in range(3))

    for row in mesh.mortars.tolist():
        e0, s0 = row[0], row[1]
        N0 = int(deg[e0])
        sl0 = int(mesh.slot[e0])
        u0 = face_slice(U[N0][sl0:sl0 + 1], s0)[0]            # [nvar, n0, n0]
        g0 = face_slice(G5[N0][sl0:sl0 + 1], s0)[0]           # [3, nvar, n0, n0]
        big = torch.zeros_like(u0)
        for ek, sk, ok, kp, kq in mortar_halves(row):
            Nk = int(deg[ek])
            slk = int(mesh.slot[ek])
            uv = split_apply(lambda k: ops1d.mortar_interp(N0, k), u0, kp, kq)
            gv = split_apply(lambda k: ops1d.mortar_interp(N0, k), g0, kp, kq)
            tk = to_left(face_slice(U[Nk][slk:slk + 1], sk), ok)[0]
            gk = to_left(face_slice(G5[Nk][slk:slk + 1], sk), ok)[0]
            nk = -to_left(mesh.groups[Nk].outward_normal(sk)[slk:slk + 1], ok)[0]
            M = max(N0, Nk)
            if N0 < M:
                V0 = _t(ops1d.interp(N0, M))
                uv, gv = apply2(V0, uv), apply2(V0, gv)
            if Nk < M:
                Vk = _t(ops1d.interp(Nk, M))
                tk, gk, nk = apply2(Vk, tk), apply2(Vk, gk), apply2(Vk, nk)
            F = 0.5 * (flux_n(uv, gv, nk) + flux_n(tk, gk, nk))   # [nvar, M+1, M+1], out of the big side
            Fk = apply2(_t(ops1d.project(M, Nk)), F) if Nk < M else F
            side[Nk][slk][sk] = -to_right(Fk[None], ok)[0]
            Fb = apply2(_t(ops1d.project(M, N0)), F) if N0 < M else F
            big = big + split_apply(lambda k: ops1d.mortar_project(N0, k), Fb, kp, kq)
        side[N0][sl0][s0] = big


class ViscousRhs:
    """``R(u, alpha) = R^c(u, alpha) + R^v(u)`` (module docstring, last reading)."""

    def __init__(self, convective, mesh: OracleMesh, gas: Gas, tr: Transport):
        self.convective = convective
        self.mesh, self.gas, self.tr = mesh, gas, tr

    def __call__(self, u: torch.Tensor, alpha) -> torch.Tensor:
        return self.convective(u, alpha) + viscous_rhs(self.mesh, self.gas, self.tr, u)
