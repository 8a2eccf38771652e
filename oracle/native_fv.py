"""FV-stored elements with a second-order minmod reconstruction (oracle).

Test infrastructure: a plain, slow reference.  Only the tests, the smoke check
and the benchmark's CPU-baseline leg use it.

Section 3.1.2 evolves, on an FV element, the integral means of N_FV^3
equidistant reference sub-cells (eq. semidiscrete_fv): the rate of a mean is
minus the sum of its six sub-face fluxes ``F* s`` over the sub-cell's volume
ratio, and the fluxes see a second-order TVD reconstruction limited with
minmod (after Sonntag and Munz).  Section 3.2 switches elements between the
two representations with ``V^{DG->FV}`` (sub-cell integration) and its
pseudo-inverse ``V^{FV->DG}``, and couples FV and DG elements at their faces
through the DG side's sub-face means (fig. h_coupling).

The state is a pair: the nodal DG state ``u[nvar, n_node]`` (used on DG
elements) and the sub-cell means ``ufv[K, nvar, s3, s2, s1]`` (used on FV
elements, ``s1`` fastest), with ``flag[K]`` true on FV elements.

Readings where the paper is silent:

* the sub-cell means are J-weighted, ``ubar = V3(J u) / V3(J)``, and the rate
  is ``d ubar / dt = -(sum of outward sub-face fluxes) / (h^3 Jbar)`` with
  ``Jbar = V3(J)``, so that ``h^3 Jbar ubar`` is the sub-cell's content;
* the reconstruction acts on the primitive variables (rho, v, p[, Y1]), cell
  by cell along each reference direction, in reference index space (the
  sub-cells are equidistant there): slope ``sigma_c = minmod(w_c - w_{c-1},
  w_{c+1} - w_c)``, face values ``w_c +- sigma_c / 2``;
* across an element face the neighbour of a boundary sub-cell (its ghost) is
  the adjacent sub-cell mean of an FV neighbour, or the DG neighbour's nodal
  trace mapped to the sub-face grid with ``V^{DG->FV}`` in both face
  directions;
* a DG side's value on a face with an FV side is that mapped trace, unlimited
  and first order (fig. h_coupling); the one sub-face flux serves the FV
  side directly and the DG side through ``V^{FV->DG} / h^2`` (as for blended
  elements);
* sub-face normals are ``h^2`` times the mean of ``Ja^d`` over the sub-face
  (the same as for blended elements);
* mortars (Section 3.2.3): where neither side is FV the DG mortar flux; else
  the FV variant on each small side's sub-face grid, as for blended
  elements, with the reconstruction above: an FV small side reconstructs
  from its boundary and next layers with the big side's data on its half as
  ghost (the big side's boundary means through ``M^FV_0k``, or a DG big
  side's half trace through ``V^{DG->FV}``); an FV big side's ghost on each
  of its sub-faces is the mean of the small sides' boundary data over it,
  ``(1/2)^s sum_k M^FV_k0 c_k``, and its reconstructed face values reach the
  halves through ``M^FV_0k``; the small side takes the flux reversed, the big
  side ``sum_k M^FV_k0`` of it (FV) or ``sum_k M_k0`` of its ``V^{FV->DG} /
  h^2`` (DG);
* switching: DG -> FV ``ubar = V3(J u) / V3(J)``; FV -> DG
  ``u = V3^+(ubar V3(J)) / J``, the least-squares DG state whose J-weighted
  sub-cell contents are those of ``ubar`` (exactly them for ``N_FV = N + 1``).
"""
from __future__ import annotations

import numpy as np
import torch

from . import ops1d
from .geometry import OracleMesh, apply3, apply_axis, face_slice, _t
from .physics import Gas, prim_to_cons, riemann, to_prim
from .rhs import Params, Rhs, apply2, mortar_halves, split_apply, to_left, to_right, volume_term

T = torch.float64


def minmod(a: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
    """``sign(a) min(|a|, |b|)`` where ``a`` and ``b`` have one sign, else 0."""
    return torch.where(a * b > 0, torch.sign(a) * torch.minimum(a.abs(), b.abs()), torch.zeros_like(a))


def to_w(u: torch.Tensor, gas: Gas) -> torch.Tensor:
    """Conservative ``[nvar, ...]`` -> primitive (rho, v1, v2, v3, p[, Y1])."""
    q = to_prim(u, gas)
    comps = [q.rho, q.v[0], q.v[1], q.v[2], q.p]
    if gas.nvar == 6:
        comps.append(q.Y)
    return torch.stack(comps)


def layer(f: torch.Tensor, side: int, depth: int) -> torch.Tensor:
    """Sub-cell layer ``depth`` (0 = at the side) of ``f[..., s3, s2, s1]``, as ``[..., q, p]``."""
    d, last = side // 2, side % 2
    idx = -1 - depth if last else depth
    if d == 0:
        return f[..., :, :, idx]
    if d == 1:
        return f[..., :, idx, :]
    return f[..., idx, :, :]


def face_value(wb: torch.Tensor, wi: torch.Tensor, wg: torch.Tensor) -> torch.Tensor:
    """Reconstructed value at the face of a boundary sub-cell (primitives).

    ``wb`` the boundary cell, ``wi`` the next one inwards, ``wg`` the ghost
    across the face: ``wb + minmod(wb - wi, wg - wb) / 2``.
    """
    return wb + 0.5 * minmod(wb - wi, wg - wb)


class NativeRhs:
    """Rates of the pair (DG nodal state, FV sub-cell means) on one mesh."""

    def __init__(self, mesh: OracleMesh, gas: Gas, params: Params):
        self.mesh = mesh
        self.gas = gas
        self.params = params
        self.h = 2.0 / mesh.n_fv

    # ---- geometry of the sub-cells ---------------------------------------
    def jbar(self, N: int) -> torch.Tensor:
        """``V3(J)``, the sub-cell means of J, for the degree-N group ``[E, s3, s2, s1]``."""
        g = self.mesh.groups[N]
        return apply3(_t(ops1d.dg2fv(N, self.mesh.n_fv)), g.J)

    def internal_normals(self, N: int, d: int) -> torch.Tensor:
        """``h^2`` x mean of ``Ja^d`` over every sub-cell face normal to ``xi_d``.

        ``[E, 3, ...]`` with ``N_FV + 1`` planes along axis d (the outer two
        are the element's sides).
        """
        g = self.mesh.groups[N]
        V = _t(ops1d.dg2fv(N, self.mesh.n_fv))
        If = _t(ops1d.face_interp(N, self.mesh.n_fv))
        nd = g.Ja[:, d]
        for ax in range(3):
            nd = apply_axis(If if ax == d else V, nd, ax)
        return nd * (self.h * self.h)

    # ---- the rates -------------------------------------------------------
    def __call__(self, u: torch.Tensor, ufv: torch.Tensor, flag):
        """``(R, Rfv)``: nodal rates of the DG elements (0 on FV elements) and the
        rates of the FV elements' means (0 on DG elements)."""
        m, gas, prm = self.mesh, self.gas, self.params
        nvar = gas.nvar
        NFV, h = m.n_fv, self.h
        flag = np.asarray(flag, dtype=bool)
        U = {N: m.gather(u, N) for N in m.groups}

        Fdg = [[None] * 6 for _ in range(m.K)]        # DG surface flux per side, at the element degree
        Ffv = [[None] * 6 for _ in range(m.K)]        # FV side fluxes on the sub-face grid
        ghost = [[None] * 6 for _ in range(m.K)]      # FV elements: conservative ghost layer per side

        def nodal_trace(e, s):
            N = int(m.degree[e])
            return face_slice(U[N][m.slot[e]], s)                  # [nvar, q, p]

        def dg_face_means(e, s):
            N = int(m.degree[e])
            return apply2(_t(ops1d.dg2fv(N, NFV)), nodal_trace(e, s))

        for f in range(len(m.faces)):
            eL, sL, eR, sR, o = (int(x) for x in m.faces[f])
            NL, NR = int(m.degree[eL]), int(m.degree[eR])
            gL = m.groups[NL]
            nvec = gL.outward_normal(sL)[m.slot[eL]]                # [3, nL, nL] left grid
            if not flag[eL] and not flag[eR]:
                # both DG: common degree, Riemann flux, projection back (fig. p_coupling)
                M = max(NL, NR)
                tL = nodal_trace(eL, sL)
                tR = to_left(nodal_trace(eR, sR), o)
                if NL < M:
                    VL = _t(ops1d.interp(NL, M))
                    tL, nvec = apply2(VL, tL), apply2(VL, nvec)
                if NR < M:
                    tR = apply2(_t(ops1d.interp(NR, M)), tR)
                Fs = riemann(prm.face_flux_dg, tL, tR, nvec, gas, prm.volume_flux)
                FL = apply2(_t(ops1d.project(M, NL)), Fs) if NL < M else Fs
                FR = apply2(_t(ops1d.project(M, NR)), Fs) if NR < M else Fs
                Fdg[eL][sL] = FL
                Fdg[eR][sR] = -to_right(FR, o)
                continue
            # a face with an FV side: one flux per sub-face (fig. h_coupling)
            cL = layer(ufv[eL], sL, 0) if flag[eL] else dg_face_means(eL, sL)      # left grid
            cR = layer(ufv[eR], sR, 0) if flag[eR] else dg_face_means(eR, sR)      # right grid
            gL_ = to_left(cR, o)             # the left side's ghost, on the left grid
            gR_ = to_right(cL, o)            # the right side's ghost, on the right grid
            if flag[eL]:
                wL = face_value(to_w(cL, gas), to_w(layer(ufv[eL], sL, 1), gas), to_w(gL_, gas))
                vL = prim_to_cons(wL, gas)
                ghost[eL][sL] = gL_
            else:
                vL = cL
            if flag[eR]:
                wR = face_value(to_w(cR, gas), to_w(layer(ufv[eR], sR, 1), gas), to_w(gR_, gas))
                vR = to_left(prim_to_cons(wR, gas), o)
                ghost[eR][sR] = gR_
            else:
                vR = to_left(cR, o)
            nsub = h * h * apply2(_t(ops1d.dg2fv(NL, NFV)), nvec)
            Fs = riemann(prm.face_flux_fv, vL, vR, nsub, gas, prm.volume_flux)     # [nvar, NFV, NFV]
            if flag[eL]:
                Ffv[eL][sL] = Fs
            else:
                Fdg[eL][sL] = apply2(_t(ops1d.fv2dg(NL, NFV)), Fs) / (h * h)
            if flag[eR]:
                Ffv[eR][sR] = -to_right(Fs, o)
            else:
                Fdg[eR][sR] = -to_right(apply2(_t(ops1d.fv2dg(NR, NFV)), Fs) / (h * h), o)

        if len(m.mortars):
            self._mortars(U, ufv, flag, Fdg, Ffv, ghost)

        R = {}
        Rfv = torch.zeros_like(ufv)
        for N, g in m.groups.items():
            elems = g.elems.numpy()
            n = N + 1
            E = len(elems)
            dg = np.nonzero(~flag[elems])[0]
            RN = torch.zeros(E, nvar, n, n, n, dtype=T)
            if len(dg):
                sl = torch.as_tensor(dg, dtype=torch.long)
                vol = volume_term(U[N][sl], g.Ja[sl], g.D, gas, prm.volume_flux)
                side = [torch.stack([Fdg[int(elems[s])][sd] for s in dg]) for sd in range(6)]
                lift = Rhs._lift(side, len(dg), nvar, n, g.w[0])
                RN[sl] = -(vol + lift) / g.J[sl][:, None]
            R[N] = RN
            fv = np.nonzero(flag[elems])[0]
            if len(fv):
                jb = self.jbar(N)
                nrm = [self.internal_normals(N, d) for d in range(3)]
                for s in fv.tolist():
                    e = int(elems[s])
                    Rfv[e] = self._fv_rate(ufv[e], [ghost[e][sd] for sd in range(6)],
                                           [Ffv[e][sd] for sd in range(6)], [nd[s] for nd in nrm], jb[s])
        return m.scatter(R, nvar), Rfv

    def _mortars(self, U, ufv, flag, Fdg, Ffv, ghost):
        """Side fluxes (and the FV sides' ghost layers) of the mortars (module docstring, mortars)."""
        m, gas, prm = self.mesh, self.gas, self.params
        NFV, h2 = m.n_fv, self.h * self.h
        deg = m.degree
        for row in m.mortars.tolist():
            e0, s0 = row[0], row[1]
            N0 = int(deg[e0])
            t0 = face_slice(U[N0][m.slot[e0]], s0)                 # [nvar, n0, n0], the big side's grid
            share = 0.5 ** (1 + (row[2] == 3))
            small = []
            for ek, sk, ok, kp, kq in mortar_halves(row):
                Nk = int(deg[ek])
                tk = to_left(face_slice(U[Nk][m.slot[ek]], sk), ok)
                nk = -to_left(m.groups[Nk].outward_normal(sk)[m.slot[ek]], ok)
                ck = to_left(layer(ufv[ek], sk, 0), ok) if flag[ek] else apply2(_t(ops1d.dg2fv(Nk, NFV)), tk)
                small.append((ek, sk, ok, kp, kq, Nk, tk, nk, ck))
            if flag[e0]:
                g0 = sum(share * split_apply(lambda k: ops1d.mortar_fv_project(NFV, k), c[8], c[3], c[4])
                         for c in small)                         # the big side's ghost, its own grid
                ghost[e0][s0] = g0
                vb = prim_to_cons(face_value(to_w(layer(ufv[e0], s0, 0), gas), to_w(layer(ufv[e0], s0, 1), gas),
                                             to_w(g0, gas)), gas)
                Fbig = torch.zeros(gas.nvar, NFV, NFV, dtype=T)
            else:
                Fbig = torch.zeros_like(t0)
            for ek, sk, ok, kp, kq, Nk, tk, nk, ck in small:
                uv = split_apply(lambda k: ops1d.mortar_interp(N0, k), t0, kp, kq)
                if not flag[e0] and not flag[ek]:                 # the DG mortar flux
                    M = max(N0, Nk)
                    if N0 < M:
                        uv = apply2(_t(ops1d.interp(N0, M)), uv)
                    if Nk < M:
                        Vk = _t(ops1d.interp(Nk, M))
                        tk, nk = apply2(Vk, tk), apply2(Vk, nk)
                    F = riemann(prm.face_flux_dg, uv, tk, nk, gas, prm.volume_flux)
                    Fs = apply2(_t(ops1d.project(M, Nk)), F) if Nk < M else F
                    Fdg[ek][sk] = -to_right(Fs[None], ok)[0]
                    Fb = apply2(_t(ops1d.project(M, N0)), F) if N0 < M else F
                    Fbig = Fbig + split_apply(lambda k: ops1d.mortar_project(N0, k), Fb, kp, kq)
                    continue
                if flag[e0]:
                    vb_k = split_apply(lambda k: ops1d.mortar_fv_interp(NFV, k), vb, kp, kq)
                else:
                    vb_k = apply2(_t(ops1d.dg2fv(N0, NFV)), uv)
                if flag[ek]:
                    cg = split_apply(lambda k: ops1d.mortar_fv_interp(NFV, k), layer(ufv[e0], s0, 0), kp, kq) \
                        if flag[e0] else vb_k
                    ghost[ek][sk] = to_right(cg[None], ok)[0]
                    vs = prim_to_cons(face_value(to_w(ck, gas), to_w(to_left(layer(ufv[ek], sk, 1), ok), gas),
                                                 to_w(cg, gas)), gas)
                else:
                    vs = ck
                Fs = riemann(prm.face_flux_fv, vb_k, vs, h2 * apply2(_t(ops1d.dg2fv(Nk, NFV)), nk), gas,
                             prm.volume_flux)                      # [nvar, NFV, NFV] on the half's grid
                if flag[ek]:
                    Ffv[ek][sk] = -to_right(Fs[None], ok)[0]
                else:
                    Fdg[ek][sk] = -to_right((apply2(_t(ops1d.fv2dg(Nk, NFV)), Fs) / h2)[None], ok)[0]
                if flag[e0]:
                    Fbig = Fbig + split_apply(lambda k: ops1d.mortar_fv_project(NFV, k), Fs, kp, kq)
                else:
                    Fbig = Fbig + split_apply(lambda k: ops1d.mortar_project(N0, k),
                                              apply2(_t(ops1d.fv2dg(N0, NFV)), Fs) / h2, kp, kq)
            if flag[e0]:
                Ffv[e0][s0] = Fbig
            else:
                Fdg[e0][s0] = Fbig

    def _fv_rate(self, ub, ghosts, sides, nrm, jb):
        """Rate of one FV element's means (eq. semidiscrete_fv with the minmod reconstruction)."""
        gas, prm, h = self.gas, self.params, self.h
        w = to_w(ub, gas)                                        # [nvar, s3, s2, s1]
        dC = torch.zeros_like(ub)
        for d in range(3):
            dim = ub.dim() - 1 - d
            wm = torch.movedim(w, dim, -1)                      # [nvar, a, b, NFV]
            lo = to_w(ghosts[2 * d], gas)[..., None]            # [nvar, a, b, 1]
            hi = to_w(ghosts[2 * d + 1], gas)[..., None]
            ext = torch.cat([lo, wm, hi], dim=-1)               # ghosts at both ends
            sigma = minmod(ext[..., 1:-1] - ext[..., :-2], ext[..., 2:] - ext[..., 1:-1])
            wl = (wm + 0.5 * sigma)[..., :-1]                   # left state of internal face c + 1/2
            wr = (wm - 0.5 * sigma)[..., 1:]                    # right state
            ndm = torch.movedim(nrm[d], dim, -1)                # [3, a, b, NFV + 1]
            Fi = riemann(prm.face_flux_fv, prim_to_cons(wl, gas), prim_to_cons(wr, gas), ndm[..., 1:-1], gas,
                         prm.volume_flux)                        # [nvar, a, b, NFV - 1]
            G = torch.cat([-sides[2 * d][..., None], Fi, sides[2 * d + 1][..., None]], dim=-1)
            dC = dC - torch.movedim(G[..., 1:] - G[..., :-1], -1, dim)
        return dC / (h ** 3 * jb[None])


# ---- switching between the representations (Section 3.2) ------------------
def dg_to_fv(mesh: OracleMesh, u: torch.Tensor, elems) -> torch.Tensor:
    """J-weighted sub-cell means ``V3(J u) / V3(J)`` of elements ``elems``: ``[len, nvar, s3, s2, s1]``."""
    out = []
    for e in np.asarray(elems, dtype=np.int64).tolist():
        N = int(mesh.degree[e])
        g = mesh.groups[N]
        V = _t(ops1d.dg2fv(N, mesh.n_fv))
        J = g.J[mesh.slot[e]]
        Ue = mesh.gather(u, N)[mesh.slot[e]]
        out.append(apply3(V, J[None] * Ue) / apply3(V, J)[None])
    return torch.stack(out) if out else torch.zeros(0)


def fv_to_dg(mesh: OracleMesh, ufv: torch.Tensor, elems) -> dict:
    """Nodal states ``V3^+(ubar V3(J)) / J`` of elements ``elems``: ``{e: [nvar, n, n, n]}``."""
    out = {}
    for e in np.asarray(elems, dtype=np.int64).tolist():
        N = int(mesh.degree[e])
        g = mesh.groups[N]
        V = _t(ops1d.dg2fv(N, mesh.n_fv))
        Vp = _t(ops1d.fv2dg(N, mesh.n_fv))
        J = g.J[mesh.slot[e]]
        out[e] = apply3(Vp, ufv[e] * apply3(V, J)[None]) / J[None]
    return out


def switch(mesh: OracleMesh, u: torch.Tensor, ufv: torch.Tensor, flag_old, flag_new):
    """Convert the elements whose flag changes; returns the new ``(u, ufv)``."""
    flag_old = np.asarray(flag_old, dtype=bool)
    flag_new = np.asarray(flag_new, dtype=bool)
    u = u.clone()
    ufv = ufv.clone()
    to_fv = np.nonzero(~flag_old & flag_new)[0]
    to_dg = np.nonzero(flag_old & ~flag_new)[0]
    if len(to_fv):
        ufv[torch.as_tensor(to_fv)] = dg_to_fv(mesh, u, to_fv)
    for e, ue in fv_to_dg(mesh, ufv, to_dg).items():
        a, b = int(mesh.offset[e]), int(mesh.offset[e + 1])
        u[:, a:b] = ue.reshape(ue.shape[0], -1)
    return u, ufv


def stage(fn, u, ufv, k, kfv, s: int, dt: float, A, B):
    """One 2N stage of the pair: ``k <- A_s k + dt R``, ``u <- u + B_s k`` on both parts."""
    R, Rfv = fn(u, ufv)
    k = dt * R if s == 0 else A[s] * k + dt * R
    kfv = dt * Rfv if s == 0 else A[s] * kfv + dt * Rfv
    return u + B[s] * k, ufv + B[s] * kfv, k, kfv
