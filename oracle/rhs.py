"""Right-hand side of the hybrid DG/FV semi-discretisation (oracle).

Test infrastructure: a plain, slow reference.  Only the tests, the smoke check
and the benchmark's CPU-baseline leg use it.

For every element ``e`` with degree ``N_e`` and blending factor ``alpha_e``:

    R_e = (1 - alpha_e) R^DG_e + alpha_e R^FV_e

DG part (eq. semidiscrete in the split form of Section 3.5, LGL nodes):

    R^DG_ijk = -1/J_ijk [ sum_{m != i} 2 D_im F#1(ijk, mjk) + sum_{n != j} 2 D_jn F#2
                          + sum_{o != k} 2 D_ko F#3 + sum_sides delta F*_out / w_0 ]

with ``F#d(a, b) = f#(u_a, u_b) . (Ja^d_a + Ja^d_b)/2``.  The boundary-node
terms of the strong split form cancel against ``2 D_00 = -1/w_0`` and
``2 D_NN = 1/w_N``, which leaves only the outward numerical flux divided by
the end weight (the surface lift with ``l_hat(+-1)``).

Interfaces (Section 3.2.1):
* both sides DG (``alpha = 0``): traces are brought to the common degree
  ``M = max(N_L, N_R)`` with ``V^{N->M}``, the Riemann flux is evaluated on the
  ``M`` nodes with the left side's normal, and each side receives the modal
  projection ``V^{M->N}`` of it;
* otherwise (an FV face): traces are sub-face means on the ``N_FV^2`` grid,
  taken from the sub-cell means of a blended side or from ``V^{DG->FV}`` of a
  DG side's nodal trace; one Riemann flux per sub-face serves the FV operators
  of blended sides directly and the DG surface terms of both sides through
  ``V^{FV->DG}``.

Non-conforming faces (Section 3.2.3, mortar types 1-3, DG sides): see
``Rhs._mortar_fluxes``; the big side's flux is the sum over its halves or
quarters of ``M_{k0}`` applied to their fluxes (``ops1d.mortar_project``).
Readings: the small side's own normal (reversed) carries the flux, so the
big side's share needs no surface-element factor (``M_{k0}`` is the L2
projection of twice the half's flux per direction of the split); the FV
variants (a blended side at a mortar) take the flux on the small side's
sub-face grid, with ``M^FV_{0k}`` and ``M^FV_{k0}`` the overlap maps between
the big side's sub-faces and those of its halves.

FV part (eq. semidiscrete_fv, first order): sub-cell contents
``C = h^3 V3(J u)`` and volumes ``h^3 V3(J)`` give the means
``ubar = C / vol``; each sub-cell face carries a Riemann flux with normal
``h^2 x (mean of Ja^d over the sub-face)``; ``dC/dt = -(sum of outward
fluxes)`` and the nodal rate is ``R^FV = V3^+(dC/dt) / (h^3 J)``.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

from . import ops1d
from .geometry import OracleMesh, apply_axis, apply3, face_slice, _t
from .physics import Gas, riemann, to_prim, two_point

T = torch.float64


@dataclass(frozen=True)
class Params:
    volume_flux: int = 0          # 0 Ranocha EC, 1 Pirozzoli KEP, 2 central
    face_flux_dg: int = 0         # 0 Roe-HH, 1 LLF, 2 EC two-point (the volume flux)
    face_flux_fv: int = 1


def _vars_first(U: torch.Tensor) -> torch.Tensor:
    """[E, nvar, ...] -> [nvar, E, ...]."""
    return U.transpose(0, 1)


def volume_term(U: torch.Tensor, Ja: torch.Tensor, D: torch.Tensor, gas: Gas, kind: int,
                chunk: int | None = None) -> torch.Tensor:
    """``sum_d sum_{m != i} 2 D_im F#d(i, m)`` for a degree group, ``[E, nvar, n, n, n]``."""
    E, nvar, n = U.shape[0], U.shape[1], U.shape[2]
    if chunk is None:
        chunk = max(1, (1 << 19) // n ** 5)
    D2 = 2.0 * D * (1.0 - torch.eye(n, dtype=T))               # diagonal excluded
    outs = []
    for c0 in range(0, E, chunk):
        Uc = _vars_first(U[c0:c0 + chunk])                     # [nvar, e, k, j, i]
        Jc = Ja[c0:c0 + chunk]                                 # [e, 3(d), 3(n), k, j, i]
        acc = torch.zeros_like(Uc)
        for d in range(3):
            dim = Uc.dim() - 1 - d
            Ud = torch.movedim(Uc, dim, -1)                    # [..., n(line)]
            Ad = torch.movedim(Jc[:, d].transpose(0, 1), dim, -1)   # [3, e, ..., n]
            qi = to_prim(Ud[..., :, None], gas)
            qm = to_prim(Ud[..., None, :], gas)
            a = 0.5 * (Ad[..., :, None] + Ad[..., None, :])
            F = two_point(kind, qi, qm, a, gas)                # [nvar, ..., n(i), n(m)]
            vol = torch.einsum("...im,im->...i", F, D2)
            acc = acc + torch.movedim(vol, -1, dim)
        outs.append(acc.transpose(0, 1))
    return torch.cat(outs, dim=0)


def _orient_index(o: int, n: int) -> torch.Tensor:
    """Flat index into a right-side ``[q', p']`` face grid for every left ``(q, p)``."""
    idx = torch.empty(n, n, dtype=torch.long)
    for q in range(n):
        for p in range(n):
            a, b = (q, p) if (o & 4) else (p, q)
            pp = n - 1 - a if (o & 1) else a
            qq = n - 1 - b if (o & 2) else b
            idx[q, p] = qq * n + pp
    return idx.reshape(-1)


def to_left(tR: torch.Tensor, o: int) -> torch.Tensor:
    """Right-side face data ``[..., n, n]`` re-indexed on the left side's face grid."""
    n = tR.shape[-1]
    flat = tR.reshape(*tR.shape[:-2], n * n)
    return flat[..., _orient_index(o, n)].reshape(*tR.shape)


def to_right(tL: torch.Tensor, o: int) -> torch.Tensor:
    """Inverse of :func:`to_left`."""
    n = tL.shape[-1]
    idx = _orient_index(o, n)
    flat = tL.reshape(*tL.shape[:-2], n * n)
    out = torch.empty_like(flat)
    out[..., idx] = flat
    return out.reshape(*tL.shape)


def apply2(A: torch.Tensor, f: torch.Tensor) -> torch.Tensor:
    """``A (x) A`` on the last two dims (a face grid)."""
    return apply_axis(A, apply_axis(A, f, 0), 1)


def mortar_halves(row):
    """(small element, side, orientation, split index along p or None, along q or None) per small side."""
    mt = row[2]
    nsub = 4 if mt == 3 else 2
    for k in range(nsub):
        kp, kq = (k, None) if mt == 1 else ((None, k) if mt == 2 else (k % 2, k // 2))
        yield row[3 + k], row[7 + k], row[11 + k], kp, kq


def split_apply(A_of, f: torch.Tensor, kp, kq) -> torch.Tensor:
    """Apply ``A_of(k)`` along p (the last axis) for kp and along q for kq."""
    if kp is not None:
        f = apply_axis(_t(A_of(kp)), f, 0)
    if kq is not None:
        f = apply_axis(_t(A_of(kq)), f, 1)
    return f


class Rhs:
    """Evaluates R(u) on one mesh; ``alpha`` is frozen per call."""

    def __init__(self, mesh: OracleMesh, gas: Gas, params: Params):
        self.mesh = mesh
        self.gas = gas
        self.params = params

    # ------------------------------------------------------------------
    def subcell_means(self, U: torch.Tensor, N: int, sel: torch.Tensor) -> torch.Tensor:
        """J-weighted sub-cell means ``V3(J u) / V3(J)`` for group slots ``sel``."""
        g = self.mesh.groups[N]
        V = _t(ops1d.dg2fv(N, self.mesh.n_fv))
        J = g.J[sel][:, None]
        return apply3(V, J * U[sel]) / apply3(V, J)

    def __call__(self, u: torch.Tensor, alpha: torch.Tensor) -> torch.Tensor:
        m, gas, prm = self.mesh, self.gas, self.params
        nvar = gas.nvar
        NFV = m.n_fv
        hfv = 2.0 / NFV
        alpha = torch.as_tensor(alpha, dtype=T)
        alpha_np = alpha.detach().numpy()
        U = {N: m.gather(u, N) for N in m.groups}

        # sub-cell means of blended elements (slot-indexed dict per group)
        blended = {N: torch.as_tensor(np.nonzero(alpha_np[g.elems.numpy()] > 0)[0], dtype=torch.long)
                   for N, g in m.groups.items()}
        ubar = {}
        for N in m.groups:
            if len(blended[N]):
                ub = self.subcell_means(U[N], N, blended[N])
                full = torch.zeros(len(m.groups[N].elems), nvar, NFV, NFV, NFV, dtype=T)
                full = full.index_put((blended[N],), ub)
                ubar[N] = full

        # side flux buffers: DG part at the element degree, FV part on the sub-face grid
        Fdg = {N: [[None] * 6 for _ in range(len(g.elems))] for N, g in m.groups.items()}
        Ffv = {N: [[None] * 6 for _ in range(len(g.elems))] for N, g in m.groups.items()}

        faces = m.faces
        deg = m.degree
        is_fv = np.maximum(alpha_np[faces[:, 0]], alpha_np[faces[:, 2]]) > 0
        keys = np.stack([deg[faces[:, 0]], deg[faces[:, 2]], faces[:, 1], faces[:, 3], faces[:, 4],
                         is_fv.astype(np.int64)], axis=1)
        uniq, inv = np.unique(keys, axis=0, return_inverse=True)
        inv = inv.reshape(-1)
        for gi, (NL, NR, sL, sR, o, fv) in enumerate(uniq.tolist()):
            fsel = np.nonzero(inv == gi)[0]
            eL, eR = faces[fsel, 0], faces[fsel, 2]
            slL = torch.as_tensor(m.slot[eL], dtype=torch.long)
            slR = torch.as_tensor(m.slot[eR], dtype=torch.long)
            gL, gR = m.groups[NL], m.groups[NR]
            tL = face_slice(U[NL][slL], sL)                    # [F, nvar, n, n]
            tR = to_left(face_slice(U[NR][slR], sR), o)
            nvec = gL.outward_normal(sL)[slL]                  # [F, 3, n, n]
            if not fv:
                M = max(NL, NR)
                if NL < M:
                    VL = _t(ops1d.interp(NL, M))
                    tL, nvec = apply2(VL, tL), apply2(VL, nvec)
                if NR < M:
                    tR = apply2(_t(ops1d.interp(NR, M)), tR)
                Fs = riemann(prm.face_flux_dg, _vars_first(tL), _vars_first(tR),
                             _vars_first(nvec), gas, prm.volume_flux)
                Fs = _vars_first(Fs)                           # [F, nvar, M+1, M+1]
                FL = apply2(_t(ops1d.project(M, NL)), Fs) if NL < M else Fs
                FR = apply2(_t(ops1d.project(M, NR)), Fs) if NR < M else Fs
                FR = -to_right(FR, o)
                for r, (a, b) in enumerate(zip(slL.tolist(), slR.tolist())):
                    Fdg[NL][a][sL] = FL[r]
                    Fdg[NR][b][sR] = FR[r]
            else:
                aL = torch.as_tensor(alpha_np[eL] > 0)
                aR = torch.as_tensor(alpha_np[eR] > 0)
                VL = _t(ops1d.dg2fv(NL, NFV))
                VR = _t(ops1d.dg2fv(NR, NFV))
                tLf = apply2(VL, tL)
                tRf = apply2(VR, tR)
                if NL in ubar:
                    bL = face_slice(ubar[NL][slL], sL)
                    tLf = torch.where(aL[:, None, None, None], bL, tLf)
                if NR in ubar:
                    bR = to_left(face_slice(ubar[NR][slR], sR), o)
                    tRf = torch.where(aR[:, None, None, None], bR, tRf)
                nsub = hfv * hfv * apply2(VL, nvec)
                Fs = _vars_first(riemann(prm.face_flux_fv, _vars_first(tLf), _vars_first(tRf),
                                         _vars_first(nsub), gas, prm.volume_flux))
                FL = apply2(_t(ops1d.fv2dg(NL, NFV)), Fs) / (hfv * hfv)
                FR = -to_right(apply2(_t(ops1d.fv2dg(NR, NFV)), Fs) / (hfv * hfv), o)
                FsR = -to_right(Fs, o)
                for r, (a, b) in enumerate(zip(slL.tolist(), slR.tolist())):
                    Fdg[NL][a][sL] = FL[r]
                    Fdg[NR][b][sR] = FR[r]
                    Ffv[NL][a][sL] = Fs[r]
                    Ffv[NR][b][sR] = FsR[r]

        if len(m.mortars):
            self._mortar_fluxes(U, Fdg, Ffv, ubar, alpha_np)

        out = {}
        for N, g in m.groups.items():
            n = N + 1
            E = len(g.elems)
            vol = volume_term(U[N], g.Ja, g.D, gas, prm.volume_flux)
            side = [torch.stack([Fdg[N][e][s] for e in range(E)]) for s in range(6)]
            lift = self._lift(side, E, nvar, n, g.w[0])
            Rdg = -(vol + lift) / g.J[:, None]
            a_el = alpha[g.elems][:, None, None, None, None]
            if len(blended[N]):
                sel = blended[N]
                sidefv = [torch.stack([Ffv[N][e][s] for e in sel.tolist()]) for s in range(6)]
                Rfv = self._fv_residual(N, g, sel, ubar[N][sel], sidefv)
                Rfv_full = torch.zeros_like(Rdg).index_put((sel,), Rfv)
                R = (1.0 - a_el) * Rdg + a_el * Rfv_full
            else:
                R = Rdg
            out[N] = R
        return m.scatter(out, nvar)

    # ------------------------------------------------------------------
    def _mortar_fluxes(self, U, Fdg, Ffv, ubar, alpha_np):
        """Side fluxes of the non-conforming faces (Section 3.2.3, its five steps).

        For each small side k of a big side, when both are DG: the big side's
        trace interpolated to the virtual small side (``M_{0k}`` along the split
        directions, at the big side's degree N_0); the small side's trace brought
        onto that grid by the orientation; both, and the small side's normal (its
        outward one reversed, so that it carries the small side's surface
        element), on the common degree ``max(N_0, N_k)``; the Riemann flux there;
        the small side receives its projection to N_k, reversed; the big side
        receives the projection to N_0 mapped with ``M_{k0}`` along the split
        directions, summed over k.

        When either is FV-blended (the FV variants): the flux is taken on the
        small side's ``N_FV^2`` sub-face grid, as at a conforming FV face, from
        the big side's boundary sub-cell means mapped with ``M^FV_{0k}`` (or its
        DG virtual side through ``V^{DG->FV}``) and the small side's sub-cell
        means (or ``V^{DG->FV}`` of its trace), with the sub-face means of the
        reversed normal times ``h_FV^2``; the small side takes it reversed, its
        DG part through ``V^{FV->DG}`` over ``h_FV^2``; the big side's DG part
        takes ``V^{FV->DG}`` of it at N_0 over ``h_FV^2`` mapped with ``M_{k0}``,
        a blended big side's FV part the sub-face fluxes summed with ``M^FV_{k0}``.
        """
        m, gas, prm = self.mesh, self.gas, self.params
        deg = m.degree
        NFV = m.n_fv
        h2 = (2.0 / NFV) ** 2
        for row in m.mortars.tolist():
            e0, s0, mt = row[0], row[1], row[2]
            N0 = int(deg[e0])
            sl0 = int(m.slot[e0])
            a0 = alpha_np[e0] > 0
            u0 = face_slice(U[N0][sl0:sl0 + 1], s0)[0]           # [nvar, n0, n0] on the big side's grid
            F0 = torch.zeros_like(u0)
            F0fv = torch.zeros(u0.shape[0], NFV, NFV, dtype=T) if a0 else None
            b0 = face_slice(ubar[N0][sl0:sl0 + 1], s0)[0] if a0 else None   # boundary sub-cell means
            nsub = 4 if mt == 3 else 2
            for k in range(nsub):
                ek, sk, ok = row[3 + k], row[7 + k], row[11 + k]
                kp, kq = (k, None) if mt == 1 else ((None, k) if mt == 2 else (k % 2, k // 2))
                uv = u0
                if kp is not None:
                    uv = apply_axis(_t(ops1d.mortar_interp(N0, kp)), uv, 0)
                if kq is not None:
                    uv = apply_axis(_t(ops1d.mortar_interp(N0, kq)), uv, 1)
                Nk = int(deg[ek])
                slk = int(m.slot[ek])
                gk = m.groups[Nk]
                tk = to_left(face_slice(U[Nk][slk:slk + 1], sk), ok)[0]
                nk = -to_left(gk.outward_normal(sk)[slk:slk + 1], ok)[0]
                ak = alpha_np[ek] > 0
                if a0 or ak:
                    if a0:
                        vf = b0
                        if kp is not None:
                            vf = apply_axis(_t(ops1d.mortar_fv_interp(NFV, kp)), vf, 0)
                        if kq is not None:
                            vf = apply_axis(_t(ops1d.mortar_fv_interp(NFV, kq)), vf, 1)
                    else:
                        vf = apply2(_t(ops1d.dg2fv(N0, NFV)), uv)
                    Vk = _t(ops1d.dg2fv(Nk, NFV))
                    sf = to_left(face_slice(ubar[Nk][slk:slk + 1], sk), ok)[0] if ak else apply2(Vk, tk)
                    Fs = riemann(prm.face_flux_fv, vf, sf, h2 * apply2(Vk, nk), gas, prm.volume_flux)
                    Fdg[Nk][slk][sk] = -to_right(apply2(_t(ops1d.fv2dg(Nk, NFV)), Fs)[None] / h2, ok)[0]
                    if ak:
                        Ffv[Nk][slk][sk] = -to_right(Fs[None], ok)[0]
                    Fb = apply2(_t(ops1d.fv2dg(N0, NFV)), Fs) / h2
                    if kp is not None:
                        Fb = apply_axis(_t(ops1d.mortar_project(N0, kp)), Fb, 0)
                    if kq is not None:
                        Fb = apply_axis(_t(ops1d.mortar_project(N0, kq)), Fb, 1)
                    F0 = F0 + Fb
                    if a0:
                        Fv = Fs
                        if kp is not None:
                            Fv = apply_axis(_t(ops1d.mortar_fv_project(NFV, kp)), Fv, 0)
                        if kq is not None:
                            Fv = apply_axis(_t(ops1d.mortar_fv_project(NFV, kq)), Fv, 1)
                        F0fv = F0fv + Fv
                    continue
                M = max(N0, Nk)
                if N0 < M:
                    uv = apply2(_t(ops1d.interp(N0, M)), uv)
                if Nk < M:
                    Vk = _t(ops1d.interp(Nk, M))
                    tk, nk = apply2(Vk, tk), apply2(Vk, nk)
                F = riemann(prm.face_flux_dg, uv, tk, nk, gas, prm.volume_flux)   # [nvar, M+1, M+1]
                Fs = apply2(_t(ops1d.project(M, Nk)), F) if Nk < M else F
                Fdg[Nk][slk][sk] = -to_right(Fs[None], ok)[0]
                Fb = apply2(_t(ops1d.project(M, N0)), F) if N0 < M else F
                if kp is not None:
                    Fb = apply_axis(_t(ops1d.mortar_project(N0, kp)), Fb, 0)
                if kq is not None:
                    Fb = apply_axis(_t(ops1d.mortar_project(N0, kq)), Fb, 1)
                F0 = F0 + Fb
            Fdg[N0][sl0][s0] = F0
            if a0:
                Ffv[N0][sl0][s0] = F0fv

    @staticmethod
    def _lift(side, E, nvar, n, w0):
        """Place each side's outward flux on its boundary nodes, divided by the end weight."""
        L = torch.zeros(E, nvar, n, n, n, dtype=T)
        inv_w = 1.0 / w0
        L[..., :, :, 0] = L[..., :, :, 0] + side[0] * inv_w
        L[..., :, :, -1] = L[..., :, :, -1] + side[1] * inv_w
        L[..., :, 0, :] = L[..., :, 0, :] + side[2] * inv_w
        L[..., :, -1, :] = L[..., :, -1, :] + side[3] * inv_w
        L[..., 0, :, :] = L[..., 0, :, :] + side[4] * inv_w
        L[..., -1, :, :] = L[..., -1, :, :] + side[5] * inv_w
        return L

    def _fv_residual(self, N, g, sel, ub, sidefv):
        """First-order sub-cell operator mapped back to nodal rates (eq. semidiscrete_fv)."""
        gas, prm = self.gas, self.params
        NFV = self.mesh.n_fv
        h = 2.0 / NFV
        V = _t(ops1d.dg2fv(N, NFV))
        Vp = _t(ops1d.fv2dg(N, NFV))
        If = _t(ops1d.face_interp(N, NFV))
        Ja = g.Ja[sel]                                         # [E,3,3,n,n,n]
        dC = torch.zeros_like(ub)                              # [E,nvar,s3,s2,s1]
        for d in range(3):
            # sub-face normals: mean of Ja^d over each sub-cell face, times h^2
            nd = Ja[:, d]
            for ax in range(3):
                nd = apply_axis(If if ax == d else V, nd, ax)
            nd = nd * (h * h)                                  # [E,3, ...(NFV+1 along d)]
            dim = ub.dim() - 1 - d
            ubm = torch.movedim(ub, dim, -1)                   # [E,nvar,a,b,NFV]
            ndm = torch.movedim(nd, dim, -1)                   # [E,3,a,b,NFV+1]
            uL = _vars_first(ubm[..., :-1])
            uR = _vars_first(ubm[..., 1:])
            Fi = _vars_first(riemann(prm.face_flux_fv, uL, uR, _vars_first(ndm[..., 1:-1]), gas,
                                     prm.volume_flux))         # [E,nvar,a,b,NFV-1]
            lo = -sidefv[2 * d]                                # flux in +xi_d at the minus side
            hi = sidefv[2 * d + 1]
            G = torch.cat([lo[..., None], Fi, hi[..., None]], dim=-1)   # [E,nvar,a,b,NFV+1]
            div = G[..., 1:] - G[..., :-1]
            dC = dC - torch.movedim(div, -1, dim)
        JR = apply3(Vp, dC) / h ** 3
        return JR / g.J[sel][:, None]


def rhs(mesh: OracleMesh, gas: Gas, params: Params, u: torch.Tensor, alpha=None) -> torch.Tensor:
    if alpha is None:
        alpha = torch.zeros(mesh.K, dtype=T)
    return Rhs(mesh, gas, params)(u, alpha)
