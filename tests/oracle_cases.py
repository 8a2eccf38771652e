"""Small seeded problems for the oracle pins and the parity tests."""
import numpy as np
import torch

from oracle import ops1d, problem
from oracle.physics import prim_to_cons
from paper_2502_19342_amd import workloads as W

T = torch.float64


def curved_mixed(n=3, nmin=2, nmax=4, n_var=5, scramble=None, amp=0.05, seed=7,
                 volume_flux=W.VOL_RANOCHA, face_dg=W.RIEMANN_ROE_HH, face_fv=W.RIEMANN_LLF,
                 n_fv=None, metric_degree=None, prim=None):
    """Curved periodic unit cube, seeded mixed degrees, optionally scrambled frames."""
    deg = W.degree_field(seed, nmin, nmax) if nmax > nmin else nmin
    disp = W.sine_displacement((0, 0, 0), (1, 1, 1), amp) if amp else None
    m = W.structured_mesh(n, (0, 0, 0), (1, 1, 1), deg, displacement=disp, scramble_seed=scramble)
    kw = {}
    if n_var == 6:
        kw = dict(kappa=W.GAS_AIR_H2["kappa"], R=W.GAS_AIR_H2["R"])
    wl = W.Workload("case", m, n_var, prim or W.density_wave, volume_flux, face_dg, face_fv,
                    n_fv=n_fv or nmax + 1,
                    metric_degree=min(2, nmin) if metric_degree is None else metric_degree, **kw)
    return wl


def oracle_of(wl):
    return problem.build(wl)


def state(mesh, gas, prim_fn):
    return problem.initial_state(mesh, gas, prim_fn)


def seeded_alpha(K, seed, values=(0.0, 0.0, 0.4, 1.0)):
    return torch.as_tensor(np.random.default_rng(seed).choice(values, size=K), dtype=T)


def smooth_state(seed, n_var=5):
    """A smooth seeded periodic state with O(0.1) variations."""
    phis = [W.fourier_field(seed * 17 + i, 4, 2) for i in range(6)]

    def f(x):
        ph = [g(x) for g in phis]
        comps = [1.0 + 0.2 * ph[0], 0.3 * ph[1], 0.3 * ph[2], 0.3 * ph[3], 1.0 + 0.2 * ph[4]]
        if n_var == 6:
            comps.append(0.5 + 0.4 * ph[5])
        return np.stack(comps)
    return f


def operator_scale(mesh, rhs_fn, u):
    """Magnitude of the individual terms of R: max |R| of the state with the flux scale of u."""
    return float(rhs_fn(u, torch.zeros(mesh.K, dtype=T)).abs().max())


# ---------------------------------------------------------------------------
# full-size inputs and sampled patches
# ---------------------------------------------------------------------------

def trilinear_nodes(corners: np.ndarray, N: int) -> np.ndarray:
    """Physical coordinates [E, (N+1)^3, 3] of the LGL nodes (i fastest) of trilinear elements."""
    x, _ = ops1d.lgl(N)
    s = 0.5 * (1.0 + np.asarray(x, dtype=np.float64))
    one = np.stack([1.0 - s, s], axis=1)                        # [n, 2]
    wts = np.einsum("kz,jy,ix->kjizyx", one, one, one).reshape(-1, 8)   # corner z*4 + y*2 + x
    return np.einsum("nc,ecd->end", wts, corners)


def c5_state(wl, chunk=8192):
    spec = wl.mesh
    N = int(spec.degree[0])
    gas = problem.gas_of(wl)
    n3 = (N + 1) ** 3
    u = torch.empty(wl.n_var, spec.n_elem * n3, dtype=T)
    for a in range(0, spec.n_elem, chunk):
        b = min(spec.n_elem, a + chunk)
        X = trilinear_nodes(spec.corners[a:b], N).reshape(-1, 3)
        w = torch.as_tensor(np.asarray(wl.prim(X))[: wl.n_var], dtype=T)
        u[:, a * n3:b * n3] = prim_to_cons(w, gas)
    return u


def patch(spec, centres):
    """Sub-mesh of the centres and their face neighbours; uncovered sides get self-faces."""
    faces = np.asarray(spec.faces, dtype=np.int64)
    touch = np.isin(faces[:, 0], centres) | np.isin(faces[:, 2], centres)
    elems = np.unique(np.concatenate([centres, faces[touch, 0], faces[touch, 2]]))
    local = {int(e): i for i, e in enumerate(elems)}
    inside = np.isin(faces[:, 0], elems) & np.isin(faces[:, 2], elems)
    sub = faces[inside].copy()
    sub[:, 0] = [local[int(e)] for e in sub[:, 0]]
    sub[:, 2] = [local[int(e)] for e in sub[:, 2]]
    covered = np.zeros((len(elems), 6), dtype=bool)
    covered[sub[:, 0], sub[:, 1]] = True
    covered[sub[:, 2], sub[:, 3]] = True
    for i in range(len(elems)):
        for s in range(6):
            if not covered[i, s]:
                assert int(elems[i]) not in set(centres.tolist())
                sub = np.vstack([sub, [i, s, i, s, 0]])
    pspec = W.MeshSpec(n=spec.n, lo=spec.lo, hi=spec.hi, corners=spec.corners[elems],
                       faces=sub.astype(np.int32), degree=spec.degree[elems])
    return elems, local, pspec


def node_index(offsets, elems):
    return np.concatenate([np.arange(offsets[e], offsets[e + 1]) for e in elems])


# ---------------------------------------------------------------------------
# face traces and the Harten-Hyman switch (coverage checks of parity cases)
# ---------------------------------------------------------------------------

def face_traces(mesh, u):
    """Left and right states and left outward n*s at every node of every face.

    Faces with equal degree only; returns ``(uL, uR, nvec)`` as ``[nvar, P]``,
    ``[nvar, P]`` and ``[3, P]`` over all face nodes P.
    """
    from oracle.geometry import face_slice
    from oracle.rhs import to_left
    UL, UR, NV = [], [], []
    for eL, sL, eR, sR, o in np.asarray(mesh.faces).tolist():
        NL, NR = int(mesh.degree[eL]), int(mesh.degree[eR])
        if NL != NR:
            continue
        g = mesh.groups[NL]
        tL = face_slice(mesh.gather(u, NL)[int(mesh.slot[eL])], sL)
        tR = to_left(face_slice(mesh.gather(u, NR)[int(mesh.slot[eR])], sR), o)
        UL.append(tL.reshape(tL.shape[0], -1))
        UR.append(tR.reshape(tR.shape[0], -1))
        nv = g.outward_normal(sL)[int(mesh.slot[eL])]
        NV.append(nv.reshape(3, -1))
    return torch.cat(UL, 1), torch.cat(UR, 1), torch.cat(NV, 1)


def harten_hyman_active(uL, uR, nvec, gamma):
    """Per face node: is the entropy fix active on an acoustic wave of the Roe solver?

    Roe averages with sqrt(rho) weights, wave speeds v.n -+ c of the average and
    of each side; the fix replaces |lam~| where |lam~| < max(0, lam~ - lam_L, lam_R - lam~).
    """
    n = nvec / torch.sqrt((nvec * nvec).sum(0))

    def prim(u):
        rho = u[0]
        v = u[1:4] / rho
        p = (gamma - 1.0) * (u[4] - 0.5 * rho * (v * v).sum(0))
        return rho, v, p, (u[4] + p) / rho

    rL, vL, pL, HL = prim(uL)
    rR, vR, pR, HR = prim(uR)
    wl, wr = torch.sqrt(rL), torch.sqrt(rR)
    v = (wl * vL + wr * vR) / (wl + wr)
    H = (wl * HL + wr * HR) / (wl + wr)
    c = torch.sqrt((gamma - 1.0) * (H - 0.5 * (v * v).sum(0)))
    vn, vnL, vnR = (v * n).sum(0), (vL * n).sum(0), (vR * n).sum(0)
    cL, cR = torch.sqrt(gamma * pL / rL), torch.sqrt(gamma * pR / rR)
    act = torch.zeros_like(vn, dtype=torch.bool)
    for sg in (-1.0, 1.0):
        lt, lL, lR = vn + sg * c, vnL + sg * cL, vnR + sg * cR
        delta = torch.clamp(torch.maximum(lt - lL, lR - lt), min=0.0)
        act |= lt.abs() < delta
    return act


def transonic_state(seed):
    """Smooth state whose velocity along x stays within a few per cent of the sound speed."""
    phis = [W.fourier_field(seed * 19 + i, 4, 2) for i in range(4)]

    def f(x):
        ph = [g(x) for g in phis]
        c0 = np.sqrt(1.4)
        vx = c0 * (1.0 + 0.03 * np.sin(2 * np.pi * x[:, 0]) + 0.01 * ph[1])
        return np.stack([1.0 + 0.2 * ph[0], vx, 0.2 * ph[2], 0.2 * ph[3], np.ones(len(x))])
    return f
