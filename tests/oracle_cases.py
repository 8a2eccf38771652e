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
                    n_fv=n_fv or nmax + 1, metric_degree=metric_degree or min(2, nmin), **kw)
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
