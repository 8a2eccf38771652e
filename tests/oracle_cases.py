"""Small seeded problems for the oracle pins and the parity tests."""
import numpy as np
import torch

from oracle import problem
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
