"""Helpers of the GPU parity tests: one seeded problem, evaluated by the oracle and the HIP library."""
import sys

import numpy as np
import torch

from oracle import problem
from oracle.indicator import indicator as oracle_indicator

T = torch.float64


def announce(msg: str):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


class Case:
    """A workload with its oracle objects, an oracle-generated state and the GPU mesh."""

    def __init__(self, wl, prim=None, alpha=None, noise=0.0, seed=0):
        from paper_2502_19342_amd import dgfv
        self.wl = wl
        self.mesh, self.gas, self.f = problem.build(wl)
        self.u = problem.initial_state(self.mesh, self.gas, prim or wl.prim)
        if noise:
            rng = np.random.default_rng(seed)
            self.u = self.u * (1.0 + noise * torch.as_tensor(rng.standard_normal(tuple(self.u.shape))))
        K = self.mesh.K
        self.alpha = torch.zeros(K, dtype=T) if alpha is None else torch.as_tensor(alpha, dtype=T)
        self.gmesh = dgfv.Mesh.from_workload(wl)
        self.params = dgfv.params_of(wl)
        assert self.gmesh.n_node == self.mesh.n_node
        assert np.array_equal(self.gmesh.elem_offset, self.mesh.offset)

    def gpu(self, t):
        return t.to("cuda").contiguous()

    def oracle_rhs(self, u=None):
        return self.f(self.u if u is None else u, self.alpha)

    def gpu_rhs(self, u=None, alpha="case"):
        from paper_2502_19342_amd import dgfv
        a = self.gpu(self.alpha) if alpha == "case" else alpha
        r = dgfv.rhs(self.gmesh, self.params, self.gpu(self.u if u is None else u), a)
        torch.cuda.synchronize()
        return r.cpu()

    def oracle_indicator(self, u=None):
        wl = self.wl
        return oracle_indicator(self.mesh, self.gas, self.u if u is None else u, wl.ind_T, wl.ind_dT,
                                wl.ind_vars)


def rel_err(a: torch.Tensor, ref: torch.Tensor) -> float:
    """max_v ||a_v - ref_v||_inf / ||ref_v||_inf over the variables."""
    num = (a - ref).abs().amax(dim=1)
    den = ref.abs().amax(dim=1).clamp_min(1e-300)
    return float((num / den).max())


def abs_err(a, ref) -> float:
    return float((a - ref).abs().max())
