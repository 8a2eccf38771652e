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


def oracle_spread(c: "Case", trials: int = 2, seed: int = 0) -> float:
    """Largest rel_err of the oracle's own RHS under random 1-ulp relative perturbations of u.

    The FV sub-cell map V^{FV->DG} amplifies rounding by up to ||V^+||^3 (about
    2.7e3 at N=5, 6e4 at N=7), so no two correct evaluation orders can agree
    better than this spread on blended elements.
    """
    g = torch.Generator().manual_seed(seed)
    r0 = c.oracle_rhs()
    worst = 0.0
    for _ in range(trials):
        up = c.u * (1.0 + 2.0 ** -52 * torch.randn(tuple(c.u.shape), generator=g, dtype=T))
        worst = max(worst, rel_err(c.f(up, c.alpha), r0))
    return worst


def rhs_tol(c: "Case", base: float = 1e-12) -> float:
    """1e-12, or four times the oracle's own 1-ulp spread where the FV map makes that larger."""
    if not bool((c.alpha > 0).any()):
        return base
    return max(base, 4.0 * oracle_spread(c))


def rel_err(a: torch.Tensor, ref: torch.Tensor) -> float:
    """max_v ||a_v - ref_v||_inf / ||ref_v||_inf over the variables."""
    num = (a - ref).abs().amax(dim=1)
    den = ref.abs().amax(dim=1).clamp_min(1e-300)
    return float((num / den).max())


def abs_err(a, ref) -> float:
    return float((a - ref).abs().max())
