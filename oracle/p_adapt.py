"""Dynamic p-adaptation: the degree decision and the state transfer (oracle).

Test infrastructure: a plain, slow reference.  Only the tests, the smoke check
and the benchmark's CPU-baseline leg use it.

Section 3.4 drives the local ansatz degree by the modal decay indicator of
the density, ``I_p-adapt = I(rho)``, compared with thresholds of its own;
Section 3.2 maps an element's solution between degrees: to a higher degree by
interpolation ``V^{N->M}`` (exact), to a lower one by projection ``V^{M->N}``
(the modal L2 truncation, which keeps the Legendre modes up to the lower
degree).

Readings where the paper is silent (it defers the thresholds to earlier work):

* decision per element, one degree per adaptation: ``I < T_refine`` (slow
  modal decay, under-resolved) raises N by one, ``I > T_coarsen`` (fast decay,
  over-resolved) lowers it by one, clamped to ``[N_min, N_max]``; both
  thresholds are configuration values (parity unpinned in value);
  ``T_refine < T_coarsen``; ``I = +inf`` (a constant density) coarsens;
* the maps act on the conservative state ``u`` itself in reference space, as
  the face maps of Section 3.2.1 act on traces: constants and polynomials of
  the lower degree are kept exactly, a raise followed by a lowering returns
  the state, and on affine elements (constant J) the element's content
  ``sum w J u`` is kept as well.
"""
from __future__ import annotations

import numpy as np
import torch

from . import ops1d
from .geometry import OracleMesh, apply3, _t
from .indicator import indicator
from .physics import Gas

T = torch.float64


def degrees(mesh: OracleMesh, gas: Gas, u: torch.Tensor, t_refine: float, t_coarsen: float, n_min: int,
            n_max: int) -> np.ndarray:
    """New degree of every element from ``I(rho)`` (module docstring)."""
    I, _ = indicator(mesh, gas, u, 0.0, 1.0, ind_vars=2)
    N = mesh.degree.copy()
    I = I.numpy()
    up = I < t_refine
    down = I > t_coarsen
    N = np.where(up, np.minimum(N + 1, n_max), np.where(down, np.maximum(N - 1, n_min), N))
    return N.astype(np.int64)


def map1d(n_from: int, n_to: int) -> np.ndarray:
    """The 1D map from degree ``n_from`` to ``n_to``: interpolation up, modal truncation down."""
    if n_to > n_from:
        return ops1d.interp(n_from, n_to)
    if n_to < n_from:
        return ops1d.project(n_from, n_to)
    return np.eye(n_from + 1)


def transfer(mesh_from: OracleMesh, mesh_to: OracleMesh, u: torch.Tensor) -> torch.Tensor:
    """The state on ``mesh_to`` (same elements, new degrees), element by element."""
    parts = {N: [] for N in mesh_to.groups}
    for N_to, g in mesh_to.groups.items():
        for e in g.elems.tolist():
            N_from = int(mesh_from.degree[e])
            a, b = int(mesh_from.offset[e]), int(mesh_from.offset[e + 1])
            n = N_from + 1
            ue = u[:, a:b].reshape(u.shape[0], n, n, n)
            parts[N_to].append(apply3(_t(map1d(N_from, N_to)), ue))
    return mesh_to.scatter({N: torch.stack(v) for N, v in parts.items()}, u.shape[0])
