"""Assemble a synthetic workload into oracle objects (test infrastructure only)."""
from __future__ import annotations

import numpy as np
import torch

from .geometry import OracleMesh
from .physics import Gas, prim_to_cons
from .rhs import Params, Rhs
from .viscous import Transport, ViscousRhs

T = torch.float64


def gas_of(wl) -> Gas:
    return Gas(nvar=wl.n_var, gamma=wl.gamma, kappa=tuple(wl.kappa), R=tuple(wl.R))


def params_of(wl) -> Params:
    return Params(wl.volume_flux, wl.face_flux_dg, wl.face_flux_fv)


def transport_of(wl) -> Transport:
    return Transport(mu=tuple(wl.mu), Pr=tuple(wl.Pr), D=tuple(wl.D))


def build(wl):
    """Mesh, gas and ``R(u, alpha)``; with the viscous terms when the workload has any."""
    mesh = OracleMesh(wl.mesh, wl.n_fv, wl.metric_degree)
    gas = gas_of(wl)
    f = Rhs(mesh, gas, params_of(wl))
    if getattr(wl, "viscous", False):
        f = ViscousRhs(f, mesh, gas, transport_of(wl))
    return mesh, gas, f


def initial_state(mesh: OracleMesh, gas: Gas, prim_fn) -> torch.Tensor:
    """Sample a primitive-state function at the oracle's nodes, return conservative ``[nvar, n_node]``."""
    x = mesh.node_coords().numpy().T                           # [n_node, 3]
    w = torch.as_tensor(np.asarray(prim_fn(x)), dtype=T)
    if w.shape[0] != gas.nvar:
        w = w[: gas.nvar]
    return prim_to_cons(w, gas)
