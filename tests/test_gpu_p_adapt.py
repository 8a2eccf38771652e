"""Dynamic p-adaptation on the GPU against the oracle (Sections 3.2 and 3.4).

The degree decision from I(rho), the transfer of the state to the new
degrees, and an adaptive run: RK steps on one mesh, a decision, the mesh of the
new degrees (its own buckets, work lists and captured graphs), the transfer,
and RK steps there, each compared with the oracle doing the same.
"""
import dataclasses

import numpy as np
import pytest
import torch

from oracle import lsrk, p_adapt, problem
from oracle.geometry import OracleMesh
from oracle.indicator import indicator
from paper_2502_19342_amd import workloads as W

from gpu_common import announce, rel_err
from oracle_cases import curved_mixed, smooth_state

pytestmark = pytest.mark.gpu
T = torch.float64


def _oracle_redegree(mesh, new):
    return OracleMesh(dataclasses.replace(mesh.spec, degree=np.asarray(new).astype(np.int8)), mesh.n_fv, mesh.NJ)


@pytest.mark.parametrize("n_var", [5, 6])
def test_p_degrees_and_transfer(n_var):
    announce(f"p-adaptation decision + transfer n_var={n_var}")
    from paper_2502_19342_amd import dgfv
    flux = {} if n_var == 5 else dict(volume_flux=W.VOL_PIROZZOLI, face_dg=W.RIEMANN_LLF)
    wl = curved_mixed(n=4, nmin=2, nmax=6, n_var=n_var, scramble=13, metric_degree=0, n_fv=8, **flux)
    mesh, gas, _ = problem.build(wl)
    u = problem.initial_state(mesh, gas, smooth_state(37, n_var))
    u = u * (1.0 + 1e-2 * torch.as_tensor(np.random.default_rng(2).standard_normal(tuple(u.shape))))
    I, _ = indicator(mesh, gas, u, 0.0, 1.0, ind_vars=2)
    t_ref, t_coarse = float(np.quantile(I.numpy(), 0.3)), float(np.quantile(I.numpy(), 0.7))
    want = p_adapt.degrees(mesh, gas, u, t_ref, t_coarse, 1, 7)
    gm = dgfv.Mesh.from_workload(wl)
    prm = dgfv.params_of(wl)
    ug = u.to("cuda").contiguous()
    got = dgfv.p_degrees(gm, prm, ug, t_ref, t_coarse, 1, 7)
    assert np.array_equal(got.astype(np.int64), want)
    gm2 = gm.redegree(got)
    m2 = _oracle_redegree(mesh, want)
    assert gm2.n_node == m2.n_node
    u2 = dgfv.transfer_degree(gm, gm2, ug)
    torch.cuda.synchronize()
    assert rel_err(u2.cpu(), p_adapt.transfer(mesh, m2, u)) <= 1e-13


def test_adaptive_run():
    announce("p-adaptive run")
    from paper_2502_19342_amd import dgfv
    wl = curved_mixed(n=4, nmin=2, nmax=5, scramble=17, metric_degree=0, n_fv=8)
    mesh, gas, f = problem.build(wl)
    u = problem.initial_state(mesh, gas, smooth_state(41))
    u = u * (1.0 + 1e-3 * torch.as_tensor(np.random.default_rng(3).standard_normal(tuple(u.shape))))
    alpha = torch.zeros(mesh.K, dtype=T)
    dt = 0.3 * lsrk.timestep(mesh, gas, u, 0.5)
    gm = dgfv.Mesh.from_workload(wl)
    prm = dgfv.params_of(wl)
    ug = u.to("cuda").contiguous()
    k = torch.zeros_like(ug)
    gm.graphs(True)
    uo = u.clone()
    for _ in range(3):
        dgfv.rk_step(gm, prm, dt, ug, k, None)
        uo = lsrk.step(lambda v: f(v, alpha), uo, dt)
    I, _ = indicator(mesh, gas, uo, 0.0, 1.0, ind_vars=2)
    t_ref, t_coarse = float(np.quantile(I.numpy(), 0.35)), float(np.quantile(I.numpy(), 0.65))
    new = dgfv.p_degrees(gm, prm, ug, t_ref, t_coarse, 2, 6)
    assert np.array_equal(new.astype(np.int64), p_adapt.degrees(mesh, gas, uo, t_ref, t_coarse, 2, 6))
    gm2 = gm.redegree(new)
    gm2.graphs(True)
    m2 = _oracle_redegree(mesh, new)
    f2 = problem.Rhs(m2, gas, problem.params_of(wl))
    ug2 = dgfv.transfer_degree(gm, gm2, ug)
    uo2 = p_adapt.transfer(mesh, m2, uo)
    k2 = torch.zeros_like(ug2)
    alpha2 = torch.zeros(m2.K, dtype=T)
    for _ in range(3):
        dgfv.rk_step(gm2, prm, dt, ug2, k2, None)
        uo2 = lsrk.step(lambda v: f2(v, alpha2), uo2, dt)
    torch.cuda.synchronize()
    assert rel_err(ug2.cpu(), uo2) <= 1e-10
