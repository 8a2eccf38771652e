"""Pins of the oracle's p-adaptation (Sections 3.2 and 3.4).

* the decision: a table of indicator values against the thresholds and the
  degree bounds; and on a state with one sharp density front the elements at
  the front refine while the smooth far field coarsens;
* the maps: raising and lowering again returns the state; lowering returns a
  field of the lower degree exactly and keeps the Legendre modes up to the
  lower degree; constants stay constant on curved meshes; on affine meshes
  every element's content is kept, up and down.
"""
import dataclasses

import numpy as np
import torch

from oracle import ops1d, p_adapt, problem
from oracle.geometry import OracleMesh, apply3, _t
from oracle.indicator import indicator
from paper_2502_19342_amd import workloads as W

from oracle_cases import curved_mixed, smooth_state

T = torch.float64


def redegree(mesh: OracleMesh, new) -> OracleMesh:
    spec = dataclasses.replace(mesh.spec, degree=np.asarray(new).astype(np.int8))
    return OracleMesh(spec, mesh.n_fv, mesh.NJ)


def test_decision_table(monkeypatch):
    spec = W.structured_mesh(2, (0, 0, 0), (1, 1, 1), lambda c: np.array([1, 2, 3, 4, 5, 6, 7, 4]))
    mesh = OracleMesh(spec, 8, 1)
    I = torch.tensor([0.5, 0.5, 3.0, 9.0, 0.1, 0.5, 9.0, float("inf")], dtype=T)
    monkeypatch.setattr(p_adapt, "indicator", lambda *a, **k: (I, None))
    got = p_adapt.degrees(mesh, None, None, t_refine=1.0, t_coarsen=5.0, n_min=2, n_max=6)
    # 1 -> 2 (refine), 2 -> 3 (refine), 3 stays, 4 -> 3 (coarsen), 5 -> 6, 6 stays at the cap,
    # 7 -> 6 (coarsen), +inf coarsens 4 -> 3
    assert got.tolist() == [2, 3, 3, 3, 6, 6, 6, 3]


def test_front_refines_far_field_coarsens():
    wl = curved_mixed(n=4, nmin=4, nmax=4, scramble=None, amp=0.0, n_fv=5)
    mesh, gas, _ = problem.build(wl)

    def front(x):
        r = np.linalg.norm(x - 0.5, axis=-1)
        rho = 1.0 + 0.5 * np.tanh((r - 0.3) / 0.01)
        z = np.zeros_like(rho)
        return np.stack([rho, z, z, z, np.ones_like(rho)])
    u = problem.initial_state(mesh, gas, front)
    I, _ = indicator(mesh, gas, u, 0.0, 1.0, ind_vars=2)
    N = p_adapt.degrees(mesh, gas, u, 2.0, 6.0, 2, 6)
    centres = mesh.node_coords().reshape(3, mesh.K, -1).mean(dim=2).T.numpy()
    dist = np.abs(np.linalg.norm(centres - 0.5, axis=1) - 0.3)
    near, far = dist < 0.2, dist > 0.2          # the front crosses the first set, not the second
    assert near.any() and far.any()
    assert (N[near] == 5).all(), (I[torch.as_tensor(near)], N[near])
    assert (N[far] == 3).all(), (I[torch.as_tensor(far)], N[far])


def _case(curved, seed=3):
    wl = curved_mixed(n=3, nmin=2, nmax=5, scramble=7, metric_degree=0, n_fv=8, amp=0.05 if curved else 0.0,
                      seed=seed)
    mesh, gas, _ = problem.build(wl)
    rng = np.random.default_rng(seed)
    new = np.clip(mesh.degree + rng.integers(-1, 2, size=mesh.K), 1, 7)
    return mesh, gas, new


def test_up_then_down_returns_the_state_and_constants_stay():
    mesh, gas, _ = _case(curved=True)
    u = problem.initial_state(mesh, gas, smooth_state(5))
    m_up = redegree(mesh, np.minimum(mesh.degree + 1, 7))
    back = p_adapt.transfer(m_up, mesh, p_adapt.transfer(mesh, m_up, u))
    assert torch.allclose(back, u, rtol=1e-13, atol=1e-13)
    c = problem.initial_state(mesh, gas, lambda x: W.freestream(x, 5))
    for m2 in (m_up, redegree(mesh, np.maximum(mesh.degree - 1, 1))):
        c2 = p_adapt.transfer(mesh, m2, c)
        assert torch.allclose(c2, c[:, :1].expand(-1, c2.shape[1]), rtol=1e-13, atol=1e-13)


def test_down_is_exact_on_lower_degree_fields_and_keeps_low_modes():
    mesh, gas, _ = _case(curved=False)
    down = np.maximum(mesh.degree - 1, 1)
    m_down = redegree(mesh, down)
    rng = np.random.default_rng(9)
    u = torch.zeros(5, mesh.n_node, dtype=T)
    low = {}
    for e in range(mesh.K):                       # a field of the lower degree in every element
        N, Nd = int(mesh.degree[e]), int(down[e])
        v = torch.as_tensor(rng.standard_normal((5, Nd + 1, Nd + 1, Nd + 1)))
        low[e] = v
        up = apply3(_t(ops1d.interp(Nd, N)), v) if Nd < N else v
        a, b = int(mesh.offset[e]), int(mesh.offset[e + 1])
        u[:, a:b] = up.reshape(5, -1)
    ud = p_adapt.transfer(mesh, m_down, u)
    for e in range(mesh.K):
        c, d = int(m_down.offset[e]), int(m_down.offset[e + 1])
        assert torch.allclose(ud[:, c:d], low[e].reshape(5, -1), rtol=1e-12, atol=1e-12)
    # a general field: the Legendre modes up to the lower degree are kept
    w = problem.initial_state(mesh, gas, smooth_state(11))
    wd = p_adapt.transfer(mesh, m_down, w)
    for e in range(mesh.K):
        N, Nd = int(mesh.degree[e]), int(down[e])
        a, b = int(mesh.offset[e]), int(mesh.offset[e + 1])
        c, d = int(m_down.offset[e]), int(m_down.offset[e + 1])
        mo = apply3(_t(ops1d.vleg_inv(N)), w[:, a:b].reshape(5, N + 1, N + 1, N + 1))
        md = apply3(_t(ops1d.vleg_inv(Nd)), wd[:, c:d].reshape(5, Nd + 1, Nd + 1, Nd + 1))
        assert torch.allclose(md, mo[:, :Nd + 1, :Nd + 1, :Nd + 1], rtol=1e-11, atol=1e-12)


def test_contents_kept_on_affine_meshes():
    mesh, gas, new = _case(curved=False)
    u = problem.initial_state(mesh, gas, smooth_state(8))
    m2 = redegree(mesh, new)
    u2 = p_adapt.transfer(mesh, m2, u)
    w1 = mesh.weights_flat() * mesh.jacobian_flat()
    w2 = m2.weights_flat() * m2.jacobian_flat()
    for e in range(mesh.K):
        a, b = int(mesh.offset[e]), int(mesh.offset[e + 1])
        c, d = int(m2.offset[e]), int(m2.offset[e + 1])
        assert torch.allclose((u[:, a:b] * w1[a:b]).sum(1), (u2[:, c:d] * w2[c:d]).sum(1), rtol=1e-13, atol=1e-15)
