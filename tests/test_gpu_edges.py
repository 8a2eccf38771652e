"""Degenerate and boundary cases of the hybrid right-hand side, through the C ABI.

* The smallest periodic mesh the generator builds (2 x 2 x 2 elements): every
  element meets the same neighbour across both faces of a direction, so each
  element pair shares two faces; degrees 1..7 and blended elements at once.
* Every element blended (alpha = 1): only FV faces, the blended list holds the
  whole mesh, every element takes the pure FV residual.
* alpha = 0 everywhere, passed as an array: the blended list is empty, and the
  result and an RK stage are bit for bit those of alpha = NULL.
* One element per degree bucket next to full buckets: a 3 x 3 x 3 mesh with
  degrees 1..7 puts a few elements in each bucket, so every element-kernel
  workgroup of the small degrees is partly empty (ragged tails).
Bars as in the other parity tests: 1e-12 relative, or four times the oracle's
1-ulp spread where elements are blended.
"""
import numpy as np
import pytest
import torch

from oracle import lsrk
from paper_2502_19342_amd import workloads as W

from gpu_common import Case, announce, rel_err, rhs_tol
from oracle_cases import curved_mixed, seeded_alpha, smooth_state

pytestmark = pytest.mark.gpu
T = torch.float64


def test_smallest_periodic_mesh_mixed_blended():
    announce("2^3 periodic mesh, degrees 1..7, blended")
    wl = curved_mixed(n=2, nmin=1, nmax=7, scramble=31, metric_degree=1, n_fv=8)
    c = Case(wl, prim=smooth_state(91), noise=1e-3, seed=11)
    c.alpha = seeded_alpha(c.mesh.K, 32, values=(0.0, 0.5, 1.0))
    assert rel_err(c.gpu_rhs(), c.oracle_rhs()) <= rhs_tol(c)


def test_every_element_blended():
    announce("alpha = 1 everywhere")
    wl = curved_mixed(n=3, nmin=2, nmax=4, scramble=33, metric_degree=1, n_fv=5)
    c = Case(wl, prim=smooth_state(92), noise=1e-3, seed=12)
    c.alpha = torch.ones(c.mesh.K, dtype=T)
    assert rel_err(c.gpu_rhs(), c.oracle_rhs()) <= rhs_tol(c)


def test_zero_alpha_array_equals_pure_dg():
    announce("alpha = 0 array vs NULL")
    from paper_2502_19342_amd import dgfv
    wl = curved_mixed(n=3, nmin=1, nmax=7, scramble=34, metric_degree=1, n_fv=8)
    c = Case(wl, prim=smooth_state(93), noise=1e-3, seed=13)
    zero = torch.zeros(c.mesh.K, dtype=T, device="cuda")
    r_none = c.gpu_rhs(alpha=None)
    r_zero = c.gpu_rhs(alpha=zero)
    assert torch.equal(r_none, r_zero)
    assert rel_err(r_none, c.oracle_rhs()) <= 1e-12
    dt, stage = 1e-4, 2
    k0 = 1e-3 * c.u.roll(1, dims=1)
    u1, k1 = c.gpu(c.u), c.gpu(k0)
    u2, k2 = c.gpu(c.u), c.gpu(k0)
    dgfv.rk_stage(c.gmesh, c.params, stage, dt, u1, k1, None)
    dgfv.rk_stage(c.gmesh, c.params, stage, dt, u2, k2, zero)
    torch.cuda.synchronize()
    assert torch.equal(u1, u2) and torch.equal(k1, k2)
    k_ref = float(lsrk.A[stage - 1]) * k0 + dt * c.oracle_rhs()
    assert rel_err(k1.cpu(), k_ref) <= 1e-12


def test_ragged_degree_buckets():
    announce("3^3 mesh, degrees 1..7, ragged buckets")
    wl = curved_mixed(n=3, nmin=1, nmax=7, scramble=35, metric_degree=1, n_fv=8)
    c = Case(wl, prim=smooth_state(94), noise=1e-3, seed=14)
    counts = np.bincount(np.asarray(wl.mesh.degree), minlength=8)[1:]
    assert (counts > 0).sum() >= 5                 # several buckets, most far from a full workgroup
    c.alpha = seeded_alpha(c.mesh.K, 36, values=(0.0, 0.0, 1.0))
    assert rel_err(c.gpu_rhs(), c.oracle_rhs()) <= rhs_tol(c)


def test_nonphysical_state_is_reported():
    """rho <= 0 in the state read by an RK stage: DGFV_ERR_STATE from the next call once the
    flag copy has landed (DG elements and pure FV elements at N >= 6), and from dgfv_check_state."""
    announce("non-physical state flag")
    from paper_2502_19342_amd import dgfv
    wl = curved_mixed(n=2, nmin=6, nmax=7, scramble=37, metric_degree=1, n_fv=8)
    c = Case(wl, prim=smooth_state(95), noise=1e-3, seed=15)
    dt = 1e-5
    u, k = c.gpu(c.u), torch.zeros_like(c.gpu(c.u))
    dgfv.rk_step(c.gmesh, c.params, dt, u, k, None)
    torch.cuda.synchronize()
    dgfv.rk_step(c.gmesh, c.params, dt, u, k, None)     # sees the first step's copy: clean
    dgfv.check_state(c.gmesh)
    node = int(c.gmesh.elem_offset[3]) + 5               # a node of element 3
    for alpha in (None, torch.ones(c.mesh.K, dtype=T, device="cuda")):
        u, k = c.gpu(c.u), torch.zeros_like(c.gpu(c.u))
        u[0, node] = -1.0
        dgfv.rk_stage(c.gmesh, c.params, 1, dt, u, k, alpha)
        torch.cuda.synchronize()
        with pytest.raises(dgfv.DgfvError) as err:
            dgfv.rk_stage(c.gmesh, c.params, 2, dt, u, k, alpha)
        assert err.value.status == dgfv.ERR_STATE
        dgfv.check_state(c.gmesh)                        # reported once, then cleared
    u = c.gpu(c.u)
    u[4, node] = float("nan")
    dgfv.rhs(c.gmesh, c.params, u, None)
    with pytest.raises(dgfv.DgfvError) as err:
        dgfv.check_state(c.gmesh)
    assert err.value.status == dgfv.ERR_STATE
    dgfv.check_state(c.gmesh)
    r = dgfv.rhs(c.gmesh, c.params, c.gpu(c.u), None)   # a good state again: no report
    dgfv.check_state(c.gmesh)
    assert rel_err(r.cpu(), c.oracle_rhs()) <= 1e-12
