"""Fused face fluxes: element kernels of degree 6 and 7 evaluate their conforming DG faces.

The fused path evaluates the same Riemann flux (eq. conv_flux) from the same
operands as the separate face kernel.  Compiled into another kernel, its
products and sums may be contracted into fused multiply-adds differently, so
the fused right-hand side equals the separate path's to rounding (a few ulps of
the face flux, magnified by the cancellation between volume and surface terms;
the CPU build, which contracts nothing, shows them equal bit for bit), and the
oracle's to the parity bar.  Graph replays of the fused step (stages
alternating between two state buffers) equal its eager steps bit for bit.
"""
import pytest
import torch

from oracle import lsrk
from paper_2502_19342_amd import workloads as W

from gpu_common import Case, announce, rel_err, rhs_tol
from oracle_cases import curved_mixed, seeded_alpha, smooth_state

pytestmark = pytest.mark.gpu


def _steps(c, dt, n, alpha, fused, graphs=False):
    from paper_2502_19342_amd import dgfv
    c.gmesh.face_fusion(fused)
    c.gmesh.graphs(graphs)
    u = c.gpu(c.u)
    k = torch.full_like(u, float("nan"))
    out = []
    for _ in range(n):
        dgfv.rk_step(c.gmesh, c.params, dt, u, k, alpha)
        out.append(u.clone())
    torch.cuda.synchronize()
    c.gmesh.graphs(False)
    c.gmesh.face_fusion(False)
    return out


@pytest.mark.parametrize("n_var", [5, 6])
def test_fused_faces_equal_separate_face_kernels(n_var):
    announce(f"fused faces n_var={n_var}")
    flux = {} if n_var == 5 else dict(volume_flux=W.VOL_PIROZZOLI, face_dg=W.RIEMANN_LLF)
    wl = curved_mixed(n=4, nmin=5, nmax=7, n_var=n_var, scramble=29, metric_degree=0, n_fv=8, **flux)
    c = Case(wl, prim=smooth_state(61, n_var), noise=1e-3, seed=9)
    c.alpha = seeded_alpha(c.mesh.K, 17, values=(0.0, 0.0, 0.0, 0.4, 1.0))
    alpha = c.gpu(c.alpha)
    c.gmesh.face_fusion(True)
    fused = c.gpu_rhs()
    c.gmesh.face_fusion(False)
    separate = c.gpu_rhs()
    d = rel_err(fused, separate)
    print(f"[fusion] rhs fused vs separate: {d:.3e}", flush=True)
    assert d <= 1e-13
    assert rel_err(fused, c.oracle_rhs()) <= rhs_tol(c)
    dt = lsrk.timestep(c.mesh, c.gas, c.u, 0.4, c.alpha)
    a = _steps(c, dt, 3, alpha, True)
    b = _steps(c, dt, 3, alpha, False)
    g = _steps(c, dt, 3, alpha, True, graphs=True)
    for i in range(3):
        d = rel_err(a[i].cpu(), b[i].cpu())
        print(f"[fusion] step {i} fused vs separate: {d:.3e}", flush=True)
        assert d <= 1e-12, f"step {i}: fused vs separate"
        assert torch.equal(g[i], a[i]), f"step {i}: graph replay != eager"
    ref = c.u
    for _ in range(3):
        ref = lsrk.step(lambda v: c.f(v, c.alpha), ref, dt)
    assert rel_err(a[2].cpu(), ref) <= max(1e-11, 10 * rhs_tol(c))


def test_fused_faces_uniform_n7_pure_dg():
    # the shear-layer shape at small size: one degree, every face fused
    announce("fused faces N=7 pure DG")
    wl = curved_mixed(n=4, nmin=7, nmax=7, scramble=None, amp=0.0, n_fv=8)
    c = Case(wl, prim=smooth_state(67), noise=1e-3, seed=3)
    c.gmesh.face_fusion(True)
    fused = c.gpu_rhs()
    c.gmesh.face_fusion(False)
    separate = c.gpu_rhs()
    d = rel_err(fused, separate)
    print(f"[fusion] N=7 rhs fused vs separate: {d:.3e}", flush=True)
    assert d <= 1e-13
    assert rel_err(fused, c.oracle_rhs()) <= 1e-12
    dt = lsrk.timestep(c.mesh, c.gas, c.u, 0.5, c.alpha)
    a = _steps(c, dt, 2, None, True)
    b = _steps(c, dt, 2, None, False)
    assert rel_err(a[1].cpu(), b[1].cpu()) <= 1e-12
