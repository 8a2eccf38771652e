"""Launch batching: hipGraph replays and concurrent degree buckets give the eager results.

Each replay is checked bit for bit against the eager (graphs off) step from the
same input, with unrelated device work and synchronisations between replays.
The per-degree branches write disjoint data, so concurrency does not change
any rounding.
"""
import pytest
import torch

from paper_2502_19342_amd import workloads as W

from gpu_common import Case, announce
from oracle_cases import curved_mixed, seeded_alpha, smooth_state

pytestmark = pytest.mark.gpu


def _eager_steps(c, dt, n, alpha, mode=None):
    from paper_2502_19342_amd import dgfv
    c.gmesh.launch_mode(dgfv.LAUNCH_SERIAL if mode is None else mode)
    u = c.gpu(c.u)
    k = torch.full_like(u, float("nan"))
    out = []
    for _ in range(n):
        dgfv.rk_step(c.gmesh, c.params, dt, u, k, alpha)
        out.append(u.clone())
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("blend", [False, True])
def test_graph_replays_match_eager_steps(blend):
    announce(f"graph replays blend={blend}")
    from paper_2502_19342_amd import dgfv
    wl = curved_mixed(n=4, nmin=1, nmax=5, scramble=41, metric_degree=1, n_fv=6)
    c = Case(wl, prim=smooth_state(97), noise=1e-3, seed=12)
    alpha = c.gpu(seeded_alpha(c.mesh.K, 42, values=(0.0, 0.0, 0.5, 1.0))) if blend else None
    dt = 1e-4
    ref = _eager_steps(c, dt, 4, alpha)
    branches = _eager_steps(c, dt, 4, alpha, mode=dgfv.LAUNCH_BRANCHES)
    for i in range(4):
        assert torch.equal(branches[i], ref[i]), f"concurrent buckets, step {i}"
    c.gmesh.graphs(True)
    u = c.gpu(c.u)
    k = torch.full_like(u, float("nan"))
    scratch = torch.randn(1 << 20, dtype=torch.float64, device="cuda")
    for i in range(4):
        dgfv.rk_step(c.gmesh, c.params, dt, u, k, alpha)     # the first call captures, later ones replay
        scratch.mul_(1.0001).add_(0.5)                       # eager work between replays
        torch.cuda.synchronize()
        assert torch.equal(u, ref[i]), f"replay {i}"
    # stages as separate graphs, and a new dt, are captured anew
    u2 = c.gpu(c.u)
    k2 = torch.full_like(u2, float("nan"))
    for s in range(1, 6):
        dgfv.rk_stage(c.gmesh, c.params, s, dt, u2, k2, alpha)
    torch.cuda.synchronize()
    assert torch.equal(u2, ref[0])
    c.gmesh.graphs(False)


def test_graph_recaptures_on_new_alpha_pointer():
    announce("graph new alpha")
    from paper_2502_19342_amd import dgfv
    wl = curved_mixed(n=3, nmin=2, nmax=4, scramble=43, n_fv=5)
    c = Case(wl, prim=smooth_state(99), noise=1e-3, seed=13)
    a1 = c.gpu(seeded_alpha(c.mesh.K, 44, values=(0.0, 1.0)))
    a2 = c.gpu(seeded_alpha(c.mesh.K, 45, values=(0.0, 0.3, 1.0)))
    dt = 1e-4
    r1 = _eager_steps(c, dt, 1, a1)[0]
    r2 = _eager_steps(c, dt, 1, a2)[0]
    c.gmesh.graphs(True)
    for a, r in ((a1, r1), (a2, r2), (a1, r1)):
        u = c.gpu(c.u)
        k = torch.zeros_like(u)
        dgfv.rk_step(c.gmesh, c.params, dt, u, k, a)
        torch.cuda.synchronize()
        assert torch.equal(u, r)
    c.gmesh.graphs(False)


def test_element_shapes_and_autotune():
    announce("element shapes + autotune")
    from paper_2502_19342_amd import dgfv
    from gpu_common import rel_err, rhs_tol
    wl = curved_mixed(n=3, nmin=1, nmax=5, scramble=47, metric_degree=1, n_fv=6)
    c = Case(wl, prim=smooth_state(101), noise=1e-3, seed=14)
    c.alpha = seeded_alpha(c.mesh.K, 48, values=(0.0, 0.0, 0.5, 1.0))
    out = []
    for shape in (0, 1):
        for N in range(1, 6):
            c.gmesh.set_element_shape(N, shape)
        out.append(c.gpu_rhs())
    # the shape only changes how many elements share a workgroup: identical arithmetic
    assert torch.equal(out[0], out[1])
    assert rel_err(out[1], c.oracle_rhs()) <= rhs_tol(c)
    with pytest.raises(dgfv.DgfvError):
        c.gmesh.set_element_shape(7, 1)          # one shape only at N = 7
    ms = c.gmesh.autotune(c.params, c.gpu(c.u), c.gpu(c.alpha))
    assert set(ms) <= {1, 2, 3, 4, 5} and all(a > 0 and b > 0 for a, b in ms.values())
    assert torch.equal(c.gpu_rhs(), out[0])


def test_launch_mode_and_shape_arguments_are_checked():
    announce("launch mode / shape argument checks")
    from paper_2502_19342_amd import dgfv
    wl = curved_mixed(n=2, nmin=2, nmax=3, scramble=49)
    c = Case(wl, prim=smooth_state(103))
    with pytest.raises(dgfv.DgfvError) as e:
        c.gmesh.launch_mode(3)
    assert e.value.status == dgfv.ERR_ARG
    with pytest.raises(dgfv.DgfvError):
        c.gmesh.set_element_shape(0, 0)
    with pytest.raises(dgfv.DgfvError):
        c.gmesh.set_element_shape(2, 2)
    # every mode gives the same step
    out = []
    for mode in (dgfv.LAUNCH_SERIAL, dgfv.LAUNCH_BRANCHES, dgfv.LAUNCH_GRAPH):
        c.gmesh.launch_mode(mode)
        u = c.gpu(c.u)
        k = torch.zeros_like(u)
        for _ in range(2):
            dgfv.rk_step(c.gmesh, c.params, 1e-4, u, k)
        torch.cuda.synchronize()
        out.append(u)
    assert torch.equal(out[0], out[1]) and torch.equal(out[0], out[2])
    c.gmesh.launch_mode(dgfv.LAUNCH_BRANCHES)
