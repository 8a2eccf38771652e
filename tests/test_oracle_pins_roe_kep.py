"""Pins of the Harten-Hyman branch of the Roe solver and of Pirozzoli's two-point flux.

Roe + Harten-Hyman (Section 3.1.1, the convective interface flux): the oracle's
wave-by-wave Roe flux is compared with one built here from a numerical
eigen-decomposition of the flux Jacobian (torch autograd of the physical
flux, itself pinned by consistency) at the Roe-averaged state, whose Roe
property ``A (uR - uL) = f(uR) - f(uL)`` is checked first.  The states are
transonic rarefactions, so the entropy fix is active; a stationary expansion
shock shows that the fix is what removes the entropy-violating solution; the
flux is continuous where the fix switches on.

Pirozzoli's flux (Section 3.5): kinetic-energy preservation on a periodic
curved mesh (the kinetic-energy rate of the split-form DG operator equals a
pressure-work sum that does not involve the mass flux), and the textbook
identity between flux differencing with ``{rho}{v}{phi}`` products and the
Kennedy-Gruber split form, which fixes every component of the flux.
"""
import numpy as np
import pytest
import torch

from oracle import ops1d, physics, problem
from oracle.geometry import face_slice
from oracle.physics import Gas, entropy_vars, euler_flux, prim_to_cons, riemann, sound_speed, to_prim
from oracle.rhs import to_left, volume_term
from paper_2502_19342_amd import workloads as W

from oracle_cases import curved_mixed, smooth_state

T = torch.float64
G1 = Gas(nvar=5, gamma=1.4)


def cons(w):
    return prim_to_cons(torch.as_tensor(np.asarray(w, dtype=np.float64)[:, None], dtype=T), G1)


def normal_state(rho, un, ut1, ut2, p, n):
    """Conservative state with normal velocity ``un`` along ``n`` and two tangential parts."""
    nn = n / np.linalg.norm(n)
    t1 = np.cross(nn, [0.3, 1.0, 0.2])
    t1 /= np.linalg.norm(t1)
    t2 = np.cross(nn, t1)
    v = un * nn + ut1 * t1 + ut2 * t2
    return cons([rho, *v, p])


def roe_by_eigendecomposition(uL, uR, nvec, fix=True):
    """Roe flux F* s from eig of the Jacobian of f(u).n at the Roe-averaged state.

    Returns the flux, the Roe-property residual, and per acoustic wave
    (lambda~, lambda(uL), lambda(uR)) as speeds along the unit normal.
    """
    g = G1.gamma
    n = torch.as_tensor(np.asarray(nvec, dtype=np.float64)[:, None], dtype=T)
    s = float(torch.linalg.norm(n))
    qL, qR = to_prim(uL, G1), to_prim(uR, G1)
    wL, wR = torch.sqrt(qL.rho), torch.sqrt(qR.rho)
    v = (wL * qL.v + wR * qR.v) / (wL + wR)
    H = (wL * (qL.E + qL.p) / qL.rho + wR * (qR.E + qR.p) / qR.rho) / (wL + wR)
    rho = wL * wR
    p = rho * (g - 1.0) / g * (H - 0.5 * (v * v).sum(0))
    ut = prim_to_cons(torch.cat([rho[None], v, p[None]]), G1)[:, 0]

    def f(x):
        return euler_flux(to_prim(x[:, None], G1), n)[:, 0]

    A = torch.autograd.functional.jacobian(f, ut)
    du = (uR - uL)[:, 0]
    roe_res = float((A @ du - (f(uR[:, 0]) - f(uL[:, 0]))).abs().max())
    # the eigenvalue v.n is triple; LAPACK may return a complex basis for it,
    # which stays a basis only if it is kept complex
    lam, R = np.linalg.eig(A.numpy())
    lam = lam.real
    alam = np.abs(lam)
    nn = n[:, 0] / s
    vnL, vnR = float((qL.v[:, 0] * nn).sum()), float((qR.v[:, 0] * nn).sum())
    cL, cR = float(sound_speed(qL)), float(sound_speed(qR))
    waves = []
    for k, sg in ((int(np.argmin(lam)), -1.0), (int(np.argmax(lam)), 1.0)):
        lt, lL, lR = lam[k] / s, vnL + sg * cL, vnR + sg * cR
        waves.append((lt, lL, lR))
        delta = max(0.0, lt - lL, lR - lt)
        if fix and abs(lt) < delta:           # Harten-Hyman: |lam| -> (lam^2/delta + delta)/2
            alam[k] = 0.5 * (lt * lt / delta + delta) * s
    diss = (R @ np.diag(alam) @ np.linalg.solve(R, du.numpy().astype(complex))).real
    F = 0.5 * (f(uL[:, 0]) + f(uR[:, 0])).numpy() - 0.5 * diss
    return F, roe_res, waves


def entropy_production(uL, uR, F, nvec):
    """(w_R - w_L) . F* - (psi_R - psi_L) . n with psi = rho v; <= 0 for an entropy-stable flux."""
    wL, wR = entropy_vars(uL, G1)[:, 0].numpy(), entropy_vars(uR, G1)[:, 0].numpy()
    qL, qR = to_prim(uL, G1), to_prim(uR, G1)
    dpsi = float(((qR.rho * qR.v - qL.rho * qL.v)[:, 0] * torch.as_tensor(nvec, dtype=T)).sum())
    return float((wR - wL) @ F) - dpsi


TRANSONIC = [  # (rho, u_n, u_t1, u_t2, p) left / right: lam_1(uL) < 0 < lam_1(uR)
    ((1.0, 0.5, 0.1, -0.2, 1.0), (0.5, 2.0, 0.3, 0.1, 0.5)),
    ((1.0, 0.2, 0.0, 0.4, 1.0), (0.3, 1.9, -0.2, 0.0, 0.2)),
    ((1.0, 0.75, 0.2, 0.2, 1.0), (0.125, 1.8, 0.0, -0.3, 0.1)),
    ((0.4, -2.0, 0.1, 0.0, 0.3), (1.0, -0.4, 0.0, 0.1, 1.0)),      # wave 5: lam_5(uL) < 0 < lam_5(uR)
]


@pytest.mark.parametrize("left,right", TRANSONIC)
def test_roe_harten_hyman_on_transonic_rarefactions(left, right):
    nvec = np.array([0.6, 0.0, 0.8]) * 1.7
    uL, uR = normal_state(*left, nvec), normal_state(*right, nvec)
    F_ref, roe_res, waves = roe_by_eigendecomposition(uL, uR, nvec)
    assert roe_res <= 1e-13
    # the fix is active on one acoustic wave: lam(uL) < 0 < lam(uR) and |lam~| < delta
    active = []
    for lt, lL, lR in waves:
        delta = max(0.0, lt - lL, lR - lt)
        active.append(lL < 0.0 < lR and abs(lt) < delta)
    assert any(active)
    n = torch.as_tensor(nvec[:, None], dtype=T)
    F = riemann(0, uL, uR, n, G1)[:, 0].numpy()
    assert np.abs(F - F_ref).max() <= 1e-13 * max(1.0, np.abs(F_ref).max())
    F_nofix, _, _ = roe_by_eigendecomposition(uL, uR, nvec, fix=False)
    assert np.abs(F - F_nofix).max() > 1e-3                      # the fix changes the flux here
    assert entropy_production(uL, uR, F, nvec) <= 0.0


def test_roe_harten_hyman_removes_the_expansion_shock():
    # A Mach-2 normal shock with its two states swapped is a stationary expansion
    # shock: f(uL) = f(uR) and lam~_1 = 0.  Plain Roe keeps it (no dissipation, entropy
    # produced); with the fix the flux dissipates.
    g, M = 1.4, 2.0
    r2 = (g + 1) * M * M / ((g - 1) * M * M + 2)
    p2 = 1 + 2 * g / (g + 1) * (M * M - 1)
    u1 = M * np.sqrt(g)
    nvec = np.array([1.0, 0.0, 0.0])
    uL, uR = cons([r2, u1 / r2, 0, 0, p2]), cons([1.0, u1, 0, 0, 1.0])
    n = torch.as_tensor(nvec[:, None], dtype=T)
    assert float((euler_flux(to_prim(uL, G1), n) - euler_flux(to_prim(uR, G1), n)).abs().max()) <= 1e-14
    F_ref, _, waves = roe_by_eigendecomposition(uL, uR, nvec)
    assert abs(waves[0][0]) <= 1e-14
    F_nofix, _, _ = roe_by_eigendecomposition(uL, uR, nvec, fix=False)
    F = riemann(0, uL, uR, n, G1)[:, 0].numpy()
    assert np.abs(F - F_ref).max() <= 1e-13 * np.abs(F_ref).max()
    assert entropy_production(uL, uR, F_nofix, nvec) > 0.1          # plain Roe: entropy violation
    assert entropy_production(uL, uR, F, nvec) < -0.1


def test_roe_harten_hyman_is_continuous_where_the_fix_switches():
    # family uR(t): the right normal velocity t; the fix switches on wave 1 at some t*
    nvec = np.array([0.0, 1.0, 0.0])
    left = (1.0, 0.5, 0.2, 0.0, 1.0)

    def state_pair(t):
        return normal_state(*left, nvec), normal_state(0.5, t, 0.1, 0.0, 0.5, nvec)

    def active(t):
        uL, uR = state_pair(t)
        lt, lL, lR = roe_by_eigendecomposition(uL, uR, nvec)[2][0]
        return abs(lt) < max(0.0, lt - lL, lR - lt)

    lo, hi = 0.0, 2.0
    assert not active(lo) and active(hi)
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        lo, hi = (lo, mid) if active(mid) else (mid, hi)
    n = torch.as_tensor(nvec[:, None], dtype=T)
    eps = 1e-7
    Fa = riemann(0, *state_pair(lo - eps), n, G1)[:, 0].numpy()
    Fb = riemann(0, *state_pair(hi + eps), n, G1)[:, 0].numpy()
    # Lipschitz across the switch: the jump is of the order of the step, not of delta
    assert np.abs(Fa - Fb).max() <= 1e-5
    # at |lam~| = delta the replacement (lam~^2/delta + delta)/2 equals |lam~|, so the
    # fixed and the plain Roe flux agree there
    uL, uR = state_pair(hi)
    F_nofix, _, _ = roe_by_eigendecomposition(uL, uR, nvec, fix=False)
    assert np.abs(riemann(0, uL, uR, n, G1)[:, 0].numpy() - F_nofix).max() <= 1e-6


# ---------------------------------------------------------------------------
# Pirozzoli's flux
# ---------------------------------------------------------------------------

def kinetic_energy_rate_and_pressure_work(wl, u):
    """sum omega J (v . R_rho v - |v|^2/2 R_rho) of the oracle's R, and the pressure-work sum.

    With a KEP two-point flux (momentum part f_rho {v} + {p} a) in the volume and
    at the faces, the terms carrying the mass flux cancel: SBP makes the
    symmetric volume part a boundary term, and at faces the two sides' parts
    cancel.  What remains is
      W = - sum_e sum_i omega_i sum_d sum_{m != i} 2 D_im {p}_im a_im . v_i
          - sum_faces sum_nodes omega_p omega_q {p} n . (v_L - v_R),
    with a_im = (Ja^d_i + Ja^d_m)/2 and n the left side's outward normal.
    """
    mesh, gas, f = problem.build(wl)
    R = f(u, torch.zeros(mesh.K, dtype=T))
    wJ = mesh.weights_flat() * mesh.jacobian_flat()
    q = to_prim(u, gas)
    ke = (wJ * ((q.v * R[1:4]).sum(0) - 0.5 * (q.v * q.v).sum(0) * R[0])).sum()
    Wv = torch.zeros((), dtype=T)
    Ws = torch.zeros((), dtype=T)
    for N, g in mesh.groups.items():
        U = mesh.gather(u, N)                                  # [E, nvar, k, j, i]
        qq = to_prim(U.transpose(0, 1), gas)
        p, v = qq.p, qq.v                                      # [E,k,j,i], [3,E,k,j,i]
        w1 = g.w
        w3 = w1[:, None, None] * w1[None, :, None] * w1[None, None, :]
        D2 = 2.0 * g.D * (1.0 - torch.eye(N + 1, dtype=T))
        for d in range(3):
            dim = 3 - d                                        # axis of xi_{d+1} in [E,k,j,i]
            pm = torch.movedim(p, dim, -1)
            vm = torch.movedim(v, dim + 1, -1)
            Am = torch.movedim(g.Ja[:, d].transpose(0, 1), dim + 1, -1)   # [3,E,...,n]
            pbar = 0.5 * (pm[..., :, None] + pm[..., None, :])
            a = 0.5 * (Am[..., :, None] + Am[..., None, :])
            av = (a * vm[..., :, None]).sum(0)                 # a_im . v_i
            term = torch.einsum("...im,im->...i", pbar * av, D2)
            Wv = Wv - (torch.movedim(term, -1, dim) * w3).sum()
        del U
    faces = mesh.faces
    for fi in range(len(faces)):
        eL, sL, eR, sR, o = (int(x) for x in faces[fi])
        NL = int(mesh.degree[eL])
        gL, gR = mesh.groups[NL], mesh.groups[int(mesh.degree[eR])]
        sl, sr = int(mesh.slot[eL]), int(mesh.slot[eR])
        tL = face_slice(mesh.gather(u, NL)[sl], sL)
        tR = to_left(face_slice(mesh.gather(u, int(mesh.degree[eR]))[sr], sR), o)
        qL, qR = to_prim(tL, gas), to_prim(tR, gas)
        nvec = gL.outward_normal(sL)[sl]
        wf = gL.w[:, None] * gL.w[None, :]
        Ws = Ws - (wf * 0.5 * (qL.p + qR.p) * (nvec * (qL.v - qR.v)).sum(0)).sum()
        del gR
    return float(ke), float(Wv + Ws), float(Wv.abs() + Ws.abs())


def _kep_case(volume_flux):
    wl = curved_mixed(n=3, nmin=3, nmax=3, scramble=41, volume_flux=volume_flux, face_dg=W.RIEMANN_EC,
                      metric_degree=3)
    mesh, gas, _ = problem.build(wl)
    u = problem.initial_state(mesh, gas, smooth_state(43))
    return wl, u


def test_pirozzoli_kinetic_energy_balance_on_curved_periodic_mesh():
    wl, u = _kep_case(W.VOL_PIROZZOLI)
    ke, work, scale = kinetic_energy_rate_and_pressure_work(wl, u)
    assert scale > 1e-2
    assert abs(ke - work) <= 1e-13 * scale


def test_kinetic_energy_balance_fails_without_the_kep_structure(monkeypatch):
    # a mistake planted in the oracle: the momentum flux takes the left velocity
    # instead of the mean, f_rho v_L + {p} a (consistent, symmetric in the mass part)
    wl, u = _kep_case(W.VOL_PIROZZOLI)

    def wrong(qL, qR, a):
        rho_bar = 0.5 * (qL.rho + qR.rho)
        vbar = 0.5 * (qL.v + qR.v)
        pbar = 0.5 * (qL.p + qR.p)
        Hbar = 0.5 * ((qL.E + qL.p) / qL.rho + (qR.E + qR.p) / qR.rho)
        f_rho = rho_bar * (vbar * a).sum(0)
        vs = 0.5 * (qL.v * qL.rho + qR.v * qR.rho) / rho_bar   # density-weighted mean: not KEP
        return torch.stack([f_rho] + [f_rho * vs[d] + pbar * a[d] for d in range(3)] + [f_rho * Hbar])

    monkeypatch.setattr(physics, "flux_pirozzoli", wrong)
    ke, work, scale = kinetic_energy_rate_and_pressure_work(wl, u)
    assert abs(ke - work) > 1e-6 * scale
    monkeypatch.undo()
    # and the central flux (not KEP) fails it as well
    wl2, u2 = _kep_case(W.VOL_CENTRAL)
    ke, work, scale = kinetic_energy_rate_and_pressure_work(wl2, u2)
    assert abs(ke - work) > 1e-6 * scale


def test_pirozzoli_flux_differencing_equals_kennedy_gruber_split_form():
    # On an element with constant metric a, flux differencing with the products
    # {a}{b} and {a}{b}{c} equals the quadratic and cubic split forms:
    #   sum_m 2 D_im {a}{b}_im       = (a D b + b D a + D(ab)) / 2
    #   sum_m 2 D_im {a}{b}{c}_im    = (ab Dc + ac Db + bc Da + a D(bc) + b D(ac) + c D(ab) + D(abc)) / 4
    #   sum_m 2 D_im {p}_im          = D p
    # (sums over all m; the oracle leaves out m = i, whose term is 2 D_ii f(u_i).a).
    gas = Gas(nvar=6, kappa=(1.4, 1.41), R=(287.0, 4124.0))
    N = 4
    n = N + 1
    rng = np.random.default_rng(5)
    rho = 1 + 0.3 * rng.uniform(-1, 1, (n, n, n))
    vel = rng.uniform(-1, 1, (3, n, n, n))
    p = 1 + 0.3 * rng.uniform(-1, 1, (n, n, n))
    Y = rng.uniform(0.1, 0.9, (n, n, n))
    U = prim_to_cons(torch.as_tensor(np.stack([rho, *vel, p, Y])), gas)[None]   # [1,nvar,k,j,i]
    a_dir = torch.tensor([0.7, -0.2, 1.3], dtype=T)
    Ja = torch.zeros(1, 3, 3, n, n, n, dtype=T)
    Ja[0, 0] = a_dir[:, None, None, None]                      # only xi_1 carries a metric
    D = torch.as_tensor(ops1d.dmat(N), dtype=T)
    vol = volume_term(U, Ja, D, gas, 1)[0]                     # [nvar,k,j,i]
    q = to_prim(U[0], gas)
    diag = euler_flux(q, a_dir[:, None, None, None].expand(3, n, n, n))
    vol = vol + 2.0 * torch.diagonal(D)[None, None, None, :] * diag   # add the m = i terms

    def Dx(f):                                                 # derivative along xi_1 (last dim)
        return torch.einsum("im,...m->...i", D, f)

    vn = (q.v * a_dir[:, None, None, None]).sum(0)
    H = (q.E + q.p) / q.rho

    def quad(x, y):
        return 0.5 * (x * Dx(y) + y * Dx(x) + Dx(x * y))

    def cubic(x, y, z):
        return 0.25 * (x * y * Dx(z) + x * z * Dx(y) + y * z * Dx(x) + x * Dx(y * z) + y * Dx(x * z)
                       + z * Dx(x * y) + Dx(x * y * z))

    ref = [quad(q.rho, vn)]
    ref += [cubic(q.rho, vn, q.v[c]) + a_dir[c] * Dx(q.p) for c in range(3)]
    ref += [cubic(q.rho, vn, H), cubic(q.rho, vn, q.Y)]
    ref = torch.stack(ref)
    assert float((vol - ref).abs().max()) <= 1e-12 * float(ref.abs().max())
