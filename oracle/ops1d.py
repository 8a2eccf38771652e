"""One-dimensional operators of the DGSEM and the FV sub-cell maps (oracle).

Test infrastructure: a plain, slow reference.  Only the tests, the smoke check
and the benchmark's CPU-baseline leg use it.

Everything here is computed in 40-digit arithmetic (mpmath) and rounded once
to float64.

* Legendre-Gauss-Lobatto nodes and weights, the Lagrange basis and its
  nodal derivative matrix ``D_ij = l_j'(xi_i)`` (Section 3.1.1, the collocated
  tensor-product DGSEM, eq. dgsem_abbrev).
* The orthonormal Legendre Vandermonde ``V_Leg`` used by the modal indicator
  (Section 3.4, eq. solution_expansion).
* ``V^{N->M}``: interpolation to a higher degree; ``V^{M->N}``: the modal L2
  projection to a lower degree (Section 3.2, the degree-change maps).
* ``V^{DG->FV}``: sub-cell integral means of the Lagrange basis on an
  equidistant ``N_FV`` grid, and ``V^{FV->DG}`` its pseudo-inverse
  (Section 3.2, the DG/FV switching maps).
* ``I^{face}``: the Lagrange basis evaluated at the ``N_FV + 1`` sub-cell
  interfaces (used for sub-cell face normals).
"""
from __future__ import annotations

import functools

import mpmath as mp
import numpy as np

mp.mp.dps = 40


def _legendre(n: int, x):
    """P_n(x) and P_n'(x) by the three-term recurrence."""
    if n == 0:
        return mp.mpf(1), mp.mpf(0)
    p0, p1 = mp.mpf(1), x
    for k in range(2, n + 1):
        p0, p1 = p1, ((2 * k - 1) * x * p1 - (k - 1) * p0) / k
    # derivative from (x^2 - 1) P_n' = n (x P_n - P_{n-1})
    if abs(x) == 1:
        dp = mp.mpf(n * (n + 1)) / 2 * (x ** (n + 1))
    else:
        dp = n * (x * p1 - p0) / (x * x - 1)
    return p1, dp


@functools.lru_cache(maxsize=None)
def lgl_mp(N: int):
    """LGL nodes (ascending) and weights in mp precision."""
    if N < 1:
        raise ValueError("N >= 1")
    x = [mp.mpf(-1)]
    for j in range(1, N):
        # interior nodes are the roots of P_N'; Newton from Chebyshev-Lobatto guesses
        z = -mp.cos(mp.pi * j / N)
        for _ in range(100):
            p, dp = _legendre(N, z)
            ddp = (2 * z * dp - N * (N + 1) * p) / (1 - z * z)
            dz = dp / ddp
            z -= dz
            if abs(dz) < mp.mpf(10) ** (-38):
                break
        x.append(z)
    x.append(mp.mpf(1))
    w = []
    for xi in x:
        p, _ = _legendre(N, xi)
        w.append(mp.mpf(2) / (N * (N + 1) * p * p))
    return x, w


def _bary_weights(x):
    n = len(x)
    return [1 / mp.fprod(x[j] - x[k] for k in range(n) if k != j) for j in range(n)]


def _lagrange_row(x, t):
    """[l_0(t), ..., l_N(t)] for nodes x."""
    n = len(x)
    row = []
    for j in range(n):
        v = mp.mpf(1)
        for k in range(n):
            if k != j:
                v *= (t - x[k]) / (x[j] - x[k])
        row.append(v)
    return row


def _f64(rows) -> np.ndarray:
    return np.array([[float(v) for v in r] for r in rows], dtype=np.float64)


@functools.lru_cache(maxsize=None)
def lgl(N: int):
    """(nodes, weights) as float64 arrays."""
    x, w = lgl_mp(N)
    return np.array([float(v) for v in x]), np.array([float(v) for v in w])


@functools.lru_cache(maxsize=None)
def dmat_mp(N: int):
    x, _ = lgl_mp(N)
    bw = _bary_weights(x)
    n = N + 1
    D = [[mp.mpf(0)] * n for _ in range(n)]
    for i in range(n):
        for j in range(n):
            if i != j:
                D[i][j] = (bw[j] / bw[i]) / (x[i] - x[j])
        D[i][i] = -mp.fsum(D[i][j] for j in range(n) if j != i)
    return D


@functools.lru_cache(maxsize=None)
def dmat(N: int) -> np.ndarray:
    """Nodal derivative matrix D_ij = l_j'(xi_i) (eq. dgsem_abbrev)."""
    return _f64(dmat_mp(N))


@functools.lru_cache(maxsize=None)
def vleg_mp(N: int):
    x, _ = lgl_mp(N)
    rows = []
    for xi in x:
        r = []
        for j in range(N + 1):
            p, _ = _legendre(j, xi)
            r.append(mp.sqrt(mp.mpf(2 * j + 1) / 2) * p)
        rows.append(r)
    return mp.matrix(rows)


@functools.lru_cache(maxsize=None)
def vleg(N: int) -> np.ndarray:
    """V_Leg[i, j] = orthonormal Legendre polynomial j at LGL node i."""
    m = vleg_mp(N)
    return _f64(m.tolist())


@functools.lru_cache(maxsize=None)
def vleg_inv(N: int) -> np.ndarray:
    """Nodal -> modal map (inverse of V_Leg)."""
    return _f64((vleg_mp(N) ** -1).tolist())


@functools.lru_cache(maxsize=None)
def interp(N: int, M: int) -> np.ndarray:
    """V^{N->M}[i, j] = l^N_j(xi^M_i): evaluate a degree-N nodal polynomial at degree-M nodes."""
    xN, _ = lgl_mp(N)
    xM, _ = lgl_mp(M)
    return _f64([_lagrange_row(xN, t) for t in xM])


def _ld(rows) -> np.ndarray:
    return np.array([[np.longdouble(mp.nstr(v, 30)) for v in r] for r in rows], dtype=np.longdouble)


@functools.lru_cache(maxsize=None)
def lgl_ld(N: int) -> np.ndarray:
    """LGL nodes in long double (for metric terms rounded once)."""
    x, _ = lgl_mp(N)
    return _ld([x])[0]


@functools.lru_cache(maxsize=None)
def dmat_ld(N: int) -> np.ndarray:
    """D in long double."""
    return _ld(dmat_mp(N))


@functools.lru_cache(maxsize=None)
def interp_ld(N: int, M: int) -> np.ndarray:
    """V^{N->M} in long double."""
    xN, _ = lgl_mp(N)
    xM, _ = lgl_mp(M)
    return _ld([_lagrange_row(xN, t) for t in xM])


@functools.lru_cache(maxsize=None)
def project(M: int, N: int) -> np.ndarray:
    """V^{M->N} for M > N: modal L2 truncation of a degree-M nodal polynomial to degree N."""
    if M < N:
        raise ValueError("projection needs M >= N")
    trunc = mp.zeros(N + 1, M + 1)
    for i in range(N + 1):
        trunc[i, i] = 1
    P = vleg_mp(N) * trunc * (vleg_mp(M) ** -1)
    return _f64(P.tolist())


def _poly_from_roots(roots):
    """Monomial coefficients (ascending) of prod (t - r)."""
    c = [mp.mpf(1)]
    for r in roots:
        nc = [mp.mpf(0)] * (len(c) + 1)
        for k, ck in enumerate(c):
            nc[k + 1] += ck
            nc[k] -= r * ck
        c = nc
    return c


def _integral(coef, a, b):
    return mp.fsum(ck * (b ** (k + 1) - a ** (k + 1)) / (k + 1) for k, ck in enumerate(coef))


@functools.lru_cache(maxsize=None)
def dg2fv_mp(N: int, NFV: int):
    x, _ = lgl_mp(N)
    h = mp.mpf(2) / NFV
    rows = []
    for s in range(NFV):
        a, b = -1 + s * h, -1 + (s + 1) * h
        r = []
        for j in range(N + 1):
            others = [x[k] for k in range(N + 1) if k != j]
            scale = mp.fprod(x[j] - xk for xk in others)
            r.append(_integral(_poly_from_roots(others), a, b) / scale / h)
        rows.append(r)
    return mp.matrix(rows)


@functools.lru_cache(maxsize=None)
def dg2fv(N: int, NFV: int) -> np.ndarray:
    """V^{DG->FV}[s, j]: mean of l_j over sub-cell s of width h = 2/NFV."""
    return _f64(dg2fv_mp(N, NFV).tolist())


@functools.lru_cache(maxsize=None)
def fv2dg(N: int, NFV: int) -> np.ndarray:
    """V^{FV->DG}: Moore-Penrose pseudo-inverse of V^{DG->FV} (NFV >= N+1)."""
    if NFV < N + 1:
        raise ValueError("NFV >= N+1 required")
    V = dg2fv_mp(N, NFV)
    P = ((V.T * V) ** -1) * V.T
    return _f64(P.tolist())


@functools.lru_cache(maxsize=None)
def face_interp(N: int, NFV: int) -> np.ndarray:
    """I[q, j] = l_j(-1 + q h), q = 0..NFV: basis values at the sub-cell interfaces."""
    x, _ = lgl_mp(N)
    h = mp.mpf(2) / NFV
    return _f64([_lagrange_row(x, -1 + q * h) for q in range(NFV + 1)])


# ---------------------------------------------------------------------------
# mortars (Section 3.2.3): a big side and its two halves along one direction
# ---------------------------------------------------------------------------
@functools.lru_cache(maxsize=None)
def mortar_interp(N: int, k: int) -> np.ndarray:
    """``M_{0k}[i, j] = l_j((s_i + 2k - 1) / 2)``: the big side's degree-N polynomial at the
    degree-N nodes ``s_i`` of its half ``k`` (0: [-1, 0], 1: [0, 1]) in the half's own coordinate."""
    x, _ = lgl_mp(N)
    return _f64([_lagrange_row(x, (t + 2 * k - 1) / 2) for t in x])


@functools.lru_cache(maxsize=None)
def mortar_project(N: int, k: int) -> np.ndarray:
    """``M_{k0}``: the big side's share of a degree-N polynomial ``F_k`` given on half ``k``.

    The big side's flux is the L2 projection onto degree N over [-1, 1] of the
    function that equals ``2 F_k`` on half k (the half's surface element is half
    the big side's, so its flux per unit of its own length is half), zero on the
    other half: with Legendre polynomials ``L_j``,
    ``c_j = (2j + 1)/2 int_{-1}^{1} F_k(s) L_j((s + 2k - 1)/2) ds``,
    ``F_0(xi_i) = sum_j c_j L_j(xi_i)``.  Summed over both halves this projects
    the piecewise flux; it keeps ``sum_i w_i F_0`` equal to the halves' sums,
    and ``(M_{00} M_{00} + M_{10} M_{01}) / 2`` (projection after interpolation
    to each half) is the identity: a big-side polynomial comes back.
    """
    x, _ = lgl_mp(N)
    n = N + 1
    gx, gw = _gauss_legendre(n + 1)                  # exact for the degree-2N integrands
    C = [[mp.mpf(0)] * n for _ in range(n)]          # C[j][l] = (2j+1)/2 int l_l(s) L_j(...) ds
    for s, w in zip(gx, gw):
        lrow = _lagrange_row(x, s)
        t = (s + 2 * k - 1) / 2
        for j in range(n):
            pj, _ = _legendre(j, t)
            f = mp.mpf(2 * j + 1) / 2 * w * pj
            for l in range(n):
                C[j][l] += f * lrow[l]
    rows = []
    for xi in x:
        Lrow = [_legendre(j, xi)[0] for j in range(n)]
        rows.append([sum(Lrow[j] * C[j][l] for j in range(n)) for l in range(n)])
    return _f64(rows)


def _gauss_legendre(m: int):
    """Nodes and weights of the m-point Gauss-Legendre rule (Newton on P_m)."""
    xs, ws = [], []
    for i in range(1, m + 1):
        z = mp.cos(mp.pi * (i - mp.mpf(1) / 4) / (m + mp.mpf(1) / 2))
        for _ in range(100):
            p, dp = _legendre(m, z)
            dz = p / dp
            z -= dz
            if abs(dz) < mp.mpf(10) ** (-35):
                break
        p, dp = _legendre(m, z)
        xs.append(z)
        ws.append(2 / ((1 - z * z) * dp * dp))
    return xs, ws


def _overlap_half(NFV: int, k: int) -> np.ndarray:
    """[j, i] = length of the overlap of sub-face j of half k with sub-face i of the big side,
    over the length of sub-face j (both on the big side's axis, in units of its sub-faces)."""
    A = np.zeros((NFV, NFV))
    for j in range(NFV):
        lo = (j + k * NFV) / 2.0
        hi = lo + 0.5
        for i in range(NFV):
            A[j, i] = max(0.0, min(hi, i + 1.0) - max(lo, float(i))) / 0.5
    return A


@functools.lru_cache(maxsize=None)
def mortar_fv_interp(NFV: int, k: int) -> np.ndarray:
    """``M^FV_{0k}``: the mean of the big side's piecewise-constant sub-face data over each
    sub-face of half k (a copy when N_FV is even: every sub-face of the half lies in one of the big side's)."""
    return _overlap_half(NFV, k)


@functools.lru_cache(maxsize=None)
def mortar_fv_project(NFV: int, k: int) -> np.ndarray:
    """``M^FV_{k0}``: sub-face fluxes of half k (integrated over its sub-faces) summed into the
    big side's sub-faces, each by the fraction of it that lies there."""
    return _overlap_half(NFV, k).T.copy()
