"""Element geometry of the oracle: trilinear map, nodes, metric terms.

Test infrastructure: a plain, slow reference.  Only the tests, the smoke check
and the benchmark's CPU-baseline leg use it.

Section 3.1.1 maps each hexahedron to the reference cube and writes the
equations with the Jacobian determinant and the contravariant flux.  The
contravariant basis ``Ja^d`` (``J`` times the contravariant vector ``a^d``)
is built here in Kopriva's conservative curl form,
``Ja^d_n = -( curl_xi ( X_l grad_xi X_m ) )_d`` with ``(n, m, l)`` cyclic.
Two constructions are offered:

* one mesh-wide degree ``N_J`` (``metric_degree >= 1``): the curl form on the
  degree-``N_J`` nodes, interpolated exactly to every element degree; a
  divergence-free polynomial of degree ``N_J``, identical on both sides of
  every face, but only as accurate as degree ``N_J``;
* per element (``metric_degree = 0``): the curl form at the element's own
  degree ``N``.  Free-stream preservation needs the face normal, the
  tangential curl of ``W = X_l grad X_m`` on the face, to be the same
  polynomial on both sides.  On a face shared with a neighbour of lower
  degree ``N_f`` the tangential components of ``W`` on the face are therefore
  replaced by their degree-``N_f`` interpolant before the curl is taken; the
  neighbour's own curl sees the same interpolant.  For trilinear elements the
  component of ``W`` along an edge is linear along that edge, so two faces of
  one element never ask for different values on their common edge.  The
  volume field stays the curl of a polynomial, hence divergence-free, and is
  exact wherever ``N, N_f >= 2`` (``W`` has degree <= 2 in each variable).

``J`` is evaluated pointwise from the trilinear map.

Array layout: node arrays are ``[..., k, j, i]`` with ``i`` (xi1) fastest.
"""
from __future__ import annotations

import numpy as np
import torch

from . import ops1d

T = torch.float64


def _t(a) -> torch.Tensor:
    return torch.as_tensor(np.asarray(a), dtype=T)


def apply_axis(A: torch.Tensor, f: torch.Tensor, axis: int) -> torch.Tensor:
    """Contract a 1D matrix ``A[r, c]`` with reference axis ``axis`` of ``f[..., k, j, i]``.

    axis 0 is xi1 (last dim), 1 is xi2, 2 is xi3.
    """
    dim = f.dim() - 1 - axis
    f = torch.movedim(f, dim, -1)
    g = torch.matmul(f, A.T)
    return torch.movedim(g, -1, dim)


def apply3(A: torch.Tensor, f: torch.Tensor) -> torch.Tensor:
    """Tensor-product map ``A (x) A (x) A`` on the last three dims."""
    for ax in range(3):
        f = apply_axis(A, f, ax)
    return f


def _apply_axis_ld(A: np.ndarray, f: np.ndarray, axis: int) -> np.ndarray:
    """:func:`apply_axis` for long-double numpy arrays."""
    dim = f.ndim - 1 - axis
    g = np.moveaxis(f, dim, -1) @ A.T
    return np.moveaxis(g, -1, dim)


def trilinear_grid_ld(corners: np.ndarray, x0, x1, x2):
    """Position ``X[E, 3, n2, n1, n0]`` and ``dX_n/dxi_a`` as ``G[E, 3, 3, n2, n1, n0]``
    of the trilinear map on the tensor grid of 1D reference points (long double)."""
    LD = np.longdouble
    xs = [np.asarray(x, dtype=LD).reshape(-1) for x in (x0, x1, x2)]
    phi = [np.stack([(1 - x) / 2, (1 + x) / 2]) for x in xs]
    dphi = [np.stack([np.full_like(x, -0.5), np.full_like(x, 0.5)]) for x in xs]
    E = corners.shape[0]
    shp = (len(xs[2]), len(xs[1]), len(xs[0]))
    X = np.zeros((E, 3) + shp, dtype=LD)
    G = np.zeros((E, 3, 3) + shp, dtype=LD)
    for c in range(8):
        b = (c & 1, (c >> 1) & 1, (c >> 2) & 1)
        w = phi[2][b[2]][:, None, None] * phi[1][b[1]][None, :, None] * phi[0][b[0]][None, None, :]
        X += corners[:, c, :, None, None, None] * w
        for a in range(3):
            f = [dphi[d][b[d]] if d == a else phi[d][b[d]] for d in range(3)]
            wa = f[2][:, None, None] * f[1][None, :, None] * f[0][None, None, :]
            G[:, :, a] += corners[:, c, :, None, None, None] * wa
    return X, G


def curl_metrics_matched(corners: torch.Tensor, N: int, nbr_degree: np.ndarray) -> torch.Tensor:
    """Per-element curl-form metrics ``Ja[E, d, n, k, j, i]`` at degree ``N`` whose face
    normals match the neighbours' (module docstring).  Formed in long double and
    rounded once, so that the two sides of a face hold the same normal to rounding.

    ``nbr_degree[E, 6]``: degree of the element across each side.
    """
    LD = np.longdouble
    c = np.asarray(corners.numpy(), dtype=LD)
    x = ops1d.lgl_ld(N)
    D = ops1d.dmat_ld(N)
    E = c.shape[0]
    X, _ = trilinear_grid_ld(c, x, x, x)                       # [E,3,n,n,n]
    Ja = np.zeros((E, 3, 3, N + 1, N + 1, N + 1), dtype=LD)
    nbr_degree = np.asarray(nbr_degree)
    for nn in range(3):
        m, l = (nn + 1) % 3, (nn + 2) % 3
        W = [X[:, l] * _apply_axis_ld(D, X[:, m], a) for a in range(3)]
        for side in range(6):
            d, end = side // 2, LD(2 * (side % 2) - 1)
            idx = -1 if side % 2 else 0
            for Nf in sorted(set(nbr_degree[:, side].tolist())):
                if Nf >= N:
                    continue
                sel = np.nonzero(nbr_degree[:, side] == Nf)[0]
                xf = ops1d.lgl_ld(Nf)
                grid = [xf, xf, xf]
                grid[d] = np.array([end], dtype=LD)
                Xf, Gf = trilinear_grid_ld(c[sel], *grid)    # points of the degree-Nf face grid
                Vf = ops1d.interp_ld(Nf, N)
                for a in range(3):
                    if a == d:
                        continue
                    Wf = Xf[:, l] * Gf[:, m, a]              # [e, ...] with axis d of length 1
                    Wf = Wf[..., 0] if d == 0 else (Wf[..., 0, :] if d == 1 else Wf[:, 0])   # [e, q, p]
                    Wn = _apply_axis_ld(Vf, _apply_axis_ld(Vf, Wf, 0), 1)   # interpolant at the N nodes
                    if d == 0:
                        W[a][sel, ..., idx] = Wn
                    elif d == 1:
                        W[a][sel, ..., idx, :] = Wn
                    else:
                        W[a][sel, idx] = Wn
        curl = [_apply_axis_ld(D, W[2], 1) - _apply_axis_ld(D, W[1], 2),
                _apply_axis_ld(D, W[0], 2) - _apply_axis_ld(D, W[2], 0),
                _apply_axis_ld(D, W[1], 0) - _apply_axis_ld(D, W[0], 1)]
        for d in range(3):
            Ja[:, d, nn] = -curl[d]
    return torch.as_tensor(Ja.astype(np.float64))


def trilinear(corners: torch.Tensor, xi: torch.Tensor) -> torch.Tensor:
    """Physical coordinates ``[E, 3, n, n, n]`` of the reference points ``xi`` (per axis)."""
    phi = torch.stack([(1 - xi) / 2, (1 + xi) / 2])            # [2, n]
    E = corners.shape[0]
    n = xi.shape[0]
    X = torch.zeros(E, 3, n, n, n, dtype=T)
    for c in range(8):
        b0, b1, b2 = c & 1, (c >> 1) & 1, (c >> 2) & 1
        w = phi[b2][:, None, None] * phi[b1][None, :, None] * phi[b0][None, None, :]
        X += corners[:, c, :, None, None, None] * w
    return X


def trilinear_jacobian(corners: torch.Tensor, xi: torch.Tensor) -> torch.Tensor:
    """``dX_n / dxi_a`` as ``[E, 3 (n), 3 (a), n, n, n]``."""
    phi = torch.stack([(1 - xi) / 2, (1 + xi) / 2])
    dphi = torch.stack([torch.full_like(xi, -0.5), torch.full_like(xi, 0.5)])
    E = corners.shape[0]
    n = xi.shape[0]
    G = torch.zeros(E, 3, 3, n, n, n, dtype=T)
    for c in range(8):
        b = (c & 1, (c >> 1) & 1, (c >> 2) & 1)
        for a in range(3):
            f = [dphi[b[d]] if d == a else phi[b[d]] for d in range(3)]
            w = f[2][:, None, None] * f[1][None, :, None] * f[0][None, None, :]
            G[:, :, a] += corners[:, c, :, None, None, None] * w
    return G


def curl_metrics(corners: torch.Tensor, NJ: int) -> torch.Tensor:
    """``Ja[E, d, n, k, j, i]`` on the degree-``NJ`` LGL nodes, conservative curl form."""
    xJ, _ = ops1d.lgl(NJ)
    D = _t(ops1d.dmat(NJ))
    X = trilinear(corners, _t(xJ))                             # [E,3,..]
    Ja = torch.zeros(corners.shape[0], 3, 3, NJ + 1, NJ + 1, NJ + 1, dtype=T)
    for n in range(3):
        m, l = (n + 1) % 3, (n + 2) % 3
        W = [X[:, l] * apply_axis(D, X[:, m], a) for a in range(3)]
        curl = [apply_axis(D, W[2], 1) - apply_axis(D, W[1], 2),
                apply_axis(D, W[0], 2) - apply_axis(D, W[2], 0),
                apply_axis(D, W[1], 0) - apply_axis(D, W[0], 1)]
        for d in range(3):
            Ja[:, d, n] = -curl[d]
    return Ja


def face_slice(f: torch.Tensor, side: int) -> torch.Tensor:
    """Trace of ``f[..., k, j, i]`` on a side, as ``[..., q, p]`` (p along the lower tangential axis)."""
    d, last = side // 2, side % 2
    idx = -1 if last else 0
    if d == 0:
        return f[..., :, :, idx]          # [k, j] = [q, p]
    if d == 1:
        return f[..., :, idx, :]          # [k, i]
    return f[..., idx, :, :]              # [j, i]


class ElementGroup:
    """All elements of one polynomial degree, with their geometry at that degree."""

    def __init__(self, N: int, elems: np.ndarray, corners: torch.Tensor, NJ: int,
                 nbr_degree: np.ndarray | None = None):
        self.N = N
        self.elems = torch.as_tensor(elems, dtype=torch.long)
        x, w = ops1d.lgl(N)
        self.x = _t(x)
        self.w = _t(w)
        self.D = _t(ops1d.dmat(N))
        c = corners[self.elems]
        self.X = trilinear(c, self.x)                           # [E,3,n,n,n]
        if NJ == 0:                                             # per element, matched faces
            self.Ja = curl_metrics_matched(c, N, nbr_degree[elems])
        else:
            JaJ = curl_metrics(c, NJ)
            V = _t(ops1d.interp(NJ, N))
            self.Ja = apply3(V, JaJ)                            # [E,3,3,n,n,n]
        G = trilinear_jacobian(c, self.x)                       # [E,3,3,...]
        self.J = torch.linalg.det(G.permute(0, 3, 4, 5, 1, 2))  # [E,n,n,n]
        if torch.any(self.J <= 0):
            raise ValueError("non-positive Jacobian")

    def outward_normal(self, side: int) -> torch.Tensor:
        """``n s`` at the side's nodes: +-Ja^d restricted to the side, ``[E, 3, q, p]``."""
        d = side // 2
        sign = 1.0 if side % 2 else -1.0
        return sign * face_slice(self.Ja[:, d], side)


class OracleMesh:
    """Geometry of a whole mesh, grouped by element degree."""

    def __init__(self, spec, n_fv: int, metric_degree: int):
        self.spec = spec
        self.K = spec.n_elem
        self.degree = np.asarray(spec.degree, dtype=np.int64)
        self.n_fv = int(n_fv)
        self.NJ = int(metric_degree)                             # 0: per element (matched faces)
        if self.NJ < 0 or self.NJ > self.degree.min():
            raise ValueError("metric degree must be 0 or at most the lowest element degree")
        corners = _t(spec.corners)
        faces = np.asarray(spec.faces, dtype=np.int64)
        nbr = np.zeros((self.K, 6), dtype=np.int64)
        nbr[faces[:, 0], faces[:, 1]] = self.degree[faces[:, 2]]
        nbr[faces[:, 2], faces[:, 3]] = self.degree[faces[:, 0]]
        self.groups = {}
        for N in sorted(set(self.degree.tolist())):
            elems = np.nonzero(self.degree == N)[0]
            self.groups[N] = ElementGroup(N, elems, corners, self.NJ, nbr)
        self.slot = np.zeros(self.K, dtype=np.int64)            # position inside its group
        for N, g in self.groups.items():
            self.slot[g.elems.numpy()] = np.arange(len(g.elems))
        self.offset = spec.elem_offset()
        self.n_node = int(self.offset[-1])
        self.faces = np.asarray(spec.faces, dtype=np.int64)
        self.mortars = np.asarray(getattr(spec, "mortars", np.zeros((0, 15))), dtype=np.int64).reshape(-1, 15)
        if len(self.mortars) and self.NJ == 0:
            raise ValueError("meshes with mortars take a mesh-wide metric degree (metric_degree >= 1)")

    # ---- flat <-> grouped state ----------------------------------------
    def gather(self, u: torch.Tensor, N: int) -> torch.Tensor:
        """Flat ``[nvar, n_node]`` -> ``[E_N, nvar, n, n, n]`` for the degree-N group."""
        g = self.groups[N]
        n = N + 1
        idx = torch.as_tensor(self.offset[g.elems.numpy()], dtype=torch.long)
        ar = torch.arange(n ** 3)
        flat = (idx[:, None] + ar[None, :]).reshape(-1)
        v = u[:, flat].reshape(u.shape[0], len(idx), n, n, n)
        return v.permute(1, 0, 2, 3, 4)

    def scatter(self, parts: dict, nvar: int) -> torch.Tensor:
        """Inverse of :meth:`gather` for a dict ``{N: [E_N, nvar, n, n, n]}``."""
        out = [None] * self.K
        for N, val in parts.items():
            g = self.groups[N]
            for s, e in enumerate(g.elems.tolist()):
                out[e] = val[s].reshape(nvar, -1)
        return torch.cat(out, dim=1)

    def node_coords(self) -> torch.Tensor:
        """Physical coordinates of all nodes, flat ``[3, n_node]``."""
        return self.scatter({N: g.X for N, g in self.groups.items()}, 3)

    def jacobian_flat(self) -> torch.Tensor:
        return self.scatter({N: g.J[:, None] for N, g in self.groups.items()}, 1)[0]

    def weights_flat(self) -> torch.Tensor:
        """Tensor LGL weights omega_i omega_j omega_k per node, flat."""
        parts = {}
        for N, g in self.groups.items():
            w3 = g.w[None, None, :] * g.w[None, :, None] * g.w[:, None, None]
            parts[N] = w3.expand(len(g.elems), 1, N + 1, N + 1, N + 1)
        return self.scatter(parts, 1)[0]
