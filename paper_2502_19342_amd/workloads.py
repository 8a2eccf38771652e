"""Seeded synthetic workloads for the hybrid DG/FV right-hand side.

This module is shared by the tests, the benchmark and the oracle-side tests.
It holds none of the discretisation's arithmetic: no quadrature nodes,
metric terms, equation of state or fluxes.  It produces

* hexahedral meshes as trilinear element corners plus a face table
  ``(eL, sideL, eR, sideR, orient)``,
* a per-element polynomial degree,
* initial states as closed-form functions of the physical position, in
  primitive variables ``(rho, v1, v2, v3, p[, Y1])``, so that every consumer
  samples them at its own nodes,
* seeded noise and cotangent arrays.

Conventions (the interface format both implementations read):

* Elements of an ``n^3`` structured grid are numbered ``e = ix + n*(iy + n*iz)``.
* Corner ``c`` of an element sits at local coordinates
  ``xi_d = -1 + 2*bit_d(c)``, bit 0 for xi1, bit 1 for xi2, bit 2 for xi3.
* Side ``s`` is the face ``xi_{s//2} = -1`` (s even) or ``+1`` (s odd).
* A face's local grid indices are ``(p, q)``: ``p`` runs along the lower of
  the two tangential reference directions, ``q`` along the higher one.
* ``orient`` maps the left side's face index ``(p, q)`` to the right side's
  ``(p', q')`` on an ``n x n`` face grid: first ``(a, b) = (q, p)`` if bit 2
  is set, else ``(p, q)``; then ``p' = n-1-a`` if bit 0 is set, else ``a``,
  and ``q' = n-1-b`` if bit 1 is set, else ``b``.
"""
from __future__ import annotations

import dataclasses

import itertools
import math
from dataclasses import dataclass, field

import numpy as np

# ---------------------------------------------------------------------------
# meshes
# ---------------------------------------------------------------------------


@dataclass
class MeshSpec:
    """A conforming periodic hexahedral mesh (host arrays)."""

    n: int                      # elements per direction
    lo: np.ndarray              # box lower corner [3]
    hi: np.ndarray              # box upper corner [3]
    corners: np.ndarray         # [K, 8, 3] float64, physical corner positions
    faces: np.ndarray           # [F, 5] int32 (eL, sideL, eR, sideR, orient)
    degree: np.ndarray          # [K] int8
    rotation: np.ndarray = field(default=None)  # [K] int, index into ROTATIONS
    # non-conforming faces, one row per big side (see mortar_mesh):
    # (big element, big side, type, small elements[4], small sides[4], orientations[4])
    mortars: np.ndarray = field(default_factory=lambda: np.zeros((0, 15), dtype=np.int32))

    @property
    def n_elem(self) -> int:
        return int(self.corners.shape[0])

    @property
    def n_face(self) -> int:
        return int(self.faces.shape[0])

    def node_counts(self) -> np.ndarray:
        return (self.degree.astype(np.int64) + 1) ** 3

    def elem_offset(self) -> np.ndarray:
        off = np.zeros(self.n_elem + 1, dtype=np.int64)
        off[1:] = np.cumsum(self.node_counts())
        return off


def _proper_rotations() -> list[np.ndarray]:
    """The 24 signed permutation matrices with determinant +1."""
    rots = []
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product((1, -1), repeat=3):
            m = np.zeros((3, 3), dtype=np.int64)
            for r in range(3):
                m[r, perm[r]] = signs[r]
            if round(np.linalg.det(m)) == 1:
                rots.append(m)
    return rots


ROTATIONS = _proper_rotations()
assert len(ROTATIONS) == 24 and np.array_equal(ROTATIONS[0], np.eye(3, dtype=np.int64))


def orient_map(o: int, p: int, q: int, n: int) -> tuple[int, int]:
    """Face-grid index map of the orientation code (see module docstring)."""
    a, b = (q, p) if (o & 4) else (p, q)
    if o & 1:
        a = n - 1 - a
    if o & 2:
        b = n - 1 - b
    return a, b


def _local_face_corner(side: int, p: int, q: int) -> np.ndarray:
    """Local reference coordinates (+-1) of corner (p, q) in {0,1}^2 of a side."""
    d = side // 2
    t = [a for a in range(3) if a != d]
    xi = np.zeros(3, dtype=np.int64)
    xi[d] = 1 if side % 2 else -1
    xi[t[0]] = 2 * p - 1
    xi[t[1]] = 2 * q - 1
    return xi



def _scrambled_faces(n: int, cell: np.ndarray, rot: np.ndarray) -> list:
    """Face table of a grid whose elements carry rotated local frames."""
    K = cell.shape[0]
    faces = []

    def key(E, Rm, side, p, q):
        off = (Rm @ _local_face_corner(side, p, q) + 1) // 2
        return tuple(int(v) % n for v in cell[E] + off)

    for e in range(K):
        for X in range(3):
            nb = cell[e].copy()
            nb[X] = (nb[X] + 1) % n
            f = int(nb[0] + n * (nb[1] + n * nb[2]))
            RA, RB = ROTATIONS[rot[e]], ROTATIONS[rot[f]]
            dcan = np.zeros(3, dtype=np.int64)
            dcan[X] = 1
            # the canonical +X side of A and -X side of B in their local frames
            dA = RA.T @ dcan
            dB = RB.T @ (-dcan)
            sA = int(2 * np.argmax(np.abs(dA)) + (1 if dA.sum() > 0 else 0))
            sB = int(2 * np.argmax(np.abs(dB)) + (1 if dB.sum() > 0 else 0))
            cornA = {key(e, RA, sA, p, q): (p, q) for p in (0, 1) for q in (0, 1)}
            cornB = {(p, q): key(f, RB, sB, p, q) for p in (0, 1) for q in (0, 1)}
            found = None
            for o in range(8):
                if all(cornB[orient_map(o, p, q, 2)] == ka for ka, (p, q) in cornA.items()):
                    found = o
                    break
            if found is None:
                raise RuntimeError("face orientation not found")
            faces.append((e, sA, f, sB, found))
    return faces

def structured_mesh(n: int, lo, hi, degree, displacement=None,
                    scramble_seed: int | None = None) -> MeshSpec:
    """Periodic ``n^3`` hexahedral grid of the box [lo, hi].

    ``degree`` is an int or a callable ``f(centres[K,3]) -> int array``.
    ``displacement`` is ``None`` or a callable ``g(x[...,3]) -> dx[...,3]``
    that must be periodic on the box; it moves every grid vertex.
    ``scramble_seed`` rotates each element's local reference frame by a seeded
    proper cube rotation (the physical element is unchanged).
    """
    if n < 2:
        raise ValueError("need n >= 2 elements per direction")
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    h = (hi - lo) / n
    K = n ** 3
    idx = np.arange(K)
    ix, iy, iz = idx % n, (idx // n) % n, idx // (n * n)
    cell = np.stack([ix, iy, iz], axis=1)                      # [K,3]

    rng = np.random.default_rng(scramble_seed) if scramble_seed is not None else None
    rot = np.zeros(K, dtype=np.int64) if rng is None else rng.integers(0, 24, size=K)

    # canonical corner offsets, bit d of c -> +1 in direction d
    bits = np.array([[(c >> d) & 1 for d in range(3)] for c in range(8)], dtype=np.int64)

    def vertex_pos(gridpt):                                    # gridpt [...,3] int (unwrapped)
        x = lo + gridpt * h
        if displacement is not None:
            x = x + displacement(x)
        return x

    corners = np.zeros((K, 8, 3))
    for r in np.unique(rot):
        sel = np.nonzero(rot == r)[0]
        R = ROTATIONS[r]
        for c in range(8):
            off = (R @ (2 * bits[c] - 1) + 1) // 2
            corners[sel, c] = vertex_pos(cell[sel] + off)

    if rng is None:
        # identity frames: the +X side of A meets the -X side of B, orientation 0
        faces = []
        for X in range(3):
            nb = cell.copy()
            nb[:, X] = (nb[:, X] + 1) % n
            f = nb[:, 0] + n * (nb[:, 1] + n * nb[:, 2])
            faces.append(np.stack([idx, np.full(K, 2 * X + 1), f, np.full(K, 2 * X),
                                   np.zeros(K, dtype=np.int64)], axis=1))
        faces = np.concatenate(faces, axis=0)
    else:
        faces = _scrambled_faces(n, cell, rot)
    faces = np.asarray(faces, dtype=np.int32)

    centres = corners.mean(axis=1)
    if callable(degree):
        deg = np.asarray(degree(centres), dtype=np.int8)
    else:
        deg = np.full(K, int(degree), dtype=np.int8)
    return MeshSpec(n=n, lo=lo, hi=hi, corners=corners, faces=faces, degree=deg, rotation=rot)


def mortar_mesh(n: int, refine: str = "yz", degree=3, scramble_seed: int | None = None,
                amp: float = 0.0) -> MeshSpec:
    """Periodic unit box, coarse for x < 1/2 and refined for x > 1/2: a 2:1 non-conforming interface
    at x = 1/2 and at x = 0 (= 1).

    Coarse cells have side h = 1/n (n even, >= 4); fine cells halve h in the
    directions of ``refine`` ("y": each coarse face meets two fine faces,
    mortar type 1 or 2 depending on the big side's frame; "yz": four, type 3).
    ``degree``: an int, or a pair (coarse, fine), or a callable of the centres.
    ``scramble_seed`` rotates each element's local frame; ``amp`` displaces the
    vertices by ``amp prod_d sin 2 pi (x_d + 1/8)`` (box units, non-zero on the
    interfaces), the fine vertices hanging on a
    coarse face then placed on that face's bilinear surface, so that the small
    faces tile the big one exactly (with a metric degree of at least 2 the
    face-normal polynomials are exact and a small side's normal is the
    restriction of the big side's).

    Mortar rows: ``(big element, big side, type, e_0..e_3, s_0..s_3, o_0..o_3)``
    (unused entries -1).  Type 1 splits the big side's face grid along ``p``
    into halves k = 0, 1 (p in [-1, 0], [0, 1]); type 2 along ``q``; type 3 both,
    k = kp + 2 kq.  ``o_k`` maps the half's face grid, with ``p``, ``q`` along
    the big side's, to the small side's grid as a face orientation does (the
    big side as the left one).
    """
    if n < 4 or n % 2:
        raise ValueError("need an even n >= 4 (below it the periodic corner keys of two faces coincide)")
    if refine not in ("y", "yz"):
        raise ValueError("refine is 'y' or 'yz'")
    Lt = 2 * n                                           # lattice points per direction (unit h/2)
    cells = []                                           # (lattice min corner, lattice size)
    for iz in range(n):
        for iy in range(n):
            for ix in range(n // 2):
                cells.append(((2 * ix, 2 * iy, 2 * iz), (2, 2, 2)))
    fy = 1 if "y" in refine else 2
    fz = 1 if "z" in refine else 2
    for iz in range(0, Lt, fz):
        for iy in range(0, Lt, fy):
            for ix in range(n, Lt, 2):
                cells.append(((ix, iy, iz), (2, fy, fz)))
    K = len(cells)
    cmin = np.array([c[0] for c in cells], dtype=np.int64)
    csz = np.array([c[1] for c in cells], dtype=np.int64)
    rng = np.random.default_rng(scramble_seed) if scramble_seed is not None else None
    rot = np.zeros(K, dtype=np.int64) if rng is None else rng.integers(0, 24, size=K)
    bits = np.array([[(c >> d) & 1 for d in range(3)] for c in range(8)], dtype=np.int64)

    def corner_lattice(e, xi):                           # local reference corner (+-1) -> lattice point
        off = (ROTATIONS[rot[e]] @ xi + 1) // 2
        return cmin[e] + off * csz[e]

    # vertex positions: displaced lattice points; hanging ones on the coarse faces' bilinear surfaces
    h2 = 0.5 / n

    def disp(pt):
        x = pt * h2
        if amp:                                          # phase 1/8: non-zero on the interfaces x = 0, 1/2
            w = np.prod(np.sin(2 * np.pi * (x + 0.125)))
            x = x + amp * w
        return x

    def vertex(pt):
        pt = np.asarray(pt, dtype=np.int64)
        hang = (pt[0] % Lt in (0, n)) and (pt[1] % 2 or pt[2] % 2)
        if not hang:
            return disp(pt)
        ys = [pt[1]] if pt[1] % 2 == 0 else [pt[1] - 1, pt[1] + 1]
        zs = [pt[2]] if pt[2] % 2 == 0 else [pt[2] - 1, pt[2] + 1]
        return np.mean([disp(np.array([pt[0], y, z])) for y in ys for z in zs], axis=0)

    corners = np.zeros((K, 8, 3))
    for e in range(K):
        for c in range(8):
            corners[e, c] = vertex(corner_lattice(e, 2 * bits[c] - 1))

    def key(pt):
        return tuple(int(v) % Lt for v in pt)

    def side_corners(e, side):                           # lattice corner of (p, q) in {0,1}^2
        return {(p, q): corner_lattice(e, _local_face_corner(side, p, q)) for p in (0, 1) for q in (0, 1)}

    sides = {}                                           # corner-key set -> the sides that have it
    for e in range(K):
        for sd in range(6):
            sc = side_corners(e, sd)
            sides.setdefault(frozenset(key(v) for v in sc.values()), []).append(
                (e, sd, {key(v): pq for pq, v in sc.items()}))

    def orientation(big_keys, small):                    # big_keys[(a, b)] -> key; small: (e, s, key -> (p', q'))
        for o in range(8):
            if all(small[2].get(big_keys[(a, b)]) == orient_map(o, a, b, 2) for a in (0, 1) for b in (0, 1)):
                return o
        raise RuntimeError("mortar orientation not found")

    faces, mortars, done = [], [], set()
    for e in range(K):
        for sd in range(6):
            if (e, sd) in done:
                continue
            sc = side_corners(e, sd)
            ks = frozenset(key(v) for v in sc.values())
            other = [v for v in sides[ks] if (v[0], v[1]) != (e, sd)]
            if other:
                f, sf, kmap = other[0]
                o = orientation({pq: key(v) for pq, v in sc.items()}, other[0])
                faces.append((e, sd, f, sf, o))
                done.update({(e, sd), (f, sf)})
                continue
            # a big side: find its halves or quarters among the other sides
            P = {pq: v.astype(np.float64) for pq, v in sc.items()}

            def at(u, v):                                # bilinear lattice point of the big face, (u, v) in [0,1]^2
                x = (1 - u) * (1 - v) * P[(0, 0)] + u * (1 - v) * P[(1, 0)] + (1 - u) * v * P[(0, 1)] + u * v * P[(1, 1)]
                return np.rint(x).astype(np.int64)
            found = None
            for mtype, parts in ((3, [(kp, kq) for kq in (0, 1) for kp in (0, 1)]), (1, [(0, None), (1, None)]),
                                 (2, [(None, 0), (None, 1)])):
                subs = []
                for kp, kq in parts:
                    up = (0.0, 0.5) if kp == 0 else ((0.5, 1.0) if kp == 1 else (0.0, 1.0))
                    vq = (0.0, 0.5) if kq == 0 else ((0.5, 1.0) if kq == 1 else (0.0, 1.0))
                    bk = {(a, b): key(at(up[a], vq[b])) for a in (0, 1) for b in (0, 1)}
                    cand = sides.get(frozenset(bk.values()), [])
                    if len(cand) != 1:
                        break
                    sm = cand[0]
                    subs.append((sm, orientation(bk, sm)))
                else:
                    found = (mtype, subs)
                    break
            if found is None:
                raise RuntimeError(f"side {sd} of element {e} has no partner")
            mtype, subs = found
            row = [e, sd, mtype] + [-1] * 12
            for k, (sm, o) in enumerate(subs):
                row[3 + k], row[7 + k], row[11 + k] = sm[0], sm[1], o
                done.add((sm[0], sm[1]))
            mortars.append(row)
            done.add((e, sd))
    centres = corners.mean(axis=1)
    if callable(degree):
        deg = np.asarray(degree(centres), dtype=np.int8)
    elif isinstance(degree, tuple):
        deg = np.where(centres[:, 0] < 0.5, degree[0], degree[1]).astype(np.int8)
    else:
        deg = np.full(K, int(degree), dtype=np.int8)
    return MeshSpec(n=n, lo=np.zeros(3), hi=np.ones(3), corners=corners, faces=np.asarray(faces, dtype=np.int32),
                    degree=deg, rotation=rot, mortars=np.asarray(mortars, dtype=np.int32).reshape(-1, 15))


def sine_displacement(lo, hi, amp: float):
    """``amp * sin(2 pi x) sin(2 pi y) sin(2 pi z)`` on every coordinate, in box units."""
    lo = np.asarray(lo, dtype=np.float64)
    L = np.asarray(hi, dtype=np.float64) - lo

    def g(x):
        s = (x - lo) / L
        w = np.sin(2 * np.pi * s[..., 0]) * np.sin(2 * np.pi * s[..., 1]) * np.sin(2 * np.pi * s[..., 2])
        return amp * L * w[..., None]
    return g


# ---------------------------------------------------------------------------
# seeded smooth fields
# ---------------------------------------------------------------------------


def fourier_field(seed: int, n_modes: int = 4, kmax: int = 2, lo=(0, 0, 0), hi=(1, 1, 1)):
    """Seeded periodic field: a sum of ``n_modes`` Fourier modes, |k_d| <= kmax.

    Returns ``phi(x[...,3])`` scaled into [-1, 1] by the extreme values of the
    mode sum (bounded by the sum of amplitudes).
    """
    rng = np.random.default_rng(seed)
    ks = []
    while len(ks) < n_modes:
        k = rng.integers(-kmax, kmax + 1, size=3)
        if np.any(k != 0):
            ks.append(k)
    ks = np.asarray(ks, dtype=np.float64)
    amp = rng.uniform(0.5, 1.0, size=n_modes)
    ph = rng.uniform(0, 2 * np.pi, size=n_modes)
    lo = np.asarray(lo, dtype=np.float64)
    L = np.asarray(hi, dtype=np.float64) - lo
    norm = amp.sum()

    def phi(x):
        s = (np.asarray(x) - lo) / L
        arg = 2 * np.pi * (s @ ks.T) + ph
        return (np.sin(arg) * amp).sum(axis=-1) / norm
    return phi


def degree_field(seed: int, nmin: int = 1, nmax: int = 7):
    """Per-element degree ``nmin + min(nmax-nmin, floor((nmax-nmin+1)*phi01))``.

    ``phi01`` is the min-max normalisation over the element centres of a seeded
    smooth Fourier field.
    """
    phi = fourier_field(seed, 4, 2)
    span = nmax - nmin

    def f(centres):
        v = phi(centres)
        v01 = (v - v.min()) / max(v.max() - v.min(), 1e-300)
        return nmin + np.minimum(span, np.floor((span + 1) * v01)).astype(np.int64)
    return f


# ---------------------------------------------------------------------------
# initial states (primitive variables)
# ---------------------------------------------------------------------------


def density_wave(x):
    """rho = 1 + 0.1 sin(2 pi (x+y+z)), v = (1,1,1), p = 1."""
    rho = 1.0 + 0.1 * np.sin(2 * np.pi * (x[..., 0] + x[..., 1] + x[..., 2]))
    one = np.ones_like(rho)
    return np.stack([rho, one, one, one, one], axis=0)


def density_wave_exact(x, t):
    """The density wave advected with v = (1,1,1) to time t on the unit-period box."""
    rho = 1.0 + 0.1 * np.sin(2 * np.pi * (x[..., 0] + x[..., 1] + x[..., 2] - 3.0 * t))
    one = np.ones_like(rho)
    return np.stack([rho, one, one, one, one], axis=0)


def taylor_green(mach: float = 0.1, gamma: float = 1.4):
    """Taylor-Green vortex on the unit-period box (k = 2 pi): rho = 1,
    v = (sin kx cos ky cos kz, -cos kx sin ky cos kz, 0),
    p = 1/(gamma Ma^2) + (cos 2kx + cos 2ky)(cos 2kz + 2)/16."""
    k = 2 * np.pi

    def f(x):
        sx, sy, sz = (np.sin(k * x[..., d]) for d in range(3))
        cx, cy, cz = (np.cos(k * x[..., d]) for d in range(3))
        p = 1.0 / (gamma * mach ** 2) + (np.cos(2 * k * x[..., 0]) + np.cos(2 * k * x[..., 1])) \
            * (np.cos(2 * k * x[..., 2]) + 2.0) / 16.0
        return np.stack([np.ones_like(p), sx * cy * cz, -cx * sy * cz, np.zeros_like(p), p], axis=0)
    return f


def freestream(x, n_var: int = 5):
    """Uniform state rho = 1, v = (1,1,1), p = 1 (and Y1 = 0.5)."""
    one = np.ones(x.shape[:-1])
    comps = [one, one, one, one, one]
    if n_var == 6:
        comps.append(0.5 * one)
    return np.stack(comps, axis=0)


def blast_wave(x, centre=(0.5, 0.5, 0.5), r0=0.25, width=0.0):
    """Spherical blast: r < r0 -> rho=1, p=10; else rho=0.125, p=0.1; v=0.

    ``width > 0`` replaces the jump by ``(1 - tanh((r - r0)/width))/2`` so that
    polynomial sub-cell means of the nodal data stay positive.
    """
    r = np.linalg.norm(x - np.asarray(centre), axis=-1)
    if width > 0:
        s = 0.5 * (1.0 - np.tanh((r - r0) / width))
    else:
        s = (r < r0).astype(np.float64)
    rho = 0.125 + (1.0 - 0.125) * s
    p = 0.1 + (10.0 - 0.1) * s
    z = np.zeros_like(rho)
    return np.stack([rho, z, z, z, p], axis=0)


def smoothed_blast(width: float):
    """The spherical blast with a tanh front of the given width."""
    def f(x):
        return blast_wave(x, width=width)
    return f


def shocked_two_species(seed: int):
    """Smooth seeded 2-species fields plus a planar Mach-2 shock at x = 0.5.

    Upstream (x >= 0.5): rho = 1 + 0.1 phi1, v = 0.1 (phi2, phi3, phi4),
    p = 1 + 0.1 phi5, Y1 = 0.5 + 0.4 phi6.  Downstream (x < 0.5) the
    Rankine-Hugoniot jump of a Mach-2 shock in a gamma = 1.4 gas scales rho by
    8/3 and p by 4.5 and adds 1.479 to v1.
    """
    phis = [fourier_field(seed * 101 + i, 4, 2) for i in range(6)]

    def f(x):
        ph = [g(x) for g in phis]
        rho = 1.0 + 0.1 * ph[0]
        v1, v2, v3 = 0.1 * ph[1], 0.1 * ph[2], 0.1 * ph[3]
        p = 1.0 + 0.1 * ph[4]
        Y1 = 0.5 + 0.4 * ph[5]
        down = x[..., 0] < 0.5
        rho = np.where(down, rho * 8.0 / 3.0, rho)
        p = np.where(down, p * 4.5, p)
        v1 = np.where(down, v1 + 1.479, v1)
        return np.stack([rho, v1, v2, v3, p, Y1], axis=0)
    return f


def isentropic_vortex(eps: float = 5.0, gamma: float = 1.4):
    """Isentropic vortex around the z axis, background (1, (1,1,0), 1)."""
    def f(x):
        r2 = x[..., 0] ** 2 + x[..., 1] ** 2
        ex = np.exp(0.5 * (1.0 - r2))
        du = eps / (2 * np.pi) * ex
        v1 = 1.0 - du * x[..., 1]
        v2 = 1.0 + du * x[..., 0]
        v3 = np.zeros_like(v1)
        T = 1.0 - (gamma - 1.0) * eps ** 2 / (8.0 * gamma * np.pi ** 2) * ex ** 2
        rho = T ** (1.0 / (gamma - 1.0))
        p = rho * T
        return np.stack([rho, v1, v2, v3, p], axis=0)
    return f


def kelvin_helmholtz(seed: int):
    """Shear layer on [-0.5,0.5]^3: |y| < 0.25 -> rho=2, v1=0.5; else rho=1, v1=-0.5.

    p = 2.5, v2 = 0.01 psi(x, z) with psi a seeded smooth field, v3 = 0.
    """
    psi = fourier_field(seed, 4, 2, lo=(-0.5, -0.5, -0.5), hi=(0.5, 0.5, 0.5))

    def f(x):
        inner = np.abs(x[..., 1]) < 0.25
        rho = np.where(inner, 2.0, 1.0)
        v1 = np.where(inner, 0.5, -0.5)
        xz = x.copy()
        xz[..., 1] = 0.0
        v2 = 0.01 * psi(xz)
        v3 = np.zeros_like(rho)
        p = np.full_like(rho, 2.5)
        return np.stack([rho, v1, v2, v3, p], axis=0)
    return f


# ---------------------------------------------------------------------------
# configurations
# ---------------------------------------------------------------------------

# flux selectors shared by the interface format
VOL_RANOCHA, VOL_PIROZZOLI, VOL_CENTRAL = 0, 1, 2
RIEMANN_ROE_HH, RIEMANN_LLF, RIEMANN_EC = 0, 1, 2

GAS_AIR_H2 = dict(gamma=1.4, kappa=(1.4, 1.41), R=(287.0, 4124.0))


@dataclass
class Workload:
    name: str
    mesh: MeshSpec
    n_var: int
    prim: object                 # callable x[...,3] -> prim[n_var, ...]
    volume_flux: int
    face_flux_dg: int
    face_flux_fv: int
    n_fv: int
    metric_degree: int
    gamma: float = 1.4
    kappa: tuple = (1.4, 1.4)
    R: tuple = (287.0, 287.0)
    ind_T: float = 2.0
    ind_dT: float = 1.0
    ind_vars: int = 1            # bit 0: pressure, bit 1: density, bit 2: Y1
    cfl: float = 0.5
    steps: int = 10
    seed: int = 0
    noise: float = 0.0
    blend_fraction: float | None = None
    limiter: bool = False        # positivity limiter after every Runge-Kutta stage
    # viscous terms (species 1 first; one species uses index 0): dynamic viscosity,
    # Prandtl number, diffusion coefficient; all zero mu and D: inviscid
    mu: tuple = (0.0, 0.0)
    Pr: tuple = (0.72, 0.72)
    D: tuple = (0.0, 0.0)

    @property
    def viscous(self) -> bool:
        return any(x != 0.0 for x in tuple(self.mu) + tuple(self.D))


def make_workload(name: str, n: int | None = None, scramble_seed: int | None = None) -> Workload:
    """The five workloads C1..C5 (``n`` overrides the elements per direction)."""
    if name == "C1":
        n = n or 4
        mesh = structured_mesh(n, (0, 0, 0), (1, 1, 1), 3, scramble_seed=scramble_seed)
        return Workload("C1", mesh, 5, density_wave, VOL_RANOCHA, RIEMANN_ROE_HH, RIEMANN_LLF,
                        n_fv=4, metric_degree=1, steps=10, seed=1,
                        ind_T=-1.0, ind_dT=0.5)
    if name == "C2":
        n = n or 16
        mesh = structured_mesh(n, (0, 0, 0), (1, 1, 1), 5, scramble_seed=scramble_seed)
        # the configured jump; the positivity limiter keeps density and pressure
        # positive at the nodes and at the sub-cell means of blended elements
        return Workload("C2", mesh, 5, blast_wave, VOL_RANOCHA, RIEMANN_ROE_HH,
                        RIEMANN_LLF, n_fv=6, metric_degree=1, steps=100, seed=2,
                        ind_T=2.5, ind_dT=0.5, limiter=True)
    if name == "C3":
        n = n or 32
        mesh = structured_mesh(n, (0, 0, 0), (1, 1, 1), degree_field(3, 1, 7),
                               displacement=sine_displacement((0, 0, 0), (1, 1, 1), 0.05),
                               scramble_seed=scramble_seed)
        # curved: per-element metrics (metric_degree 0); the affine boxes of the other
        # workloads have constant metrics, which every metric degree reproduces exactly
        return Workload("C3", mesh, 6, shocked_two_species(3), VOL_PIROZZOLI, RIEMANN_LLF,
                        RIEMANN_LLF, n_fv=8, metric_degree=0, seed=3,
                        kappa=GAS_AIR_H2["kappa"], R=GAS_AIR_H2["R"],
                        ind_T=2.0, ind_dT=1.0, ind_vars=1 | 4)
    if name == "C4":
        n = n or 16
        mesh = structured_mesh(n, (-5, -5, -5), (5, 5, 5), 4, scramble_seed=scramble_seed)
        return Workload("C4", mesh, 5, isentropic_vortex(5.0), VOL_RANOCHA, RIEMANN_ROE_HH,
                        RIEMANN_LLF, n_fv=5, metric_degree=1, steps=50, seed=4, noise=1e-3,
                        ind_T=-1.0, ind_dT=0.5)
    if name == "C5":
        n = n or 64
        mesh = structured_mesh(n, (-0.5, -0.5, -0.5), (0.5, 0.5, 0.5), 7,
                               scramble_seed=scramble_seed)
        return Workload("C5", mesh, 5, kelvin_helmholtz(5), VOL_RANOCHA, RIEMANN_ROE_HH,
                        RIEMANN_LLF, n_fv=8, metric_degree=1, seed=5,
                        ind_T=2.0, ind_dT=1.0, blend_fraction=0.10)
    if name == "M3":
        # non-conforming: coarse for x < 1/2, halved in y and z beyond (type-3 mortars
        # at x = 1/2 and x = 0), N = 7, a tenth of the elements blended as in C5 (the
        # FV variants of the mortars where a blended element meets one)
        n = n or 24
        mesh = mortar_mesh(n, "yz", 7, scramble_seed=scramble_seed)
        return Workload("M3", mesh, 5, density_wave, VOL_RANOCHA, RIEMANN_ROE_HH, RIEMANN_LLF,
                        n_fv=8, metric_degree=1, seed=7, ind_T=-1.0, ind_dT=0.5, blend_fraction=0.10)
    if name == "M3V":
        # M3 with the viscous terms (mu = 1e-3, Pr = 0.71): BR1 lifting and viscous
        # fluxes through the mortars as well
        return dataclasses.replace(make_workload("M3", n, scramble_seed), name="M3V", mu=(1e-3, 0.0),
                                   Pr=(0.71, 0.71))
    if name == "TGV":
        # viscous Taylor-Green vortex, Re = 1600 on the length 1/(2 pi), Ma = 0.1, Pr = 0.71;
        # smooth, so every element is DG (no blending)
        n = n or 64
        mesh = structured_mesh(n, (0, 0, 0), (1, 1, 1), 7, scramble_seed=scramble_seed)
        return Workload("TGV", mesh, 5, taylor_green(0.1), VOL_RANOCHA, RIEMANN_ROE_HH,
                        RIEMANN_LLF, n_fv=8, metric_degree=1, seed=6,
                        ind_T=-1.0, ind_dT=0.5, mu=(1.0 / (1600.0 * 2 * np.pi), 0.0), Pr=(0.71, 0.71))
    raise KeyError(name)


def noise(seed: int, shape, scale: float) -> np.ndarray:
    """i.i.d. normal noise of standard deviation ``scale``."""
    return np.random.default_rng(seed).normal(0.0, scale, size=shape)


def cotangents(seed: int, shape) -> np.ndarray:
    """i.i.d. standard normal cotangent vectors."""
    return np.random.default_rng(seed).standard_normal(size=shape)


def quantile_mask(values: np.ndarray, fraction: float) -> np.ndarray:
    """Boolean mask of the ``fraction`` of entries with the lowest values (ties by index)."""
    k = int(math.ceil(fraction * values.size))
    order = np.argsort(values, kind="stable")
    m = np.zeros(values.size, dtype=bool)
    m[order[:k]] = True
    return m
