"""Pins of the oracle's one-dimensional operators against closed forms and exact identities."""
import math

import numpy as np
import pytest

from oracle import ops1d


def test_lgl_closed_forms():
    # N=1: nodes +-1, weights 1;  N=2: 0, +-1 with 4/3, 1/3;  N=3: +-1/sqrt(5), +-1 with 5/6, 1/6
    x, w = ops1d.lgl(1)
    assert np.allclose(x, [-1, 1], atol=0) and np.allclose(w, [1, 1], atol=1e-16)
    x, w = ops1d.lgl(2)
    assert np.allclose(x, [-1, 0, 1], atol=1e-16) and np.allclose(w, [1 / 3, 4 / 3, 1 / 3], atol=1e-15)
    x, w = ops1d.lgl(3)
    s = 1 / math.sqrt(5)
    assert np.allclose(x, [-1, -s, s, 1], atol=1e-16)
    assert np.allclose(w, [1 / 6, 5 / 6, 5 / 6, 1 / 6], atol=1e-15)


@pytest.mark.parametrize("N", range(1, 10))
def test_lgl_quadrature_exactness(N):
    # exact for polynomials of degree 2N-1, symmetric nodes, weights sum to 2
    x, w = ops1d.lgl(N)
    assert abs(w.sum() - 2) < 1e-14
    assert np.allclose(x, -x[::-1], atol=1e-15)
    for d in range(2 * N):
        exact = 0.0 if d % 2 else 2.0 / (d + 1)
        assert abs((w * x ** d).sum() - exact) < 1e-14


@pytest.mark.parametrize("N", range(1, 10))
def test_derivative_matrix(N):
    x, w = ops1d.lgl(N)
    D = ops1d.dmat(N)
    # differentiates polynomials of degree <= N exactly
    for d in range(N + 1):
        ref = d * x ** (d - 1) if d else 0 * x
        assert np.allclose(D @ x ** d, ref, atol=1e-12 * max(1, N ** 2))
    # summation by parts: W D + (W D)^T = diag(-1, 0, ..., 0, 1)
    Q = np.diag(w) @ D
    B = np.zeros((N + 1, N + 1))
    B[0, 0], B[-1, -1] = -1, 1
    assert np.allclose(Q + Q.T, B, atol=1e-14)
    # boundary diagonal entries -N(N+1)/4 and N(N+1)/4; interior diagonal 0
    assert abs(D[0, 0] + N * (N + 1) / 4) < 1e-13
    assert abs(D[-1, -1] - N * (N + 1) / 4) < 1e-13
    assert np.allclose(np.diag(D)[1:-1], 0, atol=1e-13)
    # 2 D_00 = -1/w_0: the boundary terms of the strong split form cancel
    assert abs(2 * D[0, 0] + 1 / w[0]) < 1e-12


@pytest.mark.parametrize("N", range(1, 8))
def test_legendre_vandermonde(N):
    x, w = ops1d.lgl(N)
    V = ops1d.vleg(N)
    # orthonormal under the LGL quadrature up to the last mode (degree 2N is not exact)
    G = V.T @ np.diag(w) @ V
    assert np.allclose(G[:N, :N], np.eye(N), atol=1e-13)
    assert np.allclose(V @ ops1d.vleg_inv(N), np.eye(N + 1), atol=1e-13)
    # first two modes: 1/sqrt(2) and sqrt(3/2) x
    assert np.allclose(V[:, 0], 1 / math.sqrt(2))
    assert np.allclose(V[:, 1], math.sqrt(1.5) * x)


@pytest.mark.parametrize("N,M", [(1, 2), (1, 7), (2, 5), (3, 4), (4, 7), (6, 7)])
def test_degree_maps(N, M):
    xN, _ = ops1d.lgl(N)
    xM, wM = ops1d.lgl(M)
    up = ops1d.interp(N, M)
    down = ops1d.project(M, N)
    # interpolation is exact for degree <= N
    for d in range(N + 1):
        assert np.allclose(up @ xN ** d, xM ** d, atol=1e-13)
    # projection after interpolation is the identity
    assert np.allclose(down @ up, np.eye(N + 1), atol=1e-13)
    # projection preserves the integral of any degree-M polynomial
    _, wN = ops1d.lgl(N)
    f = np.random.default_rng(N * 10 + M).standard_normal(M + 1)
    assert abs(wN @ (down @ f) - wM @ f) < 1e-13
    # and is the L2 projection: residual orthogonal to degree-N polynomials (exact M-point quadrature)
    r = up @ (down @ f) - f
    for d in range(N + 1):
        assert abs(wM @ (r * xM ** d)) < 1e-13


@pytest.mark.parametrize("N,NFV", [(1, 2), (2, 3), (3, 4), (3, 8), (5, 6), (7, 8), (2, 7), (4, 9)])
def test_subcell_maps(N, NFV):
    x, w = ops1d.lgl(N)
    V = ops1d.dg2fv(N, NFV)
    Vp = ops1d.fv2dg(N, NFV)
    h = 2.0 / NFV
    # exact sub-cell means of monomials
    for d in range(N + 1):
        a = -1 + h * np.arange(NFV)
        b = a + h
        ref = (b ** (d + 1) - a ** (d + 1)) / (d + 1) / h
        assert np.allclose(V @ x ** d, ref, atol=1e-13)
    # pseudo-inverse identities (the FV->DG map of Section 3.2)
    assert np.allclose(Vp @ V, np.eye(N + 1), atol=1e-12)
    assert np.allclose(h * np.ones(NFV) @ V, w, atol=1e-14)         # w^T = h 1^T V
    assert np.allclose(w @ Vp, h * np.ones(NFV), atol=1e-13)         # w^T V^+ = h 1^T
    If = ops1d.face_interp(N, NFV)
    assert np.allclose(If[0], np.eye(N + 1)[0]) and np.allclose(If[-1], np.eye(N + 1)[-1])
    assert np.allclose(If.sum(1), 1, atol=1e-13)
