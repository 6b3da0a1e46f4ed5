"""Pins of the FP64 texture-gradient preconditioner (CPU only): closed forms
and invariants of (I + lambda L)^-1 on the texel grid."""
import math

import numpy as np
import pytest

from oracle import precond as P


def test_zero_lambda_is_identity():
    g = np.random.Generator(np.random.PCG64(0)).normal(size=7 * 5 * 3)
    np.testing.assert_allclose(P.precondition(g, 7, 5, 3, 0.0), g, rtol=1e-14)


def test_constant_field_is_unchanged_and_sums_are_kept():
    g = np.tile(np.array([0.3, -1.5, 2.0]), 9 * 11)
    np.testing.assert_allclose(P.precondition(g, 9, 11, 3, 25.0), g, rtol=1e-12)
    # 1^T L = 0: every channel keeps its sum
    r = np.random.Generator(np.random.PCG64(1)).normal(size=(9 * 11, 3))
    y = P.precondition(r.reshape(-1), 9, 11, 3, 7.0).reshape(-1, 3)
    np.testing.assert_allclose(y.sum(0), r.sum(0), rtol=1e-11, atol=1e-12)


@pytest.mark.parametrize("h,w,ky,kx", [(8, 8, 0, 1), (6, 10, 3, 7), (13, 4, 12, 2), (1, 9, 0, 4)])
def test_grid_cosines_are_eigenvectors(h, w, ky, kx):
    # the Neumann cosines cos(pi k (i + 1/2) / n) are eigenvectors of the path
    # graph's Laplacian with eigenvalue 2 - 2 cos(pi k / n); on the grid the
    # eigenvalues of the two axes add
    lam = 3.5
    ys, xs = np.meshgrid(np.arange(h), np.arange(w), indexing="ij")
    f = np.cos(math.pi * ky * (ys + 0.5) / h) * np.cos(math.pi * kx * (xs + 0.5) / w)
    mu = (2 - 2 * math.cos(math.pi * ky / h)) + (2 - 2 * math.cos(math.pi * kx / w))
    g = np.stack([f, -2 * f], -1).reshape(-1)
    y = P.precondition(g, h, w, 2, lam)
    np.testing.assert_allclose(y, g / (1 + lam * mu), rtol=1e-10, atol=1e-13)


def test_two_by_two_grid_by_hand():
    # 2x2 texels: a 4-cycle 0-1-3-2-0, every node of degree 2
    lam = 0.5
    M = np.array([[1 + 2 * lam, -lam, -lam, 0],
                  [-lam, 1 + 2 * lam, 0, -lam],
                  [-lam, 0, 1 + 2 * lam, -lam],
                  [0, -lam, -lam, 1 + 2 * lam]])
    g = np.array([1.0, 2.0, -3.0, 0.5])
    y = P.precondition(g, 2, 2, 1, lam)
    np.testing.assert_allclose(M @ y, g, rtol=1e-13)


def test_channels_are_independent_and_map_is_symmetric():
    gen = np.random.Generator(np.random.PCG64(4))
    a = gen.normal(size=(5 * 6, 4))
    b = a.copy()
    b[:, 2] = gen.normal(size=30)
    ya = P.precondition(a.reshape(-1), 5, 6, 4, 2.0).reshape(-1, 4)
    yb = P.precondition(b.reshape(-1), 5, 6, 4, 2.0).reshape(-1, 4)
    np.testing.assert_array_equal(ya[:, [0, 1, 3]], yb[:, [0, 1, 3]])
    # (I + lam L)^-1 is symmetric: <P u, v> = <u, P v>
    u, v = gen.normal(size=30), gen.normal(size=30)
    Pu, Pv = (P.precondition(x, 5, 6, 1, 2.0) for x in (u, v))
    assert abs(Pu @ v - u @ Pv) <= 1e-12 * abs(Pu @ v)
