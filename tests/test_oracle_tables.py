"""Pins of the oracle's 1D rules and SBP operator (section "Nodal bases, quadrature,
and mass matrices"; eq. euler-sbp) against closed forms and numpy's Gauss rule."""
import math

import numpy as np
import pytest

import oracle as O

GLL_CLOSED = {
    1: ([-1, 1], [1, 1]),
    2: ([-1, 0, 1], [1 / 3, 4 / 3, 1 / 3]),
    3: ([-1, -1 / math.sqrt(5), 1 / math.sqrt(5), 1], [1 / 6, 5 / 6, 5 / 6, 1 / 6]),
    4: ([-1, -math.sqrt(3 / 7), 0, math.sqrt(3 / 7), 1], [1 / 10, 49 / 90, 32 / 45, 49 / 90, 1 / 10]),
}


@pytest.mark.parametrize("r", [1, 2, 3, 4])
def test_gll_closed_forms(r):
    x, w = O.gll(r)
    np.testing.assert_allclose(x, GLL_CLOSED[r][0], atol=1e-15)
    np.testing.assert_allclose(w, GLL_CLOSED[r][1], atol=1e-15)


def test_gll_degree0_midpoint():
    x, w = O.gll(0)
    assert x.tolist() == [0.0] and w.tolist() == [2.0]


@pytest.mark.parametrize("k", range(0, 7))
def test_gauss_matches_numpy(k):
    x, w = O.gauss(k)
    xr, wr = np.polynomial.legendre.leggauss(k + 1)
    np.testing.assert_allclose(x, xr, atol=1e-15)
    np.testing.assert_allclose(w, wr, atol=1e-15)


@pytest.mark.parametrize("r", range(1, 9))
def test_gll_exactness(r):
    x, w = O.gll(r)
    for deg in range(0, 2 * r):  # exact through degree 2r-1
        exact = 0.0 if deg % 2 else 2.0 / (deg + 1)
        assert abs((w * x ** deg).sum() - exact) < 1e-14
    # and not exact at degree 2r (lumping error)
    assert abs((w * x ** (2 * r)).sum() - 2.0 / (2 * r + 1)) > 1e-6


@pytest.mark.parametrize("r", range(1, 9))
def test_sbp_identity(r):
    x, w = O.gll(r)
    D = O.diff_matrix(r)
    Q = np.diag(w) @ D
    B = np.zeros((r + 1, r + 1)); B[0, 0] = -1; B[-1, -1] = 1
    np.testing.assert_allclose(Q + Q.T, B, atol=1e-13)
    # D differentiates polynomials of degree <= r exactly
    for deg in range(r + 1):
        np.testing.assert_allclose(D @ x ** deg, deg * x ** max(deg - 1, 0) if deg else 0 * x, atol=1e-12)
