"""Pins of the LGL basis (Section 3) against closed forms."""

import json
import math
import os

import numpy as np
import pytest

from oracle import gll

GOLD = os.path.join(os.path.dirname(__file__), "golden", "lgl_closed_forms.json")


def _ev(s):
    return eval(s, {"sqrt": math.sqrt})


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 6])
def test_lgl_closed_forms(N):
    g = json.load(open(GOLD))["cases"][str(N)]
    x = np.array([_ev(s) for s in g["nodes"]])
    w = np.array([_ev(s) for s in g["weights"]])
    np.testing.assert_allclose(gll.lgl_nodes(N), x, atol=2e-16, rtol=0)
    np.testing.assert_allclose(gll.lgl_weights(N), w, atol=1e-15, rtol=0)


@pytest.mark.parametrize("N", range(1, 13))
def test_quadrature_exactness(N):
    """sum w = 2 and exact integrals of x^k for k <= 2N-1."""
    x, w = gll.lgl_nodes(N), gll.lgl_weights(N)
    assert abs(w.sum() - 2.0) < 1e-14
    for k in range(2 * N):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.dot(w, x**k) - exact) < 1e-13
    # 2N is not integrated exactly (LGL has degree of exactness 2N-1)
    assert abs(np.dot(w, x ** (2 * N)) - 2.0 / (2 * N + 1)) > 1e-9


@pytest.mark.parametrize("N", range(1, 13))
def test_derivative_exact_on_polynomials(N):
    """D x^k = k x^(k-1) for k <= N; D 1 = 0."""
    x = gll.lgl_nodes(N)
    D = gll.derivative_matrix(N)
    for k in range(N + 1):
        ref = k * x ** (k - 1) if k > 0 else np.zeros_like(x)
        np.testing.assert_allclose(D @ x**k, ref, atol=5e-13 * max(1, N * N))
    assert np.abs(D.sum(axis=1)).max() < 1e-12 * N * N


@pytest.mark.parametrize("N", range(1, 13))
def test_summation_by_parts(N):
    """W D + D^T W = diag(-1, 0, ..., 0, 1) (exact for LGL, degree 2N-1)."""
    w = gll.lgl_weights(N)
    D = gll.derivative_matrix(N)
    Q = np.diag(w) @ D
    B = np.zeros((N + 1, N + 1))
    B[0, 0], B[-1, -1] = -1.0, 1.0
    np.testing.assert_allclose(Q + Q.T, B, atol=1e-12 * N * N)


def test_lagrange_cardinal_and_polynomial():
    N = 7
    x = gll.lgl_nodes(N)
    np.testing.assert_allclose(gll.lagrange_matrix(x, x), np.eye(N + 1), atol=1e-14)
    s = np.linspace(-1, 1, 23)
    P = lambda t: 3 * t**7 - t**4 + 0.5 * t - 2
    np.testing.assert_allclose(gll.lagrange_matrix(x, s) @ P(x), P(s), atol=1e-12)
