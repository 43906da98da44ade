"""Pins of the oracle's 1D tables against closed forms and exactness properties."""
import math
import os

import numpy as np
import pytest
from numpy.polynomial import legendre as L

from oracle import basis, rng

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("k", range(1, 9))
def test_gll_nodes_roots_and_symmetry(k):
    x = basis.gll_nodes(k)
    assert len(x) == k + 1
    assert x[0] == 0.0 and x[-1] == 1.0
    assert np.all(np.diff(x) > 0)
    np.testing.assert_allclose(x + x[::-1], 1.0, atol=1e-15)
    t = 2 * x - 1
    resid = (1 - t ** 2) * L.Legendre.basis(k).deriv()(t)
    assert np.max(np.abs(resid)) < 1e-13


def test_gll_known_values():
    np.testing.assert_allclose(basis.gll_nodes(2), [0, 0.5, 1], atol=1e-16)
    s = 1 / math.sqrt(5)
    np.testing.assert_allclose(basis.gll_nodes(3), 0.5 * (np.array([-1, -s, s, 1]) + 1), atol=1e-15)
    s = math.sqrt(3 / 7)
    np.testing.assert_allclose(basis.gll_nodes(4), 0.5 * (np.array([-1, -s, 0, s, 1]) + 1), atol=1e-15)


@pytest.mark.parametrize("k", range(1, 9))
def test_gll_weights_closed_form(k):
    # GLL weights on [-1,1]: 2 / (k (k+1) P_k(x_i)^2); halved on [0,1]
    x = 2 * basis.gll_nodes(k) - 1
    w = 1.0 / (k * (k + 1) * L.Legendre.basis(k)(x) ** 2)
    np.testing.assert_allclose(basis.gll_weights(k), w, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("nq", range(1, 11))
def test_gauss_exactness(nq):
    x, w = basis.gauss_rule(nq)
    assert abs(w.sum() - 1.0) < 1e-15
    for p in range(2 * nq):
        assert abs(w @ x ** p - 1.0 / (p + 1)) < 2e-15
    # not exact one degree higher (the rule is exactly of degree 2nq-1); the
    # error for x^(2nq) on [0,1] is (nq!)^4 / ((2nq+1) ((2nq)!)^2)
    err = math.factorial(nq) ** 4 / ((2 * nq + 1) * math.factorial(2 * nq) ** 2)
    assert abs((1.0 / (2 * nq + 1) - w @ x ** (2 * nq)) - err) < 1e-15 + 1e-6 * err


@pytest.mark.parametrize("k", range(1, 9))
def test_lagrange_cardinal_and_derivative(k):
    nodes = basis.gll_nodes(k)
    np.testing.assert_allclose(basis.lagrange_values(nodes, nodes), np.eye(k + 1), atol=1e-14)
    xs = np.linspace(-0.2, 1.3, 17)
    p = lambda t: (t - 0.3) ** k + 2 * t - 1
    dp = lambda t: k * (t - 0.3) ** (k - 1) + 2
    np.testing.assert_allclose(basis.lagrange_values(nodes, xs) @ p(nodes), p(xs), atol=1e-13)
    np.testing.assert_allclose(basis.lagrange_derivatives(nodes, xs) @ p(nodes), dp(xs), atol=1e-11)


def test_conv_points_rule():
    assert [basis.default_conv_points(k) for k in (3, 4, 5)] == [6, 7, 9]


def test_splitmix64_published_vector():
    vals = [int(l) for l in open(os.path.join(GOLDEN, "splitmix64_seed1234567.txt")) if not l.startswith("#")]
    assert [int(v) for v in rng.splitmix64(1234567, 5)] == vals
    u = rng.uniform_pm1(7, 100000)
    assert u.min() >= -1 and u.max() < 1 and abs(u.mean()) < 0.01
