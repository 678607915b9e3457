"""Pins of the oracle's quadrature rules against closed-form integrals."""
import math

import numpy as np
import pytest

from oracle import quadrature as quad


def test_gauss_legendre_exact_on_polynomials():
    R = 7.249309
    for m in (4, 8, 16):
        x, w = quad.gauss_legendre(m, R)
        assert np.all((x > 0) & (x < R))
        for k in range(2 * m):
            exact = R ** (k + 1) / (k + 1)
            assert abs((w * x ** k).sum() - exact) <= 1e-13 * exact
        # prod (x - x_a)^2 (degree 2m) vanishes at every node but has a
        # positive integral: the rule is not exact beyond degree 2m - 1
        xs = np.linspace(0, R, 20001)
        node_poly = np.prod((xs[:, None] - x[None, :]) ** 2, axis=1)
        assert np.trapezoid(node_poly, xs) > 0
        assert abs((w * np.prod((x[:, None] - x[None, :]) ** 2, axis=1)).sum()) == 0.0


def test_circle_rule_exact_on_trig():
    for m in (8, 16):
        s, w = quad.circle_rule(m)
        t = np.arctan2(s[:, 1], s[:, 0])
        assert abs(w.sum() - 2 * math.pi) < 1e-14
        for j in range(1, m):
            assert abs((w * np.cos(j * t)).sum()) < 1e-13
        assert abs((w * np.cos(m * t)).sum() - 2 * math.pi) < 1e-12


def _sphere_monomial(a, b, c):
    if a % 2 or b % 2 or c % 2:
        return 0.0
    g = math.gamma
    return 2.0 * g((a + 1) / 2) * g((b + 1) / 2) * g((c + 1) / 2) / g((a + b + c + 3) / 2)


def test_lebedev38_degree9_exact():
    s, w = quad.lebedev38()
    assert s.shape == (38, 3)
    assert np.allclose((s ** 2).sum(axis=1), 1.0, atol=1e-15)
    worst = 0.0
    for deg in range(0, 10):
        for a in range(deg + 1):
            for b in range(deg + 1 - a):
                c = deg - a - b
                val = (w * s[:, 0] ** a * s[:, 1] ** b * s[:, 2] ** c).sum()
                worst = max(worst, abs(val - _sphere_monomial(a, b, c)))
    assert worst < 1e-13
    # degree 10 is not exact (x^10)
    val = (w * s[:, 0] ** 10).sum()
    assert abs(val - _sphere_monomial(10, 0, 0)) > 1e-4


def test_rules_are_antipodal():
    for d in (2, 3):
        s, w = quad.sphere_rule(d)
        bb = quad.antipode_index(s)
        assert np.allclose(s[bb], -s)
        assert np.allclose(w[bb], w)
