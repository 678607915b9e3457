"""Quadrature rules of the collision solver (oracle; test infrastructure only).

The paper evaluates the collision operator with the fast Fourier spectral
methods it cites (Sec. 2.1) and does not list their quadrature; the readings
taken here are:
  * radial: Gauss-Legendre with m_rho nodes on [0, R];
  * circle (d = 2): m_sigma equispaced angles 2*pi*b/m_sigma, weight 2*pi/m_sigma;
  * sphere (d = 3): the 38-point Lebedev rule (exact for polynomials of degree
    <= 9), weights scaled to sum to 4*pi.
All three rules are symmetric under sigma -> -sigma.

Pinned in tests/test_oracle_quadrature.py against closed-form integrals.
"""
from __future__ import annotations

import math

import numpy as np


def gauss_legendre(m: int, R: float):
    """Nodes rho_a and weights w_a of the m-point Gauss-Legendre rule on [0, R]."""
    x, w = np.polynomial.legendre.leggauss(m)
    return 0.5 * R * (x + 1.0), 0.5 * R * w


def circle_rule(m: int):
    """Unit vectors sigma_b = (cos t_b, sin t_b), t_b = 2 pi b / m; weights 2 pi / m."""
    t = 2.0 * math.pi * np.arange(m) / m
    return np.stack([np.cos(t), np.sin(t)], axis=1), np.full(m, 2.0 * math.pi / m)


def lebedev38():
    """38-point Lebedev rule on the unit sphere, weights summing to 4 pi.

    Orbits: 6 vertices (+-1,0,0) of weight 1/105; 8 cube corners
    (+-1,+-1,+-1)/sqrt(3) of weight 9/280; 24 points (+-p,+-q,0) with every
    placement of the zero, weight 1/35, where p = 0.4597008433809831 and
    q = sqrt(1 - p^2)."""
    pts, wts = [], []
    for ax in range(3):
        for s in (1.0, -1.0):
            e = [0.0, 0.0, 0.0]
            e[ax] = s
            pts.append(e)
            wts.append(1.0 / 105.0)
    c = 1.0 / math.sqrt(3.0)
    for sx in (1.0, -1.0):
        for sy in (1.0, -1.0):
            for sz in (1.0, -1.0):
                pts.append([sx * c, sy * c, sz * c])
                wts.append(9.0 / 280.0)
    p = 0.4597008433809831
    q = math.sqrt(1.0 - p * p)
    for zero_ax in range(3):
        others = [a for a in range(3) if a != zero_ax]
        for (u, w) in ((p, q), (q, p)):
            for su in (1.0, -1.0):
                for sw in (1.0, -1.0):
                    e = [0.0, 0.0, 0.0]
                    e[others[0]] = su * u
                    e[others[1]] = sw * w
                    pts.append(e)
                    wts.append(1.0 / 35.0)
    return np.array(pts), 4.0 * math.pi * np.array(wts)


def sphere_rule(d: int, m_sigma: int = 0):
    if d == 2:
        return circle_rule(m_sigma or 8)
    if d == 3:
        if m_sigma not in (0, 38):
            raise ValueError("3D sphere rule: only the 38-point Lebedev rule is provided")
        return lebedev38()
    raise ValueError("d must be 2 or 3")


def antipode_index(sig: np.ndarray) -> np.ndarray:
    """bbar[b] with sigma[bbar[b]] = -sigma[b]."""
    m = sig.shape[0]
    out = np.empty(m, dtype=np.int64)
    for b in range(m):
        dist = np.abs(sig + sig[b]).sum(axis=1)
        j = int(np.argmin(dist))
        if dist[j] > 1e-12:
            raise ValueError("rule is not antipodally symmetric")
        out[b] = j
    return out
