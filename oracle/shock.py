"""Mott-Smith description of a normal shock (oracle).

TEST INFRASTRUCTURE ONLY -- see oracle/__init__.py.

Source: Sec. 4 of the paper.  For a strong shock the distribution across the
wave is close to a blend f = a(x_1) f_L + (1 - a(x_1)) f_R of the two
Rankine-Hugoniot Maxwellians.  Taking the v_1^2 moment of the stationary
equation v_1 df/dx_1 = Q(f, f) turns the blend into an ordinary differential
equation for a whose solution is the logistic profile

    a(x_1) = 1 / (exp(beta x_1) + 1),
    beta   = alpha / ((d - 1) rho_L u_L R (T_L - T_R)),
    alpha  = int v_1^2 (Q(f_L, f_R) + Q(f_R, f_L)) dv   (eq. alpha),

(gas constant R = 1 here), and the density across the wave is

    rho(x_1) / rho_L = (1 + (rho_R / rho_L) exp(beta x_1)) / (1 + exp(beta x_1)),

with rho_R / rho_L = (d + 1) M^2 / (M^2 + d) from the Rankine-Hugoniot
relations.  alpha is evaluated here with the oracle's discrete operator and
the grid quadrature dv^d sum_q.
"""
from __future__ import annotations

import numpy as np

from . import collision as oc


def mott_smith_alpha(fL: np.ndarray, fR: np.ndarray, vs: oc.VelocitySetup,
                     conserve: bool = False) -> float:
    """alpha = int v_1^2 (Q(f_L, f_R) + Q(f_R, f_L)) dv  (eq. alpha), i.e. twice
    the v_1^2 moment of the pair collision Q_s(f_L, f_R)."""
    q, _ = oc.q_pairs(np.array([np.ravel(fL), np.ravel(fR)]), [(0, 1)], vs, conserve=conserve)
    v1 = oc.grid(vs)[0].reshape(-1)
    return float(2.0 * vs.dv ** vs.d * np.dot(v1 * v1, q[0]))


def mott_smith_beta(alpha: float, d: int, left, right) -> float:
    """beta = alpha / ((d - 1) rho_L u_L R (T_L - T_R)), R = 1; left and right
    are the end states (rho, u_1, T)."""
    (rl, ul, Tl), (_, _, Tr) = left, right
    return alpha / ((d - 1) * rl * ul * (Tl - Tr))


def mott_smith_density(x: np.ndarray, beta: float, left, right) -> np.ndarray:
    """rho(x_1) of the Mott-Smith blend: a rho_L + (1 - a) rho_R with the
    logistic a(x_1) = 1 / (exp(beta x_1) + 1)."""
    rl, rr = left[0], right[0]
    a = 1.0 / (np.exp(beta * np.asarray(x)) + 1.0)
    return a * rl + (1.0 - a) * rr
