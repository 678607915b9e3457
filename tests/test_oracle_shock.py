"""Pins of the Mott-Smith quantities of Sec. 4 (oracle/shock.py).

alpha = int v_1^2 (Q(f_L, f_R) + Q(f_R, f_L)) dv for the two Rankine-Hugoniot
Maxwellians.  For Maxwell molecules (B = C) the weak form of Q gives, with
q = v - v* and the post-collision velocities of eq. (collision velocity),

    phi(v') + phi(v*') - phi(v) - phi(v*) = (|q|^2 sigma_1^2 - q_1^2) / 2,   phi = v_1^2,

and int sigma_1^2 dsigma = |S^{d-1}| / d, so alpha = (C |S^{d-1}| / 2) *
rho_L rho_R E[|q|^2 / d - q_1^2], q ~ N((u_L - u_R) e_1, (T_L + T_R) I).  The
operator on the grid truncates the kernel at |q| <= R; the same expectation
restricted to the ball |q| <= R reduces, after the angular integral, to

    2D:  -(C / 2) rho_L rho_R / s^2 * int_0^R r^3 exp(-(r^2 + mu^2) / 2s^2) I_2(mu r / s^2) dr
    3D:  -(4/3) C (2 pi)^(1/2) ... (see _alpha_ball)

(I_2 the modified Bessel function, i_2 the modified spherical one), computed
here by adaptive quadrature: nothing of the spectral operator enters it.  As
R -> infinity it must equal the untruncated closed form
-C |S^{d-1}| (d-1)/(2d) rho_L rho_R (u_L - u_R)^2 (temperatures drop out).
The oracle's alpha (its discrete operator on Maxwellians) must approach the
truncated value when the grid resolves the Maxwellians and the box holds
their relative-velocity support without wrap-around.
"""
import math

import numpy as np
import pytest
import scipy.integrate as si
import scipy.special as ss

import synth
from oracle import collision as oc
from oracle import shock


def _alpha_ball(d, C, R, left, right):
    (rl, ul, Tl), (rr, ur, Tr) = left, right
    mu, s2 = abs(ul - ur), Tl + Tr
    if d == 2:
        # |q|^2/2 - q_1^2 = -(r^2/2) cos 2theta; int cos 2theta e^{k cos theta} = 2 pi I_2(k)
        f = lambda r: r ** 3 * math.exp(-(r * r + mu * mu) / (2 * s2)) * ss.iv(2, mu * r / s2)
        I = si.quad(f, 0.0, R, epsabs=0, epsrel=1e-13, limit=200)[0]
        return 0.5 * C * 2 * math.pi * rl * rr * (-0.5) / (2 * math.pi * s2) * 2 * math.pi * I
    # |q|^2/3 - q_1^2 = -(2/3) r^2 P_2(cos theta); int P_2(x) e^{k x} dx over [-1,1] = 2 i_2(k)
    f = lambda r: r ** 4 * math.exp(-(r * r + mu * mu) / (2 * s2)) * ss.spherical_in(2, mu * r / s2)
    I = si.quad(f, 0.0, R, epsabs=0, epsrel=1e-13, limit=200)[0]
    return (0.5 * C * 4 * math.pi * rl * rr * (-2.0 / 3.0) * (2 * math.pi * s2) ** -1.5
            * 4 * math.pi * I)


def _maxwellians(d, n, L, mach):
    left, right = synth.rh_downstream(mach, d)
    v = synth.vgrid_points(d, n, L)
    fL = synth.maxwellian(v, left[0], (left[1],) + (0.0,) * (d - 1), left[2]).reshape(-1)
    fR = synth.maxwellian(v, right[0], (right[1],) + (0.0,) * (d - 1), right[2]).reshape(-1)
    return left, right, fL, fR


@pytest.mark.parametrize("d,mach", [(2, 1.4), (2, 3.0), (3, 1.4), (3, 2.5)])
def test_ball_integral_tends_to_the_closed_form(d, mach):
    C = 1 / (2 * math.pi) if d == 2 else 1 / (4 * math.pi)
    left, right = synth.rh_downstream(mach, d)
    S = 2 * math.pi if d == 2 else 4 * math.pi
    closed = -C * S * (d - 1) / (2 * d) * left[0] * right[0] * (left[1] - right[1]) ** 2
    assert abs(_alpha_ball(d, C, 80.0, left, right) - closed) < 1e-12 * abs(closed)
    # truncation only removes a tail of the same sign
    assert 0 < _alpha_ball(d, C, 7.0, left, right) / closed < 1.0


@pytest.mark.parametrize("d,n,L,m_rho,m_sigma,tol", [(2, 64, 12.0, 16, 32, 1e-9),
                                                     (3, 24, 8.0, 16, 38, 1e-5)])
def test_alpha_of_the_discrete_operator(d, n, L, m_rho, m_sigma, tol):
    C = 1 / (2 * math.pi) if d == 2 else 1 / (4 * math.pi)
    spec = synth.VGridSpec(d=d, n=n, L=L, gamma=0.0, C=C, m_rho=m_rho, m_sigma=m_sigma)
    vs = oc.setup_from_spec(spec)
    left, right, fL, fR = _maxwellians(d, n, L, 1.4)
    a = shock.mott_smith_alpha(fL, fR, vs)
    ref = _alpha_ball(d, C, vs.R, left, right)
    assert abs(a - ref) <= tol * abs(ref)


def test_logistic_profile_solves_the_moment_equation():
    """a(x) = 1/(exp(beta x)+1) solves (d-1) rho_L u_L (T_L - T_R) a' = -alpha a (1-a)
    (Sec. 4), and the density runs from rho_L to rho_R."""
    d, mach, alpha = 2, 1.4, -0.155
    left, right = synth.rh_downstream(mach, d)
    beta = shock.mott_smith_beta(alpha, d, left, right)
    assert beta > 0
    x = np.linspace(-20, 20, 4001)
    rho = shock.mott_smith_density(x, beta, left, right)
    a = (rho - right[0]) / (left[0] - right[0])
    da = np.gradient(a, x)
    lhs = (d - 1) * left[0] * left[1] * (left[2] - right[2]) * da
    assert np.abs(lhs[1:-1] + alpha * a[1:-1] * (1 - a[1:-1])).max() < 1e-5
    far = shock.mott_smith_density(np.array([-40 / beta, 40 / beta]), beta, left, right)
    assert abs(far[0] - left[0]) < 1e-12 and abs(far[1] - right[0]) < 1e-12
