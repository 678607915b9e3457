"""Pins of the Carleman-form collision operator (oracle/carleman.py).

* The fast form (filtered transforms, products, direction sum) equals the
  weighted direct sum that defines the discrete operator.
* The closed-form filters equal their defining integrals, evaluated by
  adaptive quadrature (the 3D disc integral in polar coordinates, so J1 is
  not used on the reference side).
* Mass is conserved exactly (beta(l, -l) = beta(l, l)); in 2D with an even
  number of directions the gain is symmetric in its arguments.
* The BKW closed-form solution (2D Maxwell molecules): Q(f, f) = df/dt.
* Mott-Smith alpha for the Rankine-Hugoniot Maxwellians against the
  untruncated closed form: 2D Maxwell molecules -rho_L rho_R (u_L - u_R)^2 / 4
  (from the weak form, see test_oracle_shock.py); 3D hard spheres
  (C/2) 4 pi rho_L rho_R E[|q| (|q|^2/3 - q_1^2)], q ~ N((u_L - u_R) e_1,
  (T_L + T_R) I), reduced to a radial integral with the modified spherical
  Bessel function i_2 and evaluated by adaptive quadrature.  A large box
  makes truncation and wrap-around negligible.
* On smooth inputs it agrees with the (rho, sigma) form of oracle/collision.py
  (two discretisations of the same operator).
"""
import math

import numpy as np
import pytest
import scipy.integrate as si
import scipy.special as ss

import synth
from oracle import carleman as ca
from oracle import collision as oc


def _cs(d, N, L=8.0, M=0):
    return ca.setup(d, N, L, 1 / (2 * math.pi) if d == 2 else 1.0, M)


@pytest.mark.parametrize("d,N,M", [(2, 16, 8), (2, 16, 6), (3, 8, 38)])
def test_fast_form_equals_definition(d, N, M):
    cs = _cs(d, N, M=M)
    spec = synth.VGridSpec(d=d, n=N, L=8.0, gamma=d - 2, C=cs.C, m_rho=4,
                           m_sigma=M if d == 2 else 38)
    V = synth.smooth_basis(2, spec, seed=3)
    a, ap, am = ca.q_direct(V[0], V[1], cs, parts=True)
    b, bp, bm = ca.q_fft(V[0], V[1], cs, parts=True)
    scale = np.abs(bp).max()
    assert np.abs(a - b).max() < 1e-13 * scale
    assert np.abs(ap - bp).max() < 1e-13 * scale
    assert abs(a.sum()) < 1e-14 * np.abs(bp).sum()          # exact mass conservation


@pytest.mark.parametrize("s", [0.0, 0.3, 1.7, 5.0, 12.5])
def test_filters_equal_their_integrals(s):
    for d in (2, 3):
        cs = _cs(d, 16)
        ref = si.quad(lambda r: abs(r) ** (d - 2) * math.cos(math.pi * r * s / cs.L), -cs.R, cs.R,
                      epsabs=1e-13, limit=400)[0]
        assert abs(float(ca.phi(cs, s)) - ref) < 1e-10 * max(1.0, abs(ref))
    cs = _cs(3, 16)
    k = np.array([s, 0.5 * s, -1.0]).reshape(3, 1)
    for p in (0, 4, 11):
        e = cs.dirs[p]
        kp = k[:, 0] - (k[:, 0] @ e) * e                    # component in the disc's plane
        b = math.pi * np.linalg.norm(kp) / cs.L
        ref = si.dblquad(lambda t, r: r * math.cos(b * r * math.cos(t)), 0, cs.R, 0, 2 * math.pi,
                         epsabs=1e-11)[0]
        assert abs(float(ca.psi(cs, k, p)[0]) - ref) < 1e-9 * max(1.0, abs(ref))


def test_2d_gain_is_symmetric():
    cs = _cs(2, 32, M=8)
    spec = synth.VGridSpec(d=2, n=32, L=8.0, gamma=0.0, C=cs.C, m_rho=4, m_sigma=8)
    V = synth.smooth_basis(2, spec, seed=8)
    _, g1, _ = ca.q_fft(V[0], V[1], cs, parts=True)
    _, g2, _ = ca.q_fft(V[1], V[0], cs, parts=True)
    assert np.abs(g1 - g2).max() < 1e-14 * np.abs(g1).max()


def test_bkw_2d():
    spec = synth.VGridSpec(d=2, n=64, L=8.0, gamma=0.0, C=1 / (2 * math.pi), m_rho=4, m_sigma=8)
    cs = _cs(2, 64, M=8)
    f, dfdt = synth.c2_bkw(0.5, spec)
    q = ca.q_fft(f, f, cs)
    assert np.abs(q - dfdt).max() < 1e-6 * np.abs(dfdt).max()


def _alpha(cs, mach):
    d = cs.d
    left, right = synth.rh_downstream(mach, d)
    v = synth.vgrid_points(d, cs.N, cs.L)
    fL = synth.maxwellian(v, left[0], (left[1],) + (0.0,) * (d - 1), left[2]).reshape(-1)
    fR = synth.maxwellian(v, right[0], (right[1],) + (0.0,) * (d - 1), right[2]).reshape(-1)
    q, _ = ca.q_pairs(np.array([fL, fR]), [(0, 1)], cs, conserve=False)
    return 2.0 * cs.dv ** d * float(np.dot(v[0].reshape(-1) ** 2, q[0])), left, right


def test_mott_smith_alpha_2d_maxwell():
    cs = ca.setup(2, 128, 16.0, 1 / (2 * math.pi), 16)
    a, left, right = _alpha(cs, 1.4)
    closed = -0.25 * left[0] * right[0] * (left[1] - right[1]) ** 2
    assert abs(a - closed) < 1e-8 * abs(closed)


@pytest.mark.slow
def test_mott_smith_alpha_3d_hard_spheres():
    cs = ca.setup(3, 64, 16.0, 1.0, 38)
    a, left, right = _alpha(cs, 1.4)
    mu, s2 = abs(left[1] - right[1]), left[2] + right[2]
    f = lambda r: r ** 5 * math.exp(-(r * r + mu * mu) / (2 * s2)) * ss.spherical_in(2, mu * r / s2)
    I = si.quad(f, 0.0, 80.0, epsabs=0, epsrel=1e-13, limit=400)[0]
    closed = (0.5 * 4 * math.pi * left[0] * right[0] * (-2.0 / 3.0) * (2 * math.pi * s2) ** -1.5
              * 4 * math.pi * I)
    assert abs(a - closed) < 1e-6 * abs(closed)


def test_agrees_with_the_rho_sigma_form():
    spec = synth.VGridSpec(d=2, n=32, L=8.0, gamma=0.0, C=1 / (2 * math.pi), m_rho=16,
                           m_sigma=32)
    V = synth.smooth_basis(2, spec, seed=5)
    q1, g1 = oc.q_pairs(V, [(0, 1)], oc.setup_from_spec(spec), conserve=False)
    q2, _ = ca.q_pairs(V, [(0, 1)], _cs(2, 32, M=16), conserve=False)
    assert np.linalg.norm(q1 - q2) < 1e-4 * np.linalg.norm(g1)
