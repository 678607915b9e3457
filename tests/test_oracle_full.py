"""Pins of the oracle's full-tensor reference step (eq. scheme:fullupwind of
Sec. 2.2 with forward Euler, walls of Sec. 2.3, err_full of eq. err full grid).

* A profile linear in x, the same for every velocity, with ghosts on the same
  line: both one-sided differences equal the slope b exactly, so the step is
  f - dt b (v^+ + v^-) = f - dt b v_1 in every cell (no collisions).
* A uniform Maxwellian with matching inflow stays put and err_full = 0.
* Discrete balance of mass, momentum and energy: the upwind differences
  telescope over the cells and Q_s conserves the collision invariants, so the
  change of each moment is the boundary flux alone,
  dM_k = -dt dv^d sum_q phi_k [v^+ (f_{nx-1} - g_L) + v^- (g_R - f_0)].
"""
import math

import numpy as np

import synth
from oracle import collision as oc
from oracle import dlr


def _spec2(N=16, m_rho=8):
    return synth.VGridSpec(d=2, n=N, L=8.0, gamma=0.0, C=1 / (2 * math.pi), m_rho=m_rho,
                           m_sigma=8)


def _no_collision(V, pairs, vs, conserve):
    z = np.zeros((len(pairs), V.shape[1]))
    return z, z


def test_linear_profile_is_advected_exactly():
    spec = _spec2(N=8)
    vs = oc.setup_from_spec(spec)
    nx, a, b, dt = 7, 0.3, 0.05, 0.01
    prob = dlr.Problem1D(vs=vs, nx=nx, x_lo=-3.5, x_hi=3.5, fL=None, fR=None,
                         collision=_no_collision)
    x = synth.xgrid_centres(nx, prob.x_lo, prob.x_hi)
    n = vs.n
    F = (a + b * x)[:, None] * np.ones((1, n))
    prob.fL = np.full(n, a + b * (x[0] - prob.dx))
    prob.fR = np.full(n, a + b * (x[-1] + prob.dx))
    Fn, err = dlr.full_step(F, prob, dt)
    v1 = prob.v1()
    expect = F - dt * b * v1[None, :]
    assert np.abs(Fn - expect).max() < 1e-15
    assert abs(err - math.sqrt(prob.dx * prob.dvd * nx * ((dt * b * v1) ** 2).sum())) < 1e-15


def test_uniform_equilibrium_is_steady():
    spec = _spec2(N=8)
    vs = oc.setup_from_spec(spec)
    v = synth.vgrid_points(2, spec.n, spec.L)
    M = synth.maxwellian(v, 1.2, (0.7, 0.0), 0.9).reshape(-1)
    prob = dlr.Problem1D(vs=vs, nx=5, x_lo=0.0, x_hi=1.0, fL=M, fR=M, collision=_no_collision)
    F = np.tile(M, (5, 1))
    Fn, err = dlr.full_step(F, prob, 0.05)
    assert np.array_equal(Fn, F)
    assert err == 0.0


def test_moment_balance_is_the_boundary_flux():
    spec = _spec2(N=16, m_rho=8)
    vs = oc.setup_from_spec(spec)
    nx, dt = 10, 0.02
    ini = synth.shock_initial(1.6, spec, nx, -4.0, 4.0, pert=1e-2, pert_rank=3, seed=11)
    prob = dlr.Problem1D(vs=vs, nx=nx, x_lo=-4.0, x_hi=4.0, fL=ini["fL"], fR=ini["fR"],
                         conserve=True)
    F = ini["f0"]
    Fn, _ = dlr.full_step(F, prob, dt)
    C = oc.moment_matrix(vs)                       # rows dv^d {1, v_1, v_2, |v|^2}
    dM = prob.dx * (Fn - F).sum(axis=0) @ C.T      # change of the x-integrated moments
    v1 = prob.v1()
    vp, vm = np.maximum(v1, 0.0), np.minimum(v1, 0.0)
    gL = np.where(v1 > 0, prob.fL, F[0])
    gR = np.where(v1 < 0, prob.fR, F[-1])
    flux = -dt * (vp * (F[-1] - gL) + vm * (gR - F[0]))
    expect = flux @ C.T
    scale = np.abs(prob.dx * np.abs(F).sum(axis=0) @ np.abs(C).T).max()
    assert np.abs(dM - expect).max() < 1e-13 * scale
    # without the projection the collision moments no longer vanish exactly
    prob.conserve = False
    Fn2, _ = dlr.full_step(F, prob, dt)
    dM2 = prob.dx * (Fn2 - F).sum(axis=0) @ C.T
    assert np.abs(dM2 - expect).max() > 10 * np.abs(dM - expect).max()
