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
* Maxwell diffusive walls: the assembled boundary row (wall Maxwellian on
  the incoming half, the adjacent cell on the outgoing half) carries no net
  mass flux, so two walls conserve the total mass to rounding while energy
  flows in from the hotter wall; for gas leaving as rho M_T the wall density
  converges to the continuum half-range balance rho sqrt(T / T_w) with the
  second-order error term that Euler-Maclaurin predicts for the half-range
  sums (integrands with a kink at v_1 = 0).
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


def _wall_problem(nx=10, N=16, pert=1e-2):
    spec = _spec2(N=N, m_rho=8)
    vs = oc.setup_from_spec(spec)
    ini = synth.wall_initial(spec, nx, 0.0, 2.0, T_walls=(1.0, 1.2), pert=pert, pert_rank=3,
                             seed=5)
    prob = dlr.Problem1D(vs=vs, nx=nx, x_lo=0.0, x_hi=2.0, fL=ini["fL"], fR=ini["fR"],
                         conserve=True, wall_left=True, wall_right=True)
    return prob, ini


def test_wall_rows_carry_no_net_mass_flux():
    prob, ini = _wall_problem()
    F = ini["f0"]
    v1 = prob.v1()
    for side, f_adj, inflow in ((0, F[0], v1 > 0), (1, F[-1], v1 < 0)):
        row = np.where(inflow, dlr.boundary_function(side, f_adj, prob), f_adj)
        assert abs(np.sum(v1 * row)) < 1e-14 * np.sum(np.abs(v1 * row))
        assert dlr.wall_density(f_adj, prob.fL if side == 0 else prob.fR, prob, side) > 0


def test_diffusive_walls_conserve_mass():
    prob, ini = _wall_problem()
    F = ini["f0"]
    C = oc.moment_matrix(prob.vs)                 # rows dv^d {1, v_1, v_2, |v|^2}
    m0 = prob.dx * F.sum(axis=0) @ C.T
    for _ in range(5):
        F, _ = dlr.full_step(F, prob, 0.01)
    m1 = prob.dx * F.sum(axis=0) @ C.T
    assert abs(m1[0] - m0[0]) < 1e-14 * m0[0]
    assert m1[-1] - m0[-1] > 1e-4 * m0[-1]        # heat flows in from the T = 1.2 wall


def test_wall_density_converges_to_the_half_range_balance():
    """Euler-Maclaurin for the half-range sums (h sum_{k>=1} g(kh) with g(0) =
    0, g'(0) = 1 per unit density after the v_2 sum, which is spectrally
    exact) gives the discrete value rho sqrt(T/T_w) (1 - h^2 (1/T - 1/T_w)/12
    + O(h^4)): the error per h^2 is pinned to that coefficient."""
    rho, T, Tw = 1.3, 0.8, 1.25
    exact = rho * math.sqrt(T / Tw)
    coef = -exact * (1.0 / T - 1.0 / Tw) / 12.0
    errs = []
    for N in (64, 128, 256):
        spec = synth.VGridSpec(d=2, n=N, L=12.0, gamma=0.0, C=1 / (2 * math.pi), m_rho=4,
                               m_sigma=8)
        vs = oc.setup_from_spec(spec)
        v = synth.vgrid_points(2, N, spec.L)
        f = synth.maxwellian(v, rho, (0.0, 0.0), T).reshape(-1)
        M = synth.maxwellian(v, 1.0, (0.0, 0.0), Tw).reshape(-1)
        prob = dlr.Problem1D(vs=vs, nx=2, x_lo=0.0, x_hi=1.0, fL=M, fR=M, wall_left=True,
                             wall_right=True)
        e = [dlr.wall_density(f, M, prob, side) - exact for side in (0, 1)]
        assert abs(e[0] - e[1]) < 1e-13                # both walls see the same balance
        errs.append(e[0] / (2.0 * spec.L / N) ** 2)
    assert abs(errs[-1] - coef) < 0.005 * abs(coef)
    assert abs(errs[-1] - coef) < abs(errs[0] - coef)


def test_uniform_gas_at_wall_temperature_is_transport_free():
    """Both walls at T_w and the gas a uniform Maxwellian at T_w: rho_w equals
    the gas density and the step changes f by dt Q(f, f) alone.  Up to the
    grid's one-sided node v_1 = -L (its mirror +L is not a node): the two
    half-range sums then differ by the Maxwellian's tail there, relative
    size exp(-L^2 / 2 T_w) ~ 3e-13."""
    spec = _spec2(N=16)
    vs = oc.setup_from_spec(spec)
    v = synth.vgrid_points(2, spec.n, spec.L)
    M = synth.maxwellian(v, 1.0, (0.0, 0.0), 1.1).reshape(-1)
    prob = dlr.Problem1D(vs=vs, nx=6, x_lo=0.0, x_hi=2.0, fL=M, fR=M, conserve=True,
                         wall_left=True, wall_right=True)
    F = np.tile(0.7 * M, (6, 1))
    dt = 0.01
    Fn, _ = dlr.full_step(F, prob, dt)
    Q, _ = dlr.evaluate_pairs(F, [(p, p) for p in range(6)], prob)
    assert np.abs(Fn - F - dt * Q).max() < 1e-12 * np.abs(F).max()
