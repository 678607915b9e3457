"""Checks of the seeded input generator (not of the method)."""
import math

import numpy as np
import pytest

import synth


@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("mach", [1.2, 1.5, 2.0, 3.0, 3.8, 6.5])
def test_rankine_hugoniot_fluxes(d, mach):
    """The closed-form downstream state conserves the fluxes of mass,
    momentum and energy (Sec. 4, eq. normal_shock_conservation2)."""
    (rl, ul, Tl), (rr, ur, Tr) = synth.rh_downstream(mach, d)
    assert abs(rl * ul - rr * ur) < 1e-13 * rl * ul
    assert abs(rl * ul ** 2 + rl * Tl - (rr * ur ** 2 + rr * Tr)) < 1e-13 * rl * ul ** 2
    e = lambda r, u, T: r * u * (u ** 2 + (d + 2) * T)
    assert abs(e(rl, ul, Tl) - e(rr, ur, Tr)) < 1e-12 * e(rl, ul, Tl)


def test_paper_d2_downstream_formulas():
    """Sec. 5.2 writes the d = 2 states as rho_R = 3M^2/(M^2+2), u_L = sqrt 2 M,
    T_R = (4M^2-1)/(3 rho_R); they agree with the general relation."""
    for M in (1.4, 3.8, 6.5):
        (rl, ul, Tl), (rr, ur, Tr) = synth.rh_downstream(M, 2)
        assert abs(ul - math.sqrt(2) * M) < 1e-14 * ul
        assert abs(rr - 3 * M * M / (M * M + 2)) < 1e-14 * rr
        assert abs(Tr - (4 * M * M - 1) / (3 * rr)) < 1e-13 * Tr


def test_lowrank_state_orthonormal_and_reconstructs():
    spec = synth.VGridSpec(d=2, n=16, L=8.0)
    ini = synth.shock_initial(1.5, spec, 32, pert_rank=3)
    dx = 60.0 / 32
    dvd = (16.0 / 16) ** 2
    X, S, V = synth.lowrank_state(ini["f0"], 12, dx, dvd)
    assert np.abs(dx * X.T @ X - np.eye(12)).max() < 1e-12
    assert np.abs(dvd * V @ V.T - np.eye(12)).max() < 1e-12
    assert np.abs(X @ S @ V - ini["f0"]).max() < 1e-6 * np.abs(ini["f0"]).max()


def test_seeded_inputs_are_deterministic():
    a = synth.c1_distribution()
    b = synth.c1_distribution()
    assert np.array_equal(a, b)
    assert np.array_equal(synth.smooth_basis(3, synth.C2, seed=4), synth.smooth_basis(3, synth.C2, seed=4))


def test_sketched_lowrank_state_matches_the_svd():
    """The randomized range finder gives the same truncation as the full SVD
    (singular values, reconstruction) on shock data, with orthonormal factors."""
    spec = synth.VGridSpec(d=2, n=16, L=8.0)
    ini = synth.shock_initial(2.0, spec, 64, pert=1e-3, pert_rank=6, seed=9)
    dx, dvd = 60.0 / 64, (16.0 / 16) ** 2
    X, S, V = synth.lowrank_state(ini["f0"], 8, dx, dvd)
    Xs, Ss, Vs = synth.lowrank_state_sketch(ini["f0"], 8, dx, dvd, seed=1)
    assert np.abs(dx * Xs.T @ Xs - np.eye(8)).max() < 1e-12
    assert np.abs(dvd * Vs @ Vs.T - np.eye(8)).max() < 1e-12
    assert np.abs(np.diag(Ss) - np.diag(S)).max() < 1e-9 * S[0, 0]
    f = X @ S @ V
    assert np.abs(Xs @ Ss @ Vs - f).max() < 1e-8 * np.abs(f).max()


def test_serving_trace_recipe():
    tr = synth.serving_trace(count=400, seed=5, rate=4.0)
    assert tr[:16] == synth.serving_trace(count=16, seed=5, rate=4.0)   # prefix-stable
    t = np.array([q["arrival"] for q in tr])
    assert t[0] == 0.0 and np.all(np.diff(t) > 0)
    gaps = np.diff(t)
    assert abs(gaps.mean() - 0.25) < 0.04          # Poisson arrivals at 4 per second
    assert abs(gaps.std() / gaps.mean() - 1.0) < 0.15   # exponential gaps: CV = 1
    for q in tr:
        assert 1.2 <= q["mach"] <= 3.0 and 5 <= q["r0"] <= 25
        assert q["nx"] in (128, 256, 512) and q["n"] in (24, 32)
        assert q["L"] == {24: 8.0, 32: 10.0}[q["n"]]
        dx = 60.0 / q["nx"]
        R = 4.0 * q["L"] / (3.0 + math.sqrt(2.0))
        nu = 4.0 * math.pi * R * synth.rh_downstream(q["mach"], 3)[1][0]
        assert q["dt"] <= 0.5 * 0.35 * dx / q["L"] + 1e-15
        assert q["dt"] * nu <= 0.75 + 1e-12
        assert q["dt"] == min(0.5 * 0.35 * dx / q["L"], 0.5 * 1.5 / nu)
