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
