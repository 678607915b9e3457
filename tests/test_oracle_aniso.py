"""Pins of the oracle's anisotropic-kernel operator (oracle/aniso.py).

* The definition (direct spectral sum with the sigma-dependent F_ab) against
  a physical-space brute force of eq. (collision_operator): trigonometric
  interpolants at the post-collision velocities and the kernel's angular
  factor B(rho, sigma . q^) under a fine rule for the direction integral.
  This shares none of the Fourier algebra (Funk-Hecke factors, signs of the
  sigma phase, the (-i)^n).
* F_ab(k) against the direction integral it stands for.
* beta = (1,) equals the isotropic operator; the FFT form equals the
  definition; mass is exact; the symmetrised pair operator does not see odd
  Legendre / Chebyshev components (B(rho, -c) enters through the antipodal
  partner).
"""
import math

import numpy as np
import pytest

import synth
from oracle import aniso as oa
from oracle import collision as oc

BETA3 = (0.8, 0.45, 0.3, -0.1)   # 3D: B / (C rho^gamma) = 0.8 + 0.45 P1 + 0.3 P2 - 0.1 P3 > 0 on [-1, 1]
BETA2 = (0.9, 0.4, 0.25)         # 2D: 0.9 + 0.4 T1 + 0.25 T2 > 0


def _vs(d):
    if d == 2:
        return oc.setup(2, 16, 8.0, 1 / (2 * math.pi), 0.0, 6, 8)
    return oc.setup(3, 8, 8.0, 1.0, 1.0, 3, 38)


def _interp(ch, vs, U):
    kc = oc.centred(vs.N).astype(np.float64)
    E = [np.exp(1j * (math.pi / vs.L) * U[:, i:i + 1] * kc[None, :]) for i in range(vs.d)]
    if vs.d == 2:
        return np.einsum("pa,pb,ab->p", E[0], E[1], ch, optimize=True)
    t = np.einsum("pc,abc->pab", E[2], ch, optimize=True)
    t = np.einsum("pb,pab->pa", E[1], t, optimize=True)
    return np.einsum("pa,pa->p", E[0], t)


def _direction_rule(d, n):
    if d == 2:
        t = 2 * math.pi * np.arange(n) / n
        return np.stack([np.cos(t), np.sin(t)], 1), np.full(n, 2 * math.pi / n)
    x, w = np.polynomial.legendre.leggauss(n)
    ph = 2 * math.pi * np.arange(2 * n) / (2 * n)
    st = np.sqrt(1 - x ** 2)
    pts = np.stack([np.outer(st, np.cos(ph)).ravel(), np.outer(st, np.sin(ph)).ravel(),
                    np.repeat(x, 2 * n)], 1)
    return pts, np.repeat(w, 2 * n) * (2 * math.pi / (2 * n))


def _band_limited(vs, K, seed):
    rng = np.random.default_rng(seed)
    kv = oc.mode_vectors(vs)
    keep = np.all(np.abs(kv) <= K, axis=0)
    c = (rng.standard_normal(keep.shape) + 1j * rng.standard_normal(keep.shape)) * keep
    return oc.synthesis(c, vs).real


def _brute_gain(g, f, vs, beta, q_idx, n_dir):
    """Q+(v) = sum_a w_a rho_a^{d-1} sum_b w_b int_S B(rho_a, sigma_b . q^)
    g~(v - rho (q^ + sigma_b)/2) f~(v - rho (q^ - sigma_b)/2) dq^."""
    gh, fh = oc.coefficients(g, vs), oc.coefficients(f, vs)
    V = oc.grid(vs).reshape(vs.d, -1).T
    qd, wd = _direction_rule(vs.d, n_dir)
    out = []
    for qi in q_idx:
        v = V[qi]
        acc = 0.0
        for a, rho in enumerate(vs.rho):
            for b in range(vs.sig.shape[0]):
                s = vs.sig[b]
                wB = oa.B(vs, beta, rho, qd @ s)
                val = _interp(gh, vs, v[None, :] - 0.5 * rho * (qd + s[None, :])) * \
                    _interp(fh, vs, v[None, :] - 0.5 * rho * (qd - s[None, :]))
                acc += vs.wrho[a] * rho ** (vs.d - 1) * vs.wsig[b] * (wd * wB * val).sum()
        out.append(acc)
    return np.array(out)


@pytest.mark.parametrize("d", [2, 3])
def test_definition_matches_physical_space_brute_force(d):
    vs = _vs(d)
    beta = BETA2 if d == 2 else BETA3
    n_dir, pts = (240, [0, 37, 119, 200]) if d == 2 else (36, [0, 219, 365])
    K = vs.N // 4 - 1
    g, f = _band_limited(vs, K, 21), _band_limited(vs, K, 22)
    q, qp, im = oa.q_direct(g, f, vs, beta, parts=True)
    bp = _brute_gain(g, f, vs, beta, pts, n_dir)
    scale = np.abs(qp).max()
    assert im < 1e-12 * scale
    assert np.abs(qp.reshape(-1)[pts] - bp.real).max() < 1e-9 * scale
    assert np.abs(bp.imag).max() < 1e-9 * scale


@pytest.mark.parametrize("d", [2, 3])
def test_funk_hecke_table_is_the_direction_integral(d):
    vs = _vs(d)
    beta = BETA2 if d == 2 else BETA3
    Ft = oa.F_table(vs, beta)
    k = oc.mode_vectors(vs).reshape(d, -1).T.astype(np.float64)
    qd, wd = _direction_rule(d, 400 if d == 2 else 48)
    for a in (0, len(vs.rho) - 1):
        th = math.pi * vs.rho[a] / (2 * vs.L)
        for b in (0, 3, 5):
            for kidx in (0, 1, 7, 23, vs.n // 2 + 3):
                direct = (wd * oa.B(vs, beta, vs.rho[a], qd @ vs.sig[b]) *
                          np.exp(-1j * th * (qd @ k[kidx]))).sum()
                assert abs(direct - Ft[a, b, kidx]) < 1e-11 * max(1.0, abs(direct))


@pytest.mark.parametrize("d", [2, 3])
def test_isotropic_limit_and_fft_form(d):
    vs = _vs(d)
    spec = synth.small_2d if d == 2 else synth.small_3d
    V = synth.smooth_basis(3, spec, seed=5, orthonormal=False)
    # beta = (1,) is the isotropic operator
    q_iso, qp_iso = oc.q_fft(V[0], V[1], vs, parts=True)
    q_a, qp_a = oa.q_fft(V[0], V[1], vs, (1.0,), parts=True)
    s = np.abs(qp_iso).max()
    assert np.abs(q_iso - q_a).max() < 1e-13 * s
    # the fast form equals the definition
    beta = BETA2 if d == 2 else BETA3
    q1, q1p, _ = oa.q_direct(V[1], V[2], vs, beta, parts=True)
    q2, q2p = oa.q_fft(V[1], V[2], vs, beta, parts=True)
    s = np.abs(q1p).max()
    assert np.abs(q1 - q2).max() < 1e-13 * s
    assert np.abs(q1p - q2p).max() < 1e-13 * s
    # mass exact
    assert abs(oc.moments(q2, vs)[0]) < 1e-13 * np.abs(oc.moments(q2p, vs)[0])


@pytest.mark.parametrize("d", [2, 3])
def test_symmetrised_pairs_see_only_even_components(d):
    vs = _vs(d)
    spec = synth.small_2d if d == 2 else synth.small_3d
    V = synth.smooth_basis(2, spec, seed=8, orthonormal=False)
    beta = BETA2 if d == 2 else BETA3
    even = tuple(b if n % 2 == 0 else 0.0 for n, b in enumerate(beta))
    a, ga = oa.q_pairs(V, [(0, 1), (1, 1)], vs, beta, conserve=False)
    b, gb = oa.q_pairs(V, [(0, 1), (1, 1)], vs, even, conserve=False)
    s = np.abs(ga).max()
    assert np.abs(a - b).max() < 1e-13 * s
    # but the unsymmetrised operator does see them
    q_odd = oa.q_fft(V[0], V[1], vs, beta) - oa.q_fft(V[0], V[1], vs, even)
    assert np.abs(q_odd).max() > 1e-3 * s
