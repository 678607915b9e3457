"""Pins of the oracle's collision operator.

The oracle's definition (direct spectral sum with the G+/G- weights) is
checked against routes that share none of its Fourier algebra:
  * a physical-space brute force of eq. (collision_operator) with the
    trigonometric interpolants of g and f, the post-collision velocities of
    eq. (collision velocity) and a fine rule for the inner direction integral;
  * the BKW closed-form solution of the homogeneous equation for Maxwell
    molecules (d f / d t = Q(f, f)), in 2D and 3D;
  * exact discrete invariants: mass, reflection / permutation / periodic
    translation equivariance, bilinearity and symmetry of the gain.
The FFT form of the operator is pinned to the definition.
"""
import math

import numpy as np
import pytest

import synth
from oracle import collision as oc


def _vs(spec, **kw):
    return oc.setup_from_spec(spec) if not kw else oc.setup(
        spec.d, spec.n, spec.L, spec.C, spec.gamma, kw.get("m_rho", spec.m_rho),
        kw.get("m_sigma", spec.m_sigma))


def _interp(ch, vs, U):
    """Trigonometric interpolant sum_k c_k exp(i (pi/L) k.u) at points U (npts, d),
    evaluated by separable explicit sums (no FFT)."""
    kc = oc.centred(vs.N).astype(np.float64)
    E = [np.exp(1j * (math.pi / vs.L) * U[:, i:i + 1] * kc[None, :]) for i in range(vs.d)]
    if vs.d == 2:
        return np.einsum("pa,pb,ab->p", E[0], E[1], ch, optimize=True)
    t = np.einsum("pc,abc->pab", E[2], ch, optimize=True)
    t = np.einsum("pb,pab->pa", E[1], t, optimize=True)
    return np.einsum("pa,pa->p", E[0], t)


def _direction_rule(d, n):
    """Fine rule on S^{d-1} for the inner (relative velocity direction) integral."""
    if d == 2:
        t = 2 * math.pi * np.arange(n) / n
        return np.stack([np.cos(t), np.sin(t)], 1), np.full(n, 2 * math.pi / n)
    x, w = np.polynomial.legendre.leggauss(n)
    ph = 2 * math.pi * np.arange(2 * n) / (2 * n)
    st = np.sqrt(1 - x ** 2)
    pts = np.stack([np.outer(st, np.cos(ph)).ravel(), np.outer(st, np.sin(ph)).ravel(),
                    np.repeat(x, 2 * n)], 1)
    wts = np.repeat(w, 2 * n) * (2 * math.pi / (2 * n))
    return pts, wts


def _brute_force(g, f, vs, q_idx, n_dir):
    """Q+(v) = sum_a w_a rho_a^{d-1} B(rho_a) sum_b w_b int_S g~(v*') f~(v') dqhat,
    v' = v - rho (qhat - sigma)/2, v*' = v - rho (qhat + sigma)/2  (q = v - v*);
    Q-(v) = f~(v) |S^{d-1}| sum_a w_a rho_a^{d-1} B(rho_a) sum_b w_b g~(v - rho_a sigma_b)."""
    gh, fh = oc.coefficients(g, vs), oc.coefficients(f, vs)
    V = oc.grid(vs).reshape(vs.d, -1).T
    qd, wd = _direction_rule(vs.d, n_dir)
    out_p, out_m = [], []
    for qi in q_idx:
        v = V[qi]
        gp = 0.0
        lm = 0.0
        for a, rho in enumerate(vs.rho):
            wa = vs.wrho[a] * rho ** (vs.d - 1) * vs.B(rho)
            for b in range(vs.sig.shape[0]):
                s = vs.sig[b]
                vstar_p = v[None, :] - 0.5 * rho * (qd + s[None, :])
                v_p = v[None, :] - 0.5 * rho * (qd - s[None, :])
                val = _interp(gh, vs, vstar_p) * _interp(fh, vs, v_p)
                gp += wa * vs.wsig[b] * (wd * val).sum()
                lm += wa * vs.wsig[b] * _interp(gh, vs, (v - rho * s)[None, :])[0]
        fv = _interp(fh, vs, v[None, :])[0]
        out_p.append(gp)
        out_m.append(vs.sphere_area * lm * fv)
    return np.array(out_p), np.array(out_m)


def _band_limited(vs, K, seed):
    """Real trigonometric polynomial with random modes |k_i| <= K (so that for
    K < N/4 no sum of two modes wraps around the grid)."""
    rng = np.random.default_rng(seed)
    kv = oc.mode_vectors(vs)
    keep = np.all(np.abs(kv) <= K, axis=0)
    c = (rng.standard_normal(keep.shape) + 1j * rng.standard_normal(keep.shape)) * keep
    h = oc.synthesis(c, vs).real          # real part = Hermitian projection
    return h


@pytest.mark.parametrize("case", ["2d", "3d"])
def test_definition_matches_physical_space_brute_force(case):
    if case == "2d":
        spec, kw, n_dir, pts = synth.small_2d, dict(m_rho=6), 200, [0, 37, 119, 136, 200]
    else:
        spec, kw, n_dir, pts = synth.small_3d, dict(m_rho=3), 32, [0, 219, 292, 365]
    vs = _vs(spec, **kw)
    K = vs.N // 4 - 1
    g = _band_limited(vs, K, 11)
    f = _band_limited(vs, K, 12)
    q, qp, im = oc.q_direct(g, f, vs, parts=True)
    bp, bm = _brute_force(g, f, vs, pts, n_dir)
    scale = np.abs(qp).max()
    assert im < 1e-12 * scale
    assert np.abs(qp.reshape(-1)[pts] - bp.real).max() < 1e-9 * scale
    assert np.abs((qp - q).reshape(-1)[pts] - bm.real).max() < 1e-9 * scale


@pytest.mark.parametrize("spec", [synth.small_2d, synth.small_3d])
def test_fft_form_equals_definition(spec):
    vs = _vs(spec)
    V = synth.smooth_basis(3, spec, seed=5, orthonormal=False)
    for (i, j) in [(0, 1), (2, 2), (1, 2)]:
        q1, q1p, _ = oc.q_direct(V[i], V[j], vs, parts=True)
        q2, q2p = oc.q_fft(V[i], V[j], vs, parts=True)
        s = np.abs(q1p).max()
        assert np.abs(q1 - q2).max() < 1e-13 * s
        assert np.abs(q1p - q2p).max() < 1e-13 * s


def test_c_and_numpy_direct_sums_agree():
    vs = _vs(synth.small_3d)
    V = synth.smooth_basis(2, synth.small_3d, seed=9, orthonormal=False)
    gh, fh = oc.coefficients(V[0], vs), oc.coefficients(V[1], vs)
    ks = np.arange(0, vs.n, 7)
    a = oc.qhat_direct(gh, fh, vs, ks=ks)
    b = oc.qhat_direct_c(gh, fh, vs, ks=ks)
    assert np.abs(a - b).max() < 1e-13 * np.abs(a).max()


def test_coefficient_convention_single_mode():
    vs = _vs(synth.small_2d)
    v = oc.grid(vs)
    k0 = np.array([3, -2])
    h = np.cos((math.pi / vs.L) * (k0[0] * v[0] + k0[1] * v[1]))
    c = oc.coefficients(h, vs)
    N = vs.N
    expect = np.zeros((N, N), dtype=complex)
    expect[k0[0] % N, k0[1] % N] = 0.5
    expect[-k0[0] % N, -k0[1] % N] = 0.5
    assert np.abs(c - expect).max() < 1e-15
    assert np.abs(oc.synthesis(c, vs).real - h).max() < 1e-14


@pytest.mark.parametrize("spec", [synth.small_2d, synth.small_3d])
def test_mass_exact_and_projection(spec):
    vs = _vs(spec)
    V = synth.smooth_basis(2, spec, seed=4, orthonormal=False)
    q, qp = oc.q_fft(V[0], V[1], vs, parts=True)
    m = oc.moments(q, vs)
    mp = oc.moments(qp, vs)
    assert abs(m[0]) < 1e-13 * abs(mp[0])
    qc = oc.conserve_project(q, vs)
    assert np.abs(oc.moments(qc, vs)).max() < 1e-12 * np.abs(mp).max()
    # the correction lies in span{1, v, |v|^2}
    C = oc.moment_matrix(vs)
    corr = q.reshape(-1) - qc
    coef, res, *_ = np.linalg.lstsq(C.T, corr, rcond=None)
    assert np.abs(C.T @ coef - corr).max() < 1e-12 * np.abs(corr).max()


def test_bkw_2d():
    for N, tol in ((32, 2e-3), (64, 2e-6)):
        spec = synth.VGridSpec(d=2, n=N, L=8.0, gamma=0.0, C=1 / (2 * math.pi), m_rho=16, m_sigma=32)
        vs = _vs(spec)
        f, dfdt = synth.c2_bkw(0.5, spec)
        q = oc.q_fft(f, f, vs)
        assert np.abs(q - dfdt).max() < tol * np.abs(dfdt).max()


@pytest.mark.slow
def test_bkw_3d():
    spec = synth.VGridSpec(d=3, n=32, L=8.0, gamma=0.0, C=1 / (4 * math.pi), m_rho=16, m_sigma=38)
    vs = _vs(spec)
    f, dfdt = synth.c2_bkw(0.5, spec)
    q = oc.q_fft(f, f, vs)
    assert np.abs(q - dfdt).max() < 1e-2 * np.abs(dfdt).max()


def test_maxwellian_equilibrium_refines():
    errs = []
    for N in (16, 32, 64):
        spec = synth.VGridSpec(d=2, n=N, L=8.0, gamma=0.0, C=1 / (2 * math.pi), m_rho=16, m_sigma=16)
        vs = _vs(spec)
        M = synth.maxwellian(synth.vgrid_points(2, N, 8.0), 1.0, (0.3, -0.2), 1.0)
        q, qp = oc.q_fft(M, M, vs, parts=True)
        errs.append(np.abs(q).max() / np.abs(qp).max())
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 5e-6


@pytest.mark.parametrize("spec", [synth.small_2d, synth.small_3d])
def test_discrete_symmetries(spec):
    vs = _vs(spec)
    N, d = vs.N, vs.d
    V = synth.smooth_basis(2, spec, seed=21, orthonormal=False)
    g, f = V[0].reshape((N,) * d), V[1].reshape((N,) * d)
    q = oc.q_fft(g, f, vs).reshape((N,) * d)
    s = np.abs(q).max()
    # reflection v_1 -> -v_1  (q -> -q mod N on the grid)
    ref = lambda h: np.roll(np.flip(h, axis=0), 1, axis=0)
    assert np.abs(oc.q_fft(ref(g), ref(f), vs).reshape(q.shape) - ref(q)).max() < 1e-13 * s
    # axis swap
    sw = lambda h: np.swapaxes(h, 0, 1)
    assert np.abs(oc.q_fft(sw(g), sw(f), vs).reshape(q.shape) - sw(q)).max() < 1e-13 * s
    # periodic translation by one cell
    tr = lambda h: np.roll(h, 1, axis=d - 1)
    assert np.abs(oc.q_fft(tr(g), tr(f), vs).reshape(q.shape) - tr(q)).max() < 1e-13 * s
    # bilinearity and symmetry of the gain
    h = V[0].reshape(q.shape) * 0.3 - 1.7 * V[1].reshape(q.shape)
    lhs = oc.q_fft(g, 2.0 * f + h, vs)
    rhs = 2.0 * q + oc.q_fft(g, h, vs)
    assert np.abs(lhs - rhs).max() < 1e-13 * s
    _, p1 = oc.q_fft(g, f, vs, parts=True)
    _, p2 = oc.q_fft(f, g, vs, parts=True)
    assert np.abs(p1 - p2).max() < 1e-13 * np.abs(p1).max()
