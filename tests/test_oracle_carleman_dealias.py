"""Pins of the oracle's de-aliased Carleman form (oracle/carleman.py): the
Galerkin sum over l + m = k exactly, the reading of the spectral method's
convolution that the de-aliased option follows (the default is the circular
sum an N-point transform computes).

* the exact direct sum (the beta(l, m) matrix of the definition) equals the
  fast form on the padded 2N-point grid;
* on inputs band-limited to |k_i| < N/4 no sum of two modes wraps, so the
  de-aliased and the circular operators coincide; on full-band inputs they
  differ;
* mass is exact;
* the reason the option exists: at the cold upstream Maxwellian of the
  Mach-3.8 shock (u_1 = 3.8 sqrt 2, T = 1) on the paper's 32^2 grid with
  L_v = 20.97, the circular operator's linearisation has an eigenvalue with
  real part about +0.11 (a growing mode; the steady solve diverges), the
  de-aliased one about +0.002.
"""
import math

import numpy as np
import pytest

import synth
from oracle import carleman as ca
from oracle import collision as oc


def _cs(d, N, L=8.0, M=0):
    return ca.setup(d, N, L, 1 / (2 * math.pi) if d == 2 else 1.0, M)


def _band_limited(cs, K, seed):
    rng = np.random.default_rng(seed)
    kv = oc.mode_vectors(cs)
    keep = np.all(np.abs(kv) <= K, axis=0)
    c = (rng.standard_normal(keep.shape) + 1j * rng.standard_normal(keep.shape)) * keep
    return oc.synthesis(c, cs).real


@pytest.mark.parametrize("d,N,M", [(2, 16, 8), (2, 16, 6), (3, 8, 38)])
def test_exact_sum_equals_padded_fast_form(d, N, M):
    cs = _cs(d, N, M=M)
    spec = synth.VGridSpec(d=d, n=N, L=8.0, gamma=d - 2, C=cs.C, m_rho=4,
                           m_sigma=M if d == 2 else 38)
    V = synth.smooth_basis(2, spec, seed=13, orthonormal=False)
    a, ap, am, im = ca.q_direct_exact(V[0], V[1], cs, parts=True)
    b, bp, bm = ca.q_fft_dealiased(V[0], V[1], cs, parts=True)
    s = np.abs(ap).max()
    assert im < 1e-13 * s
    assert np.abs(a - b).max() < 1e-13 * s
    assert np.abs(ap - bp).max() < 1e-13 * s
    assert np.abs(am - bm).max() < 1e-13 * s
    assert abs(oc.moments(a, cs)[0]) < 1e-13 * abs(oc.moments(ap, cs)[0])


@pytest.mark.parametrize("d,N", [(2, 16), (3, 8)])
def test_band_limited_inputs_do_not_wrap(d, N):
    cs = _cs(d, N)
    K = N // 4 - 1
    g, f = _band_limited(cs, K, 3), _band_limited(cs, K, 4)
    qa, qap, _ = ca.q_fft_dealiased(g, f, cs, parts=True)
    qc, qcp, _ = ca.q_fft(g, f, cs, parts=True)
    s = np.abs(qcp).max()
    assert np.abs(qa - qc).max() < 1e-13 * s
    h1, h2 = _band_limited(cs, N // 2 - 1, 5), _band_limited(cs, N // 2 - 1, 6)
    qa, _, _ = ca.q_fft_dealiased(h1, h2, cs, parts=True)
    qc, qcp, _ = ca.q_fft(h1, h2, cs, parts=True)
    assert np.abs(qa - qc).max() > 1e-3 * np.abs(qcp).max()


def _jacobian(f, cs, q):
    """d Q_s(f, f) / d f with the moment projection: column j is
    Q(f, e_j) + Q(e_j, f) (the operator is bilinear)."""
    n = f.size
    J = np.empty((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        J[:, j] = oc.conserve_project((q(f, e, cs) + q(e, f, cs)).reshape(-1), cs)
    return J


def test_dealiasing_removes_the_growing_mode_of_the_cold_upstream_state():
    L, N, mach = 20.97, 32, 3.8
    cs = ca.setup(2, N, L, 1 / (2 * math.pi), 8)
    v = oc.grid(cs)
    u = math.sqrt(2.0) * mach
    f = (np.exp(-((v[0] - u) ** 2 + v[1] ** 2) / 2.0) / (2 * math.pi)).reshape(-1)
    lam_c = np.linalg.eigvals(_jacobian(f, cs, ca.q_fft)).real.max()
    lam_d = np.linalg.eigvals(_jacobian(f, cs, ca.q_fft_dealiased)).real.max()
    print(f"largest real part: circular {lam_c:.4f}, de-aliased {lam_d:.4f}")
    assert lam_c > 0.05
    assert lam_d < 0.01
