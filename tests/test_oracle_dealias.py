"""Pins of the oracle's de-aliased operator (the Galerkin sum over l + m = k
exactly, reading of the spectral method's convolution; the default is the
circular sum an N-point transform computes).

* the exact direct sum equals the FFT form on the padded 2N-point grid (the
  definition against a route through a different grid);
* on inputs band-limited to |k_i| < N/4 no sum of two modes wraps, so the
  de-aliased and the circular operators coincide;
* on inputs with modes up to N/2 - 1 they differ (the wrap is real);
* mass is exact.
"""
import math

import numpy as np
import pytest

import synth
from oracle import collision as oc


def _vs(d):
    if d == 2:
        return oc.setup(2, 16, 8.0, 1 / (2 * math.pi), 0.0, 6, 8)
    return oc.setup(3, 8, 8.0, 1.0, 1.0, 3, 38)


def _band_limited(vs, K, seed):
    rng = np.random.default_rng(seed)
    kv = oc.mode_vectors(vs)
    keep = np.all(np.abs(kv) <= K, axis=0)
    c = (rng.standard_normal(keep.shape) + 1j * rng.standard_normal(keep.shape)) * keep
    return oc.synthesis(c, vs).real


@pytest.mark.parametrize("d", [2, 3])
def test_exact_sum_equals_padded_fft_form(d):
    vs = _vs(d)
    spec = synth.small_2d if d == 2 else synth.small_3d
    V = synth.smooth_basis(2, spec, seed=12, orthonormal=False)
    q1, q1p, im = oc.q_direct_exact(V[0], V[1], vs, parts=True)
    q2, q2p = oc.q_fft_dealiased(V[0], V[1], vs, parts=True)
    s = np.abs(q1p).max()
    assert im < 1e-13 * s
    assert np.abs(q1 - q2.reshape(q1.shape)).max() < 1e-13 * s
    assert np.abs(q1p - q2p.reshape(q1.shape)).max() < 1e-13 * s
    assert abs(oc.moments(q1, vs)[0]) < 1e-13 * abs(oc.moments(q1p, vs)[0])


@pytest.mark.parametrize("d", [2, 3])
def test_band_limited_inputs_do_not_wrap(d):
    vs = _vs(d)
    K = vs.N // 4 - 1
    g, f = _band_limited(vs, K, 3), _band_limited(vs, K, 4)
    qa, qap = oc.q_fft_dealiased(g, f, vs, parts=True)
    qc, qcp = oc.q_fft(g, f, vs, parts=True)
    s = np.abs(qcp).max()
    assert np.abs(qa.reshape(qc.shape) - qc).max() < 1e-13 * s
    # full-band inputs: the circular sum wraps, the exact one does not
    h1, h2 = _band_limited(vs, vs.N // 2 - 1, 5), _band_limited(vs, vs.N // 2 - 1, 6)
    qa, _ = oc.q_fft_dealiased(h1, h2, vs, parts=True)
    qc, qcp = oc.q_fft(h1, h2, vs, parts=True)
    assert np.abs(qa.reshape(qc.shape) - qc).max() > 1e-3 * np.abs(qcp).max()
