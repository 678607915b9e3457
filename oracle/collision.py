"""Discrete collision operator Q(g, f) on the uniform velocity grid (oracle).

TEST INFRASTRUCTURE ONLY -- see oracle/__init__.py.

Source: the bilinear operator of eq. (collision_operator) with the post-
collision velocities of eq. (collision velocity); the paper evaluates it with
a fast Fourier spectral method acting as a discrete velocity method on a
uniform grid of [-L, L]^d (Sec. 2.1) and leaves its formulas to the cited
works.  What follows is the Fourier-Galerkin construction written out, with
the readings used throughout this repository:

  grid      v_q = -L + q*dv, dv = 2L/N, q in {0..N-1}^d (C order);
  modes     K_N = {-N/2 .. N/2-1}^d; coefficients
            h^_k = N^-d sum_q h(v_q) exp(-i (pi/L) k.v_q), and every mode with
            a component equal to -N/2 (Nyquist) is set to zero;
  wrap      convolutions are circular: m = wrap(k - l) (componentwise mod N
            into K_N), i.e. what an N-point FFT pipeline computes;
  kernel    isotropic B(|v-v*|) = C |v-v*|^gamma, truncated to |v-v*| <= R,
            R = 4L/(3+sqrt 2);
  weights   with q = v - v*, rho = |q|, theta_a = pi rho_a /(2L):
      G+(l,m) = sum_a w_a rho_a^{d-1} F(wrap(l+m), rho_a) E_a(l-m),
      F(k, rho) = B(rho) A_d(pi rho |k| / (2L)),
        A_2(z) = 2 pi J0(z), A_3(z) = 4 pi sin z / z   (exact inner q^-integral),
      E_a(delta) = sum_b w_b exp(-i theta_a sigma_b . delta)   (sigma rule),
      G-(l) = |S^{d-1}| sum_a w_a rho_a^{d-1} B(rho_a) sum_b w_b exp(-2 i theta_a sigma_b . l)
            (the loss uses the same sigma rule, so G+(l,-l) = G-(l) and mass
             is conserved exactly);
  operator  Q^_k = sum_{l in K_N} [G+(l, m) - G-(l)] g^_l f^_m, m = wrap(k-l),
            Q(v_q) = Re sum_k Q^_k exp(i (pi/L) k.v_q);
  pairs     Q_s(g, f) = (Q(g, f) + Q(f, g)) / 2.

``q_direct`` is that definition (the O(N^{2d}) sum); ``q_fft`` takes the
steps of the fast algorithm (shift by the trigonometric interpolant, product,
sigma sum, transform, radial weights) with library FFTs, and is pinned to
``q_direct`` in the tests.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass

import numpy as np
import scipy.special

from . import quadrature as quad


# ----------------------------------------------------------------------------
# setup
# ----------------------------------------------------------------------------
@dataclass
class VelocitySetup:
    d: int
    N: int
    L: float
    R: float
    C: float
    gamma: float
    rho: np.ndarray      # (m_rho,)
    wrho: np.ndarray     # (m_rho,)
    sig: np.ndarray      # (m_sigma, d)
    wsig: np.ndarray     # (m_sigma,)

    @property
    def dv(self):
        return 2.0 * self.L / self.N

    @property
    def n(self):
        return self.N ** self.d

    def B(self, rho):
        return self.C * np.power(rho, self.gamma)

    @property
    def sphere_area(self):
        return 2.0 * math.pi if self.d == 2 else 4.0 * math.pi


def setup(d: int, N: int, L: float, C: float, gamma: float, m_rho: int = 16,
          m_sigma: int = 0, R: float | None = None) -> VelocitySetup:
    if R is None:
        R = 4.0 * L / (3.0 + math.sqrt(2.0))
    rho, wrho = quad.gauss_legendre(m_rho, R)
    sig, wsig = quad.sphere_rule(d, m_sigma)
    return VelocitySetup(d, N, L, R, C, gamma, rho, wrho, sig, wsig)


def setup_from_spec(spec) -> VelocitySetup:
    return setup(spec.d, spec.n, spec.L, spec.C, spec.gamma, spec.m_rho, spec.m_sigma)


def grid(vs: VelocitySetup) -> np.ndarray:
    ax = -vs.L + vs.dv * np.arange(vs.N)
    return np.stack(np.meshgrid(*([ax] * vs.d), indexing="ij"), axis=0)


def centred(N: int) -> np.ndarray:
    """Integer mode of each DFT index: 0..N/2-1, then -N/2..-1."""
    k = np.arange(N)
    return np.where(k >= N // 2, k - N, k)


def mode_vectors(vs: VelocitySetup) -> np.ndarray:
    """Centred integer mode vectors in DFT index order, shape (d, N, ..., N)."""
    c = centred(vs.N)
    return np.stack(np.meshgrid(*([c] * vs.d), indexing="ij"), axis=0)


def nyquist_mask(vs: VelocitySetup) -> np.ndarray:
    k = mode_vectors(vs)
    return np.all(k != -vs.N // 2, axis=0)


# ----------------------------------------------------------------------------
# Fourier coefficients and synthesis (convention of the module docstring)
# ----------------------------------------------------------------------------
def coefficients(h: np.ndarray, vs: VelocitySetup, zero_nyquist: bool = True):
    """h^_k = N^-d sum_q h(v_q) exp(-i (pi/L) k.v_q), in DFT index order.

    With v_q = -L + q dv the exponential equals (-1)^{sum k} exp(-2 pi i k.q/N),
    so the sum is a forward FFT times a sign."""
    h = np.asarray(h, dtype=np.float64).reshape((vs.N,) * vs.d)
    k = mode_vectors(vs)
    sign = np.where(k.sum(axis=0) % 2 == 0, 1.0, -1.0)
    c = np.fft.fftn(h) * sign / vs.n
    if zero_nyquist:
        c = c * nyquist_mask(vs)
    return c


def synthesis(c: np.ndarray, vs: VelocitySetup) -> np.ndarray:
    """sum_k c_k exp(i (pi/L) k.v_q) on the grid (complex)."""
    k = mode_vectors(vs)
    sign = np.where(k.sum(axis=0) % 2 == 0, 1.0, -1.0)
    return np.fft.ifftn(c * sign) * vs.n


# ----------------------------------------------------------------------------
# weights
# ----------------------------------------------------------------------------
def angular_factor(d: int, z):
    """A_d(z) = int_{S^{d-1}} exp(-i z e.q) dq for a unit e: 2 pi J0(z) or 4 pi sin z/z."""
    z = np.asarray(z, dtype=np.float64)
    if d == 2:
        return 2.0 * math.pi * scipy.special.j0(z)
    return 4.0 * math.pi * np.sinc(z / math.pi)


def F_table(vs: VelocitySetup) -> np.ndarray:
    """F(k, rho_a) = B(rho_a) A_d(pi rho_a |k| / (2L)) for k in DFT order; (m_rho, N..N)."""
    k = mode_vectors(vs)
    kk = np.sqrt((k.astype(np.float64) ** 2).sum(axis=0))
    out = []
    for a, rho in enumerate(vs.rho):
        out.append(vs.B(rho) * angular_factor(vs.d, math.pi * rho * kk / (2.0 * vs.L)))
    return np.array(out)


def E_table(vs: VelocitySetup) -> np.ndarray:
    """E_a(delta) = sum_b w_b exp(-i theta_a sigma_b.delta) for delta in
    [-(N-1), N-1]^d; array index delta + N - 1; shape (m_rho, 2N-1, ..., 2N-1)."""
    N, d = vs.N, vs.d
    ax = np.arange(-(N - 1), N)
    D = np.stack(np.meshgrid(*([ax] * d), indexing="ij"), axis=0).astype(np.float64)
    out = np.zeros((len(vs.rho),) + (2 * N - 1,) * d, dtype=np.complex128)
    for a, rho in enumerate(vs.rho):
        th = math.pi * rho / (2.0 * vs.L)
        for b in range(vs.sig.shape[0]):
            sd = sum(vs.sig[b, i] * D[i] for i in range(d))
            out[a] += vs.wsig[b] * np.exp(-1j * th * sd)
    return out


def loss_weight(vs: VelocitySetup) -> np.ndarray:
    """G-(l) in DFT index order (complex array, imaginary part ~ 0)."""
    k = mode_vectors(vs).astype(np.float64)
    out = np.zeros((vs.N,) * vs.d, dtype=np.complex128)
    for a, rho in enumerate(vs.rho):
        th = math.pi * rho / (2.0 * vs.L)
        acc = np.zeros_like(out)
        for b in range(vs.sig.shape[0]):
            sd = sum(vs.sig[b, i] * k[i] for i in range(vs.d))
            acc += vs.wsig[b] * np.exp(-2j * th * sd)
        out += vs.wrho[a] * rho ** (vs.d - 1) * vs.B(rho) * acc
    return vs.sphere_area * out


# ----------------------------------------------------------------------------
# the definition: direct spectral sum
# ----------------------------------------------------------------------------
def _flat_modes(vs):
    k = mode_vectors(vs).reshape(vs.d, -1).T          # (n, d) centred ints, DFT order
    return k


def qhat_direct(gh: np.ndarray, fh: np.ndarray, vs: VelocitySetup, ks=None,
                parts: bool = False):
    """Q^_k = sum_l [G+(l, wrap(k-l)) - G-(l)] g^_l f^_{wrap(k-l)} for the flat
    DFT indices ``ks`` (all modes by default).  Vectorised over l; a Python
    loop over k.  Returns Q^ (and Q^+ with ``parts``)."""
    N, d = vs.N, vs.d
    kv = _flat_modes(vs)
    n = kv.shape[0]
    if ks is None:
        ks = np.arange(n)
    ks = np.asarray(ks)
    g = gh.reshape(-1)
    f = fh.reshape(-1)
    Ft = F_table(vs).reshape(len(vs.rho), -1)                  # (m_rho, n)
    E = E_table(vs).reshape(len(vs.rho), -1)                   # (m_rho, (2N-1)^d)
    Gm = loss_weight(vs).reshape(-1)
    cw = vs.wrho * vs.rho ** (d - 1)                           # radial weight
    strides = np.array([N ** (d - 1 - i) for i in range(d)])
    estr = np.array([(2 * N - 1) ** (d - 1 - i) for i in range(d)])
    out = np.zeros(len(ks), dtype=np.complex128)
    outp = np.zeros(len(ks), dtype=np.complex128)
    for t, kidx in enumerate(ks):
        kc = kv[kidx]
        mc = kc[None, :] - kv                                  # k - l (ints)
        mc = (mc + N // 2) % N - N // 2                        # wrap into K_N
        midx = ((mc % N) * strides).sum(axis=1)
        delta = kv - mc                                        # l - m
        eidx = ((delta + N - 1) * estr).sum(axis=1)
        prod = g * f[midx]
        gplus = (cw[:, None] * Ft[:, kidx][:, None] * E[:, eidx]).sum(axis=0)
        outp[t] = (gplus * prod).sum()
        out[t] = outp[t] - (Gm * prod).sum()
    if parts:
        return out, outp
    return out


_DIRECT_LIB = None


def _direct_lib():
    global _DIRECT_LIB
    if _DIRECT_LIB is None:
        here = os.path.dirname(os.path.abspath(__file__))
        path = os.path.join(here, "_direct_sum.so")
        if not os.path.exists(path):
            from . import build_c
            build_c.build()
        lib = ctypes.CDLL(path)
        lib.oracle_qhat_direct.restype = ctypes.c_int
        _DIRECT_LIB = lib
    return _DIRECT_LIB


def qhat_direct_c(gh: np.ndarray, fh: np.ndarray, vs: VelocitySetup, ks=None,
                  parts: bool = False):
    """The same sum as ``qhat_direct`` in plain C (OpenMP over k) for N^d
    beyond what numpy finishes quickly.  Tables are built here in Python."""
    N, d = vs.N, vs.d
    n = vs.n
    if ks is None:
        ks = np.arange(n)
    ks = np.ascontiguousarray(np.asarray(ks, dtype=np.int64))
    g = np.ascontiguousarray(gh.reshape(-1).astype(np.complex128))
    f = np.ascontiguousarray(fh.reshape(-1).astype(np.complex128))
    cw = vs.wrho * vs.rho ** (d - 1)
    FtW = np.ascontiguousarray(F_table(vs).reshape(len(vs.rho), -1) * cw[:, None])
    E = np.ascontiguousarray(E_table(vs).reshape(len(vs.rho), -1).real)
    Gm = np.ascontiguousarray(loss_weight(vs).reshape(-1).real)
    out = np.zeros(len(ks), dtype=np.complex128)
    outp = np.zeros(len(ks), dtype=np.complex128)
    lib = _direct_lib()
    P = ctypes.c_void_p
    rc = lib.oracle_qhat_direct(
        ctypes.c_int(d), ctypes.c_int(N), ctypes.c_int(len(vs.rho)),
        P(g.ctypes.data), P(f.ctypes.data), P(FtW.ctypes.data), P(E.ctypes.data),
        P(Gm.ctypes.data), P(ks.ctypes.data), ctypes.c_long(len(ks)),
        P(out.ctypes.data), P(outp.ctypes.data))
    if rc != 0:
        raise RuntimeError(f"oracle direct sum failed ({rc})")
    if parts:
        return out, outp
    return out


def q_direct(g: np.ndarray, f: np.ndarray, vs: VelocitySetup, parts: bool = False,
             use_c: bool | None = None):
    """Q(g, f) on the grid from the direct sum (all modes), real part.
    With ``parts`` also returns Q+ (the gain) and max |Im| of the synthesis."""
    gh = coefficients(g, vs)
    fh = coefficients(f, vs)
    if use_c is None:
        use_c = vs.n > 4096
    fn = qhat_direct_c if use_c else qhat_direct
    qh, qhp = fn(gh, fh, vs, parts=True)
    shape = (vs.N,) * vs.d
    q = synthesis(qh.reshape(shape), vs)
    qp = synthesis(qhp.reshape(shape), vs)
    if parts:
        return q.real, qp.real, float(np.abs(q.imag).max())
    return q.real


# ----------------------------------------------------------------------------
# the fast algorithm's steps (same operator), library FFTs, float64
# ----------------------------------------------------------------------------
def q_fft(g: np.ndarray, f: np.ndarray, vs: VelocitySetup, parts: bool = False):
    """Q(g, f) via: g~(v - rho_a sigma_b / 2), f~(v + rho_a sigma_b / 2) as
    phase-shifted syntheses; P_a = sum_b w_b product; Q^+_k = sum_a w_a rho_a^{d-1}
    F(k, rho_a) P^_a(k); loss f~(v) * synthesis(G- g^)."""
    gh = coefficients(g, vs)
    fh = coefficients(f, vs)
    k = mode_vectors(vs).astype(np.float64)
    Ft = F_table(vs)
    qplus_h = np.zeros_like(gh)
    for a, rho in enumerate(vs.rho):
        th = math.pi * rho / (2.0 * vs.L)
        P = np.zeros((vs.N,) * vs.d)
        for b in range(vs.sig.shape[0]):
            ph = np.exp(-1j * th * sum(vs.sig[b, i] * k[i] for i in range(vs.d)))
            sg = synthesis(gh * ph, vs).real
            sf = synthesis(fh * np.conj(ph), vs).real
            P += vs.wsig[b] * sg * sf
        qplus_h += vs.wrho[a] * rho ** (vs.d - 1) * Ft[a] * coefficients(P, vs, zero_nyquist=False)
    qplus = synthesis(qplus_h, vs).real
    lam = synthesis(loss_weight(vs) * gh, vs).real
    fproj = synthesis(fh, vs).real
    q = qplus - fproj * lam
    if parts:
        return q, qplus
    return q


def q_sym(g, f, vs, method=q_fft):
    """Q_s(g, f) = (Q(g, f) + Q(f, g)) / 2."""
    return 0.5 * (method(g, f, vs) + method(f, g, vs))


def q_pairs(V: np.ndarray, pairs, vs: VelocitySetup, conserve: bool = True,
            method=None):
    """Q_s(V_i, V_j) for each (i, j) in ``pairs``; V is (r, n).  Optionally
    followed by the conservation projection.  Returns (npairs, n) and the
    gains Q_s^+ (npairs, n)."""
    if method is None:
        method = q_fft
    out, gains = [], []
    for (i, j) in pairs:
        a, ap = method(V[i], V[j], vs, parts=True)[:2]
        b, bp = method(V[j], V[i], vs, parts=True)[:2]
        q = 0.5 * (a + b).reshape(-1)
        if conserve:
            q = conserve_project(q, vs)
        out.append(q)
        gains.append(0.5 * (ap + bp).reshape(-1))
    return np.array(out), np.array(gains)


# ----------------------------------------------------------------------------
# moments and the conservation projection
# ----------------------------------------------------------------------------
def moment_matrix(vs: VelocitySetup) -> np.ndarray:
    """C with rows dv^d * {1, v_1, .., v_d, |v|^2}(v_q); shape (d+2, n)."""
    v = grid(vs).reshape(vs.d, -1)
    rows = [np.ones(vs.n)] + [v[i] for i in range(vs.d)] + [(v ** 2).sum(axis=0)]
    return vs.dv ** vs.d * np.array(rows)


def moments(h: np.ndarray, vs: VelocitySetup) -> np.ndarray:
    """(mass, momentum_1..d, energy*2) = C h."""
    return moment_matrix(vs) @ np.asarray(h).reshape(-1)


def conserve_project(q: np.ndarray, vs: VelocitySetup) -> np.ndarray:
    """Least-squares correction q - C^T (C C^T)^-1 C q: the smallest change in
    the Euclidean norm that makes all d+2 discrete moments vanish."""
    C = moment_matrix(vs)
    lam = np.linalg.solve(C @ C.T, C @ q.reshape(-1))
    return q.reshape(-1) - C.T @ lam


# ----------------------------------------------------------------------------
# the de-aliased convolution (reading of the Galerkin sum over l + m = k)
# ----------------------------------------------------------------------------
def qhat_direct_exact(gh: np.ndarray, fh: np.ndarray, vs: VelocitySetup, ks=None,
                      parts: bool = False):
    """Q^_k = sum_{l in K_N} [G+(l, k - l) - G-(l)] g^_l f^_{k - l} with l + m = k
    exactly (no wrap: terms whose m = k - l leaves K_N are absent), for modes
    k of K_N; G+(l, m) = sum_a w_a rho_a^{d-1} F(l + m, rho_a) E_a(l - m).
    Modes with a component -N/2 of the output are set to 0 (the rule the
    inputs follow), so the synthesis is real."""
    N, d = vs.N, vs.d
    kv = _flat_modes(vs)
    n = kv.shape[0]
    if ks is None:
        ks = np.arange(n)
    g = gh.reshape(-1)
    f = fh.reshape(-1)
    Ft = F_table(vs).reshape(len(vs.rho), -1)
    E = E_table(vs).reshape(len(vs.rho), -1)
    Gm = loss_weight(vs).reshape(-1)
    cw = vs.wrho * vs.rho ** (d - 1)
    strides = np.array([N ** (d - 1 - i) for i in range(d)])
    estr = np.array([(2 * N - 1) ** (d - 1 - i) for i in range(d)])
    out = np.zeros(len(ks), dtype=np.complex128)
    outp = np.zeros(len(ks), dtype=np.complex128)
    for t, kidx in enumerate(ks):
        kc = kv[kidx]
        if np.any(kc == -N // 2):
            continue
        mc = kc[None, :] - kv                                  # k - l, not wrapped
        inside = np.all((mc >= -N // 2) & (mc < N // 2), axis=1)
        mcl = mc[inside]
        midx = ((mcl % N) * strides).sum(axis=1)
        delta = kv[inside] - mcl
        eidx = ((delta + N - 1) * estr).sum(axis=1)
        prod = g[inside] * f[midx]
        gplus = (cw[:, None] * Ft[:, kidx][:, None] * E[:, eidx]).sum(axis=0)
        outp[t] = (gplus * prod).sum()
        out[t] = outp[t] - (Gm[inside] * prod).sum()
    if parts:
        return out, outp
    return out


def q_direct_exact(g, f, vs: VelocitySetup, parts: bool = False):
    gh, fh = coefficients(g, vs), coefficients(f, vs)
    qh, qhp = qhat_direct_exact(gh, fh, vs, parts=True)
    shape = (vs.N,) * vs.d
    q, qp = synthesis(qh.reshape(shape), vs), synthesis(qhp.reshape(shape), vs)
    if parts:
        return q.real, qp.real, float(np.abs(q.imag).max())
    return q.real


def padded_setup(vs: VelocitySetup) -> VelocitySetup:
    """The same box, truncation radius and quadrature with 2N points per axis."""
    return VelocitySetup(vs.d, 2 * vs.N, vs.L, vs.R, vs.C, vs.gamma, vs.rho, vs.wrho, vs.sig,
                         vs.wsig)


def q_fft_dealiased(g, f, vs: VelocitySetup, parts: bool = False):
    """The de-aliased operator through the FFT form on the padded grid: the
    interpolants of g and f at the 2N-point nodes, q_fft there (no sum of two
    input modes wraps), then the output coefficients of K_N without Nyquist
    components, synthesised on the N-point grid."""
    ws = padded_setup(vs)
    N, d = vs.N, vs.d

    def pad(h):
        c = coefficients(h, vs)                       # Nyquist modes dropped
        cf = np.zeros((2 * N,) * d, dtype=np.complex128)
        k = centred(N)
        idx = np.ix_(*([k % (2 * N)] * d))
        cf[idx] = c
        return synthesis(cf, ws).real

    def restrict(hf):
        cf = coefficients(hf, ws, zero_nyquist=False)
        k = centred(N)
        c = cf[np.ix_(*([k % (2 * N)] * d))]
        return synthesis(c * nyquist_mask(vs), vs).real

    q, qp = q_fft(pad(g), pad(f), ws, parts=True)
    if parts:
        return restrict(q), restrict(qp)
    return restrict(q)


def q_pairs_dealiased(V, pairs, vs: VelocitySetup, conserve: bool = True):
    out, gains = [], []
    for (i, j) in pairs:
        a, ap = q_fft_dealiased(V[i], V[j], vs, parts=True)
        b, bp = q_fft_dealiased(V[j], V[i], vs, parts=True)
        q = 0.5 * (a + b).reshape(-1)
        if conserve:
            q = conserve_project(q, vs)
        out.append(q)
        gains.append(0.5 * (ap + bp).reshape(-1))
    return np.array(out), np.array(gains)
