"""Carleman-form fast spectral collision operator (oracle).

TEST INFRASTRUCTURE ONLY -- see oracle/__init__.py.

Source: for 2D Maxwell molecules and 3D hard spheres the paper evaluates Q
with the fast spectral algorithm of the cited Mouhot-Pareschi work, cost
O(M N^d log N) with M points on the sphere (Sec. 2.1, the paragraph on the
collision solver; Sec. 5 uses it for every 2D run).  The construction,
written out from the Carleman representation of eq. (collision_operator):

  with v' = v + x, v*' = v + y, v* = v + x + y (x orthogonal to y), the
  operator reads
      Q(g, f)(v) = 2^{d-1} int int Bt(x, y) delta(x.y) [g(v+y) f(v+x) - g(v+x+y) f(v)] dx dy,
      Bt(x, y) = B(|x+y|) |x+y|^{2-d};
  for B = C |q|^gamma this is the constant b0 = 2^{d-1} C exactly when
  gamma = d - 2 (2D Maxwell molecules, 3D hard spheres), the two cases the
  paper names.

  Truncation and periodisation: x, y restricted to the ball |.| <= R,
  R = 4L/(3+sqrt 2), on the box [-L, L]^d with the grid, coefficients,
  Nyquist rule and circular wrap of oracle/collision.py.  Galerkin weights
      Q^_k = sum_{l in K_N} [beta(l, m) - beta(l, l)] g^_l f^_m,  m = wrap(k - l),
      beta(l, m) = b0 int int_{|x|,|y|<=R} delta(x.y) exp(i (pi/L)(l.y + m.x)) dx dy.

  Directions: x = rho e with e on a half sphere and rho in [-R, R]; y runs
  over the disc of radius R orthogonal to e.  Then
      beta(l, m) = b0 int_{half sphere} phi(m.e) psi(l, e) de,
      phi(s)    = int_{-R}^{R} |rho|^{d-2} exp(i pi rho s / L) d rho,
      psi(l, e) = int_{y.e=0, |y|<=R} exp(i (pi/L) l.y) dy,
  closed forms
      2D: phi(s) = 2 sin(a R)/a,  a = pi s / L   (2R at a = 0);
          psi(l, e) = phi(l.e_perp)  (the disc is a segment);
      3D: phi(s) = 2 [R sin(aR)/a - 2 sin^2(aR/2)/a^2]   (R^2 at a = 0);
          psi(l, e) = 2 pi R J1(b R) / b,  b = pi |l - (l.e) e| / L   (pi R^2 at 0).
  The direction integral is the quadrature that makes beta separable:
      2D: e_p = (cos t_p, sin t_p), t_p = p pi / M, weights pi / M (M even);
      3D: one point of each antipodal pair of the 38-point Lebedev rule, with
          its full-sphere weight (the integrand is even in e).
  So  Q+(g, f) = b0 sum_p w_p [IDFT(psi_p g^)] [IDFT(phi_p f^)]  (pointwise on
  the grid), and the loss is f times IDFT(beta(l, l) g^_l).

``q_direct`` is the weighted sum above, term by term (O(N^{2d})); ``q_fft``
follows the fast algorithm (filtered inverse transforms, products, direction
sum) with library FFTs; the tests pin them to each other and to closed forms.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import scipy.special

from . import collision as oc
from . import quadrature as quad


@dataclass
class CarlemanSetup:
    d: int
    N: int
    L: float
    R: float
    C: float
    dirs: np.ndarray     # (M, d) unit directions on a half sphere / half circle
    wdir: np.ndarray     # (M,)

    @property
    def dv(self):
        return 2.0 * self.L / self.N

    @property
    def n(self):
        return self.N ** self.d

    @property
    def b0(self):
        return 2.0 ** (self.d - 1) * self.C


def setup(d: int, N: int, L: float, C: float, M: int = 0, R: float | None = None):
    """2D: M even directions on [0, pi) (default 8); 3D: the 19 antipodal
    representatives of the Lebedev-38 rule (M must be 0 or 38)."""
    if R is None:
        R = 4.0 * L / (3.0 + math.sqrt(2.0))
    if d == 2:
        M = M or 8
        if M % 2:
            raise ValueError("2D: an even number of directions")
        t = math.pi * np.arange(M) / M
        dirs = np.stack([np.cos(t), np.sin(t)], axis=1)
        w = np.full(M, math.pi / M)
    elif d == 3:
        if M not in (0, 38):
            raise ValueError("3D: the Lebedev-38 rule only")
        sig, ws = quad.lebedev38()
        bbar = quad.antipode_index(sig)
        keep = [b for b in range(sig.shape[0]) if b < bbar[b]]
        dirs, w = sig[keep], ws[keep]
    else:
        raise ValueError("d must be 2 or 3")
    return CarlemanSetup(d, N, L, R, C, dirs, w)


def setup_from_spec(spec):
    """From a grid spec with B = C |q|^gamma; gamma must be d - 2."""
    if abs(spec.gamma - (spec.d - 2)) > 0:
        raise ValueError("the Carleman form needs gamma = d - 2 (2D Maxwell, 3D hard spheres)")
    return setup(spec.d, spec.n, spec.L, spec.C, spec.m_sigma)


# ----------------------------------------------------------------------------
# filters
# ----------------------------------------------------------------------------
def phi(cs: CarlemanSetup, s):
    """int_{-R}^{R} |rho|^{d-2} exp(i pi rho s / L) d rho (real, even in s)."""
    a = math.pi * np.asarray(s, dtype=np.float64) / cs.L
    R = cs.R
    small = np.abs(a) < 1e-12
    a_safe = np.where(small, 1.0, a)
    if cs.d == 2:
        v = 2.0 * np.sin(a_safe * R) / a_safe
        return np.where(small, 2.0 * R, v)
    # cos(aR) - 1 written as -2 sin^2(aR/2): the same value without cancellation
    v = 2.0 * (R * np.sin(a_safe * R) / a_safe - 2.0 * np.sin(0.5 * a_safe * R) ** 2 / a_safe ** 2)
    return np.where(small, R * R, v)


def psi(cs: CarlemanSetup, k: np.ndarray, p: int):
    """int over the disc {y.e_p = 0, |y| <= R} of exp(i (pi/L) k.y) dy for mode
    vectors k of shape (d, ...)."""
    e = cs.dirs[p]
    if cs.d == 2:
        eperp = np.array([-e[1], e[0]])
        return phi(cs, sum(eperp[i] * k[i] for i in range(2)))
    ke = sum(e[i] * k[i] for i in range(3))
    kperp = np.sqrt(np.maximum(sum(k[i].astype(np.float64) ** 2 for i in range(3)) - ke * ke, 0.0))
    b = math.pi * kperp / cs.L
    R = cs.R
    small = b < 1e-12
    b_safe = np.where(small, 1.0, b)
    v = 2.0 * math.pi * R * scipy.special.j1(b_safe * R) / b_safe
    return np.where(small, math.pi * R * R, v)


def filters(cs: CarlemanSetup):
    """(Phi, Psi): (M, N..N) tables of phi(k.e_p) and psi(k, e_p) in DFT order."""
    k = oc.mode_vectors(cs).astype(np.float64)
    Phi = np.array([phi(cs, sum(cs.dirs[p, i] * k[i] for i in range(cs.d)))
                    for p in range(len(cs.wdir))])
    Psi = np.array([psi(cs, k, p) for p in range(len(cs.wdir))])
    return Phi, Psi


def loss_weight(cs: CarlemanSetup) -> np.ndarray:
    """beta(l, l) in DFT order."""
    Phi, Psi = filters(cs)
    return cs.b0 * np.tensordot(cs.wdir, Psi * Phi, axes=1)


# ----------------------------------------------------------------------------
# the definition: weighted direct sum
# ----------------------------------------------------------------------------
def qhat_direct(gh: np.ndarray, fh: np.ndarray, cs: CarlemanSetup, parts: bool = False):
    """Q^_k = sum_l [beta(l, m) - beta(l, l)] g^_l f^_m over all k (DFT order)."""
    Phi, Psi = filters(cs)
    M = len(cs.wdir)
    Phi = Phi.reshape(M, -1)
    Psi = Psi.reshape(M, -1)
    beta = cs.b0 * (Psi.T * cs.wdir) @ Phi            # beta[l, m]
    K = oc.mode_vectors(cs).reshape(cs.d, -1).T       # (n, d)
    N = cs.N
    idx = np.zeros(K.shape[0], dtype=np.int64)        # DFT index of a centred mode
    g = gh.reshape(-1)
    f = fh.reshape(-1)
    gain = np.zeros(K.shape[0], dtype=np.complex128)
    loss = np.zeros_like(gain)
    dl = np.diag(beta)
    for kk in range(K.shape[0]):
        mvec = np.mod(K[kk][None, :] - K, N)          # wrap(k - l) as DFT indices
        idx = np.ravel_multi_index(tuple(mvec.T), (N,) * cs.d)
        gain[kk] = np.sum(beta[np.arange(K.shape[0]), idx] * g * f[idx])
        loss[kk] = np.sum(dl * g * f[idx])
    shape = (N,) * cs.d
    if parts:
        return (gain - loss).reshape(shape), gain.reshape(shape), loss.reshape(shape)
    return (gain - loss).reshape(shape)


def q_direct(g: np.ndarray, f: np.ndarray, cs: CarlemanSetup, parts: bool = False):
    gh, fh = oc.coefficients(g, cs), oc.coefficients(f, cs)
    q, qp, qm = qhat_direct(gh, fh, cs, parts=True)
    out = [oc.synthesis(x, cs).real for x in (q, qp, qm)]
    return tuple(out) if parts else out[0]


# ----------------------------------------------------------------------------
# the fast algorithm
# ----------------------------------------------------------------------------
def q_fft(g: np.ndarray, f: np.ndarray, cs: CarlemanSetup, parts: bool = False):
    """Filtered inverse transforms, pointwise products, direction sum."""
    gh, fh = oc.coefficients(g, cs), oc.coefficients(f, cs)
    Phi, Psi = filters(cs)
    gain = np.zeros((cs.N,) * cs.d)
    for p in range(len(cs.wdir)):
        a = oc.synthesis(Psi[p] * gh, cs).real
        b = oc.synthesis(Phi[p] * fh, cs).real
        gain += cs.wdir[p] * a * b
    gain *= cs.b0
    fp = oc.synthesis(fh, cs).real          # f with its Nyquist modes dropped
    loss = fp * oc.synthesis(loss_weight(cs) * gh, cs).real
    if parts:
        return gain - loss, gain, loss
    return gain - loss


def q_pairs(V: np.ndarray, pairs, cs: CarlemanSetup, conserve: bool = True, method=None):
    """Q_s(V_i, V_j) = (Q(V_i, V_j) + Q(V_j, V_i)) / 2 per pair, optionally
    followed by the moment projection of oracle/collision.py; also returns
    the gains."""
    method = method or q_fft
    out, gains = [], []
    for (i, j) in pairs:
        a, ap, _ = method(V[i], V[j], cs, parts=True)
        b, bp, _ = method(V[j], V[i], cs, parts=True)
        q = 0.5 * (a + b).reshape(-1)
        if conserve:
            q = oc.conserve_project(q, cs)
        out.append(q)
        gains.append(0.5 * (ap + bp).reshape(-1))
    return np.array(out), np.array(gains)


# ----------------------------------------------------------------------------
# the de-aliased convolution (the Galerkin sum over l + m = k exactly)
# ----------------------------------------------------------------------------
def qhat_direct_exact(gh: np.ndarray, fh: np.ndarray, cs: CarlemanSetup, parts: bool = False):
    """Q^_k = sum_l [beta(l, k - l) - beta(l, l)] g^_l f^_{k - l} with l + m = k
    exactly: a term whose m = k - l leaves the N-point mode set is absent (the
    circular form wraps it instead).  Output modes with a component -N/2 are
    set to 0, the rule the inputs follow."""
    Phi, Psi = filters(cs)
    M = len(cs.wdir)
    beta = cs.b0 * (Psi.reshape(M, -1).T * cs.wdir) @ Phi.reshape(M, -1)    # beta[l, m]
    K = oc.mode_vectors(cs).reshape(cs.d, -1).T                            # centred, DFT order
    N, n = cs.N, K.shape[0]
    g, f = gh.reshape(-1), fh.reshape(-1)
    dl = np.diag(beta)
    gain = np.zeros(n, dtype=np.complex128)
    loss = np.zeros_like(gain)
    for kk in range(n):
        if np.any(K[kk] == -N // 2):
            continue
        mc = K[kk][None, :] - K                                            # k - l, not wrapped
        inside = np.all((mc >= -N // 2) & (mc < N // 2), axis=1)
        ls = np.nonzero(inside)[0]
        midx = np.ravel_multi_index(tuple(np.mod(mc[inside], N).T), (N,) * cs.d)
        gain[kk] = np.sum(beta[ls, midx] * g[ls] * f[midx])
        loss[kk] = np.sum(dl[ls] * g[ls] * f[midx])
    shape = (N,) * cs.d
    if parts:
        return (gain - loss).reshape(shape), gain.reshape(shape), loss.reshape(shape)
    return (gain - loss).reshape(shape)


def q_direct_exact(g: np.ndarray, f: np.ndarray, cs: CarlemanSetup, parts: bool = False):
    gh, fh = oc.coefficients(g, cs), oc.coefficients(f, cs)
    q, qp, qm = qhat_direct_exact(gh, fh, cs, parts=True)
    out = [oc.synthesis(x, cs) for x in (q, qp, qm)]
    if parts:
        return out[0].real, out[1].real, out[2].real, float(np.abs(out[0].imag).max())
    return out[0].real


def padded_setup(cs: CarlemanSetup) -> CarlemanSetup:
    """The same box, truncation radius and directions with 2N points per axis."""
    return CarlemanSetup(cs.d, 2 * cs.N, cs.L, cs.R, cs.C, cs.dirs, cs.wdir)


def q_fft_dealiased(g: np.ndarray, f: np.ndarray, cs: CarlemanSetup, parts: bool = False):
    """The de-aliased operator through the fast form on the padded grid: the
    interpolants of g and f at the 2N-point nodes of the same box, q_fft there
    (its products hold every mode l + m of two N-point input modes without a
    wrap), then the output coefficients of the N-point mode set without
    Nyquist components, synthesised on the N-point grid."""
    ws = padded_setup(cs)
    N, d = cs.N, cs.d
    k = oc.centred(N)
    idx = np.ix_(*([k % (2 * N)] * d))

    def pad(h):
        cf = np.zeros((2 * N,) * d, dtype=np.complex128)
        cf[idx] = oc.coefficients(h, cs)              # Nyquist modes dropped
        return oc.synthesis(cf, ws).real

    def restrict(hf):
        c = oc.coefficients(hf, ws, zero_nyquist=False)[idx]
        return oc.synthesis(c * oc.nyquist_mask(cs), cs).real

    q, qp, qm = q_fft(pad(g), pad(f), ws, parts=True)
    if parts:
        return restrict(q), restrict(qp), restrict(qm)
    return restrict(q)


def q_pairs_dealiased(V: np.ndarray, pairs, cs: CarlemanSetup, conserve: bool = True):
    """q_pairs with the de-aliased operator."""
    out, gains = [], []
    for (i, j) in pairs:
        a, ap, _ = q_fft_dealiased(V[i], V[j], cs, parts=True)
        b, bp, _ = q_fft_dealiased(V[j], V[i], cs, parts=True)
        q = 0.5 * (a + b).reshape(-1)
        if conserve:
            q = oc.conserve_project(q, cs)
        out.append(q)
        gains.append(0.5 * (ap + bp).reshape(-1))
    return np.array(out), np.array(gains)
