"""Collision operator with an anisotropic kernel B(|q|, cos chi) (oracle).

TEST INFRASTRUCTURE ONLY -- see oracle/__init__.py.

The paper's collision operator (eq. collision_operator) admits a kernel that
depends on the angle chi between the pre- and post-collision relative
velocities, cos chi = sigma . q^ (Sec. 2.1; the cited fast spectral methods
treat a general B, the isotropic case lets the angular integral be done in
closed form).  Here

    B(rho, c) = C rho^gamma sum_{n=0}^{nb-1} beta_n P_n(c)     (3D, Legendre)
    B(rho, c) = C rho^gamma sum_{n=0}^{nb-1} beta_n T_n(c)     (2D, Chebyshev),

beta = (1,) being the isotropic kernel of ``collision.py``.  Everything else
(grid, coefficients, Nyquist rule, circular wrap, radial Gauss-Legendre and
sigma rules, the loss through the same sigma rule) is as in ``collision.py``.

Substituting the Fourier series of g and f into the gain with
v*' = v - rho (q^ + sigma)/2 and v' = v - rho (q^ - sigma)/2 gives

    G+(l, m) = sum_a w_a rho_a^{d-1} sum_b w_b exp(-i theta_a (l - m).sigma_b)
               F_ab(wrap(l + m)),    theta_a = pi rho_a / (2L),
    F_ab(k)  = int_{S^{d-1}} B(rho_a, sigma_b . q^) exp(-i theta_a k . q^) dq^
             = C rho_a^gamma sum_n beta_n |S^{d-1}| (-i)^n Z_n(theta_a |k|) Y_n(sigma_b . k^)

(Funk-Hecke: 3D Z_n = j_n spherical Bessel, Y_n = P_n; 2D Z_n = J_n, Y_n =
T_n).  The sigma sum no longer factors out of F, so the fast form transforms
every product S_g(a, b) S_f(a, bbar) on its own.  The loss: int B dsigma =
|S^{d-1}| C rho^gamma beta_0 for every q^, so G-(l) is beta_0 times the
isotropic loss weight (G+(l, -l) = G-(l): mass stays exact).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.special

from . import collision as oc


def angular(d: int, beta, c):
    """sum_n beta_n P_n(c) (3D) or T_n(c) (2D)."""
    c = np.asarray(c, dtype=np.float64)
    out = np.zeros_like(c)
    for n, bn in enumerate(beta):
        if bn == 0.0:
            continue
        out = out + bn * (scipy.special.eval_legendre(n, c) if d == 3 else
                          scipy.special.eval_chebyt(n, c))
    return out


def B(vs: oc.VelocitySetup, beta, rho, c):
    return vs.C * np.power(rho, vs.gamma) * angular(vs.d, beta, c)


def F_table(vs: oc.VelocitySetup, beta) -> np.ndarray:
    """F_ab(k) for every radial node a, sigma node b and mode k (DFT order),
    shape (m_rho, m_sigma, n), complex, from the Funk-Hecke formula."""
    k = oc.mode_vectors(vs).reshape(vs.d, -1).T.astype(np.float64)     # (n, d)
    kk = np.sqrt((k ** 2).sum(axis=1))
    khat = np.where(kk[:, None] > 0, k / np.where(kk > 0, kk, 1.0)[:, None], 0.0)
    out = np.zeros((len(vs.rho), vs.sig.shape[0], k.shape[0]), dtype=np.complex128)
    for a, rho in enumerate(vs.rho):
        z = math.pi * rho / (2.0 * vs.L) * kk
        pref = vs.C * rho ** vs.gamma * vs.sphere_area
        for n, bn in enumerate(beta):
            if bn == 0.0:
                continue
            Zn = scipy.special.spherical_jn(n, z) if vs.d == 3 else scipy.special.jv(n, z)
            for b in range(vs.sig.shape[0]):
                c = khat @ vs.sig[b]
                Yn = scipy.special.eval_legendre(n, c) if vs.d == 3 else scipy.special.eval_chebyt(n, c)
                out[a, b] += pref * bn * (-1j) ** n * Zn * Yn
    return out


def loss_weight(vs: oc.VelocitySetup, beta) -> np.ndarray:
    return beta[0] * oc.loss_weight(vs)


def qhat_direct(gh, fh, vs: oc.VelocitySetup, beta, ks=None, parts: bool = False):
    """Q^_k = sum_l [G+(l, wrap(k - l)) - G-(l)] g^_l f^_{wrap(k - l)}, G+ as
    in the module docstring (sum over a and b for each pair (l, m))."""
    N, d = vs.N, vs.d
    kv = oc.mode_vectors(vs).reshape(d, -1).T                 # (n, d) centred ints
    n = kv.shape[0]
    if ks is None:
        ks = np.arange(n)
    g = gh.reshape(-1)
    f = fh.reshape(-1)
    Ft = F_table(vs, beta)                                    # (m_rho, m_sigma, n)
    Gm = loss_weight(vs, beta).reshape(-1)
    cw = vs.wrho * vs.rho ** (d - 1)
    strides = np.array([N ** (d - 1 - i) for i in range(d)])
    out = np.zeros(len(ks), dtype=np.complex128)
    outp = np.zeros(len(ks), dtype=np.complex128)
    for t, kidx in enumerate(ks):
        mc = kv[kidx][None, :] - kv
        mc = (mc + N // 2) % N - N // 2                       # m = wrap(k - l)
        midx = ((mc % N) * strides).sum(axis=1)
        delta = (kv - mc).astype(np.float64)                  # l - m
        prod = g * f[midx]
        gplus = np.zeros(n, dtype=np.complex128)
        for a, rho in enumerate(vs.rho):
            th = math.pi * rho / (2.0 * vs.L)
            for b in range(vs.sig.shape[0]):
                gplus += cw[a] * vs.wsig[b] * np.exp(-1j * th * (delta @ vs.sig[b])) * Ft[a, b, kidx]
        outp[t] = (gplus * prod).sum()
        out[t] = outp[t] - (Gm * prod).sum()
    if parts:
        return out, outp
    return out


def q_direct(g, f, vs: oc.VelocitySetup, beta, parts: bool = False):
    gh, fh = oc.coefficients(g, vs), oc.coefficients(f, vs)
    qh, qhp = qhat_direct(gh, fh, vs, beta, parts=True)
    shape = (vs.N,) * vs.d
    q = oc.synthesis(qh.reshape(shape), vs)
    qp = oc.synthesis(qhp.reshape(shape), vs)
    if parts:
        return q.real, qp.real, float(np.abs(q.imag).max())
    return q.real


def q_fft(g, f, vs: oc.VelocitySetup, beta, parts: bool = False):
    """The fast algorithm's steps with the sigma sum moved into Fourier space:
    for every radial node a and sigma node b the shifted interpolants
    g~(v - rho_a sigma_b / 2), f~(v + rho_a sigma_b / 2), their product, its
    coefficients times F_ab(k) and the weights, summed; loss as in the
    isotropic form with the factor beta_0."""
    gh = oc.coefficients(g, vs)
    fh = oc.coefficients(f, vs)
    k = oc.mode_vectors(vs).astype(np.float64)
    Ft = F_table(vs, beta).reshape((len(vs.rho), vs.sig.shape[0]) + (vs.N,) * vs.d)
    qplus_h = np.zeros_like(gh)
    for a, rho in enumerate(vs.rho):
        th = math.pi * rho / (2.0 * vs.L)
        cw = vs.wrho[a] * rho ** (vs.d - 1)
        for b in range(vs.sig.shape[0]):
            ph = np.exp(-1j * th * sum(vs.sig[b, i] * k[i] for i in range(vs.d)))
            sg = oc.synthesis(gh * ph, vs).real
            sf = oc.synthesis(fh * np.conj(ph), vs).real
            P = oc.coefficients(sg * sf, vs, zero_nyquist=False)
            qplus_h += cw * vs.wsig[b] * Ft[a, b] * P
    qplus = oc.synthesis(qplus_h, vs).real
    lam = oc.synthesis(loss_weight(vs, beta) * gh, vs).real
    q = qplus - oc.synthesis(fh, vs).real * lam
    if parts:
        return q, qplus
    return q


def q_pairs(V, pairs, vs: oc.VelocitySetup, beta, conserve: bool = True):
    """Q_s(V_i, V_j) = (Q(V_i, V_j) + Q(V_j, V_i)) / 2 for each pair, optionally
    projected; returns (npairs, n) and the gains."""
    out, gains = [], []
    for (i, j) in pairs:
        a, ap = q_fft(V[i], V[j], vs, beta, parts=True)
        b, bp = q_fft(V[j], V[i], vs, beta, parts=True)
        q = 0.5 * (a + b).reshape(-1)
        if conserve:
            q = oc.conserve_project(q, vs)
        out.append(q)
        gains.append(0.5 * (ap + bp).reshape(-1))
    return np.array(out), np.array(gains)
