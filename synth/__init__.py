"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke run.

This module only *builds inputs*: velocity/space grids for evaluating test
functions, Maxwellians, the normal-shock end states from the Rankine-Hugoniot
relations (paper, Sec. 4, eq. ``relation``), shock-like initial data (Sec. 5.2)
and seeded random perturbations.  It contains none of the collision operator,
none of the low-rank integrator and none of the rank adaptivity: those live
separately in ``oracle/`` (CPU checker) and in the HIP library.

Grids are regenerated here on purpose (velocity nodes v_q = -L + q*2L/N,
spatial cell centres x_p = a + (p+1/2) dx); nothing here is imported by the
library or by the oracle's arithmetic.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "vgrid_points", "xgrid_centres", "maxwellian", "rh_downstream", "shock_states",
    "c1_distribution", "c2_bimaxwellian", "c2_bkw", "smooth_basis", "shock_initial",
    "lowrank_state", "lowrank_state_sketch", "serving_trace", "serving_trace_2d", "VGridSpec",
    "C1", "C2", "C3",
    "small_3d", "small_2d",
]


@dataclass(frozen=True)
class VGridSpec:
    """Velocity grid + kernel description of one workload (plain data)."""
    d: int
    n: int
    L: float
    gamma: float = 0.0        # B(rho) = C * rho**gamma
    C: float = 1.0
    m_rho: int = 16
    m_sigma: int = 0          # 0 -> default (8 on the circle, 38 on the sphere)

    @property
    def npts(self) -> int:
        return self.n ** self.d

    def sigma_count(self) -> int:
        if self.m_sigma:
            return self.m_sigma
        return 8 if self.d == 2 else 38


# Workload presets (sizes of the configurations the benchmark and tests use).
C1 = VGridSpec(d=2, n=32, L=8.0, gamma=0.0, C=1.0 / (2.0 * math.pi), m_rho=16, m_sigma=8)
C2 = VGridSpec(d=3, n=32, L=8.0, gamma=1.0, C=1.0, m_rho=16, m_sigma=38)
C3 = C2
small_3d = VGridSpec(d=3, n=8, L=8.0, gamma=1.0, C=1.0, m_rho=8, m_sigma=38)
small_2d = VGridSpec(d=2, n=16, L=8.0, gamma=0.0, C=1.0 / (2.0 * math.pi), m_rho=8, m_sigma=8)


def vgrid_points(d: int, n: int, L: float) -> np.ndarray:
    """Velocity nodes, shape (d, n, ..., n), C order (last axis fastest)."""
    h = 2.0 * L / n
    ax = -L + h * np.arange(n, dtype=np.float64)
    return np.stack(np.meshgrid(*([ax] * d), indexing="ij"), axis=0)


def xgrid_centres(nx: int, lo: float, hi: float) -> np.ndarray:
    dx = (hi - lo) / nx
    return lo + dx * (np.arange(nx, dtype=np.float64) + 0.5)


def maxwellian(vpts: np.ndarray, rho: float, u, T: float) -> np.ndarray:
    """rho/(2 pi T)^{d/2} exp(-|v-u|^2/(2T)) on the grid (gas constant 1)."""
    d = vpts.shape[0]
    u = np.broadcast_to(np.asarray(u, dtype=np.float64), (d,))
    r2 = sum((vpts[i] - u[i]) ** 2 for i in range(d))
    return rho / (2.0 * math.pi * T) ** (d / 2.0) * np.exp(-r2 / (2.0 * T))


def rh_downstream(mach: float, d: int, rho_l: float = 1.0, T_l: float = 1.0):
    """Downstream (rho, u, T) of a normal shock from the upstream state (Sec. 4,
    Rankine-Hugoniot relations solved in closed form, gamma=(d+2)/d, R=1)."""
    gam = (d + 2.0) / d
    u_l = mach * math.sqrt(gam * T_l)
    m2 = mach * mach
    rho_r = rho_l * (d + 1.0) * m2 / (m2 + d)
    u_r = u_l * (m2 + d) / ((d + 1.0) * m2)
    T_r = T_l * ((d + 2.0) * m2 - 1.0) * (m2 + d) / ((d + 1.0) ** 2 * m2)
    return (rho_l, u_l, T_l), (rho_r, u_r, T_r)


def shock_states(mach: float, d: int):
    return rh_downstream(mach, d)


def c1_distribution(seed: int = 1, spec: VGridSpec = C1) -> np.ndarray:
    """Two unit-temperature Maxwellians at u=(+-2,0) with 1% multiplicative
    seeded Gaussian noise (2D velocity)."""
    v = vgrid_points(spec.d, spec.n, spec.L)
    f = maxwellian(v, 1.0, (2.0, 0.0), 1.0) + maxwellian(v, 1.0, (-2.0, 0.0), 1.0)
    rng = np.random.default_rng(seed)
    return f * (1.0 + 0.01 * rng.standard_normal(f.shape))


def c2_bimaxwellian(seed: int = 2, spec: VGridSpec = C2) -> np.ndarray:
    """a*M(1,0,1) + (1-a)*M(1,(1.5,0,0),0.5), a ~ U[0.3,0.7] (seeded)."""
    v = vgrid_points(spec.d, spec.n, spec.L)
    a = np.random.default_rng(seed).uniform(0.3, 0.7)
    return a * maxwellian(v, 1.0, (0.0,) * spec.d, 1.0) + (1 - a) * maxwellian(
        v, 1.0, (1.5,) + (0.0,) * (spec.d - 1), 0.5)


def c2_bkw(t: float, spec: VGridSpec, t0: float | None = None):
    """BKW self-similar solution for Maxwell molecules and its time derivative.

    3D (B = 1/(4 pi)):  K = 1 - exp(-(t+t0)/6),
        f = exp(-|v|^2/(2K)) / (2 (2 pi K)^{3/2}) * ((5K-3)/K + (1-K)|v|^2/K^2)
    2D (B = 1/(2 pi)):  S = 1 - exp(-(t+t0)/8)/2,
        f = exp(-|v|^2/(2S)) / (2 pi S^2) * (2S - 1 + (1-S)|v|^2/(2S))
    Returns (f, df/dt) on the grid; df/dt is the analytic derivative.
    """
    v = vgrid_points(spec.d, spec.n, spec.L)
    r2 = sum(v[i] ** 2 for i in range(spec.d))
    if spec.d == 3:
        if t0 is None:
            t0 = 6.0 * math.log(2.5)
        K = 1.0 - math.exp(-(t + t0) / 6.0)
        dK = math.exp(-(t + t0) / 6.0) / 6.0

        def fK(Kv):
            return np.exp(-r2 / (2 * Kv)) / (2 * (2 * math.pi * Kv) ** 1.5) * (
                (5 * Kv - 3) / Kv + (1 - Kv) * r2 / Kv ** 2)
        f = fK(K)
        h = 1e-6
        dfdK = (fK(K + h) - fK(K - h)) / (2 * h)
        dfdK2 = (fK(K + 2 * h) - fK(K - 2 * h)) / (4 * h)
        dfdK = (4 * dfdK - dfdK2) / 3.0  # Richardson
        return f, dfdK * dK
    if t0 is None:
        t0 = 0.0
    S = 1.0 - 0.5 * math.exp(-(t + t0) / 8.0)
    dS = 0.5 * math.exp(-(t + t0) / 8.0) / 8.0

    def fS(Sv):
        return np.exp(-r2 / (2 * Sv)) / (2 * math.pi * Sv ** 2) * (
            2 * Sv - 1 + (1 - Sv) * r2 / (2 * Sv))
    f = fS(S)
    h = 1e-6
    d1 = (fS(S + h) - fS(S - h)) / (2 * h)
    d2 = (fS(S + 2 * h) - fS(S - 2 * h)) / (4 * h)
    return f, (4 * d1 - d2) / 3.0 * dS


def smooth_basis(r: int, spec: VGridSpec, seed: int = 7, orthonormal: bool = True,
                 width: float = 1.0) -> np.ndarray:
    """r smooth, decaying velocity functions (Maxwellian times random
    polynomials of degree <= 2, random centres), shape (r, n^d).

    With ``orthonormal`` the rows are orthonormalised in the weighted inner
    product dv^d * sum_q (numpy QR; input preparation only)."""
    rng = np.random.default_rng(seed)
    v = vgrid_points(spec.d, spec.n, spec.L)
    d = spec.d
    rows = []
    for _ in range(r):
        c = rng.uniform(-1.5, 1.5, size=d)
        T = width * rng.uniform(0.6, 1.4)
        base = maxwellian(v, 1.0, c, T)
        poly = rng.standard_normal()
        for i in range(d):
            poly = poly + rng.standard_normal() * (v[i] - c[i])
        for i in range(d):
            for j in range(i, d):
                poly = poly + 0.3 * rng.standard_normal() * (v[i] - c[i]) * (v[j] - c[j])
        rows.append((base * poly).reshape(-1))
    W = np.array(rows)
    if orthonormal:
        dvd = (2.0 * spec.L / spec.n) ** d
        q, _ = np.linalg.qr(W.T)
        W = q.T / math.sqrt(dvd)
    return np.ascontiguousarray(W)


def shock_initial(mach: float, spec: VGridSpec, nx: int, x_lo: float = -30.0,
                  x_hi: float = 30.0, alpha: float = 0.5, pert: float = 1e-3,
                  pert_rank: int = 10, seed: int = 3):
    """Normal-shock-like initial data f0(x, v), shape (nx, n^d), and the two
    inflow Maxwellians.

    rho, u_1, T are blended from the upstream to the downstream state by
    (tanh(alpha x)+1)/2 (Sec. 5.2 with alpha = 0.5); a seeded smooth rank-
    ``pert_rank`` perturbation of relative size ``pert`` is added.
    Returns dict(f0, fL, fR, states, x)."""
    d = spec.d
    (rl, ul, Tl), (rr, ur, Tr) = rh_downstream(mach, d)
    x = xgrid_centres(nx, x_lo, x_hi)
    v = vgrid_points(d, spec.n, spec.L)
    s = 0.5 * (np.tanh(alpha * x) + 1.0)
    rho = rl + (rr - rl) * s
    u = ul + (ur - ul) * s
    T = Tl + (Tr - Tl) * s
    n = spec.npts
    f0 = np.empty((nx, n))
    r2perp = sum(v[i] ** 2 for i in range(1, d)).reshape(-1)
    v1 = v[0].reshape(-1)
    for p in range(nx):
        f0[p] = rho[p] / (2 * math.pi * T[p]) ** (d / 2) * np.exp(
            -((v1 - u[p]) ** 2 + r2perp) / (2 * T[p]))
    if pert > 0 and pert_rank > 0:
        rng = np.random.default_rng(seed)
        xi = rng.uniform(-10.0, 10.0, size=pert_rank)
        A = np.exp(-((x[:, None] - xi[None, :]) ** 2) / 8.0)           # nx x pr
        m0 = maxwellian(v, 1.0, (0.0,) * d, 1.0).reshape(-1)
        Bv = []
        for _ in range(pert_rank):
            poly = rng.standard_normal() * np.ones(n)
            for i in range(d):
                poly += rng.standard_normal() * v[i].reshape(-1)
            for i in range(d):
                for j in range(i, d):
                    poly += rng.standard_normal() * (v[i] * v[j]).reshape(-1)
            Bv.append(m0 * poly)
        Bv = np.array(Bv)                                                 # pr x n
        P = A @ Bv
        f0 = f0 + pert * f0.max() * P / np.abs(P).max()
    fL = maxwellian(v, rl, (ul,) + (0.0,) * (d - 1), Tl).reshape(-1)
    fR = maxwellian(v, rr, (ur,) + (0.0,) * (d - 1), Tr).reshape(-1)
    return dict(f0=f0, fL=fL, fR=fR, states=((rl, ul, Tl), (rr, ur, Tr)), x=x)


# Fourier flow (Sec. 5.3): x in [0, 2], 2D velocity 32^2 on [-7.86, 7.86]^2,
# Maxwell diffusive walls at rest with T_w = 1 (x = 0) and 1.2 (x = 2),
# initial Maxwellian rho = 1, u = 0, T = 1; 2D Maxwell molecules B = 1/(2 pi)
# in the Carleman form with 8 directions (m_rho is not used by that form).
FOURIER = VGridSpec(d=2, n=32, L=7.86, gamma=0.0, C=1.0 / (2.0 * math.pi), m_rho=1, m_sigma=8)


def wall_initial(spec: VGridSpec, nx: int, x_lo: float = 0.0, x_hi: float = 2.0,
                 T_walls=(1.0, 1.2), rho0: float = 1.0, T0: float = 1.0,
                 pert: float = 0.0, pert_rank: int = 0, seed: int = 3):
    """Gas between two diffusive walls at rest: a uniform Maxwellian (rho0, 0,
    T0) in every cell plus, optionally, a seeded smooth rank-``pert_rank``
    perturbation of relative size ``pert`` (x-profiles exp(-(x - xi)^2 /
    (w^2/8)) on the interval's width w, velocity profiles a random quadratic
    times the unit Maxwellian).  fL, fR are the normalised wall Maxwellians
    (density 1, temperatures T_walls).  Returns dict(f0, fL, fR, x)."""
    d = spec.d
    x = xgrid_centres(nx, x_lo, x_hi)
    v = vgrid_points(d, spec.n, spec.L)
    n = spec.npts
    m = maxwellian(v, rho0, (0.0,) * d, T0).reshape(-1)
    f0 = np.tile(m, (nx, 1))
    if pert > 0 and pert_rank > 0:
        rng = np.random.default_rng(seed)
        w = x_hi - x_lo
        xi = rng.uniform(x_lo, x_hi, size=pert_rank)
        A = np.exp(-((x[:, None] - xi[None, :]) ** 2) / (w * w / 8.0))
        m0 = maxwellian(v, 1.0, (0.0,) * d, 1.0).reshape(-1)
        Bv = []
        for _ in range(pert_rank):
            poly = rng.standard_normal() * np.ones(n)
            for i in range(d):
                poly += rng.standard_normal() * v[i].reshape(-1)
            for i in range(d):
                for j in range(i, d):
                    poly += rng.standard_normal() * (v[i] * v[j]).reshape(-1)
            Bv.append(m0 * poly)
        P = A @ np.array(Bv)
        f0 = f0 + pert * f0.max() * P / np.abs(P).max()
    fL = maxwellian(v, 1.0, (0.0,) * d, T_walls[0]).reshape(-1)
    fR = maxwellian(v, 1.0, (0.0,) * d, T_walls[1]).reshape(-1)
    return dict(f0=f0, fL=fL, fR=fR, x=x)


def rect_field(spec: VGridSpec, nx: int, ny: int, seed: int = 3, rank: int = 3,
               pert: float = 5e-2) -> np.ndarray:
    """Seeded smooth state on an nx x ny rectangle (cell ix ny + iy): a
    Maxwellian whose temperature grows along x and y and whose bulk velocity
    varies smoothly, plus a seeded rank-``rank`` perturbation (random
    Gaussian-weighted velocity profiles) of relative size ``pert``."""
    d = spec.d
    v = vgrid_points(d, spec.n, spec.L)
    rng = np.random.default_rng(seed)
    F = np.empty((nx * ny, spec.npts))
    z = (0.0,) * (d - 2)
    for ix in range(nx):
        for iy in range(ny):
            T = 1.0 + 0.2 * ix / max(1, nx - 1) + 0.1 * iy / max(1, ny - 1)
            u = (0.3 * math.sin(ix + 0.5 * iy), 0.2 * math.cos(iy - ix)) + z
            F[ix * ny + iy] = maxwellian(v, 1.0 + 0.1 * rng.standard_normal() ** 2, u, T).reshape(-1)
    m0 = maxwellian(v, 1.0, (0.0,) * d, 1.0).reshape(-1)
    B = rng.standard_normal((rank, spec.npts)) * m0
    A = rng.standard_normal((nx * ny, rank))
    return F + pert * F.max() * (A @ B) / np.abs(A @ B).max()


def lowrank_state(f0: np.ndarray, r: int, dx: float, dvd: float):
    """Rank-r factors (X, S, V) of f0 with <X_i,X_j>_x = <V_i,V_j>_v = delta_ij,
    where <a,b>_x = dx sum a b and <a,b>_v = dv^d sum a b.

    Input preparation (numpy SVD) so that every consumer starts from identical
    factors. X: (nx, r), S: (r, r) diagonal, V: (r, n) -- V stored row-wise."""
    w = math.sqrt(dx * dvd)
    U, s, Wt = np.linalg.svd(f0 * w, full_matrices=False)
    U, s, Wt = U[:, :r], s[:r], Wt[:r]
    # sign convention: largest |entry| of each left vector positive
    for i in range(r):
        j = np.argmax(np.abs(U[:, i]))
        if U[j, i] < 0:
            U[:, i] *= -1.0
            Wt[i] *= -1.0
    X = np.ascontiguousarray(U / math.sqrt(dx))
    V = np.ascontiguousarray(Wt / math.sqrt(dvd))
    S = np.diag(s)
    return X, S, V


def lowrank_state_sketch(f0: np.ndarray, r: int, dx: float, dvd: float, seed: int = 0,
                         oversample: int = 10, power: int = 2):
    """Rank-r factors like ``lowrank_state``, from a randomized range finder
    (Gaussian sketch of ``r + oversample`` columns, ``power`` subspace
    iterations with re-orthonormalisation, then the SVD of the small
    projected matrix).  Input preparation for large f0, where a full SVD
    takes seconds; the factors are orthonormal to rounding and the rank-r
    truncation is accurate when the singular values decay fast."""
    w = math.sqrt(dx * dvd)
    A = f0 * w
    rng = np.random.default_rng(seed)
    k = min(r + oversample, min(A.shape))
    Y = A @ rng.standard_normal((A.shape[1], k))
    Qm, _ = np.linalg.qr(Y)
    for _ in range(power):
        Z, _ = np.linalg.qr(A.T @ Qm)
        Qm, _ = np.linalg.qr(A @ Z)
    B = Qm.T @ A
    Ub, s, Wt = np.linalg.svd(B, full_matrices=False)
    U = Qm @ Ub
    U, s, Wt = U[:, :r], s[:r], Wt[:r]
    for i in range(r):
        j = np.argmax(np.abs(U[:, i]))
        if U[j, i] < 0:
            U[:, i] *= -1.0
            Wt[i] *= -1.0
    X = np.ascontiguousarray(U / math.sqrt(dx))
    V = np.ascontiguousarray(Wt / math.sqrt(dvd))
    return X, np.diag(s), V


def serving_trace(count: int = 64, seed: int = 5, rate: float = 4.0, mach=(1.2, 3.0),
                  nx_choices=(128, 256, 512), n_choices=(24, 32), r0=(5, 25),
                  half_width=None, x_lo: float = -30.0, x_hi: float = 30.0, cfl: float = 0.35,
                  nu_frac: float = 1.5, safety: float = 0.5, C: float = 1.0):
    """A stream of steady normal-shock solves (hard spheres in 3D velocity):
    Poisson arrivals of the given rate (exponential gaps, first request at
    t = 0), Mach ~ U[mach], N_x and N_v drawn uniformly from the choices,
    initial rank ~ U{r0}.

    Velocity box: L_v = 8 at N_v = 24 and 10 at N_v = 32 (``half_width``
    overrides), so the grid step stays at or below 2/3 of the upstream
    thermal speed.  dt = safety * min(cfl dx / L_v, nu_frac / nu): the upwind
    CFL on the fastest grid velocity, and the relaxation limit with nu =
    4 pi C R rho_R a bound of the hard-sphere loss rate (B = C |q| truncated
    at R = 4 L_v / (3 + sqrt 2), downstream density rho_R).
    Returns a list of dicts."""
    hw = {24: 8.0, 32: 10.0} if half_width is None else dict(half_width)
    rng = np.random.default_rng(seed)
    out = []
    t = 0.0
    for k in range(count):   # one draw sequence per request: a longer trace extends a shorter one
        gap = float(rng.exponential(1.0 / rate))
        t = 0.0 if k == 0 else t + gap
        m = float(rng.uniform(*mach))
        nx = int(rng.choice(nx_choices))
        n = int(rng.choice(n_choices))
        r = int(rng.integers(r0[0], r0[1] + 1))
        L = float(hw[n])
        dx = (x_hi - x_lo) / nx
        R = 4.0 * L / (3.0 + math.sqrt(2.0))
        rho_r = rh_downstream(m, 3)[1][0]
        dt = safety * min(cfl * dx / L, nu_frac / (4.0 * math.pi * C * R * rho_r))
        out.append(dict(index=k, arrival=t, mach=m, nx=nx, n=n, r0=r, L=L,
                        dt=dt, x_lo=x_lo, x_hi=x_hi))
    return out


def serving_trace_2d(count: int = 8, seed: int = 6, rate: float = 4.0, mach=(1.2, 2.0),
                     nx_choices=(32, 64), n: int = 32, L: float = 8.0, r0=(4, 8),
                     x_lo: float = -30.0, x_hi: float = 30.0, courant: float = 0.4):
    """A stream of steady normal-shock solves in the paper's own velocity
    dimension (2D velocity, Maxwell molecules B = 1/(2 pi), the Sec. 5.2
    class): Poisson arrivals of the given rate (exponential gaps, first at
    t = 0), Mach ~ U[mach], N_x drawn from the choices on [x_lo, x_hi],
    N_v = n^2 on [-L, L]^2, initial rank ~ U{r0}; dt = courant dx / L.
    Returns a list of dicts (same keys as serving_trace)."""
    rng = np.random.default_rng(seed)
    out = []
    t = 0.0
    for k in range(count):
        gap = float(rng.exponential(1.0 / rate))
        t = 0.0 if k == 0 else t + gap
        m = float(rng.uniform(*mach))
        nx = int(rng.choice(nx_choices))
        r = int(rng.integers(r0[0], r0[1] + 1))
        dx = (x_hi - x_lo) / nx
        out.append(dict(index=k, arrival=t, mach=m, nx=nx, n=n, r0=r, L=L, d=2,
                        dt=courant * dx / L, x_lo=x_lo, x_hi=x_hi))
    return out
