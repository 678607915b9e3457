"""Fully discrete adaptive dynamical low-rank step (oracle, float64).

TEST INFRASTRUCTURE ONLY -- see oracle/__init__.py.

Follows the paper:
  * state f = sum_ij X_i S_ij V_j with <X_i,X_j>_x = <V_i,V_j>_v = delta_ij
    (eqs. lowrank decomposition, orthogonality); inner products by the
    midpoint rule, <a,b>_x = dx sum a b, <a,b>_v = dv^d sum a b (Sec. 2.4);
  * first-order upwind "discretise then project" transport, v^+ D_+ with a
    backward and v^- D_- with a forward difference (eq. scheme:fullupwind);
  * ghost values of K from the projected boundary function f^b (eq. boundary
    general), inflow Maxwellian (or a Maxwell diffusive wall with its density
    set by zero net mass flux) on the inflow half, the outflow half taken
    from the adjacent interior cell (Sec. 2.3);
  * K-step, S-step, L-step with forward Euler and QR (Sec. 2.4), the
    collision terms written with the symmetrised pair values Q_s(V_m, V_n)
    for m <= n and weights (2 - delta_mn);
  * residual err from the pieces dK, dS, dL and the cross terms I, II, III
    (eqs. err low rank1, err low rank2, Sec. 5.1);
  * adaptivity: add the boundary basis at the start of a step (Sec. 3.1),
    drop singular values of S below drop_tol = c * err at its end (Sec. 3.2,
    Sec. 5.1 with c = 0.2), err_ada evaluated exactly from the factors.

Space is one-dimensional here (x along the first velocity axis), which is the
geometry of the normal-shock workload.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import collision as oc


@dataclass
class Problem1D:
    vs: oc.VelocitySetup
    nx: int
    x_lo: float
    x_hi: float
    fL: np.ndarray            # inflow Maxwellian at the left wall, (n,)
    fR: np.ndarray            # inflow Maxwellian at the right wall, (n,)
    conserve: bool = True     # conservation projection of each Q_s
    collision: object = None  # pair evaluator: (V, pairs, vs, conserve) -> (Q, Q+)
    # Maxwell diffusive walls (Sec. 2.3): fL / fR then give the shape of the
    # wall Maxwellian exp(-|v - u_w|^2 / 2 T_w) (any positive multiple), and
    # its density rho_w is set by zero net mass flux through the wall
    wall_left: bool = False
    wall_right: bool = False

    @property
    def dx(self):
        return (self.x_hi - self.x_lo) / self.nx

    @property
    def wx(self):
        """Weight of the x-side inner product <a, b>_x = wx sum a b."""
        return self.dx

    @property
    def dvd(self):
        return self.vs.dv ** self.vs.d

    def v1(self):
        return oc.grid(self.vs)[0].reshape(-1)


@dataclass
class State:
    X: np.ndarray   # (nx, r)
    S: np.ndarray   # (r, r)
    V: np.ndarray   # (r, n), rows are V_j

    @property
    def r(self):
        return self.S.shape[0]

    def full(self):
        return self.X @ self.S @ self.V


@dataclass
class StepInfo:
    err: float = 0.0
    err_ada: float = 0.0
    drop_tol: float = 0.0
    r_in: int = 0
    r_added: int = 0
    r_out: int = 0
    sigma_dropped: float = 0.0
    extra: dict = field(default_factory=dict)


# ----------------------------------------------------------------------------
# helpers
# ----------------------------------------------------------------------------
def pair_list(r: int):
    return [(m, n) for m in range(r) for n in range(m, r)]


def qr_pos(A: np.ndarray):
    """Householder QR (numpy) with diag(R) >= 0."""
    Q, R = np.linalg.qr(A)
    s = np.where(np.diag(R) < 0, -1.0, 1.0)
    return Q * s[None, :], R * s[:, None]


def weighted_qr_cols(A: np.ndarray, w: float):
    """A = Q R with <Q_i, Q_j> = delta_ij in the inner product w * sum."""
    Q, R = qr_pos(math.sqrt(w) * A)
    return Q / math.sqrt(w), R


def transport_matrices(V: np.ndarray, prob: Problem1D):
    """A^+_{jl} = <v^+ V_j V_l>_v, A^-_{jl} = <v^- V_j V_l>_v."""
    v1 = prob.v1()
    vp = np.maximum(v1, 0.0)
    vm = np.minimum(v1, 0.0)
    return prob.dvd * (V * vp) @ V.T, prob.dvd * (V * vm) @ V.T


def wall_density(f_out: np.ndarray, M_w: np.ndarray, prob: Problem1D, side: int) -> float:
    """rho_w of a Maxwell diffusive wall (Sec. 2.3): with n the outward normal
    (-e1 at the left wall, +e1 at the right, wall velocity tangential),
        rho_w = - int_{v.n >= 0} (v.n) f dv / int_{v.n < 0} (v.n) M_w dv,
    f the distribution leaving the domain (the adjacent interior cell) and M_w
    the wall Maxwellian shape; midpoint rule in v."""
    vn = -prob.v1() if side == 0 else prob.v1()
    out = vn >= 0
    num = float(np.sum(vn[out] * f_out[out]))
    den = float(np.sum(vn[~out] * M_w[~out]))
    return -num / den


def boundary_function(side: int, f_adj: np.ndarray, prob: Problem1D) -> np.ndarray:
    """The incoming half of the boundary function f_bdy at one wall: the
    prescribed inflow Maxwellian, or rho_w M_w at a diffusive wall with rho_w
    from the outgoing flux of f_adj (the adjacent interior cell).  Values on
    the outgoing half are not used by the callers."""
    M = prob.fL if side == 0 else prob.fR
    wall = prob.wall_left if side == 0 else prob.wall_right
    if not wall:
        return M
    return wall_density(f_adj, M, prob, side) * M


def ghosts(K: np.ndarray, V: np.ndarray, prob: Problem1D):
    """Ghost values of K_j at both walls from the projected boundary function:
    K_j = <f_bdy 1_in, V_j>_v + sum_l K_l(adjacent cell) <1_out V_l V_j>_v.
    Left wall (outward normal -e1): inflow v1 > 0.  Right wall: inflow v1 < 0.
    At a diffusive wall f_bdy = rho_w M_w with rho_w from the extrapolated
    outgoing distribution sum_l K_l(adjacent cell) V_l."""
    v1 = prob.v1()
    inL = (v1 > 0).astype(np.float64)
    inR = (v1 < 0).astype(np.float64)
    outL, outR = 1.0 - inL, 1.0 - inR
    fbL = boundary_function(0, K[0] @ V, prob)
    fbR = boundary_function(1, K[-1] @ V, prob)
    gl = prob.dvd * V @ (fbL * inL) + prob.dvd * ((V * outL) @ V.T) @ K[0]
    gr = prob.dvd * V @ (fbR * inR) + prob.dvd * ((V * outR) @ V.T) @ K[-1]
    return gl, gr


def d_plus(K, gl, dx):
    """(K_p - K_{p-1}) / dx with the left ghost."""
    prev = np.vstack([gl[None, :], K[:-1]])
    return (K - prev) / dx


def d_minus(K, gr, dx):
    """(K_{p+1} - K_p) / dx with the right ghost."""
    nxt = np.vstack([K[1:], gr[None, :]])
    return (nxt - K) / dx


def collision_tensor(V, Qs, prob):
    """C_{j,(mn)} = <V_j, Q_s(V_m, V_n)>_v, shape (r, P)."""
    return prob.dvd * V @ Qs.T


def pair_products(K, pairs, wts):
    """(2 - delta_mn) K_m K_n for each pair, shape (nx, P)."""
    return np.stack([w * K[:, m] * K[:, n] for (m, n), w in zip(pairs, wts)], axis=1)


def evaluate_pairs(V, pairs, prob):
    if prob.collision is not None:
        return prob.collision(V, pairs, prob.vs, prob.conserve)
    return oc.q_pairs(V, pairs, prob.vs, conserve=prob.conserve)


def initial_state(F0: np.ndarray, r: int, wx: float, dvd: float) -> State:
    """Rank-r initial factors of a full f^0 (Sec. 2.4, first paragraph: the
    initial values of X, S, V come from a truncated SVD of f^0).  The SVD is
    taken of sqrt(wx dv^d) F0 (cells x n) so that the weights of the two
    inner products are folded into the factors: X = U_r / sqrt(wx),
    V = W_r^T / sqrt(dv^d), S = diag(sigma_1..sigma_r); then
    f_r = X S V is the best rank-r approximation in the L2(x, v) norm."""
    U, s, Wt = np.linalg.svd(math.sqrt(wx * dvd) * np.asarray(F0, dtype=np.float64),
                             full_matrices=False)
    return State(U[:, :r] / math.sqrt(wx), np.diag(s[:r]), Wt[:r] / math.sqrt(dvd))


# ----------------------------------------------------------------------------
# one fixed-rank step (Sec. 2.4)
# ----------------------------------------------------------------------------
def ksl_step(st: State, prob: Problem1D, dt: float, Qs=None):
    """One K -> S -> L step with forward Euler; returns (new State, err, pieces)."""
    if isinstance(prob, Problem2D):
        return ksl_step_2d(st, prob, dt, Qs)
    X, S, V = st.X, st.S, st.V
    r = S.shape[0]
    dx, dvd = prob.dx, prob.dvd
    pairs = pair_list(r)
    wts = np.array([1.0 if m == n else 2.0 for (m, n) in pairs])
    if Qs is None:
        Qs, _ = evaluate_pairs(V, pairs, prob)            # (P, n) reused by K, S, L
    Ap, Am = transport_matrices(V, prob)
    Cj = collision_tensor(V, Qs, prob)                    # (r, P)

    # K-step
    K = X @ S
    gl, gr = ghosts(K, V, prob)
    rhsK = -d_plus(K, gl, dx) @ Ap.T - d_minus(K, gr, dx) @ Am.T \
        + pair_products(K, pairs, wts) @ Cj.T
    K1 = K + dt * rhsK
    X1, S1 = weighted_qr_cols(K1, dx)

    # S-step (uses K^{n+1} = X1 S1 and its own ghosts)
    Kn = X1 @ S1
    gl, gr = ghosts(Kn, V, prob)
    Dp = dx * X1.T @ d_plus(Kn, gl, dx)                   # <X_i, D_+ K_l>_x, (r, r)
    Dm = dx * X1.T @ d_minus(Kn, gr, dx)
    T = dx * X1.T @ pair_products(Kn, pairs, wts)         # (r, P)
    S2 = S1 + dt * (Dp @ Ap.T + Dm @ Am.T - T @ Cj.T)

    # L-step
    L = S2 @ V                                            # (r, n)
    Kt = X1 @ S2
    gl, gr = ghosts(Kt, V, prob)
    Dpt = dx * X1.T @ d_plus(Kt, gl, dx)
    Dmt = dx * X1.T @ d_minus(Kt, gr, dx)
    Tt = dx * X1.T @ pair_products(Kt, pairs, wts)        # (r, P)
    v1 = prob.v1()
    vp, vm = np.maximum(v1, 0.0), np.minimum(v1, 0.0)
    L1 = L - dt * ((Dpt @ V) * vp[None, :] + (Dmt @ V) * vm[None, :]) + dt * Tt @ Qs
    Vq, R = weighted_qr_cols(L1.T, dvd)
    V1 = Vq.T
    Snew = R.T

    # residual from the pieces (Sec. 5.1)
    dK = K1 - K
    dS = S2 - S1
    dL = L1 - L
    kx = dx * X1.T @ dK                                   # <dK_j, X_i>, indexed [i, j]
    lv = dvd * dL @ V.T                                   # <dL_i, V_j>, [i, j]
    e2 = dx * (dK ** 2).sum() + (dS ** 2).sum() + dvd * (dL ** 2).sum() \
        + 2.0 * (kx * dS).sum() + 2.0 * (lv * dS).sum() + 2.0 * (kx * lv).sum()
    err = math.sqrt(max(e2, 0.0))
    pieces = dict(K1=K1, S1=S1, S2=S2, L1=L1, X1=X1, Qs=Qs, Cj=Cj, e2=e2)
    return State(X1, Snew, V1), err, pieces


# ----------------------------------------------------------------------------
# adaptivity (Sec. 3)
# ----------------------------------------------------------------------------
def boundary_matrix(st: State, prob: Problem1D):
    """F_b rows f^b(x_b, .) at the two walls: inflow half from the prescribed
    Maxwellian, outflow half from the adjacent interior cell."""
    if isinstance(prob, Problem2D):
        return boundary_matrix_2d(st, prob)
    v1 = prob.v1()
    K = st.X @ st.S
    fin = K[0] @ st.V
    fout = K[-1] @ st.V
    left = np.where(v1 > 0, boundary_function(0, fin, prob), fin)
    right = np.where(v1 < 0, boundary_function(1, fout, prob), fout)
    return np.vstack([left, right])


def add_boundary_basis(st: State, prob: Problem1D, add_tol: float = 1e-10,
                       r_max: int = 10 ** 9, rng=None):
    """Append the right singular vectors of F_b with sigma > add_tol (capped at
    r_max), a random X_h, zero-padded S; re-orthonormalise both sides by QR;
    S_q = S_x S^ S_v^T.  Leaves f unchanged.  On the rectangle F_b is first
    projected onto the complement of span V (with every face cell's row the
    rows far outnumber the room under the cap; the projection keeps that room
    for new directions, and gives the same span when the cap does not bind)."""
    Fb = boundary_matrix(st, prob)
    if isinstance(prob, Problem2D):
        # on the rectangle the rows outnumber the room r_max - r: take the
        # boundary information not yet in span V (rows projected onto V^perp)
        Fb = Fb - prob.dvd * (Fb @ st.V.T) @ st.V
    _, sb, Qbt = np.linalg.svd(Fb, full_matrices=False)
    rb = int((sb > add_tol).sum())
    rb = max(0, min(rb, r_max - st.r))
    if rb == 0:
        return st, 0
    if rng is None:
        rng = np.random.default_rng(0)
    Xh = rng.standard_normal((st.X.shape[0], rb))
    Xhat = np.hstack([st.X, Xh])
    Vhat = np.vstack([st.V, Qbt[:rb]])
    Shat = np.zeros((st.r + rb, st.r + rb))
    Shat[:st.r, :st.r] = st.S
    Xq, Sx = weighted_qr_cols(Xhat, prob.wx)
    Vq, Sv = weighted_qr_cols(Vhat.T, prob.dvd)
    return State(Xq, Sx @ Shat @ Sv.T, Vq.T), rb


def drop_basis(st: State, drop_tol: float, r_min: int = 1, r_max: int = 10 ** 9):
    """SVD of S; keep sigma >= drop_tol (clamped to [r_min, r_max]); rotate."""
    U, s, Qt = np.linalg.svd(st.S)
    keep = int((s >= drop_tol).sum())
    keep = max(min(keep, r_max, len(s)), min(r_min, len(s)))
    X = st.X @ U[:, :keep]
    V = Qt[:keep] @ st.V
    return State(X, np.diag(s[:keep]), V), s, keep, U, Qt


def adaptive_step(st: State, prob: Problem1D, dt: float, c: float = 0.2,
                  add: bool = True, drop: bool = True, add_tol: float = 1e-10,
                  r_min: int = 1, r_max: int = 30, rng=None):
    info = StepInfo(r_in=st.r)
    if add:
        st, rb = add_boundary_basis(st, prob, add_tol, r_max, rng)
        info.r_added = rb
    start = st
    new, err, pieces = ksl_step(st, prob, dt)
    info.err = err
    if not drop:
        info.err_ada = err
        info.r_out = new.r
        return new, info
    drop_tol = c * err
    info.drop_tol = drop_tol
    out, s, keep, U, Qt = drop_basis(new, drop_tol, r_min, r_max)
    # err_ada^2 = err^2 - |Sigma_perp|^2 + 2 <f^n, D>,  D = X1 U_p Sig_p Q_p^T V1
    sp = s[keep:]
    M = U[:, keep:] @ np.diag(sp) @ Qt[keep:]
    A = prob.wx * start.X.T @ new.X                       # <X^n_k, X1_i>
    B = prob.dvd * start.V @ new.V.T                      # <V^n_l, V1_j>
    fnD = (start.S * (A @ M @ B.T)).sum()
    e2 = err ** 2 - (sp ** 2).sum() + 2.0 * fnD
    info.err_ada = math.sqrt(max(e2, 0.0))
    info.sigma_dropped = float(math.sqrt((sp ** 2).sum()))
    info.r_out = keep
    return out, info


def steady_solve(st: State, prob: Problem1D, dt: float, res_tol: float,
                 max_steps: int, **kw):
    hist = []
    for n in range(max_steps):
        st, info = adaptive_step(st, prob, dt, **kw)
        hist.append(info)
        if info.err_ada <= res_tol:
            return st, hist, True
    return st, hist, False


# ----------------------------------------------------------------------------
# full-tensor reference step (eq. scheme:fullupwind, Sec. 2.2; walls of Sec. 2.3)
# ----------------------------------------------------------------------------
def full_step(F: np.ndarray, prob: Problem1D, dt: float):
    """One forward-Euler step of the full-tensor discretisation the low-rank
    equations are projected from: for every cell,
    f_p <- f_p - dt (v^+ D_+ f + v^- D_- f)_p + dt Q_s(f_p, f_p), the left ghost
    being the boundary function f_bdy where v1 > 0 (the adjacent cell
    elsewhere) and the right ghost likewise where v1 < 0; f_bdy is the inflow
    Maxwellian, or rho_w M_w at a diffusive wall.  F is (nx, n).  Returns
    (F_new, err_full) with err_full = ||F_new - F||_{L2(x,v)} (eq. err full grid)."""
    if isinstance(prob, Problem2D):
        return full_step_2d(F, prob, dt)
    v1 = prob.v1()
    vp, vm = np.maximum(v1, 0.0), np.minimum(v1, 0.0)
    left = np.where(v1 > 0, boundary_function(0, F[0], prob), F[0])
    right = np.where(v1 < 0, boundary_function(1, F[-1], prob), F[-1])
    Q, _ = evaluate_pairs(F, [(p, p) for p in range(F.shape[0])], prob)
    Fn = F - dt * (vp * d_plus(F, left, prob.dx) + vm * d_minus(F, right, prob.dx)) + dt * Q
    err = math.sqrt(prob.dx * prob.dvd * float(((Fn - F) ** 2).sum()))
    return Fn, err


# ----------------------------------------------------------------------------
# two-dimensional physical space (Sec. 2.2: the upwind scheme on a rectangular
# grid, one axis at a time; Sec. 2.3: the boundary on every face)
# ----------------------------------------------------------------------------
@dataclass
class Problem2D:
    """Rectangle [x_lo, x_hi] x [y_lo, y_hi] with nx x ny cells, cell p = ix ny
    + iy; velocity axis 0 along x, axis 1 along y.  faces = four (f, wall)
    pairs for x_lo, x_hi, y_lo, y_hi: f is the boundary function of the face,
    one row per face cell (ny rows on the x faces, nx on the y faces) or one
    row for all; wall=True makes it the shape of a Maxwell diffusive wall's
    Maxwellian (density rho_w per face cell from zero net mass flux).

    Obstacle (Sec. 2.3 applied to the faces of solid cells inside the
    rectangle): solid is a boolean array of nx * ny cells (or None) and
    obstacle the shape of its walls' Maxwellian.  Solid cells hold no gas.
    Every face between a gas cell and a solid neighbour is a Maxwell diffusive
    wall whose outward normal (seen from the gas) points at the solid cell:
    its ghost on the incoming half is rho_w times the obstacle's Maxwellian,
    rho_w from zero net mass flux through that face, and the gas cell itself
    on the outgoing half.  These faces are listed cell by cell (p ascending),
    and within a cell in the order -x, +x, -y, +y of the solid neighbour."""
    vs: oc.VelocitySetup
    nx: int
    ny: int
    x_lo: float
    x_hi: float
    y_lo: float
    y_hi: float
    faces: list
    conserve: bool = True
    collision: object = None
    solid: object = None
    obstacle: object = None

    @property
    def dx(self):
        return (self.x_hi - self.x_lo) / self.nx

    @property
    def dy(self):
        return (self.y_hi - self.y_lo) / self.ny

    @property
    def wx(self):
        return self.dx * self.dy

    @property
    def dvd(self):
        return self.vs.dv ** self.vs.d

    def vel(self, axis: int):
        return oc.grid(self.vs)[axis].reshape(-1)

    def face_cells(self, k: int) -> np.ndarray:
        """Cells along face k (x_lo, x_hi, y_lo, y_hi), in order of the other
        coordinate."""
        ix = np.arange(self.nx)
        iy = np.arange(self.ny)
        if k == 0:
            return iy
        if k == 1:
            return (self.nx - 1) * self.ny + iy
        if k == 2:
            return ix * self.ny
        return ix * self.ny + self.ny - 1

    def face_normal(self, k: int):
        """(velocity axis, sign of the outward normal)."""
        return (0 if k < 2 else 1), (-1.0 if k % 2 == 0 else 1.0)

    def solid_mask(self) -> np.ndarray:
        if self.solid is None:
            return np.zeros(self.nx * self.ny, dtype=bool)
        return np.asarray(self.solid, dtype=bool).reshape(-1)

    def obstacle_faces(self):
        """[(gas cell p, k)] for every gas cell whose neighbour in direction k
        (0: -x, 1: +x, 2: -y, 3: +y, the face's outward normal) is solid."""
        sol = self.solid_mask()
        out = []
        for p in range(self.nx * self.ny):
            if sol[p]:
                continue
            ix, iy = divmod(p, self.ny)
            for k, (jx, jy) in enumerate(((ix - 1, iy), (ix + 1, iy), (ix, iy - 1), (ix, iy + 1))):
                if 0 <= jx < self.nx and 0 <= jy < self.ny and sol[jx * self.ny + jy]:
                    out.append((p, k))
        return out


def _face_rows(prob: Problem2D, k: int) -> np.ndarray:
    f = np.asarray(prob.faces[k][0], dtype=np.float64)
    m = len(prob.face_cells(k))
    return np.broadcast_to(f, (m, prob.vs.n)) if f.ndim == 1 else f


def face_boundary_rows(prob: Problem2D, k: int, F_adj: np.ndarray) -> np.ndarray:
    """The boundary function of face k at each of its cells (incoming half
    used by the callers): the prescribed rows, or rho_w M_w with rho_w from
    the outgoing flux of F_adj (the adjacent cells' distributions, one row per
    face cell) through the face."""
    M = _face_rows(prob, k)
    if not prob.faces[k][1]:
        return M
    axis, sgn = prob.face_normal(k)
    vn = sgn * prob.vel(axis)
    out = vn >= 0
    num = F_adj[:, out] @ vn[out]
    den = M[:, ~out] @ vn[~out]
    return (-num / den)[:, None] * M


def _incoming(prob: Problem2D, k: int) -> np.ndarray:
    axis, sgn = prob.face_normal(k)
    return sgn * prob.vel(axis) < 0


def obstacle_boundary_row(prob: Problem2D, k: int, f_adj: np.ndarray) -> np.ndarray:
    """rho_w M_obs on an obstacle face with outward normal k, rho_w from the
    outgoing flux of the adjacent gas cell's f_adj (zero net mass flux)."""
    axis, sgn = prob.face_normal(k)
    vn = sgn * prob.vel(axis)
    out = vn >= 0
    M = np.asarray(prob.obstacle, dtype=np.float64)
    return (-(f_adj[out] @ vn[out]) / (M[~out] @ vn[~out])) * M


def obstacle_ghosts(K: np.ndarray, V: np.ndarray, prob: Problem2D):
    """Ghost rows of K on every obstacle face (same formula as ghosts_2d)."""
    out = []
    for (p, k) in prob.obstacle_faces():
        inc = _incoming(prob, k).astype(np.float64)
        fb = obstacle_boundary_row(prob, k, K[p] @ V)
        Mo = prob.dvd * (V * (1.0 - inc)) @ V.T
        out.append(prob.dvd * (fb * inc) @ V.T + K[p] @ Mo)
    return np.array(out).reshape(-1, K.shape[1])


def ghosts_2d(K: np.ndarray, V: np.ndarray, prob: Problem2D):
    """Ghost rows of K on every face cell (eq. boundary general):
    K_j = <f_bdy 1_in, V_j>_v + sum_l K_l(adjacent cell) <1_out V_l V_j>_v."""
    out = []
    for k in range(4):
        cells = prob.face_cells(k)
        inc = _incoming(prob, k).astype(np.float64)
        Kc = K[cells]
        fb = face_boundary_rows(prob, k, Kc @ V)
        Mo = prob.dvd * (V * (1.0 - inc)) @ V.T
        out.append(prob.dvd * (fb * inc) @ V.T + Kc @ Mo)
    return out


def _shift(K: np.ndarray, prob: Problem2D, axis: int, step: int, ghost: np.ndarray, og=None):
    """K at the neighbour p + step e_axis of every cell, the face ghost where
    that neighbour lies outside, the obstacle face's ghost (og, rows in the
    order of obstacle_faces) where it is solid."""
    G = K.reshape(prob.nx, prob.ny, -1)
    sh = np.roll(G, -step, axis=axis).copy()
    if axis == 0:
        sh[-1 if step > 0 else 0, :, :] = ghost
    else:
        sh[:, -1 if step > 0 else 0, :] = ghost
    sh = sh.reshape(K.shape)
    if og is not None:
        kk = 2 * axis + (1 if step > 0 else 0)
        for b, (p, k) in enumerate(prob.obstacle_faces()):
            if k == kk:
                sh[p] = og[b]
    return sh


def d_plus_2d(K, g, prob, axis, og=None):
    """(K_p - K_{p - e_axis}) / h_axis with the low face's ghost."""
    h = prob.dx if axis == 0 else prob.dy
    return (K - _shift(K, prob, axis, -1, g[2 * axis], og)) / h


def d_minus_2d(K, g, prob, axis, og=None):
    """(K_{p + e_axis} - K_p) / h_axis with the high face's ghost."""
    h = prob.dx if axis == 0 else prob.dy
    return (_shift(K, prob, axis, 1, g[2 * axis + 1], og) - K) / h


def transport_matrices_2d(V, prob: Problem2D):
    """[(A+, A-) for each axis], A+-_{jl} = <v_a^+- V_j V_l>_v."""
    res = []
    for a in range(2):
        va = prob.vel(a)
        res.append((prob.dvd * (V * np.maximum(va, 0.0)) @ V.T,
                    prob.dvd * (V * np.minimum(va, 0.0)) @ V.T))
    return res


def ksl_step_2d(st: State, prob: Problem2D, dt: float, Qs=None):
    """The K -> S -> L step of ksl_step with both axes' upwind terms."""
    X, S, V = st.X, st.S, st.V
    r = S.shape[0]
    wx, dvd = prob.wx, prob.dvd
    pairs = pair_list(r)
    wts = np.array([1.0 if m == n else 2.0 for (m, n) in pairs])
    if Qs is None:
        Qs, _ = evaluate_pairs(V, pairs, prob)
    A = transport_matrices_2d(V, prob)
    Cj = collision_tensor(V, Qs, prob)

    gas = (~prob.solid_mask()).astype(np.float64)[:, None]

    def gh(K):
        return ghosts_2d(K, V, prob), obstacle_ghosts(K, V, prob)

    def transport_K(K):
        g, og = gh(K)
        return sum(d_plus_2d(K, g, prob, a, og) @ A[a][0].T +
                   d_minus_2d(K, g, prob, a, og) @ A[a][1].T for a in range(2))

    # K-step (solid cells hold no gas)
    K = X @ S
    K1 = gas * (K + dt * (-transport_K(K) + pair_products(K, pairs, wts) @ Cj.T))
    X1, S1 = weighted_qr_cols(K1, wx)
    # S-step
    Kn = X1 @ S1
    g, og = gh(Kn)
    acc = np.zeros((r, r))
    for a in range(2):
        acc += wx * X1.T @ d_plus_2d(Kn, g, prob, a, og) @ A[a][0].T
        acc += wx * X1.T @ d_minus_2d(Kn, g, prob, a, og) @ A[a][1].T
    T = wx * X1.T @ pair_products(Kn, pairs, wts)
    S2 = S1 + dt * (acc - T @ Cj.T)
    # L-step
    L = S2 @ V
    Kt = X1 @ S2
    g, og = gh(Kt)
    L1 = L + dt * (wx * X1.T @ pair_products(Kt, pairs, wts)) @ Qs
    for a in range(2):
        va = prob.vel(a)
        L1 -= dt * (wx * X1.T @ d_plus_2d(Kt, g, prob, a, og) @ V) * np.maximum(va, 0.0)[None, :]
        L1 -= dt * (wx * X1.T @ d_minus_2d(Kt, g, prob, a, og) @ V) * np.minimum(va, 0.0)[None, :]
    Vq, R = weighted_qr_cols(L1.T, dvd)
    # residual from the pieces (Sec. 5.1)
    dK, dS, dL = K1 - K, S2 - S1, L1 - L
    kx = wx * X1.T @ dK
    lv = dvd * dL @ V.T
    e2 = wx * (dK ** 2).sum() + (dS ** 2).sum() + dvd * (dL ** 2).sum() \
        + 2.0 * (kx * dS).sum() + 2.0 * (lv * dS).sum() + 2.0 * (kx * lv).sum()
    err = math.sqrt(max(e2, 0.0))
    pieces = dict(K1=K1, S1=S1, S2=S2, L1=L1, X1=X1, Qs=Qs, Cj=Cj, e2=e2)
    return State(X1, R.T, Vq.T), err, pieces


def boundary_matrix_2d(st: State, prob: Problem2D):
    """F_b: one row f^b(x_b, .) per face cell of every face (a corner cell
    once per face; zero for a solid face cell), then one per obstacle face:
    the boundary function on the incoming half, the adjacent gas cell on the
    outgoing half."""
    K = st.X @ st.S
    rows = []
    sol = prob.solid_mask()
    for k in range(4):
        cells = prob.face_cells(k)
        Fa = K[cells] @ st.V
        Fk = np.where(_incoming(prob, k)[None, :], face_boundary_rows(prob, k, Fa), Fa)
        Fk[sol[cells]] = 0.0        # a solid face cell is no gas boundary: a zero row
        rows.append(Fk)
    for (p, k) in prob.obstacle_faces():
        fa = K[p] @ st.V
        rows.append(np.where(_incoming(prob, k), obstacle_boundary_row(prob, k, fa), fa)[None, :])
    return np.vstack(rows)


def full_step_2d(F: np.ndarray, prob: Problem2D, dt: float):
    """Full-tensor step on the rectangle: f_p <- f_p - dt sum_a (v_a^+ D^a_+ f +
    v_a^- D^a_- f)_p + dt Q_s(f_p, f_p), ghosts on every face cell the
    boundary row (boundary function on the incoming half; the outgoing half
    multiplies a zero velocity part)."""
    g = [face_boundary_rows(prob, k, F[prob.face_cells(k)]) for k in range(4)]
    og = np.array([obstacle_boundary_row(prob, k, F[p]) for (p, k) in prob.obstacle_faces()])
    Q, _ = evaluate_pairs(F, [(p, p) for p in range(F.shape[0])], prob)
    Fn = F + dt * Q
    for a in range(2):
        va = prob.vel(a)
        Fn = Fn - dt * (np.maximum(va, 0.0) * d_plus_2d(F, g, prob, a, og if len(og) else None)
                        + np.minimum(va, 0.0) * d_minus_2d(F, g, prob, a, og if len(og) else None))
    Fn = Fn * (~prob.solid_mask()).astype(np.float64)[:, None]   # solid cells hold no gas
    err = math.sqrt(prob.wx * prob.dvd * float(((Fn - F) ** 2).sum()))
    return Fn, err


def macroscopic(st: State, prob: Problem1D):
    """rho, u_1, T per cell (gas constant 1): E = rho|u|^2/2 + d rho T / 2."""
    vs = prob.vs
    C = oc.moment_matrix(vs)                              # (d+2, n)
    m = (st.X @ st.S) @ (st.V @ C.T)                      # (nx, d+2)
    rho = m[:, 0]
    u = m[:, 1:1 + vs.d] / rho[:, None]
    E = 0.5 * m[:, -1]
    T = (2.0 * E / rho - (u ** 2).sum(axis=1)) / vs.d
    return rho, u[:, 0], T
