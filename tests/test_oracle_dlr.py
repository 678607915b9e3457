"""Pins of the oracle's low-rank step (Sec. 2.4), residual (Sec. 5.1) and
basis add / drop (Sec. 3).

The factored K -> S -> L algebra is checked against a *full-tensor* route
that reconstructs f on the (x, v) grid and applies the three projected
subflows (eqs. K-step general, S-step general, L-step general) with explicit
orthogonal projectors P_V (onto span V, acting on v) and P_X (onto span X,
acting on x), the upwind operator of eq. (scheme:fullupwind) with ghost rows
P_V f^b (eq. boundary general; at a Maxwell diffusive wall the inflow half is
the wall Maxwellian scaled so that the assembled row carries no net mass
flux), and Q(f(x), f(x)) evaluated cell by cell.
It shares none of the factored formulas (A^+-, pair weights, tensors T, QR).
"""
import math

import numpy as np
import pytest

import synth
from oracle import collision as oc
from oracle import dlr


def _problem(d=2, N=16, nx=24, mach=1.5, conserve=True, m_rho=8):
    if d == 2:
        spec = synth.VGridSpec(d=2, n=N, L=8.0, gamma=0.0, C=1 / (2 * math.pi), m_rho=m_rho, m_sigma=8)
    else:
        spec = synth.VGridSpec(d=3, n=N, L=8.0, gamma=1.0, C=1.0, m_rho=m_rho, m_sigma=38)
    vs = oc.setup_from_spec(spec)
    ini = synth.shock_initial(mach, spec, nx, -30.0, 30.0, pert=1e-2, pert_rank=3, seed=3)
    prob = dlr.Problem1D(vs=vs, nx=nx, x_lo=-30.0, x_hi=30.0, fL=ini["fL"], fR=ini["fR"],
                         conserve=conserve)
    return prob, ini


def _wall_problem(d=2, N=16, nx=24, conserve=True, m_rho=8):
    """Gas between two Maxwell diffusive walls at rest (T_w = 1 and 1.2), the
    geometry of the Fourier flow, with a rank-3 perturbation."""
    if d == 2:
        spec = synth.VGridSpec(d=2, n=N, L=8.0, gamma=0.0, C=1 / (2 * math.pi), m_rho=m_rho, m_sigma=8)
    else:
        spec = synth.VGridSpec(d=3, n=N, L=8.0, gamma=1.0, C=1.0, m_rho=m_rho, m_sigma=38)
    vs = oc.setup_from_spec(spec)
    ini = synth.wall_initial(spec, nx, 0.0, 2.0, T_walls=(1.0, 1.2), pert=5e-2, pert_rank=3, seed=4)
    prob = dlr.Problem1D(vs=vs, nx=nx, x_lo=0.0, x_hi=2.0, fL=ini["fL"], fR=ini["fR"],
                         conserve=conserve, wall_left=True, wall_right=True)
    return prob, ini


def _state(prob, ini, r):
    X, S, V = synth.lowrank_state(ini["f0"], r, prob.dx, prob.dvd)
    return dlr.State(X, S, V)


# ---------------------------------------------------------------- full tensor
def _PV(g, V, dvd):
    return dvd * (g @ V.T) @ V


def _PX(g, X, dx):
    return dx * X @ (X.T @ g)


def _ghost_rows(f, V, prob):
    v1 = prob.v1()

    def row(side, f_adj):
        M = prob.fL if side == 0 else prob.fR
        inflow = v1 > 0 if side == 0 else v1 < 0
        if prob.wall_left if side == 0 else prob.wall_right:
            # the density that makes the net mass flux of the assembled row zero
            M = M * (-np.sum(v1[~inflow] * f_adj[~inflow]) / np.sum(v1[inflow] * M[inflow]))
        return np.where(inflow, M, f_adj)

    fbL, fbR = row(0, f[0]), row(1, f[-1])
    return _PV(fbL[None, :], V, prob.dvd)[0], _PV(fbR[None, :], V, prob.dvd)[0]


def _transport(f, gL, gR, prob):
    v1 = prob.v1()
    vp, vm = np.maximum(v1, 0), np.minimum(v1, 0)
    Dp = (f - np.vstack([gL[None], f[:-1]])) / prob.dx
    Dm = (np.vstack([f[1:], gR[None]]) - f) / prob.dx
    return -vp[None, :] * Dp - vm[None, :] * Dm


def _Qrows(f, prob):
    out = np.empty_like(f)
    for p in range(f.shape[0]):
        q = oc.q_fft(f[p], f[p], prob.vs).reshape(-1)
        out[p] = oc.conserve_project(q, prob.vs) if prob.conserve else q
    return out


def _full_tensor_step(st, prob, dt):
    V, dx, dvd = st.V, prob.dx, prob.dvd
    f = st.full()
    # K-step: d/dt f = P_V RHS
    gL, gR = _ghost_rows(f, V, prob)
    f1 = f + dt * _PV(_transport(f, gL, gR, prob) + _Qrows(f, prob), V, dvd)
    # new X = orthonormal basis of the column space of f1 (x side)
    U, s, _ = np.linalg.svd(math.sqrt(dx * dvd) * f1, full_matrices=False)
    X1 = U[:, :st.r] / math.sqrt(dx)
    # S-step: d/dt f = - P_X P_V RHS
    gL, gR = _ghost_rows(f1, V, prob)
    f2 = f1 - dt * _PX(_PV(_transport(f1, gL, gR, prob) + _Qrows(f1, prob), V, dvd), X1, dx)
    # L-step: d/dt f = P_X RHS
    gL, gR = _ghost_rows(f2, V, prob)
    f3 = f2 + dt * _PX(_transport(f2, gL, gR, prob) + _Qrows(f2, prob), X1, dx)
    return f3


@pytest.mark.parametrize("walls", [False, True])
@pytest.mark.parametrize("conserve", [True, False])
def test_factored_step_matches_full_tensor_projections(conserve, walls):
    prob, ini = _wall_problem(conserve=conserve) if walls else _problem(conserve=conserve)
    st = _state(prob, ini, 4)
    dt = 0.01 if walls else 0.05
    new, err, pieces = dlr.ksl_step(st, prob, dt)
    f3 = _full_tensor_step(st, prob, dt)
    scale = np.abs(f3).max()
    assert np.abs(new.full() - f3).max() < 1e-12 * scale
    # orthonormality of the new factors
    assert np.abs(prob.dx * new.X.T @ new.X - np.eye(4)).max() < 1e-13
    assert np.abs(prob.dvd * new.V @ new.V.T - np.eye(4)).max() < 1e-13
    # residual from the pieces == brute-force weighted norm of f^{n+1} - f^n
    brute = math.sqrt(prob.dx * prob.dvd * ((f3 - st.full()) ** 2).sum())
    assert abs(err - brute) < 1e-10 * brute


def test_step_independent_of_factor_gauge():
    prob, ini = _problem()
    st = _state(prob, ini, 4)
    rng = np.random.default_rng(0)
    O, _ = np.linalg.qr(rng.standard_normal((4, 4)))
    P, _ = np.linalg.qr(rng.standard_normal((4, 4)))
    st2 = dlr.State(st.X @ O, O.T @ st.S @ P, P.T @ st.V)
    a, ea, _ = dlr.ksl_step(st, prob, 0.05)
    b, eb, _ = dlr.ksl_step(st2, prob, 0.05)
    assert np.abs(a.full() - b.full()).max() < 1e-12 * np.abs(a.full()).max()
    assert abs(ea - eb) < 1e-10 * ea


def test_add_keeps_f_and_drop_identity():
    prob, ini = _problem()
    st = _state(prob, ini, 3)
    f = st.full()
    st_a, rb = dlr.add_boundary_basis(st, prob, rng=np.random.default_rng(1))
    assert rb == 2
    assert st_a.r == 5
    assert np.abs(st_a.full() - f).max() < 1e-13 * np.abs(f).max()
    assert np.abs(prob.dvd * st_a.V @ st_a.V.T - np.eye(5)).max() < 1e-12
    assert np.abs(prob.dx * st_a.X.T @ st_a.X - np.eye(5)).max() < 1e-12
    # the boundary rows now lie in span V
    Fb = dlr.boundary_matrix(st, prob)
    proj = prob.dvd * (Fb @ st_a.V.T) @ st_a.V
    assert np.abs(proj - Fb).max() < 1e-12 * np.abs(Fb).max()
    # drop: |f - fbar| = |Sigma_perp|_F
    s = np.linalg.svd(st_a.S, compute_uv=False)
    tol = 0.5 * (s[1] + s[2])
    out, sv, keep, _, _ = dlr.drop_basis(st_a, tol)
    assert keep == 2
    gap = math.sqrt(prob.dx * prob.dvd * ((out.full() - st_a.full()) ** 2).sum())
    assert abs(gap - math.sqrt((sv[keep:] ** 2).sum())) < 1e-12 * max(gap, 1e-300) + 1e-15


def test_add_step_result_independent_of_random_block():
    prob, ini = _problem()
    st = _state(prob, ini, 3)
    a, ia = dlr.adaptive_step(st, prob, 0.05, rng=np.random.default_rng(1), drop=False)
    b, ib = dlr.adaptive_step(st, prob, 0.05, rng=np.random.default_rng(2), drop=False)
    assert np.abs(a.full() - b.full()).max() < 1e-12 * np.abs(a.full()).max()
    assert abs(ia.err - ib.err) < 1e-10 * ia.err


def test_err_ada_exact_and_bound():
    prob, ini = _problem()
    st = _state(prob, ini, 4)
    for _ in range(3):
        f_before = st.full()
        st2, info = dlr.adaptive_step(st, prob, 0.05, c=0.2, rng=np.random.default_rng(3))
        brute = math.sqrt(prob.dx * prob.dvd * ((st2.full() - f_before) ** 2).sum())
        assert abs(info.err_ada - brute) < 1e-9 * brute
        r_before = info.r_in + info.r_added
        bound = math.sqrt(max(r_before - info.r_out, 0)) * info.drop_tol
        assert abs(info.err - info.err_ada) <= bound * (1 + 1e-12) + 1e-15
        assert info.sigma_dropped <= bound * (1 + 1e-12) + 1e-15
        st = st2


def test_free_stream_uniform_state_is_transport_free():
    """A uniform Maxwellian with the same inflow on both walls: ghost = interior,
    so D_+- K = 0 and, with the collision term switched off, f does not move."""
    prob, ini = _problem()
    vs = prob.vs
    M = synth.maxwellian(synth.vgrid_points(vs.d, vs.N, vs.L), 1.0, (0.5, 0.0), 1.0).reshape(-1)
    prob.fL = M
    prob.fR = M
    f0 = np.tile(M, (prob.nx, 1))
    X, S, V = synth.lowrank_state(f0, 1, prob.dx, prob.dvd)
    st = dlr.State(X, S, V)
    K = st.X @ st.S
    gl, gr = dlr.ghosts(K, st.V, prob)
    assert np.abs(gl - K[0]).max() < 1e-13 * np.abs(K).max()
    assert np.abs(gr - K[-1]).max() < 1e-13 * np.abs(K).max()
    prob.collision = lambda V, pairs, vs, conserve: (np.zeros((len(pairs), vs.n)),) * 2
    new, err, _ = dlr.ksl_step(st, prob, 0.05)
    assert err < 1e-13 * math.sqrt(prob.dx * prob.dvd * (f0 ** 2).sum())


def test_macroscopic_from_factors_matches_inputs():
    prob, ini = _problem()
    X, S, V = synth.lowrank_state(ini["f0"], 8, prob.dx, prob.dvd)
    st = dlr.State(X, S, V)
    rho, u, T = dlr.macroscopic(st, prob)
    (rl, ul, Tl), (rr, ur, Tr) = ini["states"]
    assert abs(rho[0] - rl) < 2e-2 and abs(rho[-1] - rr) < 2e-2
    assert abs(u[0] - ul) < 5e-2 and abs(T[0] - Tl) < 5e-2


# -------------------------------------------------------- initial truncation
def test_initial_state_is_the_best_rank_r_approximation():
    """Sec. 2.4's initial truncated SVD: orthonormal factors in the weighted
    inner products, and the truncation error in the L2(x, v) norm equals the
    root sum of squares of the dropped singular values (Eckart-Young); an
    input of exact rank r is reproduced."""
    prob, ini = _problem()
    F0 = ini["f0"]
    w = prob.dx * prob.dvd
    sv = np.linalg.svd(math.sqrt(w) * F0, compute_uv=False)
    for r in (1, 4, 9):
        st = dlr.initial_state(F0, r, prob.dx, prob.dvd)
        assert np.abs(prob.dx * st.X.T @ st.X - np.eye(r)).max() < 1e-13
        assert np.abs(prob.dvd * st.V @ st.V.T - np.eye(r)).max() < 1e-13
        gap = math.sqrt(w * ((F0 - st.full()) ** 2).sum())
        tail = math.sqrt((sv[r:] ** 2).sum())
        assert abs(gap - tail) <= 1e-10 * tail + 1e-15 * sv[0]
        assert np.all(np.diff(np.diag(st.S)) <= 0)
    # exact rank 3: product of seeded factors
    rng = np.random.default_rng(5)
    F3 = rng.standard_normal((prob.nx, 3)) @ rng.standard_normal((3, F0.shape[1]))
    st = dlr.initial_state(F3, 3, prob.dx, prob.dvd)
    assert np.abs(st.full() - F3).max() < 1e-13 * np.abs(F3).max()
