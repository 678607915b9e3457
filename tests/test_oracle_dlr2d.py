"""Pins of the oracle's two-dimensional physical space (Sec. 2.2: the upwind
scheme on a rectangular grid; Sec. 2.3: the boundary on every face).

* The factored low-rank step on the rectangle equals a full-tensor route
  written here with explicit loops over cells: f reconstructed on the
  (cell, v) grid, the three projected subflows (eqs. K-step, S-step, L-step
  general) with projectors P_V and P_X, both axes' upwind differences with
  ghost rows P_V f^b, the diffusive walls' rows scaled so that each row
  carries no net mass flux through its face.
* A state uniform in y whose y faces return the adjacent cells (boundary
  rows equal to those cells) has no y transport: every row of the 2D
  full-tensor step, and of the 2D low-rank K-step, equals the pinned 1D step.
  The x-uniform case against the 1D step along y (velocity axes exchanged,
  a symmetry of the grid and of the isotropic operator) pins the y axis.
* Four diffusive walls conserve the total mass to rounding.
"""
import math

import numpy as np
import pytest

import synth
from oracle import collision as oc
from oracle import dlr


def _spec(N=8, m_rho=4):
    return synth.VGridSpec(d=2, n=N, L=8.0, gamma=0.0, C=1 / (2 * math.pi), m_rho=m_rho,
                           m_sigma=8)


def _maxw(spec, rho, u, T):
    v = synth.vgrid_points(2, spec.n, spec.L)
    return synth.maxwellian(v, rho, u, T).reshape(-1)


def _field(spec, nx, ny, seed=3, rank=3, pert=5e-2):
    """Seeded smooth state on the rectangle: a Maxwellian with T and u varying
    in x and y plus a rank-`rank` perturbation."""
    rng = np.random.default_rng(seed)
    F = np.empty((nx * ny, spec.npts))
    for ix in range(nx):
        for iy in range(ny):
            T = 1.0 + 0.2 * ix / max(1, nx - 1) + 0.1 * iy / max(1, ny - 1)
            u = (0.3 * math.sin(ix + 0.5 * iy), 0.2 * math.cos(iy - ix))
            F[ix * ny + iy] = _maxw(spec, 1.0 + 0.1 * rng.standard_normal() ** 2, u, T)
    B = rng.standard_normal((rank, spec.npts)) * _maxw(spec, 1.0, (0.0, 0.0), 1.0)
    A = rng.standard_normal((nx * ny, rank))
    return F + pert * F.max() * (A @ B) / np.abs(A @ B).max()


def _problem(spec, nx, ny, faces, conserve=True):
    return dlr.Problem2D(vs=oc.setup_from_spec(spec), nx=nx, ny=ny, x_lo=0.0, x_hi=1.0, y_lo=0.0,
                         y_hi=0.8, faces=faces, conserve=conserve)


def _mixed_faces(spec, nx, ny):
    """x_lo inflow, x_hi wall (T 1.2), y_lo wall moving along x (T 1), y_hi
    inflow with a per-cell temperature."""
    top = np.array([_maxw(spec, 0.9, (0.1, -0.2), 1.0 + 0.05 * i) for i in range(nx)])
    return [(_maxw(spec, 1.0, (0.4, 0.0), 1.0), False),
            (_maxw(spec, 1.0, (0.0, 0.0), 1.2), True),
            (_maxw(spec, 1.0, (0.3, 0.0), 1.0), True),
            (top, False)]


# ------------------------------------------------------------ full-tensor route
def _bdy_row(prob, k, c, f_adj):
    """Boundary row of face k at its c-th cell, written out: incoming half the
    face function (a wall's scaled so that the row's net flux v.n vanishes),
    outgoing half the adjacent cell."""
    axis = 0 if k < 2 else 1
    sgn = -1.0 if k % 2 == 0 else 1.0
    vn = sgn * prob.vel(axis)
    fk, wall = prob.faces[k]
    M = np.asarray(fk)[c] if np.ndim(fk) == 2 else np.asarray(fk)
    inc = vn < 0
    if wall:
        M = M * (-np.sum(vn[~inc] * f_adj[~inc]) / np.sum(vn[inc] * M[inc]))
    return np.where(inc, M, f_adj)


def _transport_loops(f, V, prob, project):
    """-sum_a (v_a^+ D^a_+ + v_a^- D^a_-) f by loops over cells; ghost rows are
    the boundary rows, projected onto span V when `project`."""
    nx, ny = prob.nx, prob.ny
    out = np.zeros_like(f)
    v = [prob.vel(0), prob.vel(1)]
    P = (lambda g: prob.dvd * (g @ V.T) @ V) if project else (lambda g: g)
    for ix in range(nx):
        for iy in range(ny):
            p = ix * ny + iy
            for a, (h, i, m) in enumerate(((prob.dx, ix, nx), (prob.dy, iy, ny))):
                def nb(step):
                    j = i + step
                    if 0 <= j < m:
                        return f[(j * ny + iy) if a == 0 else (ix * ny + j)]
                    k = 2 * a + (1 if step > 0 else 0)
                    c = iy if a == 0 else ix
                    return P(_bdy_row(prob, k, c, f[p]))
                vp, vm = np.maximum(v[a], 0.0), np.minimum(v[a], 0.0)
                out[p] -= vp * (f[p] - nb(-1)) / h + vm * (nb(1) - f[p]) / h
    return out


def _Q(f, prob):
    out = np.empty_like(f)
    for p in range(f.shape[0]):
        q = oc.q_fft(f[p], f[p], prob.vs).reshape(-1)
        out[p] = oc.conserve_project(q, prob.vs) if prob.conserve else q
    return out


def _full_tensor_route(st, prob, dt):
    V, wx, dvd = st.V, prob.wx, prob.dvd
    PV = lambda g: dvd * (g @ V.T) @ V
    f = st.full()
    f1 = f + dt * PV(_transport_loops(f, V, prob, True) + _Q(f, prob))
    U, _, _ = np.linalg.svd(math.sqrt(wx * dvd) * f1, full_matrices=False)
    X1 = U[:, :st.r] / math.sqrt(wx)
    PX = lambda g: wx * X1 @ (X1.T @ g)
    f2 = f1 - dt * PX(PV(_transport_loops(f1, V, prob, True) + _Q(f1, prob)))
    return f2 + dt * PX(_transport_loops(f2, V, prob, True) + _Q(f2, prob))


@pytest.mark.parametrize("conserve", [True, False])
def test_factored_2d_step_matches_the_full_tensor_route(conserve):
    spec = _spec()
    nx, ny, r = 5, 4, 4
    prob = _problem(spec, nx, ny, _mixed_faces(spec, nx, ny), conserve)
    F0 = _field(spec, nx, ny)
    X, S, V = synth.lowrank_state(F0, r, prob.wx, prob.dvd)
    st = dlr.State(X, S, V)
    dt = 0.004
    new, err, _ = dlr.ksl_step(st, prob, dt)
    ref = _full_tensor_route(st, prob, dt)
    assert np.abs(new.full() - ref).max() < 1e-12 * np.abs(ref).max()
    brute = math.sqrt(prob.wx * prob.dvd * ((ref - st.full()) ** 2).sum())
    assert abs(err - brute) < 1e-10 * brute


def test_full_2d_step_matches_the_loops():
    spec = _spec()
    nx, ny = 4, 3
    prob = _problem(spec, nx, ny, _mixed_faces(spec, nx, ny))
    F = _field(spec, nx, ny, seed=8)
    dt = 0.004
    Fn, err = dlr.full_step(F, prob, dt)
    ref = F + dt * (_transport_loops(F, None, prob, False) + _Q(F, prob))
    assert np.abs(Fn - ref).max() < 1e-14 * np.abs(F).max()


# ------------------------------------------------------------ reductions to 1D
def _x_problem_1d(spec, nx, faces2d, conserve=True):
    return dlr.Problem1D(vs=oc.setup_from_spec(spec), nx=nx, x_lo=0.0, x_hi=1.0,
                         fL=faces2d[0][0], fR=faces2d[1][0], conserve=conserve,
                         wall_left=faces2d[0][1], wall_right=faces2d[1][1])


def test_state_uniform_in_y_steps_as_in_1d():
    spec = _spec()
    nx, ny = 6, 3
    row = _field(spec, nx, 1, seed=5)                        # (nx, n)
    F = np.repeat(row, ny, axis=0)                           # cell ix ny + iy
    xf = [(_maxw(spec, 1.0, (0.5, 0.1), 1.1), False), (_maxw(spec, 1.0, (0.0, 0.0), 1.3), True)]
    faces = xf + [(row, False), (row, False)]                # y faces return the adjacent cells
    prob = _problem(spec, nx, ny, faces)
    p1 = _x_problem_1d(spec, nx, xf)
    dt = 0.004
    Fn, _ = dlr.full_step(F, prob, dt)
    Fn1, _ = dlr.full_step(row, p1, dt)
    assert np.abs(Fn - np.repeat(Fn1, ny, axis=0)).max() < 1e-14 * np.abs(F).max()
    # the low-rank K-step: K = X S is the state itself, the y-face ghosts are
    # the adjacent cells' K and D_y K = 0 (later substeps move K away from
    # the fixed y-face rows, so only the K-step reduces to 1D)
    r = 3
    X1d, S1d, V1d = synth.lowrank_state(row, r, p1.dx, p1.dvd)
    c = math.sqrt(prob.dy * ny)                              # <X_i, X_j> over the rectangle
    st2 = dlr.State(np.repeat(X1d, ny, axis=0) / c, S1d * c, V1d)
    row_r = X1d @ S1d @ V1d                                  # the y faces return the rank-r cells
    prob_r = _problem(spec, nx, ny, xf + [(row_r, False), (row_r, False)])
    _, _, pc2 = dlr.ksl_step(st2, prob_r, dt)
    _, _, pc1 = dlr.ksl_step(dlr.State(X1d, S1d, V1d), p1, dt)
    K1 = np.repeat(pc1["K1"], ny, axis=0)
    assert np.abs(pc2["K1"] - K1).max() < 1e-13 * np.abs(K1).max()


def test_state_uniform_in_x_steps_as_in_1d_along_y():
    spec = _spec()
    nx, ny = 3, 6
    N = spec.n
    col = _field(spec, 1, ny, seed=6)                        # (ny, n) in (v1, v2) order
    F = np.tile(col, (nx, 1))                                # cell ix ny + iy
    yf = [(_maxw(spec, 1.0, (0.1, 0.5), 1.1), False), (_maxw(spec, 1.0, (0.0, 0.0), 1.3), True)]
    faces = [(col, False), (col, False)] + yf
    prob = dlr.Problem2D(vs=oc.setup_from_spec(spec), nx=nx, ny=ny, x_lo=0.0, x_hi=0.8,
                         y_lo=0.0, y_hi=1.0, faces=faces)
    T = lambda a: a.reshape(-1, N, N).transpose(0, 2, 1).reshape(a.shape)   # v1 <-> v2
    p1 = dlr.Problem1D(vs=oc.setup_from_spec(spec), nx=ny, x_lo=0.0, x_hi=1.0,
                       fL=T(yf[0][0][None])[0], fR=T(yf[1][0][None])[0], wall_left=False,
                       wall_right=True)
    dt = 0.004
    Fn, _ = dlr.full_step(F, prob, dt)
    Fn1, _ = dlr.full_step(T(col), p1, dt)
    ref = np.tile(T(Fn1), (nx, 1))
    assert np.abs(Fn - ref).max() < 1e-12 * np.abs(F).max()


def test_four_walls_conserve_mass():
    spec = _spec()
    nx, ny = 4, 4
    faces = [(_maxw(spec, 1.0, (0.0, 0.0), 1.0), True), (_maxw(spec, 1.0, (0.0, 0.0), 1.2), True),
             (_maxw(spec, 1.0, (0.0, 0.0), 1.0), True), (_maxw(spec, 1.0, (0.6, 0.0), 1.0), True)]
    prob = _problem(spec, nx, ny, faces)
    F = _field(spec, nx, ny, seed=9)
    C = oc.moment_matrix(prob.vs)
    m0 = prob.wx * F.sum(axis=0) @ C.T
    for _ in range(4):
        F, _ = dlr.full_step(F, prob, 0.004)
    m1 = prob.wx * F.sum(axis=0) @ C.T
    assert abs(m1[0] - m0[0]) < 1e-14 * m0[0]
    assert abs(m1[1] - m0[1]) > 1e-6          # the moving lid drags the gas along x


def test_adaptive_2d_step_runs_and_keeps_f():
    """The add stage on the rectangle (one boundary row per face cell) leaves
    f unchanged, and err_ada follows its definition."""
    spec = _spec()
    nx, ny, r = 4, 3, 2
    prob = _problem(spec, nx, ny, _mixed_faces(spec, nx, ny))
    F0 = _field(spec, nx, ny, seed=2)
    X, S, V = synth.lowrank_state(F0, r, prob.wx, prob.dvd)
    st = dlr.State(X, S, V)
    aug, rb = dlr.add_boundary_basis(st, prob, 1e-10, 12, np.random.default_rng(0))
    assert rb > 0 and aug.r == r + rb
    assert np.abs(aug.full() - st.full()).max() < 1e-13 * np.abs(st.full()).max()
    out, info = dlr.adaptive_step(st, prob, 0.004, c=0.2, r_max=12,
                                  rng=np.random.default_rng(0))
    new, err, _ = dlr.ksl_step(aug, prob, 0.004)
    brute = math.sqrt(prob.wx * prob.dvd * ((out.full() - st.full()) ** 2).sum())
    assert abs(info.err - err) < 1e-12 * err
    assert abs(info.err_ada - brute) < 1e-9 * brute
