"""Pins of the oracle's boundary rows F_b (Sec. 3.1, the rows f^b(x_b, .) whose
right singular vectors augment the basis; the boundary function of Sec. 2.3,
eq. boundary general) and of the augmentation's span on the rectangle.

The expected rows are written here from the definition, cell by cell and
velocity node by velocity node, on the reconstructed grid f = X S V:

* the incoming half (v.n < 0, n the face's outward normal) is the prescribed
  boundary function, or at a Maxwell diffusive wall the wall Maxwellian scaled
  so that the assembled row carries no net mass flux through the face;
* the outgoing half (v.n >= 0) is the distribution of the adjacent interior
  cell.

The velocity components come from the grid's definition (v_q = -L + q dv,
C order, axis 0 along x and axis 1 along y), not from the oracle's helpers.
A swapped inflow half, a wrong adjacent cell, a wrong face order or a wall
density with the wrong sign or normal fails one of these tests.
"""
import math

import numpy as np
import pytest

import synth
from oracle import collision as oc
from oracle import dlr


def _vcomp(d, N, L, axis):
    """Velocity component `axis` of every grid node (flat, C order)."""
    dv = 2.0 * L / N
    q = np.arange(N ** d)
    digit = (q // N ** (d - 1 - axis)) % N
    return -L + dv * digit


def _maxw(d, N, L, rho, u, T):
    return synth.maxwellian(synth.vgrid_points(d, N, L), rho, u, T).reshape(-1)


def _row_from_definition(vn, f_adj, M, wall):
    """One boundary row, node by node: vn = v.n at every node."""
    if wall:
        out_flux = sum(vn[q] * f_adj[q] for q in range(len(vn)) if vn[q] >= 0)
        in_flux_shape = sum(vn[q] * M[q] for q in range(len(vn)) if vn[q] < 0)
        rho_w = -out_flux / in_flux_shape
    row = np.empty(len(vn))
    for q in range(len(vn)):
        if vn[q] < 0:
            row[q] = rho_w * M[q] if wall else M[q]
        else:
            row[q] = f_adj[q]
    return row


# ------------------------------------------------------------------ 1D space
def _problem_1d(d, N, wall_left, wall_right, nx=12):
    L = 8.0
    if d == 2:
        spec = synth.VGridSpec(d=2, n=N, L=L, gamma=0.0, C=1 / (2 * math.pi), m_rho=4, m_sigma=8)
    else:
        spec = synth.VGridSpec(d=3, n=N, L=L, gamma=1.0, C=1.0, m_rho=4, m_sigma=38)
    vs = oc.setup_from_spec(spec)
    ini = synth.shock_initial(1.5, spec, nx, -30.0, 30.0, pert=5e-2, pert_rank=3, seed=5)
    # wall shapes: any positive multiple of the wall Maxwellian (here not normalised)
    fL = 3.0 * _maxw(d, N, L, 1.0, (0.0,) * d, 1.3) if wall_left else ini["fL"]
    fR = 0.5 * _maxw(d, N, L, 1.0, (0.0,) * d, 0.8) if wall_right else ini["fR"]
    prob = dlr.Problem1D(vs=vs, nx=nx, x_lo=-30.0, x_hi=30.0, fL=fL, fR=fR,
                         wall_left=wall_left, wall_right=wall_right)
    X, S, V = synth.lowrank_state(ini["f0"], 4, prob.dx, prob.dvd)
    return prob, dlr.State(X, S, V), spec


@pytest.mark.parametrize("d,N", [(2, 16), (3, 8)])
@pytest.mark.parametrize("wall_left,wall_right", [(False, False), (True, True),
                                                   (False, True), (True, False)])
def test_boundary_matrix_1d_from_definition(d, N, wall_left, wall_right):
    prob, st, spec = _problem_1d(d, N, wall_left, wall_right)
    F = st.X @ st.S @ st.V                      # f on the (cell, v) grid
    v1 = _vcomp(d, N, spec.L, 0)
    # left face x_lo: outward normal -e1, adjacent cell 0
    left = _row_from_definition(-v1, F[0], prob.fL, wall_left)
    # right face x_hi: outward normal +e1, adjacent cell nx-1
    right = _row_from_definition(v1, F[prob.nx - 1], prob.fR, wall_right)
    Fb = dlr.boundary_matrix(st, prob)
    assert Fb.shape == (2, N ** d)
    scale = np.abs(F).max()
    assert np.abs(Fb[0] - left).max() <= 1e-14 * scale
    assert np.abs(Fb[1] - right).max() <= 1e-14 * scale
    # physical checks of the assembled rows
    for row, vn, wall in ((Fb[0], -v1, wall_left), (Fb[1], v1, wall_right)):
        if wall:
            # no net mass flux through a diffusive wall
            assert abs(np.dot(vn, row)) <= 1e-13 * np.dot(np.abs(vn), np.abs(row))
    if wall_left:
        # the wall's incoming half (v1 > 0) differs visibly from the adjacent
        # cell's (so a row taken whole from the cell would fail above)
        inc = v1 > 0
        assert np.abs(Fb[0][inc] - F[0][inc]).max() > 1e-3 * scale


def test_boundary_matrix_1d_inflow_halves_are_the_prescribed_maxwellians():
    """Inflow faces: the row equals f_L exactly where v1 > 0 at the left face,
    f_R exactly where v1 < 0 at the right face, and never the other way round."""
    prob, st, spec = _problem_1d(2, 16, False, False)
    v1 = _vcomp(2, 16, spec.L, 0)
    Fb = dlr.boundary_matrix(st, prob)
    assert np.array_equal(Fb[0][v1 > 0], prob.fL[v1 > 0])
    assert np.array_equal(Fb[1][v1 < 0], prob.fR[v1 < 0])
    F = st.full()
    tol = 1e-15 * np.abs(F).max()
    assert np.abs(Fb[0][v1 <= 0] - F[0][v1 <= 0]).max() <= tol
    assert np.abs(Fb[1][v1 >= 0] - F[-1][v1 >= 0]).max() <= tol


# ------------------------------------------------------------ the rectangle
def _problem_2d(d, N, nx, ny, seed=3):
    L = 8.0
    if d == 2:
        spec = synth.VGridSpec(d=2, n=N, L=L, gamma=0.0, C=1 / (2 * math.pi), m_rho=4, m_sigma=8)
    else:
        spec = synth.VGridSpec(d=3, n=N, L=L, gamma=1.0, C=1.0, m_rho=4, m_sigma=38)
    z = (0.0,) * (d - 2)
    # x_lo inflow (one row for the face), x_hi wall, y_lo moving wall, y_hi
    # inflow with one row per face cell
    top = np.array([_maxw(d, N, L, 0.9, (0.1, -0.2) + z, 1.0 + 0.05 * i) for i in range(nx)])
    faces = [(_maxw(d, N, L, 1.0, (0.4, 0.0) + z, 1.0), False),
             (2.0 * _maxw(d, N, L, 1.0, (0.0, 0.0) + z, 1.2), True),
             (_maxw(d, N, L, 1.0, (0.3, 0.0) + z, 1.0), True),
             (top, False)]
    prob = dlr.Problem2D(vs=oc.setup_from_spec(spec), nx=nx, ny=ny, x_lo=0.0, x_hi=1.0,
                         y_lo=0.0, y_hi=0.8, faces=faces)
    rng = np.random.default_rng(seed)
    F0 = np.empty((nx * ny, N ** d))
    for ix in range(nx):
        for iy in range(ny):
            T = 1.0 + 0.2 * ix / max(1, nx - 1) + 0.1 * iy / max(1, ny - 1)
            u = (0.3 * math.sin(ix + 0.5 * iy), 0.2 * math.cos(iy - ix)) + z
            F0[ix * ny + iy] = _maxw(d, N, L, 1.0 + 0.1 * rng.standard_normal() ** 2, u, T)
    return prob, F0, spec


def _rect_rows_from_definition(prob, F, spec):
    """Every face's rows written out with loops: faces in the order x_lo, x_hi,
    y_lo, y_hi; along a face its cells in increasing order of the other
    coordinate; cell (ix, iy) is row ix*ny + iy of F."""
    d, N, L = spec.d, spec.n, spec.L
    v1, v2 = _vcomp(d, N, L, 0), _vcomp(d, N, L, 1)
    nx, ny = prob.nx, prob.ny
    geo = [
        (-v1, [(0, iy) for iy in range(ny)]),          # x_lo: normal -e1
        (v1, [(nx - 1, iy) for iy in range(ny)]),      # x_hi: normal +e1
        (-v2, [(ix, 0) for ix in range(nx)]),          # y_lo: normal -e2
        (v2, [(ix, ny - 1) for ix in range(nx)]),      # y_hi: normal +e2
    ]
    rows = []
    for k, (vn, cells) in enumerate(geo):
        fk, wall = prob.faces[k]
        fk = np.asarray(fk)
        for c, (ix, iy) in enumerate(cells):
            M = fk[c] if fk.ndim == 2 else fk
            rows.append(_row_from_definition(vn, F[ix * ny + iy], M, wall))
    return np.array(rows)


@pytest.mark.parametrize("d,N,nx,ny", [(2, 8, 4, 3), (2, 16, 3, 5), (3, 8, 3, 4)])
def test_boundary_matrix_2d_from_definition(d, N, nx, ny):
    prob, F0, spec = _problem_2d(d, N, nx, ny)
    X, S, V = synth.lowrank_state(F0, 3, prob.wx, prob.dvd)
    st = dlr.State(X, S, V)
    F = st.full()
    Fb = dlr.boundary_matrix_2d(st, prob)
    want = _rect_rows_from_definition(prob, F, spec)
    assert Fb.shape == want.shape == (2 * (nx + ny), N ** d)
    assert np.abs(Fb - want).max() <= 1e-14 * np.abs(F).max()
    # corner cell (0, 0) appears twice: once on x_lo (incoming v1 > 0) and once
    # on y_lo (incoming v2 > 0), each with its own face's incoming half
    v1, v2 = _vcomp(d, N, spec.L, 0), _vcomp(d, N, spec.L, 1)
    r_xlo, r_ylo = Fb[0], Fb[2 * ny]
    out_both = (v1 <= 0) & (v2 <= 0)
    tol = 1e-15 * np.abs(F).max()
    assert np.abs(r_xlo[out_both] - F[0][out_both]).max() <= tol
    assert np.abs(r_ylo[out_both] - F[0][out_both]).max() <= tol
    assert np.array_equal(r_xlo[v1 > 0], np.asarray(prob.faces[0][0])[v1 > 0])
    # wall faces carry no net mass flux through their face, per cell
    for k, (lo, hi), vn in ((1, (ny, 2 * ny), v1), (2, (2 * ny, 2 * ny + nx), -v2)):
        for row in Fb[lo:hi]:
            assert abs(np.dot(vn, row)) <= 1e-13 * np.dot(np.abs(vn), np.abs(row))


def _span_projector(B, w):
    """Orthogonal projector (in the weighted inner product w * sum) onto the
    row span of B, from an SVD."""
    U, s, Vt = np.linalg.svd(B, full_matrices=False)
    k = int((s > 1e-9 * s[0]).sum())
    return Vt[:k].T @ Vt[:k], k


def test_rectangle_augmentation_spans_the_papers_directions():
    """Sec. 3.1 appends the right singular vectors of F_b (singular values
    above 10^-10) to V and orthonormalises.  On the rectangle the oracle takes
    them from F_b projected onto the complement of span V.  When the cap
    r_max does not bind the two give the same space, span(V) + rowspace(F_b),
    and the same number of added functions; f is unchanged."""
    prob, F0, spec = _problem_2d(2, 8, 6, 5, seed=7)
    r = 3
    X, S, V = synth.lowrank_state(F0, r, prob.wx, prob.dvd)
    st = dlr.State(X, S, V)
    Fb = dlr.boundary_matrix_2d(st, prob)
    n_rows = Fb.shape[0]                    # 22 rows (numerical rank 16), 30 cells
    aug, rb = dlr.add_boundary_basis(st, prob, 1e-10, r_max=r + n_rows + 5,
                                     rng=np.random.default_rng(0))
    # the paper's construction, written out: SVD of F_b itself
    _, sb, Qbt = np.linalg.svd(Fb, full_matrices=False)
    rb_paper = int((sb > 1e-10).sum())
    Vp = np.vstack([V, Qbt[:rb_paper]])
    assert rb == rb_paper and 0 < rb <= n_rows
    assert aug.r == r + rb
    P_aug, k_aug = _span_projector(aug.V, prob.dvd)
    P_pap, k_pap = _span_projector(Vp, prob.dvd)
    P_def, k_def = _span_projector(np.vstack([V, Fb]), prob.dvd)
    assert k_aug == k_pap == k_def == r + rb
    assert np.abs(P_aug - P_def).max() < 1e-10
    assert np.abs(P_pap - P_def).max() < 1e-10
    # every boundary row lies in the new span
    res = Fb - prob.dvd * (Fb @ aug.V.T) @ aug.V
    assert np.abs(res).max() < 1e-11 * np.abs(Fb).max()
    assert np.abs(aug.full() - st.full()).max() < 1e-13 * np.abs(st.full()).max()
