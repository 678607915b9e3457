"""Pins of the oracle's obstacle (solid cells inside the rectangle, Maxwell
diffusive walls on their faces; oracle/dlr.py Problem2D.solid / obstacle).

* A solid last column is the rectangle one column shorter with a diffusive
  wall of the obstacle's Maxwellian at x_hi: the full-tensor step, the
  factored K-S-L step and the boundary rows' span agree (the shorter domain's
  wall is pinned elsewhere).  This checks the +x faces, the ghosts' incoming
  and outgoing halves and rho_w; the same with a solid first row checks -y.
* A closed box with an interior obstacle conserves the total mass (every
  wall face carries zero net flux).
* Mirror symmetry: a box, obstacle and state symmetric under y -> -y (cells
  iy <-> ny - 1 - iy, v_2 -> -v_2 on the periodic grid) stay symmetric after
  a full-tensor step and a factored step (1e-8, without the moment
  projection; the grid node v_2 = -L is its own mirror image); a swapped -y / +y face would break it.
* Solid cells hold no gas after a step.
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


def _field(spec, nx, ny, seed=3, rank=3, pert=5e-2, sym=False):
    rng = np.random.default_rng(seed)
    F = np.empty((nx * ny, spec.npts))
    for ix in range(nx):
        for iy in range(ny):
            yy = min(iy, ny - 1 - iy) if sym else iy
            T = 1.0 + 0.2 * ix / max(1, nx - 1) + 0.1 * yy / max(1, ny - 1)
            u = (0.3 * math.sin(ix + 0.5 * yy), 0.0 if sym else 0.2 * math.cos(iy - ix))
            F[ix * ny + iy] = _maxw(spec, 1.0 + 0.05 * ((ix * 7 + yy * 3) % 5), u, T)
    if sym:
        return F
    B = rng.standard_normal((rank, spec.npts)) * _maxw(spec, 1.0, (0.0, 0.0), 1.0)
    A = rng.standard_normal((nx * ny, rank))
    return F + pert * F.max() * (A @ B) / np.abs(A @ B).max()


def _prob(spec, nx, ny, faces, solid=None, obstacle=None, x_hi=1.0, y_lo=0.0, conserve=True):
    return dlr.Problem2D(vs=oc.setup_from_spec(spec), nx=nx, ny=ny, x_lo=0.0, x_hi=x_hi,
                         y_lo=y_lo, y_hi=0.8, faces=faces, solid=solid, obstacle=obstacle,
                         conserve=conserve)


def _state(F, wx, dvd, r):
    return dlr.initial_state(F, r, wx, dvd)


def _faces(spec):
    return [(_maxw(spec, 1.0, (0.4, 0.0), 1.0), False), (_maxw(spec, 1.0, (0.0, 0.0), 1.3), True),
            (_maxw(spec, 1.0, (0.2, 0.0), 1.0), True), (_maxw(spec, 0.9, (0.1, -0.2), 1.1), False)]


def test_solid_last_column_is_a_wall_at_x_hi():
    spec = _spec()
    nx, ny = 5, 4
    Mobs = _maxw(spec, 1.0, (0.0, 0.0), 1.6)
    faces = _faces(spec)
    solid = np.zeros((nx, ny), dtype=bool)
    solid[-1, :] = True
    A = _prob(spec, nx, ny, faces, solid=solid, obstacle=Mobs, x_hi=1.0)
    B = _prob(spec, nx - 1, ny, [faces[0], (Mobs, True), faces[2], faces[3]], x_hi=0.8)
    assert abs(A.dx - B.dx) < 1e-15 and len(A.obstacle_faces()) == ny
    FB = _field(spec, nx - 1, ny, seed=4)
    FA = np.vstack([FB, np.zeros((ny, spec.npts))])
    # full tensor
    FAn, eA = dlr.full_step(FA, A, 0.004)
    FBn, eB = dlr.full_step(FB, B, 0.004)
    assert np.abs(FAn[:-ny] - FBn).max() < 1e-14 * np.abs(FBn).max()
    assert np.all(FAn[-ny:] == 0.0)
    assert abs(eA - eB) < 1e-12 * eB
    # factored step from the same factors (zero X rows in the solid column)
    sB = _state(FB, B.wx, B.dvd, 4)
    sA = dlr.State(np.vstack([sB.X, np.zeros((ny, 4))]), sB.S, sB.V)
    nA, errA, _ = dlr.ksl_step(sA, A, 0.004)
    nB, errB, _ = dlr.ksl_step(sB, B, 0.004)
    fA, fB = nA.full(), nB.full()
    assert np.abs(fA[:-ny] - fB).max() < 1e-12 * np.abs(fB).max()
    assert np.abs(fA[-ny:]).max() < 1e-13 * np.abs(fB).max()
    assert abs(errA - errB) < 1e-10 * errB
    # boundary rows: the same row space (A's solid x_hi face cells give zero rows)
    RA = dlr.boundary_matrix_2d(sA, A)
    RB = dlr.boundary_matrix_2d(sB, B)
    sa = np.linalg.svd(RA, compute_uv=False)
    sb = np.linalg.svd(RB, compute_uv=False)
    assert np.abs(sa[:len(sb)] - sb).max() < 1e-12 * sb[0]
    assert np.all(sa[len(sb):] < 1e-12 * sb[0])


def test_solid_first_row_is_a_wall_at_y_lo():
    spec = _spec()
    nx, ny = 4, 5
    Mobs = _maxw(spec, 1.0, (0.0, 0.0), 0.8)
    faces = _faces(spec)
    solid = np.zeros((nx, ny), dtype=bool)
    solid[:, 0] = True
    A = _prob(spec, nx, ny, faces, solid=solid, obstacle=Mobs, y_lo=-0.2)
    B = _prob(spec, nx, ny - 1, [faces[0], faces[1], (Mobs, True), faces[3]])
    assert abs(A.dy - B.dy) < 1e-15
    FB = _field(spec, nx, ny - 1, seed=5)
    FA = np.zeros((nx * ny, spec.npts))
    for ix in range(nx):
        FA[ix * ny + 1: ix * ny + ny] = FB[ix * (ny - 1): (ix + 1) * (ny - 1)]
    gas = ~solid.reshape(-1)
    FAn, eA = dlr.full_step(FA, A, 0.004)
    FBn, eB = dlr.full_step(FB, B, 0.004)
    assert np.abs(FAn[gas] - FBn).max() < 1e-14 * np.abs(FBn).max()
    assert abs(eA - eB) < 1e-12 * eB
    sB = _state(FB, B.wx, B.dvd, 4)
    XA = np.zeros((nx * ny, 4))
    XA[gas] = sB.X
    nA, errA, _ = dlr.ksl_step(dlr.State(XA, sB.S, sB.V), A, 0.004)
    nB, errB, _ = dlr.ksl_step(sB, B, 0.004)
    assert np.abs(nA.full()[gas] - nB.full()).max() < 1e-12 * np.abs(nB.full()).max()
    assert abs(errA - errB) < 1e-10 * errB


def _closed_box(spec, nx, ny):
    faces = [(_maxw(spec, 1.0, (0.0, 0.0), 1.0), True), (_maxw(spec, 1.0, (0.0, 0.0), 1.2), True),
             (_maxw(spec, 1.0, (0.0, 0.0), 1.0), True), (_maxw(spec, 1.0, (0.5, 0.0), 1.0), True)]
    solid = np.zeros((nx, ny), dtype=bool)
    solid[2:4, 2:3] = True
    return _prob(spec, nx, ny, faces, solid=solid, obstacle=_maxw(spec, 1.0, (0.0, 0.0), 2.0))


def test_closed_box_with_an_obstacle_conserves_mass():
    spec = _spec()
    nx, ny = 6, 5
    prob = _closed_box(spec, nx, ny)
    assert len(prob.obstacle_faces()) == 6
    F = _field(spec, nx, ny, seed=9) * (~prob.solid_mask())[:, None]
    C = oc.moment_matrix(prob.vs)
    m0 = prob.wx * F.sum(axis=0) @ C.T
    for _ in range(4):
        F, _ = dlr.full_step(F, prob, 0.004)
    m1 = prob.wx * F.sum(axis=0) @ C.T
    assert abs(m1[0] - m0[0]) < 1e-14 * m0[0]
    # the obstacle exchanges heat: the energy changes
    assert abs(m1[-1] - m0[-1]) > 1e-8 * m0[-1]
    assert np.all(F[prob.solid_mask()] == 0.0)


def _mirror(F, spec, nx, ny):
    """Cells iy -> ny - 1 - iy and velocities v_2 -> -v_2."""
    N = spec.n
    G = F.reshape(nx, ny, N, N)[:, ::-1, :, :]
    # grid v_q = -L + q dv: v_2 -> -v_2 maps index q2 to N - q2 (q2 = 0 has no mirror
    # on the grid; these fields vanish there to rounding), so roll after the flip
    G = np.roll(G[:, :, :, ::-1], 1, axis=3)
    return G.reshape(nx * ny, N * N)


def test_mirror_symmetry_is_kept():
    spec = _spec(N=8)
    nx, ny = 5, 6
    M = lambda T: _maxw(spec, 1.0, (0.0, 0.0), T)
    faces = [(_maxw(spec, 1.0, (0.3, 0.0), 1.0), False), (M(1.2), True), (M(1.1), True),
             (M(1.1), True)]
    solid = np.zeros((nx, ny), dtype=bool)
    solid[2, 2:4] = True                         # symmetric about the middle of y
    # without the moment projection: its v_2 row takes -L at the node q_2 = 0,
    # which the periodic mirror maps to itself, so the projection is not
    # mirror-equivariant on the grid (the operator itself is, to 1e-15)
    prob = _prob(spec, nx, ny, faces, solid=solid, obstacle=M(1.7), conserve=False)
    F = _field(spec, nx, ny, sym=True) * (~prob.solid_mask())[:, None]
    assert np.abs(_mirror(F, spec, nx, ny) - F).max() < 1e-12 * np.abs(F).max()
    # 1e-8: the node v_2 = -L maps to itself, on the incoming half of a +y
    # face and the outgoing half of its mirror -y face; the wall Maxwellian's
    # value there (exp(-L^2 / 2 T_w) ~ 7e-9) is what is left unmatched
    Fn, _ = dlr.full_step(F, prob, 0.004)
    assert np.abs(_mirror(Fn, spec, nx, ny) - Fn).max() < 1e-8 * np.abs(Fn).max()
    st = _state(F, prob.wx, prob.dvd, 5)
    new, _, _ = dlr.ksl_step(st, prob, 0.004)
    f = new.full()
    assert np.abs(_mirror(f, spec, nx, ny) - f).max() < 1e-8 * np.abs(f).max()
