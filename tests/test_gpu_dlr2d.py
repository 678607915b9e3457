"""GPU parity of the low-rank step in two-dimensional space (a rectangle with
inflow and Maxwell diffusive wall faces, boundary functions varying along a
face) against the oracle's step on the rectangle (oracle/dlr.py, pinned by
tests/test_oracle_dlr2d.py).

FP64 collisions: f = X S V on the grid to 1e-12 of max |f| and err to 1e-10
relative, step by step; with the adaptivity (boundary rows of every face
cell added, the rank decision on S) the added counts and ranks are
identical, err and err_ada to 1e-9, f to 1e-12 of ||f|| (L2) and 1e-11 of
max |f| (see _check_adaptive_fp64).  FP32 collisions: ||f_gpu - f_ref|| <=
1e-5 dt ||sum K_m K_n Q+_mn|| (the pair operator's bound, as in one
dimension).
"""
import math

import numpy as np
import pytest

import synth
from oracle import collision as oc
from oracle import dlr

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2112_02695_amd as blr  # noqa: E402


def _check_adaptive_fp64(f_gpu, f_ref):
    """An adaptive FP64 step is held to 1e-12 of ||f|| in the L2 norm and to
    1e-11 of max |f| pointwise.  The pointwise bound is looser because the
    directions the basis augmentation adds are the boundary rows' parts
    outside span V, which can be small (at the benchmark state 2e-6 and
    5e-7 of the rows), so rounding fixes them only to about eps over that
    size; two equivalent FP64 orthogonalisations of the oracle's own then
    give steps 6e-12 apart in max |f|, in the tails of the velocity box, and
    3.6e-13 apart in L2."""
    d = f_gpu - f_ref
    l2 = np.linalg.norm(d) / np.linalg.norm(f_ref)
    mx = np.abs(d).max() / np.abs(f_ref).max()
    print(f"  f: L2 rel {l2:.2e}, max rel {mx:.2e}", flush=True)
    assert l2 < 1e-12
    assert mx < 1e-11


@pytest.fixture(scope="module")
def ctx():
    c = blr.Context(0)
    yield c
    c.close()


def _spec(d, N, m_rho):
    if d == 2:
        return synth.VGridSpec(d=2, n=N, L=8.0, gamma=0.0, C=1 / (2 * math.pi), m_rho=m_rho,
                               m_sigma=8)
    return synth.VGridSpec(d=3, n=N, L=8.0, gamma=1.0, C=1.0, m_rho=m_rho, m_sigma=38)


def _maxw(spec, rho, u, T):
    v = synth.vgrid_points(spec.d, spec.n, spec.L)
    return synth.maxwellian(v, rho, tuple(u) + (0.0,) * (spec.d - 2), T).reshape(-1)


def _setup(d, N, m_rho, nx, ny, r, seed=3):
    """x_lo inflow, x_hi wall (T 1.2), y_lo wall moving along x, y_hi inflow
    with one row per face cell."""
    spec = _spec(d, N, m_rho)
    top = np.array([_maxw(spec, 0.9, (0.1, -0.2), 1.0 + 0.05 * i) for i in range(nx)])
    faces = [(_maxw(spec, 1.0, (0.4, 0.0), 1.0), False), (_maxw(spec, 1.0, (0.0, 0.0), 1.2), True),
             (_maxw(spec, 1.0, (0.3, 0.0), 1.0), True), (top, False)]
    prob = dlr.Problem2D(vs=oc.setup_from_spec(spec), nx=nx, ny=ny, x_lo=0.0, x_hi=1.0,
                         y_lo=0.0, y_hi=0.8, faces=faces)
    F0 = synth.rect_field(spec, nx, ny, seed=seed)
    X, S, V = synth.lowrank_state(F0, r, prob.wx, prob.dvd)
    return spec, prob, dlr.State(X, S, V)


class Gpu:
    def __init__(self, ctx, spec, prob, st, r_cap):
        dev = "cuda"
        nc = prob.nx * prob.ny
        self.X = torch.zeros((r_cap, nc), dtype=torch.float64, device=dev)
        self.S = torch.zeros((r_cap, r_cap), dtype=torch.float64, device=dev)
        self.V = torch.zeros((r_cap, prob.vs.n), dtype=torch.float64, device=dev)
        r = st.r
        self.X[:r] = torch.tensor(st.X.T, device=dev)
        self.S[:r, :r] = torch.tensor(st.S, device=dev)
        self.V[:r] = torch.tensor(st.V, device=dev)
        faces = [(torch.tensor(np.ascontiguousarray(f), device=dev), w) for f, w in prob.faces]
        self.pb = ctx.make_problem2d(blr.vgrid_from_spec(spec), prob.nx, prob.ny, prob.x_lo,
                                     prob.x_hi, prob.y_lo, prob.y_hi, faces)
        self.st = ctx.make_state(self.X, self.S, self.V, r)

    def full(self):
        r = self.st.r
        return (self.X[:r].cpu().numpy().T @ self.S[:r, :r].cpu().numpy()) @ self.V[:r].cpu().numpy()


@pytest.mark.parametrize("d,N,m_rho,nx,ny,r", [(2, 16, 8, 5, 4, 4), (3, 8, 4, 4, 3, 3),
                                               (2, 16, 4, 6, 5, 7), (2, 16, 4, 1, 6, 3)])
def test_fixed_rank_steps_fp64(ctx, d, N, m_rho, nx, ny, r):
    print(f"2D-space step d={d} N={N} {nx}x{ny} r={r}", flush=True)
    spec, prob, st = _setup(d, N, m_rho, nx, ny, r)
    g = Gpu(ctx, spec, prob, st, r_cap=8)
    dt = 0.004
    cur = st
    for k in range(3):
        info = ctx.dlr_step(g.pb, g.st, blr.StepParams(dt, 0.2, 1e-10, 1, 8,
                                                       blr.BLR_STEP_FP64_COLLISION))
        cur, err, _ = dlr.ksl_step(cur, prob, dt)
        f_ref = cur.full()
        e = np.abs(g.full() - f_ref).max() / np.abs(f_ref).max()
        print(k, "f rel err", e, "err", info.err, err, flush=True)
        assert e < 1e-12
        assert abs(info.err - err) < 1e-10 * err
        assert info.r_out == r


def test_fixed_rank_step_fp32_collisions(ctx):
    spec, prob, st = _setup(2, 16, 8, 5, 4, 4)
    g = Gpu(ctx, spec, prob, st, r_cap=8)
    dt = 0.004
    info = ctx.dlr_step(g.pb, g.st, blr.StepParams(dt, 0.2, 1e-10, 1, 8, 0))
    new, err, _ = dlr.ksl_step(st, prob, dt)
    pairs = dlr.pair_list(st.r)
    wts = np.array([1.0 if m == n else 2.0 for (m, n) in pairs])
    _, gains = oc.q_pairs(st.V, pairs, prob.vs, conserve=True)
    gain_scale = np.linalg.norm(dlr.pair_products(st.X @ st.S, pairs, wts) @ gains)
    e = np.linalg.norm(g.full() - new.full()) / (dt * gain_scale)
    print("fp32 step error / (dt ||gain||)", e, flush=True)
    assert e < 1e-5
    assert abs(info.err - err) < 1e-3 * err


def test_steady_solve_runs_steps_on_the_rectangle(ctx):
    spec, prob, st = _setup(2, 16, 4, 4, 4, 3, seed=5)
    g = Gpu(ctx, spec, prob, st, r_cap=8)
    dt = 0.004
    sp = blr.SolveParams(blr.StepParams(dt, 0.2, 1e-10, 1, 8, blr.BLR_STEP_FP64_COLLISION),
                         1e-30, 4)
    info = ctx.steady_solve(g.pb, g.st, sp, allow_unconverged=True)
    cur = st
    for _ in range(4):
        cur, err, _ = dlr.ksl_step(cur, prob, dt)
    f_ref = cur.full()
    assert info.steps == 4
    assert np.abs(g.full() - f_ref).max() < 1e-12 * np.abs(f_ref).max()
    assert abs(info.err_ada - err) < 1e-10 * err


@pytest.mark.parametrize("d,N,m_rho,nx,ny,r", [(2, 16, 8, 4, 3, 3), (3, 8, 4, 3, 3, 2),
                                               (2, 16, 4, 5, 4, 4)])
def test_adaptive_steps_fp64(ctx, d, N, m_rho, nx, ny, r):
    """Add (one boundary row per face cell) and drop on the rectangle: the
    added counts, ranks, err and err_ada follow the oracle step by step."""
    print(f"2D-space adaptive d={d} N={N} {nx}x{ny} r={r}", flush=True)
    spec, prob, st = _setup(d, N, m_rho, nx, ny, r, seed=9)
    g = Gpu(ctx, spec, prob, st, r_cap=16)
    dt = 0.004
    flags = blr.BLR_STEP_FP64_COLLISION | blr.BLR_STEP_ADD | blr.BLR_STEP_DROP
    r_max = min(16, nx * ny)          # the rank never exceeds the cell count
    cur = st
    for k in range(3):
        info = ctx.dlr_step(g.pb, g.st, blr.StepParams(dt, 0.2, 1e-10, 1, r_max, flags))
        cur, oinfo = dlr.adaptive_step(cur, prob, dt, c=0.2, r_max=r_max,
                                       rng=np.random.default_rng(k))
        print(k, "r", info.r_added, info.r_out, oinfo.r_added, oinfo.r_out, "err", info.err,
              oinfo.err, "ada", info.err_ada, oinfo.err_ada, flush=True)
        assert info.r_added == oinfo.r_added and info.r_out == oinfo.r_out
        assert abs(info.err - oinfo.err) < 1e-9 * oinfo.err
        assert abs(info.err_ada - oinfo.err_ada) < 1e-9 * oinfo.err_ada
        f_ref = cur.full()
        _check_adaptive_fp64(g.full(), f_ref)


def test_augmentation_limit_is_refused(ctx):
    """2 (nx + ny) > 64 face cells: the augmentation is refused before any
    work, the state untouched."""
    spec, prob, st = _setup(2, 16, 4, 20, 13, 2)
    g = Gpu(ctx, spec, prob, st, r_cap=8)
    before = g.full()
    with pytest.raises(blr.BlrError) as ei:
        ctx.dlr_step(g.pb, g.st, blr.StepParams(0.004, 0.2, 1e-10, 1, 8, blr.BLR_STEP_ADD))
    assert ei.value.code == blr.BLR_ERR_UNSUPPORTED
    assert np.array_equal(g.full(), before)


def test_served_2d_solve_equals_the_direct_solve(ctx):
    """A steady solve on the rectangle through the server (its own slot
    context and stream) gives bitwise the factors of the same solve run
    directly."""
    spec, prob, st = _setup(2, 16, 4, 4, 4, 3, seed=6)
    sp = blr.SolveParams(blr.StepParams(0.004, 0.2, 1e-10, 1, 8, blr.BLR_STEP_FP64_COLLISION),
                         1e-30, 5)
    a = Gpu(ctx, spec, prob, st, r_cap=8)
    ia = ctx.steady_solve(a.pb, a.st, sp, allow_unconverged=True)
    b = Gpu(ctx, spec, prob, st, r_cap=8)
    torch.cuda.synchronize()
    sv = blr.Server(0, slots=1)
    try:
        sv.submit(b.pb, b.st, sp, 1)
        comps = []
        while not comps:
            got = sv.wait(timeout=120.0)
            assert got, "no progress"
            comps += got
    finally:
        sv.close()
    c = comps[0]
    assert c.status in (blr.BLR_OK, blr.BLR_ERR_NOT_CONVERGED), c.message
    assert c.info.steps == ia.steps == 5
    assert torch.equal(a.X, b.X) and torch.equal(a.S, b.S) and torch.equal(a.V, b.V)


def test_adaptive_step_at_the_rank_cap_fp64(ctx):
    """The regime of the lid-driven cavity's err_ada rise: rank 52 on 16 x 16
    cells, all four walls diffusive with a moving lid, so the 64 boundary rows
    (projected onto V^perp) offer far more directions than the room r_max - r
    = 8.  One adaptive step with FP64 collisions against the oracle's: the
    cap binds on both sides, ranks and counts identical, f, err and err_ada
    to the adaptive bounds.  The input is a seeded rank-52 state of a
    Maxwellian field plus smooth perturbations (16^2 velocity)."""
    spec = _spec(2, 16, 4)
    nx = ny = 16
    wall = _maxw(spec, 1.0, (0.0, 0.0), 1.0)
    lid = _maxw(spec, 1.0, (1.0, 0.0), 1.0)
    faces = [(wall, True), (wall, True), (wall, True), (lid, True)]
    prob = dlr.Problem2D(vs=oc.setup_from_spec(spec), nx=nx, ny=ny, x_lo=0.0, x_hi=0.5,
                         y_lo=0.0, y_hi=0.5, faces=faces)
    F0 = synth.rect_field(spec, nx, ny, seed=11, rank=60, pert=0.2)
    st = dlr.initial_state(F0, 52, prob.wx, prob.dvd)
    g = Gpu(ctx, spec, prob, st, r_cap=64)
    flags = blr.BLR_STEP_FP64_COLLISION | blr.BLR_STEP_ADD | blr.BLR_STEP_DROP
    info = ctx.dlr_step(g.pb, g.st, blr.StepParams(0.004, 0.2, 1e-10, 1, 60, flags))
    new, oinfo = dlr.adaptive_step(st, prob, 0.004, c=0.2, r_max=60)
    print("r", info.r_added, info.r_out, oinfo.r_added, oinfo.r_out, "err", info.err, oinfo.err,
          "ada", info.err_ada, oinfo.err_ada, flush=True)
    assert oinfo.r_added == 8 and info.r_added == 8
    assert info.r_out == oinfo.r_out
    assert abs(info.err - oinfo.err) < 1e-9 * oinfo.err
    assert abs(info.err_ada - oinfo.err_ada) < 1e-9 * oinfo.err_ada
    _check_adaptive_fp64(g.full(), new.full())
