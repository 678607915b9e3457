"""GPU parity of blr_dlr_step / blr_steady_solve against the oracle's step.

Factors are unique only up to rotations, so the comparison is on the
reconstructed f = X S V, the residual err, err_ada and the rank decisions.
FP64 collisions: f to 1e-12 relative.  FP32 collisions: each pair collision
carries an error below 1e-5 ||Q+|| (the collision tolerance), which enters
the step linearly through dt Q, so the bound is
||f_gpu - f_ref|| <= 1e-5 dt ||sum_mn K_m K_n Q+(V_m, V_n)||.
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


def _setup(d, N, nx, r, m_rho, mach=1.5, pert=1e-2, pert_rank=3):
    if d == 2:
        spec = synth.VGridSpec(d=2, n=N, L=8.0, gamma=0.0, C=1 / (2 * math.pi), m_rho=m_rho, m_sigma=8)
    else:
        spec = synth.VGridSpec(d=3, n=N, L=8.0, gamma=1.0, C=1.0, m_rho=m_rho, m_sigma=38)
    vs = oc.setup_from_spec(spec)
    ini = synth.shock_initial(mach, spec, nx, -30.0, 30.0, pert=pert, pert_rank=pert_rank, seed=3)
    prob = dlr.Problem1D(vs=vs, nx=nx, x_lo=-30.0, x_hi=30.0, fL=ini["fL"], fR=ini["fR"])
    X, S, V = synth.lowrank_state(ini["f0"], r, prob.dx, prob.dvd)
    return spec, prob, dlr.State(X, S, V), ini


def _wall_setup(d, N, nx, r, m_rho, walls=(True, True)):
    """Gas between Maxwell diffusive walls at rest (T_w = 1 at x = 0, 1.2 at
    x = 2; a side without a wall takes that Maxwellian as inflow)."""
    if d == 2:
        spec = synth.VGridSpec(d=2, n=N, L=8.0, gamma=0.0, C=1 / (2 * math.pi), m_rho=m_rho, m_sigma=8)
    else:
        spec = synth.VGridSpec(d=3, n=N, L=8.0, gamma=1.0, C=1.0, m_rho=m_rho, m_sigma=38)
    vs = oc.setup_from_spec(spec)
    ini = synth.wall_initial(spec, nx, 0.0, 2.0, T_walls=(1.0, 1.2), pert=5e-2, pert_rank=3, seed=4)
    prob = dlr.Problem1D(vs=vs, nx=nx, x_lo=0.0, x_hi=2.0, fL=ini["fL"], fR=ini["fR"],
                         wall_left=walls[0], wall_right=walls[1])
    X, S, V = synth.lowrank_state(ini["f0"], r, prob.dx, prob.dvd)
    return spec, prob, dlr.State(X, S, V), ini


class Gpu:
    def __init__(self, ctx, spec, prob, st, r_cap, flags=0):
        dev = "cuda"
        self.ctx = ctx
        self.nx, self.n = prob.nx, prob.vs.n
        self.X = torch.zeros((r_cap, self.nx), dtype=torch.float64, device=dev)
        self.S = torch.zeros((r_cap, r_cap), dtype=torch.float64, device=dev)
        self.V = torch.zeros((r_cap, self.n), dtype=torch.float64, device=dev)
        r = st.r
        self.X[:r] = torch.tensor(st.X.T, device=dev)
        self.S[:r, :r] = torch.tensor(st.S, device=dev)
        self.V[:r] = torch.tensor(st.V, device=dev)
        self.fL = torch.tensor(prob.fL, device=dev)
        self.fR = torch.tensor(prob.fR, device=dev)
        self.vg = blr.vgrid_from_spec(spec, flags)
        self.pb = ctx.make_problem(self.vg, prob.nx, prob.x_lo, prob.x_hi, self.fL, self.fR,
                                   wall_left=prob.wall_left, wall_right=prob.wall_right)
        self.st = ctx.make_state(self.X, self.S, self.V, r, seed=11)

    def full(self):
        r = self.st.r
        X = self.X[:r].double().cpu().numpy().T
        S = self.S[:r, :r].double().cpu().numpy()
        V = self.V[:r].double().cpu().numpy()
        return X @ S @ V

    def factors(self):
        r = self.st.r
        return (self.X[:r].cpu().numpy(), self.S[:r, :r].cpu().numpy(), self.V[:r].cpu().numpy())


def _params(dt, flags, r_max=30, r_min=1):
    return blr.StepParams(dt, 0.2, 1e-10, r_min, r_max, flags)


@pytest.mark.parametrize("d,N,nx,r,m_rho", [(2, 16, 24, 4, 8), (3, 8, 16, 3, 4), (3, 16, 40, 5, 2),
                                             (2, 16, 40, 17, 4), (2, 16, 300, 16, 4),
                                             (2, 16, 300, 40, 2)])
def test_fixed_rank_step_fp64(ctx, d, N, nx, r, m_rho):
    """r = 16 takes the widest fused x-side and Cholesky QR kernels, r = 17 the
    general ones (Householder QR, separate x-side kernels); nx = 300 spans
    two cell blocks; r = 40 takes the 64-column Householder tree (blocks of
    128 rows)."""
    print(f"fixed-rank d={d} N={N} nx={nx} r={r}", flush=True)
    spec, prob, st, _ = _setup(d, N, nx, r, m_rho)
    if r > 8:
        # the smooth state has singular values down to rounding at this rank:
        # lift them so that the comparison is well conditioned
        st = dlr.State(st.X, st.S + 1e-3 * np.abs(st.S).max() * np.eye(r), st.V)
    g = Gpu(ctx, spec, prob, st, r_cap=max(8, r))
    info = ctx.dlr_step(g.pb, g.st, _params(0.05, blr.BLR_STEP_FP64_COLLISION))
    new, err, _ = dlr.ksl_step(st, prob, 0.05)
    f_ref = new.full()
    f_gpu = g.full()
    e = np.abs(f_gpu - f_ref).max() / np.abs(f_ref).max()
    print("f rel err", e, "err", info.err, err, flush=True)
    assert e < 1e-12
    assert abs(info.err - err) < 1e-10 * err
    assert info.r_out == r and g.st.r == r
    X, S, V = g.factors()
    assert np.abs(prob.dx * X @ X.T - np.eye(r)).max() < 1e-12
    assert np.abs(prob.dvd * V @ V.T - np.eye(r)).max() < 1e-12


@pytest.mark.parametrize("d,N,nx,r,m_rho", [(2, 16, 24, 4, 8), (3, 16, 40, 5, 2)])
def test_fixed_rank_step_fp32_collisions(ctx, d, N, nx, r, m_rho):
    spec, prob, st, _ = _setup(d, N, nx, r, m_rho)
    g = Gpu(ctx, spec, prob, st, r_cap=8)
    dt = 0.05
    info = ctx.dlr_step(g.pb, g.st, _params(dt, 0))
    new, err, _ = dlr.ksl_step(st, prob, dt)
    pairs = dlr.pair_list(r)
    wts = np.array([1.0 if m == n else 2.0 for (m, n) in pairs])
    _, gains = oc.q_pairs(st.V, pairs, prob.vs, conserve=True)
    gain_scale = np.linalg.norm(dlr.pair_products(st.X @ st.S, pairs, wts) @ gains)
    e = np.linalg.norm(g.full() - new.full()) / (dt * gain_scale)
    print("fp32 step error / (dt ||gain||)", e, flush=True)
    assert e < 1e-5
    assert abs(info.err - err) < 1e-3 * err


@pytest.mark.parametrize("d,N,nx,r,m_rho", [(2, 16, 24, 3, 8), (3, 16, 40, 4, 2)])
def test_adaptive_steps_fp64(ctx, d, N, nx, r, m_rho):
    print(f"adaptive d={d} N={N}", flush=True)
    spec, prob, st, _ = _setup(d, N, nx, r, m_rho)
    g = Gpu(ctx, spec, prob, st, r_cap=12)
    flags = blr.BLR_STEP_FP64_COLLISION | blr.BLR_STEP_ADD | blr.BLR_STEP_DROP
    cur = st
    for k in range(3):
        info = ctx.dlr_step(g.pb, g.st, _params(0.05, flags, r_max=12))
        cur, oinfo = dlr.adaptive_step(cur, prob, 0.05, c=0.2, r_max=12,
                                       rng=np.random.default_rng(k))
        print(k, "r", info.r_added, info.r_out, oinfo.r_added, oinfo.r_out, "err", info.err, oinfo.err,
              "ada", info.err_ada, oinfo.err_ada, flush=True)
        assert info.r_added == oinfo.r_added and info.r_out == oinfo.r_out
        assert abs(info.err - oinfo.err) < 1e-9 * oinfo.err
        assert abs(info.err_ada - oinfo.err_ada) < 1e-9 * oinfo.err_ada
        f_ref = cur.full()
        _check_adaptive_fp64(g.full(), f_ref)
        # the bound of Sec. 5.1 holds on the GPU too
        bound = math.sqrt(max(info.r_in + info.r_added - info.r_out, 0)) * info.drop_tol
        assert abs(info.err - info.err_ada) <= bound * (1 + 1e-12) + 1e-15


@pytest.mark.parametrize("d,N,nx,r,m_rho", [(2, 16, 24, 4, 8), (3, 16, 40, 5, 2), (2, 16, 40, 17, 4)])
def test_fixed_rank_step_with_walls_fp64(ctx, d, N, nx, r, m_rho):
    """Maxwell diffusive walls on both sides: the ghosts of every substep
    carry rho_w from the adjacent cell (r = 17 takes the general kernels)."""
    print(f"walls fixed-rank d={d} N={N} nx={nx} r={r}", flush=True)
    spec, prob, st, _ = _wall_setup(d, N, nx, r, m_rho)
    if r > 8:
        st = dlr.State(st.X, st.S + 1e-3 * np.abs(st.S).max() * np.eye(r), st.V)
    g = Gpu(ctx, spec, prob, st, r_cap=max(8, r))
    dt = 0.005
    info = ctx.dlr_step(g.pb, g.st, _params(dt, blr.BLR_STEP_FP64_COLLISION))
    new, err, _ = dlr.ksl_step(st, prob, dt)
    f_ref = new.full()
    e = np.abs(g.full() - f_ref).max() / np.abs(f_ref).max()
    print("f rel err", e, "err", info.err, err, flush=True)
    assert e < 1e-12
    assert abs(info.err - err) < 1e-10 * err


@pytest.mark.parametrize("walls", [(True, True), (True, False), (False, True)])
@pytest.mark.parametrize("d,N,nx,r,m_rho", [(2, 16, 24, 3, 8), (3, 16, 40, 4, 2)])
def test_adaptive_steps_with_walls_fp64(ctx, d, N, nx, r, m_rho, walls):
    """The boundary rows of the basis augmentation carry rho_w M_w on a
    wall's incoming half: the added functions, ranks and err_ada follow the
    oracle step by step."""
    print(f"walls adaptive d={d} N={N} walls={walls}", flush=True)
    spec, prob, st, _ = _wall_setup(d, N, nx, r, m_rho, walls)
    g = Gpu(ctx, spec, prob, st, r_cap=12)
    flags = blr.BLR_STEP_FP64_COLLISION | blr.BLR_STEP_ADD | blr.BLR_STEP_DROP
    cur = st
    dt = 0.005
    for k in range(3):
        info = ctx.dlr_step(g.pb, g.st, _params(dt, flags, r_max=12))
        cur, oinfo = dlr.adaptive_step(cur, prob, dt, c=0.2, r_max=12,
                                       rng=np.random.default_rng(k))
        print(k, "r", info.r_added, info.r_out, oinfo.r_added, oinfo.r_out, "err", info.err, oinfo.err,
              "ada", info.err_ada, oinfo.err_ada, flush=True)
        assert info.r_added == oinfo.r_added and info.r_out == oinfo.r_out
        assert abs(info.err - oinfo.err) < 1e-9 * oinfo.err
        assert abs(info.err_ada - oinfo.err_ada) < 1e-9 * oinfo.err_ada
        f_ref = cur.full()
        _check_adaptive_fp64(g.full(), f_ref)


def test_wall_flags_are_checked(ctx):
    spec, prob, st, _ = _wall_setup(2, 16, 24, 3, 8)
    g = Gpu(ctx, spec, prob, st, r_cap=8)
    g.pb.wall_left = 2
    before = g.full()
    with pytest.raises(blr.BlrError) as ei:
        ctx.dlr_step(g.pb, g.st, _params(0.005, blr.BLR_STEP_FP64_COLLISION))
    assert ei.value.code == blr.BLR_ERR_ARG
    assert np.array_equal(g.full(), before)


@pytest.mark.parametrize("d,N,nx,r,m_rho", [(3, 16, 40, 4, 2)])
def test_add_projection_matches_householder(ctx, d, N, nx, r, m_rho):
    """The two ways of orthogonalising the added boundary functions give the
    same step (only the span of [V; V_b] enters the K, S and L steps)."""
    spec, prob, st, _ = _setup(d, N, nx, r, m_rho)
    out = []
    for extra in (0, blr.BLR_STEP_HOUSEHOLDER_ADD):
        g = Gpu(ctx, spec, prob, st, r_cap=12)
        flags = blr.BLR_STEP_FP64_COLLISION | blr.BLR_STEP_ADD | blr.BLR_STEP_DROP | extra
        infos = [ctx.dlr_step(g.pb, g.st, _params(0.05, flags, r_max=12)) for _ in range(2)]
        X, S, V = g.factors()
        assert np.abs(prob.dvd * V @ V.T - np.eye(g.st.r)).max() < 1e-12
        out.append((g.full(), [(i.r_added, i.r_out, i.err, i.err_ada) for i in infos]))
    (fa, ia), (fb, ib) = out
    assert np.abs(fa - fb).max() < 1e-12 * np.abs(fb).max()
    for a, b in zip(ia, ib):
        assert a[:2] == b[:2]
        assert abs(a[2] - b[2]) < 1e-10 * b[2] and abs(a[3] - b[3]) < 1e-10 * b[3]


@pytest.mark.parametrize("d,N,nx,r,m_rho", [(3, 16, 40, 5, 2), (2, 16, 300, 4, 4),
                                            (2, 16, 600, 4, 4)])
def test_cholesky_qr_matches_householder(ctx, d, N, nx, r, m_rho):
    """K- and L-step QRs by shifted Cholesky QR (default) and by Householder
    QR give the same adaptive steps.  Up to 512 rows the three passes run in
    one workgroup (nx = 40: one row per thread, 300: two); nx = 600 and the
    4096-row V side take the multi-block passes."""
    spec, prob, st, _ = _setup(d, N, nx, r, m_rho)
    out = []
    for extra in (0, blr.BLR_STEP_HOUSEHOLDER_QR):
        g = Gpu(ctx, spec, prob, st, r_cap=12)
        flags = blr.BLR_STEP_FP64_COLLISION | blr.BLR_STEP_ADD | blr.BLR_STEP_DROP | extra
        infos = [ctx.dlr_step(g.pb, g.st, _params(0.05, flags, r_max=12)) for _ in range(2)]
        X, S, V = g.factors()
        rr = g.st.r
        assert np.abs(prob.dx * X @ X.T - np.eye(rr)).max() < 1e-12
        assert np.abs(prob.dvd * V @ V.T - np.eye(rr)).max() < 1e-12
        out.append((g.full(), [(i.r_added, i.r_out, i.err, i.err_ada) for i in infos]))
    (fa, ia), (fb, ib) = out
    assert np.abs(fa - fb).max() < 1e-12 * np.abs(fb).max()
    for a, b in zip(ia, ib):
        assert a[:2] == b[:2]
        assert abs(a[2] - b[2]) < 1e-10 * b[2] and abs(a[3] - b[3]) < 1e-10 * b[3]


def test_add_count_change_is_redone(ctx):
    """The step guesses the number of added boundary functions from the
    previous step and redoes itself when the singular values disagree: a
    step with add_tol so large that nothing is added (guess 2), then one
    whose rank cap leaves room for one function (guess 0).  Both match the
    oracle."""
    spec, prob, st, _ = _setup(2, 16, 24, 3, 8)
    g = Gpu(ctx, spec, prob, st, r_cap=12)
    flags = blr.BLR_STEP_FP64_COLLISION | blr.BLR_STEP_ADD | blr.BLR_STEP_DROP
    cur = st
    plan = [(1e-10, 12), (1e10, 12), (1e-10, None)]
    for k, (add_tol, r_max) in enumerate(plan):
        r_max = r_max or g.st.r + 1
        info = ctx.dlr_step(g.pb, g.st, blr.StepParams(0.05, 0.2, add_tol, 1, r_max, flags))
        cur, oinfo = dlr.adaptive_step(cur, prob, 0.05, c=0.2, add_tol=add_tol, r_max=r_max,
                                       rng=np.random.default_rng(k))
        print(k, info.r_added, oinfo.r_added, info.r_out, oinfo.r_out, flush=True)
        assert info.r_added == oinfo.r_added == [2, 0, 1][k]
        assert info.r_out == oinfo.r_out
        assert abs(info.err - oinfo.err) < 1e-9 * oinfo.err
        assert abs(info.err_ada - oinfo.err_ada) < 1e-9 * oinfo.err_ada
        f_ref = cur.full()
        _check_adaptive_fp64(g.full(), f_ref)


def test_graph_replay_matches_eager(ctx):
    """Steps recorded as graphs and replayed give the same results as steps
    issued kernel by kernel: two copies of one state advanced side by side,
    the eager one in between the replays, compared after every step."""
    spec, prob, st, _ = _setup(2, 16, 24, 3, 8)   # rank 3 -> +2 -> 3 every step
    ga = Gpu(ctx, spec, prob, st, r_cap=12)
    ge = Gpu(ctx, spec, prob, st, r_cap=12)
    base = blr.BLR_STEP_ADD | blr.BLR_STEP_DROP
    replays = 0
    for k in range(7):
        ia = ctx.dlr_step(ga.pb, ga.st, _params(0.01, base, r_max=12))
        ie = ctx.dlr_step(ge.pb, ge.st, _params(0.01, base | blr.BLR_STEP_EAGER, r_max=12))
        torch.cuda.synchronize()
        replays += ia.ms_collision == 0.0
        assert ie.ms_collision > 0.0
        assert (ia.r_added, ia.r_out) == (ie.r_added, ie.r_out)
        assert ia.err == ie.err and ia.err_ada == ie.err_ada
        assert np.array_equal(ga.full(), ge.full())
    print("replayed steps:", replays, flush=True)
    assert replays >= 4


def test_steady_solve_runs_and_reports(ctx):
    spec, prob, st, _ = _setup(2, 16, 24, 3, 4)
    g = Gpu(ctx, spec, prob, st, r_cap=12)
    flags = blr.BLR_STEP_FP64_COLLISION | blr.BLR_STEP_ADD | blr.BLR_STEP_DROP
    sp = blr.SolveParams(_params(0.05, flags, r_max=12), 1e-30, 4)
    info = ctx.steady_solve(g.pb, g.st, sp, allow_unconverged=True)
    assert info.steps == 4 and info.converged == 0 and info.r == g.st.r
    ref = st
    for k in range(4):
        ref, oi = dlr.adaptive_step(ref, prob, 0.05, c=0.2, r_max=12, rng=np.random.default_rng(k))
    rho_g, u_g, T_g = dlr.macroscopic(dlr.State(*[np.asarray(a) for a in (
        g.factors()[0].T, g.factors()[1], g.factors()[2])]), prob)
    rho_o, u_o, T_o = dlr.macroscopic(ref, prob)
    for a, b in ((rho_g, rho_o), (u_g, u_o), (T_g, T_o)):
        assert np.abs(a - b).max() <= 1e-6 * np.abs(b).max()
    # converged immediately with a loose tolerance
    sp2 = blr.SolveParams(_params(0.05, flags, r_max=12), 1e10, 5)
    info2 = ctx.steady_solve(g.pb, g.st, sp2)
    assert info2.converged == 1 and info2.steps == 1


def test_step_errors_leave_state_untouched(ctx):
    spec, prob, st, _ = _setup(2, 16, 24, 3, 4)
    g = Gpu(ctx, spec, prob, st, r_cap=8)
    before = g.full()
    with pytest.raises(blr.BlrError) as ei:
        ctx.dlr_step(g.pb, g.st, _params(-1.0, 0))
    assert ei.value.code == 1
    bad = ctx.make_state(g.X, g.S, g.V, 9)   # r > r_cap
    with pytest.raises(blr.BlrError):
        ctx.dlr_step(g.pb, bad, _params(0.05, 0))
    assert np.array_equal(g.full(), before)
