"""GPU parity of blr_collision_pairs against the float64 oracle.

Error measure per pair: ||Q_gpu - Q_ref||_2 / ||Q+_ref||_2 (Q+ = gain part),
bounded by 1e-12 for FP64 and 1e-5 for FP32.  Inputs: seeded smooth basis
functions (Maxwellians times random quadratics) from the input generator.
"""
import math

import numpy as np
import pytest

import synth
from oracle import collision as oc

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2112_02695_amd as blr  # noqa: E402

TOL = {torch.float64: 1e-12, torch.float32: 1e-5}


@pytest.fixture(scope="module")
def ctx():
    c = blr.Context(0)
    yield c
    c.close()


def _spec(d, n, m_rho, gamma=None):
    if d == 2:
        return synth.VGridSpec(d=2, n=n, L=8.0, gamma=0.0 if gamma is None else gamma,
                               C=1 / (2 * math.pi), m_rho=m_rho, m_sigma=8)
    return synth.VGridSpec(d=3, n=n, L=8.0, gamma=1.0 if gamma is None else gamma, C=1.0,
                           m_rho=m_rho, m_sigma=38)


def _rel_err(q, qref, gref):
    return np.linalg.norm(q - qref, axis=1) / np.linalg.norm(gref, axis=1)


# 2D grids of 48 and 64 points per axis are switched off in the library (a
# GPU run of the 64-point FP64 line passes ended in a memory fault whose cause
# has not been shown); their parity cases stay here, skipped, until it is.
FAULTED_2D = pytest.mark.skip(reason="2D n = 48 / 64 switched off: a GPU run of the 64-point "
                                     "FP64 line passes faulted, cause not shown")
CASES = [(3, 8, 8, 5), (3, 16, 4, 4), (2, 16, 8, 5), (2, 32, 16, 3), (3, 24, 2, 3),
         pytest.param(2, 48, 8, 3, marks=FAULTED_2D), pytest.param(2, 64, 8, 3, marks=FAULTED_2D)]


@pytest.mark.parametrize("d,n,m_rho,r", CASES)
@pytest.mark.parametrize("dtype", ["float64", "float32"])
@pytest.mark.parametrize("conserve", [True, False])
def test_pairs_match_oracle(ctx, d, n, m_rho, r, dtype, conserve):
    print(f"case d={d} n={n} m_rho={m_rho} r={r} {dtype} conserve={conserve}", flush=True)
    dt = getattr(torch, dtype)
    spec = _spec(d, n, m_rho)
    vs = oc.setup_from_spec(spec)
    V = synth.smooth_basis(r, spec, seed=100 + n)
    pairs = blr.upper_pairs(r)
    qref, gref = oc.q_pairs(V, pairs, vs, conserve=conserve)
    flags = 0 if conserve else blr.BLR_NO_CONSERVE
    vg = blr.vgrid_from_spec(spec, flags)
    Vt = torch.tensor(V, dtype=dt, device="cuda")
    q = ctx.collision_pairs(vg, Vt, pairs)
    torch.cuda.synchronize()
    e = _rel_err(q.double().cpu().numpy(), qref, gref)
    print("max rel err", e.max(), flush=True)
    assert e.max() < TOL[dt]
    if conserve:
        mom = np.array([oc.moments(row, vs) for row in q.double().cpu().numpy()])
        scale = np.array([np.abs(oc.moments(g, vs)).max() for g in gref])
        assert (np.abs(mom).max(axis=1) / scale).max() < (1e-12 if dtype == "float64" else 1e-6)


@pytest.mark.parametrize("dtype", ["float64", "float32"])
def test_plain_schedule_equals_batched(ctx, dtype):
    dt = getattr(torch, dtype)
    spec = _spec(3, 16, 4)
    V = torch.tensor(synth.smooth_basis(4, spec, seed=3), dtype=dt, device="cuda")
    pairs = [(0, 1), (2, 2), (3, 0), (1, 3), (2, 1)]
    a = ctx.collision_pairs(blr.vgrid_from_spec(spec), V, pairs)
    b = ctx.collision_pairs(blr.vgrid_from_spec(spec, blr.BLR_PLAIN_SCHEDULE), V, pairs)
    torch.cuda.synchronize()
    s = b.abs().max().item()
    assert (a - b).abs().max().item() < (1e-13 if dtype == "float64" else 2e-6) * s


def test_pair_order_and_edge_cases(ctx):
    spec = _spec(3, 8, 4)
    V = torch.tensor(synth.smooth_basis(3, spec, seed=8), dtype=torch.float64, device="cuda")
    vg = blr.vgrid_from_spec(spec)
    a = ctx.collision_pairs(vg, V, [(0, 2)])
    b = ctx.collision_pairs(vg, V, [(2, 0)])
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    # single basis function, single pair
    c = ctx.collision_pairs(vg, V[1:2].contiguous(), [(0, 0)])
    d = ctx.collision_pairs(vg, V, [(1, 1)])
    torch.cuda.synchronize()
    assert (c - d).abs().max().item() < 1e-14 * d.abs().max().item()
    # a pair asked for twice (in either order) in one call: every row filled,
    # repeats equal to the first occurrence, all equal to single-pair calls
    for Vx, vgx in ((V, vg), (V.float(), vg)):
        rep = ctx.collision_pairs(vgx, Vx, [(0, 2), (1, 1), (2, 0), (0, 2)])
        one = ctx.collision_pairs(vgx, Vx, [(0, 2)])
        torch.cuda.synchronize()
        assert torch.equal(rep[0], rep[2]) and torch.equal(rep[0], rep[3])
        tol = 1e-14 if Vx.dtype == torch.float64 else 1e-6
        assert (rep[0] - one[0]).abs().max().item() <= tol * one[0].abs().max().item()
    # no pairs: no work, no error
    e = ctx.collision_pairs(vg, V, np.zeros((0, 2), dtype=np.int32))
    assert e.shape[0] == 0
    # errors
    with pytest.raises(blr.BlrError) as ei:
        ctx.collision_pairs(vg, V, [(0, 3)])
    assert ei.value.code == 1
    bad = blr.make_vgrid(3, 20, 8.0)
    with pytest.raises(blr.BlrError) as ei:
        ctx.collision_pairs(bad, V, [(0, 0)])
    assert ei.value.code == 4


@pytest.mark.parametrize("n", [16, 24, 32])
def test_fused_fp32_equals_generic_fp32(ctx, n):
    print(f"fused vs generic n={n}", flush=True)
    spec = _spec(3, n, 16 if n == 32 else 4)
    V = torch.tensor(synth.smooth_basis(7, spec, seed=31), dtype=torch.float32, device="cuda")
    pairs = blr.upper_pairs(7)
    a = ctx.collision_pairs(blr.vgrid_from_spec(spec), V, pairs)
    b = ctx.collision_pairs(blr.vgrid_from_spec(spec, blr.BLR_GENERIC_FFT), V, pairs)
    torch.cuda.synchronize()
    num = (a - b).double().norm(dim=1)
    den = b.double().norm(dim=1)
    assert (num / den).max().item() < 5e-6


@pytest.mark.parametrize("r", [2, 5, 8, 10, 12, 13, 20, 25])
def test_fused_fp32_tile_widths(ctx, r):
    """The sigma sums run in tiles of 4 to 12 basis functions chosen from the
    rank (one or several diagonal tiles, off-diagonal tiles above 12): every
    width and tiling against the generic FP32 pipeline, all pairs and a
    scattered subset."""
    print(f"tile widths r={r}", flush=True)
    spec = _spec(3, 16, 4)
    V = torch.tensor(synth.smooth_basis(r, spec, seed=40 + r), dtype=torch.float32, device="cuda")
    rng = np.random.default_rng(r)
    full = blr.upper_pairs(r)
    sub = [full[k] for k in sorted(rng.choice(len(full), size=max(1, len(full) // 3),
                                              replace=False))]
    for pairs in (full, sub):
        a = ctx.collision_pairs(blr.vgrid_from_spec(spec), V, pairs)
        b = ctx.collision_pairs(blr.vgrid_from_spec(spec, blr.BLR_GENERIC_FFT), V, pairs)
        torch.cuda.synchronize()
        rel = ((a - b).double().norm(dim=1) / b.double().norm(dim=1)).max().item()
        assert rel < 5e-6, (len(pairs), rel)


def _c3_basis():
    nx, r = 256, 10
    spec = synth.C3
    ini = synth.shock_initial(1.5, spec, nx, -30.0, 30.0, pert=1e-3, pert_rank=10, seed=3)
    X, S, V = synth.lowrank_state(ini["f0"], r, 60.0 / nx, (2 * spec.L / spec.n) ** 3)
    return spec, V


@pytest.mark.slow
def test_full_size_sampled_pairs_match_oracle(ctx):
    """The benchmark's launch: 55 pairs of the rank-10 shock basis at 32^3,
    FP32; sampled pairs compared whole-field against the float64 oracle."""
    spec, V = _c3_basis()
    vs = oc.setup_from_spec(spec)
    pairs = blr.upper_pairs(10)
    q = ctx.collision_pairs(blr.vgrid_from_spec(spec), torch.tensor(V, dtype=torch.float32,
                                                                    device="cuda"), pairs)
    torch.cuda.synchronize()
    q = q.double().cpu().numpy()
    for pidx in (0, 17, 54):
        i, j = pairs[pidx]
        qref, gref = oc.q_pairs(V, [(i, j)], vs, conserve=True)
        e = np.linalg.norm(q[pidx] - qref[0]) / np.linalg.norm(gref[0])
        print("pair", (i, j), "rel err", e, flush=True)
        assert e < 1e-5


@pytest.mark.slow
def test_full_size_sampled_modes_match_direct_sum(ctx):
    """Fourier coefficients of Q_s(V_0, V_3) (no projection) at sampled modes
    against the direct spectral sum (the operator's definition), one mode at a time."""
    spec, V = _c3_basis()
    vs = oc.setup_from_spec(spec)
    vg = blr.vgrid_from_spec(spec, blr.BLR_NO_CONSERVE)
    q = ctx.collision_pairs(vg, torch.tensor(V, dtype=torch.float32, device="cuda"), [(0, 3)])
    torch.cuda.synchronize()
    qh_gpu = oc.coefficients(q[0].double().cpu().numpy(), vs, zero_nyquist=False).reshape(-1)
    rng = np.random.default_rng(5)
    ks = np.concatenate([[0, 1, 32, 1024], rng.integers(0, vs.n, 16)])
    g0, g3 = oc.coefficients(V[0], vs), oc.coefficients(V[3], vs)
    a, ap = oc.qhat_direct_c(g0, g3, vs, ks=ks, parts=True)
    b, bp = oc.qhat_direct_c(g3, g0, vs, ks=ks, parts=True)
    ref = 0.5 * (a + b)
    scale = np.abs(0.5 * (ap + bp)).max()
    err = np.abs(qh_gpu[ks] - ref).max() / scale
    print("sampled-mode err", err, flush=True)
    assert err < 1e-5


@pytest.mark.parametrize("d,n,m_rho,mach", [(2, 32, 16, 1.4), (3, 16, 8, 1.5), (3, 32, 16, 1.5)])
@pytest.mark.parametrize("dtype", ["float64", "float32"])
def test_mott_smith_alpha_matches_oracle(ctx, d, n, m_rho, mach, dtype):
    """alpha = int v_1^2 (Q(f_L, f_R) + Q(f_R, f_L)) dv (Sec. 4, eq. alpha) for
    the Rankine-Hugoniot Maxwellians, from the library's pair collision
    Q_s(f_L, f_R) against the oracle's (hard spheres in 3D, Maxwell
    molecules in 2D).  FP64: 1e-12 relative.  FP32: the pair bound
    ||dQ||_2 <= 1e-5 ||Q+||_2 and Cauchy-Schwarz give
    |d alpha| <= 2 dv^d ||v_1^2||_2 1e-5 ||Q+||_2."""
    from oracle import shock
    spec = _spec(d, n, m_rho)
    vs = oc.setup_from_spec(spec)
    left, right = synth.rh_downstream(mach, d)
    v = synth.vgrid_points(d, n, spec.L)
    fL = synth.maxwellian(v, left[0], (left[1],) + (0.0,) * (d - 1), left[2]).reshape(-1)
    fR = synth.maxwellian(v, right[0], (right[1],) + (0.0,) * (d - 1), right[2]).reshape(-1)
    print(f"mott-smith alpha d={d} n={n} {dtype}", flush=True)
    a_ref = shock.mott_smith_alpha(fL, fR, vs)
    _, gain = oc.q_pairs(np.array([fL, fR]), [(0, 1)], vs, conserve=False)
    vg = blr.vgrid_from_spec(spec, blr.BLR_NO_CONSERVE)
    dt = getattr(torch, dtype)
    Q = ctx.collision_pairs(vg, torch.tensor(np.array([fL, fR]), dtype=dt, device="cuda"),
                            [(0, 1)]).double().cpu().numpy()[0]
    v1sq = (v[0].reshape(-1)) ** 2
    dvd = vs.dv ** d
    a_gpu = 2.0 * dvd * float(np.dot(v1sq, Q))
    if dt == torch.float64:
        assert abs(a_gpu - a_ref) <= 1e-12 * abs(a_ref)
    else:
        bound = 2.0 * dvd * np.linalg.norm(v1sq) * 1e-5 * np.linalg.norm(gain[0])
        assert abs(a_gpu - a_ref) <= bound
        print("fp32 alpha error", abs(a_gpu - a_ref), "bound", bound, flush=True)
