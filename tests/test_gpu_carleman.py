"""GPU parity of the Carleman form (vgrid flag BLR_CARLEMAN) against the
oracle's Carleman-form operator (oracle/carleman.py).

Error measure per pair: ||Q_gpu - Q_ref||_2 / ||Q+_ref||_2, bounded by 1e-12
(FP64) and 1e-5 (FP32), with and without the moment projection; the plain
one-pair-at-a-time schedule gives the batched result; a low-rank step whose
collisions use the Carleman form matches the oracle's step with the same
collision evaluator (f to 1e-12 in FP64).
"""
import math

import numpy as np
import pytest

import synth
from oracle import carleman as ca
from oracle import collision as oc
from oracle import dlr

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


def _spec(d, n, M):
    if d == 2:
        return synth.VGridSpec(d=2, n=n, L=8.0, gamma=0.0, C=1 / (2 * math.pi), m_rho=1,
                               m_sigma=M)
    return synth.VGridSpec(d=3, n=n, L=8.0, gamma=1.0, C=1.0, m_rho=1, m_sigma=38)


# 2D grids of 48 and 64 points per axis are switched off in the library (this
# test at 64 points in FP64 ended in a GPU memory fault whose cause has not
# been shown); the cases stay here, skipped, until it is.
FAULTED_2D = pytest.mark.skip(reason="2D n = 48 / 64 switched off: a GPU run of this test at "
                                     "64 points in FP64 faulted, cause not shown")
CASES = [(2, 16, 8, 4), (2, 32, 16, 3), (2, 32, 6, 3), (3, 8, 38, 4), (3, 16, 38, 3),
         (3, 24, 38, 3), (3, 32, 38, 2),
         pytest.param(2, 48, 8, 3, marks=FAULTED_2D), pytest.param(2, 64, 16, 3, marks=FAULTED_2D)]


@pytest.mark.parametrize("d,n,M,r", CASES)
@pytest.mark.parametrize("dtype", ["float64", "float32"])
@pytest.mark.parametrize("conserve", [True, False])
def test_pairs_match_oracle(ctx, d, n, M, r, dtype, conserve):
    print(f"carleman d={d} n={n} M={M} r={r} {dtype} conserve={conserve}", flush=True)
    spec = _spec(d, n, M)
    cs = ca.setup_from_spec(spec)
    V = synth.smooth_basis(r, spec, seed=11 + r)
    pairs = blr.upper_pairs(r)
    ref, gain = ca.q_pairs(V, pairs, cs, conserve=conserve)
    flags = blr.BLR_CARLEMAN | (0 if conserve else blr.BLR_NO_CONSERVE)
    dt = getattr(torch, dtype)
    Q = ctx.collision_pairs(blr.vgrid_from_spec(spec, flags),
                            torch.tensor(V, dtype=dt, device="cuda"), pairs)
    Q = Q.double().cpu().numpy()
    rel = np.linalg.norm(Q - ref, axis=1) / np.linalg.norm(gain, axis=1)
    print("max rel", rel.max(), flush=True)
    assert rel.max() < TOL[dt]


@pytest.mark.parametrize("dtype", ["float64", "float32"])
def test_plain_schedule_equals_batched(ctx, dtype):
    spec = _spec(3, 16, 38)
    V = synth.smooth_basis(3, spec, seed=4)
    pairs = [(0, 0), (0, 2), (1, 2), (2, 1)]
    dt = getattr(torch, dtype)
    Vd = torch.tensor(V, dtype=dt, device="cuda")
    a = ctx.collision_pairs(blr.vgrid_from_spec(spec, blr.BLR_CARLEMAN), Vd, pairs)
    b = ctx.collision_pairs(blr.vgrid_from_spec(spec, blr.BLR_CARLEMAN | blr.BLR_PLAIN_SCHEDULE),
                            Vd, pairs)
    a, b = a.double().cpu().numpy(), b.double().cpu().numpy()
    assert np.abs(a - b).max() <= (1e-13 if dtype == "float64" else 1e-6) * np.abs(a).max()


def test_2d_grids_beyond_32_are_refused(ctx):
    """2D n = 48 and 64 are switched off (see the grid validation): the call
    returns BLR_ERR_UNSUPPORTED before any launch."""
    for n in (48, 64):
        spec = _spec(2, n, 8)
        V = torch.zeros((1, n * n), dtype=torch.float64, device="cuda")
        with pytest.raises(blr.BlrError) as ei:
            ctx.collision_pairs(blr.vgrid_from_spec(spec, blr.BLR_CARLEMAN), V, [(0, 0)])
        assert ei.value.code == blr.BLR_ERR_UNSUPPORTED


def test_rejects_kernels_without_a_constant_carleman_kernel(ctx):
    spec = synth.VGridSpec(d=3, n=16, L=8.0, gamma=0.0, C=1.0, m_rho=1, m_sigma=38)
    V = torch.zeros((1, 4096), dtype=torch.float64, device="cuda")
    with pytest.raises(blr.BlrError) as ei:
        ctx.collision_pairs(blr.vgrid_from_spec(spec, blr.BLR_CARLEMAN), V, [(0, 0)])
    assert ei.value.code == blr.BLR_ERR_ARG


@pytest.mark.parametrize("d,N,nx,r,M", [(2, 32, 24, 4, 8), (3, 16, 20, 3, 38)])
def test_step_with_carleman_collisions_matches_oracle(ctx, d, N, nx, r, M):
    """One fixed-rank K-S-L step (FP64) whose pair collisions use the
    Carleman form, against the oracle's step with the oracle's Carleman
    evaluator."""
    spec = _spec(d, N, M)
    cs = ca.setup_from_spec(spec)
    ini = synth.shock_initial(1.4, spec, nx, -30.0, 30.0, pert=1e-2, pert_rank=3, seed=2)
    prob = dlr.Problem1D(vs=oc.setup(d, N, spec.L, spec.C, spec.gamma, 1, spec.m_sigma), nx=nx,
                         x_lo=-30.0, x_hi=30.0, fL=ini["fL"], fR=ini["fR"],
                         collision=lambda V, pairs, vs, conserve: ca.q_pairs(V, pairs, cs,
                                                                             conserve=conserve))
    X, S, V = synth.lowrank_state(ini["f0"], r, prob.dx, prob.dvd)
    st = dlr.State(X, S, V)
    new, err, _ = dlr.ksl_step(st, prob, 0.05)
    r_cap = 8
    Xd = torch.zeros((r_cap, nx), dtype=torch.float64, device="cuda")
    Sd = torch.zeros((r_cap, r_cap), dtype=torch.float64, device="cuda")
    Vd = torch.zeros((r_cap, V.shape[1]), dtype=torch.float64, device="cuda")
    Xd[:r] = torch.tensor(X.T, device="cuda")
    Sd[:r, :r] = torch.tensor(S, device="cuda")
    Vd[:r] = torch.tensor(V, device="cuda")
    fL = torch.tensor(ini["fL"], device="cuda")
    fR = torch.tensor(ini["fR"], device="cuda")
    pb = ctx.make_problem(blr.vgrid_from_spec(spec, blr.BLR_CARLEMAN), nx, -30.0, 30.0, fL, fR)
    sd = ctx.make_state(Xd, Sd, Vd, r)
    info = ctx.dlr_step(pb, sd, blr.StepParams(0.05, 0.2, 1e-10, 1, r_cap,
                                               blr.BLR_STEP_FP64_COLLISION))
    f_gpu = Xd[:r].cpu().numpy().T @ Sd[:r, :r].cpu().numpy() @ Vd[:r].cpu().numpy()
    f_ref = new.full()
    e = np.abs(f_gpu - f_ref).max() / np.abs(f_ref).max()
    print("carleman step f rel err", e, flush=True)
    assert e < 1e-12
    assert abs(info.err - err) < 1e-10 * err


@pytest.mark.parametrize("n", [16, 24, 32])
def test_fused_filters_equal_generic(ctx, n):
    """3D FP32: the fused filter kernel (one workgroup per field, the whole
    transform in LDS) against the generic line passes (BLR_GENERIC_FFT)."""
    spec = _spec(3, n, 38)
    V = torch.tensor(synth.smooth_basis(4, spec, seed=21), dtype=torch.float32, device="cuda")
    pairs = blr.upper_pairs(4)
    a = ctx.collision_pairs(blr.vgrid_from_spec(spec, blr.BLR_CARLEMAN), V, pairs)
    b = ctx.collision_pairs(blr.vgrid_from_spec(spec, blr.BLR_CARLEMAN | blr.BLR_GENERIC_FFT), V,
                            pairs)
    a, b = a.double().cpu().numpy(), b.double().cpu().numpy()
    ref, gain = ca.q_pairs(V.double().cpu().numpy(), pairs, ca.setup_from_spec(spec))
    for q in (a, b):
        rel = np.linalg.norm(q - ref, axis=1) / np.linalg.norm(gain, axis=1)
        assert rel.max() < 1e-5
    assert np.abs(a - b).max() <= 1e-5 * np.abs(gain).max()
