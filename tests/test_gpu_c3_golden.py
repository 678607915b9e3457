"""GPU parity of the benchmark's own workload against the oracle's stored
values (``tests/golden/c3_step.npz``, written by ``make_c3_step.py``, which
calls only the oracle and the input generator).

Workload: the Mach-1.5 shock state at N_x = 256, N_v = 32^3 on [-8, 8]^3,
hard spheres, 16 x 38 nodes, rank 10 augmented by the two boundary functions
to rank 12 (78 pairs).

* All 78 pairs of the augmented basis through the library's default FP32
  path (the fused shift kernel, the 12-wide sigma-reduction tile, the fused
  final kernel with the FP64 projection), each against the oracle's
  Q_s to 1e-5 of ||Q_s^+|| (the FP32 collision tolerance).
* The benchmark's adaptive step (add, FP32 collisions, K-S-L, residual,
  drop with c = 0.2 and r_min 10) as a replayed HIP graph: ranks identical,
  f within the FP32 collision bound 1e-5 dt ||sum (2 - delta) K_m K_n Q^+_mn||
  (a collision error enters the step linearly through dt Q_s), err and
  err_ada within the same bound.
* The same step with FP64 collisions: f to 1e-12 of ||f|| in L2 and 1e-11
  of max |f|, err and err_ada to 1e-10 relative.  The pointwise bound is the
  looser one because this state's boundary rows lie in span V up to 2e-6
  and 5e-7 of their size, so the two directions the augmentation adds are
  fixed by FP64 rounding only to about 1e-10: two equivalent FP64
  orthogonalisations within the oracle give steps 6.2e-12 apart in
  max |f| (at the corner of the velocity box, where f is 1e-10 of its
  maximum) and 3.6e-13 apart in L2; the fixed-rank step (no augmentation)
  agrees to 3e-15.
"""
import math
import os

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2112_02695_amd as blr  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden", "c3_step.npz")
NX, R0, R_MAX = 256, 10, 12


@pytest.fixture(scope="module")
def gold():
    z = np.load(GOLDEN)
    return {k: z[k] for k in z.files}


@pytest.fixture(scope="module")
def ctx():
    c = blr.Context(0)
    yield c
    c.close()


def _c3_inputs(gold):
    """The stored initial factors (the input generator's SVD is not
    reproducible across machines to the 1e-12 the FP64 step is held to) and
    the inflow Maxwellians, which are closed-form."""
    spec = synth.C3
    ini = synth.shock_initial(1.5, spec, NX, -30.0, 30.0, pert=0.0, pert_rank=0)
    dx = 60.0 / NX
    dvd = (2 * spec.L / spec.n) ** 3
    X, S, V = (np.ascontiguousarray(gold[k]) for k in ("X0", "S0", "V0"))
    return spec, ini, dx, dvd, X, S, V


def _timers(ctx):
    import ctypes
    lib = ctx.lib
    lib.blr_timing.argtypes = [ctypes.c_void_p, ctypes.c_int32]
    lib.blr_timing_read.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_char_p,
                                    ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)]
    out, i = [], 0
    buf = ctypes.create_string_buffer(256)
    ms, nl, by = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double()
    while lib.blr_timing_read(ctx.h, i, buf, 256, ctypes.byref(ms), ctypes.byref(nl),
                              ctypes.byref(by)) == 0:
        out.append(buf.value.decode())
        i += 1
    return out


def test_all_78_pairs_of_the_benchmark_basis(ctx, gold):
    print("c3 golden: 78 pairs, fp32 default path", flush=True)
    V32 = torch.tensor(np.ascontiguousarray(gold["V_aug32"]), device="cuda")
    pairs = blr.upper_pairs(R_MAX)
    vg = blr.vgrid_from_spec(synth.C3)
    ctx.lib.blr_timing(ctx.h, 2)
    ctx.lib.blr_timing(ctx.h, 1)
    Q = ctx.collision_pairs(vg, V32, pairs)
    torch.cuda.synchronize()
    ctx.lib.blr_timing(ctx.h, 0)
    names = _timers(ctx)
    assert "fast.shift" in names and "fast.reduce.g12" in names, names
    q = Q.double().cpu().numpy()
    ref = gold["q32"].astype(np.float64)
    err = np.linalg.norm(q - ref, axis=1) / gold["qplus_norm"]
    print(f"max pair error / ||Q+|| = {err.max():.3e} (pair {int(err.argmax())}), "
          f"median {np.median(err):.3e}", flush=True)
    assert np.all(np.isfinite(err))
    assert err.max() < 1e-5
    # the moments the FP64 projection zeroes
    spec = synth.C3
    v = synth.vgrid_points(3, spec.n, spec.L).reshape(3, -1)
    dvd = (2 * spec.L / spec.n) ** 3
    C = dvd * np.vstack([np.ones(v.shape[1]), v, (v ** 2).sum(axis=0)])
    mom = np.abs(q @ C.T).max(axis=0)
    scale = (np.abs(q) @ np.abs(C.T)).max(axis=0)
    assert np.all(mom <= 1e-6 * scale), mom / scale


class _Gpu:
    def __init__(self, ctx, spec, ini, X, S, V):
        dev = "cuda"
        self.init = (X, S, V)
        self.X = torch.zeros((R_MAX, NX), dtype=torch.float64, device=dev)
        self.S = torch.zeros((R_MAX, R_MAX), dtype=torch.float64, device=dev)
        self.V = torch.zeros((R_MAX, V.shape[1]), dtype=torch.float64, device=dev)
        self.fL = torch.tensor(ini["fL"], device=dev)
        self.fR = torch.tensor(ini["fR"], device=dev)
        self.pb = ctx.make_problem(blr.vgrid_from_spec(spec), NX, -30.0, 30.0, self.fL, self.fR)
        self.st = ctx.make_state(self.X, self.S, self.V, R0, seed=1)
        self.reset()

    def reset(self):
        X, S, V = self.init
        self.X.zero_()
        self.S.zero_()
        self.V.zero_()
        self.X[:R0] = torch.tensor(X.T, device="cuda")
        self.S[:R0, :R0] = torch.tensor(S, device="cuda")
        self.V[:R0] = torch.tensor(V, device="cuda")
        self.st.r = R0
        torch.cuda.synchronize()

    def full(self):
        r = self.st.r
        return (self.X[:r].cpu().numpy().T @ self.S[:r, :r].cpu().numpy()) @ self.V[:r].cpu().numpy()


def _step(ctx, g, gold, fp64):
    flags = blr.BLR_STEP_ADD | blr.BLR_STEP_DROP | (blr.BLR_STEP_FP64_COLLISION if fp64 else 0)
    sp = blr.StepParams(float(gold["dt"]), 0.2, 1e-10, R0, R_MAX, flags)
    return ctx.dlr_step(g.pb, g.st, sp)


@pytest.mark.parametrize("fp64", [False, True])
def test_benchmark_step_matches_oracle(ctx, gold, fp64):
    print(f"c3 golden: adaptive step, fp64 collisions = {fp64}", flush=True)
    spec, ini, dx, dvd, X, S, V = _c3_inputs(gold)
    g = _Gpu(ctx, spec, ini, X, S, V)
    # first call: issued directly; reset the same arrays and step again: the
    # second sighting of this configuration is recorded and replayed
    first = _step(ctx, g, gold, fp64)
    f_first = g.full()
    g.reset()
    info = _step(ctx, g, gold, fp64)
    torch.cuda.synchronize()
    print(f"first ms_collision {first.ms_collision:.3f}, replay ms_collision {info.ms_collision:.3f}",
          flush=True)
    assert info.ms_collision == 0.0          # ran as a replayed graph
    f_gpu = g.full()
    assert np.array_equal(f_gpu, f_first)    # replay == direct issue, bitwise
    f_ref = (gold["X1"] @ gold["S1"]) @ gold["V1"]
    assert (info.r_added, info.r_out, g.st.r) == (int(gold["r_added"]), int(gold["r_out"]),
                                                  int(gold["r_out"]))
    w = math.sqrt(dx * dvd)
    diff = w * np.linalg.norm(f_gpu - f_ref)
    rel_max = np.abs(f_gpu - f_ref).max() / np.abs(f_ref).max()
    bound = 1e-5 * float(gold["dt"]) * float(gold["gain_scale"])
    print(f"||f_gpu - f_ref|| = {diff:.3e}, bound {bound:.3e}, max rel {rel_max:.3e}; "
          f"err {info.err:.10e} vs {float(gold['err']):.10e}, "
          f"err_ada {info.err_ada:.10e} vs {float(gold['err_ada']):.10e}", flush=True)
    if fp64:
        assert np.linalg.norm(f_gpu - f_ref) < 1e-12 * np.linalg.norm(f_ref)
        assert rel_max < 1e-11
        assert abs(info.err - gold["err"]) < 1e-10 * gold["err"]
        assert abs(info.err_ada - gold["err_ada"]) < 1e-10 * gold["err_ada"]
    else:
        assert diff <= bound
        assert abs(info.err - gold["err"]) <= bound
        assert abs(info.err_ada - gold["err_ada"]) <= bound


def test_benchmark_fixed_rank_step_fp64(ctx, gold):
    """Without the augmentation the FP64 step meets 1e-12 of max |f|."""
    print("c3 golden: fixed-rank step, fp64 collisions", flush=True)
    spec, ini, dx, dvd, X, S, V = _c3_inputs(gold)
    g = _Gpu(ctx, spec, ini, X, S, V)
    info = ctx.dlr_step(g.pb, g.st, blr.StepParams(float(gold["dt"]), 0.2, 1e-10, R0, R_MAX,
                                                   blr.BLR_STEP_FP64_COLLISION))
    f_gpu = g.full()
    f_ref = (gold["XF"] @ gold["SF"]) @ gold["VF"]
    rel_max = np.abs(f_gpu - f_ref).max() / np.abs(f_ref).max()
    print(f"  max rel {rel_max:.2e}, err {info.err:.12e} vs {float(gold['errF']):.12e}", flush=True)
    assert g.st.r == R0
    assert rel_max < 1e-12
    assert abs(info.err - gold["errF"]) < 1e-10 * gold["errF"]
