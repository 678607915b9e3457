"""GPU parity of single evaluations Q(f, f) of the homogeneous workloads
against the oracle's stored values (``tests/golden/c1_c2_q.npz``, written by
``make_c1_c2.py``, which calls only the oracle and the input generator):

  C1  2D 32^2, Maxwell molecules, two-stream distribution with 1% noise;
  C2  3D 32^3, hard spheres on a bi-Maxwellian mix, and Maxwell molecules on
      the BKW solution (also checked against its analytic dF/dt).

Error per result: ||Q_gpu - Q_ref||_2 / ||Q^+_ref||_2, bounded by 1e-12 in
FP64 and 1e-5 in FP32, with and without the conservation projection.
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

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c1_c2_q.npz")
BKW = synth.VGridSpec(d=3, n=32, L=8.0, gamma=0.0, C=1.0 / (4.0 * math.pi), m_rho=16, m_sigma=38)
SPECS = {"c1": synth.C1, "c2b": synth.C2, "c2k": BKW}
TOL = {"float64": 1e-12, "float32": 1e-5}


@pytest.fixture(scope="module")
def gold():
    z = np.load(GOLDEN)
    return {k: z[k] for k in z.files}


@pytest.fixture(scope="module")
def ctx():
    c = blr.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("case", ["c1", "c2b", "c2k"])
@pytest.mark.parametrize("dtype", ["float64", "float32"])
@pytest.mark.parametrize("conserve", [False, True])
def test_single_evaluation_matches_oracle(ctx, gold, case, dtype, conserve):
    print(f"golden {case} {dtype} conserve={conserve}", flush=True)
    spec = SPECS[case]
    f = torch.tensor(np.ascontiguousarray(gold[f"{case}_f"]).reshape(1, -1),
                     dtype=getattr(torch, dtype), device="cuda")
    vg = blr.vgrid_from_spec(spec, 0 if conserve else blr.BLR_NO_CONSERVE)
    q = ctx.collision_pairs(vg, f, [(0, 0)])
    torch.cuda.synchronize()
    q = q.double().cpu().numpy()[0]
    ref = gold[f"{case}_qc" if conserve else f"{case}_q"]
    e = np.linalg.norm(q - ref) / float(gold[f"{case}_gain_norm"])
    print(f"  error / ||Q+|| = {e:.3e}", flush=True)
    assert e < TOL[dtype]
    if case == "c2k" and not conserve:
        # BKW: dF/dt = Q(f, f) in closed form; the discrete operator reaches it
        # to the accuracy the oracle itself has on this grid
        d = gold["c2k_dfdt"]
        eo = np.abs(ref - d).max() / np.abs(d).max()
        eg = np.abs(q - d).max() / np.abs(d).max()
        print(f"  vs analytic dF/dt: gpu {eg:.3e}, oracle {eo:.3e}", flush=True)
        assert eg < 1e-2
