"""blr_collision_pairs_noalloc (workspace in the library's fixed device
array, no allocation) against blr_collision_pairs on the same inputs.

Both run the same kernels in the same order, so their results are compared
bitwise: the fused FP32 path (3D 16^3), the general FP64 path (3D 8^3), the
one-pair-at-a-time schedule with a repeated pair and no projection, and the
Carleman form (2D 16^2).  Each case makes two calls in a row, the second with
fewer basis functions and pairs than the first; a call whose workspace would
not fit the array is refused before anything is issued.
"""
import math

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2112_02695_amd as blr  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    c = blr.Context(0)
    yield c
    c.close()


def _spec3(n, m_rho):
    return synth.VGridSpec(d=3, n=n, L=8.0, gamma=1.0, C=1.0, m_rho=m_rho, m_sigma=38)


CASES = [
    # (name, spec, flags, dtype, (r1, pairs1), (r2, pairs2))
    ("fused fp32 16^3", _spec3(16, 4), 0, torch.float32,
     (5, blr.upper_pairs(5)), (2, blr.upper_pairs(2))),
    ("general fp64 8^3", _spec3(8, 6), 0, torch.float64,
     (6, blr.upper_pairs(6)), (3, [(0, 2), (1, 1)])),
    ("plain fp32 16^3, repeated pair, no projection", _spec3(16, 2),
     blr.BLR_PLAIN_SCHEDULE | blr.BLR_NO_CONSERVE, torch.float32,
     (3, [(0, 1), (2, 2), (1, 0)]), (2, [(1, 1)])),
    ("carleman fp64 2D 16^2",
     synth.VGridSpec(d=2, n=16, L=8.0, gamma=0.0, C=1 / (2 * math.pi), m_rho=1, m_sigma=8),
     blr.BLR_CARLEMAN, torch.float64, (4, blr.upper_pairs(4)), (1, [(0, 0)])),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_noalloc_equals_collision_pairs(ctx, case):
    name, spec, flags, dt, first, second = case
    print(f"noalloc: {name}", flush=True)
    vg = blr.vgrid_from_spec(spec, flags)
    V = torch.tensor(synth.smooth_basis(first[0], spec, seed=9), dtype=dt, device="cuda")
    for r, pairs in (first, second):
        Vr = V[:r].contiguous()
        ref = ctx.collision_pairs(vg, Vr, pairs)
        out = torch.full_like(ref, float("nan"))
        ctx.collision_pairs(vg, Vr, pairs, out=out, noalloc=True)
        torch.cuda.synchronize()
        print(f"  r={r} pairs={len(pairs)}: max |diff| {float((out - ref).abs().max()):.3e}",
              flush=True)
        assert torch.equal(out, ref)


def test_oversized_call_is_refused(ctx):
    spec = _spec3(32, 16)
    vg = blr.vgrid_from_spec(spec)
    V = torch.zeros((12, spec.npts), dtype=torch.float32, device="cuda")
    out = torch.full((78, spec.npts), 7.0, dtype=torch.float32, device="cuda")
    with pytest.raises(blr.BlrError) as ei:
        ctx.collision_pairs(vg, V, blr.upper_pairs(12), out=out, noalloc=True)
    torch.cuda.synchronize()
    assert ei.value.code == blr.BLR_ERR_ARG
    assert "scratch" in str(ei.value)
    assert bool((out == 7.0).all())
