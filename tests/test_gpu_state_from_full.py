"""GPU parity of blr_state_from_full (Sec. 2.4: the initial factors are a
truncated SVD of f^0) against the oracle's truncated SVD
(``oracle.dlr.initial_state``).

Singular values are unique; the factors are unique up to signs (and
rotations within equal singular values), so the comparison is on S's
diagonal (to 1e-12 of sigma_1), on the reconstructed rank-r f (to 1e-12 of
max |f|), and on the orthonormality of X and V in the weighted inner
products.  Shapes: one-dimensional space beyond the former 64-cell limit
(the benchmark's N_x = 256 at N_v = 32^3), a rectangle, and r up to the
cell count.
"""
import math

import numpy as np
import pytest

import synth
from oracle import dlr

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


def _spec(d, N):
    if d == 2:
        return synth.VGridSpec(d=2, n=N, L=8.0, gamma=0.0, C=1 / (2 * math.pi), m_rho=4, m_sigma=8)
    return synth.VGridSpec(d=3, n=N, L=8.0, gamma=1.0, C=1.0, m_rho=4, m_sigma=38)


def _check(ctx, pb, F0, r, r_cap, wx, dvd):
    dev = "cuda"
    cells, n = F0.shape
    X = torch.zeros((r_cap, cells), dtype=torch.float64, device=dev)
    S = torch.zeros((r_cap, r_cap), dtype=torch.float64, device=dev)
    V = torch.zeros((r_cap, n), dtype=torch.float64, device=dev)
    st = ctx.make_state(X, S, V, 1)
    f0 = torch.tensor(F0, device=dev)
    ctx.state_from_full(pb, f0, r, st)
    assert st.r == r
    Xg, Sg, Vg = X[:r].cpu().numpy().T, S[:r, :r].cpu().numpy(), V[:r].cpu().numpy()
    ref = dlr.initial_state(F0, r, wx, dvd)
    sg, so = np.diag(Sg), np.diag(ref.S)
    print(f"cells {cells} n {n} r {r}: sigma err {np.abs(sg - so).max() / so[0]:.2e}", flush=True)
    assert np.abs(Sg - np.diag(sg)).max() == 0.0
    assert np.abs(sg - so).max() <= 1e-12 * so[0]
    fg, fo = Xg @ Sg @ Vg, ref.full()
    e = np.abs(fg - fo).max() / np.abs(fo).max()
    print(f"  f err {e:.2e}", flush=True)
    assert e <= 1e-12
    assert np.abs(wx * Xg.T @ Xg - np.eye(r)).max() < 1e-12
    assert np.abs(dvd * Vg @ Vg.T - np.eye(r)).max() < 1e-12


@pytest.mark.parametrize("d,N,nx,r", [(2, 16, 24, 4), (2, 16, 24, 24), (3, 16, 100, 8),
                                      (3, 32, 256, 10)])
def test_one_dimensional_space(ctx, d, N, nx, r):
    print(f"state_from_full 1D d={d} N={N} nx={nx} r={r}", flush=True)
    spec = _spec(d, N)
    ini = synth.shock_initial(1.5, spec, nx, -30.0, 30.0, pert=1e-3, pert_rank=10, seed=3)
    fL = torch.tensor(ini["fL"], device="cuda")
    fR = torch.tensor(ini["fR"], device="cuda")
    pb = ctx.make_problem(blr.vgrid_from_spec(spec), nx, -30.0, 30.0, fL, fR)
    dx, dvd = 60.0 / nx, (2 * spec.L / spec.n) ** d
    _check(ctx, pb, ini["f0"], r, max(r, 12), dx, dvd)


def test_rectangle(ctx):
    print("state_from_full 2D space 6 x 5 cells", flush=True)
    spec = _spec(2, 16)
    nx, ny = 6, 5
    F0 = synth.rect_field(spec, nx, ny, seed=3, rank=3, pert=5e-2)
    f = torch.tensor(F0[0], device="cuda")
    faces = [(f, False)] * 4
    pb = ctx.make_problem2d(blr.vgrid_from_spec(spec), nx, ny, 0.0, 1.0, 0.0, 0.8, faces)
    wx, dvd = (1.0 / nx) * (0.8 / ny), (2 * spec.L / spec.n) ** 2
    _check(ctx, pb, F0, 7, 8, wx, dvd)


def test_rank_beyond_the_cells_is_refused(ctx):
    spec = _spec(2, 16)
    nx = 6
    ini = synth.shock_initial(1.5, spec, nx, -30.0, 30.0, pert=0.0, pert_rank=0)
    fL = torch.tensor(ini["fL"], device="cuda")
    pb = ctx.make_problem(blr.vgrid_from_spec(spec), nx, -30.0, 30.0, fL, fL)
    X = torch.zeros((8, nx), dtype=torch.float64, device="cuda")
    S = torch.zeros((8, 8), dtype=torch.float64, device="cuda")
    V = torch.zeros((8, spec.npts), dtype=torch.float64, device="cuda")
    st = ctx.make_state(X, S, V, 1)
    with pytest.raises(blr.BlrError) as ei:
        ctx.state_from_full(pb, torch.tensor(ini["f0"], device="cuda"), 7, st)
    assert ei.value.code == blr.BLR_ERR_ARG
    assert st.r == 1 and float(X.abs().max()) == 0.0
