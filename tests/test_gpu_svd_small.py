"""The device SVD of small square FP64 matrices (blr_svd_small), which factors
the step's new S for the rank truncation (Sec. 3.2) and the R factor of the
boundary rows for the augmentation (Sec. 3.1).  Checked against numpy's SVD
and against its own definition: U diag(sig) W^T = A, U and W orthonormal,
sig descending; rank-deficient and zero matrices complete U to an
orthonormal basis when asked."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    import paper_2112_02695_amd as blr
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = blr.Context(0)
    yield c
    c.close()


def _run(ctx, A, trans=False, complete=True):
    U, s, W = ctx.svd_small(torch.tensor(A, device="cuda"), trans=trans, complete=complete)
    torch.cuda.synchronize()
    return U.cpu().numpy(), s.cpu().numpy(), W.cpu().numpy()


def _check_full(A, U, s, W, tol=1e-13):
    r = A.shape[0]
    sref = np.linalg.svd(A, compute_uv=False)
    scale = max(sref[0], 1e-300)
    assert np.all(np.diff(s) <= 1e-15 * scale)
    assert np.max(np.abs(s - sref)) <= tol * scale * max(1, r / 8)
    assert np.linalg.norm(U @ np.diag(s) @ W.T - A) <= tol * max(np.linalg.norm(A), 1e-300) * max(1, r / 8)
    assert np.max(np.abs(W.T @ W - np.eye(r))) <= 1e-13 * max(1, r / 8)


@pytest.mark.parametrize("r", [1, 2, 5, 16, 33, 64])
@pytest.mark.parametrize("trans", [False, True])
def test_random_matrices(ctx, r, trans):
    print(f"svd_small random r={r} trans={trans}", flush=True)
    A = np.random.default_rng(100 + r).standard_normal((r, r))
    U, s, W = _run(ctx, A, trans=trans)
    _check_full(A.T if trans else A, U, s, W)
    assert np.max(np.abs(U.T @ U - np.eye(r))) <= 1e-13 * max(1, r / 8)


@pytest.mark.parametrize("r,k", [(8, 3), (33, 7), (64, 8), (64, 1)])
def test_rank_deficient_completes_u(ctx, r, k):
    print(f"svd_small rank-deficient r={r} k={k}", flush=True)
    rng = np.random.default_rng(7 * r + k)
    A = rng.standard_normal((r, k)) @ rng.standard_normal((k, r))
    U, s, W = _run(ctx, A, complete=True)
    _check_full(A, U, s, W, tol=1e-12)
    assert np.all(s[k:] <= 1e-13 * s[0])
    # every column of U, the completed ones included, is orthonormal
    assert np.max(np.abs(U.T @ U - np.eye(r))) <= 1e-12
    # without completion the leading k columns are still the left singular vectors
    U2, s2, W2 = _run(ctx, A, complete=False)
    assert np.max(np.abs(s2 - s)) <= 1e-13 * s[0]
    assert np.max(np.abs(U2[:, :k].T @ U2[:, :k] - np.eye(k))) <= 1e-12
    assert np.linalg.norm(U2 @ np.diag(s2) @ W2.T - A) <= 1e-12 * np.linalg.norm(A)


def test_zero_matrix(ctx):
    r = 12
    A = np.zeros((r, r))
    U, s, W = _run(ctx, A, complete=True)
    assert np.all(s == 0.0)
    assert np.max(np.abs(U.T @ U - np.eye(r))) <= 1e-14
    assert np.max(np.abs(W.T @ W - np.eye(r))) <= 1e-14
    U2, s2, _ = _run(ctx, A, complete=False)
    assert np.all(U2 == 0.0) and np.all(s2 == 0.0)


def test_sizes_out_of_range_are_refused(ctx):
    import paper_2112_02695_amd as blr
    A = torch.zeros((65, 65), dtype=torch.float64, device="cuda")
    with pytest.raises(blr.BlrError):
        ctx.svd_small(A)


def test_boundary_factor_size_takes_milliseconds(ctx):
    # a 64 x 64 factor of rank 8 (the shape of a rectangle's boundary rows
    # after the projection) with its U completed
    rng = np.random.default_rng(3)
    A = torch.tensor(rng.standard_normal((64, 8)) @ rng.standard_normal((8, 64)), device="cuda")
    for _ in range(2):
        ctx.svd_small(A)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        ctx.svd_small(A)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 5
    print(f"svd_small 64 x 64, rank 8, completed: {ms:.3f} ms", flush=True)
    assert ms < 20.0
