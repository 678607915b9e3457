"""A server with batch_collisions: the FP32 pair collisions of every live
solve on the fused grids run together, one launch sequence per step over all
their bases (collision pairs of all live requests and quadrature nodes in one
fused launch, recorded as a HIP graph per composition; the sigma-sum tile
width chosen by timing).

* Each result is the same alone and in the mix: a solve served beside other
  solves (two velocity grids, and a 2D-velocity solve that is not batched)
  gives bit-identical factors, rank, step count and err_ada to the same solve
  served alone by a batching server.
* The batches really held several solves' collisions.
* Batched and unbatched solves agree to FP32 rounding (the pair transforms of
  a batch group the radial nodes two by two whatever the pair count).
* Stopping a busy batching server returns.
"""
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2112_02695_amd as blr  # noqa: E402
from test_gpu_serve import Req, _factors, _solve_params  # noqa: E402

REQS = [  # (d, n, m_rho, nx, r, mach, seed, dt, steps)
    (3, 16, 4, 24, 3, 1.5, 3, 0.02, 6),
    (3, 16, 4, 32, 4, 1.8, 7, 0.02, 5),
    (3, 16, 4, 20, 5, 1.3, 8, 0.03, 7),
    (3, 24, 4, 24, 3, 1.6, 9, 0.02, 4),
    (2, 32, 8, 40, 4, 1.8, 4, 0.02, 6),   # 2D velocity: not batched
]


@pytest.fixture(scope="module")
def helper():
    c = blr.Context(0)   # make_problem / make_state only
    yield c
    c.close()


def _serve(helper, jobs, slots, batch=True):
    sv = blr.Server(0, slots=slots, batch_collisions=batch)
    keep = {}
    try:
        for k, tag in jobs:
            d, n, m_rho, nx, r, mach, seed, dt, steps = REQS[k]
            q = Req(d, n, m_rho, nx, r, mach, seed)
            pb, st, arrs = q.device(helper)
            sv.submit(pb, st, _solve_params(dt, steps), tag)
            keep[tag] = (k, st, arrs)
        comps = []
        while len(comps) < len(jobs):
            got = sv.wait(timeout=120.0)
            assert got, "server made no progress"
            comps.extend(got)
        stats = sv.batch_stats()
    finally:
        sv.close()
    out = {}
    for c in comps:
        k, st, arrs = keep[c.tag]
        assert c.status == blr.BLR_ERR_NOT_CONVERGED, c.message
        out[k] = (c.info.steps, c.info.r, c.info.err_ada, st.r, _factors(st, arrs))
    return out, stats


@pytest.fixture(scope="module")
def alone(helper):
    res = {}
    for k in range(len(REQS)):
        print(f"batched server, request {k} alone", flush=True)
        out, _ = _serve(helper, [(k, k)], slots=1)
        res[k] = out[k]
    return res


def test_result_is_the_same_alone_and_in_the_mix(helper, alone):
    print("batched server: 5 requests on 5 slots", flush=True)
    out, (rounds, jobs) = _serve(helper, [(k, k) for k in range(len(REQS))], slots=5)
    for k in range(len(REQS)):
        steps, r, err_ada, st_r, fac = out[k]
        a_steps, a_r, a_err, a_st_r, a_fac = alone[k]
        assert steps == a_steps and r == a_r == st_r == a_st_r
        assert err_ada == a_err
        for x, y in zip(fac, a_fac):
            assert np.array_equal(x, y)
    # four solves batch; their collisions shared batches
    print(f"batches {rounds}, collisions {jobs}", flush=True)
    assert rounds > 0 and jobs > rounds


def test_batched_agrees_with_unbatched_to_fp32_rounding(helper, alone):
    print("unbatched server: the same 5 requests", flush=True)
    out, (rounds, jobs) = _serve(helper, [(k, k) for k in range(len(REQS))], slots=5, batch=False)
    assert rounds == 0 and jobs == 0
    for k in range(len(REQS)):
        steps, r, err_ada, st_r, (X, S, V) = out[k]
        a_steps, a_r, a_err, _, (Xa, Sa, Va) = alone[k]
        assert steps == a_steps and r == a_r
        assert abs(err_ada - a_err) <= 1e-5 * a_err
        f = X.T @ S @ V
        fa = Xa.T @ Sa @ Va
        assert np.max(np.abs(f - fa)) <= 1e-6 * np.max(np.abs(fa))


def test_stopping_a_busy_batching_server_returns(helper):
    print("batched server: stop while busy", flush=True)
    sv = blr.Server(0, slots=3, batch_collisions=True)
    keep = []
    try:
        for k in range(3):
            d, n, m_rho, nx, r, mach, seed, dt, steps = REQS[k]
            pb, st, arrs = Req(d, n, m_rho, nx, r, mach, seed).device(helper)
            # a step small enough for the collisions' forward Euler to stay
            # stable over many steps
            sv.submit(pb, st, _solve_params(0.002, 100000), k)
            keep.append((pb, st, arrs))
        got = sv.wait(max_out=4, timeout=0.3)
        for c in got:
            print(f"early completion tag {c.tag}: status {c.status} steps {c.info.steps} "
                  f"{c.message}", flush=True)
        # a solve that ended this early ended in error
        assert all(c.status == blr.BLR_ERR_NOT_CONVERGED for c in got)
    finally:
        t0 = time.perf_counter()
        sv.close()   # must return
        print(f"close took {time.perf_counter() - t0:.3f} s", flush=True)


def test_batches_beyond_64_basis_functions(helper):
    """Four solves entering at rank 18-20 (22 with the added boundary
    functions): a batch holds more than 64 basis functions and runs as
    several launch sequences.  Each result is still the same alone and in the
    mix."""
    reqs = [(3, 16, 4, 24, 18 + k % 3, 1.4 + 0.2 * k, 20 + k, 0.01, 3) for k in range(4)]

    def serve(jobs, slots):
        sv = blr.Server(0, slots=slots, batch_collisions=True)
        keep, comps = {}, []
        try:
            for k in jobs:
                d, n, m_rho, nx, r, mach, seed, dt, steps = reqs[k]
                pb, st, arrs = Req(d, n, m_rho, nx, r, mach, seed, r_cap=24).device(helper)
                sv.submit(pb, st, _solve_params(dt, steps, r_max=24), k)
                keep[k] = (st, arrs)
            while len(comps) < len(jobs):
                got = sv.wait(timeout=120.0)
                assert got, "server made no progress"
                comps.extend(got)
            stats = sv.batch_stats()
        finally:
            sv.close()
        out = {}
        for c in comps:
            st, arrs = keep[c.tag]
            assert c.status == blr.BLR_ERR_NOT_CONVERGED, c.message
            out[c.tag] = (c.info.steps, c.info.r, c.info.err_ada, _factors(st, arrs))
        return out, stats

    print("batched server: 4 solves of rank 18-20, alone then together", flush=True)
    alone = {}
    for k in range(4):
        alone.update(serve([k], 1)[0])
    mix, (rounds, jobs) = serve(list(range(4)), 4)
    print(f"batches {rounds}, collisions {jobs}", flush=True)
    assert jobs > rounds
    for k in range(4):
        steps, r, err_ada, fac = mix[k]
        a_steps, a_r, a_err, a_fac = alone[k]
        assert steps == a_steps and r == a_r and err_ada == a_err
        for x, y in zip(fac, a_fac):
            assert np.array_equal(x, y)
