"""The serving loop (blr_server_*): steady solves admitted into slots as slots
and device memory free up, each slot a context with its own stream and host
thread.

* Each result is the same alone and in the mix: a solve run through a server
  beside other solves gives bit-identical factors, rank, step count and
  err_ada to the same solve run alone with blr_steady_solve on a fresh
  context (every kernel of the path reduces in a fixed order, so placement
  and overlap cannot change a result).
* The memory budget serialises admissions: with room for one solve only, a
  request is admitted after the previous one ended, and results are again
  identical.
* Errors stay per request; malformed or oversized requests are refused at
  submit; stopping a busy server drops its queue and returns.
The solves themselves are the steps parity-tested against the oracle in
test_gpu_dlr.py.
"""
import math
import os
import sys
import time

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

FLAGS = blr.BLR_STEP_ADD | blr.BLR_STEP_DROP


def _spec(d, n, m_rho, L=8.0):
    if d == 2:
        return synth.VGridSpec(d=2, n=n, L=L, gamma=0.0, C=1 / (2 * math.pi), m_rho=m_rho,
                               m_sigma=8)
    return synth.VGridSpec(d=3, n=n, L=L, gamma=1.0, C=1.0, m_rho=m_rho, m_sigma=38)


class Req:
    """One seeded shock solve: host factors and fresh device copies."""

    def __init__(self, d, n, m_rho, nx, r, mach, seed, r_cap=12):
        self.spec = _spec(d, n, m_rho)
        vs = oc.setup_from_spec(self.spec)
        ini = synth.shock_initial(mach, self.spec, nx, -30.0, 30.0, pert=1e-2, pert_rank=3,
                                  seed=seed)
        prob = dlr.Problem1D(vs=vs, nx=nx, x_lo=-30.0, x_hi=30.0, fL=ini["fL"], fR=ini["fR"])
        self.nx, self.n, self.r, self.r_cap = nx, vs.n, r, r_cap
        self.X, self.S, self.V = synth.lowrank_state(ini["f0"], r, prob.dx, prob.dvd)
        self.fL, self.fR = ini["fL"], ini["fR"]

    def device(self, ctx_like):
        dev = "cuda"
        X = torch.zeros((self.r_cap, self.nx), dtype=torch.float64, device=dev)
        S = torch.zeros((self.r_cap, self.r_cap), dtype=torch.float64, device=dev)
        V = torch.zeros((self.r_cap, self.n), dtype=torch.float64, device=dev)
        X[:self.r] = torch.tensor(self.X.T, device=dev)
        S[:self.r, :self.r] = torch.tensor(self.S, device=dev)
        V[:self.r] = torch.tensor(self.V, device=dev)
        fL = torch.tensor(self.fL, device=dev)
        fR = torch.tensor(self.fR, device=dev)
        vg = blr.vgrid_from_spec(self.spec)
        pb = ctx_like.make_problem(vg, self.nx, -30.0, 30.0, fL, fR)
        st = ctx_like.make_state(X, S, V, self.r)
        # this thread's stream only: a server may be recording a step graph on
        # another thread, and HIP refuses a device-wide synchronize meanwhile
        torch.cuda.current_stream().synchronize()
        return pb, st, (X, S, V)


def _solve_params(dt, steps, res_tol=1e-30, fp64=False, r_max=12):
    flags = FLAGS | (blr.BLR_STEP_FP64_COLLISION if fp64 else 0)
    return blr.SolveParams(blr.StepParams(dt, 0.2, 1e-10, 1, r_max, flags), res_tol, steps)


def _factors(st, arrs):
    r = st.r
    X, S, V = arrs
    return X[:r].cpu().numpy(), S[:r, :r].cpu().numpy(), V[:r].cpu().numpy()


REQS = [  # (d, n, m_rho, nx, r, mach, seed, dt, steps, fp64)
    (3, 16, 4, 24, 3, 1.5, 3, 0.02, 6, False),
    (2, 32, 8, 40, 4, 1.8, 4, 0.02, 9, False),
    (2, 16, 8, 24, 3, 1.3, 5, 0.03, 7, True),
    (2, 16, 8, 30, 5, 2.2, 6, 0.02, 5, False),
]


def _alone(case):
    d, n, m_rho, nx, r, mach, seed, dt, steps, fp64 = case
    q = Req(d, n, m_rho, nx, r, mach, seed)
    ctx = blr.Context(0)
    try:
        pb, st, arrs = q.device(ctx)
        info = ctx.steady_solve(pb, st, _solve_params(dt, steps, fp64=fp64), allow_unconverged=True)
        torch.cuda.synchronize()
        return info, st.r, _factors(st, arrs)
    finally:
        ctx.close()


@pytest.fixture(scope="module")
def alone():
    return [_alone(c) for c in REQS]


@pytest.fixture(scope="module")
def helper():
    c = blr.Context(0)   # make_problem / make_state only
    yield c
    c.close()


def _run_server(helper, server, jobs):
    """jobs: (case index, tag) pairs, submitted in order."""
    keep = {}
    for k, tag in jobs:
        d, n, m_rho, nx, r, mach, seed, dt, steps, fp64 = REQS[k]
        q = Req(d, n, m_rho, nx, r, mach, seed)
        pb, st, arrs = q.device(helper)
        server.submit(pb, st, _solve_params(dt, steps, fp64=fp64), tag)
        keep[tag] = (k, st, arrs)
    comps = []
    while len(comps) < len(jobs):
        got = server.wait(timeout=120.0)
        assert got, "server made no progress"
        comps.extend(got)
    return comps, keep


def _same(c, alone_k, st, arrs):
    info, r, fac = alone_k
    assert c.status == blr.BLR_ERR_NOT_CONVERGED, c.message
    assert c.info.steps == info.steps and c.info.r == info.r == st.r == r
    assert c.info.err_ada == info.err_ada
    for a, b in zip(_factors(st, arrs), fac):
        assert np.array_equal(a, b)


def test_result_is_the_same_alone_and_in_the_mix(helper, alone):
    print("server: 4 requests on 3 slots", flush=True)
    sv = blr.Server(0, slots=3)
    try:
        comps, keep = _run_server(helper, sv, [(k, k) for k in range(4)])
    finally:
        sv.close()
    slots = set()
    for c in comps:
        k, st, arrs = keep[c.tag]
        _same(c, alone[k], st, arrs)
        slots.add(c.slot)
        assert c.t_submit <= c.t_admit <= c.t_done
    assert len(slots) >= 2   # the work was spread over slots


def test_second_pass_on_warm_slots_is_identical(helper, alone):
    """Slots keep their workspace and recorded step graphs between requests;
    a request landing on a warm slot gives the same bits."""
    print("server: two passes on 2 slots", flush=True)
    sv = blr.Server(0, slots=2)
    try:
        c1, k1 = _run_server(helper, sv, [(3, 3), (2, 2), (1, 1), (0, 0)])
        c2, k2 = _run_server(helper, sv, [(k, 10 + k) for k in range(4)])
    finally:
        sv.close()
    for comps, keep in ((c1, k1), (c2, k2)):
        for c in comps:
            k, st, arrs = keep[c.tag]
            _same(c, alone[k], st, arrs)


def _estimate(helper, case):
    """The server's admission estimate for a case, read from the refusal of
    a server whose budget is one byte."""
    d, n, m_rho, nx, r, mach, seed, dt, steps, fp64 = REQS[case]
    sv = blr.Server(0, slots=1, hbm_budget=1)
    try:
        pb, st, _ = Req(d, n, m_rho, nx, r, mach, seed).device(helper)
        with pytest.raises(blr.BlrError) as ei:
            sv.submit(pb, st, _solve_params(dt, 1, fp64=fp64), 0)
        assert ei.value.code == blr.BLR_ERR_NOMEM
        return int(str(ei.value).split("needs ", 1)[1].split(" ")[0])
    finally:
        sv.close()


def test_memory_budget_admits_one_at_a_time(helper, alone):
    print("server: budget for one solve", flush=True)
    need = _estimate(helper, 0)
    assert need > 0
    sv = blr.Server(0, slots=2, hbm_budget=int(need * 1.5))   # room for one, not two
    try:
        comps, keep = _run_server(helper, sv, [(0, 0), (0, 1)])
    finally:
        sv.close()
    comps.sort(key=lambda c: c.t_admit)
    assert comps[1].t_admit >= comps[0].t_done
    for c in comps:
        k, st, arrs = keep[c.tag]
        _same(c, alone[k], st, arrs)


def test_errors_stay_with_their_request(helper, alone):
    sv = blr.Server(0, slots=2)
    try:
        d, n, m_rho, nx, r, mach, seed, dt, steps, fp64 = REQS[0]
        pb, st, arrs = Req(d, n, m_rho, nx, r, mach, seed).device(helper)
        before = _factors(st, arrs)
        sv.submit(pb, st, _solve_params(-1.0, 3), 100)          # bad dt: fails in the step
        comps, keep = _run_server(helper, sv, [(1, 1)])
        comps += sv.wait(timeout=60.0)
        by = {c.tag: c for c in comps}
        assert by[100].status == blr.BLR_ERR_ARG
        assert b"dt" in by[100].message and by[100].info.steps == 0
        for a, b in zip(_factors(st, arrs), before):
            assert np.array_equal(a, b)
        _same(by[1], alone[1], *keep[1][1:])
        # malformed requests are refused at submit
        bad = helper.make_state(arrs[0], arrs[1], arrs[2], 13)   # r > r_cap
        with pytest.raises(blr.BlrError) as ei:
            sv.submit(pb, bad, _solve_params(0.01, 1), 101)
        assert ei.value.code == blr.BLR_ERR_ARG
    finally:
        sv.close()


def test_stop_drops_the_queue(helper):
    print("server: stop with a queue", flush=True)
    sv = blr.Server(0, slots=1)
    keep = []
    d, n, m_rho, nx, r, mach, seed, dt, steps, fp64 = REQS[2]
    for k in range(4):
        pb, st, arrs = Req(d, n, m_rho, nx, r, mach, seed).device(helper)
        sv.submit(pb, st, _solve_params(dt, 100000, fp64=fp64), k)
        keep.append(arrs)
    time.sleep(0.5)
    queued, running = sv.load()
    assert running == 1 and queued == 3
    t0 = time.time()
    sv.close()
    assert time.time() - t0 < 30.0


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "steady_shock_2d.npz")


def _golden_problem():
    sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
    import make_steady_shock as mk
    return mk.SETUP, mk.problem()


@pytest.mark.parametrize("mode", ["fp32", "fp32_defect", "fp64"])
def test_served_steady_solve_matches_the_oracle(helper, mode):
    """A served steady solve (beside a second request on another slot) of the
    small Mach-1.4 shock against the oracle's steady solve of the same setup
    (tests/golden/make_steady_shock.py, err_ada <= 1e-6).

    Bounds on rho, u_1, T per cell, relative to their maxima: FP64
    collisions 1e-9 (rounding; the step itself agrees to 1e-12); FP32
    collisions 1e-4: FP32 and FP64 runs stop within a step of each other with
    moments 2-3e-5 apart, the FP32 error of Q_s piled up over the solve's
    1700 steps.  FP32 collisions with the FP64 defect correction (a refresh
    every 4 steps) are compared at the oracle's own stopping step (the solve
    marched exactly that many steps, since near the stopping point one step
    still moves the moments by about 1e-6): bound 2e-6.  The correction
    removes the part of the FP32 error that stays the same from step to step;
    the rest, the rounding that changes with every step, leaves 0.7-1.5e-6
    here (refresh every 2 to 4 steps, 2.5e-6 every 8), so the 1e-6 target for
    steady moments is reached only at about a refresh every 2 steps."""
    fp64 = mode == "fp64"
    if not os.path.exists(GOLDEN):
        pytest.skip("expected values not generated yet: run tests/golden/make_steady_shock.py")
    g = np.load(GOLDEN)
    s, (spec, prob, ini, (X, S, V)) = _golden_problem()
    print(f"served steady solve {mode}", flush=True)
    r_cap = 16
    dev = "cuda"
    Xd = torch.zeros((r_cap, s["nx"]), dtype=torch.float64, device=dev)
    Sd = torch.zeros((r_cap, r_cap), dtype=torch.float64, device=dev)
    Vd = torch.zeros((r_cap, prob.vs.n), dtype=torch.float64, device=dev)
    Xd[:s["r0"]] = torch.tensor(X.T, device=dev)
    Sd[:s["r0"], :s["r0"]] = torch.tensor(S, device=dev)
    Vd[:s["r0"]] = torch.tensor(V, device=dev)
    fL = torch.tensor(ini["fL"], device=dev)
    fR = torch.tensor(ini["fR"], device=dev)
    pb = helper.make_problem(blr.vgrid_from_spec(spec), s["nx"], s["x_lo"], s["x_hi"], fL, fR)
    st = helper.make_state(Xd, Sd, Vd, s["r0"])
    torch.cuda.synchronize()
    flags = blr.BLR_STEP_ADD | blr.BLR_STEP_DROP | (blr.BLR_STEP_FP64_COLLISION if fp64 else 0) | (
        blr.BLR_STEP_FP64_DEFECT if mode == "fp32_defect" else 0)
    at_oracle_step = mode == "fp32_defect"
    sp = blr.SolveParams(blr.StepParams(s["dt"], s["c"], s["add_tol"], 1, s["r_max"], flags),
                         0.0 if at_oracle_step else s["res_tol"],
                         int(g["steps"]) if at_oracle_step else s["max_steps"])
    sp.defect_every = 4
    sv = blr.Server(0, slots=2)
    try:
        other, okeep = _run_server(helper, sv, [(1, 1)])
        sv.submit(pb, st, sp, 7)
        comps = []
        while not any(c.tag == 7 for c in comps):
            got = sv.wait(timeout=240.0)
            assert got, "no progress"
            comps += got
    finally:
        sv.close()
    c = [c for c in comps if c.tag == 7][0]
    assert c.status == (blr.BLR_ERR_NOT_CONVERGED if at_oracle_step else blr.BLR_OK), c.message
    r = st.r
    fac = (Xd[:r].cpu().numpy().T, Sd[:r, :r].cpu().numpy(), Vd[:r].cpu().numpy())
    rho, u, T = dlr.macroscopic(dlr.State(*fac), prob)
    rel = [float(np.abs(a - b).max() / np.abs(b).max()) for a, b in
           ((rho, g["rho"]), (u, g["u"]), (T, g["T"]))]
    print("steps", c.info.steps, "oracle", int(g["steps"]), "r", r, int(g["r"]), "rel", rel,
          flush=True)
    assert bool(g["converged"])
    assert abs(c.info.steps - int(g["steps"])) <= (0 if fp64 else 0.02 * int(g["steps"]) + 2)
    assert max(rel) <= {"fp64": 1e-9, "fp32_defect": 2e-6, "fp32": 1e-4}[mode]
