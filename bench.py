"""Benchmark of the collision hot path on one MI355X.

Workload: a Mach-1.5 normal-shock state in low-rank form (N_x = 256 cells on
[-30, 30], N_v = 32^3 on [-8, 8]^3, hard spheres B = |v - v*|, 16 Gauss-
Legendre radial nodes x 38 Lebedev sphere nodes, rank 10).

  --mode step  (default) one step = one full adaptive low-rank time step:
               add the boundary basis (rank 10 -> 12), the 78 pair
               collisions Q_s(V_i, V_j) in FP32 (+ FP64 moment projection),
               K-step, S-step, L-step with FP64 QR, the residual, and the
               drop back to rank >= 10 (SVD of S).  value = pair collisions
               evaluated per second of whole steps.
  --mode pairs one step = the 55 pair collisions of the rank-10 basis alone.

The timed steps run as the library issues them by default (from the second
step of a configuration on, as a replayed HIP graph).  A second, shorter pass
of the same steps with the library's kernel events on gives the per-kernel
times and the roofline of the dominant kernel.

Full tensor: the reference step of the same discretisation on the full grid
(Q(f(x_p), f(x_p)) for all 256 cells, FP32 collisions, and upwind transport),
three timed steps, and its time over the low-rank step's.

Latency: the wall time of each timed step (p50, p99) on the batched FP32
path, and of three steps of the same workload on the plain FP64 per-pair
schedule.  A steady solve is a sequence of such steps (one host wait each),
so its latency is the step count times these; a steady state at this size
takes more than 10^4 steps, so no solve is timed here.

Prints ONE JSON line (rank 0, N = 1 only).  Inputs are resident in HBM before
the timed region starts.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, published


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--mode", choices=["pairs", "step"], default="step")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-parity", action="store_true",
                    help="skip the comparison with the oracle's stored values (tests/golden)")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-full", action="store_true",
                    help="skip the full-tensor reference step (N_x collisions per step)")
    ap.add_argument("--generic", action="store_true", help="force the multi-pass FFT path")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving traces")
    ap.add_argument("--no-carleman", action="store_true",
                    help="skip the Carleman-form measurement")
    ap.add_argument("--paper-shock", action="store_true",
                    help="also solve the paper's normal shock (2D velocity, 32^2, N_x = 1000; "
                         "Mach from --paper-shock-mach) to steady state by the low-rank and the "
                         "full-tensor method (minutes)")
    ap.add_argument("--paper-tol", type=float, default=1e-6)
    ap.add_argument("--paper-shock-mach", type=float, default=1.4,
                    help="Mach number of --paper-shock: 1.4 (L_v = 13.11) or 3.8 (L_v = 20.97), "
                         "the paper's 32^2 shapes")
    ap.add_argument("--paper-shock-lv", type=float, default=13.11,
                    help="velocity half width for another Mach number")
    ap.add_argument("--paper-dealias", action="store_true",
                    help="de-aliased collision products in --paper-shock (always at Mach >= 3)")
    ap.add_argument("--paper-fourier", action="store_true",
                    help="also solve the paper's Fourier flow (diffusive walls at T = 1 and 1.2, "
                         "N_x = 200, 2D velocity 32^2) to err <= --fourier-tol by the low-rank "
                         "and the full-tensor method (minutes)")
    ap.add_argument("--fourier-tol", type=float, default=2e-7)
    ap.add_argument("--c4", action="store_true",
                    help="also run the 2D-space x 3D-velocity adaptive workload with an obstacle at "
                         "12 x 12 cells (24^3 velocity) by the low-rank and the full-tensor method")
    ap.add_argument("--c4-steps", type=int, default=200)
    ap.add_argument("--paper-cavity", action="store_true",
                    help="also solve the paper's lid-driven cavity (all walls diffusive, lid "
                         "u_w = (1, 0)) on 16 x 16 cells, 2D velocity 32^2, by the low-rank and "
                         "the full-tensor method (minutes)")
    ap.add_argument("--paper-thermal", action="store_true",
                    help="also solve the paper's thermally driven cavity on 16 x 16 cells (walls "
                         "y = 0, 2 at T linear in x from 1 to 1.2) by both methods (minutes)")
    ap.add_argument("--cavity-tol", type=float, default=2e-7)
    ap.add_argument("--cavity-cap", type=float, default=300.0,
                    help="wall-clock cap in seconds per method of the cavity")
    ap.add_argument("--cavity-rmax", type=int, default=30)
    ap.add_argument("--fourier-cap", type=float, default=420.0,
                    help="wall-clock cap in seconds per method of the Fourier flow")
    ap.add_argument("--serve-count", type=int, default=8,
                    help="requests of the trace both paths run")
    ap.add_argument("--serve-steps", type=int, default=10,
                    help="step cap per solve in the trace both paths run")
    ap.add_argument("--serve-long-count", type=int, default=16,
                    help="requests of the longer trace (batched path only; 0 skips it)")
    ap.add_argument("--serve-long-steps", type=int, default=200)
    ap.add_argument("--serve-slots", type=int, default=4)
    ap.add_argument("--serve-conv-count", type=int, default=8,
                    help="requests of the trace run to err_ada <= 1e-6 (2D velocity; 0 skips it)")
    ap.add_argument("--serve-conv-plain", type=int, default=1,
                    help="how many of them the plain FP64 FIFO serves")
    ap.add_argument("--serve-conv-cap", type=int, default=40000)
    ap.add_argument("--steady-compare", type=int, default=0,
                    help="also run the converged trace's first solve for this many steps with FP32 "
                         "and with FP64 collisions (no stopping rule) and compare the moments")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain 256 MiB device copy (counter calibration)")
    ap.add_argument("--traffic", default=os.path.join(ROOT, "profiles", "traffic.json"),
                    help="HBM traffic per launch from rocprofv3 counters (if present)")
    return ap.parse_args()


def read_timers(ctx):
    lib = ctx.lib
    out = []
    buf = ctypes.create_string_buffer(256)
    ms = ctypes.c_double()
    nl = ctypes.c_int64()
    by = ctypes.c_double()
    i = 0
    while lib.blr_timing_read(ctx.h, i, buf, 256, ctypes.byref(ms), ctypes.byref(nl),
                              ctypes.byref(by)) == 0:
        out.append(dict(name=buf.value.decode(), ms=ms.value, launches=nl.value, bytes=by.value))
        i += 1
    return out


def pct(xs, q):
    xs = sorted(xs)
    return xs[min(len(xs) - 1, int(math.ceil(q * len(xs))) - 1)]


def prepare_trace(trace, synth):
    """Initial low-rank factors of each request of a serving trace (host,
    before any clock): shock data of the request's Mach number, truncated to
    its initial rank."""
    out = []
    for q in trace:
        d = q.get("d", 3)
        if d == 3:
            spec = synth.VGridSpec(d=3, n=q["n"], L=q["L"], gamma=1.0, C=1.0, m_rho=16, m_sigma=38)
        else:
            spec = synth.VGridSpec(d=2, n=q["n"], L=q["L"], gamma=0.0, C=1.0 / (2.0 * math.pi),
                                   m_rho=8, m_sigma=8)
        ini = synth.shock_initial(q["mach"], spec, q["nx"], q["x_lo"], q["x_hi"], pert=1e-3,
                                  pert_rank=10 if d == 3 else 3, seed=100 + q["index"])
        dx = (q["x_hi"] - q["x_lo"]) / q["nx"]
        dvd = (2.0 * q["L"] / q["n"]) ** d
        X, S, V = synth.lowrank_state_sketch(ini["f0"], q["r0"], dx, dvd, seed=q["index"])
        out.append(dict(q=q, spec=spec, X=X, S=S, V=V, fL=ini["fL"], fR=ini["fR"]))
    return out


def progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def run_trace(blr, torch, helper, prepared, slots, plain, cap, r_cap=30, res_tol=1e-6,
              moments_of=(), batch=False, fp64=False, defect=False):
    """Serve the requests at their arrival times; latency = completion time -
    arrival (submit) time on the server's clock.  For the request indices in
    moments_of, the steady rho, u_1, T per cell are returned as well."""
    dev = torch.device("cuda:0")

    def device_request(p):
        q = p["q"]
        r = q["r0"]
        X = torch.zeros((r_cap, q["nx"]), dtype=torch.float64, device=dev)
        S = torch.zeros((r_cap, r_cap), dtype=torch.float64, device=dev)
        V = torch.zeros((r_cap, p["V"].shape[1]), dtype=torch.float64, device=dev)
        X[:r] = torch.tensor(p["X"].T, device=dev)
        S[:r, :r] = torch.tensor(p["S"], device=dev)
        V[:r] = torch.tensor(p["V"], device=dev)
        fL = torch.tensor(p["fL"], device=dev)
        fR = torch.tensor(p["fR"], device=dev)
        vg = blr.vgrid_from_spec(p["spec"], blr.BLR_PLAIN_SCHEDULE if plain else 0)
        pb = helper.make_problem(vg, q["nx"], q["x_lo"], q["x_hi"], fL, fR)
        st = helper.make_state(X, S, V, r)
        return pb, st

    def params(q, steps):
        flags = blr.BLR_STEP_ADD | blr.BLR_STEP_DROP | (
            blr.BLR_STEP_FP64_COLLISION if (plain or fp64) else 0) | (
            blr.BLR_STEP_FP64_DEFECT if defect else 0)
        p = blr.SolveParams(blr.StepParams(q["dt"], 0.2, 1e-10, 1, r_cap, flags), res_tol, steps)
        p.defect_every = 4
        return p

    progress(f"serving trace: {len(prepared)} requests, {slots} slot(s), "
             f"{'plain fp64' if plain else ('batched fp64' if fp64 else 'batched fp32')}"
             f"{' with the fp64 defect correction' if defect else ''}"
             f"{', collisions of all live solves in shared launches' if batch else ''}, "
             f"cap {cap} steps")
    sv = blr.Server(0, slots=slots, batch_collisions=batch)
    bstats = (0, 0)
    try:
        # warm-up (untimed): every slot runs two steps of the largest-rank
        # request of each velocity grid (allocations, tables, recorded graphs)
        tag = -1
        for nv in sorted({p["q"]["n"] for p in prepared}):
            big = max((p for p in prepared if p["q"]["n"] == nv), key=lambda p: p["q"]["r0"])
            for _ in range(slots):
                pb, st = device_request(big)
                # this thread's stream only: a slot may be recording a step graph,
                # and HIP refuses a device-wide synchronize meanwhile
                torch.cuda.current_stream().synchronize()
                sv.submit(pb, st, params(big["q"], 2), tag)
                tag -= 1
            got = 0
            while got < slots:
                got += len(sv.wait(timeout=300.0))
        reqs = [device_request(p) for p in prepared]
        torch.cuda.synchronize()
        comps = []
        t0 = time.perf_counter()
        i = 0
        while len(comps) < len(reqs):
            now = time.perf_counter() - t0
            while i < len(reqs) and prepared[i]["q"]["arrival"] <= now:
                sv.submit(reqs[i][0], reqs[i][1], params(prepared[i]["q"], cap), i)
                i += 1
            if i < len(reqs):
                wait = max(0.0, prepared[i]["q"]["arrival"] - (time.perf_counter() - t0))
                if sv.load() == (0, 0):
                    time.sleep(wait)   # nothing live: idle until the next arrival
                else:
                    comps += sv.wait(timeout=wait)
            else:
                got = sv.wait(timeout=600.0)
                if not got:
                    raise RuntimeError("serving trace made no progress")
                comps += got
        wall = time.perf_counter() - t0
        bstats = sv.batch_stats()
    finally:
        sv.close()
    lat = [c.t_done - c.t_submit for c in comps]
    ok = [c for c in comps if c.status in (blr.BLR_OK, blr.BLR_ERR_NOT_CONVERGED)]
    moments = {}
    import numpy as np
    for i in moments_of:
        st = reqs[i][1]
        X, S, V = (t.cpu().numpy() for t in st._keep)
        r = st.r
        F = (X[:r].T @ S[:r, :r]) @ V[:r]
        sp = prepared[i]["spec"]
        v = synth_vgrid(sp).reshape(sp.d, -1)
        w = (2.0 * sp.L / sp.n) ** sp.d
        rho = F.sum(axis=1) * w
        u = (F * v[0]).sum(axis=1) * w / rho
        e2 = (F * (v ** 2).sum(axis=0)).sum(axis=1) * w / rho
        # |u|^2 over every velocity component
        uu = sum(((F * v[k]).sum(axis=1) * w / rho) ** 2 for k in range(sp.d))
        moments[i] = (rho, u, (e2 - uu) / sp.d)
    out = {"slots": slots, "requests": len(comps), "step_cap": cap,
            "latency_s_p50": round(pct(lat, 0.50), 4), "latency_s_p99": round(pct(lat, 0.99), 4),
            "queue_wait_s_p50": round(pct([c.t_admit - c.t_submit for c in comps], 0.5), 4),
            "wall_s": round(wall, 3), "solves_per_s": round(len(comps) / wall, 3),
            "steps": int(sum(c.info.steps for c in comps)),
            "pair_evals": int(sum(c.info.pair_evals for c in comps)),
            "pair_evals_per_s": round(sum(c.info.pair_evals for c in comps) / wall, 1),
            "converged": sum(1 for c in comps if c.status == blr.BLR_OK),
            "failed": len(comps) - len(ok),
            "final_rank_range": [min(c.info.r for c in ok), max(c.info.r for c in ok)] if ok else None,
            "final_err_ada": max(c.info.err_ada for c in ok) if ok else None}
    if len(comps) <= 16:
        # per request: index, slot, submit, admit and done times (s), steps
        out["requests_detail"] = [[c.tag, c.slot, round(c.t_submit, 4), round(c.t_admit, 4),
                                   round(c.t_done, 4), c.info.steps] for c in comps]
    if batch:
        # the warm-up's batches included
        out["collision_batches"] = bstats[0]
        out["step_collisions_in_batches"] = bstats[1]
    if moments_of:
        return out, moments
    return out


def synth_vgrid(spec):
    import synth
    return synth.vgrid_points(spec.d, spec.n, spec.L)


def carleman_leg(args, blr, synth, torch, ctx, lib, spec, V, X, S, ini, nx, r, r_cap, dt):
    """The same workload with the Carleman form of the operator (the paper's
    fast algorithm for 3D hard spheres): the 55 pair collisions of the
    rank-10 basis, and the adaptive step on them; per-kernel times; the
    two forms are different discretisations of one operator (see the design
    notes for how far apart they are on this basis)."""
    dev = torch.device("cuda:0")
    pairs = blr.upper_pairs(r)
    P = len(pairs)
    vgc = blr.vgrid_from_spec(spec, blr.BLR_CARLEMAN)
    V32 = torch.tensor(V, dtype=torch.float32, device=dev)
    Q = torch.empty((P, V.shape[1]), dtype=torch.float32, device=dev)
    for _ in range(2):
        ctx.collision_pairs(vgc, V32, pairs, out=Q)
    torch.cuda.synchronize()
    reps = 10
    t0 = time.perf_counter()
    for _ in range(reps):
        ctx.collision_pairs(vgc, V32, pairs, out=Q)
    torch.cuda.synchronize()
    coll_rate = reps * P / (time.perf_counter() - t0)
    # per-kernel times of the collision batch
    lib.blr_timing(ctx.h, 2)
    lib.blr_timing(ctx.h, 1)
    ctx.collision_pairs(vgc, V32, pairs, out=Q)
    torch.cuda.synchronize()
    lib.blr_timing(ctx.h, 0)
    timers = read_timers(ctx)
    # the adaptive step with Carleman collisions
    Xd = torch.zeros((r_cap, nx), dtype=torch.float64, device=dev)
    Sd = torch.zeros((r_cap, r_cap), dtype=torch.float64, device=dev)
    Vd = torch.zeros((r_cap, V.shape[1]), dtype=torch.float64, device=dev)
    Xd[:r] = torch.tensor(X.T, device=dev)
    Sd[:r, :r] = torch.tensor(S, device=dev)
    Vd[:r] = torch.tensor(V, device=dev)
    fL = torch.tensor(ini["fL"], device=dev)
    fR = torch.tensor(ini["fR"], device=dev)
    pb = ctx.make_problem(vgc, nx, -30.0, 30.0, fL, fR)
    st = ctx.make_state(Xd, Sd, Vd, r, seed=1)
    sp = blr.StepParams(dt, 0.2, 1e-10, r, r_cap, blr.BLR_STEP_ADD | blr.BLR_STEP_DROP)
    for _ in range(3):
        ctx.dlr_step(pb, st, sp)
    torch.cuda.synchronize()
    wall, counted = [], 0
    for _ in range(max(5, args.steps)):
        ts = time.perf_counter()
        info = ctx.dlr_step(pb, st, sp)
        wall.append(time.perf_counter() - ts)
        rr = info.r_in + info.r_added
        counted += rr * (rr + 1) // 2
    return {"form": "Carleman (constant kernel 4C for hard spheres, 19 directions of the "
                    "Lebedev-38 rule, no radial quadrature)",
            "collision_only_pair_evals_per_s": round(coll_rate, 1),
            "step_pair_evals_per_s": round(counted / sum(wall), 1),
            "step_ms_p50": round(1e3 * pct(wall, 0.5), 4),
            "step_ms_p99": round(1e3 * pct(wall, 0.99), 4),
            "kernels": [{k: (round(v, 4) if isinstance(v, float) else v) for k, v in t.items()}
                        for t in sorted(timers, key=lambda t: -t["ms"])[:6]]}


def paper_shock_leg(args, blr, synth, torch, ctx):
    """The normal shock of Sec. 5.2 at the paper's shapes: d = 2, Maxwell
    molecules B = 1/(2 pi) with the Carleman form (8 directions), N_v = 32^2
    on [-L_v, L_v]^2 (L_v = 13.11 at Mach 1.4, 20.97 at Mach 3.8), N_x = 1000
    on [-30, 30], the tanh initial profile (alpha = 0.5) without
    perturbation, dt = dx / (2 L_v); de-aliased products at Mach >= 3.
    Both methods run to err <= tol (err_ada for the low-rank method, adaptive
    with c = 0.2; err_full for the full tensor); the macroscopic profiles of
    the two steady states are compared, and the density with the Mott-Smith
    logistic profile of Sec. 4 (alpha from the same pair operator)."""
    import numpy as np
    # the paper's box half widths: 13.11 (Mach 1.4), 20.97 (Mach 3.8) at 32^2
    mach, nx, N = args.paper_shock_mach, 1000, 32
    L = {1.4: 13.11, 3.8: 20.97}.get(round(mach, 2), args.paper_shock_lv)
    # the circular products make the cold upstream Maxwellian of the strong
    # shock (T = 1 on a grid of spacing 1.31) a growing mode of the discrete
    # operator; the de-aliased (Galerkin) products do not
    dealias = args.paper_dealias or mach >= 3.0
    cflags = blr.BLR_CARLEMAN | (blr.BLR_DEALIAS if dealias else 0)
    dev = torch.device("cuda:0")
    spec = synth.VGridSpec(d=2, n=N, L=L, gamma=0.0, C=1 / (2 * math.pi), m_rho=1, m_sigma=8)
    ini = synth.shock_initial(mach, spec, nx, -30.0, 30.0, pert=0.0, pert_rank=0)
    dx, dv = 60.0 / nx, 2 * L / N
    dt = 0.5 * dx / L
    vg = blr.vgrid_from_spec(spec, cflags)
    fL = torch.tensor(ini["fL"], device=dev)
    fR = torch.tensor(ini["fR"], device=dev)
    pb = ctx.make_problem(vg, nx, -30.0, 30.0, fL, fR)
    v = synth.vgrid_points(2, N, L).reshape(2, -1)

    def macro(F):
        w = dv * dv
        rho = F.sum(axis=1) * w
        u = (F * v[0]).sum(axis=1) * w / rho
        E = 0.5 * (F * (v ** 2).sum(axis=0)).sum(axis=1) * w
        T = (2 * E / rho - u * u) / 2
        return rho, u, T

    # low-rank steady solve (one library call)
    r0, rc = 4, 32
    X, S, V = synth.lowrank_state_sketch(ini["f0"], r0, dx, dv * dv, seed=1)
    Xd = torch.zeros((rc, nx), dtype=torch.float64, device=dev)
    Sd = torch.zeros((rc, rc), dtype=torch.float64, device=dev)
    Vd = torch.zeros((rc, N * N), dtype=torch.float64, device=dev)
    Xd[:r0] = torch.tensor(X.T, device=dev)
    Sd[:r0, :r0] = torch.tensor(S, device=dev)
    Vd[:r0] = torch.tensor(V, device=dev)
    st = ctx.make_state(Xd, Sd, Vd, r0)
    torch.cuda.synchronize()
    sp = blr.SolveParams(blr.StepParams(dt, 0.2, 1e-10, 1, 30,
                                        blr.BLR_STEP_ADD | blr.BLR_STEP_DROP), args.paper_tol,
                         400000)
    progress(f"paper shock (Mach {mach}): low-rank solve to {args.paper_tol}")
    t0 = time.perf_counter()
    # in pieces of 20000 steps (a progress line per piece), up to 400000 steps
    sp.max_steps = 20000
    steps_lr = 0
    while True:
        li = ctx.steady_solve(pb, st, sp, allow_unconverged=True)
        steps_lr += li.steps
        progress(f"  low rank: {steps_lr} steps, err_ada {li.err_ada:.3e}, rank {li.r}")
        if li.converged or steps_lr >= 400000:
            break
    li.steps = steps_lr
    t_lr = time.perf_counter() - t0
    r = st.r
    F_lr = (Xd[:r].cpu().numpy().T @ Sd[:r, :r].cpu().numpy()) @ Vd[:r].cpu().numpy()
    # full-tensor solve (one library call per step)
    progress(f"paper shock: full-tensor solve to {args.paper_tol}")
    F = torch.tensor(ini["f0"], device=dev)
    t0 = time.perf_counter()
    steps_full, e = 0, float("inf")
    t_prog = t0
    while e > args.paper_tol and steps_full < 400000 and time.perf_counter() - t0 < 900:
        e = ctx.full_step(pb, F, dt, blr.BLR_FP32)
        steps_full += 1
        if time.perf_counter() - t_prog > 30:
            t_prog = time.perf_counter()
            progress(f"  full tensor: {steps_full} steps, err_full {e:.3e}")
    t_full = time.perf_counter() - t0
    F_full = F.cpu().numpy()
    m_lr, m_full = macro(F_lr), macro(F_full)
    prof = {nm: float(np.abs(a - b).max() / np.abs(b).max())
            for nm, a, b in zip(("rho", "u", "T"), m_lr, m_full)}
    # Mott-Smith: alpha from the pair operator on (f_L, f_R), logistic profile
    # centred where the low-rank density crosses the mean of the end states
    Vb = torch.stack([fL, fR])
    q = ctx.collision_pairs(blr.vgrid_from_spec(spec, cflags | blr.BLR_NO_CONSERVE),
                            Vb, [(0, 1)]).cpu().numpy()[0]
    alpha = float(2 * dv * dv * np.dot(v[0] ** 2, q))
    (rl, ul, Tl), (rr, ur, Tr) = ini["states"]
    beta = alpha / (1 * rl * ul * (Tl - Tr))
    x = ini["x"]
    rho = m_lr[0]
    mid = 0.5 * (rl + rr)
    kx = int(np.argmax(rho >= mid))
    x0 = x[kx - 1] + (mid - rho[kx - 1]) * (x[kx] - x[kx - 1]) / (rho[kx] - rho[kx - 1])
    a = 1.0 / (np.exp(beta * (x - x0)) + 1.0)
    rho_ms = a * rl + (1 - a) * rr
    # thickness: max density slope of each profile, over the jump
    thick = lambda rr_: (rr - rl) / np.max(np.gradient(rr_, x))
    return {"shape": f"Mach {mach}, d=2 Maxwell molecules (Carleman form, 8 directions"
                     f"{', de-aliased products' if dealias else ''}), "
                     f"N_v=32^2 on [-{L},{L}]^2, N_x=1000 on [-30,30], dt=dx/(2 L_v), tanh initial "
                     "profile, FP32 collisions",
            "tol": args.paper_tol,
            "low_rank": {"steps": int(li.steps), "converged": int(li.converged),
                         "err_ada": li.err_ada, "rank": int(li.r), "seconds": round(t_lr, 2),
                         "ms_per_step": round(1e3 * t_lr / max(1, li.steps), 4)},
            "full_tensor": {"steps": steps_full, "converged": int(e <= args.paper_tol),
                            "err_full": e, "seconds": round(t_full, 2),
                            "ms_per_step": round(1e3 * t_full / max(1, steps_full), 4)},
            "time_ratio_full_over_low_rank": round(t_full / t_lr, 2),
            "profile_rel_diff_low_rank_vs_full": prof,
            "mott_smith": {"alpha": alpha, "beta": beta,
                           "density_max_rel_dev": float(np.abs(rho - rho_ms).max() / (rr - rl)),
                           "thickness_numerical": float(thick(rho)),
                           "thickness_mott_smith": float(thick(rho_ms))}}


def c4_leg(args, blr, synth, torch, ctx):
    """The 2D-space x 3D-velocity adaptive workload with an obstacle (the
    rectangle of Sec. 2.2, the walls of Sec. 2.3 on the obstacle's faces) at
    a reduced grid: [0, 1]^2 with 12 x 12 cells (the full 64 x 64 would need
    256 boundary rows in the augmentation, which takes 64; here 2 (12 + 12)
    + the obstacle's 12 faces = 60).  A square obstacle of 3 x 3 cells whose
    lower-left cell is drawn from [4, 6]^2 (seed 4), its faces Maxwell
    diffusive walls at T_w = 2; inflow Mach 2 on every outer face, (rho, u_1,
    T) = (1, 2 sqrt(5/3), 1); 3D velocity 24^3 on [-8, 8]^3, hard spheres
    (C = 1), M_rho = 16 x M_sigma = 38, FP32 collisions; the free stream at
    rank 1 to start, adaptive with r_max = 30, c = 0.2; dt = 1/2 min(0.35 dx
    / L_v, 1.5 / nu), nu = 4 pi C R rho_max with rho_max = 3.  The low-rank
    method and the full tensor run the same number of steps; their
    macroscopic fields are compared at the end."""
    import numpy as np
    nx = ny = 12
    spec = synth.VGridSpec(d=3, n=24, L=8.0, gamma=1.0, C=1.0, m_rho=16, m_sigma=38)
    rng = np.random.default_rng(4)
    i0, j0 = (int(x) for x in rng.integers(4, 7, size=2))
    solid = np.zeros((nx, ny), dtype=bool)
    solid[i0:i0 + 3, j0:j0 + 3] = True
    dev = torch.device("cuda:0")
    v = synth.vgrid_points(3, spec.n, spec.L)
    u_in = 2.0 * math.sqrt(5.0 / 3.0)
    f_in = synth.maxwellian(v, 1.0, (u_in, 0.0, 0.0), 1.0).reshape(-1)
    f_w = synth.maxwellian(v, 1.0, (0.0, 0.0, 0.0), 2.0).reshape(-1)
    dx = 1.0 / nx
    R = 4.0 * spec.L / (3.0 + math.sqrt(2.0))
    dt = 0.5 * min(0.35 * dx / spec.L, 1.5 / (4.0 * math.pi * 1.0 * R * 3.0))
    fin = torch.tensor(f_in, device=dev)
    obs = torch.tensor(f_w, device=dev)
    vg = blr.vgrid_from_spec(spec)
    pb = ctx.make_problem2d(vg, nx, ny, 0.0, 1.0, 0.0, 1.0, [(fin, False)] * 4, solid=solid,
                            obstacle=obs)
    gas = ~solid.reshape(-1)
    F0 = np.outer(gas.astype(np.float64), f_in)
    vv = v.reshape(3, -1)
    w = (2 * spec.L / spec.n) ** 3

    def macro(F):
        rho = F.sum(axis=1) * w
        safe = np.where(rho > 0, rho, 1.0)
        u1 = (F * vv[0]).sum(axis=1) * w / safe
        e2 = (F * (vv ** 2).sum(axis=0)).sum(axis=1) * w / safe
        return rho, u1, (e2 - u1 * u1) / 3.0

    rc = 30
    X, S, V = synth.lowrank_state(F0, 1, dx * dx, w)
    Xd = torch.zeros((rc, nx * ny), dtype=torch.float64, device=dev)
    Sd = torch.zeros((rc, rc), dtype=torch.float64, device=dev)
    Vd = torch.zeros((rc, spec.npts), dtype=torch.float64, device=dev)
    Xd[:1] = torch.tensor(X.T, device=dev)
    Sd[:1, :1] = torch.tensor(S, device=dev)
    Vd[:1] = torch.tensor(V, device=dev)
    st = ctx.make_state(Xd, Sd, Vd, 1)
    torch.cuda.synchronize()
    sp = blr.StepParams(dt, 0.2, 1e-10, 1, rc, blr.BLR_STEP_ADD | blr.BLR_STEP_DROP)
    nsteps = args.c4_steps
    ranks, pairs, times = [], 0, []
    progress(f"C4 reduced: {nsteps} low-rank steps (12 x 12 cells, 24^3, obstacle at {i0},{j0})")
    t0 = time.perf_counter()
    for k in range(nsteps):
        ts = time.perf_counter()
        info = ctx.dlr_step(pb, st, sp)
        times.append(time.perf_counter() - ts)
        rk = info.r_in + info.r_added
        pairs += rk * (rk + 1) // 2
        ranks.append(int(info.r_out))
        if k % 50 == 0 or k == nsteps - 1:
            progress(f"  step {k}: err_ada {info.err_ada:.3e}, rank {info.r_in}+{info.r_added}->"
                     f"{info.r_out}")
    t_lr = time.perf_counter() - t0
    r = st.r
    F_lr = (Xd[:r].cpu().numpy().T @ Sd[:r, :r].cpu().numpy()) @ Vd[:r].cpu().numpy()
    progress(f"C4 reduced: {nsteps} full-tensor steps")
    F = torch.tensor(F0, device=dev)
    t0 = time.perf_counter()
    for k in range(nsteps):
        e = ctx.full_step(pb, F, dt, blr.BLR_FP32)
    t_full = time.perf_counter() - t0
    m_lr, m_full = macro(F_lr), macro(F.cpu().numpy())
    diffs = {nm: float(np.abs(a[gas] - b[gas]).max() / np.abs(b[gas]).max())
             for nm, a, b in zip(("rho", "u1", "T"), m_lr, m_full)}
    times.sort()
    return {"shape": f"[0,1]^2 with 12 x 12 cells, 3x3 obstacle at cells ({i0},{j0}) (diffusive wall "
                     "T_w=2), inflow Mach 2 on every outer face, 3D velocity 24^3 on [-8,8]^3, hard "
                     "spheres M_rho=16 x M_sigma=38, FP32 collisions, adaptive r_max=30, c=0.2",
            "dt": dt, "steps": nsteps,
            "low_rank": {"seconds": round(t_lr, 3), "ms_per_step": round(1e3 * t_lr / nsteps, 3),
                         "step_ms_p50": round(1e3 * times[len(times) // 2], 3),
                         "pair_evals": pairs, "pair_evals_per_s": round(pairs / t_lr, 1),
                         "final_rank": int(r), "rank_max": max(ranks),
                         "err_ada_last": info.err_ada},
            "full_tensor": {"seconds": round(t_full, 3),
                            "ms_per_step": round(1e3 * t_full / nsteps, 3), "err_full_last": e},
            "low_rank_vs_full_max_rel_diff": diffs}


def fourier_leg(args, blr, synth, torch, ctx):
    """The Fourier flow of Sec. 5.3: x in [0, 2] with N_x = 200, 2D velocity
    32^2 on [-7.86, 7.86]^2, Maxwell diffusive walls at rest with T_w = 1
    (x = 0) and 1.2 (x = 2), initial Maxwellian rho = 1, u = 0, T = 1; Maxwell
    molecules B = 1/(2 pi) in the Carleman form (8 directions), FP32
    collisions, dt = dx / (2 L_v).  Both methods run to err <= tol (the
    paper's res_tol 2e-7): the adaptive low-rank method (c = 0.2) from the
    rank-1 initial state, and the full tensor; the temperature profiles of the
    two steady states are compared and the rank history reported."""
    import numpy as np
    spec = synth.FOURIER
    nx, N, L = 200, spec.n, spec.L
    dev = torch.device("cuda:0")
    dx, dv = 2.0 / nx, 2 * L / N
    dt = 0.5 * dx / L
    tol = args.fourier_tol
    ini = synth.wall_initial(spec, nx, 0.0, 2.0, T_walls=(1.0, 1.2))
    vg = blr.vgrid_from_spec(spec, blr.BLR_CARLEMAN)
    fL = torch.tensor(ini["fL"], device=dev)
    fR = torch.tensor(ini["fR"], device=dev)
    pb = ctx.make_problem(vg, nx, 0.0, 2.0, fL, fR, wall_left=True, wall_right=True)
    v = synth.vgrid_points(2, N, L).reshape(2, -1)

    def temperature(F):
        w = dv * dv
        rho = F.sum(axis=1) * w
        u1 = (F * v[0]).sum(axis=1) * w / rho
        u2 = (F * v[1]).sum(axis=1) * w / rho
        E = 0.5 * (F * (v ** 2).sum(axis=0)).sum(axis=1) * w
        return (2 * E / rho - u1 * u1 - u2 * u2) / 2, rho

    # low-rank: steady solves of `chunk` steps until converged (a progress
    # line between chunks; the state and its rank carry over)
    rc, chunk = 32, 10000
    X, S, V = synth.lowrank_state(ini["f0"], 1, dx, dv * dv)
    Xd = torch.zeros((rc, nx), dtype=torch.float64, device=dev)
    Sd = torch.zeros((rc, rc), dtype=torch.float64, device=dev)
    Vd = torch.zeros((rc, N * N), dtype=torch.float64, device=dev)
    Xd[:1] = torch.tensor(X.T, device=dev)
    Sd[:1, :1] = torch.tensor(S, device=dev)
    Vd[:1] = torch.tensor(V, device=dev)
    st = ctx.make_state(Xd, Sd, Vd, 1)
    torch.cuda.synchronize()
    sp = blr.SolveParams(blr.StepParams(dt, 0.2, 1e-10, 1, rc,
                                        blr.BLR_STEP_ADD | blr.BLR_STEP_DROP), tol, chunk)
    steps_lr, ranks, conv_lr, li = 0, [], False, None
    t0 = time.perf_counter()
    while not conv_lr and time.perf_counter() - t0 < args.fourier_cap:
        li = ctx.steady_solve(pb, st, sp, allow_unconverged=True)
        steps_lr += int(li.steps)
        conv_lr = bool(li.converged)
        ranks.append([steps_lr, int(li.r)])
        progress(f"fourier: low-rank {steps_lr} steps, err_ada {li.err_ada:.3e}, rank {li.r}")
    t_lr = time.perf_counter() - t0
    r = st.r
    F_lr = (Xd[:r].cpu().numpy().T @ Sd[:r, :r].cpu().numpy()) @ Vd[:r].cpu().numpy()
    # full tensor: one library call per step
    F = torch.tensor(ini["f0"], device=dev)
    steps_full, e = 0, float("inf")
    t0 = last = time.perf_counter()
    while e > tol and time.perf_counter() - t0 < args.fourier_cap:
        e = ctx.full_step(pb, F, dt, blr.BLR_FP32)
        steps_full += 1
        if time.perf_counter() - last > 20.0:
            last = time.perf_counter()
            progress(f"fourier: full tensor {steps_full} steps, err_full {e:.3e}")
    t_full = time.perf_counter() - t0
    T_lr, rho_lr = temperature(F_lr)
    T_full, rho_full = temperature(F.cpu().numpy())
    conv_full = e <= tol
    return {"shape": "Fourier flow: x in [0,2], N_x=200, 2D velocity 32^2 on [-7.86,7.86]^2, "
                     "diffusive walls at rest T_w=1 (x=0) and 1.2 (x=2), initial Maxwellian "
                     "rho=1 T=1, Maxwell molecules B=1/(2 pi) (Carleman form, 8 directions), "
                     "FP32 collisions, dt=dx/(2 L_v)",
            "tol": tol,
            "low_rank": {"steps": steps_lr, "converged": int(conv_lr),
                         "err_ada": li.err_ada if li else None, "rank": int(r),
                         "rank_history": ranks, "seconds": round(t_lr, 2),
                         "ms_per_step": round(1e3 * t_lr / max(1, steps_lr), 4)},
            "full_tensor": {"steps": steps_full, "converged": int(conv_full), "err_full": e,
                            "seconds": round(t_full, 2),
                            "ms_per_step": round(1e3 * t_full / max(1, steps_full), 4)},
            "time_ratio_full_over_low_rank": round(t_full / t_lr, 2) if conv_lr and conv_full
            else None,
            "T_rel_diff_low_rank_vs_full": float(np.abs(T_lr - T_full).max() / T_full.max()),
            "rho_rel_diff_low_rank_vs_full": float(np.abs(rho_lr - rho_full).max() /
                                                   rho_full.max()),
            "T_profile_low_rank": [round(float(x), 5) for x in T_lr[::20]],
            "T_profile_full": [round(float(x), 5) for x in T_full[::20]],
            "T_next_to_walls_low_rank": [float(T_lr[0]), float(T_lr[-1])]}


def cavity_leg(args, blr, synth, torch, ctx, kind="lid"):
    """The cavities of Sec. 5.4 at a reduced spatial grid of 16 x 16 cells (the
    paper uses 100 x 100; 16 x 16 is the largest square grid whose 2 (nx + ny)
    boundary rows the GPU augmentation takes), 2D velocity 32^2, Maxwell
    diffusive walls everywhere, Maxwell molecules B = 1/(2 pi) in the Carleman
    form (8 directions), FP32 collisions, dt = dx / (2 L_v).
      lid:     [0, 0.5]^2, L_v = 7.86, T_w = 1, the lid y = 0.5 moving at
               u_w = (1, 0); initial Maxwellian rho = 1, u = (1, 1), T = 1;
      thermal: [0, 2]^2, L_v = 6.55, walls at rest; T_w = 1 on x = 0 and x = 2,
               on y = 0 and y = 2 linear in x from 1 to 1.2 (one row per
               face cell); initial Maxwellian rho = 1, u = 0, T = 1.
    Both methods run to err <= tol (the paper's res_tol 2e-7) or the
    wall-clock cap; the adaptive low-rank method starts at rank 1 with
    r_max = --cavity-rmax."""
    import numpy as np
    nx = ny = 16
    if kind == "lid":
        spec, side, u0 = synth.FOURIER, 0.5, (1.0, 1.0)
    else:
        spec = synth.VGridSpec(d=2, n=32, L=6.55, gamma=0.0, C=1.0 / (2.0 * math.pi), m_rho=1,
                               m_sigma=8)
        side, u0 = 2.0, (0.0, 0.0)
    N, L = spec.n, spec.L
    dev = torch.device("cuda:0")
    dx, dv = side / nx, 2 * L / N
    dt = 0.5 * dx / L
    tol = args.cavity_tol
    vg = blr.vgrid_from_spec(spec, blr.BLR_CARLEMAN)
    v = synth.vgrid_points(2, N, L)
    mw = lambda u, T: synth.maxwellian(v, 1.0, u, T).reshape(-1)
    wall = torch.tensor(mw((0.0, 0.0), 1.0), device=dev)
    if kind == "lid":
        top = torch.tensor(mw((1.0, 0.0), 1.0), device=dev)
        faces = [(wall, True), (wall, True), (wall, True), (top, True)]
    else:
        xc = synth.xgrid_centres(nx, 0.0, side)
        rows = torch.tensor(np.array([mw((0.0, 0.0), 1.0 + 0.2 * x / side) for x in xc]),
                            device=dev)
        faces = [(wall, True), (wall, True), (rows, True), (rows, True)]
    pb = ctx.make_problem2d(vg, nx, ny, 0.0, side, 0.0, side, faces)
    f0 = synth.maxwellian(v, 1.0, u0, 1.0).reshape(-1)
    F0 = np.tile(f0, (nx * ny, 1))
    vv = v.reshape(2, -1)

    def moments(F):
        w = dv * dv
        rho = F.sum(axis=1) * w
        u1 = (F * vv[0]).sum(axis=1) * w / rho
        u2 = (F * vv[1]).sum(axis=1) * w / rho
        E = 0.5 * (F * (vv ** 2).sum(axis=0)).sum(axis=1) * w
        return (2 * E / rho - u1 * u1 - u2 * u2) / 2, u1, u2

    rc, chunk = max(2, args.cavity_rmax), 25
    X, S, V = synth.lowrank_state(F0, 1, dx * dx, dv * dv)
    Xd = torch.zeros((rc, nx * ny), dtype=torch.float64, device=dev)
    Sd = torch.zeros((rc, rc), dtype=torch.float64, device=dev)
    Vd = torch.zeros((rc, N * N), dtype=torch.float64, device=dev)
    Xd[:1] = torch.tensor(X.T, device=dev)
    Sd[:1, :1] = torch.tensor(S, device=dev)
    Vd[:1] = torch.tensor(V, device=dev)
    st = ctx.make_state(Xd, Sd, Vd, 1)
    torch.cuda.synchronize()
    sp = blr.SolveParams(blr.StepParams(dt, 0.2, 1e-10, 1, rc,
                                        blr.BLR_STEP_ADD | blr.BLR_STEP_DROP), tol, chunk)
    steps_lr, ranks, conv_lr, li = 0, [], False, None
    t0 = time.perf_counter()
    while not conv_lr and time.perf_counter() - t0 < args.cavity_cap:
        li = ctx.steady_solve(pb, st, sp, allow_unconverged=True)
        steps_lr += int(li.steps)
        conv_lr = bool(li.converged)
        if not ranks or ranks[-1][1] != int(li.r) or steps_lr % 2000 == 0:
            ranks.append([steps_lr, int(li.r)])
        progress(f"{kind} cavity: low-rank {steps_lr} steps, err_ada {li.err_ada:.3e}, rank {li.r}")
    t_lr = time.perf_counter() - t0
    r = st.r
    F_lr = (Xd[:r].cpu().numpy().T @ Sd[:r, :r].cpu().numpy()) @ Vd[:r].cpu().numpy()
    F = torch.tensor(F0, device=dev)
    steps_full, e = 0, float("inf")
    t0 = last = time.perf_counter()
    while e > tol and time.perf_counter() - t0 < args.cavity_cap:
        e = ctx.full_step(pb, F, dt, blr.BLR_FP32)
        steps_full += 1
        if time.perf_counter() - last > 20.0:
            last = time.perf_counter()
            progress(f"{kind} cavity: full tensor {steps_full} steps, err_full {e:.3e}")
    t_full = time.perf_counter() - t0
    m_lr, m_full = moments(F_lr), moments(F.cpu().numpy())
    diffs = {nm: float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))
             for nm, a, b in zip(("T", "u1", "u2"), m_lr, m_full)}
    shape = ("lid-driven cavity: [0,0.5]^2, L_v=7.86, diffusive walls T_w=1, lid u_w=(1,0), "
             "initial Maxwellian rho=1 u=(1,1) T=1" if kind == "lid" else
             "thermally driven cavity: [0,2]^2, L_v=6.55, diffusive walls at rest, T_w=1 on "
             "x=0 and x=2, linear in x from 1 to 1.2 on y=0 and y=2, initial Maxwellian rho=1 "
             "u=0 T=1")
    return {"shape": shape + "; 16x16 cells (paper: 100x100), 2D velocity 32^2, Maxwell "
                             "molecules B=1/(2 pi) (Carleman form, 8 directions), FP32 "
                             "collisions, dt=dx/(2 L_v)",
            "tol": tol, "r_max": rc,
            "low_rank": {"steps": steps_lr, "converged": int(conv_lr),
                         "err_ada": li.err_ada if li else None, "rank": int(r),
                         "rank_history": ranks, "seconds": round(t_lr, 2),
                         "ms_per_step": round(1e3 * t_lr / max(1, steps_lr), 4)},
            "full_tensor": {"steps": steps_full, "converged": int(e <= tol), "err_full": e,
                            "seconds": round(t_full, 2),
                            "ms_per_step": round(1e3 * t_full / max(1, steps_full), 4)},
            "max_rel_diff_low_rank_vs_full": diffs}


def steady_compare_leg(args, blr, synth, torch, helper):
    """One solve of the 2D-velocity converged-trace recipe marched a fixed
    number of steps past the stopping rule with FP32, corrected FP32 and FP64
    collisions; the steady moments of the first two against the third."""
    import numpy as np
    ct = synth.serving_trace_2d(count=1, seed=6, rate=4.0)
    cp = prepare_trace(ct, synth)
    n = args.steady_compare
    legs = {}
    for name, kw in (("fp32", {}), ("fp32_defect", {"defect": True}), ("fp64", {"fp64": True})):
        rr, mm = run_trace(blr, torch, helper, cp, 1, False, n, res_tol=0.0, moments_of=(0,), **kw)
        legs[name] = (rr, mm[0])
    return {
        "steps": n, "target": 1e-6,
        **{name: {"err_ada": legs[name][0].get("final_err_ada"), "wall_s": legs[name][0]["wall_s"],
                  "moments_max_rel_diff": {
                      nm: float(np.abs(a - c).max() / np.abs(c).max())
                      for nm, a, c in zip(("rho", "u1", "T"), legs[name][1], legs["fp64"][1])}}
           for name in ("fp32", "fp32_defect")},
        "fp64": {"err_ada": legs["fp64"][0].get("final_err_ada"),
                 "wall_s": legs["fp64"][0]["wall_s"]}}


def serving_leg(args, blr, synth, torch, helper):
    """The serving trace on the batched FP32 path (slots solves at once) and on
    the plain FP64 per-pair path (one solve at a time, first in first out),
    then a longer trace on the batched path."""
    import numpy as np
    base = dict(count=args.serve_count, seed=5, rate=4.0)
    trace = synth.serving_trace(**base)
    prepared = prepare_trace(trace, synth)
    batched = run_trace(blr, torch, helper, prepared, args.serve_slots, False, args.serve_steps)
    fused = run_trace(blr, torch, helper, prepared, args.serve_slots, False, args.serve_steps,
                      batch=True)
    plain = run_trace(blr, torch, helper, prepared, 1, True, args.serve_steps)
    out = {"trace": (f"{args.serve_count} steady normal-shock solves, seed 5, Poisson arrivals 4/s, "
                     "Mach~U[1.2,3], N_x in {128,256,512}, N_v in {24^3 (L=8), 32^3 (L=10)}, "
                     "initial rank U{5..25}, r_max 30, hard spheres M_rho=16 x M_sigma=38, "
                     f"each to err_ada<=1e-6 or {args.serve_steps} steps"),
           "batched_fp32": batched,
           "batched_fp32_shared_collision_launches": fused,
           "plain_fp64_fifo": plain,
           "plain_over_batched_latency_p50": round(plain["latency_s_p50"] /
                                                   batched["latency_s_p50"], 1)}
    if args.serve_conv_count > 0:
        ct = synth.serving_trace_2d(count=args.serve_conv_count, seed=6, rate=4.0)
        cp = prepare_trace(ct, synth)
        nplain = min(args.serve_conv_plain, len(cp))
        out["converged_trace"] = (
            f"{len(cp)} steady normal-shock solves of the paper's own class (2D velocity 32^2 on "
            "[-8,8]^2, Maxwell molecules B=1/(2 pi), M_rho=8 x M_sigma=8), seed 6, Poisson arrivals "
            "4/s, Mach~U[1.2,2], N_x in {32,64} on [-30,30], initial rank U{4..8}, dt=0.4 dx/L_v, "
            f"each run to err_ada<=1e-6 (cap {args.serve_conv_cap} steps); the plain FP64 FIFO on the "
            f"first {nplain} of them")
        out["converged_batched_fp32"] = run_trace(blr, torch, helper, cp, args.serve_slots, False,
                                                  args.serve_conv_cap)
        if nplain:
            out["converged_plain_fp64_fifo"], m64 = run_trace(
                blr, torch, helper, cp[:nplain], 1, True, args.serve_conv_cap, moments_of=(0,))
            b, m32 = run_trace(blr, torch, helper, cp[:nplain], args.serve_slots, False,
                               args.serve_conv_cap, moments_of=(0,))
            out["converged_batched_fp32_same_subset"] = b
            out["converged_plain_over_batched_latency_p50"] = round(
                out["converged_plain_fp64_fifo"]["latency_s_p50"] / b["latency_s_p50"], 1)
            # steady moments of the first request: FP32 collisions (batched) against
            # FP64 collisions (plain), each run to its own err_ada <= 1e-6
            out["converged_fp32_vs_fp64_steady_moments"] = {
                nm: float(np.abs(a - c).max() / np.abs(c).max())
                for nm, a, c in zip(("rho", "u1", "T"), m32[0], m64[0])}
            out["converged_fp32_vs_fp64_steady_moments"]["target"] = 1e-6
            # the same with the FP64 defect correction of the FP32 pairs
            bd, md = run_trace(blr, torch, helper, cp[:nplain], args.serve_slots, False,
                               args.serve_conv_cap, moments_of=(0,), defect=True)
            out["converged_fp32_defect_same_subset"] = bd
            out["converged_fp32_defect_vs_fp64_steady_moments"] = {
                nm: float(np.abs(a - c).max() / np.abs(c).max())
                for nm, a, c in zip(("rho", "u1", "T"), md[0], m64[0])}
    if args.serve_long_count > 0:
        long_trace = synth.serving_trace(count=args.serve_long_count, seed=5, rate=4.0)
        lp = prepare_trace(long_trace, synth)
        out["long_trace"] = f"the first {args.serve_long_count} requests of the same recipe, " \
                            f"each to err_ada<=1e-6 or {args.serve_long_steps} steps"
        out["long_batched_fp32"] = run_trace(blr, torch, helper, lp, args.serve_slots, False,
                                             args.serve_long_steps)
        out["long_batched_fp32_shared_collision_launches"] = run_trace(
            blr, torch, helper, lp, args.serve_slots, False, args.serve_long_steps, batch=True)
        # the same requests all arriving at once (every slot busy from the start)
        burst = [dict(p, q=dict(p["q"], arrival=0.0)) for p in lp]
        out["burst_trace"] = "the long trace's requests, all arriving at t = 0"
        out["burst_batched_fp32"] = run_trace(blr, torch, helper, burst, args.serve_slots, False,
                                              args.serve_long_steps)
        out["burst_batched_fp32_shared_collision_launches"] = run_trace(
            blr, torch, helper, burst, args.serve_slots, False, args.serve_long_steps, batch=True)
    return out


_CPU_VS = None


def _cpu_worker_init(spec):
    """Worker of the CPU baseline: one thread per process (the oracle's FFTs
    and products are single-threaded; BLAS kept to one thread as well)."""
    global _CPU_VS
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except ImportError:
        pass
    from oracle import collision as oc
    _CPU_VS = oc.setup_from_spec(spec)


def _cpu_pair(args):
    from oracle import collision as oc
    V, pair = args
    q, _ = oc.q_pairs(V, [pair], _CPU_VS, conserve=True)
    return q.shape


def cpu_baseline_leg(spec, V, pairs):
    """The float64 oracle (its FFT form) on all pairs of the rank-r basis at the
    benchmark's grid, the pairs spread over one process per host core (each
    pair is the oracle's own serial computation).  Runs before the GPU is
    touched, so the worker processes are forked from a process without GPU
    state.  Cores: the job's CPU share (OMP_NUM_THREADS where the job sets
    it), at most os.cpu_count()."""
    import multiprocessing as mp
    ncpu = os.cpu_count() or 1
    try:
        share = int(os.environ.get("OMP_NUM_THREADS", ncpu))
    except ValueError:
        share = ncpu
    workers = max(1, min(ncpu, share, len(pairs)))
    with mp.get_context("fork").Pool(workers, initializer=_cpu_worker_init, initargs=(spec,)) as pool:
        pool.map(_cpu_pair, [(V, pairs[0])] * workers)      # warm the workers
        t0 = time.perf_counter()
        pool.map(_cpu_pair, [(V, p) for p in pairs], chunksize=1)
        t = time.perf_counter() - t0
    return {"value": round(len(pairs) / t, 4), "unit": "pair evals/s", "cores": workers,
            "kind": "oracle",
            "sample": (f"all {len(pairs)} pairs Q_s(V_i,V_j) of the rank-10 basis on the full 32^3 "
                       f"grid, float64 oracle (FFT form of the operator, numpy), one pair per task "
                       f"over {workers} worker processes of one thread each"),
            "seconds": round(t, 2), "os_cpu_count": ncpu}


def parity_leg(blr, synth, torch, ctx):
    """Errors of the library against the oracle's stored values (tests/golden,
    written by scripts that call only the oracle): the benchmark's own 78
    pair collisions and adaptive step, and single evaluations of the
    homogeneous workloads.  Pair errors are ||Q - Q_ref|| / ||Q+_ref||."""
    import numpy as np
    gdir = os.path.join(ROOT, "tests", "golden")
    out = {}
    dev = "cuda"
    try:
        g = np.load(os.path.join(gdir, "c3_step.npz"))
    except OSError:
        g = None
    if g is not None:
        V32 = torch.tensor(np.ascontiguousarray(g["V_aug32"]), device=dev)
        Q = ctx.collision_pairs(blr.vgrid_from_spec(synth.C3), V32, blr.upper_pairs(12))
        torch.cuda.synchronize()
        e = np.linalg.norm(Q.double().cpu().numpy() - g["q32"].astype(np.float64), axis=1) / \
            g["qplus_norm"]
        out["c3_78_pairs_fp32_max_err"] = float(e.max())
        out["c3_78_pairs_fp32_median_err"] = float(np.median(e))
        nx, r0, rm = int(g["nx"]), int(g["r_min"]), int(g["r_max"])
        ini = synth.shock_initial(1.5, synth.C3, nx, -30.0, 30.0, pert=0.0, pert_rank=0)
        fL, fR = torch.tensor(ini["fL"], device=dev), torch.tensor(ini["fR"], device=dev)
        f_ref = (g["X1"] @ g["S1"]) @ g["V1"]
        w = math.sqrt((60.0 / nx) * (2 * synth.C3.L / synth.C3.n) ** 3)
        for name, fl in (("fp32", 0), ("fp64", blr.BLR_STEP_FP64_COLLISION)):
            X = torch.zeros((rm, nx), dtype=torch.float64, device=dev)
            S = torch.zeros((rm, rm), dtype=torch.float64, device=dev)
            V = torch.zeros((rm, g["V0"].shape[1]), dtype=torch.float64, device=dev)
            X[:r0] = torch.tensor(np.ascontiguousarray(g["X0"].T), device=dev)
            S[:r0, :r0] = torch.tensor(np.ascontiguousarray(g["S0"]), device=dev)
            V[:r0] = torch.tensor(np.ascontiguousarray(g["V0"]), device=dev)
            pb = ctx.make_problem(blr.vgrid_from_spec(synth.C3), nx, -30.0, 30.0, fL, fR)
            st = ctx.make_state(X, S, V, r0, seed=1)
            sp = blr.StepParams(float(g["dt"]), 0.2, 1e-10, r0, rm,
                                blr.BLR_STEP_ADD | blr.BLR_STEP_DROP | fl)
            info = ctx.dlr_step(pb, st, sp)
            r = st.r
            f = (X[:r].cpu().numpy().T @ S[:r, :r].cpu().numpy()) @ V[:r].cpu().numpy()
            out[f"c3_step_{name}"] = {
                "f_err_l2": float(w * np.linalg.norm(f - f_ref)),
                "f_err_max_rel": float(np.abs(f - f_ref).max() / np.abs(f_ref).max()),
                "fp32_bound_l2": float(1e-5 * float(g["dt"]) * float(g["gain_scale"])),
                "ranks_match": bool(info.r_added == int(g["r_added"]) and
                                    info.r_out == int(g["r_out"])),
                "err_rel": float(abs(info.err - float(g["err"])) / float(g["err"]))}
    try:
        h = np.load(os.path.join(gdir, "c1_c2_q.npz"))
    except OSError:
        h = None
    if h is not None:
        bkw = synth.VGridSpec(d=3, n=32, L=8.0, gamma=0.0, C=1.0 / (4.0 * math.pi), m_rho=16,
                              m_sigma=38)
        for case, spec in (("c1", synth.C1), ("c2b", synth.C2), ("c2k", bkw)):
            for dt in (torch.float64, torch.float32):
                f = torch.tensor(np.ascontiguousarray(h[f"{case}_f"]).reshape(1, -1), dtype=dt,
                                 device=dev)
                q = ctx.collision_pairs(blr.vgrid_from_spec(spec, blr.BLR_NO_CONSERVE), f,
                                        [(0, 0)])
                torch.cuda.synchronize()
                q = q.double().cpu().numpy()[0]
                key = {"c1": "c1_2d_two_stream", "c2b": "c2_3d_bimaxwellian_hard_spheres",
                       "c2k": "c2_3d_bkw_maxwell"}[case]
                tag = "fp64" if dt == torch.float64 else "fp32"
                out[f"{key}_{tag}_err"] = float(np.linalg.norm(q - h[f"{case}_q"]) /
                                                float(h[f"{case}_gain_norm"]))
                if case == "c2k":
                    d = h["c2k_dfdt"]
                    out[f"{key}_{tag}_vs_analytic_dfdt"] = float(np.abs(q - d).max() /
                                                                 np.abs(d).max())
    try:
        gs = np.load(os.path.join(gdir, "steady_shock_2d.npz"))
    except OSError:
        gs = None
    if gs is not None:
        # the oracle's steady solve of a small Mach-1.4 shock (2D velocity 32^2,
        # Maxwell molecules, 32 cells, dt 0.1, err_ada <= 1e-6) against the
        # library's in each collision precision: rho, u_1, T per cell
        spec = synth.VGridSpec(d=2, n=32, L=8.0, gamma=0.0, C=1.0 / (2.0 * math.pi), m_rho=8,
                               m_sigma=8)
        nx, r0, rc = 32, 6, 16
        ini = synth.shock_initial(1.4, spec, nx, -30.0, 30.0, pert=1e-3, pert_rank=3, seed=7)
        dvd = (2.0 * spec.L / spec.n) ** 2
        X0, S0, V0 = synth.lowrank_state(ini["f0"], r0, 60.0 / nx, dvd)
        v = synth.vgrid_points(2, spec.n, spec.L).reshape(2, -1)
        fL, fR = torch.tensor(ini["fL"], device=dev), torch.tensor(ini["fR"], device=dev)
        pb = ctx.make_problem(blr.vgrid_from_spec(spec), nx, -30.0, 30.0, fL, fR)
        res = {"oracle_steps": int(gs["steps"])}
        # each precision to its own stopping rule, and FP32 with and without
        # the defect correction marched exactly the oracle's step count (near
        # the stopping point one step moves the moments by about 1e-6)
        for name, fl, at in (("fp32", 0, False), ("fp32_defect", blr.BLR_STEP_FP64_DEFECT, False),
                             ("fp64", blr.BLR_STEP_FP64_COLLISION, False),
                             ("fp32_at_oracle_step", 0, True),
                             ("fp32_defect_at_oracle_step", blr.BLR_STEP_FP64_DEFECT, True)):
            X = torch.zeros((rc, nx), dtype=torch.float64, device=dev)
            S = torch.zeros((rc, rc), dtype=torch.float64, device=dev)
            V = torch.zeros((rc, spec.n ** 2), dtype=torch.float64, device=dev)
            X[:r0] = torch.tensor(np.ascontiguousarray(X0.T), device=dev)
            S[:r0, :r0] = torch.tensor(S0, device=dev)
            V[:r0] = torch.tensor(V0, device=dev)
            st = ctx.make_state(X, S, V, r0)
            sp = blr.SolveParams(blr.StepParams(0.1, 0.2, 1e-10, 1, 16,
                                                blr.BLR_STEP_ADD | blr.BLR_STEP_DROP | fl),
                                 0.0 if at else 1e-6, int(gs["steps"]) if at else 8000)
            sp.defect_every = 4
            info = ctx.steady_solve(pb, st, sp, allow_unconverged=at)
            r = st.r
            F = (X[:r].cpu().numpy().T @ S[:r, :r].cpu().numpy()) @ V[:r].cpu().numpy()
            rho = F.sum(axis=1) * dvd
            u = (F * v[0]).sum(axis=1) * dvd / rho
            u2 = (F * v[1]).sum(axis=1) * dvd / rho
            T = ((F * (v ** 2).sum(axis=0)).sum(axis=1) * dvd / rho - u * u - u2 * u2) / 2.0
            res[name] = {"steps": int(info.steps), "moments_max_rel_err": max(
                float(np.abs(a - b).max() / np.abs(b).max())
                for a, b in ((rho, gs["rho"]), (u, gs["u"]), (T, gs["T"])))}
        res["target"] = 1e-6
        out["steady_shock_2d_moments_vs_oracle"] = res
    out["measure"] = ("pair / single evaluations: ||Q - Q_ref||_2 / ||Q+_ref||_2 (targets 1e-5 FP32, "
                      "1e-12 FP64); step: L2(x,v) norm of f - f_ref against the FP32 collision "
                      "bound 1e-5 dt ||sum K_m K_n Q+_mn||, and max |f - f_ref| / max |f_ref|")
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "runs on one GPU only: sharding a solve across GPUs is not "
                                   "implemented (independent requests can run one process per "
                                   "GPU)", "n_gpus": args.gpus}))
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2112_02695_amd as blr
    import synth

    spec = synth.C3
    nx, r, r_cap = 256, 10, 12
    dt = 0.01
    ini = synth.shock_initial(1.5, spec, nx, -30.0, 30.0, pert=1e-3, pert_rank=10, seed=3)
    dx = 60.0 / nx
    dvd = (2 * spec.L / spec.n) ** 3
    X, S, V = synth.lowrank_state(ini["f0"], r, dx, dvd)
    pairs = blr.upper_pairs(r)
    cpu = None
    if not args.no_cpu_baseline:
        progress("cpu baseline (oracle, all 55 pairs over the host cores)")
        cpu = cpu_baseline_leg(spec, V, pairs)

    lib = blr.load_library()
    lib.blr_timing.argtypes = [ctypes.c_void_p, ctypes.c_int32]
    lib.blr_timing_read.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_char_p, ctypes.c_int32,
                                    ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64),
                                    ctypes.POINTER(ctypes.c_double)]
    P = len(pairs)
    flags = blr.BLR_GENERIC_FFT if args.generic else 0
    vg = blr.vgrid_from_spec(spec, flags)

    dev = torch.device("cuda:0")
    if args.copy_calibration:
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)   # 256 MiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    ctx = blr.Context(0)
    V32 = torch.tensor(V, dtype=torch.float32, device=dev)
    Q = torch.empty((P, V.shape[1]), dtype=torch.float32, device=dev)

    counted = [0]
    if args.mode == "pairs":
        def one_step():
            ctx.collision_pairs(vg, V32, pairs, out=Q)
            counted[0] += P
    else:
        Xd = torch.zeros((r_cap, nx), dtype=torch.float64, device=dev)
        Sd = torch.zeros((r_cap, r_cap), dtype=torch.float64, device=dev)
        Vd = torch.zeros((r_cap, V.shape[1]), dtype=torch.float64, device=dev)
        Xd[:r] = torch.tensor(X.T, device=dev)
        Sd[:r, :r] = torch.tensor(S, device=dev)
        Vd[:r] = torch.tensor(V, device=dev)
        fL = torch.tensor(ini["fL"], device=dev)
        fR = torch.tensor(ini["fR"], device=dev)
        pb = ctx.make_problem(vg, nx, -30.0, 30.0, fL, fR)
        st = ctx.make_state(Xd, Sd, Vd, r, seed=1)
        sp = blr.StepParams(dt, 0.2, 1e-10, r, r_cap, blr.BLR_STEP_ADD | blr.BLR_STEP_DROP)
        infos = []

        def one_step():
            info = ctx.dlr_step(pb, st, sp)
            rr = info.r_in + info.r_added
            counted[0] += rr * (rr + 1) // 2
            infos.append((info.r_in, info.r_added, info.r_out, info.err, info.err_ada,
                          info.ms_collision, info.ms_step))

    progress(f"{args.mode}: {args.warmup} warm-up + {args.steps} timed steps")
    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()
    counted[0] = 0
    t0 = time.perf_counter()
    step_wall = []
    for _ in range(args.steps):
        ts = time.perf_counter()
        one_step()   # a step ends with the library's one host wait (the rank decision)
        step_wall.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    n_counted = counted[0]
    # Per-kernel times: a second pass of the same steps with the library's
    # kernel events on (steps then run kernel by kernel, not as replayed
    # graphs); the dominant kernel's launches are identical in both passes.
    kpass = max(3, min(args.steps, 10))
    lib.blr_timing(ctx.h, 2)
    lib.blr_timing(ctx.h, 1)
    torch.cuda.synchronize()
    tk0 = time.perf_counter()
    for _ in range(kpass):
        one_step()
    torch.cuda.synchronize()
    tk1 = time.perf_counter()
    lib.blr_timing(ctx.h, 0)
    timers = read_timers(ctx)
    counted[0] = n_counted
    ktime = tk1 - tk0
    ms_per_step = 1e3 * elapsed / args.steps
    value = counted[0] / elapsed
    step_extra = None
    if args.mode == "step":
        last = infos[-(args.steps + kpass):-kpass]
        timed = infos[-kpass:]
        step_extra = {"rank_in_added_out": [list(x[:3]) for x in last[:3]],
                      "err_last": last[-1][3], "err_ada_last": last[-1][4],
                      "ms_step_gpu_avg": round(sum(x[6] for x in last) / len(last), 4),
                      "ms_collision_avg_kernel_pass": round(sum(x[5] for x in timed) / len(timed), 4),
                      "ms_per_step_kernel_pass": round(1e3 * ktime / kpass, 4),
                      "pairs_per_step": counted[0] / args.steps}
        # collision-only rate of the rank-10 batch, for reference
        for _ in range(2):
            ctx.collision_pairs(vg, V32, pairs, out=Q)
        torch.cuda.synchronize()
        tq = time.perf_counter()
        for _ in range(5):
            ctx.collision_pairs(vg, V32, pairs, out=Q)
        torch.cuda.synchronize()
        step_extra["collision_only_pair_evals_per_s"] = round(5 * P / (time.perf_counter() - tq), 1)

    # dominant kernel and its roofline
    dom = max(timers, key=lambda t: t["ms"]) if timers else None
    roof = None
    if dom:
        avg_s = dom["ms"] / dom["launches"] / 1e3
        bytes_per_launch = dom["bytes"] / dom["launches"]
        achieved = bytes_per_launch / avg_s / 1e9
        # HBM bytes per launch from rocprofv3 counters, valid only while the
        # kernel source is the one they were taken on
        traffic = None
        try:
            import hashlib
            with open(args.traffic) as fh:
                tr = json.load(fh)
            with open(os.path.join(ROOT, tr["source"]), "rb") as fh:
                same = hashlib.sha256(fh.read()).hexdigest() == tr.get("source_sha256")
            if tr.get("kernel") == dom["name"] and same:
                traffic = tr.get("bytes_per_launch")
        except (OSError, ValueError, KeyError):
            pass
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": dom["name"], "avg_launch_us": round(avg_s * 1e6, 2),
                "launches_timed": dom["launches"],
                "algorithmic_bytes_per_launch": bytes_per_launch,
                "share_of_step": round(dom["ms"] / (ktime * 1e3), 3)}

    latency = {"batched_step_ms_p50": round(1e3 * pct(step_wall, 0.50), 4),
               "batched_step_ms_p99": round(1e3 * pct(step_wall, 0.99), 4),
               "batched_samples": len(step_wall)}
    # the same step on the plain FP64 per-pair schedule (fresh copy of the
    # initial factors; one untimed step first)
    if args.mode == "step" and not args.no_plain:
        progress("plain fp64 per-pair steps")
        vgp = blr.vgrid_from_spec(spec, blr.BLR_PLAIN_SCHEDULE)
        pbp = ctx.make_problem(vgp, nx, -30.0, 30.0, fL, fR)
        Xp, Sp, Vp = Xd.clone(), Sd.clone(), Vd.clone()
        Xp.zero_(); Sp.zero_(); Vp.zero_()
        Xp[:r] = torch.tensor(X.T, device=dev)
        Sp[:r, :r] = torch.tensor(S, device=dev)
        Vp[:r] = torch.tensor(V, device=dev)
        stp = ctx.make_state(Xp, Sp, Vp, r, seed=1)
        spp = blr.StepParams(dt, 0.2, 1e-10, r, r_cap,
                             blr.BLR_STEP_ADD | blr.BLR_STEP_DROP | blr.BLR_STEP_FP64_COLLISION)
        ctx.dlr_step(pbp, stp, spp)
        torch.cuda.synchronize()
        pw = []
        for _ in range(3):
            ts = time.perf_counter()
            ctx.dlr_step(pbp, stp, spp)
            pw.append(time.perf_counter() - ts)
        latency.update({"plain_fp64_step_ms_p50": round(1e3 * pct(pw, 0.50), 3),
                        "plain_fp64_step_ms_max": round(1e3 * max(pw), 3),
                        "plain_samples": len(pw),
                        "plain_over_batched_p50": round(pct(pw, 0.5) / pct(step_wall, 0.5), 1)})

    # the same step with FP64 collisions on the fast schedule, and with the
    # FP64 defect correction of the FP32 pairs (a refresh step: FP64 and FP32
    # pairs; a corrected step: FP32 pairs plus the carried defect)
    if args.mode == "step" and not args.no_plain:
        progress("fp64 and defect-corrected steps")
        ms = {}
        for name, fl in (("fp64_collision", blr.BLR_STEP_FP64_COLLISION),
                         ("defect_refresh", blr.BLR_STEP_FP64_DEFECT | blr.BLR_STEP_DEFECT_REFRESH),
                         ("defect_corrected", blr.BLR_STEP_FP64_DEFECT)):
            Xq, Sq, Vq = Xd.clone(), Sd.clone(), Vd.clone()
            Xq.zero_(); Sq.zero_(); Vq.zero_()
            Xq[:r] = torch.tensor(X.T, device=dev)
            Sq[:r, :r] = torch.tensor(S, device=dev)
            Vq[:r] = torch.tensor(V, device=dev)
            stq = ctx.make_state(Xq, Sq, Vq, r, seed=1)
            spq = blr.StepParams(dt, 0.2, 1e-10, r, r_cap, blr.BLR_STEP_ADD | blr.BLR_STEP_DROP | fl)
            for _ in range(2):   # the first recording of the step graph
                ctx.dlr_step(pb, stq, spq)
            torch.cuda.synchronize()
            tw = []
            for _ in range(5):
                ts = time.perf_counter()
                ctx.dlr_step(pb, stq, spq)
                tw.append(time.perf_counter() - ts)
            ms[name] = round(1e3 * pct(tw, 0.5), 3)
        latency.update({"fp64_collision_step_ms_p50": ms["fp64_collision"],
                        "defect_refresh_step_ms_p50": ms["defect_refresh"],
                        "defect_corrected_step_ms_p50": ms["defect_corrected"],
                        "defect_every_4_step_ms": round(
                            (ms["defect_refresh"] + 3 * ms["defect_corrected"]) / 4, 3)})

    # the full-tensor reference step on the same grid (Q(f(x_p), f(x_p)) for
    # all N_x cells plus upwind transport), FP32 collisions as in the step
    full = None
    if args.mode == "step" and not args.no_full:
        progress("full-tensor steps")
        Ff = torch.tensor(ini["f0"], device=dev)
        ctx.full_step(pb, Ff, dt, blr.BLR_FP32)
        torch.cuda.synchronize()
        tf = []
        for _ in range(3):
            ts = time.perf_counter()
            e_full = ctx.full_step(pb, Ff, dt, blr.BLR_FP32)
            tf.append(time.perf_counter() - ts)
        full = {"step_ms_p50": round(1e3 * pct(tf, 0.5), 3), "samples": len(tf), "cells": nx,
                "cell_collisions_per_s": round(nx / pct(tf, 0.5), 1),
                "err_full_last": e_full,
                "low_rank_step_speedup": round(pct(tf, 0.5) / pct(step_wall, 0.5), 2)}
        del Ff

    # plain FP64 per-pair GPU path (the baseline schedule), on a few pairs
    plain = None
    if not args.no_plain:
        V64 = torch.tensor(V, dtype=torch.float64, device=dev)
        vgp = blr.vgrid_from_spec(spec, blr.BLR_PLAIN_SCHEDULE)
        sub = pairs[:3]
        ctx.collision_pairs(vgp, V64, sub[:1])
        torch.cuda.synchronize()
        tp = time.perf_counter()
        ctx.collision_pairs(vgp, V64, sub)
        torch.cuda.synchronize()
        plain = len(sub) / (time.perf_counter() - tp)

    carleman = None
    if args.mode == "step" and not args.no_carleman:
        progress("carleman form")
        carleman = carleman_leg(args, blr, synth, torch, ctx, lib, spec, V, X, S, ini, nx, r,
                                r_cap, dt)

    paper = None
    if args.paper_shock:
        paper = paper_shock_leg(args, blr, synth, torch, ctx)
    fourier = None
    if args.paper_fourier:
        fourier = fourier_leg(args, blr, synth, torch, ctx)
    cavity = None
    if args.paper_cavity:
        cavity = cavity_leg(args, blr, synth, torch, ctx, "lid")
    thermal = None
    if args.paper_thermal:
        thermal = cavity_leg(args, blr, synth, torch, ctx, "thermal")
    c4 = None
    if args.c4:
        c4 = c4_leg(args, blr, synth, torch, ctx)

    serving = None
    if args.mode == "step" and not args.no_serve:
        serving = serving_leg(args, blr, synth, torch, ctx)
    if args.steady_compare > 0:
        serving = dict(serving or {})
        serving["fixed_steps_vs_fp64"] = steady_compare_leg(args, blr, synth, torch, ctx)

    parity = None
    if not args.no_parity:
        progress("parity against the oracle's stored values")
        parity = parity_leg(blr, synth, torch, ctx)

    line = {
        "metric": "Q(V_i,V_j) evals/s at N_v=32^3 + p50/p99 solve latency, batched vs plain",
        "value": round(value, 2),
        "unit": "pair evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": ("adaptive low-rank step of a Mach-1.5 shock state (N_x=256, N_v=32^3 "
                                "on [-8,8]^3, hard spheres, M_rho=16 x M_sigma=38, rank 10 -> +2 "
                                "boundary basis -> drop to >=10; 78 pair collisions per step)")
                   if args.mode == "step" else
                   ("55 pair collisions Q_s(V_i,V_j) of the rank-10 basis of a Mach-1.5 shock "
                    "state, N_v=32^3 on [-8,8]^3, hard spheres, M_rho=16 x M_sigma=38"),
                   "mode": args.mode, "r": r, "n_v": spec.n, "nx": nx, "dt": dt,
                   "collisions": "fp32 (+fp64 moment projection)", "linear_algebra": "fp64",
                   "path": "generic" if args.generic else "default"},
        "step": step_extra,
        "roofline": roof,
        "cpu_baseline": cpu,
        "parity": parity,
        "plain_fp64_pair_evals_per_s": round(plain, 2) if plain else None,
        "latency": latency,
        "full_tensor": full,
        "carleman": carleman,
        "paper_shock": paper,
        "paper_fourier": fourier,
        "paper_cavity": cavity,
        "paper_thermal_cavity": thermal,
        "c4_reduced": c4,
        "serving": serving,
        "kernels": [{k: (round(v, 4) if isinstance(v, float) else v) for k, v in t.items()}
                    for t in sorted(timers, key=lambda t: -t["ms"])[:8]],
    }
    print(json.dumps(line))
    ctx.close()


if __name__ == "__main__":
    main()
