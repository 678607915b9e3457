"""Benchmark of the collision hot path on one MI355X.

Workload: the pair collisions Q_s(V_i, V_j), i <= j, of the rank-10 velocity
basis of a Mach-1.5 normal-shock state (N_x = 256 cells on [-30, 30],
N_v = 32^3 on [-8, 8]^3, hard spheres B = |v - v*|, 16 Gauss-Legendre radial
nodes x 38 Lebedev sphere nodes): 55 pairs per step, FP32 FFTs/products/sums
with the FP64 moment projection.  With ``--mode step`` a step is one full
adaptive low-rank time step (add -> K -> S -> L -> drop) of the same state,
whose 55 pair collisions are counted.

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
    ap.add_argument("--mode", choices=["pairs", "step"], default="pairs")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--generic", action="store_true", help="force the multi-pass FFT path")
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


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; multi-GPU sharding is described "
                                   "in DESIGN.md but not built", "n_gpus": args.gpus}))
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2112_02695_amd as blr
    import synth

    lib = blr.load_library()
    lib.blr_timing.argtypes = [ctypes.c_void_p, ctypes.c_int32]
    lib.blr_timing_read.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_char_p, ctypes.c_int32,
                                    ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64),
                                    ctypes.POINTER(ctypes.c_double)]

    spec = synth.C3
    nx, r = 256, 10
    ini = synth.shock_initial(1.5, spec, nx, -30.0, 30.0, pert=1e-3, pert_rank=10, seed=3)
    dx = 60.0 / nx
    dvd = (2 * spec.L / spec.n) ** 3
    X, S, V = synth.lowrank_state(ini["f0"], r, dx, dvd)
    pairs = blr.upper_pairs(r)
    P = len(pairs)
    flags = blr.BLR_GENERIC_FFT if args.generic else 0
    vg = blr.vgrid_from_spec(spec, flags)

    dev = torch.device("cuda:0")
    ctx = blr.Context(0)
    V32 = torch.tensor(V, dtype=torch.float32, device=dev)
    Q = torch.empty((P, V.shape[1]), dtype=torch.float32, device=dev)

    def one_step():
        ctx.collision_pairs(vg, V32, pairs, out=Q)

    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()
    lib.blr_timing(ctx.h, 2)
    lib.blr_timing(ctx.h, 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        one_step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lib.blr_timing(ctx.h, 0)
    timers = read_timers(ctx)
    elapsed = t1 - t0
    ms_per_step = 1e3 * elapsed / args.steps
    value = P * args.steps / elapsed

    # dominant kernel and its roofline
    dom = max(timers, key=lambda t: t["ms"]) if timers else None
    roof = None
    if dom:
        avg_s = dom["ms"] / dom["launches"] / 1e3
        bytes_per_launch = dom["bytes"] / dom["launches"]
        achieved = bytes_per_launch / avg_s / 1e9
        traffic = None
        try:
            with open(args.traffic) as fh:
                tr = json.load(fh)
            if tr.get("kernel") == dom["name"]:
                traffic = tr.get("bytes_per_launch")
        except (OSError, ValueError):
            pass
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": dom["name"], "avg_launch_us": round(avg_s * 1e6, 2),
                "algorithmic_bytes_per_launch": bytes_per_launch,
                "share_of_step": round(dom["ms"] / (elapsed * 1e3), 3)}

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

    cpu = None
    if not args.no_cpu_baseline:
        from oracle import collision as oc
        vs = oc.setup_from_spec(spec)
        tc = time.perf_counter()
        oc.q_pairs(V, [pairs[1]], vs, conserve=True)
        dt = time.perf_counter() - tc
        cpu = {"value": round(1.0 / dt, 5), "unit": "pair evals/s", "cores": 1, "kind": "oracle",
               "sample": "1 of the 55 pairs (Q_s(V_0,V_1)) on the full 32^3 grid, float64 oracle "
                         "(FFT form of the operator, numpy, single thread)",
               "seconds": round(dt, 2)}

    line = {
        "metric": "Q(V_i,V_j) evals/s at N_v=32^3",
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
        "config": {"workload": "55 pair collisions Q_s(V_i,V_j) of the rank-10 basis of a Mach-1.5 "
                               "shock state, N_v=32^3 on [-8,8]^3, hard spheres, M_rho=16 x M_sigma=38",
                   "mode": args.mode, "r": r, "pairs": P, "n_v": spec.n, "nx": nx,
                   "path": "generic" if args.generic else "default"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "plain_fp64_pair_evals_per_s": round(plain, 2) if plain else None,
        "kernels": [{k: (round(v, 4) if isinstance(v, float) else v) for k, v in t.items()}
                    for t in sorted(timers, key=lambda t: -t["ms"])[:8]],
    }
    print(json.dumps(line))
    ctx.close()


if __name__ == "__main__":
    main()
