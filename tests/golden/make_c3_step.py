"""Writes ``c3_step.npz``: the oracle's values for the benchmark's own workload
(the expected values of ``tests/test_gpu_c3_golden.py`` and of the parity
figures the benchmark reports).

Workload: the Mach-1.5 normal shock of Sec. 5.2 in 3D velocity, N_v = 32^3 on
[-8, 8]^3, hard spheres B = |v - v*| (C = 1), 16 Gauss-Legendre radial x 38
Lebedev sphere nodes; N_x = 256 cells on [-30, 30]; the tanh blend of the
Rankine-Hugoniot end states plus a seeded rank-10 perturbation of relative
size 1e-3, truncated to rank 10 (the input generator's factors).  One adaptive
step as the benchmark takes it: add the boundary basis (Sec. 3.1, add_tol
1e-10, r_max 12: rank 10 -> 12), the 78 pair collisions of the augmented
basis with the conservation projection, the K, S and L steps with forward
Euler dt = 0.01 (Sec. 2.4), the residual (Sec. 5.1), the drop with
c = 0.2 and r_min 10 (Sec. 3.2).

Stored:
  V_aug32     the augmented rank-12 basis rounded to float32 (the input of the
              pair test: the FP32 path computes from exactly these values);
  q32         Q_s(V_i, V_j) of all 78 pairs of V_aug32 (promoted to float64,
              oracle in float64, projection on), rounded to float32;
  qplus_norm, q_norm   ||Q_s^+||_2 and ||Q_s||_2 of each pair (float64);
  X0, S0, V0  the initial rank-10 factors (float64; X0 is nx x 10): the
              input of the step test, stored because the input generator's
              SVD differs between machines at the 1e-12 level in the
              singular vectors of the smallest singular values, and the step
              result follows such differences at the same level;
  S0_sv       singular values of the initial S;
  X1, S1, V1  the state after the step (float64; X1 is nx x r_out);
  XF, SF, VF, errF   the fixed-rank step (no augmentation, no drop) from
              the same state: K, S, L steps with the 55 pairs of rank 10;
  err, err_ada, drop_tol, r_added, r_out    the step's report;
  gain_scale  ||sum_{m<=n} (2 - delta_mn) K_m K_n Q_s^+(V_m, V_n)||_{x,v}
              with K = X S of the augmented state: the scale of the FP32
              collision bound of a step (error <= 1e-5 dt gain_scale).

Calls only the oracle and the input generator; the pair evaluations run in a
process pool (each pair is the oracle's own serial computation).
Run from the repository root:  python tests/golden/make_c3_step.py
(about three minutes on 8 cores).
"""
import math
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import collision as oc  # noqa: E402
from oracle import dlr  # noqa: E402

SETUP = dict(mach=1.5, nx=256, x_lo=-30.0, x_hi=30.0, pert=1e-3, pert_rank=10, seed=3, r0=10,
             r_max=12, dt=0.01, c=0.2, add_tol=1e-10)
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c3_step.npz")


def problem(s=SETUP):
    spec = synth.C3
    vs = oc.setup_from_spec(spec)
    ini = synth.shock_initial(s["mach"], spec, s["nx"], s["x_lo"], s["x_hi"], pert=s["pert"],
                              pert_rank=s["pert_rank"], seed=s["seed"])
    prob = dlr.Problem1D(vs=vs, nx=s["nx"], x_lo=s["x_lo"], x_hi=s["x_hi"], fL=ini["fL"],
                         fR=ini["fR"])
    X, S, V = synth.lowrank_state(ini["f0"], s["r0"], prob.dx, prob.dvd)
    return spec, prob, ini, dlr.State(X, S, V)


_VS = None


def _init_worker():
    global _VS
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except ImportError:
        pass
    _VS = oc.setup_from_spec(synth.C3)


def _one(args):
    V, pair, conserve = args
    q, g = oc.q_pairs(V, [pair], _VS, conserve=conserve)
    return q[0], g[0]


class PoolEvaluator:
    """prob.collision for the oracle step: the pairs spread over processes."""

    def __init__(self, pool):
        self.pool = pool
        self.last_gains = None

    def __call__(self, V, pairs, vs, conserve):
        res = self.pool.map(_one, [(V, p, conserve) for p in pairs], chunksize=1)
        Q = np.array([a for a, _ in res])
        G = np.array([b for _, b in res])
        self.last_gains = G
        return Q, G


def main():
    s = SETUP
    t0 = time.time()
    spec, prob, ini, st = problem()
    workers = os.cpu_count() or 1
    with mp.get_context("fork").Pool(workers, initializer=_init_worker) as pool:
        ev = PoolEvaluator(pool)
        prob.collision = ev
        # the augmented basis of the step (the random X block does not enter f)
        aug, rb = dlr.add_boundary_basis(st, prob, s["add_tol"], s["r_max"],
                                         np.random.default_rng(0))
        assert rb == 2 and aug.r == 12
        pairs = dlr.pair_list(aug.r)
        V32 = aug.V.astype(np.float32)
        print(f"pairs of the float32 basis ({len(pairs)}) ...", flush=True)
        q32, g32 = ev(V32.astype(np.float64), pairs, prob.vs, True)
        print(f"  {time.time() - t0:.0f}s; adaptive step ...", flush=True)
        new, info = dlr.adaptive_step(st, prob, s["dt"], c=s["c"], add_tol=s["add_tol"],
                                      r_min=s["r0"], r_max=s["r_max"],
                                      rng=np.random.default_rng(0))
        gains = ev.last_gains
        print(f"  {time.time() - t0:.0f}s; fixed-rank step ...", flush=True)
        fixed, errF, _ = dlr.ksl_step(st, prob, s["dt"])
    wts = np.array([1.0 if m == n else 2.0 for (m, n) in pairs])
    Kaug = aug.X @ aug.S
    gain_scale = math.sqrt(prob.dx * prob.dvd) * np.linalg.norm(
        dlr.pair_products(Kaug, pairs, wts) @ gains)
    np.savez_compressed(
        OUT, V_aug32=V32, q32=q32.astype(np.float32),
        qplus_norm=np.linalg.norm(g32, axis=1), q_norm=np.linalg.norm(q32, axis=1),
        X0=st.X, S0=st.S, V0=st.V, S0_sv=np.linalg.svd(st.S, compute_uv=False),
        X1=new.X, S1=new.S, V1=new.V, err=info.err, err_ada=info.err_ada,
        XF=fixed.X, SF=fixed.S, VF=fixed.V, errF=errF,
        drop_tol=info.drop_tol, r_added=info.r_added, r_out=info.r_out, gain_scale=gain_scale,
        dt=s["dt"], nx=s["nx"], r_max=s["r_max"], r_min=s["r0"])
    print(f"wrote {OUT}: r_added {info.r_added} r_out {info.r_out} err {info.err:.6e} "
          f"err_ada {info.err_ada:.6e} ({time.time() - t0:.0f}s)", flush=True)


if __name__ == "__main__":
    main()
