"""Writes ``steady_shock_2d.npz``: the oracle's adaptive low-rank steady solve
of a small normal shock, the expected values of the served steady-solve test.

Setup (Sec. 5.2's normal shock, scaled down): 2D velocity, Maxwell molecules
B = 1/(2 pi), N_v = 32^2 on [-8, 8]^2, 8 Gauss-Legendre radial x 8 circle
nodes; N_x = 32 cells on [-30, 30]; Mach 1.4 (the paper's weak shock) with
the Rankine-Hugoniot end states as inflow; initial data the tanh blend of
Sec. 5.2 plus a seeded rank-3 perturbation of relative size 1e-3, truncated
to rank 6; forward Euler dt = 0.1; add the boundary basis (add_tol 1e-10) and
drop with c = 0.2 every step (Sec. 3, Sec. 5.1), r_max 16; stop when err_ada
<= 1e-6 (Sec. 5.1).

Stored: rho, u_1, T per cell at the stopping step, the step count, the final
rank and the err_ada history.  Calls only the oracle and the input generator.
Run from the repository root:  python tests/golden/make_steady_shock.py
(about an hour on one core).
"""
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import collision as oc  # noqa: E402
from oracle import dlr  # noqa: E402

SETUP = dict(d=2, n=32, L=8.0, C=1.0 / (2.0 * math.pi), gamma=0.0, m_rho=8, m_sigma=8, nx=32,
             x_lo=-30.0, x_hi=30.0, mach=1.4, pert=1e-3, pert_rank=3, seed=7, r0=6, dt=0.1,
             c=0.2, add_tol=1e-10, r_max=16, res_tol=1e-6, max_steps=8000)


def problem(s=SETUP):
    spec = synth.VGridSpec(d=s["d"], n=s["n"], L=s["L"], gamma=s["gamma"], C=s["C"],
                           m_rho=s["m_rho"], m_sigma=s["m_sigma"])
    vs = oc.setup_from_spec(spec)
    ini = synth.shock_initial(s["mach"], spec, s["nx"], s["x_lo"], s["x_hi"], pert=s["pert"],
                              pert_rank=s["pert_rank"], seed=s["seed"])
    prob = dlr.Problem1D(vs=vs, nx=s["nx"], x_lo=s["x_lo"], x_hi=s["x_hi"], fL=ini["fL"],
                         fR=ini["fR"])
    X, S, V = synth.lowrank_state(ini["f0"], s["r0"], prob.dx, prob.dvd)
    return spec, prob, ini, (X, S, V)


def main():
    s = SETUP
    spec, prob, ini, (X, S, V) = problem()
    st = dlr.State(X, S, V)
    hist = []
    t0 = time.time()
    converged = False
    for k in range(s["max_steps"]):
        st, info = dlr.adaptive_step(st, prob, s["dt"], c=s["c"], add_tol=s["add_tol"],
                                     r_max=s["r_max"])
        hist.append(info.err_ada)
        if k % 100 == 0:
            print(f"step {k} err_ada {info.err_ada:.3e} r {st.r} {time.time() - t0:.0f}s", flush=True)
        if info.err_ada <= s["res_tol"]:
            converged = True
            break
    rho, u, T = dlr.macroscopic(st, prob)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "steady_shock_2d.npz")
    np.savez(out, rho=rho, u=u, T=T, steps=len(hist), r=st.r, converged=converged,
             err_ada=np.array(hist))
    print(f"wrote {out}: steps {len(hist)} converged {converged} r {st.r}", flush=True)


if __name__ == "__main__":
    main()
