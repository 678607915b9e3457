"""Writes ``c1_c2_q.npz``: the oracle's single evaluations Q(f, f) of the two
homogeneous workloads (expected values of ``tests/test_gpu_c1_c2_golden.py``
and of the per-result errors the benchmark reports).

  C1  2D velocity, N_v = 32^2 on [-8, 8]^2, Maxwell molecules B = 1/(2 pi),
      16 Gauss-Legendre radial x 8 circle nodes; f = two unit-temperature
      Maxwellians at u = (+-2, 0) times (1 + 0.01 xi), xi ~ N(0, 1), seed 1.
  C2  3D velocity, N_v = 32^3 on [-8, 8]^3, 16 radial x 38 Lebedev nodes:
      (i)  hard spheres B = |v - v*|, f = a M(1, 0, 1) + (1 - a) M(1, (1.5, 0, 0), 0.5),
           a ~ U[0.3, 0.7], seed 2;
      (ii) Maxwell molecules B = 1/(4 pi), f = the BKW solution at t = 0.5 (with the
           time shift that keeps it positive), stored with its analytic dF/dt = Q(f, f).

For each: the input f, Q(f, f) without and with the conservation projection,
and ||Q^+||_2 (the scale of the error measure).  Calls only the oracle and
the input generator.  Run from the repository root:
  python tests/golden/make_c1_c2.py      (about half a minute)
"""
import math
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import collision as oc  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c1_c2_q.npz")

BKW_SPEC = synth.VGridSpec(d=3, n=32, L=8.0, gamma=0.0, C=1.0 / (4.0 * math.pi), m_rho=16,
                           m_sigma=38)


def evaluate(f, spec):
    vs = oc.setup_from_spec(spec)
    V = np.asarray(f, dtype=np.float64).reshape(1, -1)
    q, g = oc.q_pairs(V, [(0, 0)], vs, conserve=False)
    qc = oc.conserve_project(q[0], vs)
    return q[0], qc, float(np.linalg.norm(g[0]))


def main():
    out = {}
    f1 = synth.c1_distribution(seed=1, spec=synth.C1).reshape(-1)
    out["c1_f"] = f1
    out["c1_q"], out["c1_qc"], out["c1_gain_norm"] = evaluate(f1, synth.C1)
    f2 = synth.c2_bimaxwellian(seed=2, spec=synth.C2).reshape(-1)
    out["c2b_f"] = f2
    out["c2b_q"], out["c2b_qc"], out["c2b_gain_norm"] = evaluate(f2, synth.C2)
    fk, dfdt = synth.c2_bkw(0.5, BKW_SPEC)
    out["c2k_f"] = fk.reshape(-1)
    out["c2k_dfdt"] = dfdt.reshape(-1)
    out["c2k_q"], out["c2k_qc"], out["c2k_gain_norm"] = evaluate(fk, BKW_SPEC)
    np.savez_compressed(OUT, **out)
    e = np.abs(out["c2k_q"] - out["c2k_dfdt"]).max() / np.abs(out["c2k_dfdt"]).max()
    print(f"wrote {OUT}; BKW: oracle Q vs analytic dF/dt {e:.2e} of max|dF/dt|", flush=True)


if __name__ == "__main__":
    main()
