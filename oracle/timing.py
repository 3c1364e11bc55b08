"""Time oracle steps of the cylinder workload from a saved state (the benchmark's CPU-baseline leg).

TEST INFRASTRUCTURE ONLY: run by bench.py as a child process, so that the OpenMP build of the
oracle (CGP_ORACLE_OPENMP=1, OMP_NUM_THREADS) can be timed beside the single-thread one.

    python -m oracle.timing STATE.npz TARGET_TRIS STEPS MOM_TOL P_TOL MASS_TOL

STATE.npz holds u [n_f][2], pc [n_c] and g [n_f][2].  Prints one JSON line: seconds per step, the
threads used and the last step's solver iterations.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np


def main(argv):
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import oracle
    import workloads as W
    state, tris, steps = argv[0], int(argv[1]), int(argv[2])
    tol_mom, tol_p, tol_mass = float(argv[3]), float(argv[4]), float(argv[5])
    d = np.load(state)
    case = W.case_cylinder(tris)
    P = oracle.Problem(case.mesh, 1)
    P.assemble(case.rho, case.mu, case.dt)
    u, pc = d["u"], d["pc"]
    t0 = time.perf_counter()
    for _ in range(steps):
        u, pf, pc, code, st = P.step(d["g"], u, pc, tol_mom=tol_mom, tol_p=tol_p, tol_mass=tol_mass)
    el = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", "1")) if os.environ.get("CGP_ORACLE_OPENMP") == "1" else 1
    print(json.dumps(dict(s_per_step=el / steps, steps=steps, threads=threads, code=code, p_iters=st["p_iters"])))


if __name__ == "__main__":
    main(sys.argv[1:])
