"""Write order_parameter_config2_n30000.json: the FP64 oracle's r(t) over ten
time units (RK4, dt 0.01, 1000 steps) and every community's own order
parameter at t = 10 on the power-law Kuramoto recipe at N = 30000 (community
sizes ~ s^-2 on [100, 5000], p_in 0.95, mean inter degree 5, Cauchy(0, 0.5)
frequencies, K = 3; seed 51: the largest community has 4929 nodes).

r(t) is the modulus of the mean of e^{i theta} over all nodes (App. A.4,
the first Kuramoto order parameter); r_c is the same over the nodes of
community c.  Calls only the oracle and the seeded input generators; about a
quarter of an hour on eight host cores.

    python3 tests/golden/make_order_parameter_config2.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

N, SEED, STEPS = 30000, 51, 1000
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "order_parameter_config2_n30000.json")


def main():
    P = W.scaled_kuramoto(N, seed=SEED, hi=5000)
    g = P.graph
    t0 = time.time()
    th, r = oracle.phase_integrate(g.n, g.row_ptr, g.col, P.omega, P.K, [0, 1], [0, 0], P.theta0, P.dt, STEPS)
    labs = np.unique(g.labels[g.labels >= 0])
    r_c = [float(np.abs(np.exp(1j * th[g.labels == c]).mean())) for c in labs]
    doc = {
        "what": "FP64 oracle r(t), RK4 dt 0.01 over 10 time units, and per-community r_c at t = 10",
        "source": "App. A.4 (first Kuramoto order parameter); eq. (2.1) Kuramoto network; oracle.phase_integrate",
        "recipe": {"n": N, "seed": SEED, "lo": 100, "hi": 5000, "K": P.K, "dt": P.dt, "steps": STEPS},
        "check": {"nnz": int(g.nnz), "ncomm": int(g.ncomm), "sum_omega": float(P.omega.sum()),
                  "sum_theta0": float(P.theta0.sum())},
        "r": [float(x) for x in r],
        "communities": [int(c) for c in labs],
        "r_c": r_c,
    }
    with open(OUT, "w") as f:
        json.dump(doc, f, separators=(",", ":"))
    print("wrote %s (%.0f s)" % (OUT, time.time() - t0))


if __name__ == "__main__":
    main()
