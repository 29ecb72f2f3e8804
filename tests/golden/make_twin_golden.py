"""Writes twin_theta.json: contact angles of the half-size throughput twin
(64 x 64 x 32 box, cap radius 12, g_ab = g_wall = 0.12, tau = 1, psi = rho,
seed 0) for the nine wall asymmetries in [-0.4, 0.4], after 20000 steps of
the FP64 CPU oracle.  Calls only oracle/ and workloads/.  Slow (tens of
minutes on 8 cores); the GPU test compares against the stored values.

    python tests/golden/make_twin_golden.py [steps]
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads as W  # noqa: E402


def main():
    steps = int(sys.argv[1]) if len(sys.argv) > 1 else 20000
    out = {"box": [64, 64, 32], "radius": 12.0, "g_ab": 0.12, "steps": steps, "seed": 0,
           "source": "oracle (FP64 CPU), tests/golden/make_twin_golden.py", "cases": []}
    for delta in W.THROUGHPUT_DELTAS:
        t0 = time.time()
        c = W.config_throughput_twin(delta=float(delta))
        L = oracle.Lattice(c["params"], c["solid"])
        L.init_equilibrium(c["rho_a"], c["rho_b"])
        L.step(steps)
        ca = L.contact_angle(c["ca"])
        obs = L.observables()
        rec = {"delta": float(delta), "theta_e1": ca["theta_e1"], "theta_e2": ca["theta_e2"],
               "flags": ca["flags"], "status": ca["status"], "mass": list(obs["mass"])}
        out["cases"].append(rec)
        print(json.dumps(rec), f"{time.time() - t0:.0f}s", flush=True)
    with open(os.path.join(HERE, "twin_theta.json"), "w") as f:
        json.dump(out, f, indent=1, allow_nan=True)


if __name__ == "__main__":
    main()
