"""Stability of the single-relaxation-time (BGK) run of the 256 x 128 drop with
unequal viscosities, on the FP64 oracle: tau_alpha = 1 (phi = +1) and tau_beta
from 0.55 (the workload's value, viscosity ratio 10) upward, a 90-degree wall.
Every 500 steps, up to 2 x 10^4: the peak speed within 5 nodes of the contact
points on the first fluid row (reading R15) and over the lattice, until the
conservation sums stop being finite. Writes c2_bgk_stability.json.

    python tests/golden/make_c2_bgk_stability.py

Only the oracle (oracle/) and the seeded layouts (workloads.py) are used."""
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from paper_0812_1282_amd import workloads as wl  # noqa: E402
from tests.helpers import make_oracle  # noqa: E402

STEPS, EVERY = 20000, 500
TAU_BETA = (0.55, 0.56, 0.57, 0.58, 0.6, 0.65, 0.7, 0.8, 1.0)


def near_contact_speed(phi, ux, uy, solid, radius=5.0):
    speed = np.hypot(ux, uy)
    fluid = solid == 0
    row = phi[1]
    xs = [x + row[x] / (row[x] - row[x + 1]) for x in range(len(row) - 1)
          if fluid[1, x] and fluid[1, x + 1] and row[x] * row[x + 1] < 0]
    ny, nx = phi.shape
    y, x = np.mgrid[0:ny, 0:nx]
    near = np.zeros_like(fluid)
    for xc in xs:
        near |= np.hypot(x - xc, y - 1.0) <= radius
    near &= fluid
    return (float(speed[near].max()) if near.any() else None), float(speed[fluid].max())


def main():
    out = {"workload": "C2 drop 256x128 R=60, BGK, tau_alpha = 1, 90-degree wall, FP64 oracle",
           "steps": STEPS, "every": EVERY, "runs": []}
    t0 = time.time()
    for tb in TAU_BETA:
        p, inp = wl.c2_drop("bgk", 0.0)
        p = dict(p, tau_beta=tb)
        o = make_oracle(p, inp)
        rec, dead = [], None
        for k in range(STEPS // EVERY):
            o.step(EVERY)
            d = o.diagnostics()
            if not (math.isfinite(d["sum_rho"]) and math.isfinite(d["max_u"])):
                dead = (k + 1) * EVERY
                break
            phi, rho, ux, uy = o.fields()
            near, glob = near_contact_speed(phi, ux, uy, inp["solid"])
            rec.append([(k + 1) * EVERY, near, glob])
        out["runs"].append({"tau_beta": tb, "viscosity_ratio": (1.0 - 0.5) / (tb - 0.5),
                            "nonfinite_by": dead, "records": rec})
        print(f"tau_beta {tb}: non-finite by {dead}, last record {rec[-1] if rec else None} "
              f"({time.time() - t0:.0f} s)", flush=True)
    with open(os.path.join(HERE, "c2_bgk_stability.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
