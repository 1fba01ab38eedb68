"""Write the stored FP64 oracle record of the unequal-viscosity wall drop.

Only the oracle (oracle/) and the seeded input layouts (workloads.py) are used.
Re-run after any change to the oracle's arithmetic or to the inputs:

    python tests/golden/make_wall_viscosity_record.py

wall_viscosity_60.json  a drop (R = 18 on a 128 x 48 channel, M = 1, Gamma = 2)
                        on a 60-degree wall (the wall gradient of Eq. (theory)),
                        with tau_alpha / tau_beta = 1 / 1 (MRT), 3 / 0.7 (MRT)
                        and 3 / 0.7 (BGK): the contact angle every 10^4 steps
                        to 4 x 10^4 (Sec. VI, Fig. 2(b))
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import analysis as an  # noqa: E402
from paper_0812_1282_amd import workloads as wl  # noqa: E402
from tests.helpers import make_oracle  # noqa: E402

KAPPA = A_L = 0.04
NX, NY, RADIUS, GAMMA, THETA = 128, 48, 18.0, 2.0, 60.0
STEPS, EVERY = 40000, 10000
WINDOW = (0.0, float(NX), 3.5, 43.5)
CASES = (("mrt", 1.0, 1.0), ("mrt", 3.0, 0.7), ("bgk", 3.0, 0.7))


def case_inputs(coll, ta, tb):
    p = wl.params(NX, NY, ta, tb, coll, Gamma=GAMMA)
    inp = wl.drop_on_wall(p, RADIUS, NX / 2, 0.0, 1, an.theory_dphi(THETA, KAPPA, A_L))
    return p, inp


def record(coll, ta, tb):
    p, inp = case_inputs(coll, ta, tb)
    o = make_oracle(p, inp)
    out = []
    for _ in range(STEPS // EVERY):
        o.step(EVERY)
        phi = o.fields()[0]
        out.append(an.contact_angle(phi, inp["solid"], 0.5, 1, *WINDOW)["theta"])
    return out


def main():
    t0 = time.time()
    rec = {"nx": NX, "ny": NY, "radius": RADIUS, "Gamma": GAMMA, "theta_target": THETA,
           "every": EVERY, "steps": STEPS, "window": list(WINDOW), "records": {}}
    for coll, ta, tb in CASES:
        rec["records"][f"{coll}-{ta}-{tb}"] = record(coll, ta, tb)
        print(coll, ta, tb, rec["records"][f"{coll}-{ta}-{tb}"], f"{time.time() - t0:.0f} s",
              flush=True)
    with open(os.path.join(HERE, "wall_viscosity_60.json"), "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
