"""Write the stored FP64 oracle records that the GPU tests compare against.

Only the oracle (oracle/) and the seeded input layouts (workloads.py) are used.
Re-run after any change to the oracle's arithmetic or to the inputs:

    python tests/golden/make_oracle_records.py

c3_oracle_256x32.json   capillary filling at 256 x 32 (the capillary layout of
                        the 1024 x 64 workload scaled: walls on [128, 224),
                        h = 30, 60-degree wall, MRT), viscosity ratios 1 and 10:
                        every 500 steps to 2 x 10^4 the column length l, the
                        centreline meniscus position and the advancing angle at
                        the bottom wall (Sec. VII)
c5_oracle_sample.npz    the first member of each size of the 256-member ensemble
                        (seed 5), then each size's member with the target angle
                        farthest from 90 degrees, after 10^4 steps: phi on every
                        second row and column, and the contact angle (Sec. IV)
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import analysis as an  # noqa: E402
from paper_0812_1282_amd import workloads as wl  # noqa: E402
from tests.helpers import make_oracle  # noqa: E402

KAPPA = A_L = 0.04
C3_NX, C3_NY, C3_IN, C3_OUT, C3_H = 256, 32, 128, 224, 30.0
C3_STEPS, C3_EVERY = 20000, 500
C5_STEPS = 10000


def meniscus_x(phi, x_lo, x_hi, row):
    r = phi[row]
    for x in range(max(x_lo, 0), x_hi - 1):
        if r[x] > 0 >= r[x + 1]:
            return x + r[x] / (r[x] - r[x + 1])
    return None


def c3_window(xm):
    """Crossings behind and around the meniscus, away from both walls."""
    return (xm - 24.0, xm + 12.0, 3.5, C3_NY - 4.5)


def c3_record(ratio):
    p, inp = wl.c3_capillary(C3_NX, C3_NY, ratio, an.theory_dphi(60.0, KAPPA, A_L), seed=3)
    o = make_oracle(p, inp)
    fluid = inp["solid"] == 0
    rec = []
    for k in range(C3_STEPS // C3_EVERY):
        o.step(C3_EVERY)
        phi = o.fields()[0]
        ch = slice(C3_IN, C3_OUT)
        l = float((0.5 * (1 + phi[:, ch]))[fluid[:, ch]].sum() / C3_H)
        xm = meniscus_x(phi, C3_IN - 16, C3_OUT, C3_NY // 2)
        th = None
        if xm is not None and C3_IN + 10 < xm < C3_OUT - 10:
            res = an.contact_angle(phi, inp["solid"], 0.5, 1, *c3_window(xm))
            th = None if res is None else res["theta"]
        rec.append([(k + 1) * C3_EVERY, l, xm, th])
    return rec


def c5_members():
    """The first member of each size (by width), then, for each size, the member
    whose target angle is farthest from 90 degrees (the ends of the range)."""
    ins = wl.c5_instances()
    descs, seen = [], set()
    for d in ins:
        if (d["nx"], d["ny"]) not in seen:
            seen.add((d["nx"], d["ny"]))
            descs.append(d)
    descs.sort(key=lambda d: d["nx"])
    for first in list(descs):
        same = [d for d in ins if (d["nx"], d["ny"]) == (first["nx"], first["ny"])]
        descs.append(max(same, key=lambda d: abs(d["theta"] - 90.0)))
    return descs


def c5_window(d):
    return (0.0, float(d["nx"]), 3.5, d["ny"] - 4.5)


def main():
    t0 = time.time()
    c3 = {"nx": C3_NX, "ny": C3_NY, "x_in": C3_IN, "x_out": C3_OUT, "h": C3_H,
          "every": C3_EVERY, "steps": C3_STEPS, "records": {}}
    for ratio in (1, 10):
        c3["records"][str(ratio)] = c3_record(ratio)
        print(f"c3 ratio {ratio}: l = {c3['records'][str(ratio)][-1][1]:.3f} "
              f"({time.time() - t0:.0f} s)", flush=True)
    with open(os.path.join(HERE, "c3_oracle_256x32.json"), "w") as f:
        json.dump(c3, f, indent=1)
    out = {}
    for k, d in enumerate(c5_members()):
        dphi = an.theory_dphi(d["theta"], KAPPA, A_L)
        p, inp = wl.c5_member(d, dphi)
        o = make_oracle(p, inp)
        o.step(C5_STEPS)
        phi = o.fields()[0]
        th = an.contact_angle(phi, inp["solid"], 0.5, 1, *c5_window(d))["theta"]
        out[f"phi{k}"] = phi[::2, ::2].copy()
        out[f"desc{k}"] = np.array([d["nx"], d["ny"], d["seed"], d["theta"], d["tau_beta"]])
        out[f"theta{k}"] = np.array(th)
        print(f"c5 member {d['nx']}x{d['ny']} theta {d['theta']:.2f} -> {th:.3f} "
              f"({time.time() - t0:.0f} s)", flush=True)
    np.savez_compressed(os.path.join(HERE, "c5_oracle_sample.npz"), **out)


if __name__ == "__main__":
    main()
