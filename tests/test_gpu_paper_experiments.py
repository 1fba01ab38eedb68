"""The paper's own capillary-filling experiment (Sec. VII, Fig. 5) on the GPU:
the multiple-relaxation-time advancing angle extrapolated to Ca -> 0 against
the values the paper states (tests/golden/fig5_advancing_angle.txt).

One batched launch per step advances the three mobilities together; FP32
storage (held to the FP64 oracle at 10^-3 in phi by the precision tests);
10^6 steps, about a minute on one MI355X."""
import os
import sys

import numpy as np
import pytest

from paper_0812_1282_amd import experiments

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "fig5_advancing_angle.txt")


def _golden():
    rows = [l.split() for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    return {float(m): (float(mrt), float(bgk)) for m, mrt, bgk in rows}


def test_fig5_mrt_advancing_angle_at_zero_capillary_number():
    gold = _golden()
    print("case fig5 MRT f32, M = 0.05, 0.1, 0.5", flush=True)
    sys.stdout.flush()
    res = experiments.fig5(steps=1_000_000, every=10_000, storage="f32",
                           mobilities=tuple(sorted(gold)), collisions=("mrt",))
    for run in res["runs"]:
        m = run["mobility"]
        fit = run["fit"]
        assert run["alive"] and fit is not None
        th = fit["theta_a_ca0"]
        print(f"  M = {m}: theta_a(Ca -> 0) = {th:.2f} (paper {gold[m][0]})", flush=True)
        # the paper states whole degrees read off a linear fit
        assert abs(th - gold[m][0]) <= 2.5
        # Washburn-type growth: l^2 linear in t within 20% of the closed form
        assert 0.8 < fit["washburn"]["ratio"] < 1.2
    # more mobility, more inter-diffusion at the contact line, faster filling
    finals = [run["records"][-1][1] for run in res["runs"]]
    assert np.all(np.diff(finals) > 0)


@pytest.mark.xfail(strict=True, reason=(
    "BGK theta_a(Ca -> 0) measured 67.4/67.8/67.7 degrees against the paper's 75/73/72 for "
    "M = 0.05/0.1/0.5: above MRT (59-60) as the paper finds, but 5-7 degrees below its BGK "
    "values; the paper does not state a and kappa (only gamma = 0.0188) or its BGK details"))
def test_fig5_bgk_advancing_angle_at_zero_capillary_number():
    """The single-relaxation-time column of Fig. 5 (Sec. VII): the advancing
    angle at Ca -> 0 against the paper's BGK values, within 2.5 degrees. Kept as
    a strict expected failure with the measured values (see the reason)."""
    gold = _golden()
    print("case fig5 BGK f32, M = 0.05, 0.1, 0.5", flush=True)
    res = experiments.fig5(steps=1_000_000, every=10_000, storage="f32",
                           mobilities=tuple(sorted(gold)), collisions=("bgk",))
    ths = {}
    for run in res["runs"]:
        m = run["mobility"]
        assert run["alive"] and run["fit"] is not None
        ths[m] = run["fit"]["theta_a_ca0"]
        print(f"  M = {m}: theta_a(Ca -> 0) = {ths[m]:.2f} (paper {gold[m][1]})", flush=True)
        # above the MRT value the paper states, as it finds
        assert ths[m] > gold[m][0] + 3.0
    for m, th in ths.items():
        assert abs(th - gold[m][1]) <= 2.5
