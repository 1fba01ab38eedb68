"""The oracle side of checkpoint/resume and failure detection.

Checkpoint: the state S_n is the whole of what a step depends on, so a run of
1000 steps equals 500 steps, the populations written to a file, a fresh lattice
loaded from that file, and 500 more, bit for bit (also with lattice-node
bounce-back, where wall nodes hold populations in flight). Failure detection: a
run driven unstable (tau close to 1/2 and a large velocity) ends with
non-finite sums, which is what the GPU library's periodic check reports; the
same set-up at tau = 1 stays finite; non-finite inputs are rejected."""
import numpy as np
import pytest

from oracle import analysis
from paper_0812_1282_amd import workloads as wl
from tests.helpers import make_oracle


@pytest.mark.parametrize("bounce", [0, 1])
def test_oracle_checkpoint_resume_is_bitwise(tmp_path, bounce):
    p, inp = wl.c1_drop(seed=1, dphi_wall=analysis.theory_dphi(60.0, 0.04, 0.04))
    a = make_oracle(p, inp, bounce=bounce)
    a.step(1000)
    ref = a.populations()
    b = make_oracle(p, inp, bounce=bounce)
    b.step(500)
    path = tmp_path / "state.npz"
    f, g = b.populations()
    np.savez(path, f=f, g=g)
    del b
    c = make_oracle(p, inp, bounce=bounce)
    with np.load(path) as z:
        c.set_populations(z["f"], z["g"])
    c.step(500)
    out = c.populations()
    assert np.array_equal(out[0], ref[0]) and np.array_equal(out[1], ref[1])
    assert a.diagnostics() == c.diagnostics()


def test_oracle_unstable_run_goes_non_finite():
    p = wl.params(64, 16, 0.5001, 0.5001, "bgk")
    inp = wl.random_fields(p, seed=2, amp_u=0.4)
    o = make_oracle(p, inp)
    o.step(2000)
    d = o.diagnostics()
    assert not (np.isfinite(d["kinetic"]) and np.isfinite(d["sum_rho"]))
    p = wl.params(64, 16, 1.0, 1.0, "bgk")
    inp = wl.random_fields(p, seed=2)
    o = make_oracle(p, inp)
    o.step(200)
    d = o.diagnostics()
    assert all(np.isfinite(d[k]) for k in ("sum_rho", "sum_phi", "kinetic", "max_u"))


@pytest.mark.parametrize("field", ["phi0", "rho0", "ux0", "uy0"])
@pytest.mark.parametrize("bad", [np.nan, np.inf, -np.inf])
def test_oracle_rejects_non_finite_inputs(field, bad):
    p = wl.params(10, 8, 1.0, 1.0, "bgk")
    inp = wl.random_fields(p, seed=1)
    inp[field] = inp[field].copy()
    inp[field][4, 5] = bad
    with pytest.raises(ValueError):
        make_oracle(p, inp)
