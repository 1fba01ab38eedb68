"""The persistent schedule of batched ensembles: one launch per window of steps,
work items (step, tile) taken in order, a tile swept once its neighbouring tiles
have finished the previous step. Results must equal the stepwise schedule (one
launch per step) and solo runs bit for bit; a wait that exceeds its poll limit
must surface as an error on every read of the batch, with every workgroup
leaving."""
import sys

import numpy as np
import pytest

from oracle import analysis
from paper_0812_1282_amd import lbm, workloads as wl

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _members(n=6, seed=0):
    """Members of uneven size (narrow ones on wide tiles, ragged edges)."""
    sizes = [(64, 32), (128, 64), (256, 128), (67, 13), (300, 37), (512, 96)]
    out = []
    for k in range(n):
        nx, ny = sizes[k % len(sizes)]
        d = dict(nx=nx, ny=ny, theta=40.0 + 17.0 * k, tau_beta=0.55 + 0.05 * k, seed=800 + k + seed)
        p, inp = wl.c5_member(d, analysis.theory_dphi(d["theta"], 0.04, 0.04))
        out.append((p, inp))
    return out


def _batch(members, storage, tuning, schedule, diag_every=0):
    params = [lbm.make_params(p, storage, diag_every=diag_every) for p, _ in members]
    b = lbm.lb_batch_init(params, [inp for _, inp in members], tuning=tuning)
    lbm.lb_batch_set_schedule(b, schedule)
    return b


@pytest.mark.parametrize("storage", ["f64", "f32", "f16s"])
@pytest.mark.parametrize("tuning", [(128, 4), (256, 8), (512, 3)])
def test_persistent_equals_stepwise(storage, tuning):
    members = _members()
    say(f"case persistent vs stepwise {storage} tiles {tuning}")
    a = _batch(members, storage, tuning, lbm.STEPWISE)
    b = _batch(members, storage, tuning, lbm.PERSISTENT)
    assert lbm.lb_batch_get_schedule(b) == lbm.PERSISTENT
    for n in (1, 7, 32, 45):           # windows of several lengths, both parities
        lbm.lb_batch_step(a, n)
        lbm.lb_batch_step(b, n)
    for k in range(len(members)):
        fa, ga = lbm.lb_batch_read_populations(a, k)
        fb, gb = lbm.lb_batch_read_populations(b, k)
        assert np.array_equal(fa, fb) and np.array_equal(ga, gb), k
    a.close()
    b.close()


def test_persistent_with_periodic_checks_equals_solo():
    """diag_every = 10: the checked steps run stepwise inside the windows; every
    member equals its solo lattice."""
    members = _members(4, seed=1)
    say("case persistent with checks vs solo")
    b = _batch(members, "f32", (256, 8), lbm.PERSISTENT, diag_every=10)
    lbm.lb_batch_step(b, 123)
    for k, (p, inp) in enumerate(members):
        solo = lbm.lb_init(lbm.make_params(p, "f32", diag_every=10), inp["solid"], inp["phi0"],
                           dphi=inp["dphi"], rho0=inp["rho0"])
        lbm.lb_step(solo, 123)
        fb, gb = lbm.lb_batch_read_populations(b, k)
        fs, gs = lbm.lb_read_populations(solo)
        assert np.array_equal(fb, fs) and np.array_equal(gb, gs), k
        solo.close()
    lbm.lb_batch_read_fields(b, 0)     # the checks found nothing
    b.close()


def test_persistent_rejects_unsupported_tunings():
    members = _members(3)
    b = _batch(members, "f32", (64, 8), lbm.STEPWISE)
    with pytest.raises(lbm.LbError) as e:
        lbm.lb_batch_set_schedule(b, lbm.PERSISTENT)      # block_x 64
    assert e.value.code == lbm.LB_EINVAL
    assert lbm.lb_batch_get_schedule(b) == lbm.STEPWISE
    b.close()
    b = _batch(members, "f32", (256, 2), lbm.STEPWISE)
    with pytest.raises(lbm.LbError):
        lbm.lb_batch_set_schedule(b, lbm.PERSISTENT)      # strips of 2 rows
    b.close()


def test_persistent_wait_limit_reports_an_error():
    """A poll limit of one: the second step of a one-tile member must wait for
    the first, gives up at once, and the batch reports LB_EHIP; the grid still
    drains (the next batch runs normally)."""
    members = _members(1)
    say("case persistent poll limit 1")
    b = _batch(members, "f32", (256, 8), lbm.STEPWISE)
    lbm.lb_batch_set_schedule(b, lbm.PERSISTENT, spin_limit=1)
    lbm.lb_batch_step(b, 32)
    with pytest.raises(lbm.LbError) as e:
        lbm.lb_batch_read_fields(b, 0)
    assert e.value.code == lbm.LB_EHIP
    with pytest.raises(lbm.LbError) as e:            # populations are not handed back
        lbm.lb_batch_read_populations(b, 0)
    assert e.value.code == lbm.LB_EHIP
    b.close()
    ok = _batch(members, "f32", (256, 8), lbm.PERSISTENT)
    lbm.lb_batch_step(ok, 32)
    lbm.lb_batch_read_fields(ok, 0)
    ok.close()


def test_autotuned_batch_equals_solo():
    """lb_batch_init without a tuning times both schedules; whatever it keeps,
    members equal their solo lattices."""
    members = _members(5, seed=2)
    say("case autotuned batch vs solo")
    params = [lbm.make_params(p, "f32") for p, _ in members]
    b = lbm.lb_batch_init(params, [inp for _, inp in members])
    say(f"  chose {lbm.lb_batch_get_tuning(b)} schedule {lbm.lb_batch_get_schedule(b)}")
    lbm.lb_batch_step(b, 77)
    for k, (p, inp) in enumerate(members):
        solo = lbm.lb_init(lbm.make_params(p, "f32"), inp["solid"], inp["phi0"],
                           dphi=inp["dphi"], rho0=inp["rho0"])
        lbm.lb_step(solo, 77)
        fb, gb = lbm.lb_batch_read_populations(b, k)
        fs, gs = lbm.lb_read_populations(solo)
        assert np.array_equal(fb, fs) and np.array_equal(gb, gs), k
        solo.close()
    b.close()
