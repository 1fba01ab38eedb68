"""lb_diagnostics_noalloc (the entry point that allocates nothing) against
lb_diagnostics, through the C ABI: two calls in a row on different lattices,
the second smaller, each compared bit for bit with the allocating call; the
size limit; and that a non-finite state is reported the same way."""
import numpy as np
import pytest

from paper_0812_1282_amd import lbm, workloads as wl

pytestmark = pytest.mark.gpu

KEYS = ("sum_rho", "sum_phi", "kinetic", "max_u", "n_fluid", "step", "rc")


def say(msg):
    print(msg, flush=True)


def _drop(nx, ny, storage, seed, steps):
    say(f"case noalloc: {nx}x{ny} {storage} drop, {steps} steps")
    p = wl.params(nx, ny, 1.0, 0.55, "mrt")
    inp = wl.drop_on_wall(p, 0.35 * ny, nx / 2, 0.0, seed, -0.1)
    lat = lbm.lb_init(lbm.make_params(p, storage), inp["solid"], inp["phi0"], dphi=inp["dphi"],
                      rho0=inp["rho0"], ux0=inp["ux0"], uy0=inp["uy0"])
    lbm.lb_step(lat, steps)
    return lat


@pytest.mark.parametrize("storage", ["f64", "f32", "f16s"])
def test_noalloc_matches_diagnostics_on_two_calls_second_smaller(storage):
    big = _drop(1000, 700, storage, 1, 40)      # 2734 partial records
    small = _drop(67, 13, storage, 2, 7)        # 4 records: the rest of the array is stale
    for lat in (big, small, big):
        a = lbm.lb_diagnostics(lat)
        b = lbm.lb_diagnostics_noalloc(lat)
        assert all(a[k] == b[k] for k in KEYS), (storage, a, b)
        assert b["n_fluid"] == int((lat.params.ny - 2) * lat.params.nx)
    big.close()
    small.close()


def test_noalloc_size_limit():
    """2^23 nodes is the largest lattice; one row more is rejected."""
    ok = _drop(4096, 2048, "f32", 3, 2)
    a = lbm.lb_diagnostics(ok)
    b = lbm.lb_diagnostics_noalloc(ok)
    assert all(a[k] == b[k] for k in KEYS)
    ok.close()
    over = _drop(4096, 2049, "f32", 3, 1)
    with pytest.raises(lbm.LbError) as e:
        lbm.lb_diagnostics_noalloc(over)
    assert e.value.code == lbm.LB_EINVAL
    assert lbm.lb_diagnostics(over)["rc"] == 0      # the allocating call still works
    over.close()


def test_noalloc_reports_non_finite_state():
    """A state driven non-finite (tau just above 1/2 with a strong flow) gives
    LB_ENUMERIC from both calls."""
    p = wl.params(64, 16, 0.5001, 0.5001, "bgk")
    inp = wl.random_fields(p, seed=2, amp_u=0.4)
    say("case noalloc: unstable 64x16 run, 2000 steps")
    lat = lbm.lb_init(lbm.make_params(p, "f64"), inp["solid"], inp["phi0"], dphi=inp["dphi"],
                      rho0=inp["rho0"], ux0=inp["ux0"], uy0=inp["uy0"])
    lbm.lb_step(lat, 2000)
    a = lbm.lb_diagnostics(lat, check=False)
    b = lbm.lb_diagnostics_noalloc(lat, check=False)
    assert a["rc"] == b["rc"] == lbm.LB_ENUMERIC
    lat.close()
