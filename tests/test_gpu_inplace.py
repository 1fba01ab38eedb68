"""The in-place update (lb_params.inplace = 1): one population buffer, two
alternating phases. It changes where the populations are kept, not what is
computed: every result must be bit-identical to the two-buffer path (the same
pulled values summed in the same order, and the phi of tile-border nodes formed
by the pre-pass with the sweep's own arithmetic), and the FP64 path is held to
the oracle at the FP64 tolerance. The state alternates between two layouts
(even step counts, S_0 included, leave it in the one phase 1 reads; odd counts
in the one phase 0 reads), so tests stop at both even and odd counts."""
import os
import tempfile

import numpy as np
import pytest

from oracle import analysis
from paper_0812_1282_amd import lbm, workloads as wl
from tests.test_gpu_parity import D60, gpu_lattice, run_pair, say

pytestmark = pytest.mark.gpu


def pair(p, inp, storage, **kw):
    """(two-buffer, in-place) lattices of the same case."""
    return gpu_lattice(p, inp, storage, **kw), gpu_lattice(p, inp, storage, inplace=1, **kw)


def assert_same(a, b, what):
    fa, ga = lbm.lb_read_populations(a)
    fb, gb = lbm.lb_read_populations(b)
    assert np.array_equal(fa, fb) and np.array_equal(ga, gb), what
    for x, y, name in zip(lbm.lb_read_fields(a), lbm.lb_read_fields(b), ("phi", "rho", "ux", "uy")):
        assert np.array_equal(x, y), (what, name)


def random_case(collision, tau_phi, seed=11, nx=70, ny=30):
    p = wl.params(nx, ny, 1.3, 0.6, collision, Gamma=0.3, tau_phi=tau_phi)
    inp = wl.random_fields(p, seed=seed)
    rng = np.random.default_rng(seed + 1)
    inp["dphi"] = np.where(inp["solid"] != 0, rng.uniform(-0.3, 0.3, inp["solid"].shape), 0.0)
    return p, inp


@pytest.mark.parametrize("steps", [1000, 999])
def test_inplace_f64_c1_drop_against_oracle(steps):
    p, inp = wl.c1_drop(seed=1, dphi_wall=D60)
    run_pair(p, inp, steps, what=f"C1 100x50 BGK in place, {steps} steps", inplace=1)


@pytest.mark.parametrize("collision,zf,zg", [("bgk", 0, 0), ("mrt", 1, 0), ("mrt", 1, 1)])
def test_inplace_f64_every_term_against_oracle(collision, zf, zg):
    p, inp = random_case(collision, 0.8)
    run_pair(p, inp, 201, what=f"random {collision} in place step2={zf}/{zg}", inplace=1,
             zero_u_feq=zf, zero_u_geq=zg)


@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("collision", ["bgk", "mrt"])
@pytest.mark.parametrize("tau_phi", [1.0, 0.8])
def test_inplace_bit_identical_to_two_buffers(storage, collision, tau_phi):
    """Single steps, a step run that takes the 32-step graphs, and odd counts."""
    p, inp = random_case(collision, tau_phi, seed=21)
    say(f"case in place == two buffers {storage} {collision} tau_phi={tau_phi}")
    a, b = pair(p, inp, storage)
    assert_same(a, b, "S_0")
    for n in (1, 1, 5, 64, 3):
        lbm.lb_step(a, n)
        lbm.lb_step(b, n)
        assert_same(a, b, f"after +{n} (step {lbm.lb_get_step(a)})")
    a.close()
    b.close()


@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("nx,ny", [(3, 3), (67, 13), (130, 7), (300, 37)])
def test_inplace_ragged_sizes_and_tunings(storage, nx, ny):
    """Tiles narrower than the lattice, wider than it, one row high, taller than
    it: the band pre-pass has to cover every stencil row and halo column."""
    p = wl.params(nx, ny, 1.0, 0.65, "mrt")
    inp = wl.random_fields(p, seed=nx * 100 + ny)
    inp["dphi"] = wl.wall_field(inp["solid"], 0.1)
    say(f"case in place ragged {storage} {nx}x{ny}")
    ref = gpu_lattice(p, inp, storage)
    lbm.lb_step(ref, 61)
    for bx, rows in [(64, 1), (128, 7), (256, 1024), (64, 3), (256, 32), (64, 2), (512, 9),
                     (512, 64), (1024, 32), (1024, 3)]:
        lat = gpu_lattice(p, inp, storage, inplace=1)
        lbm.lb_set_tuning(lat, bx, rows)
        lbm.lb_step(lat, 61)
        assert_same(ref, lat, f"tile {bx}x{rows}")
        lat.close()
    ref.close()


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_inplace_scattered_solids(storage):
    p = wl.params(48, 40, 1.0, 0.6, "mrt")
    inp = wl.random_fields(p, seed=5)
    rng = np.random.default_rng(6)
    solid = inp["solid"].copy()
    solid[rng.integers(2, 38, 60), rng.integers(0, 48, 60)] = 1
    solid[10, 5] = 1
    solid[11, 6] = 1
    fluid = solid == 0
    inp = {k: (np.where(fluid, v, 0.0) if isinstance(v, np.ndarray) and k != "solid" else v)
           for k, v in inp.items()}
    inp["solid"] = solid
    inp["dphi"] = np.where(solid != 0, rng.uniform(-0.3, 0.3, solid.shape), 0.0)
    say(f"case in place scattered solids {storage}")
    a, b = pair(p, inp, storage)
    for bx, rows in [(64, 5), (256, 32), (512, 32), (1024, 32)]:
        lbm.lb_set_tuning(a, bx, rows)
        lbm.lb_set_tuning(b, bx, rows)
        lbm.lb_step(a, 151)
        lbm.lb_step(b, 151)
        assert_same(a, b, f"tile {bx}x{rows}")
    a.close()
    b.close()
    if storage == "f64":
        run_pair(p, inp, 300, what="scattered solids in place", inplace=1)


@pytest.mark.parametrize("at", [33, 34])
def test_inplace_checkpoint_in_either_phase(at):
    """A checkpoint restores the layout of the phase it was taken in."""
    p, inp = random_case("mrt", 1.0, seed=31)
    say(f"case in place checkpoint at step {at}")
    a = gpu_lattice(p, inp, "f32", inplace=1)
    lbm.lb_step(a, at)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "state.ckpt")
        lbm.lb_save(a, path)
        lbm.lb_step(a, 10)
        b = gpu_lattice(p, inp, "f32", inplace=1)
        lbm.lb_load(b, path)
        assert lbm.lb_get_step(b) == at
        lbm.lb_step(b, 10)
        assert_same(a, b, f"restored at step {at}, then 10 steps")
        b.close()
    a.close()


def test_inplace_autotune_keeps_state_and_diagnostics_agree():
    p, inp = wl.c2_drop("mrt", analysis.theory_dphi(50.0, 0.04, 0.04))
    say("case in place autotune / diagnostics / contact angle")
    a, b = pair(p, inp, "f32", diag_every=8)
    lbm.lb_step(a, 7)
    lbm.lb_step(b, 7)
    lbm.lb_autotune(b, 2)
    lbm.lb_set_tuning(a, *lbm.lb_get_tuning(b))
    lbm.lb_step(a, 500)
    lbm.lb_step(b, 500)
    assert_same(a, b, "after autotune")
    da, db = lbm.lb_diagnostics(a), lbm.lb_diagnostics(b)
    for k in ("sum_rho", "sum_phi", "kinetic", "max_u", "n_fluid", "step"):
        assert da[k] == db[k], k
    win = (0.0, 256.0, 3.5, 120.0)
    ta = lbm.lb_contact_angle(a, *win, 0.5, 1)
    tb = lbm.lb_contact_angle(b, *win, 0.5, 1)
    assert ta == tb
    assert lbm.lb_fill_length(a, 0, 256, 1.0) == lbm.lb_fill_length(b, 0, 256, 1.0)
    a.close()
    b.close()



def _cross_channels(nx=40, ny=11):
    """Solid everywhere except a one-node-wide row and column (periodic): every
    fluid node has exactly two fluid neighbours, or four at the crossing."""
    solid = np.ones((ny, nx), dtype=np.uint8)
    solid[ny // 2, :] = 0
    solid[:, nx // 2] = 0
    return solid


@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("case", ["no walls", "one-node channels"])
def test_inplace_degenerate_geometries(storage, case):
    p = wl.params(40, 11, 1.2, 0.7, "mrt")
    inp = wl.random_fields(p, seed=41, walls=False)
    if case != "no walls":
        solid = _cross_channels()
        inp = {k: (np.where(solid == 0, v, 0.0) if isinstance(v, np.ndarray) and k != "solid"
                   else v) for k, v in inp.items()}
        inp["solid"] = solid
        inp["dphi"] = wl.wall_field(solid, -0.1)
    say(f"case in place {case} {storage}")
    a, b = pair(p, inp, storage)
    for n in (1, 40, 3):
        lbm.lb_step(a, n)
        lbm.lb_step(b, n)
        assert_same(a, b, f"{case} after +{n}")
    a.close()
    b.close()
    if storage == "f64":
        run_pair(p, inp, 100, what=f"{case} in place", inplace=1)
