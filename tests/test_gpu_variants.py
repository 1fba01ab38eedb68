"""The paper's two variants on the HIP path, held to the FP64 oracle: the tau
table of Sec. VI (lb_params.tau_lut) and lattice-node bounce-back (Fig. 9b,
lb_params.bounce = LB_LATTICE_NODE). FP64 at the FP64 tolerance; FP32 at the
reduced-precision gate; results independent of the tile shape; batch members
equal to solo runs."""
import numpy as np
import pytest

from oracle import analysis
from paper_0812_1282_amd import lbm, workloads as wl
from tests.helpers import make_oracle
from tests.test_gpu_parity import D60, compare, gpu_lattice, run_pair, say

pytestmark = pytest.mark.gpu

LN = lbm.LATTICE_NODE


def random_case(collision, seed=11, nx=70, ny=30, **over):
    p = dict(wl.params(nx, ny, 1.3, 0.6, collision, Gamma=0.3, tau_phi=0.8), **over)
    inp = wl.random_fields(p, seed=seed)
    rng = np.random.default_rng(seed + 1)
    inp["dphi"] = np.where(inp["solid"] != 0, rng.uniform(-0.3, 0.3, inp["solid"].shape), 0.0)
    return p, inp


@pytest.mark.parametrize("n", [10000, 3])
@pytest.mark.parametrize("collision", ["bgk", "mrt"])
def test_tau_table_random_fields(n, collision):
    p, inp = random_case(collision, tau_lut=n)
    run_pair(p, inp, 200, what=f"tau table n={n} {collision}")


def test_tau_table_c2_drop_viscosity_ratio():
    p, inp = wl.c2_drop("mrt", analysis.theory_dphi(60.0, 0.04, 0.04), seed=201)
    p = dict(p, tau_lut=10000)
    run_pair(p, inp, 1000, what="C2 256x128 mrt 60deg tau table")


@pytest.mark.parametrize("storage", ["f32", "f16s"])
def test_tau_table_reduced_precision(storage):
    dphi = analysis.theory_dphi(60.0, 0.04, 0.04)
    p, inp = wl.c5_member(dict(nx=128, ny=64, tau_beta=0.55, seed=777), dphi)
    p = dict(p, tau_lut=10000)
    say(f"case tau table {storage}")
    lat = gpu_lattice(p, inp, storage)
    lbm.lb_step(lat, 3000)
    orc = make_oracle(p, inp)
    orc.step(3000)
    fluid = inp["solid"] == 0
    d = np.abs(lbm.lb_read_fields(lat)[0] - orc.fields()[0])[fluid].max()
    say(f"  max|dphi| {d:.2e}")
    assert d <= 1e-3
    lat.close()


def test_lattice_node_c1_drop():
    p, inp = wl.c1_drop(seed=1, dphi_wall=D60)
    run_pair(dict(p, bounce=LN), inp, 1000, what="C1 100x50 BGK lattice-node")


@pytest.mark.parametrize("collision,zf,zg", [("bgk", 0, 0), ("mrt", 1, 0), ("mrt", 1, 1),
                                             ("mrt", 0, 0)])
def test_lattice_node_every_term(collision, zf, zg):
    p, inp = random_case(collision, bounce=LN)
    run_pair(p, inp, 201, what=f"random {collision} lattice-node step2={zf}/{zg}",
             zero_u_feq=zf, zero_u_geq=zg)


def test_lattice_node_with_tau_table_and_viscosity_ratio():
    p, inp = wl.c2_drop("mrt", analysis.theory_dphi(120.0, 0.04, 0.04), seed=201)
    run_pair(dict(p, bounce=LN, tau_lut=10000), inp, 1000,
             what="C2 256x128 mrt 120deg lattice-node + table")


def test_lattice_node_scattered_solids():
    p = dict(wl.params(48, 40, 1.0, 0.6, "mrt"), bounce=LN)
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
    run_pair(p, inp, 300, what="scattered solids lattice-node")


@pytest.mark.parametrize("nx,ny", [(3, 5), (67, 13), (130, 7)])
def test_lattice_node_ragged_sizes_and_tunings(nx, ny):
    p = dict(wl.params(nx, ny, 1.0, 0.65, "mrt"), bounce=LN)
    inp = wl.random_fields(p, seed=nx * 100 + ny)
    inp["dphi"] = wl.wall_field(inp["solid"], 0.1)
    say(f"case lattice-node ragged {nx}x{ny}")
    orc = make_oracle(p, inp)
    orc.step(60)
    ref = None
    for bx, rows in [(64, 1), (128, 7), (256, 1024), (64, 3), (512, 9), (1024, 4)]:
        lat = gpu_lattice(p, inp, "f64")
        lbm.lb_set_tuning(lat, bx, rows)
        lbm.lb_step(lat, 60)
        f, g = lbm.lb_read_populations(lat)
        if ref is None:
            ref = (f, g)
            compare(lat, orc, inp["solid"], what=f"lattice-node {nx}x{ny} tile {bx}x{rows}")
        else:
            assert np.array_equal(f, ref[0]) and np.array_equal(g, ref[1]), (bx, rows)
        lat.close()


def test_lattice_node_f32_gate():
    dphi = analysis.theory_dphi(60.0, 0.04, 0.04)
    p, inp = wl.c5_member(dict(nx=128, ny=64, tau_beta=0.55, seed=777), dphi)
    p = dict(p, bounce=LN)
    say("case lattice-node f32")
    lat = gpu_lattice(p, inp, "f32")
    lbm.lb_step(lat, 3000)
    orc = make_oracle(p, inp)
    orc.step(3000)
    fluid = inp["solid"] == 0
    d = np.abs(lbm.lb_read_fields(lat)[0] - orc.fields()[0])[fluid].max()
    say(f"  max|dphi| {d:.2e}")
    assert d <= 1e-3
    lat.close()


def test_variants_in_a_batch_equal_solo_runs():
    descs = [dict(nx=64, ny=32, theta=45.0, tau_beta=0.6, seed=91),
             dict(nx=100, ny=40, theta=120.0, tau_beta=0.55, seed=92)]
    members = []
    for d, over in zip(descs, ({"bounce": LN}, {"tau_lut": 5000})):
        p, inp = wl.c5_member(dict(d), analysis.theory_dphi(d["theta"], 0.04, 0.04))
        members.append((dict(p, **over), inp))
    say("case batch with variants")
    b = lbm.lb_batch_init([lbm.make_params(p, "f32") for p, _ in members],
                          [inp for _, inp in members], tuning=(64, 8))
    lbm.lb_batch_step(b, 150)
    for k, (p, inp) in enumerate(members):
        solo = gpu_lattice(p, inp, "f32")
        lbm.lb_set_tuning(solo, 128, 16)
        lbm.lb_step(solo, 150)
        fb, gb = lbm.lb_batch_read_populations(b, k)
        fs, gs = lbm.lb_read_populations(solo)
        assert np.array_equal(fb, fs) and np.array_equal(gb, gs), k
        solo.close()
    b.close()


def test_lattice_node_without_walls_is_mid_link():
    p = wl.params(48, 20, 1.2, 0.7, "mrt")
    inp = wl.random_fields(p, seed=43, walls=False)
    say("case lattice-node without walls")
    a = gpu_lattice(p, inp, "f64")
    b = gpu_lattice(dict(p, bounce=LN), inp, "f64")
    lbm.lb_step(a, 77)
    lbm.lb_step(b, 77)
    fa, ga = lbm.lb_read_populations(a)
    fb, gb = lbm.lb_read_populations(b)
    assert np.array_equal(fa, fb) and np.array_equal(ga, gb)
    a.close()
    b.close()


def test_lattice_node_one_node_channels():
    """A one-node-wide row and column: every fluid node but the crossing has six
    wall neighbours, so most of its populations travel through wall nodes."""
    p = dict(wl.params(40, 11, 1.2, 0.7, "mrt"), bounce=LN)
    inp = wl.random_fields(p, seed=41, walls=False)
    solid = np.ones((11, 40), dtype=np.uint8)
    solid[5, :] = 0
    solid[:, 20] = 0
    inp = {k: (np.where(solid == 0, v, 0.0) if isinstance(v, np.ndarray) and k != "solid" else v)
           for k, v in inp.items()}
    inp["solid"] = solid
    inp["dphi"] = wl.wall_field(solid, -0.1)
    run_pair(p, inp, 150, what="one-node channels lattice-node")


def test_tau_table_compressed_formats():
    """The table applies to every storage format: F64C against the oracle at the
    FP64 tolerance, F32C at the reduced-precision gate."""
    p, inp = wl.c2_drop("mrt", analysis.theory_dphi(60.0, 0.04, 0.04), seed=201)
    p = dict(p, tau_lut=10000)
    run_pair(p, inp, 500, storage="f64c", what="C2 256x128 mrt tau table f64c")
    say("case tau table f32c")
    lat = gpu_lattice(p, inp, "f32c")
    lbm.lb_step(lat, 2000)
    orc = make_oracle(p, inp)
    orc.step(2000)
    fluid = inp["solid"] == 0
    d = np.abs(lbm.lb_read_fields(lat)[0] - orc.fields()[0])[fluid].max()
    say(f"  max|dphi| {d:.2e}")
    assert d <= 1e-3
    lat.close()


@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("collision", ["bgk", "mrt"])
@pytest.mark.parametrize("bounce", [lbm.MIDLINK, LN])
def test_channel_mode_decay_between_walls_on_gpu(storage, collision, bounce):
    """On the GPU alone: the lowest shear mode between two no-slip walls of
    either bounce-back kind decays at nu (pi/H)^2, H the number of fluid rows
    (the wall plane halfway between the solid row and the first fluid row)."""
    nx, ny, tau = 8, 34, 0.8
    H = ny - 2
    p = wl.params(nx, ny, tau, tau, collision, bounce=bounce)
    y = np.arange(ny)[:, None] * np.ones((1, nx))
    solid = wl.walls_mask(nx, ny)
    prof = np.sin(np.pi * (y - 0.5) / H)
    inp = {"solid": solid, "dphi": wl.wall_field(solid, 0.0), "phi0": np.ones((ny, nx)),
           "rho0": np.ones((ny, nx)), "ux0": np.where(solid == 0, 1e-2 * prof, 0.0),
           "uy0": np.zeros((ny, nx))}
    say(f"case channel mode {storage} {collision} bounce={bounce}")
    lat = gpu_lattice(p, inp, storage, zero_u_feq=0)
    ts, amps = [], []
    for k in range(20):
        lbm.lb_step(lat, 100)
        ux = lbm.lb_read_fields(lat)[2]
        amps.append((ux[1:-1, 0] * prof[1:-1, 0]).sum() / (prof[1:-1, 0] ** 2).sum())
        ts.append((k + 1) * 100)
    lat.close()
    rate = -np.polyfit(ts[4:], np.log(amps[4:]), 1)[0]
    ratio = rate / ((tau - 0.5) / 3 * (np.pi / H) ** 2)
    say(f"  decay rate / (nu (pi/H)^2) = {ratio:.4f}")
    assert ratio == pytest.approx(1.0, abs=0.01)


@pytest.mark.parametrize("bounce", [lbm.MIDLINK, LN])
def test_wall_film_reaches_the_discrete_wall_equilibrium_on_gpu(bounce):
    """On the GPU alone (FP64): a film of phi = +1 under phi = -1 between a
    60-degree and a 110-degree wall, at rest, settles on the discrete wall
    equilibrium (A phi + B phi^3 - kappa lap phi = mu0 on every fluid row, ghost
    rows phi_1 - d_perp phi; Sec. II), solved by Newton at the same total phi,
    with either bounce-back kind: lattice-node bounce-back only delays what
    meets a wall, so its rest state is mid-link's."""
    nx, ny = 4, 40
    d_lo = analysis.theory_dphi(60.0, 0.04, 0.04)
    d_hi = analysis.theory_dphi(110.0, 0.04, 0.04)
    p = wl.params(nx, ny, 1.0, 1.0, "bgk", Gamma=2.0, bounce=bounce)
    solid = wl.walls_mask(nx, ny)
    y = np.arange(ny)[:, None] * np.ones((1, nx))
    dphi = np.zeros((ny, nx))
    dphi[0], dphi[ny - 1] = d_lo, d_hi
    inp = {"solid": solid, "dphi": dphi,
           "phi0": np.where(solid == 0, np.tanh((14.0 - y) / np.sqrt(2.0)), 0.0),
           "rho0": np.where(solid == 0, 1.0, 0.0), "ux0": np.zeros((ny, nx)),
           "uy0": np.zeros((ny, nx))}
    say(f"case wall film at rest, bounce={bounce}, 80000 steps")
    lat = gpu_lattice(p, inp)
    lbm.lb_step(lat, 80000)
    phi, rho, ux, uy = lbm.lb_read_fields(lat)
    lat.close()
    prof, _ = analysis.wall_film_profile(phi[1:ny - 1, 0], -0.04, 0.04, 0.04, d_lo, d_hi)
    err = np.abs(phi[1:ny - 1] - prof[:, None]).max()
    say(f"  max|phi - Newton| {err:.2e}")
    assert err < 1e-8
    assert np.hypot(ux, uy)[1:ny - 1].max() < 1e-10
