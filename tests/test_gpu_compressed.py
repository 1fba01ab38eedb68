"""The compressed-g formats (tau_phi = 1): a node stores (phi, Gamma mu, u of
g^eq) instead of g_0..g_8, and a receiving node forms g^eq_i of its neighbour.

The dynamics are the method's. LB_F64C is held to the FP64 oracle at the FP64
tolerance after at least one step, populations included: after the first
collision every g is an equilibrium, so the pulled g of S_n (n >= 1) is
defined the same way on both sides. The g populations of S_0 are represented
only by their sum phi_0; that difference is checked here. LB_F32C is held to
the reduced-precision gate against the oracle, and batch members are
bit-identical to solo runs."""
import numpy as np
import pytest

from oracle import analysis
from paper_0812_1282_amd import lbm, workloads as wl
from tests.helpers import make_oracle
from tests.test_gpu_parity import D60, TOL64, compare, gpu_lattice, run_pair, say

pytestmark = pytest.mark.gpu


def _random_case(collision, seed=11):
    p = wl.params(70, 30, 1.3, 0.6, collision, Gamma=0.3)
    inp = wl.random_fields(p, seed=seed)
    rng = np.random.default_rng(seed + 1)
    inp["dphi"] = np.where(inp["solid"] != 0, rng.uniform(-0.3, 0.3, inp["solid"].shape), 0.0)
    return p, inp


def test_f64c_c1_drop_1000_steps():
    p, inp = wl.c1_drop(seed=1, dphi_wall=D60)
    run_pair(p, inp, 1000, storage="f64c", what="C1 100x50 BGK f64c")


@pytest.mark.parametrize("collision,zf,zg", [("bgk", 0, 0), ("mrt", 1, 0), ("mrt", 1, 1),
                                             ("bgk", 1, 1)])
def test_f64c_every_term_random_fields(collision, zf, zg):
    p, inp = _random_case(collision)
    run_pair(p, inp, 200, storage="f64c", what=f"random {collision} f64c step2={zf}/{zg}",
             zero_u_feq=zf, zero_u_geq=zg)


def test_f64c_viscosity_ratio_and_capillary():
    p, inp = wl.c2_drop("mrt", analysis.theory_dphi(130.0, 0.04, 0.04), seed=201)
    run_pair(p, inp, 1000, storage="f64c", what="C2 256x128 mrt 130deg f64c")
    p, inp = wl.c3_capillary(256, 32, 10, D60, seed=3)
    run_pair(p, inp, 500, storage="f64c", what="capillary 256x32 f64c")


def test_f64c_irregular_solid_mask():
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
    run_pair(p, inp, 300, storage="f64c", what="scattered solids f64c")


@pytest.mark.parametrize("nx,ny", [(3, 3), (67, 13), (130, 7)])
def test_f64c_ragged_sizes_and_tunings(nx, ny):
    p = wl.params(nx, ny, 1.0, 0.65, "mrt")
    inp = wl.random_fields(p, seed=nx * 100 + ny)
    inp["dphi"] = wl.wall_field(inp["solid"], 0.1)
    say(f"case ragged f64c {nx}x{ny}")
    orc = make_oracle(p, inp)
    orc.step(60)
    ref = None
    for bx, rows in [(64, 1), (128, 7), (256, 1024), (64, 3), (256, 32), (512, 9), (512, 32)]:
        lat = gpu_lattice(p, inp, "f64c")
        lbm.lb_set_tuning(lat, bx, rows)
        lbm.lb_step(lat, 60)
        f, g = lbm.lb_read_populations(lat)
        if ref is None:
            ref = (f, g)
            compare(lat, orc, inp["solid"], what=f"ragged f64c {nx}x{ny} tile {bx}x{rows}")
        else:
            assert np.array_equal(f, ref[0]) and np.array_equal(g, ref[1]), (bx, rows)
        lat.close()


@pytest.mark.parametrize("storage", ["f64c", "f32c"])
def test_compressed_initial_state(storage):
    """S_0: f and every moment as in the oracle; g represented by its sum."""
    p = wl.params(40, 24, 1.0, 0.7, "mrt")
    inp = wl.random_fields(p, seed=3)
    say(f"case S_0 {storage}")
    lat = gpu_lattice(p, inp, storage)
    orc = make_oracle(p, inp)
    fluid = inp["solid"] == 0
    f, g = lbm.lb_read_populations(lat)
    of, og = orc.populations()
    tol = 1e-14 if storage == "f64c" else 1e-6
    assert np.abs(f - of)[:, fluid].max() <= tol
    phi = lbm.lb_read_fields(lat)[0]
    assert np.abs(phi - orc.fields()[0])[fluid].max() <= tol
    assert np.abs(g[0] - og.sum(axis=0))[fluid].max() <= tol
    assert np.all(g[1:] == 0)
    lat.close()


@pytest.mark.parametrize("storage,tol", [("f64c", 1e-12), ("f32c", 1e-5)])
def test_compressed_conserves_mass_and_phi(storage, tol):
    p, inp = wl.c2_drop("mrt", analysis.theory_dphi(50.0, 0.04, 0.04))
    say(f"case conservation {storage}")
    lat = gpu_lattice(p, inp, storage)
    d0 = lbm.lb_diagnostics(lat)
    lbm.lb_step(lat, 3000)
    d1 = lbm.lb_diagnostics(lat)
    n = d0["n_fluid"]
    say(f"  d sum rho {d1['sum_rho'] - d0['sum_rho']:.3e}  d sum phi "
        f"{d1['sum_phi'] - d0['sum_phi']:.3e} over {n} nodes")
    assert abs(d1["sum_rho"] - d0["sum_rho"]) <= tol * n
    assert abs(d1["sum_phi"] - d0["sum_phi"]) <= tol * n
    lat.close()


def test_f32c_against_fp64_oracle():
    """The reduced-precision gate: 128 x 64 MRT drop, viscosity ratio 10, 60 degree
    wall, 10^4 steps: max |d phi| <= 1e-3, contact angle within 0.5 degrees."""
    dphi = analysis.theory_dphi(60.0, 0.04, 0.04)
    p, inp = wl.c5_member(dict(nx=128, ny=64, tau_beta=0.55, seed=777), dphi)
    say("case precision f32c")
    lat = gpu_lattice(p, inp, "f32c")
    lbm.lb_step(lat, 10000)
    phi = lbm.lb_read_fields(lat)[0]
    orc = make_oracle(p, inp)
    orc.step(10000)
    ophi = orc.fields()[0]
    fluid = inp["solid"] == 0
    dphi_max = np.abs(phi - ophi)[fluid].max()
    win = (0.0, 128.0, 3.5, 60.0)
    th = lbm.lb_contact_angle(lat, *win, 0.5, 1)["theta"]
    oth = analysis.contact_angle(ophi, inp["solid"], 0.5, 1, *win)["theta"]
    say(f"  f32c: max|dphi| {dphi_max:.3e} theta {th:.4f} oracle {oth:.4f}")
    assert dphi_max <= 1e-3
    assert abs(th - oth) <= 0.5
    lat.close()


def test_f32c_batch_members_equal_solo_runs():
    descs = [dict(nx=64, ny=32, theta=45.0, tau_beta=0.6, seed=91),
             dict(nx=100, ny=40, theta=120.0, tau_beta=0.55, seed=92),
             dict(nx=67, ny=13, theta=70.0, tau_beta=0.7, seed=94)]
    members = [wl.c5_member(dict(d), analysis.theory_dphi(d["theta"], 0.04, 0.04))
               for d in descs]
    say("case batch f32c")
    b = lbm.lb_batch_init([lbm.make_params(p, "f32c") for p, _ in members],
                          [inp for _, inp in members], tuning=(64, 8))
    lbm.lb_batch_step(b, 150)
    for k, (p, inp) in enumerate(members):
        solo = gpu_lattice(p, inp, "f32c")
        lbm.lb_set_tuning(solo, 128, 16)
        lbm.lb_step(solo, 150)
        fb, gb = lbm.lb_batch_read_populations(b, k)
        fs, gs = lbm.lb_read_populations(solo)
        assert np.array_equal(fb, fs) and np.array_equal(gb, gs), k
        solo.close()
    b.close()
