"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerance for the FP64 path, after up to 1000 steps: max |GPU - oracle| /
max |oracle| <= 1e-12 for the populations f and g (the state) and for phi and
rho; the velocity, a difference of O(0.1) populations divided by rho ~ 1, has an
absolute rounding floor, so it is held to max |GPU - oracle| <= 1e-12 (lattice
units, c = 1). The two sides differ only in rounding order (fused multiply-adds,
moment-space MRT, pull vs push streaming)."""
import os
import sys

import numpy as np
import pytest

import oracle
from oracle import analysis
from paper_0812_1282_amd import lbm, workloads as wl
from tests.helpers import make_oracle

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
D60 = analysis.theory_dphi(60.0, 0.04, 0.04)


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel(a, b, mask=None):
    if mask is not None:
        a, b = a[..., mask], b[..., mask]
    den = np.abs(b).max()
    return np.abs(a - b).max() / (den if den > 0 else 1.0)


def gpu_lattice(p, inp, storage="f64", **kw):
    return lbm.lb_init(lbm.make_params(p, storage, **kw), inp["solid"], inp["phi0"],
                       dphi=inp["dphi"], rho0=inp["rho0"], ux0=inp["ux0"], uy0=inp["uy0"])


def compare(lat, orc, solid, tol=TOL64, what=""):
    fluid = solid == 0
    f, g = lbm.lb_read_populations(lat)
    of, og = orc.populations()
    fields = lbm.lb_read_fields(lat)
    ofields = orc.fields()
    errs = {"f": rel(f, of, fluid), "g": rel(g, og, fluid)}
    for name, a, b in zip(("phi", "rho"), fields[:2], ofields[:2]):
        errs[name] = rel(a, b, fluid)
    for name, a, b in zip(("ux", "uy"), fields[2:], ofields[2:]):
        errs[name] = np.abs(a - b)[fluid].max()
    say(f"  {what}: " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()))
    for k, v in errs.items():
        assert v <= tol, (what, k, v)
    assert np.all(f[:, ~fluid] == 0) and np.all(g[:, ~fluid] == 0)
    return errs


def run_pair(p, inp, steps, storage="f64", tol=TOL64, what="", **kw):
    say(f"case {what}: {p['nx']}x{p['ny']} {p['collision']} {storage} steps={steps} {kw}")
    lat = gpu_lattice(p, inp, storage, **kw)
    orc = make_oracle(p, inp, **{k: v for k, v in kw.items() if k.startswith("zero_u")})
    lbm.lb_step(lat, steps)
    orc.step(steps)
    errs = compare(lat, orc, inp["solid"], tol, what)
    lat.close()
    return errs


def test_initial_state_is_equilibrium_of_inputs():
    p = wl.params(40, 24, 1.0, 0.7, "mrt")
    inp = wl.random_fields(p, seed=3)
    inp["dphi"] = wl.wall_field(inp["solid"], -0.2)
    run_pair(p, inp, 0, tol=1e-14, what="S_0")


def test_c1_drop_bgk_1000_steps():
    p, inp = wl.c1_drop(seed=1, dphi_wall=D60)
    run_pair(p, inp, 1000, what="C1 100x50 BGK 60deg")


def test_c1_configured_run_2000_steps():
    """The 100 x 50 BGK drop on a 60-degree wall at its configured 2000 steps:
    populations and fields within the FP64 tolerance of the oracle, the outputs
    the run reports (contact angle, sum rho, sum phi) equal to the oracle's, and
    sum rho, sum phi conserved from S_0 to 1e-13 relative (Sec. III)."""
    p, inp = wl.c1_drop(seed=1, dphi_wall=D60)
    say("case C1 100x50 BGK 60deg configured run: 2000 steps")
    lat = gpu_lattice(p, inp)
    orc = make_oracle(p, inp)
    d0 = lbm.lb_diagnostics(lat)
    lbm.lb_step(lat, 2000)
    orc.step(2000)
    compare(lat, orc, inp["solid"], TOL64, "C1 2000 steps")
    win = (0.0, 100.0, 3.5, 45.5)
    th = lbm.lb_contact_angle(lat, *win, 0.5, 1)["theta"]
    oth = analysis.contact_angle(orc.fields()[0], inp["solid"], 0.5, 1, *win)["theta"]
    d = lbm.lb_diagnostics(lat)
    od = orc.diagnostics()
    lat.close()
    say(f"  theta {th:.9f} (oracle {oth:.9f}); sum rho {d['sum_rho']:.15e} "
        f"(oracle {od['sum_rho']:.15e}); sum phi {d['sum_phi']:.12e} (oracle {od['sum_phi']:.12e})")
    assert abs(th - oth) < 1e-8
    for key in ("sum_rho", "sum_phi"):
        assert abs(d[key] - od[key]) <= 1e-12 * abs(od[key])
        assert abs(d[key] - d0[key]) <= 1e-13 * abs(d0[key])


@pytest.mark.parametrize("collision,zf,zg", [("bgk", 0, 0), ("bgk", 1, 0), ("mrt", 1, 0),
                                             ("mrt", 0, 0), ("mrt", 1, 1)])
def test_every_term_random_fields(collision, zf, zg):
    """Random phi, rho and u with walls, unequal tau, tau_phi != 1 and a wall field."""
    p = wl.params(70, 30, 1.3, 0.6, collision, Gamma=0.3, tau_phi=0.8)
    inp = wl.random_fields(p, seed=11)
    rng = np.random.default_rng(12)
    inp["dphi"] = np.where(inp["solid"] != 0, rng.uniform(-0.3, 0.3, inp["solid"].shape), 0.0)
    run_pair(p, inp, 200, what=f"random {collision} step2={zf}/{zg}", zero_u_feq=zf,
             zero_u_geq=zg)


@pytest.mark.parametrize("collision", ["bgk", "mrt"])
@pytest.mark.parametrize("theta", [30.0, 130.0])
def test_c2_viscosity_ratio_10(collision, theta):
    """BGK with tau = 0.55 in the phi = -1 phase is unstable in this model (the
    oracle goes non-finite near step 600, also at uniform tau = 0.55), so BGK is
    compared over the first 300 steps; MRT over 1000."""
    p, inp = wl.c2_drop(collision, analysis.theory_dphi(theta, 0.04, 0.04), seed=201)
    run_pair(p, inp, 1000 if collision == "mrt" else 300,
             what=f"C2 256x128 {collision} {theta}deg")


def test_c2_bgk_instability_reproduced_and_flagged():
    """Both sides blow up on the BGK C2 case; the GPU reports it through the
    periodic check as LB_ENUMERIC."""
    p, inp = wl.c2_drop("bgk", analysis.theory_dphi(30.0, 0.04, 0.04), seed=201)
    say("case C2 bgk instability")
    orc = make_oracle(p, inp)
    orc.step(1000)
    assert not np.isfinite(orc.diagnostics()["kinetic"])
    lat = lbm.lb_init(lbm.make_params(p, "f64", diag_every=100), inp["solid"], inp["phi0"],
                      dphi=inp["dphi"], rho0=inp["rho0"])
    lbm.lb_step(lat, 1000)
    with pytest.raises(lbm.LbError) as e:
        lbm.lb_read_fields(lat)
    assert e.value.code == lbm.LB_ENUMERIC
    lat.close()


def test_capillary_geometry_plate_ends():
    """Walls on part of the lattice only: plate ends (corner ghosts) and solid nodes
    with fluid on one side within a wall-free periodic column."""
    p, inp = wl.c3_capillary(256, 32, 10, D60, seed=3)
    run_pair(p, inp, 500, what="capillary 256x32 mrt")


def test_irregular_solid_mask():
    """Scattered solid nodes: diagonal-only ghosts, bounce-back from all sides."""
    p = wl.params(48, 40, 1.0, 0.6, "mrt")
    inp = wl.random_fields(p, seed=5)
    rng = np.random.default_rng(6)
    solid = inp["solid"].copy()
    solid[rng.integers(2, 38, 60), rng.integers(0, 48, 60)] = 1
    solid[20, 10:14] = 1
    solid[21:24, 30] = 1
    solid[10, 5] = 1
    solid[11, 6] = 1          # diagonal pair: each sees the other only diagonally
    fluid = solid == 0
    inp = {k: (np.where(fluid, v, 0.0) if isinstance(v, np.ndarray) and k != "solid" else v)
           for k, v in inp.items()}
    inp["solid"] = solid
    inp["dphi"] = np.where(solid != 0, rng.uniform(-0.3, 0.3, solid.shape), 0.0)
    run_pair(p, inp, 300, what="scattered solids")


@pytest.mark.parametrize("nx,ny", [(3, 3), (67, 13), (130, 7), (64, 5)])
def test_ragged_sizes_and_tunings(nx, ny):
    """Sizes that are not multiples of the tile, and every tile shape, give the same
    bits, and match the oracle."""
    p = wl.params(nx, ny, 1.0, 0.65, "mrt")
    inp = wl.random_fields(p, seed=nx * 100 + ny)
    inp["dphi"] = wl.wall_field(inp["solid"], 0.1)
    say(f"case ragged {nx}x{ny}")
    orc = make_oracle(p, inp)
    orc.step(60)
    ref = None
    for bx, rows in [(64, 1), (128, 7), (256, 1024), (64, 3), (256, 32), (512, 9), (512, 32),
                     (1024, 5)]:
        lat = gpu_lattice(p, inp, "f64")
        lbm.lb_set_tuning(lat, bx, rows)
        lbm.lb_step(lat, 60)
        f, g = lbm.lb_read_populations(lat)
        if ref is None:
            ref = (f, g)
            compare(lat, orc, inp["solid"], what=f"ragged {nx}x{ny} tile {bx}x{rows}")
        else:
            assert np.array_equal(f, ref[0]) and np.array_equal(g, ref[1]), (bx, rows)
        lat.close()


def test_diagnostics_fields_and_fill_length():
    p, inp = wl.c3_capillary(256, 32, 10, D60, seed=3)
    say("case diagnostics capillary 256x32")
    lat = gpu_lattice(p, inp, "f64")
    orc = make_oracle(p, inp)
    lbm.lb_step(lat, 300)
    orc.step(300)
    d = lbm.lb_diagnostics(lat)
    od = orc.diagnostics()
    assert d["n_fluid"] == od["n_fluid"]
    assert d["step"] == 300
    assert d["sum_rho"] == pytest.approx(od["sum_rho"], rel=1e-13)
    assert d["sum_phi"] == pytest.approx(od["sum_phi"], rel=1e-12, abs=1e-10)
    assert d["kinetic"] == pytest.approx(od["kinetic"], rel=1e-9)
    assert d["max_u"] == pytest.approx(od["max_u"], rel=1e-9)
    phi = orc.fields()[0]
    l_gpu = lbm.lb_fill_length(lat, 128, 224, 30.0)
    l_orc = (0.5 * (1 + phi[:, 128:224]))[inp["solid"][:, 128:224] == 0].sum() / 30.0
    assert l_gpu == pytest.approx(l_orc, rel=1e-12)
    lat.close()


def test_conservation_on_gpu():
    p, inp = wl.c2_drop("mrt", analysis.theory_dphi(50.0, 0.04, 0.04))
    say("case conservation C2 mrt 3000 steps")
    lat = gpu_lattice(p, inp, "f64")
    d0 = lbm.lb_diagnostics(lat)
    lbm.lb_step(lat, 3000)
    d1 = lbm.lb_diagnostics(lat)
    assert abs(d1["sum_rho"] - d0["sum_rho"]) <= 1e-12 * d0["sum_rho"]
    assert abs(d1["sum_phi"] - d0["sum_phi"]) <= 1e-12 * d0["n_fluid"]
    lat.close()


def test_contact_angle_matches_oracle_measurement():
    p, inp = wl.c1_drop(seed=1, dphi_wall=D60)
    say("case contact angle C1 5000 steps")
    lat = gpu_lattice(p, inp, "f64")
    orc = make_oracle(p, inp)
    lbm.lb_step(lat, 5000)
    orc.step(5000)
    win = (0.0, 100.0, 3.5, 47.0)
    ca = lbm.lb_contact_angle(lat, *win, 0.5, 1)
    oca = analysis.contact_angle(orc.fields()[0], inp["solid"], 0.5, 1, *win)
    say(f"  gpu {ca['theta']:.6f} (n={ca['n']}) oracle {oca['theta']:.6f} (n={oca['n']})")
    assert ca["n"] == oca["n"]
    assert ca["theta"] == pytest.approx(oca["theta"], abs=1e-8)
    assert ca["R"] == pytest.approx(oca["R"], rel=1e-9)
    # Eq. (theory) with equal viscosities: 60 degrees (within the lattice error).
    assert abs(ca["theta"] - 60.0) < 3.0
    lat.close()


def test_mrt_at_unit_rates_is_bgk_tau_one():
    """Sec. III.B: with tau = 1 in both phases every non-conserved MRT rate is 1,
    so MRT and BGK both relax f to f^eq in one step, Step 2 off (with Step 2 on
    they differ by design: MRT keeps the momentum of f at boundary nodes, BGK
    takes that of f^eq, which is zero there). A check of the GPU path against
    itself, independent of the oracle: the two operators take different
    arithmetic, so they agree to rounding."""
    p, inp = wl.c1_drop(seed=1, dphi_wall=D60)
    say("case MRT at unit rates vs BGK tau = 1")
    a = gpu_lattice(dict(p, collision="bgk"), inp, "f64", zero_u_feq=0)
    b = gpu_lattice(dict(p, collision="mrt"), inp, "f64", zero_u_feq=0)
    lbm.lb_step(a, 300)
    lbm.lb_step(b, 300)
    fa, ga = lbm.lb_read_populations(a)
    fb, gb = lbm.lb_read_populations(b)
    df = np.abs(fa - fb).max() / np.abs(fa).max()
    dg = np.abs(ga - gb).max() / np.abs(ga).max()
    say(f"  max rel diff f {df:.2e}, g {dg:.2e}")
    assert df <= 1e-13 and dg <= 1e-13
    a.close()
    b.close()


@pytest.mark.parametrize("storage", ["f64", "f32", "f16s"])
@pytest.mark.parametrize("collision", ["bgk", "mrt"])
@pytest.mark.parametrize("phase", [1.0, -1.0, 0.7, -0.7])
def test_shear_wave_viscosity_on_gpu(storage, collision, phase):
    """A shear wave u_x = U sin(k y) in a uniform fluid at phi decays at nu k^2
    with nu = (tau(phi) - 1/2)/3, tau(phi) = tau_beta + (phi + 1)/2 (tau_alpha -
    tau_beta): the bulk phases phi = +1, -1 and mixtures at +-0.7, outside the
    spinodal, which stay uniform (Eqs. (tau), (kine); MRT through its stress
    modes). A check of the GPU path alone, in the headline format too."""
    nx, ny = 8, 48
    ta, tb = 1.3, 0.7
    p = wl.params(nx, ny, ta, tb, collision)
    y = np.arange(ny)[:, None] * np.ones((1, nx))
    inp = {"solid": np.zeros((ny, nx), np.uint8), "dphi": None,
           "phi0": np.full((ny, nx), phase), "rho0": np.ones((ny, nx)),
           "ux0": 1e-2 * np.sin(2 * np.pi * y / ny), "uy0": np.zeros((ny, nx))}
    say(f"case shear wave {storage} {collision} phi={phase}")
    lat = gpu_lattice(p, inp, storage, zero_u_feq=0)
    ts, amps = [], []
    for k in range(20):
        lbm.lb_step(lat, 50)
        ux = lbm.lb_read_fields(lat)[2]
        amps.append((ux[:, 0] * np.sin(2 * np.pi * np.arange(ny) / ny)).sum() * 2 / ny)
        ts.append((k + 1) * 50)
    lat.close()
    rate = -np.polyfit(ts[4:], np.log(amps[4:]), 1)[0]
    nu = (tb + 0.5 * (phase + 1.0) * (ta - tb) - 0.5) / 3
    ratio = rate / (nu * (2 * np.pi / ny) ** 2)
    say(f"  decay rate / (nu k^2) = {ratio:.4f}")
    assert ratio == pytest.approx(1.0, abs=0.02)


@pytest.mark.parametrize("storage", ["f64", "f16s"])
@pytest.mark.parametrize("collision", ["bgk", "mrt"])
@pytest.mark.parametrize("clamp, phase", [(1, 1.2), (1, -1.2), (0, 1.2)])
def test_shear_wave_viscosity_with_tau_clamp_on_gpu(storage, collision, clamp, phase):
    """tau_clamp on the GPU alone: a uniform fluid at phi = +-1.2 has its bulk
    phase's viscosity with the clamp and the linear continuation of Eq. (tau)
    without it, from the decay of a shear wave (Eq. (kine))."""
    nx, ny = 8, 96
    ta, tb = 3.0, 0.7
    p = wl.params(nx, ny, ta, tb, collision, tau_clamp=clamp)
    y = np.arange(ny)[:, None] * np.ones((1, nx))
    inp = {"solid": np.zeros((ny, nx), np.uint8), "dphi": None,
           "phi0": np.full((ny, nx), phase), "rho0": np.ones((ny, nx)),
           "ux0": 1e-2 * np.sin(2 * np.pi * y / ny), "uy0": np.zeros((ny, nx))}
    say(f"case shear wave tau_clamp={clamp} {storage} {collision} phi={phase}")
    lat = gpu_lattice(p, inp, storage, zero_u_feq=0)
    ts, amps = [], []
    for k in range(20):
        lbm.lb_step(lat, 50)
        ux = lbm.lb_read_fields(lat)[2]
        amps.append((ux[:, 0] * np.sin(2 * np.pi * np.arange(ny) / ny)).sum() * 2 / ny)
        ts.append((k + 1) * 50)
    lat.close()
    rate = -np.polyfit(ts[4:], np.log(amps[4:]), 1)[0]
    c = max(-1.0, min(1.0, phase)) if clamp else phase
    nu = (tb + 0.5 * (c + 1.0) * (ta - tb) - 0.5) / 3
    ratio = rate / (nu * (2 * np.pi / ny) ** 2)
    say(f"  decay rate / (nu k^2) = {ratio:.4f}")
    assert ratio == pytest.approx(1.0, abs=0.02)


@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("collision", ["bgk", "mrt"])
def test_stratified_shear_decay_on_gpu(storage, collision):
    """tau(phi) through interfaces on the GPU alone: a periodic stripe with a
    shear flow along its flat interfaces decays as d_y(nu(y) d_y u) predicts,
    nu(y) from the measured phi and Eq. (tau), viscosity ratio 15."""
    from tests.test_oracle_physics import _slowest_excited_rate, stratified_shear_case
    ny, ta, tb = 64, 2.0, 0.6
    p, inp = stratified_shear_case(ny, ta, tb, collision)
    say(f"case stratified shear {storage} {collision}")
    lat = gpu_lattice(p, inp, storage, zero_u_feq=0)
    ts, es = [], []
    for k in range(60):
        lbm.lb_step(lat, 100)
        phi, rho, ux, uy = lbm.lb_read_fields(lat)
        ts.append((k + 1) * 100)
        es.append((rho[:, 0] * ux[:, 0] ** 2).sum())
    lat.close()
    lam = -np.polyfit(ts[30:], np.log(es[30:]), 1)[0] / 2
    lam0 = _slowest_excited_rate(phi[:, 0], ta, tb, np.sin(2 * np.pi * np.arange(ny) / ny))
    say(f"  rate / slowest excited rate of the continuum operator = {lam / lam0:.4f}")
    assert lam / lam0 == pytest.approx(1.0, abs=0.015)


@pytest.mark.parametrize("storage", ["f64", "f16s"])
def test_laplace_pressure_on_gpu(storage):
    """Free drops of radius 8, 12, 16 in a periodic 64 x 64 box: p0 inside minus
    outside against 1/R has the slope of the discrete flat interface's tension
    (Eq. (pressten); Sec. II gives sqrt(8 kappa a / 9) for the continuum),
    from GPU runs alone; the radius is fitted to the phi = 0 crossings."""
    from tests.test_oracle_physics import _discrete_surface_tension
    gam = _discrete_surface_tension()
    pts = []
    for R in (8.0, 12.0, 16.0):
        p = wl.params(64, 64, 1.0, 1.0, "bgk", Gamma=1.0)
        inp = wl.free_drop(p, R, seed=7)
        say(f"case Laplace {storage} R={R}")
        lat = gpu_lattice(p, inp, storage)
        lbm.lb_step(lat, 3000)
        phi, rho, ux, uy = lbm.lb_read_fields(lat)
        lat.close()
        p0 = rho / 3 + p["A"] * phi ** 2 / 2 + 3 * p["B"] * phi ** 4 / 4
        xs, ys = analysis.crossing_points(phi, inp["solid"], 0, 64, 0, 64)[0].T
        _, _, Rf = analysis.fit_circle(np.stack([xs, ys], 1))
        pts.append((1.0 / Rf, p0[32, 32] - p0[0, 0]))
    pts = np.array(pts)
    slope = np.polyfit(pts[:, 0], pts[:, 1], 1)[0]
    say(f"  slope {slope:.5f}, discrete tension {gam:.5f}")
    assert slope == pytest.approx(gam, rel=0.03)


_BGK60 = pytest.mark.xfail(strict=True, reason=(
    "measured 56.6 degrees, converged (the same to 0.1 degree from 3e4 to 2.4e5 "
    "steps, for either fit window): with the wetting ghost rule the wall wets "
    "3.4 degrees more than Eq. (theory) here, 0.4 degree beyond the 3-degree "
    "reading of good agreement; reported, not re-tuned"))


@pytest.mark.parametrize("storage", ["f64", "f16s"])
@pytest.mark.parametrize("collision,theta", [
    pytest.param("bgk", 60.0, marks=_BGK60), ("mrt", 60.0), ("bgk", 90.0), ("mrt", 90.0),
    ("bgk", 120.0), ("mrt", 120.0)])
def test_equilibrium_angle_follows_theory_on_gpu(storage, collision, theta):
    """Fig. 2(a) set-up, equal viscosities (tau = 1), Gamma = 0.5: a semicircle of
    radius 35 on the wall of a 300 x 100 box, 3e4 steps at the wall gradient
    Eq. (theory) gives for theta; the fitted angle (the library's measurement)
    is within 3 degrees of theta, the agreement the paper reports as good.
    The wall gradient comes from the test's own copy of Eq. (theory). Measured
    (FP64 = FP16S to 0.01 degree): BGK 56.6, 89.4, 122.4; MRT 57.1, 89.5,
    122.2."""
    p = wl.params(300, 100, 1.0, 1.0, collision, Gamma=0.5)
    inp = wl.drop_on_wall(p, 35.0, 150.0, 0.0, seed=3,
                          dphi_wall=analysis.theory_dphi(theta, 0.04, 0.04))
    say(f"case equilibrium angle {storage} {collision} {theta}")
    lat = gpu_lattice(p, inp, storage)
    lbm.lb_step(lat, 30000)
    got = lbm.lb_contact_angle(lat, 0.0, 300.0, 3.5, 90.0, 0.5, 1)["theta"]
    lat.close()
    say(f"  theta {got:.2f} (target {theta})")
    assert abs(got - theta) <= 3.0


UNIFORM_TOL = {"f64": 1e-13, "f64c": 1e-13, "f32": 1e-6, "f32c": 1e-6, "f16s": 1e-3, "bf16s": 1e-3}


@pytest.mark.parametrize("storage", list(UNIFORM_TOL))
@pytest.mark.parametrize("collision", ["bgk", "mrt"])
@pytest.mark.parametrize("case", ["uniform flow, periodic", "rest between walls"])
def test_uniform_states_are_fixed_points(storage, collision, case):
    """A uniform state is a fixed point of the method: all gradients vanish, the
    equilibria carry exactly the state's rho, j and phi (Appendix A), streaming
    moves equal values, and at rest bounce-back returns what it receives while
    the wetting ghosts (wall gradient 0) repeat the uniform phi. phi = 0.3 keeps
    mu and the g^eq terms nonzero. A check of the GPU path alone: the fields must
    stay at their initial values to the storage format's rounding (the stored
    values re-encode to themselves after the first step)."""
    nx, ny = 64, 32
    walls = case != "uniform flow, periodic"
    p = wl.params(nx, ny, 1.3, 0.7, collision, tau_phi=1.0 if storage.endswith("c") else 0.8)
    solid = wl.walls_mask(nx, ny) if walls else np.zeros((ny, nx), dtype=np.uint8)
    fluid = solid == 0
    u0 = (0.0, 0.0) if walls else (0.04, -0.03)
    inp = {"solid": solid, "dphi": np.zeros((ny, nx)), "phi0": np.where(fluid, 0.3, 0.0),
           "rho0": np.where(fluid, 1.0, 0.0), "ux0": np.where(fluid, u0[0], 0.0),
           "uy0": np.where(fluid, u0[1], 0.0)}
    say(f"case uniform state {case} {storage} {collision}")
    lat = gpu_lattice(p, inp, storage, zero_u_feq=0)
    lbm.lb_step(lat, 200)
    phi, rho, ux, uy = lbm.lb_read_fields(lat)
    lat.close()
    err = max(np.abs(phi - 0.3)[fluid].max(), np.abs(rho - 1.0)[fluid].max(),
              np.abs(ux - u0[0])[fluid].max(), np.abs(uy - u0[1])[fluid].max())
    say(f"  max deviation {err:.2e}")
    assert err <= UNIFORM_TOL[storage], err


def test_checkpoint_resume_is_bitwise(tmp_path):
    p, inp = wl.c2_drop("mrt", analysis.theory_dphi(110.0, 0.04, 0.04))
    say("case checkpoint")
    a = gpu_lattice(p, inp, "f64")
    lbm.lb_step(a, 401)
    a_f = lbm.lb_read_populations(a)
    lbm.lb_step(a, 399)
    ref = lbm.lb_read_populations(a)
    b = gpu_lattice(p, inp, "f64")
    lbm.lb_step(b, 401)
    path = tmp_path / "state.ckpt"
    lbm.lb_save(b, path)
    b.close()
    c = gpu_lattice(p, inp, "f64")
    lbm.lb_load(c, path)
    assert lbm.lb_get_step(c) == 401
    mid = lbm.lb_read_populations(c)
    assert np.array_equal(mid[0], a_f[0]) and np.array_equal(mid[1], a_f[1])
    lbm.lb_step(c, 399)
    out = lbm.lb_read_populations(c)
    assert np.array_equal(out[0], ref[0]) and np.array_equal(out[1], ref[1])
    a.close()
    c.close()


def test_checkpoint_rejects_other_cases(tmp_path):
    """A checkpoint loads into a handle of the same case whatever its check
    cadence, and is refused by one whose parameters or mask differ."""
    p, inp = wl.c1_drop(seed=1, dphi_wall=D60)
    say("case checkpoint matching")
    a = gpu_lattice(p, inp, "f64")
    lbm.lb_step(a, 7)
    path = tmp_path / "state.ckpt"
    lbm.lb_save(a, path)
    ok = lbm.lb_init(lbm.make_params(p, "f64", diag_every=5), inp["solid"], inp["phi0"],
                     dphi=inp["dphi"], rho0=inp["rho0"])
    lbm.lb_load(ok, path)
    assert lbm.lb_get_step(ok) == 7
    fa, ga = lbm.lb_read_populations(a)
    fb, gb = lbm.lb_read_populations(ok)
    assert np.array_equal(fa, fb) and np.array_equal(ga, gb)
    ok.close()
    other = gpu_lattice(dict(p, tau_beta=0.9), inp, "f64")
    with pytest.raises(lbm.LbError) as e:
        lbm.lb_load(other, path)
    assert e.value.code == lbm.LB_EINVAL
    other.close()
    solid = inp["solid"].copy()
    solid[10, 3] = 1
    moved = dict(inp, solid=solid)
    for k in ("phi0", "rho0"):
        moved[k] = np.where(solid != 0, 0.0, inp[k])
    other = gpu_lattice(p, moved, "f64")
    with pytest.raises(lbm.LbError) as e:
        lbm.lb_load(other, path)
    assert e.value.code == lbm.LB_EINVAL
    other.close()
    a.close()


def test_determinism_graph_and_memory_paths():
    """Two runs are bitwise equal; the captured-graph path (>= 32 steps per call)
    equals single-step calls; library-allocated and torch-allocated memory agree."""
    p, inp = wl.c2_drop("mrt", analysis.theory_dphi(70.0, 0.04, 0.04))
    say("case determinism")
    runs = []
    for mem, chunk in [("torch", 96), ("torch", 96), ("torch", 1), ("library", 96)]:
        lat = lbm.lb_init(lbm.make_params(p, "f64"), inp["solid"], inp["phi0"], dphi=inp["dphi"],
                          rho0=inp["rho0"], device_memory=mem)
        for _ in range(96 // chunk):
            lbm.lb_step(lat, chunk)
        runs.append(lbm.lb_read_populations(lat))
        lat.close()
    for r in runs[1:]:
        assert np.array_equal(r[0], runs[0][0]) and np.array_equal(r[1], runs[0][1])


@pytest.mark.parametrize("inplace", [0, 1])
@pytest.mark.parametrize("every", [8, 48, 100])
def test_graph_windows_with_periodic_checks(every, inplace):
    """With a check every 8 steps the 32-step graph carries four checks; with 48
    or 100 a window replays the graph with one check at its start or the one
    with none, and steps near a check are launched singly. All of it equals
    single-step calls, and the diagnostics agree."""
    p, inp = wl.c2_drop("mrt", analysis.theory_dphi(70.0, 0.04, 0.04))
    say(f"case graph windows, check every {every}, inplace {inplace}")
    out = []
    for chunks in ([3, 300, 1, 97], [1] * 401):
        params = lbm.make_params(p, "f64", diag_every=every, inplace=inplace)
        lat = lbm.lb_init(params, inp["solid"], inp["phi0"], dphi=inp["dphi"], rho0=inp["rho0"])
        for c in chunks:
            lbm.lb_step(lat, c)
        out.append((lbm.lb_read_populations(lat), lbm.lb_diagnostics(lat)))
        lat.close()
    (a, da), (b, db) = out
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert da == db


@pytest.mark.parametrize("every", [10, 100])
def test_periodic_check_reports_nonfinite_state(every):
    """diag_every > 0 enqueues the conservation sums; a run driven unstable (tau
    close to 1/2 and a large velocity) is reported as LB_ENUMERIC, also when the
    checks sit inside replayed 32-step graphs (every = 100)."""
    p = wl.params(64, 16, 0.5001, 0.5001, "bgk")
    inp = wl.random_fields(p, seed=2, amp_u=0.4)
    say(f"case unstable run with periodic check every {every}")
    lat = lbm.lb_init(lbm.make_params(p, "f64", diag_every=every), inp["solid"], inp["phi0"],
                      dphi=inp["dphi"], rho0=inp["rho0"], ux0=inp["ux0"], uy0=inp["uy0"])
    lbm.lb_step(lat, 2000)
    with pytest.raises(lbm.LbError) as e:
        lbm.lb_read_fields(lat)
    assert e.value.code == lbm.LB_ENUMERIC
    lat.close()
    # A stable run with the same check enabled stays clean.
    p = wl.params(64, 16, 1.0, 1.0, "bgk")
    inp = wl.random_fields(p, seed=2)
    lat = lbm.lb_init(lbm.make_params(p, "f64", diag_every=10), inp["solid"], inp["phi0"])
    lbm.lb_step(lat, 200)
    lbm.lb_read_fields(lat)
    assert lbm.lb_diagnostics(lat)["rc"] == 0
    lat.close()


def test_set_wall_dphi_matches_oracle():
    p, inp = wl.c1_drop(seed=1, dphi_wall=0.0)
    say("case wall gradient update")
    lat = gpu_lattice(p, inp, "f64")
    orc = make_oracle(p, inp)
    lbm.lb_step(lat, 100)
    orc.step(100)
    new = wl.wall_field(inp["solid"], D60)
    lbm.lb_set_wall_dphi(lat, new)
    orc.set_wall_dphi(new)
    lbm.lb_step(lat, 200)
    orc.step(200)
    compare(lat, orc, inp["solid"], what="after wall update")
    lat.close()
