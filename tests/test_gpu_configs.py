"""The workloads checked against the FP64 oracle over their stated records, and
the paper's Fig. 2(b) finding, on the GPU.

C3 (capillary filling, FP32 storage) follows the oracle's filling record at the
oracle size 256 x 32 to 2 x 10^4 steps; the ensemble's members of every size
(FP32, batched) match the oracle after 10^4 steps. The oracle records are
stored by tests/golden/make_oracle_records.py, which runs the oracle only."""
import json
import os
import sys

import numpy as np
import pytest

from oracle import analysis
from paper_0812_1282_amd import lbm, workloads as wl
from tests.helpers import max_u_near_contact

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
KAPPA = A_L = 0.04


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _meniscus_x(phi, x_lo, x_hi, row):
    r = phi[row]
    for x in range(max(x_lo, 0), x_hi - 1):
        if r[x] > 0 >= r[x + 1]:
            return x + r[x] / (r[x] - r[x + 1])
    return None


@pytest.mark.parametrize("ratio", [1, 10])
def test_c3_filling_record_follows_the_oracle(ratio):
    """Sec. VII, the capillary layout at the oracle size (walls on [128, 224),
    h = 30, 60-degree wall, MRT, FP32 storage): every 500 steps to 2 x 10^4 the
    column length l within 0.02 of the oracle's, the meniscus within 0.05 nodes
    and the advancing angle within 0.5 degrees."""
    g = json.load(open(os.path.join(GOLDEN, "c3_oracle_256x32.json")))
    rec = g["records"][str(ratio)]
    nx, ny, x_in, x_out, h = g["nx"], g["ny"], g["x_in"], g["x_out"], g["h"]
    p, inp = wl.c3_capillary(nx, ny, ratio, analysis.theory_dphi(60.0, KAPPA, A_L), seed=3)
    say(f"case C3 capillary 256x32 ratio {ratio} f32, {g['steps']} steps")
    lat = lbm.lb_init(lbm.make_params(p, "f32"), inp["solid"], inp["phi0"], dphi=inp["dphi"],
                      rho0=inp["rho0"], ux0=inp["ux0"], uy0=inp["uy0"])
    worst = dict(l=0.0, xm=0.0, th=0.0)
    n_th = 0
    for step, l_o, xm_o, th_o in rec:
        lbm.lb_step(lat, g["every"])
        l = lbm.lb_fill_length(lat, x_in, x_out, h)
        worst["l"] = max(worst["l"], abs(l - l_o))
        phi = lbm.lb_read_fields(lat)[0]
        xm = _meniscus_x(phi, x_in - 16, x_out, ny // 2)
        assert (xm is None) == (xm_o is None), step
        if xm is not None:
            worst["xm"] = max(worst["xm"], abs(xm - xm_o))
        if th_o is not None:
            th = lbm.lb_contact_angle(lat, xm_o - 24.0, xm_o + 12.0, 3.5, ny - 4.5, 0.5,
                                      1)["theta"]
            worst["th"] = max(worst["th"], abs(th - th_o))
            n_th += 1
    say(f"  worst |dl| {worst['l']:.2e}  |dx_meniscus| {worst['xm']:.2e}  "
        f"|dtheta_a| {worst['th']:.2e} over {len(rec)} records ({n_th} angles); "
        f"final l {l:.3f} (oracle {rec[-1][1]:.3f})")
    assert worst["l"] < 0.02 and worst["xm"] < 0.05 and worst["th"] < 0.5
    assert n_th >= 10
    assert rec[-1][1] > rec[0][1] + 10.0       # it fills
    lat.close()


def test_c5_members_of_every_size_follow_the_oracle():
    """Eight members of the 256-member ensemble (MRT, tau_beta = 0.5 + 0.5 /
    ratio, tau clamp): the first of each size (64 x 32 .. 512 x 256) and each
    size's member with the target angle farthest from 90 degrees (30 to 150
    degrees, one at viscosity ratio 81), FP32 storage in one batch, against the
    FP64 oracle after 10^4 steps: contact angle within 0.5 degrees and max
    |d phi| <= 1e-3 (on every second row and column)."""
    z = np.load(os.path.join(GOLDEN, "c5_oracle_sample.npz"))
    n = len([k for k in z.files if k.startswith("phi")])
    descs = []
    for k in range(n):
        nx, ny, seed, theta, tb = z[f"desc{k}"]
        descs.append(dict(nx=int(nx), ny=int(ny), seed=int(seed), theta=float(theta),
                          tau_beta=float(tb)))
    assert n == 8 and sorted(set(d["nx"] for d in descs)) == [64, 128, 256, 512]
    assert min(d["theta"] for d in descs) < 35.0 and max(d["theta"] for d in descs) > 145.0
    say(f"case C5 sample of {n} members, f32 batched, 10^4 steps")
    members, params = [], []
    for d in descs:
        p, inp = wl.c5_member(d, analysis.theory_dphi(d["theta"], KAPPA, A_L))
        members.append(inp)
        params.append(lbm.make_params(p, "f32"))
    b = lbm.lb_batch_init(params, members)
    lbm.lb_batch_step(b, 10000)
    for k, (d, inp) in enumerate(zip(descs, members)):
        phi = lbm.lb_batch_read_fields(b, k)[0]
        ophi = z[f"phi{k}"]
        fluid = inp["solid"][::2, ::2] == 0
        dphi = np.abs(phi[::2, ::2] - ophi)[fluid].max()
        th = lbm.lb_batch_contact_angle(b, k, 0.0, float(d["nx"]), 3.5, d["ny"] - 4.5, 0.5, 1)
        oth = float(z[f"theta{k}"])
        say(f"  member {d['nx']}x{d['ny']} target {d['theta']:.1f}: theta {th:.3f} "
            f"oracle {oth:.3f}  max|dphi| {dphi:.2e}")
        assert abs(th - oth) <= 0.5
        assert dphi <= 1e-3
    b.close()


def test_c2_mrt_full_length_follows_the_oracle():
    """C2 at its stated length (256 x 128, R = 60, viscosity ratio 10, MRT with
    Step 2, FP64) on the 30- and 150-degree walls, against the stored FP64 oracle
    record after 20,000 steps: phi and u on every second node within 1e-9, the
    contact angle within 1e-6 degree, the peak spurious |u| at the contact points
    (Sec. V) within 1e-6 of its value, and sum rho, sum phi within 1e-10
    relative. Both sides are FP64 with different summation orders; the drop is
    close to rest, so their difference stays near rounding."""
    z = np.load(os.path.join(GOLDEN, "c2_oracle_256x128.npz"))
    win = tuple(float(v) for v in z["window"])
    for k, theta in enumerate(z["thetas"]):
        p, inp = wl.c2_drop("mrt", analysis.theory_dphi(float(theta), KAPPA, A_L), seed=201)
        say(f"case C2 mrt {theta:.0f} degrees, {int(z['steps'])} steps, f64")
        lat = lbm.lb_init(lbm.make_params(p, "f64"), inp["solid"], inp["phi0"],
                          dphi=inp["dphi"], rho0=inp["rho0"], ux0=inp["ux0"], uy0=inp["uy0"])
        lbm.lb_step(lat, int(z["steps"]))
        phi, rho, ux, uy = lbm.lb_read_fields(lat)
        th = lbm.lb_contact_angle(lat, *win, 0.5, 1)["theta"]
        lat.close()
        fluid = inp["solid"] == 0
        sub = fluid[::2, ::2]
        errs = [np.abs(a[::2, ::2] - z[f"{n}{k}"])[sub].max()
                for a, n in ((phi, "phi"), (ux, "ux"), (uy, "uy"))]
        umax = max_u_near_contact(phi, ux, uy, inp["solid"])
        oumax = float(z[f"umax_contact{k}"])
        sums = np.array([rho[fluid].sum(), phi[fluid].sum()])
        osums = z[f"sums{k}"]
        say(f"  theta {th:.6f} (oracle {float(z[f'theta{k}']):.6f}); max|dphi|, |dux|, |duy| "
            f"{errs[0]:.2e} {errs[1]:.2e} {errs[2]:.2e}; peak |u| at contacts {umax:.6e} "
            f"(oracle {oumax:.6e})")
        assert max(errs) < 1e-9
        assert abs(th - float(z[f"theta{k}"])) < 1e-6
        assert abs(umax - oumax) <= 1e-6 * oumax
        assert np.all(np.abs(sums - osums) <= 1e-10 * np.abs(osums))


@pytest.mark.parametrize("storage", ["f32", "f16s"])
def test_c2_reduced_precision_at_the_angle_extremes(storage):
    """The precision gate away from the neutral wall: the C2 drop on the 30- and
    150-degree walls with FP32 or FP16 shifted storage (FP32 arithmetic), after
    20,000 steps against the stored FP64 oracle record: max |d phi| <= 1e-3 on
    every second node and the contact angle within 0.5 degree."""
    z = np.load(os.path.join(GOLDEN, "c2_oracle_256x128.npz"))
    win = tuple(float(v) for v in z["window"])
    for k, theta in enumerate(z["thetas"]):
        p, inp = wl.c2_drop("mrt", analysis.theory_dphi(float(theta), KAPPA, A_L), seed=201)
        say(f"case C2 mrt {theta:.0f} degrees, {int(z['steps'])} steps, {storage}")
        lat = lbm.lb_init(lbm.make_params(p, storage), inp["solid"], inp["phi0"],
                          dphi=inp["dphi"], rho0=inp["rho0"], ux0=inp["ux0"], uy0=inp["uy0"])
        lbm.lb_step(lat, int(z["steps"]))
        phi = lbm.lb_read_fields(lat)[0]
        th = lbm.lb_contact_angle(lat, *win, 0.5, 1)["theta"]
        lat.close()
        sub = (inp["solid"] == 0)[::2, ::2]
        dphi = np.abs(phi[::2, ::2] - z[f"phi{k}"])[sub].max()
        dth = abs(th - float(z[f"theta{k}"]))
        say(f"  max|dphi| {dphi:.2e}  dtheta {dth:.2e} degrees")
        assert dphi <= 1e-3 and dth <= 0.5


def _neutral_angle(ta, tb, coll, steps):
    p, inp = wl.fig2_drop(ta, tb, coll)
    lat = lbm.lb_init(lbm.make_params(p, "f64"), inp["solid"], inp["phi0"], dphi=inp["dphi"],
                      rho0=inp["rho0"], ux0=inp["ux0"], uy0=inp["uy0"])
    lbm.lb_set_tuning(lat, 64, 8)
    lbm.lb_step(lat, steps)
    th = lbm.lb_contact_angle(lat, 0.0, 300.0, 3.5, 95.5, 0.5, 1)["theta"]
    lat.close()
    return th


def test_fig2b_neutral_wall_bgk_off_mrt_on():
    """Fig. 2(b) and Sec. V: the 300 x 100 drop (R = 35, Gamma = 0.5) on a
    neutral wall with tau_alpha = 3, tau_beta = 0.7: BGK settles more than 5
    degrees above 90 (the paper: about 10), MRT with Step 2 within 2 degrees;
    with tau = 1 both are within 1 degree."""
    res = {}
    for ta, tb in ((3.0, 0.7), (1.0, 1.0)):
        for coll in ("bgk", "mrt"):
            say(f"case fig2b neutral wall tau {ta}/{tb} {coll}, 10^5 steps")
            res[(ta, coll)] = _neutral_angle(ta, tb, coll, 100000)
            say(f"  theta = {res[(ta, coll)]:.3f}")
    assert res[(3.0, "bgk")] - 90.0 > 5.0
    assert abs(res[(3.0, "mrt")] - 90.0) < 2.0
    assert abs(res[(1.0, "bgk")] - 90.0) < 1.0 and abs(res[(1.0, "mrt")] - 90.0) < 1.0


def test_unequal_viscosity_at_a_wetting_wall_follows_the_oracle():
    """Sec. VI, Fig. 2(b), on a 60-degree wall: the FP64 GPU path follows the
    stored oracle record of the drop with tau 1/1 (MRT), 3/0.7 (MRT) and 3/0.7
    (BGK) every 10^4 steps to 4 x 10^4 within 0.01 degree, and reproduces the
    finding the record holds: MRT with unequal viscosities within 1.5 degrees
    of the equal-viscosity angle, BGK more than 3 degrees above it."""
    with open(os.path.join(GOLDEN, "wall_viscosity_60.json")) as f:
        rec = json.load(f)
    nx, ny = rec["nx"], rec["ny"]
    dphi = analysis.theory_dphi(rec["theta_target"], KAPPA, A_L)
    got = {}
    for key, ref in rec["records"].items():
        coll, ta, tb = key.split("-")
        p = wl.params(nx, ny, float(ta), float(tb), coll, Gamma=rec["Gamma"])
        inp = wl.drop_on_wall(p, rec["radius"], nx / 2, 0.0, 1, dphi)
        lat = lbm.lb_init(lbm.make_params(p, "f64"), inp["solid"], inp["phi0"], dphi=inp["dphi"],
                          rho0=inp["rho0"], ux0=inp["ux0"], uy0=inp["uy0"])
        say(f"case wall viscosity 60 degrees {key}, {rec['steps']} steps")
        th = []
        for _ in range(rec["steps"] // rec["every"]):
            lbm.lb_step(lat, rec["every"])
            th.append(lbm.lb_contact_angle(lat, *rec["window"], 0.5, 1)["theta"])
        lat.close()
        say(f"  theta {['%.4f' % t for t in th]} oracle {['%.4f' % t for t in ref]}")
        assert np.max(np.abs(np.array(th) - np.array(ref))) < 0.01
        got[key] = th[-1]
    ref11 = got["mrt-1.0-1.0"]
    assert abs(got["mrt-3.0-0.7"] - ref11) < 1.5
    assert got["bgk-3.0-0.7"] - ref11 > 3.0
