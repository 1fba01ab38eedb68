"""Parity at the full 4096 x 2048 size of the large-drop workload, in the tile
shape the benchmark times.

After k steps the state at a node depends only on the initial fields within a
bounded distance (streaming reaches 1 node per step, the phi stencil and its
wall ghosts 2 more), so the oracle can compute sampled outputs exactly on small
windows cut from the same initial fields: inside a margin of 3k + 4 nodes from a
window's edges the window run equals the full-lattice run. Where a window is cut
next to a wall, one extra solid row closes it so that the real wall row sees
the same solid neighbours as in the full lattice."""
import sys

import numpy as np
import pytest

from paper_0812_1282_amd import lbm, workloads as wl
from tests.helpers import make_oracle

pytestmark = pytest.mark.gpu

K = 10
MARGIN = 3 * K + 4
W = 112
TILES = {"f64": (512, 32), "f64c": (256, 16)}   # the shapes bench.py times


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _window(inp, x0, y0, nx, ny, close_top=False, close_bottom=False):
    """Cut [x0, x0+W) x [y0, y0+W) (x periodic). close_*: replace the edge row with
    solid so the window's periodic seam does not put fluid next to a wall."""
    xs = (np.arange(x0, x0 + W)) % nx
    ys = np.arange(y0, y0 + W)
    sub = {k: (None if v is None else v[np.ix_(ys, xs)].copy()) for k, v in inp.items()}
    if close_top:
        sub["solid"][-1, :] = 1
    if close_bottom:
        sub["solid"][0, :] = 1
    for k in ("phi0", "rho0", "ux0", "uy0"):
        sub[k][sub["solid"] != 0] = 0.0
    return sub


@pytest.mark.parametrize("storage", ["f64", "f64c"])
def test_full_size_sampled_windows(storage):
    p, inp = wl.c4_drop()
    nx, ny = p["nx"], p["ny"]
    say(f"case full size {nx}x{ny} {storage}, {K} steps, bench tiles")
    lat = lbm.lb_init(lbm.make_params(p, storage), inp["solid"], inp["phi0"], dphi=inp["dphi"],
                      rho0=inp["rho0"])
    lbm.lb_set_tuning(lat, *TILES[storage])
    bx, rows = lbm.lb_get_tuning(lat)
    say(f"  tiles {bx}x{rows}")
    d0 = lbm.lb_diagnostics(lat)
    lbm.lb_step(lat, K)
    d1 = lbm.lb_diagnostics(lat)
    assert abs(d1["sum_rho"] - d0["sum_rho"]) <= 1e-13 * d0["sum_rho"]
    assert abs(d1["sum_phi"] - d0["sum_phi"]) <= 1e-12 * d0["n_fluid"]
    fields = lbm.lb_read_fields(lat)
    lat.close()
    compare_windows(p, inp, fields, 1e-12)


def compare_windows(p, inp, fields, tol):
    """Every field of the full-lattice run against the oracle on four windows
    (contact line, drop apex, periodic seam, top wall): phi and rho relative to
    their scale, u absolutely (lattice units; u is a difference of O(0.1)
    populations). Returns the largest error of each field."""
    nx, ny = p["nx"], p["ny"]
    worst = {}
    cases = [
        ("contact line, bottom wall", nx // 2 + 800 - W // 2, 0, False, True),
        ("drop apex", nx // 2 - W // 2, 800 - W // 2, False, False),
        ("periodic seam", nx - W // 2, 1000, False, False),
        ("top wall", 100, ny - W + 1, True, False),
    ]
    for name, x0, y0, top, bottom in cases:
        if top:          # the window's first row stands for the solid row below
            sub = _window(inp, x0, y0 - 1, nx, ny, close_bottom=True)
            y_lo = y0 - 1
        else:
            sub = _window(inp, x0, y0, nx, ny, close_top=bottom)
            y_lo = y0
        wp = dict(p)
        wp["nx"], wp["ny"] = W, W
        orc = make_oracle(wp, sub)
        orc.step(K)
        ofields = orc.fields()
        # rows/cols that are exact: away from cut edges (walls are real edges)
        r0 = 0 if bottom else MARGIN
        r1 = W if top else W - MARGIN
        c0, c1 = MARGIN, W - MARGIN
        xs = np.arange(x0 + c0, x0 + c1) % nx
        ys = np.arange(y_lo + r0, y_lo + r1)
        for fname, g, o in zip(("phi", "rho", "ux", "uy"), fields, ofields):
            gw = g[np.ix_(ys, xs)]
            ow = o[r0:r1, c0:c1]
            scale = max(np.abs(ow).max(), 1e-300) if fname in ("phi", "rho") else 1.0
            err = np.abs(gw - ow).max() / scale
            worst[fname] = max(worst.get(fname, 0.0), err)
            say(f"  {name}: {fname} err {err:.2e} (max |value| {np.abs(ow).max():.2e})")
            assert err <= tol, (name, fname, err)
    return worst


# Reduced-precision formats at the tiles the benchmark times. Each stored
# population (or stored phi, Gamma mu, u of the compressed-g formats) carries a
# relative rounding error of at most 2^-24 (FP32), 2^-11 (FP16) or 2^-8 (BF16);
# a node's phi, rho and u sum nine such values, and over 10 steps the
# collision relaxes rather than amplifies them. The bounds: 1e-5 for FP32
# storage, 1e-3 for FP16 (the benchmark's accuracy gate on phi) and 1e-2 for
# BF16.
REDUCED = [("f32", (512, 32), 1e-5), ("f32c", (512, 32), 1e-5), ("f16s", (1024, 32), 1e-3),
           ("bf16s", (512, 32), 1e-2)]


@pytest.mark.parametrize("storage,tiles,tol", REDUCED)
def test_full_size_reduced_formats_sampled_windows(storage, tiles, tol):
    p, inp = wl.c4_drop()
    say(f"case full size {p['nx']}x{p['ny']} {storage}, {K} steps, tiles {tiles}")
    lat = lbm.lb_init(lbm.make_params(p, storage), inp["solid"], inp["phi0"], dphi=inp["dphi"],
                      rho0=inp["rho0"])
    lbm.lb_set_tuning(lat, *tiles)
    lbm.lb_step(lat, K)
    fields = lbm.lb_read_fields(lat)
    lat.close()
    worst = compare_windows(p, inp, fields, tol)
    say(f"  worst {storage}: " + ", ".join(f"{k} {v:.2e}" for k, v in worst.items()))


@pytest.mark.parametrize("storage,tiles", [("f64", (1024, 32)), ("f32", (1024, 32))])
def test_full_size_in_place_equals_two_buffers(storage, tiles):
    """The in-place update at full size and at the tiles the benchmark times for
    it: bit-identical to the two-buffer path after an odd and an even number of
    steps (both layouts), the 32-step graphs included."""
    p, inp = wl.c4_drop()
    say(f"case full size in place {storage}, tiles {tiles}")
    lats = []
    for inplace in (0, 1):
        lat = lbm.lb_init(lbm.make_params(p, storage, inplace=inplace), inp["solid"],
                          inp["phi0"], dphi=inp["dphi"], rho0=inp["rho0"])
        lbm.lb_set_tuning(lat, *tiles)
        lats.append(lat)
    for n in (33, 32):
        for lat in lats:
            lbm.lb_step(lat, n)
        a, b = (lbm.lb_read_fields(lat) for lat in lats)
        for x, y, name in zip(a, b, ("phi", "rho", "ux", "uy")):
            assert np.array_equal(x, y), (n, name)
        say(f"  step {lbm.lb_get_step(lats[0])}: fields identical")
    fa, ga = lbm.lb_read_populations(lats[0])
    fb, gb = lbm.lb_read_populations(lats[1])
    assert np.array_equal(fa, fb) and np.array_equal(ga, gb)
    for lat in lats:
        lat.close()


# The widest lattice the library accepts: a row block of the FP64 layout (18
# planes of the padded width, 8 bytes each) must stay under 2^31 bytes, so that
# every in-row byte offset fits the 32-bit offsets of the buffer accesses.
NX_MAX = ((1 << 31) - 1) // (18 * 8) // 64 * 64


def _widest_case(ny=6):
    """NX_MAX x ny, walls in the first and last rows, phi varying on scales of
    13-40 nodes along x (so the x pulls and the stencil carry real differences
    all along the row), a small density and velocity pattern."""
    nx = NX_MAX
    p = wl.params(nx, ny, 1.2, 0.8, "mrt")
    x = np.arange(nx, dtype=np.float64)
    y = np.arange(ny, dtype=np.float64)[:, None]
    solid = np.zeros((ny, nx), dtype=np.uint8)
    solid[0, :] = 1
    solid[ny - 1, :] = 1
    fluid = solid == 0
    phi0 = np.tanh(1.5 * (np.sin(2 * np.pi * x / 40 + 0.7 * y) + 0.3 * np.sin(2 * np.pi * x / 13)))
    phi0 = np.where(fluid, phi0, 0.0)
    rho0 = np.where(fluid, 1.0 + 0.01 * np.sin(2 * np.pi * x / 29), 0.0)
    ux0 = np.where(fluid, 0.01 * np.cos(2 * np.pi * x / 31), 0.0)
    uy0 = np.zeros((ny, nx))
    dphi = np.where(solid != 0, 0.05, 0.0)
    return p, {"solid": solid, "dphi": dphi, "phi0": phi0, "rho0": rho0, "ux0": ux0, "uy0": uy0}


@pytest.mark.parametrize("storage,inplace,tiles,tol", [("f64", 0, (512, 32), 1e-12),
                                                       ("f64", 1, (1024, 32), 1e-12),
                                                       ("f16s", 0, (1024, 32), 1e-3)])
def test_widest_lattice_against_oracle(storage, inplace, tiles, tol):
    """At the largest accepted width (the last tile ragged at 1024 columns),
    windows at the row start (across the periodic seam), the middle and the row
    end, whole in y, against the oracle."""
    p, inp = _widest_case()
    nx, ny = p["nx"], p["ny"]
    say(f"case widest lattice {nx}x{ny} {storage} inplace={inplace} tiles {tiles}")
    lat = lbm.lb_init(lbm.make_params(p, storage, inplace=inplace), inp["solid"], inp["phi0"],
                      dphi=inp["dphi"], rho0=inp["rho0"], ux0=inp["ux0"], uy0=inp["uy0"])
    lbm.lb_set_tuning(lat, *tiles)
    lbm.lb_step(lat, K)
    fields = lbm.lb_read_fields(lat)
    lat.close()
    say("  GPU run done")
    for x0 in (nx - W // 2, nx // 2, nx - W):
        xs = np.arange(x0, x0 + W) % nx
        sub = {k: v[:, xs].copy() for k, v in inp.items()}
        wp = dict(p, nx=W)
        orc = make_oracle(wp, sub)
        orc.step(K)
        for fname, g, o in zip(("phi", "rho", "ux", "uy"), fields, orc.fields()):
            gw = g[:, xs[MARGIN:W - MARGIN]]
            ow = o[:, MARGIN:W - MARGIN]
            scale = max(np.abs(ow).max(), 1e-300) if fname in ("phi", "rho") else 1.0
            err = np.abs(gw - ow).max() / scale
            say(f"  window at x = {x0}: {fname} err {err:.2e}")
            assert err <= tol, (x0, fname, err)


def test_tallest_lattice_in_place_where_two_buffers_do_not_fit():
    """3 x 2^24 (the most rows the library accepts), FP64: the two-buffer layout
    needs more than the device holds; the in-place update fits and matches the
    oracle on windows at the bottom (across the periodic seam in y), the middle
    and the top."""
    import torch
    nx, ny = 3, 1 << 24
    p = wl.params(nx, ny, 1.2, 0.8, "mrt")
    need_ab = lbm.lb_workspace_bytes(lbm.make_params(p, "f64"))
    need_ip = lbm.lb_workspace_bytes(lbm.make_params(p, "f64", inplace=1))
    torch.cuda.empty_cache()
    free, total = torch.cuda.mem_get_info()
    say(f"case tallest lattice {nx}x{ny}: two buffers {need_ab / 2**30:.0f} GiB, in place "
        f"{need_ip / 2**30:.0f} GiB, device {total / 2**30:.0f} GiB ({free / 2**30:.0f} free)")
    assert need_ab > total
    if need_ip > free:
        pytest.skip("not enough free device memory for the in-place layout")
    y = np.arange(ny, dtype=np.float64)[:, None]
    x = np.arange(nx, dtype=np.float64)[None, :]
    phi0 = np.tanh(1.5 * (np.sin(2 * np.pi * y / 40 + 0.9 * x) + 0.3 * np.sin(2 * np.pi * y / 13)))
    inp = {"solid": np.zeros((ny, nx), dtype=np.uint8), "dphi": None, "phi0": phi0,
           "rho0": 1.0 + 0.01 * np.sin(2 * np.pi * y / 29) + 0 * x,
           "ux0": 0.01 * np.cos(2 * np.pi * y / 31) + 0 * x, "uy0": np.zeros((ny, nx))}
    say("  inputs ready")
    lat = lbm.lb_init(lbm.make_params(p, "f64", inplace=1), inp["solid"], inp["phi0"],
                      rho0=inp["rho0"], ux0=inp["ux0"], uy0=inp["uy0"])
    say("  initialised")
    lbm.lb_set_tuning(lat, 64, 32)
    lbm.lb_step(lat, K)
    fields = lbm.lb_read_fields(lat)
    lat.close()
    torch.cuda.empty_cache()
    say("  GPU run done")
    for y0 in (ny - W // 2, ny // 2, ny - W):
        ys = np.arange(y0, y0 + W) % ny
        sub = {k: (None if v is None else v[ys, :].copy()) for k, v in inp.items()}
        orc = make_oracle(dict(p, ny=W), sub)
        orc.step(K)
        for fname, g, o in zip(("phi", "rho", "ux", "uy"), fields, orc.fields()):
            gw = g[ys[MARGIN:W - MARGIN], :]
            ow = o[MARGIN:W - MARGIN, :]
            scale = max(np.abs(ow).max(), 1e-300) if fname in ("phi", "rho") else 1.0
            err = np.abs(gw - ow).max() / scale
            say(f"  window at y = {y0}: {fname} err {err:.2e}")
            assert err <= 1e-12, (y0, fname, err)
