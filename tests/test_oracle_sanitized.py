"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer.

A small C driver (oracle/sanitize_driver.c) links lbm_oracle.c into one
instrumented executable and runs every exported routine on one case: create,
step, wall-field update, population round trip, fields, diagnostics, and the
individual steps (moments, ghosts, gradients, both streamings, the wall
reversal, tau). Any out-of-bounds access, use after free, leak, signed overflow
or other undefined behaviour ends it with a report (every check is fatal). The
cases cover each option of the method (BGK and MRT, both Step 2 flags, the
clamp, the tau table, lattice-node bounce-back), the smallest lattice the
oracle accepts, lattices with no wall and with one-node channels, and a rejected
case. What the instrumented build computed must equal the ordinary library's
result bit for bit."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from paper_0812_1282_amd import workloads as wl

HERE = os.path.dirname(os.path.abspath(__file__))
ORACLE = os.path.join(os.path.dirname(HERE), "oracle")

SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("gcc is not available")
    exe = str(tmp_path_factory.mktemp("san") / "sanitize_driver")
    # the ordinary build's floating-point flags, so results match bit for bit
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-Wall", "-Wextra", "-Werror", *SAN, "-o", exe,
           os.path.join(ORACLE, "sanitize_driver.c"), os.path.join(ORACLE, "lbm_oracle.c"), "-lm"]
    subprocess.run(cmd, check=True)
    return exe


def run_driver(exe, d, p, inp, steps):
    os.makedirs(d, exist_ok=True)
    fields = [p["nx"], p["ny"], p["A"], p["B"], p["kappa"], p["Gamma"], p["tau_alpha"],
              p["tau_beta"], p.get("tau_phi", 1.0), 1 if p["collision"] == "mrt" else 0,
              p["zero_u_feq"], p["zero_u_geq"], p.get("tau_clamp", 0), p.get("tau_lut", 0),
              p.get("bounce", 0), steps]
    with open(os.path.join(d, "params.txt"), "w") as fp:
        fp.write(" ".join(repr(v) if isinstance(v, float) else str(v) for v in fields) + "\n")
    np.ascontiguousarray(inp["solid"], dtype=np.uint8).tofile(os.path.join(d, "solid.u8"))
    for k, name in (("dphi", "dphi"), ("phi0", "phi"), ("rho0", "rho"), ("ux0", "ux"),
                    ("uy0", "uy")):
        np.ascontiguousarray(inp[k], dtype=np.float64).tofile(os.path.join(d, f"{name}.f64"))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    return subprocess.run([exe, d], capture_output=True, text=True, env=env, timeout=300)


def oracle_side(p, inp, steps):
    ny, nx = inp["solid"].shape
    op = oracle.make_params(nx, ny, A=p["A"], B=p["B"], kappa=p["kappa"], Gamma=p["Gamma"],
                            tau_alpha=p["tau_alpha"], tau_beta=p["tau_beta"],
                            tau_phi=p.get("tau_phi", 1.0),
                            collision=oracle.MRT if p["collision"] == "mrt" else oracle.BGK,
                            zero_u_feq=p["zero_u_feq"], zero_u_geq=p["zero_u_geq"],
                            tau_clamp=p.get("tau_clamp", 0), tau_lut=p.get("tau_lut", 0),
                            bounce=p.get("bounce", 0))
    o = oracle.Oracle(op, inp["solid"], inp["phi0"], inp["dphi"], inp["rho0"], inp["ux0"],
                      inp["uy0"])
    o.step(steps)
    f, g = o.populations()
    solid = inp["solid"]
    rho, phi, ux, uy = oracle.moments(solid, f, g)
    phix = oracle.ghosts(solid, inp["dphi"], phi)
    parts = [rho, phi, ux, uy, phix, *oracle.gradients(phix, solid), oracle.stream(solid, f),
             oracle.stream_lattice_node(solid, f), oracle.reflect_walls(solid, f),
             np.array([oracle.tau(op, -1.6 + 3.2 * k / 63.0) for k in range(64)])]
    d = o.diagnostics()
    diag = [d["sum_rho"], d["sum_phi"], d["kinetic"], d["max_u"], d["n_fluid"]]
    return f, g, np.stack(o.fields()), np.array(diag, dtype=np.float64), \
        np.concatenate([a.ravel() for a in parts])


def one_node_channels(p, seed):
    inp = wl.random_fields(p, seed=seed, walls=False)
    ny, nx = p["ny"], p["nx"]
    solid = np.ones((ny, nx), dtype=np.uint8)
    solid[ny // 2, :] = 0
    solid[:, nx // 2] = 0
    inp = {k: (np.where(solid == 0, v, 0.0) if isinstance(v, np.ndarray) and k != "solid" else v)
           for k, v in inp.items()}
    inp["solid"] = solid
    inp["dphi"] = wl.wall_field(solid, -0.1)
    return inp


def case(name):
    """(params, inputs, steps) of a named case."""
    if name == "mrt step2 clamp":
        p = wl.params(30, 20, 1.3, 0.6, "mrt", Gamma=0.3, tau_phi=0.8, zero_u_feq=1,
                      zero_u_geq=1, tau_clamp=1)
        inp = wl.random_fields(p, seed=3)
        inp["dphi"] = wl.wall_field(inp["solid"], 0.05)
        return p, inp, 40
    if name == "bgk table lattice-node":
        p = wl.params(17, 9, 2.0, 0.7, "bgk", tau_lut=7, bounce=1)
        inp = wl.random_fields(p, seed=4)
        inp["dphi"] = wl.wall_field(inp["solid"], -0.08)
        return p, inp, 31
    if name == "smallest lattice":
        p = wl.params(3, 3, 1.0, 1.0, "mrt", zero_u_feq=0, zero_u_geq=0)
        return p, wl.random_fields(p, seed=5, walls=False), 9
    if name == "no walls":
        p = wl.params(11, 7, 1.2, 0.7, "mrt", zero_u_feq=0, zero_u_geq=0, tau_lut=1000)
        return p, wl.random_fields(p, seed=6, walls=False), 20
    if name == "one-node channels":
        p = wl.params(16, 9, 1.2, 0.7, "mrt", zero_u_feq=1, zero_u_geq=0, bounce=1)
        return p, one_node_channels(p, 7), 25
    raise KeyError(name)


CASES = ["mrt step2 clamp", "bgk table lattice-node", "smallest lattice", "no walls",
         "one-node channels"]


@pytest.mark.parametrize("name", CASES)
def test_sanitized_oracle_is_clean_and_identical(driver, tmp_path, name):
    p, inp, steps = case(name)
    if inp["dphi"] is None:
        inp["dphi"] = np.zeros(inp["solid"].shape)
    for k in ("zero_u_feq", "zero_u_geq"):
        p.setdefault(k, 1 if (k == "zero_u_feq" and p["collision"] == "mrt") else 0)
    r = run_driver(driver, str(tmp_path), p, inp, steps)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, r.stderr[-4000:]
    got = {k: np.fromfile(os.path.join(tmp_path, f"out_{k}.f64"))
           for k in ("f", "g", "fields", "diag", "parts")}
    f, g, fields, diag, parts = oracle_side(p, inp, steps)
    assert np.array_equal(got["f"], f.ravel())
    assert np.array_equal(got["g"], g.ravel())
    assert np.array_equal(got["fields"], fields.ravel())
    assert np.array_equal(got["diag"], diag)
    assert np.array_equal(got["parts"], parts)


def test_sanitized_oracle_rejects_cleanly(driver, tmp_path):
    p = wl.params(10, 8, 1.0, 1.0, "bgk", tau_lut=1)
    p.update(zero_u_feq=0, zero_u_geq=0)
    inp = wl.random_fields(p, seed=1)
    inp["dphi"] = wl.wall_field(inp["solid"], 0.0)
    r = run_driver(driver, str(tmp_path), p, inp, 5)
    assert r.returncode == 3, r.stderr[-4000:]
    assert "Sanitizer" not in r.stderr and "runtime error" not in r.stderr
