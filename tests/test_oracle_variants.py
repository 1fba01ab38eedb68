"""Pins of the oracle's two paper variants: the tau table of Sec. VI and
lattice-node bounce-back (Fig. 9b).

The table: brute-force nearest-entry search over an explicit list, the closed
forms of tables of two and three entries, and the quantisation bound. Lattice-
node bounce-back: a single population traced through streaming and reflection
(it must come back to the node it left, reversed, one step later than with
mid-link bounce-back), invariance of a fluid at rest, exact conservation over
fluid and wall nodes together, and identity with mid-link when there is no wall.
"""
import numpy as np
import pytest

import oracle
from paper_0812_1282_amd import workloads as wl
from tests.helpers import make_oracle

E = np.array([(0, 0), (1, 0), (-1, 0), (0, 1), (0, -1), (1, 1), (-1, -1), (-1, 1), (1, -1)])
OPP = [0, 2, 1, 4, 3, 6, 5, 8, 7]


def _nearest_by_scan(entries, t):
    d = [abs(e - t) for e in entries]
    return entries[d.index(min(d))]  # first minimum: the lower index on a tie


@pytest.mark.parametrize("n", [2, 3, 7, 101, 10000])
@pytest.mark.parametrize("ta,tb", [(3.0, 0.7), (0.7, 3.0), (1.3, 0.6)])
def test_tau_table_is_the_nearest_entry(n, ta, tb):
    P = oracle.make_params(4, 4, tau_alpha=ta, tau_beta=tb, tau_lut=n)
    exact = oracle.make_params(4, 4, tau_alpha=ta, tau_beta=tb)
    entries = [tb + k * ((ta - tb) / (n - 1)) for k in range(n)]
    rng = np.random.default_rng(n)
    phis = list(rng.uniform(-1.6, 1.6, 400)) + [-1.0, 1.0, 0.0, -1.3, 1.3]
    for phi in phis:
        t = oracle.tau(exact, phi)
        got = oracle.tau(P, phi)
        assert got == _nearest_by_scan(entries, t), (phi, t, got)
        # quantisation bound inside the bulk range; the ends outside it
        if -1.0 <= phi <= 1.0:
            assert abs(got - t) <= abs(ta - tb) / (2 * (n - 1)) * (1 + 1e-12) + 1e-15
        else:  # past a bulk value: the end entry on that side
            assert got == (entries[-1] if phi > 1.0 else entries[0])


def test_tau_table_closed_forms():
    two = oracle.make_params(4, 4, tau_alpha=3.0, tau_beta=0.7, tau_lut=2)
    assert oracle.tau(two, -0.2) == 0.7 and oracle.tau(two, 0.2) == 3.0
    assert oracle.tau(two, 0.0) == 0.7  # a tie takes the lower entry
    three = oracle.make_params(4, 4, tau_alpha=3.0, tau_beta=0.7, tau_lut=3)
    assert oracle.tau(three, 0.49) == pytest.approx(1.85)
    assert oracle.tau(three, -0.49) == pytest.approx(1.85)
    assert oracle.tau(three, 0.51) == 3.0 and oracle.tau(three, -0.51) == 0.7
    flat = oracle.make_params(4, 4, tau_alpha=0.9, tau_beta=0.9, tau_lut=50)
    assert oracle.tau(flat, 0.3) == 0.9 and oracle.tau(flat, -7.0) == 0.9


def test_tau_table_enters_the_dynamics():
    """A fine table reproduces the clamped law closely; a coarse one differs."""
    p = wl.params(40, 24, 3.0, 0.7, "mrt")
    inp = wl.random_fields(p, seed=8)
    ref = make_oracle(p, inp, tau_clamp=1)
    fine = make_oracle(p, inp, tau_lut=1 << 22)
    coarse = make_oracle(p, inp, tau_lut=3)
    for o in (ref, fine, coarse):
        o.step(60)
    fluid = inp["solid"] == 0
    f_ref = ref.populations()[0][:, fluid]
    d_fine = np.abs(fine.populations()[0][:, fluid] - f_ref).max()
    d_coarse = np.abs(coarse.populations()[0][:, fluid] - f_ref).max()
    assert d_fine < 1e-7 and d_coarse > 1e-4, (d_fine, d_coarse)


def _channel(nx=7, ny=6):
    solid = np.zeros((ny, nx), dtype=np.uint8)
    solid[0, :] = 1
    solid[ny - 1, :] = 1
    return solid


@pytest.mark.parametrize("i", [4, 6, 8])
def test_lattice_node_pulse_returns_after_two_steps(i):
    """A population sent from a fluid node toward the wall row (e_i pointing into
    it) reaches the wall node, is reversed there and arrives back at the node it
    left, moving the other way, after the second streaming; mid-link
    bounce-back returns it after the first."""
    solid = _channel()
    ny, nx = solid.shape
    x0, y0 = 3, 1
    post = np.zeros((9, ny, nx))
    post[i, y0, x0] = 1.0
    first = oracle.stream_lattice_node(solid, post)
    xw, yw = (x0 + E[i, 0]) % nx, (y0 + E[i, 1]) % ny
    assert solid[yw, xw] == 1 and first[i, yw, xw] == 1.0 and first.sum() == 1.0
    second = oracle.stream_lattice_node(solid, oracle.reflect_walls(solid, first))
    assert second[OPP[i], y0, x0] == 1.0 and second.sum() == 1.0
    mid = oracle.stream(solid, post)
    assert mid[OPP[i], y0, x0] == 1.0 and mid.sum() == 1.0


def test_lattice_node_streaming_brute_force():
    """Every population of a fluid or wall node moves one link; what would enter
    a solid node with no fluid neighbour is dropped."""
    rng = np.random.default_rng(9)
    ny, nx = 7, 6
    solid = np.zeros((ny, nx), dtype=np.uint8)
    solid[0:2, :] = 1        # row 0 is interior solid (no fluid neighbour)
    solid[4, 3] = 1
    post = rng.standard_normal((9, ny, nx))

    def wall(x, y):
        return solid[y, x] and any(not solid[(y + E[k, 1]) % ny, (x + E[k, 0]) % nx]
                                   for k in range(1, 9))

    expect = np.zeros_like(post)
    for y in range(ny):
        for x in range(nx):
            if solid[y, x] and not wall(x, y):
                continue
            for i in range(9):
                xd, yd = (x + E[i, 0]) % nx, (y + E[i, 1]) % ny
                if not solid[yd, xd] or wall(xd, yd):
                    expect[i, yd, xd] = post[i, y, x]
    np.testing.assert_array_equal(oracle.stream_lattice_node(solid, post), expect)
    rev = oracle.reflect_walls(solid, post)
    for y in range(ny):
        for x in range(nx):
            want = post[OPP, y, x] if wall(x, y) else np.zeros(9)
            np.testing.assert_array_equal(rev[:, y, x], want)


@pytest.mark.parametrize("collision", ["bgk", "mrt"])
def test_lattice_node_rest_state_is_invariant(collision):
    """A uniform bulk phase at rest between walls stays exactly at rest."""
    p = wl.params(12, 9, 1.3, 0.8, collision)
    solid = _channel(12, 9)
    inp = {"solid": solid, "phi0": np.ones((9, 12)), "dphi": np.zeros((9, 12)),
           "rho0": np.ones((9, 12)), "ux0": np.zeros((9, 12)), "uy0": np.zeros((9, 12))}
    o = make_oracle(p, inp, bounce=1)
    f0 = o.populations()[0].copy()
    o.step(50)
    phi, rho, ux, uy = o.fields()
    fluid = solid == 0
    assert np.abs(ux[fluid]).max() < 1e-15 and np.abs(uy[fluid]).max() < 1e-15
    np.testing.assert_allclose(o.populations()[0][:, fluid], f0[:, fluid], atol=1e-15)


@pytest.mark.parametrize("collision", ["bgk", "mrt"])
def test_lattice_node_conserves_fluid_plus_wall_mass(collision):
    p = wl.params(30, 20, 1.2, 0.7, collision, tau_phi=0.8)
    inp = wl.random_fields(p, seed=4)
    inp["dphi"] = wl.wall_field(inp["solid"], -0.1)
    o = make_oracle(p, inp, bounce=1)
    f0, g0 = (a.sum() for a in o.populations())
    o.step(120)
    f1, g1 = (a.sum() for a in o.populations())
    assert abs(f1 - f0) <= 1e-12 * abs(f0) and abs(g1 - g0) <= 1e-11 * max(1.0, abs(g0))


def test_lattice_node_is_mid_link_without_walls():
    p = wl.params(16, 12, 1.2, 0.7, "mrt")
    inp = wl.random_fields(p, seed=2, walls=False)
    a = make_oracle(p, inp)
    b = make_oracle(p, inp, bounce=1)
    a.step(40)
    b.step(40)
    np.testing.assert_array_equal(a.populations()[0], b.populations()[0])
    np.testing.assert_array_equal(a.populations()[1], b.populations()[1])


def test_variant_parameters_are_validated():
    p = wl.params(10, 8)
    inp = wl.random_fields(p, seed=1)
    for over in ({"bounce": 2}, {"tau_lut": 1}, {"tau_lut": -5}):
        with pytest.raises(ValueError):
            make_oracle(p, inp, **over)
