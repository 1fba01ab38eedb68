"""Seeded synthetic inputs: lattice geometry, initial fields and parameter sets.

This module only lays out inputs (solid masks, wall-gradient fields, initial
phi/rho/u arrays and parameter dictionaries). It performs none of the lattice
Boltzmann arithmetic and imports neither the HIP binding nor the oracle, so the
same arrays feed both sides of every comparison.

Conventions: arrays are (ny, nx), node (x, y) at [y, x]; the lattice is doubly
periodic and walls are rows of solid nodes, so a wall plane sits half-way
between a solid row and the first fluid row (mid-link bounce-back).

Initial conditions (the paper does not print them): phi follows the flat
interface solution tanh(d / sqrt(2 kappa / a)) across each interface, plus
uniform noise in [-1e-3, 1e-3] at fluid nodes drawn from
numpy.random.default_rng(seed); rho = 1 and u = 0.
"""
import math

import numpy as np

# Landau parameters used by every workload: a = kappa = 0.04 (Sec. IV), written
# as mu = A phi + B phi^3 - kappa lap phi with A = -a, B = a.
BASE = dict(A=-0.04, B=0.04, kappa=0.04, Gamma=0.1, tau_phi=1.0, rho_ref=1.0)


def params(nx, ny, tau_alpha=1.0, tau_beta=1.0, collision="bgk", **kw):
    """Parameter dictionary (plain numbers) for one lattice."""
    p = dict(BASE)
    p.update(nx=int(nx), ny=int(ny), tau_alpha=float(tau_alpha), tau_beta=float(tau_beta),
             collision=collision)
    p.update(kw)
    return p


def _width(p):
    a = -p["A"]
    return math.sqrt(2.0 * p["kappa"] / a)


def walls_mask(nx, ny):
    """Solid rows y = 0 and y = ny - 1 (wall planes at y = 0.5 and ny - 1.5)."""
    solid = np.zeros((ny, nx), dtype=np.uint8)
    solid[0, :] = 1
    solid[ny - 1, :] = 1
    return solid


def wall_field(solid, value):
    """Wall gradient d_perp phi = value at every solid node, zero elsewhere."""
    return np.where(solid != 0, float(value), 0.0)


def noise(shape, seed, amp=1e-3):
    return np.random.default_rng(seed).uniform(-amp, amp, shape)


def drop_on_wall(p, radius, xc, yc, seed, dphi_wall, walls=True):
    """A circular drop (phi = +1 inside) centred at node (xc, yc) on the bottom
    wall, phi = -1 elsewhere; returns dict(solid, dphi, phi0, rho0, ux0, uy0)."""
    nx, ny = p["nx"], p["ny"]
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    d = np.hypot(x - xc, y - yc)
    phi = np.tanh((radius - d) / _width(p))
    solid = walls_mask(nx, ny) if walls else np.zeros((ny, nx), dtype=np.uint8)
    fluid = solid == 0
    phi = np.where(fluid, phi + noise((ny, nx), seed), 0.0)
    return dict(solid=solid, dphi=wall_field(solid, dphi_wall), phi0=phi,
                rho0=np.where(fluid, 1.0, 0.0), ux0=np.zeros((ny, nx)), uy0=np.zeros((ny, nx)))


def free_drop(p, radius, seed=0):
    """A drop in the middle of a doubly periodic box (no walls)."""
    nx, ny = p["nx"], p["ny"]
    return drop_on_wall(p, radius, nx / 2.0, ny / 2.0, seed, 0.0, walls=False)


def stripe(p, half_width, seed=0, walls=True, axis="x"):
    """A band of phi = +1 of half width `half_width` centred in x (across the
    walls) in a box that is periodic in x (and in y when walls is False)."""
    nx, ny = p["nx"], p["ny"]
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    c = (nx - 1) / 2.0 if axis == "x" else (ny - 1) / 2.0
    s = x if axis == "x" else y
    phi = np.tanh((half_width - np.abs(s - c)) / _width(p))
    solid = walls_mask(nx, ny) if walls else np.zeros((ny, nx), dtype=np.uint8)
    fluid = solid == 0
    if seed is not None:
        phi = phi + noise((ny, nx), seed)
    phi = np.where(fluid, phi, 0.0)
    return dict(solid=solid, dphi=wall_field(solid, 0.0), phi0=phi,
                rho0=np.where(fluid, 1.0, 0.0), ux0=np.zeros((ny, nx)), uy0=np.zeros((ny, nx)))


def capillary(p, seed, dphi_wall, x_in=None, x_out=None):
    """Capillary filling layout: a walled channel on [x_in, x_out) (solid rows
    0 and ny-1 there, wetting gradient on every solid node), wall-free periodic
    reservoirs elsewhere. phi = +1 for x < x_in, -1 beyond, with tanh fronts at
    the channel entrance and at the periodic seam x = 0."""
    nx, ny = p["nx"], p["ny"]
    x_in = nx // 2 if x_in is None else x_in
    x_out = (7 * nx) // 8 if x_out is None else x_out
    solid = np.zeros((ny, nx), dtype=np.uint8)
    solid[0, x_in:x_out] = 1
    solid[ny - 1, x_in:x_out] = 1
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    # Signed distance to the nearer front, positive inside the +1 column
    # (-0.5, x_in - 0.5): the fronts sit between nodes.
    inside = x < x_in
    d = np.where(inside, np.minimum(x + 0.5, x_in - 0.5 - x),
                 -np.minimum(x - (x_in - 0.5), nx - 0.5 - x))
    phi = np.tanh(d / _width(p))
    fluid = solid == 0
    phi = np.where(fluid, phi + noise((ny, nx), seed), 0.0)
    return dict(solid=solid, dphi=wall_field(solid, dphi_wall), phi0=phi,
                rho0=np.where(fluid, 1.0, 0.0), ux0=np.zeros((ny, nx)), uy0=np.zeros((ny, nx)))


def random_fields(p, seed, walls=True, amp_u=0.02):
    """Smooth random phi in [-1, 1] with random rho ~ 1 and small random u, for
    parity tests that exercise every term of the method."""
    nx, ny = p["nx"], p["ny"]
    rng = np.random.default_rng(seed)
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    phi = np.zeros((ny, nx))
    for _ in range(4):
        kx, ky = rng.integers(1, 3, size=2)
        ph = rng.uniform(0, 2 * np.pi, size=2)
        phi += np.sin(2 * np.pi * kx * x / nx + ph[0]) * np.cos(2 * np.pi * ky * y / ny + ph[1])
    phi = np.tanh(2.0 * phi / 4.0)
    solid = walls_mask(nx, ny) if walls else np.zeros((ny, nx), dtype=np.uint8)
    fluid = solid == 0
    rho = 1.0 + 0.01 * rng.uniform(-1, 1, (ny, nx))
    ux = amp_u * rng.uniform(-1, 1, (ny, nx))
    uy = amp_u * rng.uniform(-1, 1, (ny, nx))
    z = lambda a: np.where(fluid, a, 0.0)
    return dict(solid=solid, dphi=None, phi0=z(phi), rho0=z(rho), ux0=z(ux), uy0=z(uy))


# ------------------------------------------------------------------ workloads

def c1_drop(seed=1, dphi_wall=None):
    """100x50 BGK drop, equal viscosities, tau = 1, R = 25 at (50, 0), 60 degree wall."""
    p = params(100, 50, 1.0, 1.0, "bgk")
    return p, drop_on_wall(p, 25.0, 50.0, 0.0, seed, dphi_wall)


def c2_drop(collision, dphi_wall, seed=201):
    """256x128 drop, R = 60 at (128, 0), tau 0.55 (phi = -1) to 1.0 (phi = +1)."""
    p = params(256, 128, 1.0, 0.55, collision)
    return p, drop_on_wall(p, 60.0, 128.0, 0.0, seed, dphi_wall)


def c3_capillary(nx, ny, ratio, dphi_wall, seed=3, collision="mrt"):
    """Capillary filling, viscosity ratio 1 (tau 1/1) or 10 (tau 1/0.55)."""
    tb = 1.0 if ratio == 1 else 0.55
    p = params(nx, ny, 1.0, tb, collision)
    return p, capillary(p, seed, dphi_wall)


def c4_drop(nx=4096, ny=2048, radius=800.0, seed=4):
    """Large MRT drop, viscosity ratio 10, 90 degree wall (d_perp phi = 0)."""
    p = params(nx, ny, 1.0, 0.55, "mrt")
    return p, drop_on_wall(p, radius, nx / 2.0, 0.0, seed, 0.0)


C5_SIZES = ((64, 32), (128, 64), (256, 128), (512, 256))


def c5_instances(n=256, seed=5):
    """Ensemble description: per instance (nx, ny, theta_deg, ratio, tau_beta,
    noise seed). Sizes uniform over C5_SIZES, theta ~ U[30, 150], log10 ratio ~
    U[0, 2], tau_beta = 0.5 + 0.5 / ratio so that tau_alpha = 1 is the more
    viscous phase."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        nx, ny = C5_SIZES[int(rng.integers(0, len(C5_SIZES)))]
        theta = float(rng.uniform(30.0, 150.0))
        ratio = float(10.0 ** rng.uniform(0.0, 2.0))
        out.append(dict(nx=nx, ny=ny, theta=theta, ratio=ratio,
                        tau_beta=0.5 + 0.5 / ratio, seed=5001 + i))
    return out


def c5_member(desc, dphi_wall):
    """One ensemble member. tau(phi) clamps phi to [-1, 1]: with tau_beta as low
    as 0.505, the overshoot of phi to about -1.12 next to a non-wetting wall
    would take the unclamped law below 1/2."""
    p = params(desc["nx"], desc["ny"], 1.0, desc["tau_beta"], "mrt", tau_clamp=1)
    return p, drop_on_wall(p, 0.4 * desc["ny"], desc["nx"] / 2.0, 0.0, desc["seed"], dphi_wall)


def fig5_capillary(mobility, collision, dphi_wall, seed=6, a=0.02, kappa=0.02):
    """The capillary-filling geometry of Sec. VII (Fig. 5): a channel of length
    640 and width h = 50 between two 480 x 200 reservoirs, joined through the
    periodic seam so that their pressures are equal. The lattice is 1600 x 200.
    The channel walls are solid blocks over x in [480, 1120), outside the fluid
    rows 75..124 (wall planes at y = 74.5 and 124.5). phi = +1 (fluid alpha,
    nu = 0.83) in the left reservoir, -1 (fluid beta, nu = 0.03) in the channel
    and the right reservoir. gamma = 0.0188 gives a = kappa = 0.02; the mobility
    M = Gamma (tau_phi - 1/2) gives Gamma = 2 M at tau_phi = 1. Other (a, kappa)
    with 8 kappa a / 9 = gamma^2 give the same tension with another interface
    width (the paper states gamma only)."""
    nx, ny, x_in, x_out, y_lo, y_hi = 1600, 200, 480, 1120, 75, 125
    p = params(nx, ny, 3 * 0.83 + 0.5, 3 * 0.03 + 0.5, collision,
               A=-a, B=a, kappa=kappa, Gamma=2.0 * mobility)
    solid = np.zeros((ny, nx), dtype=np.uint8)
    solid[:y_lo, x_in:x_out] = 1
    solid[y_hi:, x_in:x_out] = 1
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    # signed distance to the nearer front, positive in the left reservoir
    # (-0.5, x_in - 0.5): fronts at the channel entrance and at the seam
    inside = x < x_in
    d = np.where(inside, np.minimum(x + 0.5, x_in - 0.5 - x),
                 -np.minimum(x - (x_in - 0.5), nx - 0.5 - x))
    phi = np.tanh(d / _width(p))
    fluid = solid == 0
    phi = np.where(fluid, phi + noise((ny, nx), seed), 0.0)
    geom = dict(x_in=x_in, x_out=x_out, y_lo=y_lo, y_hi=y_hi, h=float(y_hi - y_lo))
    return p, dict(solid=solid, dphi=wall_field(solid, dphi_wall), phi0=phi,
                   rho0=np.where(fluid, 1.0, 0.0), ux0=np.zeros((ny, nx)),
                   uy0=np.zeros((ny, nx)), geometry=geom)


def fig2_drop(tau_alpha, tau_beta, collision, seed=7):
    """The equilibrium-angle set-up of Sec. IV (Fig. 2): 300 x 100, walls at the
    bottom and top rows, a semicircle of radius 35 on the bottom wall at 90
    degrees, a = kappa = 0.04, Gamma = 0.5, tau_phi = 1."""
    p = params(300, 100, tau_alpha, tau_beta, collision, Gamma=0.5)
    return p, drop_on_wall(p, 35.0, 150.0, 0.0, seed, 0.0)
