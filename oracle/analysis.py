"""Oracle-side measurements and closed forms (TEST INFRASTRUCTURE, numpy).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark use
this module. Nothing here is shared with the HIP library.

  theory_dphi / theory_angle   Sec. IV, Eq. (theory): wall gradient vs angle
  cahn_angle                   Young's law Eq. (Young) with the wall tensions
                               of the Landau free energy Eqs. (freeen), (bulkfe)
                               (an independent route to the same curve)
  surface_tension, width       Sec. II and Sec. IV: gamma = sqrt(8 kappa a / 9),
                               W = 2 sqrt(2 kappa / a)
  contact_angle                Sec. IV: phi = 0 crossings on lattice links by
                               linear interpolation, least-squares circle,
                               angle with the wall
  flat_profile                 the discrete flat interface: Eq. (chempot) with
                               the Laplacian of Eq. (best) and uniform mu
  wall_film_profile            the discrete equilibrium of a film between two
                               wetting walls (Sec. II, ghost rows of reading R4)
                               at a given total phi, by Newton
  wall_tension,                the discrete wall and interface tensions of the
  discrete_interface_tension   free energy of Eqs. (freeen), (bulkfe) on the
                               lattice (bulk term per node, kappa/2 (d phi)^2 per
                               link, the wall term at the first fluid row)
  discrete_young_angle         Eq. (Young) with those discrete tensions
"""
import math

import numpy as np


def surface_tension(kappa, a):
    return math.sqrt(8.0 * kappa * a / 9.0)


def interface_width(kappa, a):
    return 2.0 * math.sqrt(2.0 * kappa / a)


def theory_dphi(theta_deg, kappa, a):
    """Eq. (theory): d_perp phi at the wall for an equilibrium angle theta."""
    th = math.radians(theta_deg)
    alpha = math.acos(math.sin(th) ** 2)
    c = math.cos(alpha / 3.0)
    s = math.copysign(1.0, th - math.pi / 2) if abs(th - math.pi / 2) > 0 else 0.0
    return 2.0 * s * math.sqrt(c * (1.0 - c)) / math.sqrt(2.0 * kappa / a)


def theory_angle(dphi, kappa, a):
    """Inverse of Eq. (theory) by bisection (the right side is monotonic in theta)."""
    lo, hi = 0.0, 180.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if theory_dphi(mid, kappa, a) < dphi:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def cahn_angle(dphi, kappa, a):
    """Young's angle from the wall tensions of the free energy with surface term
    xi*phi, xi = kappa * d_perp phi (Sec. II). For a semi-infinite phase the
    profile obeys kappa/2 phi'^2 = a/4 (1 - phi^2)^2, the wall value follows from
    kappa phi'(0) = xi, and gamma_s = xi phi_s + int kappa phi'^2 dz."""
    xi = kappa * dphi
    om = dphi * math.sqrt(2.0 * kappa / a)
    if abs(om) >= 1.0:
        return float("nan")
    s = math.sqrt(kappa * a / 2.0)
    pa = math.sqrt(1.0 - om)   # wall value under bulk phi = +1
    pb = -math.sqrt(1.0 + om)  # wall value under bulk phi = -1
    g_as = xi * pa + s * (2.0 / 3.0 - pa + pa ** 3 / 3.0)
    g_bs = xi * pb + s * (2.0 / 3.0 + pb - pb ** 3 / 3.0)
    cos_t = (g_bs - g_as) / surface_tension(kappa, a)
    return math.degrees(math.acos(max(-1.0, min(1.0, cos_t))))


# ---------------------------------------------------------------- contact angle

def crossing_points(phi, solid, x_lo, x_hi, y_lo, y_hi):
    """phi = 0 crossings on axis links between two fluid nodes (Sec. IV).

    Returns (pts, pos_end): crossing coordinates (k, 2) and the coordinates of
    the phi > 0 end of each link. x and y are unwrapped (periodic lattice) to the
    image nearest the centre of the window [x_lo, x_hi) x [y_lo, y_hi]."""
    ny, nx = phi.shape
    cx = 0.5 * (x_lo + x_hi)
    cy = 0.5 * (y_lo + y_hi)
    fluid = ~np.asarray(solid, dtype=bool)
    pts, pos = [], []
    for dx, dy in ((1, 0), (0, 1)):
        phi_b = np.roll(phi, shift=(-dy, -dx), axis=(0, 1))    # phi at (x+dx, y+dy)
        fluid_b = np.roll(fluid, shift=(-dy, -dx), axis=(0, 1))
        sel = fluid & fluid_b & (((phi > 0) & (phi_b < 0)) | ((phi < 0) & (phi_b > 0)))
        ys, xs = np.nonzero(sel)
        a, b = phi[ys, xs], phi_b[ys, xs]
        t = a / (a - b)
        px, py = xs + t * dx, ys + t * dy
        ex = np.where(a > 0, xs, xs + dx).astype(float)
        ey = np.where(a > 0, ys, ys + dy).astype(float)
        sx = nx * np.round((px - cx) / nx)
        sy = ny * np.round((py - cy) / ny)
        px, py, ex, ey = px - sx, py - sy, ex - sx, ey - sy
        keep = (px >= x_lo) & (px < x_hi) & (py >= y_lo) & (py <= y_hi)
        pts.append(np.stack([px[keep], py[keep]], axis=1))
        pos.append(np.stack([ex[keep], ey[keep]], axis=1))
    return np.concatenate(pts).reshape(-1, 2), np.concatenate(pos).reshape(-1, 2)


def fit_circle(pts):
    """Algebraic least-squares circle x^2 + y^2 + D x + E y + F = 0."""
    x, y = pts[:, 0], pts[:, 1]
    A = np.stack([x, y, np.ones_like(x)], axis=1)
    rhs = -(x * x + y * y)
    (D, E, F), *_ = np.linalg.lstsq(A, rhs, rcond=None)
    xc, yc = -D / 2.0, -E / 2.0
    return xc, yc, math.sqrt(max(xc * xc + yc * yc - F, 0.0))


def contact_angle(phi, solid, y_wall, wall_dir, x_lo, x_hi, y_lo, y_hi):
    """Angle (degrees, through the phi > 0 phase) between the fitted circle and
    the wall plane y = y_wall, whose normal into the fluid is (0, wall_dir).

    Returns dict(theta, xc, yc, R, n) or None when fewer than 3 points are found
    or the circle does not reach the wall."""
    pts, pos = crossing_points(phi, solid, x_lo, x_hi, y_lo, y_hi)
    if len(pts) < 3:
        return None
    xc, yc, R = fit_circle(pts)
    if not R > 0 or abs(yc - y_wall) > R:
        return None
    inside = np.hypot(pos[:, 0] - xc, pos[:, 1] - yc) < R
    phi_pos_inside = 2 * int(inside.sum()) > len(inside)
    cos_in = -wall_dir * (yc - y_wall) / R
    th = math.degrees(math.acos(max(-1.0, min(1.0, cos_in))))
    if not phi_pos_inside:
        th = 180.0 - th
    return {"theta": th, "xc": xc, "yc": yc, "R": R, "n": len(pts)}


# ---------------------------------------------------------------- flat interface

def flat_profile(phi_init, A, B, kappa, iters=60):
    """Newton solve, on a periodic 1-D lattice, of A phi + B phi^3 - kappa L phi = mu0
    with L phi_j = phi_{j+1} + phi_{j-1} - 2 phi_j (Eq. (best) on a field that is
    constant across the other axis), mu0 unknown and sum(phi) fixed."""
    phi = np.array(phi_init, dtype=float)
    n = phi.size
    total = phi.sum()
    mu0 = 0.0
    for _ in range(iters):
        lap = np.roll(phi, -1) + np.roll(phi, 1) - 2.0 * phi
        res = np.concatenate([A * phi + B * phi ** 3 - kappa * lap - mu0, [phi.sum() - total]])
        J = np.zeros((n + 1, n + 1))
        idx = np.arange(n)
        J[idx, idx] = A + 3.0 * B * phi ** 2 + 2.0 * kappa
        J[idx, (idx + 1) % n] -= kappa
        J[idx, (idx - 1) % n] -= kappa
        J[idx, n] = -1.0
        J[n, :n] = 1.0
        step = np.linalg.solve(J, -res)
        phi += step[:n]
        mu0 += step[n]
        if np.max(np.abs(step)) < 1e-15:
            break
    return phi, mu0


# ---------------------------------------------------------------- flat walls

def _walled_newton(phi, A, B, kappa, d_lo, d_hi, total, iters=80):
    """Newton solve of A phi + B phi^3 - kappa L phi = mu0 on the fluid rows
    1..n of a channel whose solid rows 0 and n+1 carry the ghost values of the
    wall condition (Sec. II, d_perp phi = xi / kappa, the gradient taken across
    the mid-link wall plane): phi_0 = phi_1 - d_lo, phi_{n+1} = phi_n - d_hi.
    L phi_j = phi_{j+1} + phi_{j-1} - 2 phi_j is Eq. (best) on a field constant
    along the wall. With `total` given, sum(phi) is fixed and mu0 is an unknown;
    otherwise mu0 = 0 and the far end (d_hi = None) is held at its bulk value."""
    phi = np.array(phi, dtype=float)
    n = phi.size
    fixed_far = d_hi is None
    far = phi[-1]
    mu0 = 0.0
    m = n + (1 if total is not None else 0)
    for _ in range(iters):
        lo = phi[0] - d_lo
        hi = far if fixed_far else phi[-1] - d_hi
        ext = np.concatenate([[lo], phi, [hi]])
        lap = ext[2:] + ext[:-2] - 2.0 * phi
        res = A * phi + B * phi ** 3 - kappa * lap - mu0
        J = np.zeros((m, m))
        idx = np.arange(n)
        J[idx, idx] = A + 3.0 * B * phi ** 2 + 2.0 * kappa
        J[idx[:-1], idx[:-1] + 1] -= kappa
        J[idx[1:], idx[1:] - 1] -= kappa
        J[0, 0] -= kappa                 # the ghost phi_0 follows phi_1
        if not fixed_far:
            J[n - 1, n - 1] -= kappa     # the ghost phi_{n+1} follows phi_n
        if total is not None:
            J[idx, n] = -1.0
            J[n, :n] = 1.0
            res = np.concatenate([res, [phi.sum() - total]])
        step = np.linalg.solve(J, -res)
        phi += step[:n]
        if total is not None:
            mu0 += step[n]
        if np.max(np.abs(step)) < 1e-15:
            break
    return phi, mu0


def wall_film_profile(phi_init, A, B, kappa, d_lo, d_hi):
    """The discrete equilibrium across a channel between two flat walls with
    wall gradients d_lo (bottom) and d_hi (top), at the total phi of phi_init
    (the fluid rows only). Returns (phi, mu0)."""
    phi_init = np.asarray(phi_init, dtype=float)
    return _walled_newton(phi_init, A, B, kappa, d_lo, d_hi, phi_init.sum())


def wall_tension(dphi, bulk, A, B, kappa, n=80):
    """Tension of a flat wall against the bulk phase phi = bulk (+1 or -1) in the
    discrete free energy whose stationary points the lattice reaches: the sum
    over fluid rows of psi(phi) - psi(bulk), the gradient energy kappa/2 (dphi)^2
    of every link between fluid rows, and the surface term xi phi_1 of Sec. II,
    xi = kappa d_perp phi, at the first fluid row. Its stationarity condition at
    row 1 is the chemical potential with the ghost row phi_0 = phi_1 - d_perp phi."""
    phi, _ = _walled_newton(np.full(n, float(bulk)), A, B, kappa, dphi, None, None)
    psi = lambda p: 0.5 * A * p ** 2 + 0.25 * B * p ** 4
    ext = np.concatenate([phi, [float(bulk)]])
    return ((psi(phi) - psi(float(bulk))).sum() + 0.5 * kappa * (np.diff(ext) ** 2).sum()
            + kappa * dphi * phi[0])


def discrete_interface_tension(A, B, kappa, n=400):
    """Tension of a flat interface in the same discrete free energy (bulk
    energy per node plus kappa/2 (dphi)^2 per link), from the Newton profile."""
    a = -A
    x = np.arange(float(n))
    w = math.sqrt(2.0 * kappa / a)
    prof, _ = flat_profile(np.tanh((n / 4 - np.abs(x - (n - 1) / 2)) / w), A, B, kappa)
    psi = lambda p: 0.5 * A * p ** 2 + 0.25 * B * p ** 4 - (0.5 * A + 0.25 * B)
    return 0.5 * (psi(prof).sum() + 0.5 * kappa * ((np.roll(prof, -1) - prof) ** 2).sum())


def discrete_young_angle(dphi, A, B, kappa):
    """Young's law, Eq. (Young), with the wall and interface tensions of the
    discrete free energy: the equilibrium angle (degrees, through phi > 0) that
    the lattice's wetting condition implies for a drop large against W."""
    g_as = wall_tension(dphi, 1.0, A, B, kappa)
    g_bs = wall_tension(dphi, -1.0, A, B, kappa)
    c = (g_bs - g_as) / discrete_interface_tension(A, B, kappa)
    return math.degrees(math.acos(max(-1.0, min(1.0, c))))
