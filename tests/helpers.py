"""Shared test helpers: turn a workload dictionary into oracle parameters."""
import numpy as np

import oracle

COLL = {"bgk": oracle.BGK, "mrt": oracle.MRT}


def orc_params(p, **over):
    q = dict(p)
    q.update(over)
    return oracle.make_params(q["nx"], q["ny"], A=q["A"], B=q["B"], kappa=q["kappa"],
                              Gamma=q["Gamma"], tau_alpha=q["tau_alpha"],
                              tau_beta=q["tau_beta"], tau_phi=q["tau_phi"],
                              collision=COLL[q["collision"]],
                              zero_u_feq=q.get("zero_u_feq"),
                              zero_u_geq=q.get("zero_u_geq", 0),
                              tau_clamp=q.get("tau_clamp", 0),
                              tau_lut=q.get("tau_lut", 0), bounce=q.get("bounce", 0))


def make_oracle(p, inp, **over):
    return oracle.Oracle(orc_params(p, **over), inp["solid"], inp["phi0"], dphi=inp["dphi"],
                         rho0=inp["rho0"], ux0=inp["ux0"], uy0=inp["uy0"])


def max_u_near_contact(phi, ux, uy, solid, radius=5.0):
    """Peak |u| over fluid nodes within `radius` of the phi = 0 crossings of the
    first fluid row above the bottom wall (the spurious velocity at the contact
    points), or None without crossings."""
    speed = np.hypot(ux, uy)
    fluid = solid == 0
    row = phi[1]
    xs = [x + row[x] / (row[x] - row[x + 1]) for x in range(len(row) - 1)
          if fluid[1, x] and fluid[1, x + 1] and row[x] * row[x + 1] < 0]
    ny, nx = phi.shape
    y, x = np.mgrid[0:ny, 0:nx]
    near = np.zeros_like(fluid)
    for xc in xs:
        near |= np.hypot(x - xc, y - 1.0) <= radius
    near &= fluid
    return float(speed[near].max()) if near.any() else None
