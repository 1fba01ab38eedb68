"""Shared test helpers: turn a workload dictionary into oracle parameters."""
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
