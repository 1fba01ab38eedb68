"""The C ABI: the library loads, exports every symbol of include/lb.h, and
validates arguments on the host (no GPU needed for these calls)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_0812_1282_amd import lbm, workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "lb.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lb_[a-z_0-9]+)\s*\(", text)))


def test_header_and_binding_agree():
    assert _declared_functions() == sorted(lbm.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = lbm.load_library()
    for name in _declared_functions():
        assert hasattr(L, name), name


def test_default_params_and_workspace():
    L = lbm.load_library()
    p = lbm.lb_params()
    assert L.lb_default_params(100, 50, ctypes.byref(p)) == 0
    assert (p.nx, p.ny, p.collision, p.storage) == (100, 50, lbm.BGK, lbm.F64)
    assert p.A == -0.04 and p.B == 0.04 and p.kappa == 0.04
    n64 = lbm.lb_workspace_bytes(p)
    p.storage = lbm.F32
    n32 = lbm.lb_workspace_bytes(p)
    p.storage = lbm.F16S
    n16 = lbm.lb_workspace_bytes(p)
    # two population buffers of 18 planes, pitch 128 x 50 rows, dominate
    assert n64 > 2 * 18 * 128 * 50 * 8 > n32 > 2 * 18 * 128 * 50 * 4 > n16
    # compressed g: 13 planes instead of 18
    p.storage = lbm.F64C
    n64c = lbm.lb_workspace_bytes(p)
    p.storage = lbm.F32C
    n32c = lbm.lb_workspace_bytes(p)
    assert n64 > n64c > 2 * 13 * 128 * 50 * 8 and n32 > n32c > 2 * 13 * 128 * 50 * 4


@pytest.mark.parametrize("storage", ["F64C", "F32C"])
def test_compressed_formats_need_tau_phi_one(storage):
    p = lbm.lb_params()
    lbm.load_library().lb_default_params(16, 8, ctypes.byref(p))
    p.storage = getattr(lbm, storage)
    p.tau_phi = 0.8
    with pytest.raises(lbm.LbError) as e:
        lbm.lb_workspace_bytes(p)
    assert e.value.code == lbm.LB_EINVAL


def test_inplace_workspace_is_one_buffer_plus_a_plane():
    for st in ("f64", "f32"):
        p = wl.params(1000, 500)
        two = lbm.lb_workspace_bytes(lbm.make_params(p, st))
        one = lbm.lb_workspace_bytes(lbm.make_params(p, st, inplace=1))
        per = {"f64": 144, "f32": 72}[st]
        nodes = 1024 * 500  # rows padded to a multiple of 64
        assert two - one == per * nodes - 8 * nodes, (st, two, one)


@pytest.mark.parametrize("storage", ["F16S", "BF16S", "F64C", "F32C"])
def test_inplace_only_for_f64_and_f32(storage):
    p = lbm.lb_params()
    lbm.load_library().lb_default_params(16, 8, ctypes.byref(p))
    p.storage = getattr(lbm, storage)
    p.inplace = 1
    with pytest.raises(lbm.LbError) as e:
        lbm.lb_workspace_bytes(p)
    assert e.value.code == lbm.LB_EINVAL


@pytest.mark.parametrize("storage,inplace", [("f16s", 0), ("f64c", 0), ("f32c", 0), ("f32", 1)])
def test_lattice_node_bounce_back_formats(storage, inplace):
    p = dict(wl.params(16, 8), tau_phi=1.0, bounce=lbm.LATTICE_NODE)
    with pytest.raises(lbm.LbError) as e:
        lbm.lb_workspace_bytes(lbm.make_params(p, storage, inplace=inplace))
    assert e.value.code == lbm.LB_EINVAL
    assert lbm.lb_workspace_bytes(lbm.make_params(p, "f32")) > 0


def test_inplace_rejected_in_batches():
    """Rejected while validating, before any device work."""
    p = wl.params(8, 6)
    inp = wl.random_fields(p, seed=0)
    P = (lbm.lb_params * 1)(lbm.make_params(p, "f32", inplace=1))
    solid = np.ascontiguousarray(inp["solid"], dtype=np.uint8)
    phi0 = np.ascontiguousarray(inp["phi0"], dtype=np.float64)
    solids = (ctypes.POINTER(ctypes.c_uint8) * 1)(solid.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
    phis = (ctypes.POINTER(ctypes.c_double) * 1)(phi0.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    h = ctypes.c_void_p()
    rc = lbm.load_library().lb_batch_init(1, P, solids, None, phis, None, None, None, None, None,
                                          ctypes.byref(h))
    assert rc == lbm.LB_EINVAL and not h.value
    assert b"single lattices" in lbm.load_library().lb_last_error()


@pytest.mark.parametrize("field,value", [
    ("nx", 2), ("ny", 0), ("tau_alpha", 0.5), ("tau_beta", 0.3), ("tau_phi", 0.5),
    ("collision", 7), ("storage", 9), ("zero_u_feq", 2), ("diag_every", -1), ("tau_clamp", 2),
    ("inplace", 2), ("tau_lut", 1), ("tau_lut", -3), ("tau_lut", (1 << 24) + 1), ("bounce", 2),
    ("kappa", float("nan")), ("rho_ref", 0.0),
])
def test_init_rejects_bad_params_before_any_device_work(field, value):
    p = wl.params(8, 6)
    inp = wl.random_fields(p, seed=0)
    P = lbm.make_params(p)
    setattr(P, field, value)
    shape = (max(P.ny, 0), max(P.nx, 0))
    solid = np.zeros(shape, dtype=np.uint8) if field in ("nx", "ny") else inp["solid"]
    phi0 = np.zeros(shape) if field in ("nx", "ny") else inp["phi0"]
    with pytest.raises(lbm.LbError) as e:
        lbm.lb_init(P, solid, phi0, device_memory="library")
    assert e.value.code == lbm.LB_EINVAL


def test_init_rejects_bad_inputs():
    p = wl.params(8, 6)
    P = lbm.make_params(p)
    inp = wl.random_fields(p, seed=0)
    bad = inp["phi0"].copy()
    bad[2, 3] = np.inf
    with pytest.raises(lbm.LbError) as e:
        lbm.lb_init(P, inp["solid"], bad, device_memory="library")
    assert e.value.code == lbm.LB_EINVAL
    rho = inp["rho0"].copy()
    rho[2, 2] = -1.0
    with pytest.raises(lbm.LbError):
        lbm.lb_init(P, inp["solid"], inp["phi0"], rho0=rho, device_memory="library")
    enclosed = np.ones((6, 8), dtype=np.uint8)
    enclosed[3, 3] = 0
    with pytest.raises(lbm.LbError) as e:
        lbm.lb_init(P, enclosed, inp["phi0"], device_memory="library")
    assert "no fluid neighbour" in str(e.value)


def test_dphi_for_angle_host_helper():
    # Eq. (theory): 90 degrees is a neutral wall and the curve is odd about it.
    assert lbm.lb_dphi_for_angle(90.0, 0.04, -0.04, 0.04) == 0.0
    for th in (30.0, 60.0, 110.0):
        a = lbm.lb_dphi_for_angle(th, 0.04, -0.04, 0.04)
        b = lbm.lb_dphi_for_angle(180.0 - th, 0.04, -0.04, 0.04)
        assert a == pytest.approx(-b, abs=1e-15)
    assert lbm.lb_dphi_for_angle(60.0, 0.04, -0.04, 0.04) < 0
    with pytest.raises(lbm.LbError):
        lbm.lb_dphi_for_angle(200.0, 0.04, -0.04, 0.04)
    with pytest.raises(lbm.LbError):
        lbm.lb_dphi_for_angle(60.0, 0.04, -0.04, 0.05)


def test_dphi_for_angle_matches_oracle_closed_form():
    from oracle import analysis
    for th in np.linspace(0, 180, 37):
        assert lbm.lb_dphi_for_angle(th, 0.04, -0.04, 0.04) == pytest.approx(
            analysis.theory_dphi(th, 0.04, 0.04), abs=1e-14)


def test_null_handle_calls_fail_cleanly():
    L = lbm.load_library()
    assert L.lb_step(None, 1) == lbm.LB_EINVAL
    assert L.lb_free(None) == 0
    assert L.lb_batch_free(None) == 0
    assert b"NULL" in L.lb_last_error() or L.lb_last_error()


def test_size_limits():
    """The largest lattices the layout can address are accepted, larger ones are
    rejected before any allocation (host-side computation only)."""
    L = lbm.load_library()

    def params(nx, ny, storage="f32"):
        p = lbm.lb_params()
        L.lb_default_params(nx, ny, ctypes.byref(p))
        p.storage = lbm.STORAGE[storage]
        return p

    assert lbm.lb_workspace_bytes(params(14_000_000, 3, "f64")) > 14_000_000 * 3 * 288
    for nx, ny, st in [((1 << 24) + 1, 3, "f32"), (15_000_000, 3, "f64"), (1 << 20, (1 << 14) + 1, "f32")]:
        with pytest.raises(lbm.LbError) as e:
            lbm.lb_workspace_bytes(params(nx, ny, st))
        assert e.value.code == lbm.LB_EINVAL, (nx, ny, st)
