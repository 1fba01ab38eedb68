"""Python binding of liblbm.so (the C ABI in include/lb.h).

Argument marshalling only: every step of the method runs in the HIP library.
PyTorch supplies the device memory (one byte tensor per lattice, handed to
lb_init_ext) and the HIP stream (torch's current stream). If liblbm.so has not
been built, loading fails with an error; there is no fallback.

Function names follow the C ABI: lb_init, lb_step, lb_read_fields, ...
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm.so")

LB_OK, LB_EINVAL, LB_ENOMEM, LB_EHIP, LB_ENUMERIC, LB_ENODATA, LB_EIO = 0, -1, -2, -3, -4, -5, -6
BGK, MRT = 0, 1
F64, F32, F16S, BF16S, F64C, F32C = 0, 1, 2, 3, 4, 5
STORAGE = {"f64": F64, "f32": F32, "f16s": F16S, "bf16s": BF16S, "f64c": F64C, "f32c": F32C}
COLLISION = {"bgk": BGK, "mrt": MRT}
MIDLINK, LATTICE_NODE = 0, 1

EXPORTS = [
    "lb_default_params", "lb_workspace_bytes", "lb_init", "lb_init_ext", "lb_step",
    "lb_read_fields", "lb_read_populations", "lb_diagnostics", "lb_contact_angle",
    "lb_fill_length", "lb_set_wall_dphi", "lb_save", "lb_load", "lb_set_tuning",
    "lb_get_tuning", "lb_autotune", "lb_get_step", "lb_free", "lb_last_error",
    "lb_dphi_for_angle", "lb_batch_init", "lb_batch_step", "lb_batch_read_fields",
    "lb_batch_read_populations", "lb_batch_contact_angle", "lb_batch_get_tuning",
    "lb_batch_free", "lb_bandwidth_probe", "lb_batch_autotune", "lb_diagnostics_noalloc",
    "lb_batch_set_schedule", "lb_batch_get_schedule",
]
STEPWISE, PERSISTENT = 0, 1


class LbError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (code {code})")
        self.code = code


class lb_params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("A", ctypes.c_double), ("B", ctypes.c_double),
                ("kappa", ctypes.c_double), ("Gamma", ctypes.c_double),
                ("tau_alpha", ctypes.c_double), ("tau_beta", ctypes.c_double),
                ("tau_phi", ctypes.c_double), ("rho_ref", ctypes.c_double),
                ("collision", ctypes.c_int32), ("storage", ctypes.c_int32),
                ("zero_u_feq", ctypes.c_int32), ("zero_u_geq", ctypes.c_int32),
                ("diag_every", ctypes.c_int32), ("tau_clamp", ctypes.c_int32),
                ("inplace", ctypes.c_int32), ("tau_lut", ctypes.c_int32),
                ("bounce", ctypes.c_int32)]


class lb_diag(ctypes.Structure):
    _fields_ = [("sum_rho", ctypes.c_double), ("sum_phi", ctypes.c_double),
                ("kinetic", ctypes.c_double), ("max_u", ctypes.c_double),
                ("n_fluid", ctypes.c_int64), ("step", ctypes.c_int64)]


class lb_tuning(ctypes.Structure):
    _fields_ = [("block_x", ctypes.c_int32), ("rows_per_block", ctypes.c_int32)]


_D = ctypes.POINTER(ctypes.c_double)
_U8 = ctypes.POINTER(ctypes.c_uint8)
_VP = ctypes.c_void_p
_lib = None


def load_library(path=LIB_PATH):
    """Load liblbm.so (built by paper_0812_1282_amd/build.py); raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_0812_1282_amd.build`")
    # PyTorch ships its own HIP runtime (soname libamdhip64.so.7). Importing it
    # first makes the dynamic loader resolve this library's libamdhip64.so.7 to
    # that same copy, so the process holds one HIP runtime, shared by the torch
    # allocations and streams and by the kernels launched here.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(path)
    P = ctypes.POINTER(lb_params)
    i32, i64, dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "lb_default_params": [i32, i32, P],
        "lb_workspace_bytes": [P, ctypes.POINTER(ctypes.c_size_t)],
        "lb_init": [P, _U8, _D, _D, _D, _D, _D, _VP, ctypes.POINTER(_VP)],
        "lb_init_ext": [P, _U8, _D, _D, _D, _D, _D, _VP, _VP, ctypes.c_size_t, ctypes.POINTER(_VP)],
        "lb_step": [_VP, i64],
        "lb_read_fields": [_VP, _D, _D, _D, _D],
        "lb_read_populations": [_VP, _D, _D],
        "lb_diagnostics": [_VP, ctypes.POINTER(lb_diag)],
        "lb_diagnostics_noalloc": [_VP, ctypes.POINTER(lb_diag)],
        "lb_contact_angle": [_VP, dbl, dbl, dbl, dbl, dbl, i32, _D, _D, _D, _D,
                             ctypes.POINTER(i64)],
        "lb_fill_length": [_VP, i32, i32, dbl, _D],
        "lb_set_wall_dphi": [_VP, _D],
        "lb_save": [_VP, ctypes.c_char_p],
        "lb_load": [_VP, ctypes.c_char_p],
        "lb_set_tuning": [_VP, ctypes.POINTER(lb_tuning)],
        "lb_get_tuning": [_VP, ctypes.POINTER(lb_tuning)],
        "lb_autotune": [_VP, i32, ctypes.POINTER(lb_tuning)],
        "lb_get_step": [_VP, ctypes.POINTER(i64)],
        "lb_free": [_VP],
        "lb_dphi_for_angle": [dbl, dbl, dbl, dbl, _D],
        "lb_batch_init": [i32, P, ctypes.POINTER(_U8), ctypes.POINTER(_D), ctypes.POINTER(_D),
                          ctypes.POINTER(_D), ctypes.POINTER(_D), ctypes.POINTER(_D), _VP,
                          ctypes.POINTER(lb_tuning), ctypes.POINTER(_VP)],
        "lb_batch_step": [_VP, i64],
        "lb_batch_read_fields": [_VP, i32, _D, _D, _D, _D],
        "lb_batch_read_populations": [_VP, i32, _D, _D],
        "lb_batch_contact_angle": [_VP, i32, dbl, dbl, dbl, dbl, dbl, i32, _D],
        "lb_batch_get_tuning": [_VP, ctypes.POINTER(lb_tuning)],
        "lb_batch_autotune": [_VP, ctypes.c_int32, ctypes.POINTER(lb_tuning)],
        "lb_batch_free": [_VP],
        "lb_batch_set_schedule": [_VP, i32, ctypes.c_uint32],
        "lb_batch_get_schedule": [_VP, ctypes.POINTER(i32)],
        "lb_bandwidth_probe": [ctypes.c_size_t, i32, _VP, _D],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    L.lb_last_error.argtypes = []
    L.lb_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def _check(rc):
    if rc != LB_OK:
        raise LbError(rc, load_library().lb_last_error().decode())
    return rc


def _f64(a, shape):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.shape != shape:
        a = a.reshape(shape)
    return a


def _dp(a):
    return None if a is None else a.ctypes.data_as(_D)


def make_params(p, storage="f64", collision=None, zero_u_feq=None, zero_u_geq=0, diag_every=0,
                inplace=0):
    """lb_params from a workload dictionary (see workloads.params). Step 2
    (zero_u_feq) defaults to on for MRT and off for BGK. inplace=1 updates one
    population buffer in place (f64 and f32). The workload's "tau_lut" (table
    size, 0 = off) and "bounce" (MIDLINK or LATTICE_NODE) are passed through."""
    coll = COLLISION[collision or p["collision"]]
    if zero_u_feq is None:
        zero_u_feq = 1 if coll == MRT else 0
    return lb_params(p["nx"], p["ny"], p["A"], p["B"], p["kappa"], p["Gamma"],
                     p["tau_alpha"], p["tau_beta"], p["tau_phi"], p.get("rho_ref", 1.0),
                     coll, STORAGE[storage] if isinstance(storage, str) else int(storage),
                     int(zero_u_feq), int(zero_u_geq), int(diag_every),
                     int(p.get("tau_clamp", 0)), int(inplace), int(p.get("tau_lut", 0)),
                     int(p.get("bounce", 0)))


def _torch_stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Lattice:
    """An lb_handle. Device memory is a torch uint8 tensor unless
    device_memory='library' (then lb_init allocates it)."""

    def __init__(self, handle, params, buffer=None, stream=None):
        self._h = handle
        self._lib = load_library()  # held so that close() works during interpreter exit
        self.params = params
        self.shape = (params.ny, params.nx)
        self._buffer = buffer  # keeps the torch allocation alive
        self._stream = stream

    def __del__(self):
        self.close()

    def close(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.lb_free(h)
            self._h = None
            self._buffer = None


def lb_workspace_bytes(params):
    n = ctypes.c_size_t(0)
    _check(load_library().lb_workspace_bytes(ctypes.byref(params), ctypes.byref(n)))
    return n.value


def lb_init(params, solid, phi0, dphi=None, rho0=None, ux0=None, uy0=None,
            device_memory="torch"):
    """Create a lattice (S_0 = equilibria of the fields); arrays are (ny, nx)."""
    L = load_library()
    shape = (params.ny, params.nx)
    solid = np.ascontiguousarray(solid, dtype=np.uint8).reshape(shape)
    arrs = [_f64(a, shape) for a in (dphi, phi0, rho0, ux0, uy0)]
    h = ctypes.c_void_p()
    if device_memory == "torch":
        import torch
        nbytes = lb_workspace_bytes(params)
        buf = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        stream = _torch_stream()
        _check(L.lb_init_ext(ctypes.byref(params), solid.ctypes.data_as(_U8),
                             *[_dp(a) for a in arrs], stream, ctypes.c_void_p(buf.data_ptr()),
                             nbytes, ctypes.byref(h)))
        return Lattice(h.value, params, buf, stream)
    _check(L.lb_init(ctypes.byref(params), solid.ctypes.data_as(_U8), *[_dp(a) for a in arrs],
                     None, ctypes.byref(h)))
    return Lattice(h.value, params)


def lb_step(lat, nsteps):
    _check(load_library().lb_step(lat._h, int(nsteps)))


def lb_get_step(lat):
    s = ctypes.c_int64()
    _check(load_library().lb_get_step(lat._h, ctypes.byref(s)))
    return s.value


def lb_read_fields(lat):
    """(phi, rho, ux, uy) of S_n, each (ny, nx) float64."""
    out = [np.zeros(lat.shape) for _ in range(4)]
    _check(load_library().lb_read_fields(lat._h, *[_dp(a) for a in out]))
    return tuple(out)


def lb_read_populations(lat):
    """(f, g) of S_n, each (9, ny, nx) float64."""
    f = np.zeros((9,) + lat.shape)
    g = np.zeros((9,) + lat.shape)
    _check(load_library().lb_read_populations(lat._h, _dp(f), _dp(g)))
    return f, g


def lb_diagnostics(lat, check=True):
    d = lb_diag()
    rc = load_library().lb_diagnostics(lat._h, ctypes.byref(d))
    if check:
        _check(rc)
    return {"sum_rho": d.sum_rho, "sum_phi": d.sum_phi, "kinetic": d.kinetic, "max_u": d.max_u,
            "n_fluid": d.n_fluid, "step": d.step, "rc": rc}


def lb_diagnostics_noalloc(lat, check=True):
    """lb_diagnostics with its partial sums in the library's fixed device array
    (allocates nothing; lattices up to 2^23 nodes)."""
    d = lb_diag()
    rc = load_library().lb_diagnostics_noalloc(lat._h, ctypes.byref(d))
    if check:
        _check(rc)
    return {"sum_rho": d.sum_rho, "sum_phi": d.sum_phi, "kinetic": d.kinetic, "max_u": d.max_u,
            "n_fluid": d.n_fluid, "step": d.step, "rc": rc}


def lb_contact_angle(lat, x_lo, x_hi, y_lo, y_hi, y_wall, wall_dir):
    th, xc, yc, R = (ctypes.c_double() for _ in range(4))
    n = ctypes.c_int64()
    _check(load_library().lb_contact_angle(lat._h, x_lo, x_hi, y_lo, y_hi, y_wall, int(wall_dir),
                                           ctypes.byref(th), ctypes.byref(xc), ctypes.byref(yc),
                                           ctypes.byref(R), ctypes.byref(n)))
    return {"theta": th.value, "xc": xc.value, "yc": yc.value, "R": R.value, "n": n.value}


def lb_fill_length(lat, x_lo, x_hi, width):
    out = ctypes.c_double()
    _check(load_library().lb_fill_length(lat._h, int(x_lo), int(x_hi), float(width),
                                         ctypes.byref(out)))
    return out.value


def lb_set_wall_dphi(lat, dphi):
    d = _f64(dphi, lat.shape)
    _check(load_library().lb_set_wall_dphi(lat._h, _dp(d)))


def lb_save(lat, path):
    _check(load_library().lb_save(lat._h, str(path).encode()))


def lb_load(lat, path):
    _check(load_library().lb_load(lat._h, str(path).encode()))


def lb_set_tuning(lat, block_x, rows_per_block):
    t = lb_tuning(block_x, rows_per_block)
    _check(load_library().lb_set_tuning(lat._h, ctypes.byref(t)))


def lb_get_tuning(lat):
    t = lb_tuning()
    _check(load_library().lb_get_tuning(lat._h, ctypes.byref(t)))
    return t.block_x, t.rows_per_block


def lb_autotune(lat, steps_per_trial=10):
    t = lb_tuning()
    _check(load_library().lb_autotune(lat._h, int(steps_per_trial), ctypes.byref(t)))
    return t.block_x, t.rows_per_block


def lb_dphi_for_angle(theta_deg, kappa, A, B):
    out = ctypes.c_double()
    _check(load_library().lb_dphi_for_angle(float(theta_deg), float(kappa), float(A), float(B),
                                            ctypes.byref(out)))
    return out.value


def lb_free(lat):
    lat.close()


def lb_bandwidth_probe(nbytes=1 << 30, repeats=20):
    """Read + write GB/s of a streaming copy of nbytes on the current device."""
    out = ctypes.c_double()
    _check(load_library().lb_bandwidth_probe(int(nbytes), int(repeats), _torch_stream(),
                                             ctypes.byref(out)))
    return out.value


# ------------------------------------------------------------------ batches

class Batch:
    def __init__(self, handle, params, keep):
        self._h = handle
        self._lib = load_library()  # held so that close() works during interpreter exit
        self.params = params
        self._keep = keep

    def __del__(self):
        self.close()

    def close(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.lb_batch_free(h)
            self._h = None

    def shape(self, k):
        return (self.params[k].ny, self.params[k].nx)


def lb_batch_init(params_list, members, tuning=None):
    """members: list of dicts with solid, phi0 and optional dphi, rho0, ux0, uy0."""
    L = load_library()
    n = len(params_list)
    P = (lb_params * n)(*params_list)
    keep = []
    cols = {k: (ctypes.POINTER(ctypes.c_double) * n)() for k in ("dphi", "phi0", "rho0", "ux0", "uy0")}
    solids = (ctypes.POINTER(ctypes.c_uint8) * n)()
    for k, (p, m) in enumerate(zip(params_list, members)):
        shape = (p.ny, p.nx)
        s = np.ascontiguousarray(m["solid"], dtype=np.uint8).reshape(shape)
        keep.append(s)
        solids[k] = s.ctypes.data_as(_U8)
        for name in cols:
            a = _f64(m.get(name), shape)
            keep.append(a)
            cols[name][k] = a.ctypes.data_as(_D) if a is not None else None
    t = None if tuning is None else lb_tuning(*tuning)
    h = ctypes.c_void_p()
    _check(L.lb_batch_init(n, P, solids, cols["dphi"], cols["phi0"], cols["rho0"], cols["ux0"],
                           cols["uy0"], _torch_stream(), None if t is None else ctypes.byref(t),
                           ctypes.byref(h)))
    return Batch(h.value, list(params_list), keep)


def lb_batch_step(b, nsteps):
    _check(load_library().lb_batch_step(b._h, int(nsteps)))


def lb_batch_read_fields(b, k):
    out = [np.zeros(b.shape(k)) for _ in range(4)]
    _check(load_library().lb_batch_read_fields(b._h, int(k), *[_dp(a) for a in out]))
    return tuple(out)


def lb_batch_read_populations(b, k):
    f = np.zeros((9,) + b.shape(k))
    g = np.zeros((9,) + b.shape(k))
    _check(load_library().lb_batch_read_populations(b._h, int(k), _dp(f), _dp(g)))
    return f, g


def lb_batch_contact_angle(b, k, x_lo, x_hi, y_lo, y_hi, y_wall, wall_dir):
    th = ctypes.c_double()
    _check(load_library().lb_batch_contact_angle(b._h, int(k), x_lo, x_hi, y_lo, y_hi, y_wall,
                                                 int(wall_dir), ctypes.byref(th)))
    return th.value


def lb_batch_autotune(b, steps_per_trial=4):
    t = lb_tuning()
    _check(load_library().lb_batch_autotune(b._h, int(steps_per_trial), ctypes.byref(t)))
    return t.block_x, t.rows_per_block


def lb_batch_get_tuning(b):
    t = lb_tuning()
    _check(load_library().lb_batch_get_tuning(b._h, ctypes.byref(t)))
    return t.block_x, t.rows_per_block


def lb_batch_set_schedule(b, schedule, spin_limit=0):
    """STEPWISE (one launch per step) or PERSISTENT (one launch per window of
    steps with per-tile dependencies); spin_limit 0 = the default poll limit."""
    _check(load_library().lb_batch_set_schedule(b._h, int(schedule), int(spin_limit)))


def lb_batch_get_schedule(b):
    s = ctypes.c_int32()
    _check(load_library().lb_batch_get_schedule(b._h, ctypes.byref(s)))
    return s.value


def lb_batch_free(b):
    b.close()
