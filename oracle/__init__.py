"""FP64 CPU oracle of the binary free-energy lattice Boltzmann method of Pooley,
Kusumaatmaja and Yeomans (arXiv:0812.1282).

TEST INFRASTRUCTURE: only the tests, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package. The product
path (the HIP library and its binding) never does, and shares no code with it.

The stepping is C (``lbm_oracle.c``, built by ``oracle/build.py``); this module
is the ctypes marshalling around it. The measurement routines (contact angle,
closed forms) are in ``oracle/analysis.py``.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

BGK, MRT = 0, 1


class OrcParams(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("A", ctypes.c_double), ("B", ctypes.c_double),
                ("kappa", ctypes.c_double), ("Gamma", ctypes.c_double),
                ("tau_alpha", ctypes.c_double), ("tau_beta", ctypes.c_double),
                ("tau_phi", ctypes.c_double),
                ("collision", ctypes.c_int32),
                ("zero_u_feq", ctypes.c_int32), ("zero_u_geq", ctypes.c_int32),
                ("tau_clamp", ctypes.c_int32), ("tau_lut", ctypes.c_int32),
                ("bounce", ctypes.c_int32)]


_D = ctypes.POINTER(ctypes.c_double)
_U8 = ctypes.POINTER(ctypes.c_uint8)
_I32 = ctypes.POINTER(ctypes.c_int32)


def lib():
    """Load liboracle.so, building it first if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _build
        _build.build()
    L = ctypes.CDLL(_LIB_PATH)
    P = ctypes.POINTER(OrcParams)
    L.orc_create.restype = ctypes.c_void_p
    L.orc_create.argtypes = [P, _U8, _D, _D, _D, _D, _D]
    L.orc_free.argtypes = [ctypes.c_void_p]
    L.orc_step.argtypes = [ctypes.c_void_p, ctypes.c_int64]
    L.orc_step_count.restype = ctypes.c_int64
    L.orc_step_count.argtypes = [ctypes.c_void_p]
    L.orc_set_wall_dphi.argtypes = [ctypes.c_void_p, _D]
    L.orc_fields.argtypes = [ctypes.c_void_p, _D, _D, _D, _D]
    L.orc_get_populations.argtypes = [ctypes.c_void_p, _D, _D]
    L.orc_set_populations.argtypes = [ctypes.c_void_p, _D, _D]
    L.orc_diagnostics.argtypes = [ctypes.c_void_p, _D]
    L.orc_lattice.argtypes = [_I32, _I32, _D, _D, _D, _D]
    L.orc_mrt_matrices.argtypes = [_D, _D]
    L.orc_moments.argtypes = [ctypes.c_int32, ctypes.c_int32, _U8, _D, _D, _D, _D, _D, _D]
    L.orc_ghosts.argtypes = [ctypes.c_int32, ctypes.c_int32, _U8, _D, _D, _D]
    L.orc_gradients.argtypes = [ctypes.c_int32, ctypes.c_int32, _U8, _D, _D, _D, _D]
    L.orc_equilibria_node.argtypes = [P] + [ctypes.c_double] * 9 + [_D, _D]
    L.orc_collide_node.argtypes = [P, ctypes.c_double, _D, _D, _D, _D, _D, _D]
    L.orc_stream.argtypes = [ctypes.c_int32, ctypes.c_int32, _U8, _D, _D]
    L.orc_stream_lattice_node.argtypes = [ctypes.c_int32, ctypes.c_int32, _U8, _D, _D]
    L.orc_reflect_walls.argtypes = [ctypes.c_int32, ctypes.c_int32, _U8, _D, _D]
    L.orc_tau.restype = ctypes.c_double
    L.orc_tau.argtypes = [P, ctypes.c_double]
    L.orc_set_threads.argtypes = [ctypes.c_int32]
    L.orc_get_threads.restype = ctypes.c_int32
    _lib = L
    return L


def _dp(a):
    return None if a is None else a.ctypes.data_as(_D)


def _f64(a, shape=None):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None and a.shape != shape:
        a = a.reshape(shape)
    return a


def make_params(nx, ny, A=-0.04, B=0.04, kappa=0.04, Gamma=0.1, tau_alpha=1.0,
                tau_beta=1.0, tau_phi=1.0, collision=BGK, zero_u_feq=None,
                zero_u_geq=0, tau_clamp=0, tau_lut=0, bounce=0):
    """Oracle parameters; Step 2 defaults to on for MRT and off for BGK.
    tau_lut >= 2: tau from the table of Sec. VI; bounce = 1: lattice-node
    bounce-back (Fig. 9b)."""
    if zero_u_feq is None:
        zero_u_feq = 1 if collision == MRT else 0
    return OrcParams(nx, ny, A, B, kappa, Gamma, tau_alpha, tau_beta, tau_phi,
                     collision, zero_u_feq, zero_u_geq, tau_clamp, tau_lut, bounce)


class Oracle:
    """One lattice advanced by the FP64 oracle.

    State S_n is the post-streaming population set (f, g), shape (9, ny, nx).
    """

    def __init__(self, params: OrcParams, solid, phi0, dphi=None, rho0=None,
                 ux0=None, uy0=None):
        L = lib()
        self.params = params
        nx, ny = params.nx, params.ny
        self.shape = (ny, nx)
        self.solid = np.ascontiguousarray(solid, dtype=np.uint8).reshape(self.shape)
        args = [_f64(a, self.shape) for a in (dphi, phi0, rho0, ux0, uy0)]
        self._keep = args
        h = L.orc_create(ctypes.byref(params), self.solid.ctypes.data_as(_U8),
                         *[_dp(a) for a in args])
        if not h:
            raise ValueError("oracle rejected the parameters or inputs")
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_free(h)
            self._h = None

    def step(self, n=1):
        lib().orc_step(self._h, int(n))

    @property
    def step_count(self):
        return int(lib().orc_step_count(self._h))

    def set_wall_dphi(self, dphi):
        d = _f64(dphi, self.shape)
        lib().orc_set_wall_dphi(self._h, _dp(d))

    def fields(self):
        """(phi, rho, ux, uy) of S_n, each (ny, nx); zero at solid nodes."""
        out = [np.zeros(self.shape) for _ in range(4)]
        lib().orc_fields(self._h, *[_dp(a) for a in out])
        return tuple(out)

    def populations(self):
        ny, nx = self.shape
        f = np.zeros((9, ny, nx))
        g = np.zeros((9, ny, nx))
        lib().orc_get_populations(self._h, _dp(f), _dp(g))
        return f, g

    def set_populations(self, f, g):
        ny, nx = self.shape
        f = _f64(f, (9, ny, nx))
        g = _f64(g, (9, ny, nx))
        lib().orc_set_populations(self._h, _dp(f), _dp(g))

    def diagnostics(self):
        out = np.zeros(5)
        lib().orc_diagnostics(self._h, _dp(out))
        return {"sum_rho": out[0], "sum_phi": out[1], "kinetic": out[2],
                "max_u": out[3], "n_fluid": int(out[4])}


# ---- the individual steps, for the pins ----

def lattice():
    ex = np.zeros(9, dtype=np.int32)
    ey = np.zeros(9, dtype=np.int32)
    w, wxx, wyy, wxy = (np.zeros(9) for _ in range(4))
    lib().orc_lattice(ex.ctypes.data_as(_I32), ey.ctypes.data_as(_I32),
                      _dp(w), _dp(wxx), _dp(wyy), _dp(wxy))
    return ex, ey, w, wxx, wyy, wxy


def mrt_matrices():
    M = np.zeros((9, 9))
    Minv = np.zeros((9, 9))
    lib().orc_mrt_matrices(_dp(M), _dp(Minv))
    return M, Minv


def moments(solid, f, g):
    ny, nx = solid.shape
    solid = np.ascontiguousarray(solid, dtype=np.uint8)
    f = _f64(f, (9, ny, nx))
    g = _f64(g, (9, ny, nx))
    out = [np.zeros((ny, nx)) for _ in range(4)]
    lib().orc_moments(nx, ny, solid.ctypes.data_as(_U8), _dp(f), _dp(g),
                      *[_dp(a) for a in out])
    return tuple(out)  # rho, phi, ux, uy


def ghosts(solid, dphi, phi):
    ny, nx = solid.shape
    solid = np.ascontiguousarray(solid, dtype=np.uint8)
    dphi = _f64(dphi, (ny, nx))
    phi = _f64(phi, (ny, nx))
    out = np.zeros((ny, nx))
    lib().orc_ghosts(nx, ny, solid.ctypes.data_as(_U8), _dp(dphi), _dp(phi), _dp(out))
    return out


def gradients(phix, solid=None):
    ny, nx = phix.shape
    phix = _f64(phix)
    s = None if solid is None else np.ascontiguousarray(solid, dtype=np.uint8)
    out = [np.zeros((ny, nx)) for _ in range(3)]
    lib().orc_gradients(nx, ny, None if s is None else s.ctypes.data_as(_U8),
                        _dp(phix), *[_dp(a) for a in out])
    return tuple(out)  # dx, dy, lap


def equilibria_node(params, rho, phi, ux, uy, dxphi, dyphi, lapphi, ux_f=None, uy_f=None):
    feq = np.zeros(9)
    geq = np.zeros(9)
    ux_f = ux if ux_f is None else ux_f
    uy_f = uy if uy_f is None else uy_f
    lib().orc_equilibria_node(ctypes.byref(params), rho, phi, ux, uy, ux_f, uy_f,
                              dxphi, dyphi, lapphi, _dp(feq), _dp(geq))
    return feq, geq


def collide_node(params, phi, f, feq, g, geq):
    fo = np.zeros(9)
    go = np.zeros(9)
    args = [_f64(a) for a in (f, feq, g, geq)]
    lib().orc_collide_node(ctypes.byref(params), phi, *[_dp(a) for a in args],
                           _dp(fo), _dp(go))
    return fo, go


def stream(solid, post):
    ny, nx = solid.shape
    solid = np.ascontiguousarray(solid, dtype=np.uint8)
    post = _f64(post, (9, ny, nx))
    nxt = np.zeros((9, ny, nx))
    lib().orc_stream(nx, ny, solid.ctypes.data_as(_U8), _dp(post), _dp(nxt))
    return nxt


def stream_lattice_node(solid, post):
    """Lattice-node streaming (Fig. 9b) of a (9, ny, nx) post-collision set."""
    solid = np.ascontiguousarray(solid, dtype=np.uint8)
    ny, nx = solid.shape
    post = _f64(post)
    out = np.zeros_like(post)
    lib().orc_stream_lattice_node(nx, ny, solid.ctypes.data_as(_U8), _dp(post), _dp(out))
    return out


def reflect_walls(solid, pre, post=None):
    """Wall nodes' reversal (Fig. 9b): post_i = pre_opp(i) at every wall node;
    other nodes keep the values of post (zeros if None)."""
    solid = np.ascontiguousarray(solid, dtype=np.uint8)
    ny, nx = solid.shape
    pre = _f64(pre)
    out = np.zeros_like(pre) if post is None else np.array(post, dtype=np.float64)
    lib().orc_reflect_walls(nx, ny, solid.ctypes.data_as(_U8), _dp(pre), _dp(out))
    return out


def tau(params, phi):
    return lib().orc_tau(ctypes.byref(params), phi)


def set_threads(n):
    lib().orc_set_threads(int(n))


def get_threads():
    return int(lib().orc_get_threads())
