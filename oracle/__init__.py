"""CPU oracle of the two-belt pseudopotential lattice Boltzmann step (FP64).

TEST INFRASTRUCTURE ONLY.  Tests, the smoke check and the benchmark's CPU-baseline leg may
import this package; the product path (the HIP library and its binding) must not, and this
package imports nothing from it.  The compiled part is ``lb_oracle.cpp`` (plain loops, one
stage at a time); this module compiles it with g++ and wraps it with ctypes.
"""

import ctypes
import os
import subprocess
from dataclasses import dataclass, field
from typing import Sequence

import numpy as np

from . import weights as _weights

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lb_oracle.cpp")
_LIB = os.path.join(_HERE, "liblb_oracle.so")
_SRC3 = os.path.join(_HERE, "lb_oracle3d.cpp")
_LIB3 = os.path.join(_HERE, "liblb_oracle3d.so")
# LB_ORACLE_LIB_DIR: load prebuilt oracle libraries from that directory instead (the sanitizer
# run builds instrumented copies there)
_ALT = os.environ.get("LB_ORACLE_LIB_DIR")
if _ALT:
    _LIB = os.path.join(_ALT, "liblb_oracle.so")
    _LIB3 = os.path.join(_ALT, "liblb_oracle3d.so")
# Plain FP64: no contraction of a*b+c into fma, no fast-math reassociation.
_CXXFLAGS = ["-O2", "-std=c++17", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-fno-fast-math"]

_lib = None


def build(force=True):
    """Compile the oracle shared libraries (2-D and 3-D) with g++ (called by the build entry
    point)."""
    for src, lib in ((_SRC, _LIB), (_SRC3, _LIB3)):
        if force or not os.path.exists(lib):
            tmp = lib + ".tmp"
            subprocess.run(["g++", *_CXXFLAGS, src, "-o", tmp], check=True)
            os.replace(tmp, lib)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not _ALT and (not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC)):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    vp, dp, ip = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int
    lib.orc_create.restype = vp
    lib.orc_create.argtypes = [ctypes.POINTER(OrcConfig)]
    lib.orc_destroy.argtypes = [vp]
    lib.orc_set_threads.argtypes = [ip]
    lib.orc_get_threads.restype = ip
    lib.orc_init_rest.argtypes = [vp, dp]
    lib.orc_set_f.argtypes = [vp, dp]
    lib.orc_get_f.argtypes = [vp, dp]
    lib.orc_time.argtypes = [vp]
    lib.orc_time.restype = ctypes.c_int64
    lib.orc_step.argtypes = [vp, ip, dp]
    lib.orc_fields.argtypes = [vp, dp, dp, dp, dp, dp, dp]
    lib.orc_cs_grad.argtypes = [ctypes.POINTER(OrcConfig), dp, ip, dp, ip, ctypes.c_double, dp, dp]
    _lib = lib
    return lib


class OrcConfig(ctypes.Structure):
    _fields_ = [
        ("lx", ctypes.c_int32), ("ly", ctypes.c_int32), ("ns", ctypes.c_int32), ("walls", ctypes.c_int32),
        ("g1", ctypes.c_double * 2), ("g2", ctypes.c_double * 2), ("gab", ctypes.c_double),
        ("w", ctypes.c_double * 5), ("p", ctypes.c_double * 5), ("t", ctypes.c_double * 2),
        ("body", ctypes.c_double * 2), ("rho_wall", ctypes.c_double * 2), ("tau", ctypes.c_double * 2),
        ("psi0", ctypes.c_double), ("rho0", ctypes.c_double),
        ("cross_psi", ctypes.c_int32), ("pad_", ctypes.c_int32), ("u_wall", ctypes.c_double * 2),
    ]


def default_w():
    return _weights.as_float_list(_weights.weights_w())


def default_p():
    return _weights.as_float_list(_weights.weights_p())


def default_t():
    t = _weights.weights_t()
    return [float(t[1]), float(t[2])]


@dataclass
class Params:
    """Physical parameters of one simulation (lattice units)."""
    lx: int
    ly: int
    ns: int = 1
    walls: int = 0
    g1: Sequence[float] = (0.0, 0.0)
    g2: Sequence[float] = (0.0, 0.0)
    gab: float = 0.0
    body: Sequence[float] = (0.0, 0.0)
    rho_wall: Sequence[float] = (0.0, 0.0)
    tau: Sequence[float] = (1.0, 1.0)
    psi0: float = 1.0
    rho0: float = 1.0
    w: Sequence[float] = field(default_factory=default_w)
    p: Sequence[float] = field(default_factory=default_p)
    t: Sequence[float] = field(default_factory=default_t)
    cross_psi: int = 0
    u_wall: Sequence[float] = (0.0, 0.0)

    def to_c(self):
        c = OrcConfig()
        c.lx, c.ly, c.ns, c.walls = self.lx, self.ly, self.ns, self.walls
        for k in range(2):
            c.g1[k], c.g2[k] = self.g1[k], self.g2[k]
            c.body[k], c.rho_wall[k], c.tau[k] = self.body[k], self.rho_wall[k], self.tau[k]
        c.gab = self.gab
        for q in range(5):
            c.w[q], c.p[q] = self.w[q], self.p[q]
        c.t[0], c.t[1] = self.t[0], self.t[1]
        c.psi0, c.rho0 = self.psi0, self.rho0
        c.cross_psi = self.cross_psi
        c.u_wall[0], c.u_wall[1] = self.u_wall[0], self.u_wall[1]
        return c

    def shell_k(self, s=0):
        """Folded per-shell coupling K(q) = G1 w(q) + G2 p(q) for species s."""
        return [self.g1[s] * self.w[q] + self.g2[s] * self.p[q] for q in range(5)]


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def set_threads(n):
    _load().orc_set_threads(int(n))


def get_threads():
    return _load().orc_get_threads()


class Oracle:
    """One simulation on the CPU; state = pre-collision populations f[s][l][y][x]."""

    def __init__(self, params: Params, rho_init=None, f=None):
        self.params = params
        self._lib = _load()
        self._cfg = params.to_c()
        self._h = self._lib.orc_create(ctypes.byref(self._cfg))
        self.shape = (params.ns, 9, params.ly, params.lx)
        if f is not None:
            self.set_f(f)
        elif rho_init is not None:
            r = np.ascontiguousarray(np.broadcast_to(rho_init, (params.ns, params.ly, params.lx)), dtype=np.float64)
            self._lib.orc_init_rest(self._h, _dp(r))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.orc_destroy(h)
            self._h = None

    @property
    def time(self):
        return self._lib.orc_time(self._h)

    def set_f(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(self.shape)
        self._lib.orc_set_f(self._h, _dp(f))

    def get_f(self):
        out = np.empty(self.shape, dtype=np.float64)
        self._lib.orc_get_f(self._h, _dp(out))
        return out

    def step(self, n=1, record=False):
        """Advance n steps; with record=True return the (n, 8) per-step observables
        [mass_0, mass_1, P_x, P_y, W_bot, W_top, Q, 0]."""
        if record:
            rec = np.zeros((n, 8), dtype=np.float64)
            self._lib.orc_step(self._h, int(n), _dp(rec))
            return rec
        self._lib.orc_step(self._h, int(n), None)
        return None

    def fields(self, fstar=False):
        """rho [ns,ly,lx], psi [ns,ly,lx], force [ns,2,ly,lx], u [2,ly,lx], j [ns,2,ly,lx],
        and optionally the post-collision populations of the current step."""
        P = self.params
        rho = np.empty((P.ns, P.ly, P.lx))
        psi = np.empty_like(rho)
        force = np.empty((P.ns, 2, P.ly, P.lx))
        u = np.empty((2, P.ly, P.lx))
        j = np.empty_like(force)
        fs = np.empty(self.shape) if fstar else None
        self._lib.orc_fields(self._h, _dp(rho), _dp(psi), _dp(force), _dp(u), _dp(j),
                             _dp(fs) if fstar else None)
        out = dict(rho=rho, psi=psi, force=force, u=u, j=j)
        if fstar:
            out["fstar"] = fs
        return out


def cs_grad(params: Params, f0, nsteps, loss_weights, param, h=1e-30):
    """Complex-step dL/dtheta of L = lw0 <(W_bot+W_top)/2> + lw1 <Q> over nsteps steps.
    param: 0 G1, 1 G2, 2 G_AB, 3 g_x.  Returns (L, dL/dtheta)."""
    lib = _load()
    cfg = params.to_c()
    f0 = np.ascontiguousarray(f0, dtype=np.float64)
    lw = np.ascontiguousarray(loss_weights, dtype=np.float64)
    loss = ctypes.c_double()
    dloss = ctypes.c_double()
    lib.orc_cs_grad(ctypes.byref(cfg), _dp(f0), int(nsteps), _dp(lw), int(param), float(h),
                    ctypes.byref(loss), ctypes.byref(dloss))
    return loss.value, dloss.value


# D2Q9 tables of the oracle, exposed for the diagnostics (same values as in lb_oracle.cpp).
CX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
CY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])
WL = np.array([4 / 9, 1 / 9, 1 / 9, 1 / 9, 1 / 9, 1 / 36, 1 / 36, 1 / 36, 1 / 36])


# ----------------------------------------------------------------------------------------
# Three dimensions (D3Q19; lb_oracle3d.cpp)
# ----------------------------------------------------------------------------------------

_lib3 = None


def _load3():
    global _lib3
    if _lib3 is not None:
        return _lib3
    if not _ALT and (not os.path.exists(_LIB3) or os.path.getmtime(_LIB3) < os.path.getmtime(_SRC3)):
        build(force=True)
    lib = ctypes.CDLL(_LIB3)
    vp, dp, ip = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int
    lib.orc3_create.restype = vp
    lib.orc3_create.argtypes = [ctypes.POINTER(Orc3Config)]
    lib.orc3_destroy.argtypes = [vp]
    lib.orc3_init_rest.argtypes = [vp, dp]
    lib.orc3_set_f.argtypes = [vp, dp]
    lib.orc3_get_f.argtypes = [vp, dp]
    lib.orc3_time.argtypes = [vp]
    lib.orc3_time.restype = ctypes.c_int64
    lib.orc3_nlinks.argtypes = [vp]
    lib.orc3_nlinks.restype = ip
    lib.orc3_step.argtypes = [vp, ip, dp]
    lib.orc3_fields.argtypes = [vp, dp, dp, dp, dp, dp]
    _lib3 = lib
    return lib


class Orc3Config(ctypes.Structure):
    _fields_ = [
        ("lx", ctypes.c_int32), ("ly", ctypes.c_int32), ("lz", ctypes.c_int32), ("ns", ctypes.c_int32),
        ("walls", ctypes.c_int32), ("cross_psi", ctypes.c_int32),
        ("g1", ctypes.c_double * 2), ("g2", ctypes.c_double * 2), ("gab", ctypes.c_double),
        ("w", ctypes.c_double * 7), ("p", ctypes.c_double * 7), ("t", ctypes.c_double * 2),
        ("body", ctypes.c_double * 3), ("rho_wall", ctypes.c_double * 2), ("tau", ctypes.c_double * 2),
        ("psi0", ctypes.c_double), ("rho0", ctypes.c_double),
    ]


def default_w3():
    return _weights.as_float_list3(_weights.weights3_w())


def default_p3():
    return _weights.as_float_list3(_weights.weights3_p())


def default_t3():
    t = _weights.weights3_t()
    return [float(t[1]), float(t[2])]


@dataclass
class Params3:
    """Parameters of one 3-D simulation (lattice units); walls bound y as in two dimensions."""
    lx: int
    ly: int
    lz: int
    ns: int = 1
    walls: int = 0
    g1: Sequence[float] = (0.0, 0.0)
    g2: Sequence[float] = (0.0, 0.0)
    gab: float = 0.0
    body: Sequence[float] = (0.0, 0.0, 0.0)
    rho_wall: Sequence[float] = (0.0, 0.0)
    tau: Sequence[float] = (1.0, 1.0)
    psi0: float = 1.0
    rho0: float = 1.0
    w: Sequence[float] = field(default_factory=default_w3)
    p: Sequence[float] = field(default_factory=default_p3)
    t: Sequence[float] = field(default_factory=default_t3)
    cross_psi: int = 0

    def to_c(self):
        c = Orc3Config()
        c.lx, c.ly, c.lz, c.ns, c.walls, c.cross_psi = self.lx, self.ly, self.lz, self.ns, self.walls, self.cross_psi
        for k in range(2):
            c.g1[k], c.g2[k] = self.g1[k], self.g2[k]
            c.rho_wall[k], c.tau[k] = self.rho_wall[k], self.tau[k]
        for k in range(3):
            c.body[k] = self.body[k]
        c.gab = self.gab
        for q in range(7):
            c.w[q], c.p[q] = self.w[q], self.p[q]
        c.t[0], c.t[1] = self.t[0], self.t[1]
        c.psi0, c.rho0 = self.psi0, self.rho0
        return c

    def shell_k(self, s=0):
        """K(q) = G1 w(q) + G2 p(q) for species s, q in (1, 2, 3, 4, 5, 6, 8)."""
        return [self.g1[s] * self.w[q] + self.g2[s] * self.p[q] for q in range(7)]


class Oracle3:
    """One 3-D simulation on the CPU; state = pre-collision populations f[s][l][z][y][x]."""

    def __init__(self, params: Params3, rho_init=None, f=None):
        self.params = params
        self._lib = _load3()
        self._cfg = params.to_c()
        self._h = self._lib.orc3_create(ctypes.byref(self._cfg))
        self.shape = (params.ns, 19, params.lz, params.ly, params.lx)
        if f is not None:
            self.set_f(f)
        elif rho_init is not None:
            r = np.ascontiguousarray(np.broadcast_to(rho_init, (params.ns, params.lz, params.ly, params.lx)),
                                     dtype=np.float64)
            self._lib.orc3_init_rest(self._h, _dp(r))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.orc3_destroy(h)
            self._h = None

    @property
    def time(self):
        return self._lib.orc3_time(self._h)

    @property
    def nlinks(self):
        return self._lib.orc3_nlinks(self._h)

    def set_f(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(self.shape)
        self._lib.orc3_set_f(self._h, _dp(f))

    def get_f(self):
        out = np.empty(self.shape, dtype=np.float64)
        self._lib.orc3_get_f(self._h, _dp(out))
        return out

    def step(self, n=1, record=False):
        """Advance n steps; with record=True return the (n, 8) per-step observables
        [mass_0, mass_1, P_x, P_y, P_z, W_bot, W_top, Q]."""
        if record:
            rec = np.zeros((n, 8), dtype=np.float64)
            self._lib.orc3_step(self._h, int(n), _dp(rec))
            return rec
        self._lib.orc3_step(self._h, int(n), None)
        return None

    def fields(self):
        """rho, psi [ns,lz,ly,lx]; force, j [ns,3,lz,ly,lx]; u [3,lz,ly,lx]."""
        P = self.params
        rho = np.empty((P.ns, P.lz, P.ly, P.lx))
        psi = np.empty_like(rho)
        force = np.empty((P.ns, 3, P.lz, P.ly, P.lx))
        u = np.empty((3, P.lz, P.ly, P.lx))
        j = np.empty_like(force)
        self._lib.orc3_fields(self._h, _dp(rho), _dp(psi), _dp(force), _dp(u), _dp(j))
        return dict(rho=rho, psi=psi, force=force, u=u, j=j)


# D3Q19 tables of the 3-D oracle (same values and order as in lb_oracle3d.cpp).
CX3 = np.array([0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0])
CY3 = np.array([0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1])
CZ3 = np.array([0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1])
WL3 = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
