"""ctypes wrapper of the plain FP64 CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY: tests/, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may use it; the product package never
imports it. Arrays use the oracle's own layout: ghosted fields are
``float64[nv, nz+2g, ny+2g, nx+2g]`` (x fastest), interior fields are
``float64[5, nz, ny, nx]``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

BC_PERIODIC, BC_WALL, BC_EXTRAP, BC_FROZEN = 0, 1, 2, 3
Y_UNIFORM, Y_TANH2, Y_TANH1 = 0, 1, 2
CONV_X, CONV_Y, CONV_Z, VISC, ALL = 1, 2, 4, 8, 15
NDIAG = 16


def build(force: bool = True) -> str:
    """Compile the oracle with strict IEEE semantics (no contraction)."""
    if force or not os.path.exists(_LIB):
        subprocess.check_call([
            "gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
            "-shared", "-fPIC", _SRC, "-o", _LIB, "-lm"])
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("lx", ctypes.c_double), ("ly", ctypes.c_double), ("lz", ctypes.c_double),
        ("y0", ctypes.c_double),
        ("ymap", ctypes.c_int), ("beta", ctypes.c_double),
        ("bc", ctypes.c_int * 6),
        ("gamma", ctypes.c_double), ("mach", ctypes.c_double),
        ("reynolds", ctypes.c_double), ("prandtl", ctypes.c_double),
        ("visc_exp", ctypes.c_double), ("t_wall", ctypes.c_double),
        ("central_order", ctypes.c_int), ("weno_order", ctypes.c_int),
        ("visc_order", ctypes.c_int),
        ("sensor", ctypes.c_int), ("sensor_thr", ctypes.c_double),
        ("sensor_eps", ctypes.c_double), ("weno_eps", ctypes.c_double),
        ("central_flux", ctypes.c_int), ("keep_n", ctypes.c_int),
        ("bulk_forcing", ctypes.c_int),
        ("thermo", ctypes.c_int), ("nasa", ctypes.c_double * 5), ("t_ref", ctypes.c_double),
    ]


@dataclass
class Params:
    nx: int
    ny: int
    nz: int
    lx: float
    ly: float
    lz: float
    y0: float = 0.0
    ymap: int = Y_UNIFORM
    beta: float = 0.0
    bc: tuple = (BC_PERIODIC,) * 6
    gamma: float = 1.4
    mach: float = 0.1
    reynolds: float = 1600.0
    prandtl: float = 0.72
    visc_exp: float = 0.76
    t_wall: float = 1.0
    central_order: int = 6
    weno_order: int = 5
    visc_order: int = 6
    sensor: int = 0
    sensor_thr: float = 0.5
    sensor_eps: float = 1.0
    weno_eps: float = 1e-6
    central_flux: int = 0      # 0 split form, 1 KEEP-n
    keep_n: int = 0            # KEEP-n series terms beyond the first (< 0: exact log means)
    bulk_forcing: int = 0      # 1: uniform streamwise force holding the bulk momentum
    thermo: int = 0            # 1: thermally perfect gas, c_p/R = sum_k nasa[k] (T t_ref)^k
    nasa: tuple = (3.5, 0.0, 0.0, 0.0, 0.0)
    t_ref: float = 300.0       # kelvin at T = 1

    def c(self) -> _Params:
        p = _Params()
        for name, _ in _Params._fields_:
            if name == "bc":
                p.bc[:] = list(self.bc)
            elif name == "nasa":
                p.nasa[:] = [float(x) for x in self.nasa]
            else:
                setattr(p, name, getattr(self, name))
        return p


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER(_Params)
        dp = ctypes.POINTER(ctypes.c_double)
        up = ctypes.POINTER(ctypes.c_ubyte)
        ip = ctypes.POINTER(ctypes.c_int)
        L.orc_validate.argtypes = [P]
        L.orc_ng.argtypes = [P]
        L.orc_y_nodes.argtypes = [P, ctypes.c_int, ctypes.c_int, dp]
        L.orc_metrics.argtypes = [P, dp, dp]
        L.orc_fill_ghosts.argtypes = [P, dp]
        L.orc_primitives.argtypes = [P, dp, dp]
        L.orc_theta.argtypes = [P, dp, dp]
        L.orc_face_flags.argtypes = [P, dp, up, up, up]
        L.orc_rhs.argtypes = [P, dp, dp, ctypes.c_uint, up, up, up]
        L.orc_rhs_points.argtypes = [P, dp, ctypes.c_int, ip, dp, ctypes.c_uint]
        L.orc_rk3_step.argtypes = [P, dp, dp, ctypes.c_double]
        L.orc_compute_dt.argtypes = [P, dp, ctypes.c_double]
        L.orc_compute_dt.restype = ctypes.c_double
        L.orc_diagnostics.argtypes = [P, dp, dp, dp]
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_set_num_threads.argtypes = [ctypes.c_int]
        L.orc_thermo_eval.argtypes = [P, ctypes.c_double, dp]
        L.orc_thermo_T.argtypes = [P, ctypes.c_double]
        L.orc_thermo_T.restype = ctypes.c_double
        L.orc_fd_coeffs.argtypes = [ctypes.c_int, dp, dp]
        L.orc_weno_left.argtypes = [ctypes.c_int, ctypes.c_double, dp]
        L.orc_weno_left.restype = ctypes.c_double
        L.orc_weno_smoothness.argtypes = [ctypes.c_int, dp, dp]
        L.orc_char_basis.argtypes = [ctypes.c_double] * 5 + [dp, dp]
        L.orc_face_flux_1d.argtypes = [ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_double, ctypes.c_int, dp, dp]
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"], (a.dtype, a.flags)
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _up(a):
    if a is None:
        return None
    assert a.dtype == np.uint8 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte))


class Oracle:
    """Stateless wrapper bound to one parameter set."""

    def __init__(self, params: Params):
        self.params = params
        self._c = params.c()
        rc = lib().orc_validate(ctypes.byref(self._c))
        if rc != 0:
            raise ValueError(f"oracle rejects parameters (code {rc})")
        self.ng = lib().orc_ng(ctypes.byref(self._c))
        g = self.ng
        self.ghosted_shape = (params.nz + 2 * g, params.ny + 2 * g, params.nx + 2 * g)
        self.interior_shape = (params.nz, params.ny, params.nx)

    # -- shapes / helpers -------------------------------------------------
    def empty_state(self) -> np.ndarray:
        return np.zeros((5,) + self.ghosted_shape)

    def interior(self, W: np.ndarray) -> np.ndarray:
        g = self.ng
        return W[:, g:W.shape[1] - g, g:W.shape[2] - g, g:W.shape[3] - g]

    def y_nodes(self, jlo: int, jhi: int) -> np.ndarray:
        y = np.zeros(jhi - jlo)
        lib().orc_y_nodes(ctypes.byref(self._c), jlo, jhi, _dp(y))
        return y

    def metrics(self):
        ye = np.zeros(self.params.ny)
        yee = np.zeros(self.params.ny)
        lib().orc_metrics(ctypes.byref(self._c), _dp(ye), _dp(yee))
        return ye, yee

    # -- solver pieces ----------------------------------------------------
    def fill_ghosts(self, W: np.ndarray) -> None:
        lib().orc_fill_ghosts(ctypes.byref(self._c), _dp(W))

    def primitives(self, W: np.ndarray) -> np.ndarray:
        Q = np.zeros((7,) + self.ghosted_shape)
        lib().orc_primitives(ctypes.byref(self._c), _dp(W), _dp(Q))
        return Q

    def theta(self, W: np.ndarray) -> np.ndarray:
        th = np.zeros(self.ghosted_shape)
        self.fill_ghosts(W)
        lib().orc_theta(ctypes.byref(self._c), _dp(W), _dp(th))
        return th

    def face_flags(self, W: np.ndarray):
        p = self.params
        th = self.theta(W)
        fx = np.zeros((p.nz, p.ny, p.nx + 1), np.uint8)
        fy = np.zeros((p.nz, p.ny + 1, p.nx), np.uint8)
        fz = np.zeros((p.nz + 1, p.ny, p.nx), np.uint8)
        lib().orc_face_flags(ctypes.byref(self._c), _dp(th), _up(fx), _up(fy), _up(fz))
        return fx, fy, fz

    def face_flags_from_theta(self, theta: np.ndarray):
        """Face flags of a given ghosted sensor field (the hybrid switch
        alone, without the sensor evaluation)."""
        p = self.params
        theta = np.ascontiguousarray(theta, dtype=np.float64)
        assert theta.shape == self.ghosted_shape
        fx = np.zeros((p.nz, p.ny, p.nx + 1), np.uint8)
        fy = np.zeros((p.nz, p.ny + 1, p.nx), np.uint8)
        fz = np.zeros((p.nz + 1, p.ny, p.nx), np.uint8)
        lib().orc_face_flags(ctypes.byref(self._c), _dp(theta), _up(fx), _up(fy), _up(fz))
        return fx, fy, fz

    def rhs(self, W: np.ndarray, mask: int = ALL, flags=None) -> np.ndarray:
        R = np.zeros((5,) + self.interior_shape)
        fx = fy = fz = None
        if flags is not None:
            fx, fy, fz = (np.ascontiguousarray(f, dtype=np.uint8) for f in flags)
        lib().orc_rhs(ctypes.byref(self._c), _dp(W), _dp(R), mask, _up(fx), _up(fy), _up(fz))
        return R

    def rhs_points(self, W: np.ndarray, ijk: np.ndarray, mask: int = ALL) -> np.ndarray:
        ijk = np.ascontiguousarray(ijk, dtype=np.int32)
        out = np.zeros((ijk.shape[0], 5))
        lib().orc_rhs_points(ctypes.byref(self._c), _dp(W), ijk.shape[0],
                             ijk.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _dp(out), mask)
        return out

    def rk3_step(self, W: np.ndarray, Rprev: np.ndarray, dt: float) -> None:
        lib().orc_rk3_step(ctypes.byref(self._c), _dp(W), _dp(Rprev), dt)

    def compute_dt(self, W: np.ndarray, cfl: float) -> float:
        return lib().orc_compute_dt(ctypes.byref(self._c), _dp(W), cfl)

    def thermo_eval(self, T: float):
        """(c_p, c_v, e, dc_p/dT) of the gas at temperature T."""
        out = np.zeros(4)
        lib().orc_thermo_eval(ctypes.byref(self._c), float(T), _dp(out))
        return out

    def thermo_T(self, e: float) -> float:
        return lib().orc_thermo_T(ctypes.byref(self._c), float(e))

    def diagnostics(self, W: np.ndarray, R: np.ndarray | None = None) -> np.ndarray:
        out = np.zeros(NDIAG)
        lib().orc_diagnostics(ctypes.byref(self._c), _dp(W), None if R is None else _dp(R), _dp(out))
        return out


# -- 1-D building blocks ----------------------------------------------------
def fd_coeffs(order: int):
    a = np.zeros(5)
    b = np.zeros(5)
    lib().orc_fd_coeffs(order, _dp(a), _dp(b))
    return a, b


def weno_left(order: int, eps: float, v) -> float:
    v = np.ascontiguousarray(v, dtype=np.float64)
    return lib().orc_weno_left(order, eps, _dp(v))


def weno_smoothness(order: int, v) -> np.ndarray:
    v = np.ascontiguousarray(v, dtype=np.float64)
    beta = np.zeros(4)
    lib().orc_weno_smoothness(order, _dp(v), _dp(beta))
    return beta[:(order + 1) // 2]


def char_basis(gamma, un, ut1, ut2, H):
    Rm = np.zeros(25)
    Lm = np.zeros(25)
    lib().orc_char_basis(gamma, un, ut1, ut2, H, _dp(Rm), _dp(Lm))
    return Rm.reshape(5, 5), Lm.reshape(5, 5)


def face_flux_1d(gamma, W8, central_order=6, weno_order=5, weno_eps=1e-6, use_weno=False):
    W8 = np.ascontiguousarray(W8, dtype=np.float64).reshape(8, 5)
    F = np.zeros(5)
    lib().orc_face_flux_1d(gamma, central_order, weno_order, weno_eps, int(use_weno), _dp(W8), _dp(F))
    return F


def num_threads() -> int:
    return lib().orc_num_threads()


def set_num_threads(n: int) -> None:
    """OpenMP thread count of later oracle calls."""
    lib().orc_set_num_threads(int(n))
