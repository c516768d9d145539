"""Thin ctypes binding of the C ABI in include/sx.h (argument marshalling only).

Every step of the hot path runs in the HIP library ``libsx.so``; this module
only converts Python values to C structs and torch tensors to device
pointers. Importing it fails loudly if the library has not been built.
Torch provides device memory and streams.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsx.so")

SX_OK, SX_EINVAL, SX_EUNSUPPORTED, SX_EHIP, SX_ENOMEM, SX_ENONFINITE, SX_ESTATE = range(7)
SX_BC_PERIODIC, SX_BC_WALL, SX_BC_EXTRAP, SX_BC_FROZEN = range(4)
SX_Y_UNIFORM, SX_Y_TANH2, SX_Y_TANH1 = range(3)
SX_CONV_X, SX_CONV_Y, SX_CONV_Z, SX_VISC, SX_ALL = 1, 2, 4, 8, 15
SX_FP64, SX_FP32_FLUX = 0, 1
SX_FLUX_SPLIT, SX_FLUX_KEEP = 0, 1


class SxError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"sx error {code}: {msg}")
        self.code = code


class sx_grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("lx", ctypes.c_double), ("ly", ctypes.c_double), ("lz", ctypes.c_double),
                ("y0", ctypes.c_double), ("ymap", ctypes.c_int), ("beta", ctypes.c_double),
                ("bc", ctypes.c_int * 6)]


class sx_gas(ctypes.Structure):
    _fields_ = [("gamma", ctypes.c_double), ("mach", ctypes.c_double),
                ("reynolds", ctypes.c_double), ("prandtl", ctypes.c_double),
                ("visc_exp", ctypes.c_double), ("t_wall", ctypes.c_double),
                ("thermo", ctypes.c_int), ("nasa", ctypes.c_double * 5), ("t_ref", ctypes.c_double)]


class sx_scheme(ctypes.Structure):
    _fields_ = [("central_order", ctypes.c_int), ("weno_order", ctypes.c_int),
                ("visc_order", ctypes.c_int), ("sensor", ctypes.c_int),
                ("sensor_thr", ctypes.c_double), ("sensor_eps", ctypes.c_double),
                ("weno_eps", ctypes.c_double), ("precision", ctypes.c_int),
                ("central_flux", ctypes.c_int), ("keep_n", ctypes.c_int),
                ("bulk_forcing", ctypes.c_int)]


class sx_layout(ctypes.Structure):
    _fields_ = [("ng", ctypes.c_int), ("ox", ctypes.c_int), ("px", ctypes.c_longlong),
                ("py", ctypes.c_longlong), ("pz", ctypes.c_longlong),
                ("var_stride", ctypes.c_longlong), ("elems", ctypes.c_longlong),
                ("interior", ctypes.c_longlong)]


class sx_diag(ctypes.Structure):
    _fields_ = [("mass", ctypes.c_double), ("momentum", ctypes.c_double * 3),
                ("energy", ctypes.c_double), ("kinetic", ctypes.c_double),
                ("max_mach", ctypes.c_double), ("min_rho", ctypes.c_double),
                ("min_p", ctypes.c_double), ("nonfinite", ctypes.c_double),
                ("nonphysical", ctypes.c_double), ("residual_rhou", ctypes.c_double),
                ("weno_fraction", ctypes.c_double * 3), ("volume", ctypes.c_double)]

    def as_array(self) -> np.ndarray:
        return np.array([self.mass, *self.momentum, self.energy, self.kinetic, self.max_mach,
                         self.min_rho, self.min_p, self.nonfinite, self.nonphysical,
                         self.residual_rhou, *self.weno_fraction, self.volume])


class sx_tiling(ctypes.Structure):
    _fields_ = [("tile_x", ctypes.c_int), ("tile_y", ctypes.c_int), ("zchunk", ctypes.c_int),
                ("workgroups", ctypes.c_int), ("work_items", ctypes.c_int),
                ("ms_per_substep", ctypes.c_double)]


EXPORTS = ["sx_init", "sx_finalize", "sx_get_layout", "sx_bind", "sx_current", "sx_fill_ghosts",
           "sx_rhs", "sx_rk3_step", "sx_compute_dt", "sx_diagnostics", "sx_set_flag_override",
           "sx_get_flags", "sx_diagnostics_noalloc",
           "sx_timing_enable", "sx_timing_read", "sx_init_batch", "sx_get_box", "sx_set_tiling",
           "sx_get_tiling", "sx_autotune", "sx_set_graph", "sx_last_error"]

_lib = None


def load() -> ctypes.CDLL:
    """Load libsx.so (built by paper_2304_05494_amd.build); raise if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"HIP library not built: {LIB_PATH} is missing "
                          "(run python -m paper_2304_05494_amd.build)")
    L = ctypes.CDLL(LIB_PATH)
    H = ctypes.c_void_p
    dp = ctypes.c_void_p
    L.sx_init.argtypes = [ctypes.POINTER(sx_grid), ctypes.POINTER(sx_gas),
                          ctypes.POINTER(sx_scheme), ctypes.POINTER(H)]
    L.sx_finalize.argtypes = [H]
    L.sx_finalize.restype = None
    L.sx_get_layout.argtypes = [H, ctypes.POINTER(sx_layout)]
    L.sx_bind.argtypes = [H, dp, dp, dp, ctypes.c_void_p]
    L.sx_current.argtypes = [H, ctypes.POINTER(ctypes.c_int)]
    L.sx_fill_ghosts.argtypes = [H, dp]
    L.sx_rhs.argtypes = [H, dp, dp, ctypes.c_uint]
    L.sx_rk3_step.argtypes = [H, ctypes.c_double]
    L.sx_compute_dt.argtypes = [H, ctypes.c_double, ctypes.POINTER(ctypes.c_double)]
    L.sx_diagnostics.argtypes = [H, dp, ctypes.POINTER(sx_diag)]
    L.sx_set_flag_override.argtypes = [H, dp, dp, dp]
    L.sx_get_flags.argtypes = [H, dp, dp, dp]
    L.sx_diagnostics_noalloc.argtypes = [H, dp, dp]
    L.sx_timing_enable.argtypes = [H, ctypes.c_int]
    L.sx_timing_read.argtypes = [H, ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(ctypes.c_double)]
    L.sx_init_batch.argtypes = [ctypes.c_int, ctypes.POINTER(sx_grid), ctypes.POINTER(sx_gas),
                                ctypes.POINTER(sx_scheme), ctypes.POINTER(H)]
    L.sx_get_box.argtypes = [H, ctypes.c_int, ctypes.POINTER(sx_layout),
                             ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(ctypes.c_longlong)]
    L.sx_set_tiling.argtypes = [H, ctypes.POINTER(sx_tiling)]
    L.sx_get_tiling.argtypes = [H, ctypes.POINTER(sx_tiling)]
    L.sx_autotune.argtypes = [H, ctypes.c_char_p, ctypes.POINTER(sx_tiling)]
    L.sx_set_graph.argtypes = [H, ctypes.c_int]
    L.sx_last_error.argtypes = [H]
    L.sx_last_error.restype = ctypes.c_char_p
    for name in EXPORTS:
        getattr(L, name)
    _lib = L
    return L


def make_structs(case, precision: int = SX_FP64):
    """Build the three description structs from an input case (plain data)."""
    g = sx_grid(case.nx, case.ny, case.nz, case.lx, case.ly, case.lz, case.y0, case.ymap,
                case.beta)
    g.bc[:] = list(case.bc)
    gas = sx_gas(case.gamma, case.mach, case.reynolds, case.prandtl, case.visc_exp, case.t_wall,
                 getattr(case, "thermo", 0))
    gas.nasa[:] = [float(x) for x in getattr(case, "nasa", (3.5, 0.0, 0.0, 0.0, 0.0))]
    gas.t_ref = float(getattr(case, "t_ref", 300.0))
    sc = sx_scheme(case.central_order, case.weno_order, case.visc_order, case.sensor,
                   case.sensor_thr, case.sensor_eps, case.weno_eps, precision,
                   getattr(case, "central_flux", 0), getattr(case, "keep_n", 0),
                   getattr(case, "bulk_forcing", 0))
    return g, gas, sc


def _ptr(t) -> int:
    return 0 if t is None else int(t.data_ptr())


class Handle:
    """Owns one sx_handle and the torch tensors bound to it."""

    def __init__(self, case, precision: int = SX_FP64):
        import torch
        self.lib = load()
        self.case = case
        g, gas, sc = make_structs(case, precision)
        h = ctypes.c_void_p()
        rc = self.lib.sx_init(ctypes.byref(g), ctypes.byref(gas), ctypes.byref(sc), ctypes.byref(h))
        if rc != SX_OK:
            raise SxError(rc, "sx_init rejected the description")
        self.h = h
        lay = sx_layout()
        self._check(self.lib.sx_get_layout(h, ctypes.byref(lay)))
        self.layout = lay
        self.shape = (5, lay.pz, lay.py, lay.px)
        self.ng, self.ox = lay.ng, lay.ox
        self.W = None
        self.torch = torch

    # -- errors -------------------------------------------------------------
    def _check(self, rc):
        if rc != SX_OK:
            raise SxError(rc, self.lib.sx_last_error(self.h).decode())
        return rc

    def close(self):
        if getattr(self, "h", None):
            self.lib.sx_finalize(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- layout marshalling -------------------------------------------------
    def to_layout(self, Wn: np.ndarray):
        """Neutral ghosted array [5, nz+2g, ny+2g, nx+2g] -> library layout
        (padding columns zero) as a float64 device tensor."""
        g, ox = self.ng, self.ox
        assert Wn.shape[1:] == (self.case.nz + 2 * g, self.case.ny + 2 * g, self.case.nx + 2 * g)
        out = np.zeros(self.shape)
        out[:, :, :, ox - g:ox + self.case.nx + g] = Wn
        return self.torch.from_numpy(out).to("cuda")

    def from_layout(self, W) -> np.ndarray:
        g, ox = self.ng, self.ox
        a = W.detach().cpu().numpy()
        return np.ascontiguousarray(a[:, :, :, ox - g:ox + self.case.nx + g])

    def interior(self, W) -> np.ndarray:
        g, ox = self.ng, self.ox
        c = self.case
        a = W.detach().cpu().numpy() if hasattr(W, "detach") else W
        return np.ascontiguousarray(a[:, g:g + c.nz, g:g + c.ny, ox:ox + c.nx])

    # -- C ABI, same names --------------------------------------------------
    def sx_bind(self, W0, W1=None, Rprev=None, stream=None):
        torch = self.torch
        if W1 is None:
            W1 = torch.empty_like(W0)
        if Rprev is None:
            Rprev = torch.empty((5, self.case.nz, self.case.ny, self.case.nx), dtype=torch.float64,
                                device=W0.device)
        if stream is None:
            stream = torch.cuda.current_stream()
        self.W = [W0, W1]
        self.Rprev = Rprev
        self.stream = stream
        self._check(self.lib.sx_bind(self.h, _ptr(W0), _ptr(W1), _ptr(Rprev),
                                     ctypes.c_void_p(stream.cuda_stream)))

    def sx_current(self) -> int:
        c = ctypes.c_int()
        self._check(self.lib.sx_current(self.h, ctypes.byref(c)))
        return c.value

    @property
    def state(self):
        return self.W[self.sx_current()]

    def sx_fill_ghosts(self, W):
        self._check(self.lib.sx_fill_ghosts(self.h, _ptr(W)))

    def sx_rhs(self, W, R=None, mask: int = SX_ALL):
        if R is None:
            R = self.torch.empty((5, self.case.nz, self.case.ny, self.case.nx),
                                 dtype=self.torch.float64, device=W.device)
        self._check(self.lib.sx_rhs(self.h, _ptr(W), _ptr(R), mask))
        return R

    def sx_rk3_step(self, dt: float):
        self._check(self.lib.sx_rk3_step(self.h, dt))

    def sx_compute_dt(self, cfl: float) -> float:
        dt = ctypes.c_double()
        self._check(self.lib.sx_compute_dt(self.h, cfl, ctypes.byref(dt)))
        return dt.value

    def sx_set_flag_override(self, flags=None):
        """flags = (fx, fy, fz) uint8 arrays/tensors in the face layout, or
        None to return to the sensor."""
        if flags is None:
            self._check(self.lib.sx_set_flag_override(self.h, None, None, None))
            return
        import numpy as _np
        arrs = [_np.ascontiguousarray(f, dtype=_np.uint8) for f in flags]
        self._check(self.lib.sx_set_flag_override(self.h, *[a.ctypes.data for a in arrs]))

    def sx_get_flags(self):
        """Face flags of the last hybrid evaluation as numpy uint8 arrays
        (fx [nz][ny][nx+1], fy [nz][ny+1][nx], fz [nz+1][ny][nx])."""
        c = self.case
        out = [np.zeros((c.nz, c.ny, c.nx + 1), np.uint8), np.zeros((c.nz, c.ny + 1, c.nx), np.uint8),
               np.zeros((c.nz + 1, c.ny, c.nx), np.uint8)]
        self._check(self.lib.sx_get_flags(self.h, *[a.ctypes.data for a in out]))
        return out

    def sx_diagnostics_noalloc(self, out, R=None):
        """Diagnostics into `out` (a float64 device tensor of 16 values),
        asynchronously, using the library's fixed scratch array."""
        self._check(self.lib.sx_diagnostics_noalloc(self.h, _ptr(R), _ptr(out)))
        return out

    def sx_timing_enable(self, enable: bool = True):
        self._check(self.lib.sx_timing_enable(self.h, int(enable)))

    def sx_timing_read(self):
        n = ctypes.c_longlong()
        ms = ctypes.c_double()
        self._check(self.lib.sx_timing_read(self.h, ctypes.byref(n), ctypes.byref(ms)))
        return n.value, ms.value

    def sx_diagnostics(self, R=None) -> sx_diag:
        d = sx_diag()
        rc = self.lib.sx_diagnostics(self.h, _ptr(R), ctypes.byref(d))
        if rc not in (SX_OK, SX_ENONFINITE):
            self._check(rc)
        d.status = rc
        return d


class BatchHandle(Handle):
    """Owns a batch sx_handle (many periodic blocks, one scheme) and its
    state / register arenas."""

    def __init__(self, cases, precision: int = SX_FP64):
        import torch
        self.lib = load()
        self.cases = list(cases)
        n = len(self.cases)
        grids = (sx_grid * n)()
        gases = (sx_gas * n)()
        sc = None
        for b, c in enumerate(self.cases):
            g, gas, s = make_structs(c, precision)
            grids[b] = g
            gases[b] = gas
            sc = sc or s
        h = ctypes.c_void_p()
        rc = self.lib.sx_init_batch(n, grids, gases, ctypes.byref(sc), ctypes.byref(h))
        if rc != SX_OK:
            raise SxError(rc, "sx_init_batch rejected the description")
        self.h = h
        lay = sx_layout()
        self._check(self.lib.sx_get_layout(h, ctypes.byref(lay)))
        self.layout = lay
        self.boxes = []
        for b in range(n):
            bl = sx_layout()
            wo, ro = ctypes.c_longlong(), ctypes.c_longlong()
            self._check(self.lib.sx_get_box(h, b, ctypes.byref(bl), ctypes.byref(wo), ctypes.byref(ro)))
            self.boxes.append((bl, wo.value, ro.value))
        self.ng, self.ox = lay.ng, lay.ox
        self.W = None
        self.torch = torch

    def box_view(self, A, b):
        """View of block b's ghosted state [5, pz, py, px] inside a state arena."""
        bl, wo, _ = self.boxes[b]
        return A[wo:wo + bl.elems].view(5, bl.pz, bl.py, bl.px)

    def box_rhs_view(self, R, b):
        c = self.cases[b]
        _, _, ro = self.boxes[b]
        n = c.nx * c.ny * c.nz
        return R[ro:ro + 5 * n].view(5, c.nz, c.ny, c.nx)

    def to_arena(self, fields):
        """Neutral ghosted arrays (one per block) -> a float64 device state arena."""
        out = np.zeros(self.layout.elems)
        g = self.ng
        for b, (Wn, c) in enumerate(zip(fields, self.cases)):
            bl, wo, _ = self.boxes[b]
            v = out[wo:wo + bl.elems].reshape(5, bl.pz, bl.py, bl.px)
            v[:, :, :, bl.ox - g:bl.ox + c.nx + g] = Wn
        return self.torch.from_numpy(out).to("cuda")

    def box_interior(self, A, b) -> np.ndarray:
        c = self.cases[b]
        bl, _, _ = self.boxes[b]
        g = self.ng
        a = self.box_view(A, b).detach().cpu().numpy()
        return np.ascontiguousarray(a[:, g:g + c.nz, g:g + c.ny, bl.ox:bl.ox + c.nx])

    def sx_bind(self, W0, W1=None, Rprev=None, stream=None):
        torch = self.torch
        if Rprev is None:
            Rprev = torch.empty(5 * self.layout.interior, dtype=torch.float64, device=W0.device)
        super().sx_bind(W0, W1, Rprev, stream)

    def sx_rhs(self, W, R=None, mask: int = SX_ALL):
        if R is None:
            R = self.torch.zeros(5 * self.layout.interior, dtype=self.torch.float64, device=W.device)
        self._check(self.lib.sx_rhs(self.h, _ptr(W), _ptr(R), mask))
        return R

    def sx_set_tiling(self, tile_x: int, zchunk: int, workgroups: int = 0):
        t = sx_tiling(tile_x, 0, zchunk, workgroups, 0, 0.0)
        self._check(self.lib.sx_set_tiling(self.h, ctypes.byref(t)))
        return self.sx_get_tiling()

    def sx_get_tiling(self) -> sx_tiling:
        t = sx_tiling()
        self._check(self.lib.sx_get_tiling(self.h, ctypes.byref(t)))
        return t

    def sx_autotune(self, cache_path=None) -> sx_tiling:
        t = sx_tiling()
        p = None if cache_path is None else str(cache_path).encode()
        self._check(self.lib.sx_autotune(self.h, p, ctypes.byref(t)))
        return t

    def sx_set_graph(self, enable: bool = True):
        self._check(self.lib.sx_set_graph(self.h, int(enable)))
