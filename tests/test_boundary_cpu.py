"""CPU-side checks of the C ABI: the library loads, exports every function
include/sx.h declares, the binding's structs match the header, and invalid
descriptions are rejected before any device call (no GPU needed)."""
import ctypes
import os
import re

import pytest

from paper_2304_05494_amd import inputs, sx

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "sx.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sx_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_binding_exports():
    assert declared_functions() == sorted(sx.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(sx.LIB_PATH)
    for name in declared_functions():
        assert hasattr(L, name), name


def test_struct_layouts_match_the_c_header(tmp_path):
    """Compile the header with gcc and compare every field offset and struct
    size with the ctypes mirrors used by the binding."""
    import subprocess
    structs = [sx.sx_grid, sx.sx_gas, sx.sx_scheme, sx.sx_layout, sx.sx_diag, sx.sx_tiling]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "sx.h"', 'int main(void){']
    for st in structs:
        n = st.__name__
        lines.append(f'printf("{n} size %zu\\n", sizeof({n}));')
        for f, _ in st._fields_:
            lines.append(f'printf("{n} {f} %zu\\n", offsetof({n}, {f}));')
    lines.append('return 0;}')
    src = tmp_path / "probe.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "probe"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    out = subprocess.check_output([str(exe)]).decode().split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for st in structs:
        n = st.__name__
        assert got[(n, "size")] == ctypes.sizeof(st), n
        for f, _ in st._fields_:
            assert got[(n, f)] == getattr(st, f).offset, (n, f)


def _init(case, **patch):
    L = sx.load()
    g, gas, sc = sx.make_structs(case)
    for k, v in patch.items():
        for s in (g, gas, sc):
            if hasattr(s, k):
                setattr(s, k, v)
    h = ctypes.c_void_p()
    rc = L.sx_init(ctypes.byref(g), ctypes.byref(gas), ctypes.byref(sc), ctypes.byref(h))
    return rc, h


@pytest.mark.parametrize("patch,code", [
    ({"central_order": 5}, sx.SX_EINVAL),
    ({"central_order": 10}, sx.SX_EINVAL),
    ({"visc_order": 3}, sx.SX_EINVAL),
    ({"weno_order": 9}, sx.SX_EINVAL),
    ({"nx": 2}, sx.SX_EINVAL),
    ({"gamma": 1.0}, sx.SX_EINVAL),
    ({"lx": 0.0}, sx.SX_EINVAL),
    ({"ymap": 9}, sx.SX_EINVAL),
    ({"nx": 1024, "ny": 1024, "nz": 1024}, sx.SX_EINVAL),   # over 4 GiB per variable
    ({"central_flux": 2}, sx.SX_EINVAL),
    ({"central_flux": 1, "keep_n": 17}, sx.SX_EINVAL),
    # KEEP-n is built for FP64, sensor off, equal convective and viscous orders
    ({"central_flux": 1, "precision": sx.SX_FP32_FLUX}, sx.SX_EUNSUPPORTED),
    ({"central_flux": 1, "sensor": 1}, sx.SX_EUNSUPPORTED),
    ({"central_flux": 1, "visc_order": 4}, sx.SX_EUNSUPPORTED),
    ({"bulk_forcing": 2}, sx.SX_EINVAL),
    ({"thermo": 2}, sx.SX_EINVAL),
    ({"thermo": 1, "t_ref": 0.0}, sx.SX_EINVAL),
    # the thermally perfect gas is built for the central split form, equal orders
    ({"thermo": 1, "sensor": 1}, sx.SX_EUNSUPPORTED),
    ({"thermo": 1, "central_flux": 1}, sx.SX_EUNSUPPORTED),
    ({"thermo": 1, "visc_order": 4}, sx.SX_EUNSUPPORTED),
    ({"bulk_forcing": 1, "sensor": 1}, sx.SX_EUNSUPPORTED),
])
def test_invalid_descriptions_rejected_without_device(patch, code):
    rc, h = _init(inputs.tgv_case(16), **patch)
    assert rc == code
    assert not h.value


def test_unpaired_periodic_face_rejected():
    case = inputs.tgv_case(16)
    L = sx.load()
    g, gas, sc = sx.make_structs(case)
    g.bc[0] = sx.SX_BC_WALL      # x-lo wall with x-hi periodic
    h = ctypes.c_void_p()
    assert L.sx_init(ctypes.byref(g), ctypes.byref(gas), ctypes.byref(sc), ctypes.byref(h)) == sx.SX_EINVAL


def test_null_arguments():
    L = sx.load()
    h = ctypes.c_void_p()
    assert L.sx_init(None, None, None, ctypes.byref(h)) == sx.SX_EINVAL
    assert L.sx_rk3_step(None, ctypes.c_double(1.0)) == sx.SX_EINVAL
    assert L.sx_last_error(None) == b"null handle"
    L.sx_finalize(None)


def _init_batch(cases, **patch):
    L = sx.load()
    n = len(cases)
    grids, gases = (sx.sx_grid * n)(), (sx.sx_gas * n)()
    sc = None
    for b, c in enumerate(cases):
        g, gas, s = sx.make_structs(c)
        for k, v in patch.items():
            if hasattr(g, k):
                setattr(g, k, v)
            if hasattr(s, k):
                setattr(s, k, v)
            if hasattr(gas, k):
                setattr(gas, k, v)
        grids[b], gases[b] = g, gas
        sc = sc or s
    h = ctypes.c_void_p()
    rc = L.sx_init_batch(n, grids, gases, ctypes.byref(sc), ctypes.byref(h))
    return rc, h


def test_batch_rejections_without_device():
    cases = [inputs.tgv_case(16), inputs.tgv_case(24)]
    L = sx.load()
    h = ctypes.c_void_p()
    g, gas, sc = sx.make_structs(cases[0])
    assert L.sx_init_batch(0, ctypes.byref(g), ctypes.byref(gas), ctypes.byref(sc), ctypes.byref(h)) == sx.SX_EINVAL
    assert L.sx_init_batch(1, None, None, None, ctypes.byref(h)) == sx.SX_EINVAL
    # the batched form is the central path on periodic blocks
    assert _init_batch(cases, sensor=1)[0] == sx.SX_EUNSUPPORTED
    ch = inputs.channel_case(32, 16, 8)
    assert _init_batch([ch])[0] == sx.SX_EUNSUPPORTED
    assert _init_batch(cases, central_order=5)[0] == sx.SX_EINVAL
    # the persistent kernels take one order for convective and viscous terms,
    # the split-form flux and no bulk forcing
    assert _init_batch(cases, visc_order=4)[0] == sx.SX_EUNSUPPORTED
    assert _init_batch(cases, central_flux=1)[0] == sx.SX_EUNSUPPORTED
    assert _init_batch(cases, bulk_forcing=1)[0] == sx.SX_EUNSUPPORTED
    assert _init_batch(cases, thermo=1)[0] == sx.SX_EUNSUPPORTED
    # blocks narrower than twice the ghost width cannot hold periodic images
    small = inputs.Case(**{**inputs.tgv_case(16).__dict__, "nz": 5})
    assert _init_batch([small])[0] == sx.SX_EUNSUPPORTED
    t = sx.sx_tiling()
    assert L.sx_get_box(None, 0, None, None, None) == sx.SX_EINVAL
    assert L.sx_set_tiling(None, ctypes.byref(t)) == sx.SX_EINVAL
    assert L.sx_autotune(None, None, None) == sx.SX_EINVAL
    assert L.sx_set_graph(None, 1) == sx.SX_EINVAL
