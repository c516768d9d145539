"""GPU parity of the KEEP-n central flux (the optional kinetic-energy and
entropy preserving scheme of Section 2) against the CPU oracle: per-term
right-hand sides on a periodic block and on a walled, stretched block, for
series cuts n = 0, 2 and the exact logarithmic means, orders C4/C6/C8, and
RK3 steps."""
import math

import numpy as np
import pytest

from paper_2304_05494_amd import inputs, sx
from tests.helpers import oracle_for, rel_err_per_field

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _case(kind, order, keep_n):
    if kind == "periodic":
        two_pi = 2 * math.pi
        return inputs.Case(name="tgv-keep", nx=40, ny=20, nz=12, lx=two_pi, ly=two_pi, lz=two_pi,
                           central_order=order, visc_order=order, mach=0.4, reynolds=200.0,
                           central_flux=1, keep_n=keep_n)
    base = inputs.channel_case(70, 36, 20)
    return inputs.Case(**{**base.__dict__, "name": "channel-keep", "central_order": order,
                          "visc_order": order, "central_flux": 1, "keep_n": keep_n})


def _close(got, ref, tol):
    scale = np.abs(ref).max(axis=(1, 2, 3))
    scale[1:4] = np.sqrt((ref[1:4] ** 2).sum(axis=0)).max()
    err = np.abs(got - ref).max(axis=(1, 2, 3)) / np.where(scale > 0, scale, 1.0)
    assert np.all(err < tol), err


@pytest.mark.parametrize("keep_n", [0, 2, -1], ids=["n0", "n2", "exact"])
@pytest.mark.parametrize("order", [4, 6, 8])
@pytest.mark.parametrize("kind", ["periodic", "walls"])
def test_keep_rhs_term_parity(kind, order, keep_n):
    case = _case(kind, order, keep_n)
    Wn = np.ascontiguousarray(inputs.fields(case))
    h = sx.Handle(case)
    W = h.to_layout(Wn)
    h.sx_bind(W)
    o = oracle_for(case)
    for mask in (sx.SX_CONV_X, sx.SX_CONV_Y, sx.SX_CONV_Z, sx.SX_ALL):
        R = h.sx_rhs(W, mask=mask)
        torch.cuda.synchronize()
        _close(R.cpu().numpy(), o.rhs(Wn.copy(), mask=mask), 1e-11)


@pytest.mark.parametrize("kind", ["periodic", "walls"])
def test_keep_rk3_steps_parity(kind):
    case = _case(kind, 6, 1)
    Wn = np.ascontiguousarray(inputs.fields(case))
    o = oracle_for(case)
    dt = o.compute_dt(Wn.copy(), case.cfl)
    h = sx.Handle(case)
    h.sx_bind(h.to_layout(Wn))
    for _ in range(5):
        h.sx_rk3_step(dt)
    torch.cuda.synchronize()
    Wo = Wn.copy()
    Rp = np.zeros((5, case.nz, case.ny, case.nx))
    for _ in range(5):
        o.rk3_step(Wo, Rp, dt)
    err = rel_err_per_field(h.interior(h.state), o.interior(Wo))
    assert np.all(err < 1e-12), err
