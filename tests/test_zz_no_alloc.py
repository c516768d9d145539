"""The allocation-free diagnostics entry point (sx_diagnostics_noalloc)
through the C ABI against sx_diagnostics on the same handle: bitwise-equal
values, on two calls in a row where the second has a smaller input (the
fixed scratch array keeps the first call's contents), for a single block, a
hybrid block with the sensor on (flagged-face fractions) and a batch."""
import numpy as np
import pytest

from paper_2304_05494_amd import inputs, sx

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _single(case):
    h = sx.Handle(case)
    W = h.to_layout(np.ascontiguousarray(inputs.fields(case)))
    h.sx_bind(W)
    return h, W


def _check(h, R=None):
    out = torch.full((16,), float("nan"), dtype=torch.float64, device="cuda")
    h.sx_diagnostics_noalloc(out, R)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    ref = h.sx_diagnostics(R).as_array()
    assert np.array_equal(got, ref), np.stack([got, ref])
    return got


def test_noalloc_single_block_two_calls():
    big, Wb = _single(inputs.tgv_case(24, mach=0.3))
    Rb = big.sx_rhs(Wb)
    a = _check(big, Rb)
    small, Ws = _single(inputs.tgv_case(12, mach=0.2))
    b = _check(small, small.sx_rhs(Ws))
    assert a[15] != b[15] or a[0] != b[0]           # different inputs, different sums
    # and the first handle again after the smaller call
    _check(big, Rb)
    _check(big)


def test_noalloc_hybrid_block_two_calls():
    big, _ = _single(inputs.shock_bl_case(96, 48, 12))
    a = _check(big)
    assert a[12] > 0.0
    small, _ = _single(inputs.shock_bl_case(64, 32, 8))
    _check(small)


def test_noalloc_batch_two_calls():
    cases = inputs.batch_cases(5)
    fields = [np.ascontiguousarray(inputs.fields(c)) for c in cases]
    bh = sx.BatchHandle(cases)
    bh.sx_bind(bh.to_arena(fields))
    _check(bh)
    bh2 = sx.BatchHandle(cases[:2])
    bh2.sx_bind(bh2.to_arena(fields[:2]))
    _check(bh2)


def test_noalloc_rejections():
    h, _ = _single(inputs.tgv_case(12))
    L = sx.load()
    assert L.sx_diagnostics_noalloc(h.h, None, None) == sx.SX_EINVAL
    unbound = sx.Handle(inputs.tgv_case(12))
    out = torch.zeros(16, dtype=torch.float64, device="cuda")
    assert L.sx_diagnostics_noalloc(unbound.h, None, out.data_ptr()) == sx.SX_ESTATE
