"""GPU checks of the batched form: every block of a batch advances exactly as
the same block does alone (bitwise, for both tile shapes, ragged z-chunks,
both precision forms), matches the CPU oracle after 10 RK3 steps, the
captured step graph replays exactly what direct launches compute, and the
autotuner keeps results unchanged and reuses its JSON cache. The full-size
48-block batch is checked on sampled blocks."""
import json
import math

import numpy as np
import pytest

from paper_2304_05494_amd import inputs, sx
from tests.helpers import oracle_for, rel_err_per_field

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SIZES = [(16, 16, 16), (24, 24, 24), (32, 16, 24), (20, 28, 12), (40, 24, 16), (16, 32, 20)]


def small_batch():
    cases = []
    for b, (nx, ny, nz) in enumerate(SIZES):
        kind = "tgv" if b % 2 == 0 else "hit"
        h = 2.0 * math.pi / max(nx, ny, nz)
        cases.append(inputs.Case(name=f"box{b}-{kind}{nx}x{ny}x{nz}", nx=nx, ny=ny, nz=nz,
                                 lx=nx * h, ly=ny * h, lz=nz * h, mach=0.1 + 0.08 * b,
                                 reynolds=1600.0, steps=10, seed=700 + b, extra={"kind": kind}))
    return cases


def make_batch(cases, precision=sx.SX_FP64, fields=None):
    bh = sx.BatchHandle(cases, precision)
    fields = fields if fields is not None else [np.ascontiguousarray(inputs.fields(c)) for c in cases]
    bh.sx_bind(bh.to_arena(fields))
    return bh, fields


def single_run(case, Wn, dt, steps, precision=sx.SX_FP64):
    h = sx.Handle(case, precision)
    h.sx_bind(h.to_layout(Wn))
    for _ in range(steps):
        h.sx_rk3_step(dt)
    torch.cuda.synchronize()
    return h.interior(h.state)


@pytest.mark.parametrize("precision", [sx.SX_FP64, sx.SX_FP32_FLUX], ids=["fp64", "fp32flux"])
@pytest.mark.parametrize("tile_x,zchunk", [(64, 1000), (32, 8), (64, 5)])
def test_batch_equals_single_block_runs(precision, tile_x, zchunk):
    cases = small_batch()
    bh, fields = make_batch(cases, precision)
    t = bh.sx_set_tiling(tile_x, zchunk)
    assert t.tile_x == tile_x and t.work_items > len(cases)
    dt = bh.sx_compute_dt(0.5)
    for _ in range(3):
        bh.sx_rk3_step(dt)
    torch.cuda.synchronize()
    for b, c in enumerate(cases):
        ref = single_run(c, fields[b], dt, 3, precision)
        got = bh.box_interior(bh.state, b)
        assert np.array_equal(got, ref), (b, np.abs(got - ref).max())


def test_batch_matches_oracle_after_ten_steps():
    cases = [small_batch()[0], small_batch()[3]]
    bh, fields = make_batch(cases)
    dts = [oracle_for(c).compute_dt(f.copy(), 0.5) for c, f in zip(cases, fields)]
    dt = min(dts)
    assert bh.sx_compute_dt(0.5) == pytest.approx(dt, rel=1e-13)
    for _ in range(10):
        bh.sx_rk3_step(dt)
    torch.cuda.synchronize()
    for b, c in enumerate(cases):
        o = oracle_for(c)
        Wo = fields[b].copy()
        Rp = np.zeros((5, c.nz, c.ny, c.nx))
        for _ in range(10):
            o.rk3_step(Wo, Rp, dt)
        err = rel_err_per_field(bh.box_interior(bh.state, b), o.interior(Wo))
        assert np.all(err < 1e-12), (b, err)


def test_batch_fp32_flux_matches_oracle_after_ten_steps():
    """The batched FP32-flux form against the FP64 oracle: each block's
    state after 10 RK3 steps within the FP32-flux bound of the single-block
    form (relative 1e-5 per field; the FP32 rounding of the stencil sums,
    far above the FP64 path's 1e-12)."""
    cases = [small_batch()[0], small_batch()[3]]
    bh, fields = make_batch(cases, sx.SX_FP32_FLUX)
    dt = min(oracle_for(c).compute_dt(f.copy(), 0.5) for c, f in zip(cases, fields))
    for _ in range(10):
        bh.sx_rk3_step(dt)
    torch.cuda.synchronize()
    for b, c in enumerate(cases):
        o = oracle_for(c)
        Wo = fields[b].copy()
        Rp = np.zeros((5, c.nz, c.ny, c.nx))
        for _ in range(10):
            o.rk3_step(Wo, Rp, dt)
        err = rel_err_per_field(bh.box_interior(bh.state, b), o.interior(Wo))
        assert np.all(err < 1e-5), (b, err)
        assert np.any(err > 1e-12), (b, err)   # it does run in FP32


def test_graph_replay_equals_direct_launches():
    cases = small_batch()
    ga, fields = make_batch(cases)
    gb, _ = make_batch(cases, fields=fields)
    gb.sx_set_graph(False)
    ga.sx_set_tiling(32, 7)
    gb.sx_set_tiling(32, 7)
    dt = ga.sx_compute_dt(0.5)
    for step in range(6):
        if step == 3:
            dt *= 0.7          # new dt: the captured graphs read it from device memory
        ga.sx_rk3_step(dt)
        gb.sx_rk3_step(dt)
        # eager work and a synchronisation between replays
        da, db = ga.sx_diagnostics(), gb.sx_diagnostics()
        assert da.mass == db.mass
        assert torch.equal(ga.state, gb.state), step


def test_rhs_and_diagnostics_per_block():
    cases = small_batch()
    bh, fields = make_batch(cases)
    R = bh.sx_rhs(bh.state)
    d = bh.sx_diagnostics(R)
    torch.cuda.synchronize()
    tot = np.zeros(16)
    dts = []
    for b, c in enumerate(cases):
        h = sx.Handle(c)
        W = h.to_layout(fields[b])
        h.sx_bind(W)
        Rs = h.sx_rhs(W)
        torch.cuda.synchronize()
        assert torch.equal(bh.box_rhs_view(R, b), Rs), b
        ds = h.sx_diagnostics(Rs).as_array()
        for k in (0, 1, 2, 3, 4, 5, 9, 10, 11, 15):
            tot[k] += ds[k]
        tot[6] = max(tot[6], ds[6]) if b else ds[6]
        tot[7] = min(tot[7], ds[7]) if b else ds[7]
        tot[8] = min(tot[8], ds[8]) if b else ds[8]
        dts.append(h.sx_compute_dt(0.5))
    got = d.as_array()
    np.testing.assert_allclose(got, tot, rtol=1e-14, atol=1e-300)
    assert bh.sx_compute_dt(0.5) == min(dts)


def test_autotune_keeps_results_and_reuses_cache(tmp_path):
    cases = small_batch()
    cache = tmp_path / "tune.json"
    bh, fields = make_batch(cases)
    before = bh.state.clone()
    t1 = bh.sx_autotune(cache)
    assert torch.equal(bh.state, before)
    assert t1.tile_x in (32, 64) and t1.zchunk >= 1 and t1.ms_per_substep > 0
    entries = json.loads(cache.read_text())
    assert len(entries) == 1
    (entry,) = entries.values()
    assert entry["tile_x"] == t1.tile_x and entry["zchunk"] == t1.zchunk
    dt = bh.sx_compute_dt(0.5)
    for _ in range(2):
        bh.sx_rk3_step(dt)
    ref, _ = make_batch(cases, fields=fields)
    for _ in range(2):
        ref.sx_rk3_step(dt)
    torch.cuda.synchronize()
    assert torch.equal(bh.state, ref.state)
    # a second handle takes the cached choice without timing
    bh2, _ = make_batch(cases, fields=fields)
    t2 = bh2.sx_autotune(cache)
    assert (t2.tile_x, t2.zchunk) == (t1.tile_x, t1.zchunk)
    assert t2.ms_per_substep == pytest.approx(entry["ms_per_substep"], abs=1e-6)


def test_batch_timing_counts_three_launches_per_step():
    cases = small_batch()[:2]
    bh, _ = make_batch(cases)
    bh.sx_timing_enable(True)
    dt = bh.sx_compute_dt(0.5)
    for _ in range(2):
        bh.sx_rk3_step(dt)
    n, ms = bh.sx_timing_read()
    assert n == 6 and ms > 0


def test_full_size_batch_sampled_blocks():
    """The 48-block batch (sizes 32^3 .. 128x64x64): one step of the batch,
    sampled blocks (largest, smallest, one of each kind) against the same
    blocks advanced alone."""
    cases = inputs.batch_cases(48)
    print(f"batch of {len(cases)} blocks, {sum(c.nx * c.ny * c.nz for c in cases)} points", flush=True)
    fields = [np.ascontiguousarray(inputs.fields(c)) for c in cases]
    bh, _ = make_batch(cases, fields=fields)
    bh.sx_autotune()
    dt = bh.sx_compute_dt(0.5)
    bh.sx_rk3_step(dt)
    torch.cuda.synchronize()
    vol = [c.nx * c.ny * c.nz for c in cases]
    kinds = [c.extra["kind"] for c in cases]
    pick = {int(np.argmax(vol)), int(np.argmin(vol)), kinds.index("tgv"), kinds.index("hit")}
    for b in sorted(pick):
        ref = single_run(cases[b], fields[b], dt, 1)
        assert np.array_equal(bh.box_interior(bh.state, b), ref), b
    d = bh.sx_diagnostics()
    assert d.status == sx.SX_OK and d.nonfinite == 0
