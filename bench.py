"""Benchmark of the RHS + RK3 hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Headline workload: the channel-like block 512x256x256 in FP64 (periodic
x/z, isothermal tanh-stretched walls in y, bulk Mach 1.5, Re_b 6000,
sixth-order central split-form convection + sixth-order Laplacian viscous
terms), seeded synthetic input, inputs resident in HBM before the timed
region. One step = one full RK3 step (three fused RHS/update substeps +
ghost fills).

Prints one JSON line: throughput (grid-point updates per second per RK3
step), the roofline of the dominant kernel (the fused RHS/update kernel,
timed live with HIP events on its stream) and the CPU oracle baseline,
plus side legs: the same block in the FP32-flux form (and its per-variable
difference from the FP64 path after 100 steps), the Taylor-Green vortex
32^3, the shock/boundary-layer block 1024x256x128 with the sensor and WENO-5,
and the 48-block batched form in FP64 and FP32-flux.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP64_PEAK_TFLOPS = 78.6        # MI355X FP64 vector
FP32_PEAK_TFLOPS = 157.3       # MI355X FP32 vector (packed; unpacked issue is half)
# Algorithmic HBM bytes per interior point of one RK3 step: 3 reads + 3
# writes of the 5 FP64 conserved variables, the RK register written in
# substeps 1-2 and read in substeps 2-3 -> (6 + 4) * 40 B.
ALG_BYTES_PER_POINT_STEP = 400.0
SUBSTEPS = 3


def progress(msg):
    """A progress line on stderr (the JSON result stays the only stdout line)."""
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--reps", type=int, default=5,
                    help="repetitions of the K timed steps; the median one is reported")
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the oracle timing (profiling runs)")
    ap.add_argument("--cpu-sample-steps", type=int, default=4)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run only a plain device copy of 2 GiB (counter calibration)")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-form legs")
    ap.add_argument("--no-legs", action="store_true",
                    help="skip the TGV, shock/boundary-layer and FP32-error legs")
    ap.add_argument("--sweep", action="store_true",
                    help="add the stencil-order sweep (channel, C2..C8, FP64 and FP32-flux) and "
                         "the WENO-activation sweep (shock/boundary-layer block, injected flags)")
    ap.add_argument("--sweep-f2", action="store_true",
                    help="add the viscous-order (C6 V2..V8), WENO-order (W1..W7 on every face), "
                         "thread-masking (the four grids of the paper's masking study) and "
                         "grid-size (0.25 M to 134 M points) sweeps")
    ap.add_argument("--weno-order-only", action="store_true",
                    help="run only the WENO-order sweep and print it (counter runs)")
    ap.add_argument("--tune-cache", default=None,
                    help="JSON autotune cache of the batched form (default: tune afresh)")
    return ap.parse_args()


def calibrate_copy():
    """A plain copy of known size: 2 GiB read + 2 GiB written, three times.
    Its FETCH_SIZE / WRITE_SIZE counters give the scale factor between what
    those counters report and bytes actually moved."""
    import torch
    n = (2 << 30) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"calibration": "copy", "bytes_read_per_launch": n * 8,
                      "bytes_written_per_launch": n * 8, "launches": 3}), flush=True)


def load_traffic(kernel: str):
    """Counter-measured HBM bytes per launch from profiles/, if recorded for
    the current kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
        import hashlib
        src = os.path.join(ROOT, "paper_2304_05494_amd", "csrc", "sx_rhs.hip")
        digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
        if rec.get("kernel") != kernel or rec.get("source_sha256") != digest:
            return None
        return float(rec["bytes_per_launch"])
    except Exception:
        return None


def load_flops(kernel: str):
    """Counter-measured VALU flops per launch (profiles/valu_flops.json), if
    recorded for the current kernel source."""
    path = os.path.join(ROOT, "profiles", "valu_flops.json")
    try:
        import hashlib
        rec = json.load(open(path))
        src = os.path.join(ROOT, "paper_2304_05494_amd", "csrc", "sx_rhs.hip")
        if rec.get("source_sha256") != hashlib.sha256(open(src, "rb").read()).hexdigest():
            return None
        return rec["kernels"].get(kernel)
    except Exception:
        return None


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(case, Wn, dt, steps, single_nz=32, single_steps=2):
    """The oracle, as is, timed on this host: `steps` RK3 steps of the full
    grid on all OpenMP threads, and (single-thread rate) `single_steps` RK3
    steps of a z-slab of the same flow (same x-y planes, single_nz planes,
    periodic in z like the full block)."""
    import dataclasses
    import numpy as np
    import oracle as O
    from paper_2304_05494_amd import inputs
    p = O.Params(**{k: getattr(case, k) for k in O.Params.__dataclass_fields__})
    o = O.Oracle(p)
    W = Wn.copy()
    Rp = np.zeros((5, case.nz, case.ny, case.nx))
    cores = O.num_threads()
    t0 = time.perf_counter()
    for _ in range(steps):
        o.rk3_step(W, Rp, dt)
    el = time.perf_counter() - t0
    del W, Rp
    slab = dataclasses.replace(case, nz=single_nz)
    ps = O.Params(**{k: getattr(slab, k) for k in O.Params.__dataclass_fields__})
    os_ = O.Oracle(ps)
    Ws = np.ascontiguousarray(inputs.fields(slab))
    Rs = np.zeros((5, slab.nz, slab.ny, slab.nx))
    O.set_num_threads(1)
    try:
        t1 = time.perf_counter()
        for _ in range(single_steps):
            os_.rk3_step(Ws, Rs, dt)
        el1 = time.perf_counter() - t1
    finally:
        O.set_num_threads(cores)
    return {"value": case.points * steps / el, "unit": "grid-point updates/s per RK3 step",
            "cores": cores, "kind": "oracle", "cpu_model": cpu_model(),
            "sample": f"{steps} RK3 step(s) of the full {case.nx}x{case.ny}x{case.nz} workload "
                      f"({el:.1f} s, OpenMP over z-planes, {cores} threads)",
            "single_thread": {"value": slab.points * single_steps / el1, "cores": 1,
                              "sample": f"{single_steps} RK3 step(s) of a {slab.nx}x{slab.ny}x{slab.nz} "
                                        f"z-slab of the same flow ({el1:.1f} s, one thread)"}}


def time_steps(h, dt, steps, warmup, reps=3):
    """Wall time per RK3 step (HIP events on the bound stream) and the
    per-launch time of the fused RHS/update kernel: the median of `reps`
    repetitions of `steps` steps."""
    import torch
    for _ in range(warmup):
        h.sx_rk3_step(dt)
    torch.cuda.synchronize()
    h.sx_timing_enable(True)
    h.sx_timing_read()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    res = []
    for _ in range(reps):
        start.record()
        for _ in range(steps):
            h.sx_rk3_step(dt)
        stop.record()
        torch.cuda.synchronize()
        n, kms = h.sx_timing_read()
        res.append((start.elapsed_time(stop) / steps, kms / n))
    h.sx_timing_enable(False)
    res.sort()
    return res[len(res) // 2]


def bench_tgv(args):
    """Taylor-Green vortex 32^3 (the small correctness case): launch-bound,
    rate reported without a roofline claim."""
    import numpy as np
    from paper_2304_05494_amd import inputs, sx
    case = inputs.tgv_case(32)
    h = sx.Handle(case)
    h.sx_bind(h.to_layout(np.ascontiguousarray(inputs.fields(case))))
    dt = h.sx_compute_dt(case.cfl)
    ms, _ = time_steps(h, dt, 10, args.warmup)
    return {"value": case.points / (ms * 1e-3), "ms_per_step": ms, "steps": 10,
            "workload": "Taylor-Green vortex 32^3, M0 0.1, Re 1600, C6 + V6, FP64"}


def bench_shock_bl(args):
    """Shock / boundary-layer block 1024x256x128 with the Ducros sensor and
    WENO-5 characteristic fluxes on flagged faces (FP64 and FP32-flux)."""
    import numpy as np
    import torch
    from paper_2304_05494_amd import inputs, sx
    case = inputs.shock_bl_case()
    Wn = np.ascontiguousarray(inputs.fields(case))
    out = {"workload": "shock/boundary-layer block 1024x256x128: Mach 2 flat-plate boundary "
                       "layer + 8 deg oblique shock, W5 where the Ducros sensor exceeds 0.5, "
                       "C6 + V6 elsewhere",
           "points": case.points}
    dt = None
    ms64 = None
    for prec, name in ((sx.SX_FP64, "fp64"), (sx.SX_FP32_FLUX, "fp32_flux")):
        h = sx.Handle(case, prec)
        h.sx_bind(h.to_layout(Wn))
        if dt is None:
            dt = h.sx_compute_dt(case.cfl)
            d = h.sx_diagnostics()
            out["weno_face_fraction"] = list(d.weno_fraction)
        ms, kms = time_steps(h, dt, args.steps, args.warmup)
        d = h.sx_diagnostics()
        out[name] = {"value": case.points / (ms * 1e-3), "ms_per_step": ms,
                     "central_kernel_ms": kms, "state_ok": d.status == sx.SX_OK}
        if ms64 is None:
            ms64 = ms
        else:
            out[name]["speedup_vs_fp64"] = ms64 / ms
        del h
        torch.cuda.empty_cache()
    return out


def bench_order_sweep(args, Wn, dt):
    """The channel block at central/viscous orders 2, 4, 6, 8 in both
    precision forms: RK3 step time, fused-kernel launch time and its
    fraction of the HBM roofline (the algorithmic bytes do not depend on the
    order; the arithmetic and the halo grow with it)."""
    import numpy as np
    import torch
    from paper_2304_05494_amd import inputs, sx
    out = {}
    for order in (2, 4, 6, 8):
        case = inputs.channel_case(central_order=order, visc_order=order)
        # C8 needs four ghost layers: the same recipe on the wider ghosted array
        Wo = Wn if case.ng == inputs.channel_case().ng else np.ascontiguousarray(inputs.fields(case))
        row = {}
        for prec, name in ((sx.SX_FP64, "fp64"), (sx.SX_FP32_FLUX, "fp32_flux")):
            h = sx.Handle(case, prec)
            h.sx_bind(h.to_layout(Wo))
            ms, kms = time_steps(h, dt, args.steps, args.warmup)
            d = h.sx_diagnostics()
            row[name] = {"ms_per_step": ms, "launch_ms": kms,
                         "roofline_frac": ALG_BYTES_PER_POINT_STEP / SUBSTEPS * case.points
                         / (kms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                         "state_ok": d.status == sx.SX_OK}
            del h
            torch.cuda.empty_cache()
        out[f"C{order}V{order}"] = row
        progress(f"order sweep C{order}V{order} done")
    return out


def bench_visc_order_sweep(args, Wn, dt):
    """The channel block with sixth-order convection and viscous orders 2, 4,
    6, 8 (the paper varies V2..V8 apart from C2..C8), FP64."""
    import numpy as np
    import torch
    from paper_2304_05494_amd import inputs, sx
    out = {}
    for vo in (2, 4, 6, 8):
        case = inputs.channel_case(central_order=6, visc_order=vo)
        Wo = Wn if case.ng == inputs.channel_case().ng else np.ascontiguousarray(inputs.fields(case))
        h = sx.Handle(case)
        h.sx_bind(h.to_layout(Wo))
        ms, kms = time_steps(h, dt, args.steps, args.warmup)
        d = h.sx_diagnostics()
        out[f"C6V{vo}"] = {"ms_per_step": ms, "launch_ms": kms,
                           "roofline_frac": ALG_BYTES_PER_POINT_STEP / SUBSTEPS * case.points
                           / (kms * 1e-3) / 1e9 / HBM_PEAK_GBS, "state_ok": d.status == sx.SX_OK}
        progress(f"viscous-order sweep C6V{vo} done")
        del h
        torch.cuda.empty_cache()
    return out


def bench_weno_order_sweep(args):
    """WENO orders 1, 3, 5, 7 on every face of the channel block (sensor
    threshold below zero), C6 + V6, FP64: RK3 step time against the order
    (the paper's W1..W7 study)."""
    import numpy as np
    import torch
    from paper_2304_05494_amd import inputs, sx
    out = {}
    dt = None
    for wo in (1, 3, 5, 7):
        case = inputs.channel_case(sensor=1, sensor_thr=-1.0, weno_order=wo)
        Wo = np.ascontiguousarray(inputs.fields(case))
        h = sx.Handle(case)
        h.sx_bind(h.to_layout(Wo))
        if dt is None:
            dt = h.sx_compute_dt(case.cfl)
        ms, kms = time_steps(h, dt, max(3, args.steps // 4), args.warmup)
        d = h.sx_diagnostics()
        out[f"W{wo}"] = {"ms_per_step": ms, "central_kernel_ms": kms,
                         "weno_face_fraction": list(d.weno_fraction), "state_ok": d.status == sx.SX_OK}
        progress(f"WENO-order sweep W{wo} done")
        del h, Wo
        torch.cuda.empty_cache()
    return out


MASKING_GRIDS = ((384, 256, 384), (384, 256, 350), (420, 256, 350), (420, 250, 320))


def bench_thread_masking(args):
    """The paper's thread-masking grids (multiples of 128 in three, two, one
    and no direction), channel-like flow, FP64: grind time (ms per RK3 step
    per 1e8 points) for the central scheme and with WENO-5 on every face."""
    import numpy as np
    import torch
    from paper_2304_05494_amd import inputs, sx
    out = {}
    for n, (nx, ny, nz) in enumerate(MASKING_GRIDS, 1):
        row = {"grid": [nx, ny, nz]}
        for name, kw in (("central", {}), ("weno", {"sensor": 1, "sensor_thr": -1.0})):
            case = inputs.channel_case(nx, ny, nz, **kw)
            Wo = np.ascontiguousarray(inputs.fields(case))
            h = sx.Handle(case)
            h.sx_bind(h.to_layout(Wo))
            dt = h.sx_compute_dt(case.cfl)
            steps = args.steps if name == "central" else max(3, args.steps // 4)
            ms, kms = time_steps(h, dt, steps, args.warmup)
            row[name] = {"ms_per_step": ms, "grind_ms_per_1e8_points": ms * 1e8 / case.points,
                         "fused_kernel_ms": kms}
            del h, Wo
            torch.cuda.empty_cache()
        out[f"grid{n}"] = row
        progress(f"thread-masking grid {n} done")
    return out


def bench_grid_size_sweep(args):
    """Grind time against the number of points (the paper's grid-size study):
    channel-like blocks from 0.25 M to 134 M points, doubling, FP64 central."""
    import numpy as np
    import torch
    from paper_2304_05494_amd import inputs, sx
    out = {}
    shapes = [(64, 64, 64), (128, 64, 64), (128, 128, 64), (128, 128, 128), (256, 128, 128),
              (256, 256, 128), (256, 256, 256), (512, 256, 256), (512, 512, 256), (512, 512, 512)]
    for nx, ny, nz in shapes:
        case = inputs.channel_case(nx, ny, nz)
        Wo = np.ascontiguousarray(inputs.fields(case))
        h = sx.Handle(case)
        h.sx_bind(h.to_layout(Wo))
        dt = h.sx_compute_dt(case.cfl)
        ms, kms = time_steps(h, dt, args.steps, args.warmup)
        out[f"{nx}x{ny}x{nz}"] = {"points": case.points, "ms_per_step": ms,
                                  "grind_ms_per_1e8_points": ms * 1e8 / case.points,
                                  "fused_kernel_ms": kms}
        del h, Wo
        torch.cuda.empty_cache()
        progress(f"grid-size sweep {nx}x{ny}x{nz} done")
    return out


def bench_activation_sweep(args):
    """The shock/boundary-layer block 1024x256x128 (FP64, W5 + C6 + V6) with
    seeded random face flags injected at a given fraction of the faces of
    every direction (the sensor pass is replaced by the injected flags):
    RK3 step time against the WENO fraction."""
    import numpy as np
    import torch
    from paper_2304_05494_amd import inputs, sx
    case = inputs.shock_bl_case()
    Wn = np.ascontiguousarray(inputs.fields(case))
    nx, ny, nz = case.nx, case.ny, case.nz
    out = {}
    dt = None
    for frac in (0.0, 0.05, 0.1, 0.25, 0.5, 1.0):
        rng = np.random.Generator(np.random.PCG64(11))
        flags = [(rng.random(shape, dtype=np.float32) < frac).astype(np.uint8)
                 for shape in ((nz, ny, nx + 1), (nz, ny + 1, nx), (nz + 1, ny, nx))]
        h = sx.Handle(case)
        h.sx_bind(h.to_layout(Wn))
        if dt is None:
            dt = h.sx_compute_dt(case.cfl)
        h.sx_set_flag_override(flags)
        ms, kms = time_steps(h, dt, args.steps, args.warmup)
        d = h.sx_diagnostics()
        out[f"{frac:g}"] = {"ms_per_step": ms, "central_kernel_ms": kms,
                            "weno_face_fraction": [float(f.mean()) for f in flags],
                            "state_ok": d.status == sx.SX_OK}
        del h, flags
        progress(f"WENO-activation sweep {frac:g} done")
        torch.cuda.empty_cache()
    base = out["0"]["ms_per_step"]
    for v in out.values():
        v["relative_to_no_weno"] = v["ms_per_step"] / base
    return out


def fp32_error(case, Wn, dt, steps):
    """Per-variable relative L2 and Linf difference between the FP32-flux
    form and the FP64 path after `steps` RK3 steps from the same state."""
    import numpy as np
    import torch
    from paper_2304_05494_amd import sx
    res = []
    for prec in (sx.SX_FP64, sx.SX_FP32_FLUX):
        h = sx.Handle(case, prec)
        h.sx_bind(h.to_layout(Wn))
        for _ in range(steps):
            h.sx_rk3_step(dt)
        torch.cuda.synchronize()
        res.append(h.interior(h.state))
        del h
        torch.cuda.empty_cache()
    a, b = res[1], res[0]
    names = ["rho", "rho_u", "rho_v", "rho_w", "rho_E"]
    out = {}
    for v, nm in enumerate(names):
        d = a[v] - b[v]
        ref2 = float(np.sqrt(np.mean(b[v] ** 2)))
        refi = float(np.abs(b[v]).max())
        # momentum components are scaled by the momentum magnitude
        if 1 <= v <= 3:
            mag = np.sqrt(b[1] ** 2 + b[2] ** 2 + b[3] ** 2)
            ref2, refi = float(np.sqrt(np.mean(mag ** 2))), float(mag.max())
        out[nm] = {"l2_rel": float(np.sqrt(np.mean(d ** 2))) / ref2,
                   "linf_rel": float(np.abs(d).max()) / refi}
    return out


def bench_batch(args, precision, fields=None):
    """The batched form: 48 uneven periodic blocks (TGV / decaying
    turbulence, 32^3 .. 128x64x64), one persistent launch per substep, the
    step replayed from a captured graph, work-item shape autotuned."""
    import numpy as np
    import torch
    from paper_2304_05494_amd import inputs, sx
    cases = inputs.batch_cases(48)
    if fields is None:
        fields = [np.ascontiguousarray(inputs.fields(c)) for c in cases]
    bh = sx.BatchHandle(cases, precision)
    bh.sx_bind(bh.to_arena(fields))
    t = bh.sx_autotune(args.tune_cache)
    dt = bh.sx_compute_dt(0.5)
    for _ in range(args.warmup):
        bh.sx_rk3_step(dt)
    torch.cuda.synchronize()
    bh.sx_timing_enable(True)
    bh.sx_timing_read()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(args.steps):
        bh.sx_rk3_step(dt)
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / args.steps
    n, kms = bh.sx_timing_read()
    d = bh.sx_diagnostics()
    pts = sum(c.points for c in cases)
    alg = ALG_BYTES_PER_POINT_STEP / SUBSTEPS * pts
    out = {
        "value": pts / (ms * 1e-3), "ms_per_step": ms, "blocks": len(cases), "points": pts,
        "launch_ms": kms / n, "roofline_frac": alg / (kms / n * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "tiling": {"tile_x": t.tile_x, "tile_y": t.tile_y, "zchunk": t.zchunk,
                   "workgroups": t.workgroups, "work_items": t.work_items},
        "graph": True, "state_ok": d.status == sx.SX_OK,
    }
    del bh
    torch.cuda.empty_cache()
    return out, fields


def main():
    args = parse()
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2304_05494_amd import inputs, sx

    if args.weno_order_only:
        print(json.dumps({"weno_order_sweep": bench_weno_order_sweep(args)}), flush=True)
        return
    case = inputs.channel_case()
    Wn = np.ascontiguousarray(inputs.fields(case))
    h = sx.Handle(case)
    W0 = h.to_layout(Wn)
    h.sx_bind(W0)
    dt = h.sx_compute_dt(case.cfl)
    for _ in range(args.warmup):
        h.sx_rk3_step(dt)
    torch.cuda.synchronize()

    # REPS repetitions of K timed steps; the median repetition is reported
    h.sx_timing_enable(True)
    h.sx_timing_read()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = []
    wall = 0.0
    for _ in range(args.reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        start.record()
        for _ in range(args.steps):
            h.sx_rk3_step(dt)
        stop.record()
        torch.cuda.synchronize()
        wall += time.perf_counter() - t0
        n_l, k_ms = h.sx_timing_read()
        reps.append((start.elapsed_time(stop), n_l, k_ms))
    h.sx_timing_enable(False)
    reps.sort(key=lambda r: r[0])
    ms_total, launches, kern_ms = reps[len(reps) // 2]

    d = h.sx_diagnostics()
    ok = d.status == sx.SX_OK
    ms_per_step = ms_total / args.steps
    value = case.points / (ms_per_step * 1e-3)
    avg_launch_s = kern_ms / launches * 1e-3
    alg_bytes_launch = ALG_BYTES_PER_POINT_STEP / SUBSTEPS * case.points
    achieved = alg_bytes_launch / avg_launch_s / 1e9
    kernel = "k_rhs_central<3, 3, 32, 8, 2, double, true, false, true, 0>"
    traffic = load_traffic(kernel)
    line = {
        "metric": "grid-point updates/s per RK3 step (FP64 vs FP32-flux) + % HBM roofline",
        "value": value,
        "unit": "grid-point updates/s per RK3 step",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "channel-like block 512x256x256 FP64: periodic x/z, isothermal no-slip "
                        "walls in y (tanh stretching beta=1.8), bulk Mach 1.5, Re_b 6000, "
                        "laminar profile + 5% seeded Gaussian velocity noise (seed 2), "
                        "C6 central split-form convection + V6 Laplacian viscous terms, "
                        "RK3 (Wray) at CFL 0.5",
            "nx": case.nx, "ny": case.ny, "nz": case.nz, "points": case.points,
            "dt": dt, "precision": "fp64",
        },
        "alg_fraction": value * ALG_BYTES_PER_POINT_STEP / (HBM_PEAK_GBS * 1e9),
        "roofline": {
            "bound": "hbm",
            "kernel": kernel,
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": None if traffic is None else traffic,
            # counter bytes (FETCH_SIZE x 2 + WRITE_SIZE, copy-calibrated) over the live launch time
            "hw_frac": None if traffic is None else traffic / avg_launch_s / 1e9 / HBM_PEAK_GBS,
            "launch_ms": avg_launch_s * 1e3,
            "launches": launches,
            "alg_bytes_per_launch": alg_bytes_launch,
        },
        "state_ok": ok,
        "timing": f"median of {args.reps} repetitions of {args.steps} steps (HIP events on the bound stream)",
        "ms_per_step_reps": [r[0] / args.steps for r in reps],
        "wall_s_timed": wall,
    }
    fl = load_flops(kernel)
    if fl is not None:
        tf = fl["fp64_flops_per_launch"] / avg_launch_s / 1e12
        line["valu"] = {"bound": "alu", "achieved": tf, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                        "frac": tf / FP64_PEAK_TFLOPS,
                        "flops_per_launch": fl["fp64_flops_per_launch"],
                        "source": "SQ_INSTS_VALU_*_F64 counters (profiles/valu_flops.json) / live launch time"}
    # the same workload in the FP32-flux precision form
    h32 = sx.Handle(case, precision=sx.SX_FP32_FLUX)
    W32 = h32.to_layout(Wn)
    h32.sx_bind(W32)
    ms32, l32 = time_steps(h32, dt, args.steps, args.warmup, args.reps)
    fl32 = load_flops("k_rhs_central<3, 3, 64, 8, 2, float, true, false, false, 0>")
    line["fp32_flux"] = {
        "valu_fp32_tflops": None if fl32 is None else fl32["fp32_flops_per_launch"] / (l32 * 1e-3) / 1e12,
        "value": case.points / (ms32 * 1e-3),
        "ms_per_step": ms32,
        "speedup_vs_fp64": ms_per_step / ms32,
        "launch_ms": l32,
        "roofline_frac": ALG_BYTES_PER_POINT_STEP / SUBSTEPS * case.points / (l32 * 1e-3) / 1e9 / HBM_PEAK_GBS,
    }
    del h32, W32
    if not args.no_batch:
        b64, bf = bench_batch(args, sx.SX_FP64)
        b32, _ = bench_batch(args, sx.SX_FP32_FLUX, bf)
        b32["speedup_vs_fp64"] = b64["ms_per_step"] / b32["ms_per_step"]
        line["batched"] = {"workload": "48 periodic blocks (seed 5; sizes 32^3, 48^3, 64^3, 96^3, "
                                       "128x64x64; TGV or decaying turbulence; Mach 0.1-0.5), "
                                       "C6 + V6, one graph-replayed persistent launch per substep",
                           "fp64": b64, "fp32_flux": b32}
    if not args.no_legs:
        line["tgv32"] = bench_tgv(args)
        line["shock_bl"] = bench_shock_bl(args)
        line["fp32_flux"]["error_vs_fp64_after_100_steps"] = fp32_error(case, Wn, dt, 100)
    if args.sweep_f2:
        line["visc_order_sweep"] = bench_visc_order_sweep(args, Wn, dt)
        line["weno_order_sweep"] = bench_weno_order_sweep(args)
        line["thread_masking"] = bench_thread_masking(args)
        line["grid_size_sweep"] = bench_grid_size_sweep(args)
    if args.sweep:
        line["order_sweep"] = bench_order_sweep(args, Wn, dt)
        line["weno_activation_sweep"] = bench_activation_sweep(args)
    if not args.no_cpu_baseline:
        del h, W0
        torch.cuda.empty_cache()
        line["cpu_baseline"] = cpu_baseline(case, Wn, dt, args.cpu_sample_steps)
    else:
        line["cpu_baseline"] = None
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
