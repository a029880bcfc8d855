#!/usr/bin/env python3
"""Benchmark of the batched orthonormal 2D DCT on one MI355X.

Workload (one "step"): the six square sizes N = 8, 16, 32, 64, 128, 256, each a batch
of 2^27 / N^2 row-major float32 arrays (512 MiB) of seeded N(0,1) values resident in
HBM, transformed in place by the forward, inverse and fused round-trip calls of the C
ABI (18 calls).  Algorithmic traffic is one float32 read and one float32 write per
element per call (8 N^2 bytes per array), so the step moves 18 x 1 GiB.

Before any timing, every call is checked on a full-size copy of its batch, on every
array, against closed forms that need no oracle (the round trip returns its input;
forward and inverse keep each array's norm and invert each other).

Reported: whole-step GB/s; per size and direction the median over 21 individually
timed calls with a bootstrap 95 % interval, GB/s, transforms/s and the fractions of
the 8 TB/s peak and of the library's copy kernel timed in the same run; the
roofline of the dominant kernel (HIP events on the stream the kernels run on); the
float32 vs split-precision matrix paths on the C3 arrays (N <= 64) and on the C2
mixture (65536 16x16 tiles, eight rotating buffer sets) in all three directions; the
spectral filter, rectangle orientations and the ragged C4 batch.  The CPU-baseline leg
times the FP64 oracle on a bounded sample of the same arrays on the host cores and
scores every reported GPU configuration against it (e_rel of Section 6 eq. 5 on
arrays spread over each batch), plus the boundary diagnostics of Section 6.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "2D DCT GB/s & %HBM peak, N=8..256 fp32; split-BF16 MFMA vs plain FP32"
HBM_PEAK_GBS = 8000.0
SIZES = (8, 16, 32, 64, 128, 256)
DIRS = ("forward", "inverse", "roundtrip")
GATE = {"forward": 2e-6, "inverse": 2e-6, "roundtrip": 4e-6}
PATHS = ("fp32", "bf16x3", "bf16x6", "fp16x3", "bf16", "fp16", "fp8")
C2_PATHS = ("fp32", "bf16x3", "bf16x6", "fp16x3")
SAMPLES = 64  # arrays per configuration scored against the oracle


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--reps", type=int, default=21, help="individually timed calls per case (median, CI)")
    ap.add_argument("--sizes", default=",".join(map(str, SIZES)))
    ap.add_argument("--precision", default="auto", help="path used by the step (auto = library default)")
    ap.add_argument("--compare", default=",".join(PATHS),
                    help="paths timed per size (N<=64) for the float32 vs split comparison")
    ap.add_argument("--cpu-frac", type=float, default=0.75, help="fraction of each batch the oracle is timed on")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle leg (timing and every e_rel)")
    ap.add_argument("--log2-floats", type=int, default=27, help="floats per size (default 2^27 = 512 MiB)")
    ap.add_argument("--no-tune", action="store_true", help="skip the (untimed) autotuning pass")
    ap.add_argument("--save-policy", default="", help="write the tuned policy (autotune cache, JSON) here")
    ap.add_argument("--load-policy", default="", help="freeze this saved policy instead of tuning")
    ap.add_argument("--no-ragged", action="store_true", help="skip the ragged-batch (one graph launch) measurement")
    ap.add_argument("--no-filter", action="store_true", help="skip the spectral-filter measurement")
    ap.add_argument("--no-rect", action="store_true",
                    help="skip the rectangle-orientation and long-axis (512, 1024) measurements")
    ap.add_argument("--no-c2", action="store_true", help="skip the C2 mixture timing")
    return ap.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# ---- timing statistics ----------------------------------------------------------------------

def median_ci(ms, boot=2000, seed=0):
    """Median of the timings and a bootstrap 95 % interval of the median."""
    a = np.asarray(ms, np.float64)
    g = np.random.default_rng(seed)
    meds = np.median(a[g.integers(0, a.size, (boot, a.size))], axis=1)
    return float(np.median(a)), float(np.percentile(meds, 2.5)), float(np.percentile(meds, 97.5))


def time_calls(fn, reps, stream):
    """Times `reps` calls of fn(i) one by one with HIP events on `stream`; list of ms."""
    import torch
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for i, (a, b) in enumerate(ev):
        a.record(stream)
        fn(i)
        b.record(stream)
    torch.cuda.synchronize()
    return [a.elapsed_time(b) for a, b in ev]


def rate(nbytes, ms, transforms=None, copy_gbs=None):
    """GB/s row of one case from its timings (median over reps, 95 % bootstrap interval)."""
    med, lo, hi = median_ci(ms)
    gbs = nbytes / (med * 1e-3) / 1e9
    row = {"ms": round(med, 5), "ms_ci95": [round(lo, 5), round(hi, 5)], "reps": len(ms),
           "GB/s": round(gbs, 1), "GB/s_ci95": [round(nbytes / (hi * 1e-3) / 1e9, 1),
                                               round(nbytes / (lo * 1e-3) / 1e9, 1)],
           "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}
    if transforms is not None:
        row["transforms_per_s"] = round(transforms / (med * 1e-3), 1)
    if copy_gbs:
        row["copy_frac"] = round(gbs / copy_gbs, 4)
    return row


# ---- pre-timing self-check (closed forms, no oracle) ------------------------------------------

def per_array(t, ref):
    """||t_i - ref_i|| / ||ref_i|| over every array (float64 on the GPU)."""
    import torch
    d = (t.double() - ref.double()).reshape(t.shape[0], -1)
    n = ref.double().reshape(ref.shape[0], -1)
    return torch.linalg.vector_norm(d, dim=1) / torch.linalg.vector_norm(n, dim=1)


def norm_change(t, ref):
    import torch
    a = torch.linalg.vector_norm(t.double().reshape(t.shape[0], -1), dim=1)
    b = torch.linalg.vector_norm(ref.double().reshape(ref.shape[0], -1), dim=1)
    return (a - b).abs() / b


def self_check(dct, bufs, sizes, precision, stream):
    """Every call the step times, on a full-size copy, in its timed launch configuration; every
    array checked.  Round trip: returns its input within 4e-6.  Forward (inverse): keeps each
    array's norm within 2e-6, and the opposite call returns the input within 4e-6."""
    report = {}
    for n in sizes:
        x = bufs[n]
        worst = {}
        t = x.clone()
        dct.transform(t, t, "roundtrip", precision, stream=stream)
        worst["roundtrip"] = float(per_array(t, x).max())
        for d, back in (("forward", "inverse"), ("inverse", "forward")):
            t.copy_(x)
            dct.transform(t, t, d, precision, stream=stream)
            worst[d + "_norm"] = float(norm_change(t, x).max())
            dct.transform(t, t, back, precision, stream=stream)
            worst[d + "_then_" + back] = float(per_array(t, x).max())
        del t
        ok = (worst["roundtrip"] <= GATE["roundtrip"] and worst["forward_norm"] <= GATE["forward"]
              and worst["inverse_norm"] <= GATE["inverse"] and worst["forward_then_inverse"] <= GATE["roundtrip"]
              and worst["inverse_then_forward"] <= GATE["roundtrip"])
        if not ok:
            log("self-check failed N=%d: %s" % (n, worst))
            sys.exit(1)
        report[str(n)] = {k: float("%.3e" % v) for k, v in worst.items()}
    import torch
    torch.cuda.empty_cache()
    return report


# ---- main -----------------------------------------------------------------------------------

def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the batched transform needs no communication, "
              "a multi-GPU run would be N independent copies of this one, each on its share of the "
              "arrays.", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2609_28519_amd as dct
    import workloads

    sizes = [int(s) for s in args.sizes.split(",") if s]
    dct.init(0)
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()

    # ---- inputs resident in HBM ----------------------------------------------------------
    host = {}
    bufs = {}
    for n in sizes:
        batch = (1 << args.log2_floats) // (n * n)
        x = workloads.c3_normal(n, batch=batch).x
        host[n] = x
        bufs[n] = torch.from_numpy(x).to(dev)
        log("input N=%d batch=%d (%.0f MiB)" % (n, batch, x.nbytes / 2 ** 20))
    torch.cuda.synchronize()

    # ---- autotune (untimed, on the library's own scratch data, before any measurement) ----
    tuned = {}
    if args.load_policy:
        dct.load_policy(args.load_policy)
    elif not args.no_tune:
        for n in sizes:
            for d in DIRS:
                # tunes the variants of every float32-accurate path, freezes the fastest path for "auto"
                dct.tune(n, n, d, "auto", batch=(1 << args.log2_floats) // (n * n), stream=stream)
            if not args.no_filter:
                dct.tune(n, n, "filter", "fp32", batch=(1 << args.log2_floats) // (n * n), stream=stream)
        torch.cuda.synchronize()
        log("tuned")
    if args.save_policy:
        dct.save_policy(args.save_policy)
    for n in sizes:
        for d in DIRS:
            path = dct.get_variant(n, n, d, "auto")
            name = {v: k for k, v in dct.PRECISIONS.items()}[path]
            tuned["%d/%s" % (n, d)] = "%s/v%d" % (name, dct.get_variant(n, n, d, name))
        tuned["%d/filter" % n] = "fp32/v%d" % dct.get_variant(n, n, "filter", "fp32")

    def call(n, d, prec, t):
        return dct.transform(t, t, d, prec, stream=stream)

    checked = self_check(dct, bufs, sizes, args.precision, stream)
    log("self-check passed")

    # ---- warmup + timed steps --------------------------------------------------------------
    for _ in range(args.warmup):
        for n in sizes:
            for d in DIRS:
                call(n, d, args.precision, bufs[n])
    torch.cuda.synchronize()
    ev = {(n, d): [] for n in sizes for d in DIRS}
    step_start = torch.cuda.Event(enable_timing=True)
    step_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step_start.record(stream)
    for _ in range(args.steps):
        for n in sizes:
            for d in DIRS:
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                a.record(stream)
                call(n, d, args.precision, bufs[n])
                b.record(stream)
                ev[(n, d)].append((a, b))
    step_end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    total_ms = step_start.elapsed_time(step_end)
    ms_per_step = total_ms / args.steps
    bytes_per_step = sum(8 * n * n * host[n].shape[0] for n in sizes) * len(DIRS)
    value = bytes_per_step / (ms_per_step * 1e-3) / 1e9
    step_call_ms = {k: float(np.mean([a.elapsed_time(b) for a, b in v])) for k, v in ev.items()}
    log("timed %d steps: %.3f ms/step" % (args.steps, ms_per_step))

    # ---- the copy ceiling (library kernel, same run) ---------------------------------------
    copy_rows = copy_ceiling(dct, bufs[sizes[0]], stream, args.reps)
    copy_gbs = copy_rows["out_of_place"]["GB/s"]
    valu = valu_ceiling(dct, stream)

    # ---- per-case statistics: 21 individually timed calls each -------------------------------
    per = {}
    for n in sizes:
        per[str(n)] = {}
        nb = 8 * n * n * host[n].shape[0]
        for d in DIRS:
            ms = time_calls(lambda i: call(n, d, args.precision, bufs[n]), args.reps, stream)
            per[str(n)][d] = rate(nb, ms, host[n].shape[0], copy_gbs)
            per[str(n)][d]["step_mean_ms"] = round(step_call_ms[(n, d)], 5)
            per[str(n)][d]["variant"] = tuned["%d/%s" % (n, d)]

    # dominant kernel: the call with the largest share of the step among calls that are one
    # kernel launch (the event pair then brackets exactly that kernel); its average over the
    # timed steps
    names = {(n, d): kernel_name(n, d, tuned["%d/%s" % (n, d)]) for n in sizes for d in DIRS}
    single = [k for k in names if names[k]]
    dom = max(single, key=lambda k: step_call_ms[k]) if single else max(step_call_ms, key=step_call_ms.get)
    n_dom, d_dom = dom
    alg_bytes = 8 * n_dom * n_dom * host[n_dom].shape[0]
    achieved = alg_bytes / (step_call_ms[dom] * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": counted_traffic(names[dom]) if names.get(dom) else None,
                "kernel": names.get(dom) or "%s N=%d" % (d_dom, n_dom), "call": "%s N=%d" % (d_dom, n_dom),
                "avg_ms": round(step_call_ms[dom], 5), "algorithmic_bytes_per_launch": alg_bytes,
                "copy_frac": round(achieved / copy_gbs, 4)}

    # ---- float32 vs split-precision matrix paths on the C3 arrays (N <= 64) -------------------
    compare = compare_paths(dct, bufs, host, sizes, [p for p in args.compare.split(",") if p], stream, args.reps,
                            copy_gbs)
    c2 = None if args.no_c2 else c2_rates(dct, stream, args.reps, copy_gbs)
    filt = None if args.no_filter else filter_rates(dct, bufs, host, sizes, stream, per, args.reps)
    rect = None if args.no_rect else rect_rates(dct, bufs[sizes[0]], stream,
                                                tune=not (args.no_tune or args.load_policy))
    long_axes = None if args.no_rect else long_axis_rates(dct, bufs[sizes[0]], stream)
    ragged = None if args.no_ragged else ragged_c4(dct, stream, args.reps)
    del bufs
    torch.cuda.empty_cache()

    out = {"metric": METRIC, "value": round(value, 1), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "six square sizes N=8..256, 2^%d float32 per size (batch 2^%d/N^2), N(0,1); "
                                  "forward + inverse + fused round trip, in place" % (args.log2_floats,
                                                                                     args.log2_floats),
                      "sizes": sizes, "batch": {str(n): int(host[n].shape[0]) for n in sizes},
                      "precision": args.precision, "variants": tuned},
           "hbm_frac": round(value / HBM_PEAK_GBS, 4), "copy_ceiling_GBps": round(copy_gbs, 1),
           "copy": copy_rows, "valu_ceiling": valu, "wall_s": round(wall, 3), "self_check": checked,
           "roofline": roofline, "per_size": per, "compare": compare, "c2_mixture": c2, "ragged_c4": ragged,
           "filter": filt, "rectangles": rect, "long_axes": long_axes}

    # ---- CPU baseline: the FP64 oracle timed on the host, and every row scored against it ------
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(dct, host, sizes, args, out, stream)
    print(json.dumps(out), flush=True)


# ---- reported beside the step -------------------------------------------------------------------

def copy_ceiling(dct, buf, stream, reps):
    """The library's reference copy kernel (dct2d_copy) over one 512 MiB buffer, out of place and in
    place: one read and one write per element, the practical ceiling of a transform."""
    import torch
    out = torch.empty_like(buf)
    dct.copy(buf, out, stream=stream)
    nb = 2 * buf.numel() * 4
    rows = {"out_of_place": rate(nb, time_calls(lambda i: dct.copy(buf, out, stream=stream), reps, stream))}
    rows["in_place"] = rate(nb, time_calls(lambda i: dct.copy(out, out, stream=stream), reps, stream))
    del out
    torch.cuda.empty_cache()
    return rows


def compare_paths(dct, bufs, host, sizes, paths, stream, reps, copy_gbs):
    """Every arithmetic path on the same C3 arrays (N <= 64), out of place, all three directions."""
    import torch
    res = {}
    for n in sizes:
        if n > 64:
            continue
        scratch = torch.empty_like(bufs[n])
        for p in paths:
            for d in DIRS:
                try:
                    dct.transform(bufs[n], scratch, d, p, stream=stream)
                except dct.DCT2DError:
                    continue
                ms = time_calls(lambda i: dct.transform(bufs[n], scratch, d, p, stream=stream), reps, stream)
                res.setdefault(p, {}).setdefault(str(n), {})[d] = rate(8 * n * n * host[n].shape[0], ms,
                                                                      host[n].shape[0], copy_gbs)
        del scratch
    torch.cuda.empty_cache()
    return res


C2_SETS = 8


def c2_rates(dct, stream, reps, copy_gbs):
    """The C2 mixture (65536 16x16 tiles: uniform, normal, ramps with a 1e-6 component, 2^+-100
    amplitudes) through the float32 and split-precision paths in all three directions, out of place,
    rotating over 8 buffer sets (512 MiB of inputs) so the 256 MB memory-side cache cannot serve
    them."""
    import torch

    import workloads
    sets = [torch.from_numpy(workloads.c2_mixture16(seed=workloads.SEEDS["c2"] + s).x).cuda()
            for s in range(C2_SETS)]
    outs = [torch.empty_like(sets[0]) for _ in range(C2_SETS)]
    nb = 8 * sets[0].numel()
    res = {}
    for p in C2_PATHS:
        for d in DIRS:
            try:
                dct.transform(sets[0], outs[0], d, p, stream=stream)
            except dct.DCT2DError:
                continue
            ms = time_calls(lambda i: dct.transform(sets[i % C2_SETS], outs[i % C2_SETS], d, p, stream=stream),
                            reps, stream)
            res.setdefault(p, {})[d] = rate(nb, ms, sets[0].shape[0], copy_gbs)
    del sets, outs
    torch.cuda.empty_cache()
    return res


def poisson_multipliers(n):
    """Neumann Poisson solve on an n x n grid: 1 / (2 cos(pi k/n) + 2 cos(pi l/n) - 4), 0 at (0, 0)."""
    k = np.arange(n)[:, None]
    l = np.arange(n)[None, :]
    mu = 2.0 * np.cos(np.pi * k / n) + 2.0 * np.cos(np.pi * l / n) - 4.0
    lam = np.zeros((n, n))
    lam[mu != 0] = 1.0 / mu[mu != 0]
    return lam.astype(np.float32)


def filter_rates(dct, bufs, host, sizes, stream, per, reps):
    """The fused spectral filter (Prop. 1, eq. 4) on the same batches, one shared Poisson
    operator, out of place: one read and one write per array like the round trip, so its
    GB/s uses the same 8 N^2 bytes per array.  Reported beside the step, not part of it."""
    import torch
    res = {}
    for n in sizes:
        lam = torch.from_numpy(poisson_multipliers(n)).to(bufs[n].device)
        scratch = torch.empty_like(bufs[n])
        dct.filter(bufs[n], lam, out=scratch, stream=stream)
        ms = time_calls(lambda i: dct.filter(bufs[n], lam, out=scratch, stream=stream), reps, stream)
        res[str(n)] = rate(8 * n * n * host[n].shape[0], ms, host[n].shape[0])
        res[str(n)]["vs_roundtrip"] = round(res[str(n)]["GB/s"] / per[str(n)]["roundtrip"]["GB/s"], 3)
        del scratch
    torch.cuda.empty_cache()
    return res


RECT_PAIRS = ((8, 64), (64, 8), (16, 32), (32, 16), (8, 256), (256, 8), (32, 256), (256, 32), (64, 256), (256, 64),
              (128, 256), (256, 128))
# shapes with an axis of 512 or 1024 (the two-pass long-axis kernels behind the basic calls)
LONG_SHAPES = ((512, 512), (1024, 1024), (8, 1024), (1024, 64), (512, 64), (64, 512))


def rect_rates(dct, buf, stream, tune=True, reps=9):
    """Orientation of rectangles (Section 7.1): h x w against w x h on the same 2^27 floats
    (the batch buffer of the first size, viewed as (2^27 / (h w), h, w)), out of place, float32
    path, each (shape, direction) autotuned first (untimed) like the square sizes; GB/s of
    8 h w bytes per array.  Reported beside the step, not part of it."""
    import torch
    res = {}
    scratch = torch.empty_like(buf)
    for h, w in RECT_PAIRS:
        batch = buf.numel() // (h * w)
        x = buf[:batch * h * w].view(batch, h, w)
        y = scratch[:batch * h * w].view(batch, h, w)
        key = "%dx%d" % (h, w)
        res[key] = {}
        for d in DIRS:
            if tune:
                dct.tune(h, w, d, "fp32", batch=batch, stream=stream)
            res[key]["variant/" + d] = dct.get_variant(h, w, d, "fp32")
            dct.transform(x, y, d, "fp32", stream=stream)
            ms = time_calls(lambda i: dct.transform(x, y, d, "fp32", stream=stream), reps, stream)
            res[key][d] = rate(8 * h * w * batch, ms, batch)
    del scratch
    torch.cuda.empty_cache()
    return res


def long_axis_rates(dct, buf, stream, reps=5):
    """Axes of 512 and 1024 through the basic calls (a row pass and an in-place column pass of the
    long-axis kernels; an axis <= 256 of such a shape runs the short line passes), out of place on
    the same 2^27 floats; GB/s of 8 h w bytes per array.  Reported beside the step, not part of it."""
    import torch
    res = {}
    scratch = torch.empty_like(buf)
    for h, w in LONG_SHAPES:
        batch = buf.numel() // (h * w)
        x = buf[:batch * h * w].view(batch, h, w)
        y = scratch[:batch * h * w].view(batch, h, w)
        key = "%dx%d" % (h, w)
        res[key] = {}
        for d in DIRS:
            dct.transform(x, y, d, "fp32", stream=stream)
            ms = time_calls(lambda i: dct.transform(x, y, d, "fp32", stream=stream), reps, stream)
            res[key][d] = rate(8 * h * w * batch, ms, batch)
    del scratch
    torch.cuda.empty_cache()
    return res


def valu_ceiling(dct, stream, iters=4096):
    """The vector-ALU issue reference (dct2d_fma_issue): independent float32 FMAs with 1, 2, 4 and 8
    wavefronts per SIMD; wave64 instructions issued per SIMD and cycle (at the nominal 2.4 GHz) and the
    FMA rate in TFLOP/s.  The VALU share of a kernel is judged against the rate at its occupancy."""
    import torch
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    sink = torch.zeros(1, device="cuda")
    res = {"cus": cus, "clock_GHz": 2.4, "iters": iters}
    for w in (1, 2, 4, 8):
        blocks = cus * w
        dct.fma_issue(sink, blocks, 64, stream=stream)
        ms = float(np.median(time_calls(lambda i: dct.fma_issue(sink, blocks, iters, stream=stream), 5, stream)))
        instr = 16.0 * iters * 4 * blocks
        per = instr / (ms * 1e-3 * 2.4e9 * cus * 4)
        res["waves_per_simd_%d" % w] = {"ms": round(ms, 4), "instr_per_cycle_per_simd": round(per, 4),
                                        "fma_TFLOPs": round(instr * 64 * 2 / (ms * 1e-3) / 1e12, 1)}
    return res


def ragged_c4(dct, stream, reps):
    """The ragged configuration: 200k blocks (8..256) + 4 x 1024^2 + 4 x 512x384 images, U[-1,1] with 5%
    of items x 1e30, forward in place, one hipGraphLaunch per execution (plan recorded before timing)."""
    import torch

    import workloads
    rg = workloads.c4_ragged()
    buf = torch.from_numpy(rg.data).cuda()
    plan = dct.RaggedPlan(rg.offsets, rg.rows, rg.cols, "forward", "auto")
    info = plan.info()
    plan.execute(buf, stream)
    ms = time_calls(lambda i: plan.execute(buf, stream), reps, stream)
    alg = int(8 * (rg.rows.astype(np.int64) * rg.cols).sum())
    plan.close()
    del buf
    torch.cuda.empty_cache()
    row = rate(alg, ms, rg.count)
    row.update({"items": info["items"], "classes": info["classes"], "graph_nodes": info["graph_nodes"],
                "launches_per_execution": 1, "algorithmic_bytes": alg})
    return row


def kernel_name(n, d, tuned):
    """Kernel that one call launches (as rocprofv3 names it), or None for multi-kernel schedules.
    `tuned` is "path/vK" as frozen by the policy."""
    path, v = tuned.split("/v")
    v = int(v)
    di = DIRS.index(d)
    if path != "fp32":
        return None
    if n <= 64:
        if n == 64 and v >= 13:
            return "k_split64<%d>" % di
        if v == 0 or v >= 3:
            stage = v == 4 or (v >= 5 and (v - 5) % 2 == 1)
            return "k_wave<%d, %d, %d, %s>" % (n, n, di, "true" if stage else "false")
        return "k_fused<%d, %d, %d>" % (n, n, di) if v == 1 else None
    if n == 128:
        if v == 0 or v >= 3:
            return "k_split128<%d, %s>" % (di, "true" if v in (3, 4) else "false")
        return "k_fused<128, 128, %d>" % di if v == 1 else None
    if n == 256:
        return None if v == 1 else "k_split256<%d>" % di
    return None


KERNEL_SOURCES = ("kern_fp32.hip", "kern_rect256.hip", "fp32_common.hpp", "split256.hpp", "dct1d.hpp", "internal.hpp")


def source_digest():
    """SHA-256 over the sources of the float32 transform kernels; ties counter-derived traffic figures
    to the kernel code they measured."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2609_28519_amd", "csrc")
    for name in KERNEL_SOURCES:
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def counted_traffic(kernel):
    """Calibrated HBM bytes per dispatch of `kernel` (FETCH_SIZE x fetch factor + WRITE_SIZE x write
    factor, from two rocprofv3 counter passes, recorded in profiles/hbm_traffic.json), or None when
    the counters were taken on other kernel sources or do not cover this kernel."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256") != source_digest() or kernel not in rec.get("kernels", {}):
        return None
    k = rec["kernels"][kernel]
    return int(k["read_bytes"] + k["write_bytes"])


# ---- the oracle leg ------------------------------------------------------------------------------

def spread(batch, k, seed):
    """About k array indices spread over the whole batch (one per equal segment, first and last)."""
    g = np.random.default_rng(seed)
    k = max(1, min(k, batch))
    edges = np.linspace(0, batch, k + 1).astype(np.int64)
    idx = [int(g.integers(lo, hi)) for lo, hi in zip(edges[:-1], edges[1:]) if hi > lo]
    return np.unique(np.array(idx + [0, batch - 1], dtype=np.int64))


def cpu_baseline(dct, host, sizes, args, out, stream):
    """Times the FP64 oracle (as it stands) on the first `cpu_frac` of every size's arrays, on the host's
    cores, for forward, inverse and round trip; then scores the GPU result of every reported
    configuration against the oracle: the calls are repeated once on fresh copies of their inputs in
    the launch configuration that was timed, and arrays spread over each batch are compared (e_rel of
    Section 6 eq. 5; the round trip against its input).  The errors are written into the rows above."""
    import oracle
    threads = oracle.default_threads()
    total_bytes = 0
    total_s = 0.0
    for n in sizes:
        m = max(1, int(host[n].shape[0] * args.cpu_frac))
        xs = host[n][:m]
        t0 = time.perf_counter()
        oracle.forward(xs, threads=threads)
        oracle.inverse(xs, threads=threads)
        oracle.roundtrip(xs, threads=threads)
        total_s += time.perf_counter() - t0
        total_bytes += 8 * n * n * m * 3
    log("oracle timed: %.1f s" % total_s)
    res = {"value": round(total_bytes / total_s / 1e9, 4), "unit": "GB/s", "cores": threads, "kind": "oracle",
           "sample": "first %.0f%% of each size's C3 batch (forward + inverse + round trip, FP64 direct "
                     "definition, %d threads)" % (100 * args.cpu_frac, threads),
           "seconds": round(total_s, 2)}
    res["e_rel_max"] = score_all(dct, oracle, host, sizes, args, out, stream)
    return res


def _refs(oracle, xs):
    return {"forward": oracle.forward(xs), "inverse": oracle.inverse(xs), "roundtrip": xs.astype(np.float64)}


def _sampled_output(dct, x_host, idx, d, prec, stream, inplace=True):
    import torch
    t = torch.from_numpy(x_host).cuda()
    o = t if inplace else torch.empty_like(t)
    dct.transform(t, o, d, prec, stream=stream)
    torch.cuda.synchronize()
    y = o[torch.from_numpy(idx).cuda()].cpu().numpy()
    del t, o
    return y


def score_all(dct, oracle, host, sizes, args, out, stream):
    """e_rel (max over sampled arrays) of every row; also written into each row as "e_rel"."""
    import torch

    import workloads
    summary = {}
    # the step's calls, in place, full size
    for n in sizes:
        idx = spread(host[n].shape[0], SAMPLES, n)
        xs = host[n][idx]
        refs = _refs(oracle, xs)
        for d in DIRS:
            e = float(oracle.e_rel(_sampled_output(dct, host[n], idx, d, args.precision, stream), refs[d], xs).max())
            out["per_size"][str(n)][d]["e_rel"] = float("%.3e" % e)
            out["per_size"][str(n)][d]["gate"] = GATE[d]
            summary["%d/%s" % (n, d)] = float("%.3e" % e)
        # every compared path (out of place, as timed)
        for p, rows in out["compare"].items():
            if str(n) in rows:
                for d in rows[str(n)]:
                    e = float(oracle.e_rel(_sampled_output(dct, host[n], idx, d, p, stream, False), refs[d],
                                           xs).max())
                    rows[str(n)][d]["e_rel"] = float("%.3e" % e)
        torch.cuda.empty_cache()
    log("scored the step and the paths")
    # C2 mixture: the first buffer set, every tile, per category, plus the weak-component error
    if out.get("c2_mixture"):
        bt = workloads.c2_mixture16()
        refs = _refs(oracle, bt.x)
        ramp = np.flatnonzero(bt.category == workloads.CAT_RAMP_WEAK)
        for p, rows in out["c2_mixture"].items():
            for d in rows:
                y = _sampled_output(dct, bt.x, np.arange(bt.x.shape[0]), d, p, stream, False)
                e = oracle.e_rel(y, refs[d], bt.x)
                rows[d]["e_rel"] = float("%.3e" % e.max())
                rows[d]["e_rel_by_category"] = {int(c): float("%.3e" % e[bt.category == c].max())
                                                for c in np.unique(bt.category)}
                if d == "forward":
                    w = [oracle.weak_component_error(y[i], refs[d][i], *bt.weak_kl[i]) for i in ramp]
                    rows[d]["weak_component_rel_error"] = {"median": float("%.3e" % np.median(w)),
                                                           "max": float("%.3e" % np.max(w))}
        log("scored C2")
    # filter (Poisson operator), out of place: ||X'_gpu - X'_oracle|| / (max|L| ||X||)
    if out.get("filter"):
        for n in sizes:
            idx = spread(host[n].shape[0], SAMPLES, 3 * n)
            xs = host[n][idx]
            lam = poisson_multipliers(n)
            t = torch.from_numpy(host[n]).cuda()
            o = dct.filter(t, torch.from_numpy(lam).cuda(), stream=stream)
            torch.cuda.synchronize()
            y = o[torch.from_numpy(idx).cuda()].cpu().numpy()
            del t, o
            ref = oracle.filter(xs, lam.astype(np.float64))
            num = np.sqrt(((y - ref) ** 2).sum(axis=(1, 2)))
            den = np.abs(lam).max() * np.sqrt((xs.astype(np.float64) ** 2).sum(axis=(1, 2)))
            out["filter"][str(n)]["e_rel"] = float("%.3e" % (num / den).max())
        torch.cuda.empty_cache()
    # rectangles, out of place, in the tuned variants
    if out.get("rectangles"):
        base = host[sizes[0]].reshape(-1)
        for key, row in out["rectangles"].items():
            h, w = (int(v) for v in key.split("x"))
            batch = base.size // (h * w)
            x = base[:batch * h * w].reshape(batch, h, w)
            idx = spread(batch, 32, h * 7 + w)
            xs = x[idx]
            refs = _refs(oracle, xs)
            for d in DIRS:
                y = _sampled_output(dct, x, idx, d, "fp32", stream, False)
                row[d]["e_rel"] = float("%.3e" % oracle.e_rel(y, refs[d], xs).max())
        torch.cuda.empty_cache()
    # axes of 512 and 1024 through the basic calls, out of place
    if out.get("long_axes"):
        base = host[sizes[0]].reshape(-1)
        for key, row in out["long_axes"].items():
            h, w = (int(v) for v in key.split("x"))
            batch = base.size // (h * w)
            x = base[:batch * h * w].reshape(batch, h, w)
            idx = spread(batch, 6, h + 3 * w)
            xs = x[idx]
            refs = _refs(oracle, xs)
            for d in DIRS:
                y = _sampled_output(dct, x, idx, d, "fp32", stream, False)
                row[d]["e_rel"] = float("%.3e" % oracle.e_rel(y, refs[d], xs).max())
        torch.cuda.empty_cache()
    # ragged C4: per shape class, up to 24 items (2 per image class)
    if out.get("ragged_c4"):
        rg = workloads.c4_ragged()
        buf = torch.from_numpy(rg.data).cuda()
        plan = dct.RaggedPlan(rg.offsets, rg.rows, rg.cols, "forward", "auto")
        plan.execute(buf, stream)
        torch.cuda.synchronize()
        got = buf.cpu().numpy()
        plan.close()
        del buf
        by_class = {}
        g = np.random.default_rng(4)
        shapes = sorted(set(zip(rg.rows.tolist(), rg.cols.tolist())))
        for h, w in shapes:
            members = np.flatnonzero((rg.rows == h) & (rg.cols == w))
            pick = members if members.size <= 2 else g.choice(members, 2 if max(h, w) > 256 else 24, replace=False)
            worst = 0.0
            for i in pick:
                xi = rg.item(int(i))
                yi = rg.item(int(i), got)
                worst = max(worst, float(oracle.e_rel(yi, oracle.forward(xi), xi)[0]))
            by_class["%dx%d" % (h, w)] = float("%.3e" % worst)
        out["ragged_c4"]["e_rel_by_class"] = by_class
        out["ragged_c4"]["e_rel"] = max(by_class.values())
        torch.cuda.empty_cache()
    # boundary diagnostics (Section 6), reported, not gated
    diag = {}
    for n in sizes:
        bs = workloads.boundary_set(n)
        finite = [i for i in range(bs.x.shape[0]) if np.isfinite(bs.x[i]).all()]
        refs = _refs(oracle, bs.x[finite])
        cell = {}
        for d in DIRS:
            y = _sampled_output(dct, bs.x, np.arange(bs.x.shape[0]), d, args.precision, stream, False)
            for i, name in enumerate(workloads.BOUNDARY_CASES):
                fin = float(np.isfinite(y[i]).mean())
                entry = {"finite_frac": round(fin, 4)}
                if i in finite and fin == 1.0:
                    with np.errstate(all="ignore"):
                        entry["e_rel"] = float("%.3e" % oracle.e_rel(y[i], refs[d][finite.index(i)], bs.x[i])[0])
                cell.setdefault(name, {})[d] = entry
        diag[str(n)] = cell
    out["boundary_diagnostics"] = diag
    log("scored everything")
    return summary


if __name__ == "__main__":
    main()
