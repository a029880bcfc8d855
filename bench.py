#!/usr/bin/env python3
"""Benchmark of the batched orthonormal 2D DCT on one MI355X.

Workload (one "step"): the six square sizes N = 8, 16, 32, 64, 128, 256, each a batch
of 2^27 / N^2 row-major float32 arrays (512 MiB) of seeded N(0,1) values resident in
HBM, transformed in place by the forward, inverse and fused round-trip calls of the C
ABI (18 calls).  Algorithmic traffic is one float32 read and one float32 write per
element per call (8 N^2 bytes per array), so the step moves 18 x 1 GiB.

Reported: whole-step GB/s, per-size/per-direction GB/s and %HBM, the roofline of the
dominant kernel (HIP-event timing on the stream the kernels run on), a float32 vs
split-precision matrix-path comparison where it exists, and the FP64 oracle timed on a
bounded sample of the same arrays on the host cores (the CPU baseline).
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


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--sizes", default=",".join(map(str, SIZES)))
    ap.add_argument("--precision", default="auto", help="path used by the step (auto = library default)")
    ap.add_argument("--compare", default="fp32,bf16x3,bf16x6,fp16x3,bf16,fp16,fp8",
                    help="paths timed per size for the float32 vs split comparison (N<=32 for splits)")
    ap.add_argument("--cpu-frac", type=float, default=0.75, help="fraction of each batch the oracle runs on")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--log2-floats", type=int, default=27, help="floats per size (default 2^27 = 512 MiB)")
    ap.add_argument("--no-tune", action="store_true", help="skip the (untimed) autotuning pass")
    ap.add_argument("--save-policy", default="", help="write the tuned policy (autotune cache, JSON) here")
    ap.add_argument("--load-policy", default="", help="freeze this saved policy instead of tuning")
    ap.add_argument("--no-ragged", action="store_true", help="skip the ragged-batch (one graph launch) measurement")
    ap.add_argument("--no-filter", action="store_true", help="skip the spectral-filter measurement")
    ap.add_argument("--no-rect", action="store_true", help="skip the rectangle-orientation measurement")
    return ap.parse_args()


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

    # ---- inputs resident in HBM ------------------------------------------------------
    host = {}
    bufs = {}
    for n in sizes:
        batch = (1 << args.log2_floats) // (n * n)
        x = workloads.c3_normal(n, batch=batch).x
        host[n] = x
        bufs[n] = torch.from_numpy(x).to(dev)
        print("input N=%d batch=%d (%.0f MiB)" % (n, batch, x.nbytes / 2 ** 20), file=sys.stderr, flush=True)
    torch.cuda.synchronize()

    # ---- autotune (untimed, on the library's own scratch data, before any measurement) --
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

    # ---- self-check before timing (the round trip must return the input) -------------
    # Runs on a full-size copy so every launch of a kernel in this process has the same size.
    for n in sizes:
        t = bufs[n].clone()
        call(n, "roundtrip", args.precision, t)
        torch.cuda.synchronize()
        num = torch.linalg.vector_norm((t[:256] - bufs[n][:256]).double().reshape(256, -1), dim=1)
        den = torch.linalg.vector_norm(bufs[n][:256].double().reshape(256, -1), dim=1)
        worst = float((num / den).max())
        del t
        if worst > GATE["roundtrip"]:
            print("self-check failed N=%d e_rel %.3e" % (n, worst), file=sys.stderr)
            sys.exit(1)

    # ---- warmup + timed steps ----------------------------------------------------------
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

    per = {}
    call_ms = {}
    for n in sizes:
        per[str(n)] = {}
        for d in DIRS:
            ms = float(np.mean([a.elapsed_time(b) for a, b in ev[(n, d)]]))
            call_ms[(n, d)] = ms
            gbs = 8 * n * n * host[n].shape[0] / (ms * 1e-3) / 1e9
            per[str(n)][d] = {"ms": round(ms, 4), "GB/s": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
                              "transforms_per_s": round(host[n].shape[0] / (ms * 1e-3), 1)}

    # dominant kernel: the call with the largest share of the step among calls that are one
    # kernel launch (the event pair then brackets exactly that kernel)
    names = {(n, d): kernel_name(n, d, tuned["%d/%s" % (n, d)]) for n in sizes for d in DIRS}
    single = [k for k in names if names[k]]
    dom = max(single, key=lambda k: call_ms[k]) if single else max(call_ms, key=call_ms.get)
    n_dom, d_dom = dom
    alg_bytes = 8 * n_dom * n_dom * host[n_dom].shape[0]
    achieved = alg_bytes / (call_ms[dom] * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": counted_traffic(names[dom]) if names.get(dom) else None,
                "kernel": names.get(dom) or "%s N=%d" % (d_dom, n_dom), "call": "%s N=%d" % (d_dom, n_dom),
                "avg_ms": round(call_ms[dom], 4), "algorithmic_bytes_per_launch": alg_bytes}

    # ---- float32 vs split-precision matrix paths (same GPU, same inputs) --------------
    compare = {}
    for p in [c for c in args.compare.split(",") if c]:
        for n in sizes:
            if p != "fp32" and n > 64:
                continue
            scratch = torch.empty_like(bufs[n])
            try:
                dct.transform(bufs[n], scratch, "forward", p, stream=stream)
            except dct.DCT2DError:
                continue
            torch.cuda.synchronize()
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            reps = 5
            a.record(stream)
            for _ in range(reps):
                dct.transform(bufs[n], scratch, "forward", p, stream=stream)
            b.record(stream)
            torch.cuda.synchronize()
            ms = a.elapsed_time(b) / reps
            compare.setdefault(p, {})[str(n)] = round(8 * n * n * host[n].shape[0] / (ms * 1e-3) / 1e9, 1)
            del scratch

    filt = None if args.no_filter else filter_rates(dct, bufs, host, sizes, stream, per)
    rect = None if args.no_rect else rect_rates(dct, bufs[sizes[0]], stream,
                                                tune=not (args.no_tune or args.load_policy))
    ragged = None if args.no_ragged else ragged_c4(dct, stream, args.steps)
    copy_gbs = copy_ceiling(bufs[sizes[0]], stream)
    for n in sizes:
        for d in DIRS:
            per[str(n)][d]["copy_frac"] = round(per[str(n)][d]["GB/s"] / copy_gbs, 4)

    out = {"metric": METRIC, "value": round(value, 1), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "six square sizes N=8..256, 2^%d float32 per size (batch 2^%d/N^2), N(0,1); "
                                  "forward + inverse + fused round trip, in place" % (args.log2_floats,
                                                                                     args.log2_floats),
                      "sizes": sizes, "batch": {str(n): int(host[n].shape[0]) for n in sizes},
                      "precision": args.precision, "variants": tuned},
           "hbm_frac": round(value / HBM_PEAK_GBS, 4), "copy_ceiling_GBps": round(copy_gbs, 1),
           "wall_s": round(wall, 3),
           "roofline": roofline, "per_size": per, "compare_forward_GBps": compare, "ragged_c4": ragged,
           "filter": filt, "rectangles": rect}

    # ---- CPU baseline: the FP64 oracle on a bounded sample of the same arrays -----------
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(host, sizes, args.cpu_frac, bufs, stream)
    print(json.dumps(out), flush=True)


def poisson_multipliers(n):
    """Neumann Poisson solve on an n x n grid: 1 / (2 cos(pi k/n) + 2 cos(pi l/n) - 4), 0 at (0, 0)."""
    k = np.arange(n)[:, None]
    l = np.arange(n)[None, :]
    mu = 2.0 * np.cos(np.pi * k / n) + 2.0 * np.cos(np.pi * l / n) - 4.0
    lam = np.zeros((n, n))
    lam[mu != 0] = 1.0 / mu[mu != 0]
    return lam.astype(np.float32)


def filter_rates(dct, bufs, host, sizes, stream, per, reps=5):
    """The fused spectral filter (Prop. 1, eq. 4) on the same batches, one shared Poisson
    operator, out of place: one read and one write per array like the round trip, so its
    GB/s uses the same 8 N^2 bytes per array.  Reported beside the step, not part of it."""
    import torch
    res = {}
    for n in sizes:
        lam = torch.from_numpy(poisson_multipliers(n)).to(bufs[n].device)
        scratch = torch.empty_like(bufs[n])
        dct.filter(bufs[n], lam, out=scratch, stream=stream)
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            dct.filter(bufs[n], lam, out=scratch, stream=stream)
        b.record(stream)
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / reps
        gbs = 8 * n * n * host[n].shape[0] / (ms * 1e-3) / 1e9
        res[str(n)] = {"ms": round(ms, 4), "GB/s": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
                       "vs_roundtrip": round(gbs / per[str(n)]["roundtrip"]["GB/s"], 3)}
        del scratch
    torch.cuda.empty_cache()
    return res


RECT_PAIRS = ((8, 64), (64, 8), (16, 32), (32, 16), (8, 256), (256, 8), (64, 256), (256, 64))


def rect_rates(dct, buf, stream, tune=True, reps=5):
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
        res["%dx%d" % (h, w)] = {}
        for d in DIRS:
            if tune:
                dct.tune(h, w, d, "fp32", batch=batch, stream=stream)
            res["%dx%d" % (h, w)]["variant/" + d] = dct.get_variant(h, w, d, "fp32")
            dct.transform(x, y, d, "fp32", stream=stream)
            torch.cuda.synchronize()
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            for _ in range(reps):
                dct.transform(x, y, d, "fp32", stream=stream)
            b.record(stream)
            torch.cuda.synchronize()
            ms = a.elapsed_time(b) / reps
            res["%dx%d" % (h, w)][d] = round(8 * h * w * batch / (ms * 1e-3) / 1e9, 1)
    del scratch
    torch.cuda.empty_cache()
    return res


def copy_ceiling(buf, stream, reps=10):
    """GB/s of a plain device-to-device copy of one 512 MiB buffer (read + write bytes), the practical
    ceiling a one-read-one-write kernel is compared against."""
    import torch
    out = torch.empty_like(buf)
    out.copy_(buf)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(reps):
        out.copy_(buf)
    b.record(stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    del out
    torch.cuda.empty_cache()
    return 2 * buf.numel() * 4 / (ms * 1e-3) / 1e9


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


def source_digest():
    """SHA-256 over the kernel sources; ties counter-derived traffic figures to the code they measured."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2609_28519_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".hpp", ".cpp")):
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


def ragged_c4(dct, stream, steps):
    """The ragged configuration: 200k blocks (8..256) + 4 x 1024^2 + 4 x 512x384 images, U[-1,1] with 5%
    of items x 1e30, forward in place, one hipGraphLaunch per step (plan recorded before timing)."""
    import torch

    import workloads
    rg = workloads.c4_ragged()
    buf = torch.from_numpy(rg.data).cuda()
    plan = dct.RaggedPlan(rg.offsets, rg.rows, rg.cols, "forward", "auto")
    info = plan.info()
    plan.execute(buf, stream)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(steps):
        plan.execute(buf, stream)
    b.record(stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / steps
    alg = int(8 * (rg.rows.astype(np.int64) * rg.cols).sum())
    plan.close()
    del buf
    torch.cuda.empty_cache()
    return {"ms": round(ms, 4), "GB/s": round(alg / (ms * 1e-3) / 1e9, 1),
            "hbm_frac": round(alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4), "items": info["items"],
            "classes": info["classes"], "graph_nodes": info["graph_nodes"], "launches_per_step": 1,
            "algorithmic_bytes": alg}


def cpu_baseline(host, sizes, frac, bufs, stream):
    """Times the FP64 oracle (as it stands) on the first `frac` of every size's arrays, on the host's
    cores, for forward, inverse and round trip; also scores the GPU forward of that sample."""
    import torch

    import oracle
    import paper_2609_28519_amd as dct

    threads = oracle.default_threads()
    total_bytes = 0
    total_s = 0.0
    worst = {}
    for n in sizes:
        m = max(1, int(host[n].shape[0] * frac))
        xs = host[n][:m]
        t0 = time.perf_counter()
        y = oracle.forward(xs, threads=threads)
        oracle.inverse(xs, threads=threads)
        oracle.roundtrip(xs, threads=threads)
        total_s += time.perf_counter() - t0
        total_bytes += 8 * n * n * m * 3
        # error of the GPU calls on part of the sample, vs the oracle (stated for every result): the
        # forward against the oracle's forward, the inverse of the same arrays read as spectra against
        # the oracle's inverse, the fused round trip against the input itself
        k = min(m, 256)
        ref = {"forward": y[:k], "inverse": oracle.inverse(xs[:k], threads=threads),
               "roundtrip": xs[:k].astype(np.float64)}
        worst[str(n)] = {}
        for d in DIRS:
            g = torch.from_numpy(xs[:k]).cuda()
            dct.transform(g, g, d, "auto", stream=stream)
            torch.cuda.synchronize()
            worst[str(n)][d] = float(oracle.e_rel(g.cpu().numpy(), ref[d], xs[:k]).max())
    return {"value": round(total_bytes / total_s / 1e9, 4), "unit": "GB/s", "cores": threads, "kind": "oracle",
            "sample": "first %.0f%% of each size's batch (forward + inverse + round trip, FP64 direct definition)"
                      % (100 * frac),
            "seconds": round(total_s, 2), "gpu_max_e_rel_vs_oracle": worst}


if __name__ == "__main__":
    main()
