#!/usr/bin/env python3
"""Throughput of the 3D complex64 DFT on one MI355X.

A step is one forward 3D DFT of the 1024 x 1024 x 1024 complex64 workload
(input iid uniform[-1, 1) from seed 2, already resident in HBM) with the
plan's schedule (default: auto).  value = 5 N log2 N / step time in GFLOP/s.

The JSON line also carries:
  roofline      the pass kernel (every pass reads and writes the whole
                array: 16 N algorithmic bytes per launch) against 8 TB/s;
                its average launch time is the step time (HIP events on the
                launch stream over the timed region) over the passes per
                step; traffic is the HBM bytes per launch from the rocprofv3
                byte counters recorded in profiles/ (null once the kernel
                source differs from the one profiled);
  cpu_baseline  the FP64 oracle (recursive radix-2 FFT, all host threads)
                timed on a bounded sample of the same pencils;
  configs       (unless --no-extras) the other workloads: 64^3 forward and
                inverse (latency), every schedule at 1024^3, every leaf
                precision at 256^3 and 1024^3, 96 uneven problems batched
                per pass level against one plan at a time,
                2048 x 1024 x 512 auto vs pencil, FP32 vs bf16x6 leaves,
                lengths that are not powers of two (1000^3, 1009^3, 96^3), and
                rocFFT through torch.fft.fftn on the same shapes as a timed
                vendor-library context (never a correctness reference).
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("3D c64 DFT GFLOP/s (5N·log2N) + HBM GB/s at 1024³; "
          "plain vs MFMA/batched")
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def time_plan(plan, x, out, steps, warmup, inverse=False):
    """Mean ms per step over the timed region (HIP events on the launch
    stream, one between consecutive steps), the wall-clock seconds of the
    region, and the per-step times (for the median and the minimum)."""
    import torch
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        plan.execute(x, out, inverse=inverse, stream=stream)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    t0 = time.perf_counter()
    ev[0].record(stream)
    for i in range(steps):
        plan.execute(x, out, inverse=inverse, stream=stream)
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = [ev[i].elapsed_time(ev[i + 1]) for i in range(steps)]
    return ev[0].elapsed_time(ev[steps]) / steps, wall, per


def cpu_baseline(x_host, budget_s=25.0, chunk=32768):
    """The oracle (O2, FP64, all host threads) on the pencils of every axis
    of the same input, in chunks, until all are done or the time budget is
    spent; GFLOP/s over the pencils it finished (5 n log2 n per pencil)."""
    import oracle
    n0, n1, n2 = x_host.shape
    flops = 0.0
    t = 0.0
    done = []
    for axis, n in ((2, n2), (1, n1), (0, n0)):
        total = x_host.size // n
        first = 0
        while first < total and t < budget_s:
            count = min(chunk, total - first)
            t0 = time.perf_counter()
            oracle.fft_pencils(x_host, axis, first, count, -1)
            t += time.perf_counter() - t0
            flops += 5.0 * n * math.log2(n) * count
            first += count
        done.append(f"{first}/{total} pencils of length {n} along axis {axis}")
    return {"value": round(flops / t / 1e9, 3), "unit": "GFLOP/s",
            "cores": oracle.num_threads(), "kind": "oracle",
            "sample": "O2 recursive radix-2 FFT in FP64 on " + "; ".join(done) +
                      f" of the benchmark input ({t:.1f} s)"}


def traffic_from_profile(path):
    """HBM bytes per launch of the pass kernel recorded in a profiles/
    summary, or None if the kernel source changed since it was taken."""
    import hashlib
    try:
        text = open(path).read()
    except OSError:
        return None
    fields = dict(l.split(": ", 1) for l in text.splitlines()
                  if l.startswith(("traffic_bytes_per_launch: ",
                                   "kernel_source_sha256_16: ")))
    src = b"".join(open(os.path.join(ROOT, "paper_1904_10119_amd", "csrc", f),
                        "rb").read() for f in ("pass_kernel.h", "fft_device.h"))
    if hashlib.sha256(src).hexdigest()[:16] != fields.get("kernel_source_sha256_16"):
        return None
    return float(fields["traffic_bytes_per_launch"])


def timed(fn, reps, warm=2):
    """Average ms of fn() over reps runs (HIP events on the current stream)."""
    import torch
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def extras(x1024_host, args):
    """The other workloads, each timed on the GPU (no accuracy checks here:
    the tests carry those)."""
    import torch
    from paper_1904_10119_amd import dft3d, inputs
    out = {}

    def plan_ms(shape, x, y, reps, inverse=False, **kw):
        p = dft3d.Plan(shape, **kw)
        ms = timed(lambda: p.execute(x, y, inverse=inverse), reps)
        n = p.num_passes
        p.close()
        return ms, n

    # 64^3, forward and inverse: latency-bound (2 MiB).  Pencil (three
    # passes) and auto (slab: fused plane pass + depth pass), each also
    # captured once in a HIP graph (torch's capture) and replayed, which
    # removes the per-call host overhead of the launches
    shape = (64, 64, 64)
    x = torch.from_numpy(inputs.uniform_c64(shape, 1)).cuda()
    y = torch.empty_like(x)
    small = {}
    for sch in ("pencil", "auto"):
        f, n = plan_ms(shape, x, y, 200, schedule=sch)
        i, _ = plan_ms(shape, x, y, 200, inverse=True, schedule=sch)
        p = dft3d.Plan(shape, sch)
        p.bind_workspace(x.device)
        p.execute(x, y)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        cs = torch.cuda.Stream()
        cs.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(cs):
            with torch.cuda.graph(g, stream=cs):
                for _ in range(20):
                    p.execute(x, y)
        torch.cuda.current_stream().wait_stream(cs)
        gr = timed(g.replay, 20) / 20
        del g
        p.close()
        small[sch] = {"schedule": dft3d.describe(shape, sch)["schedule"], "passes": n,
                      "fwd_us": round(f * 1e3, 2), "inv_us": round(i * 1e3, 2),
                      "fwd_graph_us": round(gr * 1e3, 2)}
    out["64^3"] = small
    log(f"bench: 64^3 {small}")

    # 1024^3 under every schedule
    N = 1 << 30
    fl = 5.0 * N * 30
    x = torch.from_numpy(x1024_host).cuda()
    y = torch.empty_like(x)
    sched = {}
    for s in ("pencil", "slab", "volumetric"):
        f, n = plan_ms((1024,) * 3, x, y, 5, schedule=s)
        i, _ = plan_ms((1024,) * 3, x, y, 5, inverse=True, schedule=s)
        sched[s] = {"passes": n, "fwd_ms": round(f, 3), "inv_ms": round(i, 3),
                    "fwd_gflops": round(fl / (f * 1e-3) / 1e9, 1),
                    "hbm_gbs_per_pass": round(16.0 * N / (f / n * 1e-3) / 1e9, 1)}
        log(f"bench: 1024^3 {s} {sched[s]}")
    # volumetric leaving the shuffled (digit-exchanged) order, and its inverse
    # from that order
    f, n = plan_ms((1024,) * 3, x, y, 5, schedule="volumetric", layout="shuffled")
    i, _ = plan_ms((1024,) * 3, x, y, 5, inverse=True, schedule="volumetric",
                   layout="shuffled")
    sched["volumetric shuffled"] = {
        "passes": n, "fwd_ms": round(f, 3), "inv_ms": round(i, 3),
        "fwd_gflops": round(fl / (f * 1e-3) / 1e9, 1),
        "hbm_gbs_per_pass": round(16.0 * N / (f / n * 1e-3) / 1e9, 1)}
    log(f"bench: 1024^3 volumetric shuffled {sched['volumetric shuffled']}")
    out["1024^3 schedules"] = sched
    prec = {}
    for pr in ("fp32", "bf16x6", "bf16x9", "fp16x3"):
        f, _ = plan_ms((1024,) * 3, x, y, 3, schedule="pencil", precision=pr)
        prec[pr] = {"fwd_ms": round(f, 3), "fwd_gflops": round(fl / (f * 1e-3) / 1e9, 1)}
    out["1024^3 pencil leaf precision"] = prec
    log(f"bench: 1024^3 precisions {prec}")
    del x, y
    torch.cuda.empty_cache()

    # 256^3, Gaussian + 8 plane waves, every leaf precision
    shape = (256, 256, 256)
    N = 1 << 24
    xh, _, _ = inputs.gaussian_waves_c64(shape, 3)
    x = torch.from_numpy(xh).cuda()
    y = torch.empty_like(x)
    prec = {}
    for pr in ("fp32", "bf16x1", "fp16x1", "bf16x6", "bf16x9", "fp16x3"):
        f, _ = plan_ms(shape, x, y, 20, schedule="pencil", precision=pr)
        prec[pr] = {"fwd_ms": round(f, 4),
                    "fwd_gflops": round(5.0 * N * 24 / (f * 1e-3) / 1e9, 1)}
    out["256^3 pencil leaf precision"] = prec
    log(f"bench: 256^3 precisions {prec}")
    del x, y
    torch.cuda.empty_cache()

    # 96 uneven problems: batched per pass level vs one plan at a time
    shapes = inputs.batch_shapes(96, 104)
    xs = [torch.from_numpy(inputs.uniform_c64(sh, 400 + k)).cuda()
          for k, sh in enumerate(shapes)]
    ys = [torch.empty_like(v) for v in xs]
    pts = sum(v.numel() for v in xs)
    flops = sum(5.0 * v.numel() * math.log2(v.numel()) for v in xs)
    b_ms = timed(lambda: dft3d.fftn_batched(xs, outs=ys), 20)
    plans = [dft3d.get_plan(v.shape, "auto") for v in xs]
    for p, v in zip(plans, xs):
        p.bind_workspace(v.device)
    l_ms = timed(lambda: [p.execute(v, w) for p, v, w in zip(plans, xs, ys)], 20)
    loop_launches = sum(p.num_passes for p in plans)
    del plans
    # autotune every distinct shape, then the batch again with tuned plans
    tuned = {}
    for sh in sorted(set(shapes)):
        tuned["x".join(map(str, sh))] = dft3d.autotune(sh)["schedule"]
    t_ms = timed(lambda: dft3d.fftn_batched(xs, outs=ys), 20)
    out["batched 96 {32,64,128}^3"] = {
        "points": pts, "batched_ms": round(b_ms, 4), "plan_loop_ms": round(l_ms, 4),
        "batched_gflops": round(flops / (b_ms * 1e-3) / 1e9, 1),
        "autotuned_batched_ms": round(t_ms, 4),
        "autotuned_schedules": sorted(set(tuned.values())),
        "launches_batched": 3, "launches_loop": loop_launches}
    log(f"bench: batched {out['batched 96 {32,64,128}^3']}")
    del xs, ys
    torch.cuda.empty_cache()

    # 2048 x 1024 x 512: auto vs fixed pencil, FP32 vs bf16x6 leaves
    shape = (2048, 1024, 512)
    N = 1 << 30
    x = torch.from_numpy(inputs.uniform_c64(shape, 5)).cuda()
    y = torch.empty_like(x)
    r = {}
    runs = [("auto untuned", dict(schedule="auto")), ("pencil", dict(schedule="pencil")),
            ("auto bf16x6", dict(schedule="auto", precision="bf16x6"))]
    for name, kw in runs:
        f, n = plan_ms(shape, x, y, 3, **kw)
        i, _ = plan_ms(shape, x, y, 3, inverse=True, **kw)
        r[name] = {"passes": n, "fwd_ms": round(f, 3), "inv_ms": round(i, 3),
                   "fwd_gflops": round(fl / (f * 1e-3) / 1e9, 1)}
    r["autotune"] = dft3d.autotune(shape)
    f, n = plan_ms(shape, x, y, 3, schedule="auto")
    r["auto tuned"] = {"passes": n, "fwd_ms": round(f, 3),
                       "fwd_gflops": round(fl / (f * 1e-3) / 1e9, 1)}
    out["2048x1024x512"] = r
    log(f"bench: 2048x1024x512 {r}")
    del x, y
    torch.cuda.empty_cache()

    # lengths that are not powers of two, one pass per axis: 1000^3 and
    # 96^3 (mixed radix) and 1009^3 (Bluestein, convolution length 2048);
    # uniform[-1, 1) inputs drawn on the device from a seeded generator
    bl = {}
    for shape, reps in (((1000, 1000, 1000), 3), ((1009, 1009, 1009), 3),
                        ((96, 96, 96), 100)):
        g = torch.Generator(device="cuda").manual_seed(6)
        x = torch.complex(torch.rand(shape, device="cuda", generator=g) * 2 - 1,
                          torch.rand(shape, device="cuda", generator=g) * 2 - 1)
        y = torch.empty_like(x)
        f, n = plan_ms(shape, x, y, reps, schedule="auto")
        i, _ = plan_ms(shape, x, y, reps, inverse=True, schedule="auto")
        Np = x.numel()
        bl["x".join(map(str, shape))] = {
            "passes": n, "fwd_ms": round(f, 4), "inv_ms": round(i, 4),
            "fwd_gflops_5nlogn": round(5.0 * Np * math.log2(Np) / (f * 1e-3) / 1e9, 1),
            "hbm_gbs_per_pass": round(16.0 * Np / (f / n * 1e-3) / 1e9, 1)}
        del x, y
        torch.cuda.empty_cache()
    out["other lengths"] = bl
    log(f"bench: other lengths {bl}")

    # vendor-library context (timing only, never a correctness reference):
    # rocFFT through torch.fft.fftn on the same shapes, beside this library
    ctx = {}
    for shape, reps in (((1024, 1024, 1024), 5), ((2048, 1024, 512), 5),
                        ((1000, 1000, 1000), 3), ((256, 256, 256), 20), ((64, 64, 64), 100)):
        g = torch.Generator(device="cuda").manual_seed(7)
        x = torch.complex(torch.rand(shape, device="cuda", generator=g) * 2 - 1,
                          torch.rand(shape, device="cuda", generator=g) * 2 - 1)
        y = torch.empty_like(x)
        try:
            vendor = timed(lambda: torch.fft.fftn(x), reps)
        except RuntimeError as e:  # no vendor FFT in this torch build
            vendor = None
            log(f"bench: torch.fft.fftn unavailable: {e}")
        mine, _ = plan_ms(shape, x, y, reps, schedule="auto")
        ctx["x".join(map(str, shape))] = {
            "rocfft_torch_fftn_ms": None if vendor is None else round(vendor, 4),
            "dft3d_ms": round(mine, 4),
            "speedup": None if vendor is None else round(vendor / mine, 2)}
        del x, y
        torch.cuda.empty_cache()
    out["vendor context (rocFFT via torch.fft.fftn, timing only)"] = ctx
    log(f"bench: vendor context {ctx}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--shape", default="1024,1024,1024")
    ap.add_argument("--schedule", default="auto")
    ap.add_argument("--breakdown", action="store_true",
                    help="(kept for compatibility; the extras include it)")
    ap.add_argument("--no-extras", action="store_true",
                    help="time only the 1024^3 headline workload")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also time a plain device copy of the array (the "
                         "reference kernel for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: --gpus {args.gpus} is not supported "
              "(this build has no multi-GPU path)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1904_10119_amd import dft3d, inputs

    shape = tuple(int(s) for s in args.shape.split(","))
    N = shape[0] * shape[1] * shape[2]
    flops = 5.0 * N * math.log2(N)
    log(f"bench: generating {shape} input")
    x_host = inputs.uniform_c64(shape, 2)
    x = torch.from_numpy(x_host).cuda()
    out = torch.empty_like(x)

    plan = dft3d.Plan(shape, args.schedule)
    npass = plan.num_passes
    desc = dft3d.describe(shape, args.schedule)
    log(f"bench: schedule {desc['schedule']} passes "
        f"{[p['label'] for p in desc['passes']]}")
    ms, wall, per = time_plan(plan, x, out, args.steps, args.warmup)
    per_sorted = sorted(per)
    ms_median = per_sorted[len(per) // 2] if len(per) % 2 else \
        0.5 * (per_sorted[len(per) // 2 - 1] + per_sorted[len(per) // 2])
    log(f"bench: {ms:.3f} ms/step (median {ms_median:.3f}, min {per_sorted[0]:.3f}, "
        f"wall {wall / args.steps * 1e3:.3f} ms)")

    per_launch_ms = ms / npass
    achieved = 16.0 * N / (per_launch_ms * 1e-3) / 1e9
    traffic = None
    if shape == (1024, 1024, 1024) and desc["schedule"] == "pencil":
        traffic = traffic_from_profile(
            os.path.join(ROOT, "profiles", "pencil_pass1024_1024cubed.md"))
    result = {
        "metric": METRIC,
        "value": round(flops / (ms * 1e-3) / 1e9, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "ms_median": round(ms_median, 4),
        "ms_min": round(per_sorted[0], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "x".join(map(str, shape)) +
                   " complex64 forward 3D DFT", "schedule": desc["schedule"],
                   "passes": npass, "parallelism": "1 GPU"},
        "hbm_gbs_per_step": round(16.0 * N * npass / (ms * 1e-3) / 1e9, 1),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": desc["passes"][0]["label"],
                     "bytes_per_launch": 16 * N,
                     "avg_launch_ms": round(per_launch_ms, 4)},
    }
    if args.copy_calibration:
        for _ in range(2):
            out.copy_(x)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        stream = torch.cuda.current_stream()
        e0.record(stream)
        for _ in range(args.steps):
            out.copy_(x)
        e1.record(stream)
        torch.cuda.synchronize()
        cms = e0.elapsed_time(e1) / args.steps
        result["copy_calibration"] = {"bytes_per_launch": 16 * N,
                                      "avg_launch_ms": round(cms, 4),
                                      "gbs": round(16.0 * N / (cms * 1e-3) / 1e9, 1)}
        log(f"bench: device copy {result['copy_calibration']}")
    del x, out
    torch.cuda.empty_cache()
    if not args.no_extras and shape == (1024, 1024, 1024):
        result["configs"] = extras(x_host, args)
    if not args.no_cpu_baseline:
        log("bench: timing the CPU oracle on a sample")
        result["cpu_baseline"] = cpu_baseline(x_host)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
