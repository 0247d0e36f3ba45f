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
  schedules     (with --breakdown) forward and inverse time of every
                schedule.
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
    import torch
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        plan.execute(x, out, inverse=inverse, stream=stream)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        plan.execute(x, out, inverse=inverse, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1) / steps, wall


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--shape", default="1024,1024,1024")
    ap.add_argument("--schedule", default="auto")
    ap.add_argument("--breakdown", action="store_true",
                    help="also time every schedule forward and inverse")
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
    ms, wall = time_plan(plan, x, out, args.steps, args.warmup)
    log(f"bench: {ms:.3f} ms/step (wall {wall / args.steps * 1e3:.3f} ms)")

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
    if args.breakdown:
        sched = {}
        for s in ("pencil", "slab", "volumetric", "auto"):
            p = dft3d.Plan(shape, s)
            f_ms, _ = time_plan(p, x, out, max(3, args.steps // 2), 2)
            i_ms, _ = time_plan(p, x, out, max(3, args.steps // 2), 2, inverse=True)
            sched[s] = {"passes": p.num_passes, "fwd_ms": round(f_ms, 4),
                        "inv_ms": round(i_ms, 4),
                        "fwd_gflops": round(flops / (f_ms * 1e-3) / 1e9, 1),
                        "fwd_gbs_per_pass": round(
                            16.0 * N / (f_ms / p.num_passes * 1e-3) / 1e9, 1)}
            log(f"bench: {s}: {sched[s]}")
            p.close()
        result["schedules"] = sched
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
    if not args.no_cpu_baseline:
        log("bench: timing the CPU oracle on a sample")
        result["cpu_baseline"] = cpu_baseline(x_host)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
