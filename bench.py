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
  error         the headline result against the FP64 oracle over every
                element (rel_l2 and the largest element error in units of
                the reference's root mean square);
  cpu_baseline  the FP64 oracle timed on the host: the recursive radix-2 FFT
                on the whole 1024^3 input on all host threads (the figure),
                on one thread for a sample of pencils, and the direct sums at
                64^3 and 256^3; the same leg computes the FP64 references
                every error in this line is measured against;
  configs       (unless --no-extras) the other workloads, each with its
                error: 64^3 forward and inverse (latency), every schedule at
                1024^3, every leaf precision at 256^3 and 1024^3, the time
                breakdown of every schedule at 1024^3 (full passes, passes
                with the radix stages removed, plain copies), 96 uneven
                problems batched (per pass level and in one persistent
                launch) against one plan at a time, 2048 x 1024 x 512 auto
                vs pencil, FP32 vs bf16x6 leaves, lengths that are not
                powers of two (1000^3, 1009^3, 96^3), the error of the
                pencil schedule over cubes from 8^3 to 1024^3, and rocFFT
                through torch.fft.fftn on the same shapes as a timed
                vendor-library context (never a correctness reference).
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("3D c64 DFT GFLOP/s (5N·log2N) + HBM GB/s at 1024³; "
          "plain vs MFMA/batched")
HBM_PEAK_GBS = 8000.0
SAMPLE_K = [(0, 0), (1, 0), (0, 1), (3, 5), (17, 250), (511, 77), (700, 1000), (1023, 1023)]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# ---------------------------------------------------------------- errors
# Plain numpy, against FP64 references the CPU leg computed.

def _slab_sums(fn, n0, planes=4):
    """Sum the per-slab tuples fn(i, j) over slabs [i, j) of axis 0 on the
    host's threads (numpy releases the GIL in its loops)."""
    from concurrent.futures import ThreadPoolExecutor
    spans = [(i, min(n0, i + planes)) for i in range(0, n0, planes)]
    with ThreadPoolExecutor(max(1, min(16, os.cpu_count() or 1))) as ex:
        parts = list(ex.map(lambda ij: fn(*ij), spans))
    return [sum(p[k] for p in parts) if k < 2 else max(p[k] for p in parts)
            for k in range(len(parts[0]))]


def errors(got, ref):
    """(rel_l2, largest element error / rms(ref)) over every element, slab by
    slab (no full-size temporaries)."""
    def part(i, j):
        d = got[i:j].astype(np.complex128) - ref[i:j]
        e2 = d.real * d.real + d.imag * d.imag
        r = ref[i:j]
        return (float(e2.sum()), float((r.real * r.real + r.imag * r.imag).sum()),
                float(e2.max()))
    num, den, worst = _slab_sums(part, got.shape[0])
    rms = math.sqrt(den / got.size)
    return math.sqrt(num / den), math.sqrt(worst) / rms


def err_fields(got, ref):
    rel, worst = errors(got, ref)
    return {"rel_l2": float(f"{rel:.3e}"), "max_elem_err_rms": float(f"{worst:.3e}")}


def sampled_err(got_dev, k_list, pencils):
    """rel_l2 over sampled output pencils y[k0, k1, :] (device tensor)."""
    num = den = 0.0
    for (k0, k1), ref in zip(k_list, pencils):
        g = got_dev[k0, k1].cpu().numpy().astype(np.complex128)
        num += float(np.sum(np.abs(g - ref) ** 2))
        den += float(np.sum(np.abs(ref) ** 2))
    return {"rel_l2_sampled": float(f"{math.sqrt(num / den):.3e}"),
            "sampled_pencils": len(k_list)}


def roundtrip_err(x_host, back_dev):
    """rel_l2(inverse(forward(x)) / N, x)."""
    n = x_host.size
    back = back_dev.cpu().numpy()

    def part(i, j):
        b = back[i:j].astype(np.complex128) / n
        r = x_host[i:j].astype(np.complex128)
        d = b - r
        return (float((d.real ** 2 + d.imag ** 2).sum()),
                float((r.real ** 2 + r.imag ** 2).sum()))
    num, den = _slab_sums(part, x_host.shape[0])
    return float(f"{math.sqrt(num / den):.3e}")


def shuffled_to_natural_err(got, ref, factors):
    """errors() of a SHUFFLED-layout result: along each axis of length
    n = a b the natural index k' + b l' sits at position l' + a k'."""
    pos = []
    for n, a in zip(got.shape, factors):
        p = np.arange(n)
        nat = (p // a) + (n // a) * (p % a)      # natural index at position p
        inv = np.empty_like(nat)
        inv[nat] = p
        pos.append(inv)
    def part(i, j):
        g = got[pos[0][i:j]][:, pos[1]][:, :, pos[2]].astype(np.complex128)
        r = ref[i:j]
        d = g - r
        e2 = d.real ** 2 + d.imag ** 2
        return (float(e2.sum()), float((r.real ** 2 + r.imag ** 2).sum()), float(e2.max()))
    num, den, worst = _slab_sums(part, got.shape[0])
    rms = math.sqrt(den / got.size)
    return {"rel_l2": float(f"{math.sqrt(num / den):.3e}"),
            "max_elem_err_rms": float(f"{math.sqrt(worst) / rms:.3e}")}


# ------------------------------------------------------------- CPU leg

def host_info():
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    mem = None
    try:
        with open("/proc/meminfo") as f:
            mem = round(int(f.readline().split()[1]) / 2 ** 20, 1)
    except (OSError, ValueError, IndexError):
        pass
    return model, mem


def cpu_leg(x_host, extras):
    """The FP64 oracle on the host: the baseline figure (O2 on the whole
    1024^3 input, all threads), one-thread and direct-sum timings, and the
    FP64 references of every workload whose error this line reports."""
    import oracle
    from paper_1904_10119_amd import inputs
    refs = {}
    n = x_host.size
    cores = oracle.num_threads()
    t0 = time.perf_counter()
    refs["1024"] = oracle.dft3d_fft_c64(x_host, -1)
    t_all = time.perf_counter() - t0
    gflops = 5.0 * n * math.log2(n) / t_all / 1e9
    log(f"bench: oracle O2 1024^3 on {cores} threads {t_all:.1f} s ({gflops:.1f} GFLOP/s)")
    # one thread: O2 on the first 32768 pencils along the contiguous axis
    oracle.set_num_threads(1)
    cnt = 32768
    t0 = time.perf_counter()
    oracle.fft_pencils(x_host, 2, 0, cnt, -1)
    t1 = time.perf_counter() - t0
    oracle.set_num_threads(cores)
    g1 = 5.0 * 1024 * 10 * cnt / t1 / 1e9
    # O1 (direct sums) at 64^3 and 256^3, all threads
    o1 = {}
    for m in (64, 256):
        xm = inputs.uniform_c64((m, m, m), 1)
        t0 = time.perf_counter()
        ym = oracle.dft3d(xm, -1, "direct")
        o1[f"{m}^3_s"] = round(time.perf_counter() - t0, 3)
        if m == 64:
            refs["64"] = (xm, ym)
    model, mem = host_info()
    base = {"value": round(gflops, 3), "unit": "GFLOP/s", "cores": cores, "kind": "oracle",
            "sample": ("O2 recursive radix-2 FFT in FP64 on the whole 1024x1024x1024 "
                       f"benchmark input, forward, all {cores} host threads "
                       f"({t_all:.1f} s)"),
            "one_thread_gflops": round(g1, 3),
            "one_thread_sample": f"O2 on {cnt} pencils of length 1024 ({t1:.1f} s)",
            "o1_direct_seconds": o1, "cpu_model": model, "host_ram_gib": mem}
    if not extras:
        return base, refs
    # references of the other workloads (not part of the figure above)
    t0 = time.perf_counter()
    xw, _, _ = inputs.gaussian_waves_c64((256,) * 3, 3)
    refs["256w"] = (xw, oracle.dft3d(xw, -1, "fft"))
    shapes = inputs.batch_shapes(96, 104)
    xs = [inputs.uniform_c64(sh, 400 + k) for k, sh in enumerate(shapes)]
    refs["batch"] = (xs, [oracle.dft3d(v, -1, "fft") for v in xs])
    x2 = inputs.uniform_c64((2048, 1024, 512), 5)
    k0 = [a % 2048 for a, _ in SAMPLE_K]
    k1 = [b % 1024 for _, b in SAMPLE_K]
    refs["2048"] = (x2, list(zip(k0, k1)), oracle.sample_pencils(x2, k0, k1, -1))
    for m in (1000, 1009):
        xm = inputs.uniform_c64((m,) * 3, 6)
        kk = [(0, 0), (1, 2), (m // 2, 7), (m - 1, m - 3)]
        refs[str(m)] = (xm, kk, oracle.sample_pencils(xm, [a for a, _ in kk],
                                                      [b for _, b in kk], -1))
    x96 = inputs.uniform_c64((96,) * 3, 6)
    refs["96"] = (x96, oracle.dft3d(x96, -1, "direct"))
    curve = {}
    for lg in range(3, 10):
        m = 1 << lg
        xm = inputs.uniform_c64((m,) * 3, 11)
        curve[m] = (xm, oracle.dft3d_fft_c64(xm, -1))
    refs["curve"] = curve
    log(f"bench: oracle references of the other workloads {time.perf_counter() - t0:.1f} s")
    return base, refs


# ------------------------------------------------------------- GPU timing

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


def extras(x1024_host, refs):
    """The other workloads, each timed on the GPU, then checked against its
    FP64 reference (outside the timed region)."""
    import torch
    from paper_1904_10119_amd import dft3d
    out = {}
    have = bool(refs)

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
    x64h, y64 = refs["64"] if have else (None, None)
    from paper_1904_10119_amd import inputs
    x64h = inputs.uniform_c64(shape, 1) if x64h is None else x64h
    x = torch.from_numpy(x64h).cuda()
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
        small[sch] = {"schedule": dft3d.describe(shape, sch)["schedule"], "passes": n,
                      "fwd_us": round(f * 1e3, 2), "inv_us": round(i * 1e3, 2),
                      "fwd_graph_us": round(gr * 1e3, 2)}
        if have:
            p.execute(x, y)
            small[sch].update(err_fields(y.cpu().numpy(), y64))
            z = torch.empty_like(x)
            p.execute(y, z, inverse=True)
            small[sch]["roundtrip_rel_l2"] = roundtrip_err(x64h, z)
        p.close()
    out["64^3"] = small
    log(f"bench: 64^3 {small}")

    # 1024^3 under every schedule
    N = 1 << 30
    fl = 5.0 * N * 30
    x = torch.from_numpy(x1024_host).cuda()
    y = torch.empty_like(x)
    z = torch.empty_like(x)
    ref = refs.get("1024")

    def check_1024(p, sch_key, shuffled=False, roundtrip=True):
        res = {}
        if ref is None:
            return res
        p.execute(x, y)
        torch.cuda.synchronize()
        got = y.cpu().numpy()
        if shuffled:
            res.update(shuffled_to_natural_err(got, ref, dft3d.shuffle_factors(x.shape)))
        else:
            res.update(err_fields(got, ref))
        del got
        if roundtrip:
            p.execute(y, z, inverse=True)
            res["roundtrip_rel_l2"] = roundtrip_err(x1024_host, z)
        log(f"bench: 1024^3 {sch_key} error {res}")
        return res

    sched = {}
    for s, lay in (("pencil", "natural"), ("slab", "natural"), ("volumetric", "natural"),
                   ("volumetric", "shuffled")):
        key = s if lay == "natural" else "volumetric shuffled"
        p = dft3d.Plan((1024,) * 3, s, layout=lay)
        f = timed(lambda: p.execute(x, y), 5)
        i = timed(lambda: p.execute(x, y, inverse=True), 5)
        n = p.num_passes
        sched[key] = {"passes": n, "fwd_ms": round(f, 3), "inv_ms": round(i, 3),
                      "fwd_gflops": round(fl / (f * 1e-3) / 1e9, 1),
                      "hbm_gbs_per_pass": round(16.0 * N / (f / n * 1e-3) / 1e9, 1)}
        sched[key].update(check_1024(p, key, shuffled=(lay == "shuffled")))
        p.close()
        log(f"bench: 1024^3 {key} {sched[key]}")
    out["1024^3 schedules"] = sched
    prec = {}
    for pr, lf in (("fp32", 0), ("bf16x6", 16), ("bf16x9", 16), ("fp16x3", 16),
                   ("bf16x6", 32), ("bf16x9", 32), ("fp16x3", 32)):
        key = pr if lf == 0 else f"{pr} leaf{lf}"
        p = dft3d.Plan((1024,) * 3, "pencil", precision=pr, mfma_leaf=lf)
        f = timed(lambda: p.execute(x, y), 3)
        prec[key] = {"fwd_ms": round(f, 3), "fwd_gflops": round(fl / (f * 1e-3) / 1e9, 1)}
        if pr != "fp32":
            prec[key]["default_leaf"] = lf == dft3d.describe(
                (1024,) * 3, "pencil", precision=pr)["passes"][0]["mfma_leaf"]
            prec[key].update(check_1024(p, key, roundtrip=False))
        else:
            prec[key].update({k: v for k, v in sched["pencil"].items()
                              if k in ("rel_l2", "max_elem_err_rms")})
        p.close()
    out["1024^3 pencil leaf precision"] = prec
    log(f"bench: 1024^3 precisions {prec}")

    # time breakdown per schedule (the paper's split of a decomposition's
    # time into communication, packing and local DFTs, on one device): the
    # unfused pass list in full, with the radix stages removed (loads, LDS
    # exchanges and stores only) and as plain copies of the array (the HBM
    # floor of the same number of passes)
    brk = {}
    for s in ("pencil", "slab", "volumetric"):
        ms = {}
        for key, kw in (("full", {"fused_plane": 0, "fused_axes": 0}),
                        ("move_only", {"move_only": 1}), ("copy", {"move_only": 2})):
            p = dft3d.Plan((1024,) * 3, s, **kw)
            ms[key] = timed(lambda: p.execute(x, y), 5)
            n = p.num_passes
            p.close()
        brk[s] = {"passes": n, "full_ms": round(ms["full"], 3),
                  "move_only_ms": round(ms["move_only"], 3), "copy_ms": round(ms["copy"], 3),
                  "per_pass_ms": {k: round(v / n, 3) for k, v in ms.items()},
                  "butterflies_share": round((ms["full"] - ms["move_only"]) / ms["full"], 3),
                  "exchange_share": round((ms["move_only"] - ms["copy"]) / ms["full"], 3),
                  "hbm_floor_share": round(ms["copy"] / ms["full"], 3),
                  "copy_gbs": round(16.0 * N * n / (ms["copy"] * 1e-3) / 1e9, 1)}
    out["1024^3 time breakdown (move-only passes)"] = brk
    log(f"bench: 1024^3 breakdown {brk}")
    del x, y, z
    torch.cuda.empty_cache()

    # 256^3, Gaussian + 8 plane waves, every leaf precision
    shape = (256, 256, 256)
    N = 1 << 24
    xh, yref = refs["256w"] if have else (inputs.gaussian_waves_c64(shape, 3)[0], None)
    x = torch.from_numpy(xh).cuda()
    y = torch.empty_like(x)
    prec = {}
    for pr, lf in (("fp32", 0), ("bf16x1", 0), ("fp16x1", 0), ("bf16x6", 16),
                   ("bf16x9", 16), ("fp16x3", 16), ("bf16x6", 32), ("bf16x9", 32),
                   ("fp16x3", 32)):
        key = pr if lf == 0 else f"{pr} leaf{lf}"
        p = dft3d.Plan(shape, "pencil", precision=pr, mfma_leaf=lf)
        f = timed(lambda: p.execute(x, y), 20)
        prec[key] = {"fwd_ms": round(f, 4),
                     "fwd_gflops": round(5.0 * N * 24 / (f * 1e-3) / 1e9, 1)}
        if yref is not None:
            p.execute(x, y)
            prec[key].update(err_fields(y.cpu().numpy(), yref))
        p.close()
    out["256^3 pencil leaf precision"] = prec
    log(f"bench: 256^3 precisions {prec}")
    del x, y
    torch.cuda.empty_cache()

    # 96 uneven problems: batched per pass level and in one persistent
    # launch, vs one plan at a time
    shapes = inputs.batch_shapes(96, 104)
    xs_h, ys_ref = refs["batch"] if have else (
        [inputs.uniform_c64(sh, 400 + k) for k, sh in enumerate(shapes)], None)
    xs = [torch.from_numpy(v).cuda() for v in xs_h]
    ys = [torch.empty_like(v) for v in xs]
    pts = sum(v.numel() for v in xs)
    flops = sum(5.0 * v.numel() * math.log2(v.numel()) for v in xs)

    def batch_err():
        if ys_ref is None:
            return {}
        worst = max(float(np.linalg.norm(o.cpu().numpy() - r) / np.linalg.norm(r))
                    for o, r in zip(ys, ys_ref))
        return {"max_rel_l2_over_problems": float(f"{worst:.3e}")}

    b_ms = timed(lambda: dft3d.fftn_batched(xs, outs=ys), 20)
    b_err = batch_err()
    for v in ys:
        v.zero_()
    p_ms = timed(lambda: dft3d.fftn_batched(xs, outs=ys, launch="persistent"), 20)
    p_err = batch_err()
    lv = dft3d.describe_batch(shapes, "auto", "levels")
    pv = dft3d.describe_batch(shapes, "auto", "persistent")
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
        "persistent_ms": round(p_ms, 4),
        "persistent_gflops": round(flops / (p_ms * 1e-3) / 1e9, 1),
        "autotuned_batched_ms": round(t_ms, 4),
        "autotuned_schedules": sorted(set(tuned.values())),
        "launches_batched": len(lv["levels"]) if lv["batchable"] else None,
        "launches_persistent": 1 if pv["batchable"] else None,
        "launches_loop": loop_launches,
        "levels_error": b_err, "persistent_error": p_err}
    log(f"bench: batched {out['batched 96 {32,64,128}^3']}")
    del xs, ys
    torch.cuda.empty_cache()

    # 2048 x 1024 x 512: auto vs fixed pencil, FP32 vs bf16x6 leaves
    shape = (2048, 1024, 512)
    N = 1 << 30
    x2h, kk, pen = refs["2048"] if have else (inputs.uniform_c64(shape, 5), None, None)
    x = torch.from_numpy(x2h).cuda()
    y = torch.empty_like(x)
    z = torch.empty_like(x)
    r = {}
    runs = [("auto untuned", dict(schedule="auto")), ("pencil", dict(schedule="pencil")),
            ("auto bf16x6", dict(schedule="auto", precision="bf16x6")),
            ("auto bf16x6 leaf16", dict(schedule="auto", precision="bf16x6", mfma_leaf=16)),
            ("auto fp16x3", dict(schedule="auto", precision="fp16x3"))]
    for name, kw in runs:
        p = dft3d.Plan(shape, **kw)
        f = timed(lambda: p.execute(x, y), 3)
        i = timed(lambda: p.execute(x, y, inverse=True), 3)
        n = p.num_passes
        r[name] = {"passes": n, "fwd_ms": round(f, 3), "inv_ms": round(i, 3),
                   "fwd_gflops": round(fl / (f * 1e-3) / 1e9, 1)}
        if have:
            p.execute(x, y)
            r[name].update(sampled_err(y, kk, pen))
            p.execute(y, z, inverse=True)
            r[name]["roundtrip_rel_l2"] = roundtrip_err(x2h, z)
        p.close()
    r["autotune"] = dft3d.autotune(shape)
    f, n = plan_ms(shape, x, y, 3, schedule="auto")
    r["auto tuned"] = {"passes": n, "fwd_ms": round(f, 3),
                       "fwd_gflops": round(fl / (f * 1e-3) / 1e9, 1)}
    out["2048x1024x512"] = r
    log(f"bench: 2048x1024x512 {r}")
    del x, y, z
    torch.cuda.empty_cache()

    # lengths that are not powers of two, one pass per axis: 1000^3 and
    # 96^3 (mixed radix) and 1009^3 (Bluestein, convolution length 2048)
    bl = {}
    for shape, reps, sch in (((1000, 1000, 1000), 3, "auto"), ((1009, 1009, 1009), 3, "auto"),
                             ((96, 96, 96), 100, "auto"), ((1000, 1000, 1000), 3, "slab"),
                             ((1000, 1000, 1000), 3, "volumetric")):
        key = str(shape[0])
        xh = refs[key][0] if have else inputs.uniform_c64(shape, 6)
        x = torch.from_numpy(xh).cuda()
        y = torch.empty_like(x)
        p = dft3d.Plan(shape, sch)
        f = timed(lambda: p.execute(x, y), reps)
        i = timed(lambda: p.execute(x, y, inverse=True), reps)
        n = p.num_passes
        Np = x.numel()
        ent = {"passes": n, "fwd_ms": round(f, 4), "inv_ms": round(i, 4),
               "fwd_gflops_5nlogn": round(5.0 * Np * math.log2(Np) / (f * 1e-3) / 1e9, 1),
               "hbm_gbs_per_pass": round(16.0 * Np / (f / n * 1e-3) / 1e9, 1)}
        if have:
            p.execute(x, y)
            if key == "96":
                ent.update(err_fields(y.cpu().numpy(), refs[key][1]))
            else:
                ent.update(sampled_err(y, refs[key][1], refs[key][2]))
        p.close()
        bl["x".join(map(str, shape)) + ("" if sch == "auto" else " " + sch)] = ent
        del x, y
        torch.cuda.empty_cache()
    out["other lengths"] = bl
    log(f"bench: other lengths {bl}")

    # error of the default plan over cubes 8^3 .. 1024^3 (every element)
    if have:
        curve = {}
        for m, (xm, ym) in sorted(refs["curve"].items()):
            x = torch.from_numpy(xm).cuda()
            y = torch.empty_like(x)
            dft3d.fftn(x, out=y)
            torch.cuda.synchronize()
            rel, worst = errors(y.cpu().numpy(), ym)
            curve[f"{m}^3"] = {"log2N": 3 * int(math.log2(m)), "rel_l2": float(f"{rel:.3e}"),
                               "max_elem_err_rms": float(f"{worst:.3e}")}
        curve["1024^3"] = {"log2N": 30, **{k: sched["pencil"][k]
                                           for k in ("rel_l2", "max_elem_err_rms")}}
        out["error vs log2 N (auto schedule, FP32)"] = curve
        log(f"bench: error curve {curve}")

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
    ap.add_argument("--layout", default="natural",
                    help="layout of the timed plan (natural, shuffled)")
    ap.add_argument("--precision", default="fp32",
                    help="leaf arithmetic of the timed plan (fp32, bf16x6, ...)")
    ap.add_argument("--mfma-leaf", type=int, default=0,
                    help="split-precision leaf length of the timed plan (16, 32; 0 default)")
    ap.add_argument("--no-extras", action="store_true",
                    help="time only the 1024^3 headline workload")
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the oracle leg (and with it every error figure)")
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
    default = (shape == (1024, 1024, 1024) and args.precision == "fp32" and
               args.layout == "natural")
    base, refs = (None, {})
    if not args.no_cpu_baseline and default:
        log("bench: CPU leg (FP64 oracle: baseline timing and references)")
        base, refs = cpu_leg(x_host, not args.no_extras)
    x = torch.from_numpy(x_host).cuda()
    out = torch.empty_like(x)

    leaf = {"mfma_leaf": args.mfma_leaf} if args.mfma_leaf else {}
    plan = dft3d.Plan(shape, args.schedule, layout=args.layout, precision=args.precision,
                      **leaf)
    npass = plan.num_passes
    desc = dft3d.describe(shape, args.schedule, args.layout, precision=args.precision,
                          **leaf)
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
    if default and desc["schedule"] == "pencil":
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
        "dtype": "f32" if args.precision == "fp32" else args.precision,
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
    if "1024" in refs:
        torch.cuda.synchronize()
        result["error"] = err_fields(out.cpu().numpy(), refs["1024"])
        result["error"]["tol"] = float(f"{1e-6 * math.log2(N) / 18:.3e}")
        log(f"bench: headline error {result['error']}")
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
    plan.close()
    del x, out
    torch.cuda.empty_cache()
    if not args.no_extras and default:
        result["configs"] = extras(x_host, refs)
    if base is not None:
        result["cpu_baseline"] = base
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
