"""GPU parity: the HIP library against the FP64 oracle, element by element,
on seeded inputs (paper_1904_10119_amd.inputs), through the C ABI.

Tolerance: relative L2 error <= tol(N) = 1e-6 * log2(N) / 18 (1e-6 at 64^3,
growing with log N); the inverse round trip gets 2 * tol(N)."""
import os
import sys

import numpy as np
import pytest

import oracle
from paper_1904_10119_amd import dft3d, inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu_and_native_library():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dft3d.lib()
    maps = open("/proc/self/maps").read()
    assert "libdft3d.so" in maps, "native library not loaded"
    runtimes = {l.split()[-1] for l in maps.splitlines() if "libamdhip64" in l}
    assert len(runtimes) == 1, runtimes
    yield


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_fftn(x_np, schedule, inverse=False, **opts):
    x = torch.from_numpy(x_np).cuda()
    y = dft3d.fftn(x, schedule=schedule, inverse=inverse, **opts)
    torch.cuda.synchronize()
    return y.cpu().numpy()


def ref_fftn(x_np, sign):
    n = x_np.size
    method = "direct" if n <= (1 << 15) else "fft"
    return oracle.dft3d(x_np.astype(np.complex128), sign, method)


SCHEDULES = ["pencil", "slab", "volumetric", "auto"]


@pytest.mark.parametrize("schedule", SCHEDULES)
def test_64cubed_forward_inverse_roundtrip(schedule):
    """The 64^3 workload: forward within 1e-6 of the FP64 oracle, inverse
    within tol, round trip inv(fwd(x)) / N within 2 tol."""
    shape = (64, 64, 64)
    say("case 64^3", schedule)
    x = inputs.uniform_c64(shape, 1)
    y = gpu_fftn(x, schedule)
    ref = oracle.dft3d(x.astype(np.complex128), -1, "fft")
    err = oracle.rel_l2(y, ref)
    say("  fwd rel_l2", err)
    assert err <= 1e-6
    yi = gpu_fftn(x, schedule, inverse=True)
    refi = oracle.dft3d(x.astype(np.complex128), +1, "fft")
    assert oracle.rel_l2(yi, refi) <= 1e-6
    back = gpu_fftn(y, schedule, inverse=True) / x.size
    assert oracle.rel_l2(back, x) <= 2e-6


SHAPES = [
    (1, 1, 1), (2, 2, 2), (1, 4, 1), (8, 16, 4), (4, 8, 16), (32, 2, 64),
    (128, 64, 32), (32, 64, 128), (16, 512, 8), (1024, 4, 2), (2, 2, 1024),
    (2048, 2, 4), (4, 2048, 2), (2, 4, 4096), (4096, 2, 2),
]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("schedule", SCHEDULES)
def test_shapes_and_lengths(shape, schedule):
    """Every transform length 1..4096 on every schedule, anisotropic shapes
    (catch axis mix-ups), tiles larger than the batch (ragged tails)."""
    say("case", shape, schedule)
    x = inputs.uniform_c64(shape, 21)
    n = x.size
    for sign, inv in ((-1, False), (1, True)):
        y = gpu_fftn(x, schedule, inverse=inv)
        err = oracle.rel_l2(y, ref_fftn(x, sign))
        assert err <= oracle.tol(n), (shape, schedule, sign, err)


@pytest.mark.parametrize("tile", [8, 16, 32, 64, 128, 256])
def test_tile_variants(tile):
    shape = (64, 128, 32)
    x = inputs.uniform_c64(shape, 22)
    ref = ref_fftn(x, -1)
    for sched in ("pencil", "slab", "volumetric"):
        y = gpu_fftn(x, sched, tile=tile)
        assert oracle.rel_l2(y, ref) <= oracle.tol(x.size), (tile, sched)


@pytest.mark.parametrize("split_max", [2, 16, 64])
def test_pencil_with_split_axes(split_max):
    """Pencil rotation with every long axis split four-step (V1 + V2)."""
    shape = (256, 128, 64)
    x = inputs.uniform_c64(shape, 23)
    ref = ref_fftn(x, -1)
    y = gpu_fftn(x, "auto", split_max=split_max)
    assert oracle.rel_l2(y, ref) <= oracle.tol(x.size)


def test_256cubed_all_schedules():
    shape = (256, 256, 256)
    x = inputs.uniform_c64(shape, 3)
    ref = oracle.dft3d(x.astype(np.complex128), -1, "fft")
    for sched in SCHEDULES:
        say("case 256^3", sched)
        y = gpu_fftn(x, sched)
        err = oracle.rel_l2(y, ref)
        say("  rel_l2", err)
        assert err <= oracle.tol(x.size)


def test_deterministic_and_input_untouched():
    x = inputs.uniform_c64((128, 128, 128), 24)
    xt = torch.from_numpy(x).cuda()
    a = dft3d.fftn(xt, schedule="pencil")
    b = dft3d.fftn(xt, schedule="pencil")
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    assert np.array_equal(xt.cpu().numpy(), x)


def test_schedules_agree():
    x = inputs.uniform_c64((128, 256, 64), 25)
    xt = torch.from_numpy(x).cuda()
    outs = {s: dft3d.fftn(xt, schedule=s).cpu().numpy() for s in SCHEDULES}
    for s in SCHEDULES:
        assert oracle.rel_l2(outs[s], outs["pencil"]) <= 2 * oracle.tol(x.size)


def test_execute_rejects_aliasing_and_bad_sign():
    p = dft3d.Plan((8, 8, 8), "pencil")
    x = torch.zeros((8, 8, 8), dtype=torch.complex64, device="cuda")
    L = dft3d.lib()
    assert L.dft3d_execute(p.handle, x.data_ptr(), x.data_ptr(), -1, None) == \
        dft3d.ERR_INVALID_ARG
    y = torch.empty_like(x)
    assert L.dft3d_execute(p.handle, x.data_ptr(), y.data_ptr(), 0, None) == \
        dft3d.ERR_INVALID_ARG
    p.bind_workspace(x.device)
    ws = torch.empty(16, dtype=torch.uint8, device="cuda")
    assert L.dft3d_set_workspace(p.handle, ws.data_ptr(), 16) == \
        dft3d.ERR_WORKSPACE_TOO_SMALL
    p.close()


@pytest.mark.parametrize("shape", [(1024, 16, 512), (512, 1024, 8), (64, 1024, 64),
                                   (2048, 8, 16), (16, 2048, 8), (4, 4, 2048)])
@pytest.mark.parametrize("schedule", ["pencil", "slab"])
def test_persistent_matches_one_tile_per_workgroup(shape, schedule):
    """The persistent prefetching kernels and the one-tile-per-workgroup
    kernels both meet the oracle tolerance and agree with each other (the
    compiler may contract the same butterflies differently, so they are not
    compared bit for bit).  Streaming accesses are forced on so that the
    persistent kernels run at these sizes too, and the two-halves kernels
    (one form only) are off."""
    x = inputs.uniform_c64(shape, 26)
    xt = torch.from_numpy(x).cuda()
    outs = []
    for pers in (0, 1):
        d = dft3d.describe(shape, schedule, persistent=pers, nontemporal=1, halves=0)
        used = [q["persistent"] for q in d["passes"] if q["n"] in (512, 1024, 2048)]
        assert used and all(u == pers for u in used), (pers, used)
        p = dft3d.Plan(shape, schedule, persistent=pers, nontemporal=1, halves=0)
        y = torch.empty_like(xt)
        p.execute(xt, y)
        torch.cuda.synchronize()
        outs.append(y.cpu().numpy())
        p.close()
    ref = ref_fftn(x, -1)
    for o in outs:
        assert oracle.rel_l2(o, ref) <= oracle.tol(x.size)
    assert oracle.rel_l2(outs[0], outs[1]) <= oracle.tol(x.size)


def full_size_check(shape, schedule, seed, nsamp=12, **opts):
    """Full-size transform in the launch configuration bench.py times:
    sampled output pencils y[k0, k1, :] against the oracle's direct sums,
    Parseval over the whole array, and the inverse round trip."""
    say("case full size", shape, schedule, opts)
    x = inputs.uniform_c64(shape, seed)
    xt = torch.from_numpy(x).cuda()
    y = dft3d.fftn(xt, schedule=schedule, **opts)
    torch.cuda.synchronize()
    N = x.size
    g = np.random.default_rng(seed)
    k0 = np.concatenate([[0, shape[0] - 1], g.integers(0, shape[0], nsamp - 2)])
    k1 = np.concatenate([[0, shape[1] // 2], g.integers(0, shape[1], nsamp - 2)])
    got = y[torch.from_numpy(k0).cuda(), torch.from_numpy(k1).cuda(), :].cpu().numpy()
    ref = oracle.sample_pencils(x, k0, k1, -1)
    err = oracle.rel_l2(got, ref)
    say("  sampled pencils rel_l2", err)
    assert err <= oracle.tol(N)
    # Parseval: sum |y|^2 = N sum |x|^2 (float64 sums on the device)
    ex = torch.sum(torch.view_as_real(xt).double() ** 2).item()
    ey = torch.sum(torch.view_as_real(y).double() ** 2).item()
    assert abs(ey / (N * ex) - 1.0) <= 2 * oracle.tol(N)
    # round trip: inverse(forward(x)) / N == x
    back = dft3d.fftn(y, schedule=schedule, inverse=True, **opts)
    d = torch.view_as_real(back).double() / N - torch.view_as_real(xt).double()
    rt = (torch.linalg.vector_norm(d) /
          torch.linalg.vector_norm(torch.view_as_real(xt).double())).item()
    say("  round trip rel_l2", rt)
    assert rt <= 2 * oracle.tol(N)
    del xt, y, back, d
    torch.cuda.empty_cache()


@pytest.mark.parametrize("schedule", ["auto", "pencil", "slab", "volumetric"])
def test_full_1024_cubed(schedule):
    full_size_check((1024, 1024, 1024), schedule, 2)


def test_full_2048x1024x512():
    full_size_check((2048, 1024, 512), "auto", 5)


@pytest.mark.parametrize("precision", ["bf16x6", "bf16x9", "fp16x3"])
def test_full_1024_cubed_split_precision(precision):
    """The split-precision leaves at full size, as the benchmark runs them."""
    full_size_check((1024, 1024, 1024), "pencil", 2, precision=precision)


def test_full_2048x1024x512_bf16x6():
    full_size_check((2048, 1024, 512), "auto", 5, precision="bf16x6")


@pytest.mark.parametrize("shape", [(4096, 4096, 16), (16, 4096, 4096)])
def test_longest_axes(shape):
    """The longest supported axes (4096, split four-step by the auto
    schedule: five passes) in a 2 GiB array."""
    d = dft3d.describe(shape, "auto")
    assert d["schedule"] == "pencil" and len(d["passes"]) == 5
    full_size_check(shape, "auto", 7, nsamp=8)


@pytest.mark.parametrize("group", [1, 4, 16])
def test_slab_plane_groups(group):
    """Slab with the planes processed in groups (rows then columns per
    group): forward and inverse against the oracle."""
    shape = (64, 128, 64)
    x = inputs.uniform_c64(shape, 27)
    for sign, inv in ((-1, False), (1, True)):
        y = gpu_fftn(x, "slab", inverse=inv, slab_group=group)
        assert oracle.rel_l2(y, ref_fftn(x, sign)) <= oracle.tol(x.size), (group, sign)


@pytest.mark.parametrize("shape,group", [((64, 64, 64), 8), ((32, 128, 64), 4),
                                         ((16, 32, 256), 1), ((8, 16, 32), 2)])
def test_grouped_pencil_matches_oracle(shape, group):
    """Pencil schedule with its first two passes taken in groups of planes:
    forward and inverse against the oracle."""
    say("case grouped pencil", shape, group)
    x = inputs.uniform_c64(shape, 31)
    for sign, inv in ((-1, False), (1, True)):
        y = gpu_fftn(x, "pencil", inverse=inv, pencil_group=group)
        assert oracle.rel_l2(y, ref_fftn(x, sign)) <= oracle.tol(x.size), (group, sign)


def test_grouped_pencil_one_sided_kernels_bitwise():
    """(32, 1024, 1024) in groups of 8 planes runs the length-1024 passes
    with streaming loads only (first pass) and streaming stores only
    (second pass): the same arithmetic as the ungrouped schedule in the
    rotation's order (the order grouping keeps), so the results match it bit
    for bit, forward and inverse, and the oracle on sampled outputs."""
    shape = (32, 1024, 1024)
    say("case grouped pencil one-sided", shape)
    d = dft3d.describe(shape, "pencil", pencil_group=8)
    assert [p["nontemporal"] for p in d["passes"][:2]] == [2, 3] and len(d["passes"]) == 9
    x = torch.from_numpy(inputs.uniform_c64(shape, 32)).cuda()
    for inv in (False, True):
        y0 = dft3d.fftn(x, schedule="pencil", inverse=inv, pencil_group=0, pencil_order=0)
        y1 = dft3d.fftn(x, schedule="pencil", inverse=inv, pencil_group=8)
        torch.cuda.synchronize()
        assert torch.equal(y0, y1), inv
    # sampled outputs of the forward transform by direct sums
    y = dft3d.fftn(x, schedule="pencil", pencil_group=8).cpu().numpy()
    xs = x.cpu().numpy().astype(np.complex128)
    g = np.random.default_rng(3)
    ks = [tuple(int(g.integers(0, n)) for n in shape) for _ in range(4)] + [(0, 0, 0), (31, 1023, 1023)]
    for k in ks:
        w = [np.exp(-2j * np.pi * k[d] * np.arange(shape[d]) / shape[d]) for d in range(3)]
        ref = np.einsum("ijk,i,j,k->", xs, w[0], w[1], w[2])
        assert abs(y[k] - ref) <= 1e-5 * np.sqrt(np.sum(np.abs(xs) ** 2)), k


def test_grouped_pencil_plans_in_a_batch():
    """Plans with grouped first passes in one batched call, next to an
    ordinary plan: every result equals its single execution bit for bit,
    forward and inverse."""
    import ctypes
    shapes = [(16, 32, 64), (32, 64, 16), (8, 8, 8)]
    groups = [4, 8, 0]
    plans = [dft3d.Plan(s, "pencil", pencil_group=g) for s, g in zip(shapes, groups)]
    xs = [torch.from_numpy(inputs.uniform_c64(s, 70 + i)).cuda() for i, s in enumerate(shapes)]
    for p, x in zip(plans, xs):
        p.bind_workspace(x.device)
    assert sum(" group " in q["label"] for q in dft3d.describe(shapes[0], "pencil",
                                                                pencil_group=4)["passes"]) == 8
    arr = ctypes.c_void_p * len(plans)
    for inverse in (False, True):
        outs = [torch.empty_like(x) for x in xs]
        st = dft3d.lib().dft3d_execute_batched(
            arr(*[p.handle.value for p in plans]), arr(*[x.data_ptr() for x in xs]),
            arr(*[o.data_ptr() for o in outs]), len(plans), 1 if inverse else -1,
            torch.cuda.current_stream().cuda_stream)
        assert st == 0
        for p, x, o in zip(plans, xs, outs):
            single = torch.empty_like(x)
            p.execute(x, single, inverse=inverse)
            torch.cuda.synchronize()
            assert torch.equal(o, single), (x.shape, inverse)
    for p in plans:
        p.close()


def test_autotune_records_choice_for_auto_plans(tmp_path, monkeypatch):
    """The autotuner times the candidates, records the fastest, and later
    auto plans of that shape use it (and still match the oracle); the
    choice is written to and read back from the cache file."""
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("DFT3D_TUNE_CACHE", str(cache))
    shape = (128, 32, 64)
    r = dft3d.autotune(shape)
    say("autotune", shape, r)
    assert r["schedule"] in ("pencil", "slab", "volumetric") and r["ms"] > 0
    assert cache.exists() and f"{shape[0]} {shape[1]} {shape[2]}" in cache.read_text()
    x = inputs.uniform_c64(shape, 28)
    p = dft3d.Plan(shape, "auto")
    y = torch.empty(shape, dtype=torch.complex64, device="cuda")
    p.execute(torch.from_numpy(x).cuda(), y)
    torch.cuda.synchronize()
    assert oracle.rel_l2(y.cpu().numpy(), ref_fftn(x, -1)) <= oracle.tol(x.size)
    p.close()


@pytest.mark.parametrize("n1", [16, 32, 64, 128])
@pytest.mark.parametrize("n2", [16, 32, 64, 128])
def test_slab_fused_plane_kernel(n1, n2):
    """Every fused plane shape: forward and inverse against the oracle, and
    against the unfused row + column passes."""
    shape = (4, n1, n2)
    say("case fused plane", shape)
    x = inputs.uniform_c64(shape, 29)
    d = dft3d.describe(shape, "slab")
    assert d["passes"][0]["plane_rows"] == n1 and len(d["passes"]) == 2
    for sign, inv in ((-1, False), (1, True)):
        y = gpu_fftn(x, "slab", inverse=inv)
        assert oracle.rel_l2(y, ref_fftn(x, sign)) <= oracle.tol(x.size), (sign,)
        y0 = gpu_fftn(x, "slab", inverse=inv, fused_plane=0)
        assert oracle.rel_l2(y, y0) <= oracle.tol(x.size)


def test_batched_runs_fused_plane_plans_as_twins():
    """Batched execution of slab plans whose planes are fused: the batch
    runs their one-dimensional twins and matches single execution."""
    shapes = [(64, 64, 64), (32, 128, 16), (16, 16, 16), (128, 32, 64)]
    xs = [inputs.uniform_c64(s, 60 + i) for i, s in enumerate(shapes)]
    xt = [torch.from_numpy(x).cuda() for x in xs]
    for inv, sign in ((False, -1), (True, 1)):
        ys = dft3d.fftn_batched(xt, schedule="slab", inverse=inv)
        torch.cuda.synchronize()
        for x, y in zip(xs, ys):
            assert oracle.rel_l2(y.cpu().numpy(), ref_fftn(x, sign)) <= oracle.tol(x.size)


def test_error_against_size_sweep():
    """Accuracy curve from 8^3 to 256^3 (auto schedule, uniform inputs):
    every size within tol(N); the measured values are printed for the
    record."""
    errs = {}
    for n in (8, 16, 32, 64, 128, 256):
        shape = (n, n, n)
        x = inputs.uniform_c64(shape, 11)
        for sched in ("auto", "pencil"):
            y = gpu_fftn(x, sched)
            err = oracle.rel_l2(y, oracle.dft3d(x.astype(np.complex128), -1, "fft"))
            errs[(n, sched)] = err
            assert err <= oracle.tol(x.size), (n, sched, err)
    say("error curve", {f"{k[0]}^3 {k[1]}": "%.3e" % v for k, v in errs.items()})


@pytest.mark.parametrize("shape", [(2, 256, 256), (256, 256, 32), (2, 1024, 512),
                                   (1024, 512, 16), (256, 256, 256)])
def test_volumetric_fused_axes_kernels(shape):
    """Each fused volumetric two-axis kernel (split factor 16 or 32, runs
    contiguous or strided): forward and inverse against the oracle and
    against the unfused six-pass list."""
    say("case fused axes", shape)
    d = dft3d.describe(shape, "volumetric")
    assert any(p["fused_axes"] for p in d["passes"])
    x = inputs.uniform_c64(shape, 30)
    for sign, inv in ((-1, False), (1, True)):
        y = gpu_fftn(x, "volumetric", inverse=inv)
        assert oracle.rel_l2(y, ref_fftn(x, sign)) <= oracle.tol(x.size), (sign,)
        y0 = gpu_fftn(x, "volumetric", inverse=inv, fused_axes=0)
        assert oracle.rel_l2(y, y0) <= oracle.tol(x.size)
        # the persistent (prefetching) form of the fused kernels
        dp = dft3d.describe(shape, "volumetric", nontemporal=1)
        assert all(p["persistent"] for p in dp["passes"] if p["fused_axes"])
        yp = gpu_fftn(x, "volumetric", inverse=inv, nontemporal=1)
        assert oracle.rel_l2(yp, ref_fftn(x, sign)) <= oracle.tol(x.size), (sign, "pers")
