"""GPU parity for lengths that are not powers of two, through the C ABI,
against the FP64 oracle's direct sums: the mixed-radix pass (prime factors
at most 13) and the Bluestein pass (other lengths, convolution length up
to 8192).

Tolerance: each power-of-two axis of length n contributes log2(n) rounding
levels, as in tol(N); a mixed-radix axis log2(n) + 1 (its odd radices are
computed from pairs with rounded constants); a Bluestein axis (convolution
length m) 2 log2(m) + 3: two FFTs of length m plus the chirp multiply
before, the filter multiply between and the chirp multiply after them.  The
bar is 1e-6 / 18 per level, the same rate as tol(N)."""
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
    assert "libdft3d.so" in open("/proc/self/maps").read(), "native library not loaded"
    yield


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def smooth13(n):
    for f in (2, 3, 5, 7, 11, 13):
        while n % f == 0:
            n //= f
    return n == 1


def levels(shape):
    out = 0.0
    for n in shape:
        if n & (n - 1) == 0:
            out += np.log2(n) if n > 1 else 0.0
        elif smooth13(n):
            out += np.log2(n) + 1
        else:
            m = 1 << int(np.ceil(np.log2(2 * n - 1)))
            out += 2 * np.log2(m) + 3
    return max(out, 1.0)


def tol_bl(shape):
    return 1e-6 * levels(shape) / 18.0


def gpu_fftn(x_np, inverse=False, schedule="pencil"):
    y = dft3d.fftn(torch.from_numpy(x_np).cuda(), schedule=schedule, inverse=inverse)
    torch.cuda.synchronize()
    return y.cpu().numpy()


SHAPES = [
    # mixed radix (prime factors <= 13), every tile shape of the kernel
    (3, 5, 7), (6, 10, 12), (1, 1, 3), (9, 1, 1), (2, 3, 4), (11, 13, 26),
    (64, 100, 64), (12, 7, 16), (15, 8, 2048), (3, 2000, 7), (96, 96, 96),
    (33, 65, 1001), (4095, 2, 3), (3, 3000, 2), (120, 384, 5), (243, 169, 4),
    # Bluestein (a prime factor above 13), with mixed and power-of-two axes
    (1, 17, 1), (100, 30, 17), (2047, 5, 3), (5, 3, 1025), (19, 23, 31),
    (1009, 2, 6), (2039, 3, 1), (34, 37, 8),
    # Bluestein with convolution length 8192 (lengths above 2048)
    (4093, 2, 3), (3, 2062, 2),
]


_refs = {}


def direct_ref(x, sign):
    """The oracle's direct sums of x (kept for the next schedule of the same
    shape)."""
    key = (x.shape, sign)
    if key not in _refs:
        if len(_refs) > 8:
            _refs.clear()
        _refs[key] = oracle.dft3d(x.astype(np.complex128), sign, "direct")
    return _refs[key]


@pytest.mark.parametrize("schedule", ["pencil", "auto", "slab", "volumetric"])
@pytest.mark.parametrize("shape", SHAPES)
def test_other_lengths_forward_inverse(shape, schedule):
    """Every schedule: the pencil passes rotate; slab and volumetric keep the
    layout (an axis that is not a power of two runs as one pass in layout,
    with the general pencil index where the pencil counts need it)."""
    say("case other length", shape, schedule)
    x = inputs.uniform_c64(shape, 31)
    t = tol_bl(shape)
    for sign, inv in ((-1, False), (1, True)):
        y = gpu_fftn(x, inv, schedule)
        ref = direct_ref(x, sign)
        err = oracle.rel_l2(y, ref)
        say("  sign", sign, "rel_l2", err, "tol", t)
        assert err <= t, (shape, sign, err)


@pytest.mark.parametrize("shape", [(3, 5, 7), (100, 30, 17), (2047, 5, 3), (1000, 12, 9)])
def test_other_lengths_round_trip(shape):
    x = inputs.uniform_c64(shape, 32)
    y = gpu_fftn(x)
    back = gpu_fftn(y, inverse=True) / x.size
    assert oracle.rel_l2(back, x) <= 2 * tol_bl(shape)


def test_other_lengths_special_inputs():
    """Impulse at the origin gives all ones; a constant gives N at the
    origin only; a shifted impulse gives the product of the axis roots."""
    shape = (6, 10, 12)
    N = 6 * 10 * 12
    x = np.zeros(shape, np.complex64)
    x[0, 0, 0] = 1
    y = gpu_fftn(x)
    assert np.max(np.abs(y - 1)) < 1e-6
    y = gpu_fftn(np.ones(shape, np.complex64))
    ref = np.zeros(shape)
    ref[0, 0, 0] = N
    assert np.max(np.abs(y - ref)) < 1e-6 * N
    x = np.zeros(shape, np.complex64)
    x[1, 3, 5] = 1
    k = np.indices(shape)
    ref = np.exp(-2j * np.pi * (k[0] * 1 / 6 + k[1] * 3 / 10 + k[2] * 5 / 12))
    assert np.max(np.abs(gpu_fftn(x) - ref)) < 2e-6


@pytest.mark.parametrize("shape,schedule", [((1000, 1000, 100), "auto"),
                                            ((1009, 1000, 64), "auto"),
                                            ((1000, 1000, 100), "slab"),
                                            ((1009, 1000, 64), "volumetric")])
def test_other_lengths_full_size_sampled(shape, schedule):
    """1000 x 1000 x 100 (mixed radix on every axis) and 1009 x 1000 x 64
    (Bluestein, mixed radix, power of two): sampled output pencils against
    the oracle's direct sums, Parseval, round trip."""
    say("case other lengths full size", shape, schedule)
    x = inputs.uniform_c64(shape, 33)
    xt = torch.from_numpy(x).cuda()
    y = dft3d.fftn(xt, schedule=schedule)
    torch.cuda.synchronize()
    N = x.size
    t = tol_bl(shape)
    g = np.random.default_rng(33)
    k0 = np.concatenate([[0, shape[0] - 1, shape[0] // 2], g.integers(0, shape[0], 5)])
    k1 = np.concatenate([[0, 1, shape[1] - 1], g.integers(0, shape[1], 5)])
    got = y[torch.from_numpy(k0).cuda(), torch.from_numpy(k1).cuda(), :].cpu().numpy()
    ref = oracle.sample_pencils(x, k0, k1, -1)
    err = oracle.rel_l2(got, ref)
    say("  sampled pencils rel_l2", err, "tol", t)
    assert err <= t
    ex = torch.sum(torch.view_as_real(xt).double() ** 2).item()
    ey = torch.sum(torch.view_as_real(y).double() ** 2).item()
    assert abs(ey / (N * ex) - 1.0) <= 2 * t
    back = dft3d.fftn(y, schedule=schedule, inverse=True)
    d = torch.view_as_real(back).double() / N - torch.view_as_real(xt).double()
    rt = (torch.linalg.vector_norm(d) /
          torch.linalg.vector_norm(torch.view_as_real(xt).double())).item()
    say("  round trip rel_l2", rt)
    assert rt <= 2 * t
    del xt, y, back, d
    torch.cuda.empty_cache()


def test_other_lengths_in_a_batch():
    """A batch holding plans of other lengths runs plan by plan and still
    matches."""
    shapes = [(3, 5, 7), (16, 16, 16), (6, 10, 17)]
    xs = [inputs.uniform_c64(s, 40 + i) for i, s in enumerate(shapes)]
    ys = dft3d.fftn_batched([torch.from_numpy(x).cuda() for x in xs])
    torch.cuda.synchronize()
    for x, y in zip(xs, ys):
        ref = oracle.dft3d(x.astype(np.complex128), -1, "direct")
        assert oracle.rel_l2(y.cpu().numpy(), ref) <= tol_bl(x.shape)


def test_other_lengths_rejected_forms():
    """Split-precision leaves and the shuffled layout are powers of two only."""
    x = torch.zeros((3, 4, 4), dtype=torch.complex64, device="cuda")
    for sched in ("pencil", "slab", "volumetric"):
        with pytest.raises(dft3d.Dft3dError):
            dft3d.fftn(x, schedule=sched, precision="bf16x6")
    with pytest.raises(dft3d.Dft3dError):
        dft3d.fftn(x, schedule="volumetric", layout="shuffled")


@pytest.mark.parametrize("tile", [1, 2, 4, 8])
def test_bluestein_tile_variants(tile):
    """The Bluestein pass's tile variants (the tile option; lengths without a
    variant of that tile keep their default) give the same transform."""
    shape = (2039, 6, 20)  # m = 4096 on the first axis, 32 on the last
    say("case bluestein tile", tile)
    x = inputs.uniform_c64(shape, 50)
    y = dft3d.fftn(torch.from_numpy(x).cuda(), schedule="pencil", tile=tile)
    torch.cuda.synchronize()
    ref = oracle.dft3d(x.astype(np.complex128), -1, "direct")
    assert oracle.rel_l2(y.cpu().numpy(), ref) <= tol_bl(shape)


def test_every_length_up_to_300():
    """Every length 1..300 along the contiguous axis (powers of two, every
    radix packing of the mixed-radix pass, Bluestein lengths with m = 8..1024)
    against the oracle's direct sums, forward and inverse."""
    worst = 0.0
    for n in range(1, 301):
        shape = (3, 4, n)
        x = inputs.uniform_c64(shape, 1000 + n)
        for sign, inv in ((-1, False), (1, True)):
            y = gpu_fftn(x, inv)
            err = oracle.rel_l2(y, oracle.dft3d(x.astype(np.complex128), sign, "direct"))
            assert err <= tol_bl(shape), (n, sign, err)
            worst = max(worst, err / tol_bl(shape))
    say("  worst error / bar over lengths 1..300:", worst)


@pytest.mark.parametrize("n", [2047, 2049, 2050, 2053, 2187, 3001, 3003, 3125, 4093, 4095])
def test_lengths_near_the_limits(n):
    """Lengths around 2048 and up to 4095 along the outermost axis."""
    shape = (n, 2, 3)
    x = inputs.uniform_c64(shape, 2000 + n)
    y = gpu_fftn(x)
    err = oracle.rel_l2(y, oracle.dft3d(x.astype(np.complex128), -1, "direct"))
    say("  n", n, "rel_l2", err)
    assert err <= tol_bl(shape), (n, err)


@pytest.mark.parametrize("n", [48, 60, 72, 80, 96, 100, 120, 125, 144, 160, 192, 200, 240, 250,
                               300, 320, 384, 400, 480, 500, 600, 640, 768, 800, 960, 1000,
                               1200, 1536, 2000, 2400, 2500, 3000, 3072, 3200, 3600, 4000,
                               56, 112, 168, 224, 336, 448, 672, 896, 1008, 1344, 1792, 2016])
def test_fixed_length_kernels(n):
    """The lengths with a kernel compiled for them, on the innermost and the
    outermost axis, forward and inverse, against direct sums."""
    for shape in ((2, 3, n), (n, 3, 2)):
        x = inputs.uniform_c64(shape, 3000 + n)
        for sign, inv in ((-1, False), (1, True)):
            y = gpu_fftn(x, inv)
            err = oracle.rel_l2(y, oracle.dft3d(x.astype(np.complex128), sign, "direct"))
            assert err <= tol_bl(shape), (shape, sign, err)


RADIX_CASES = [((4, 2, 1000), [10, 10, 10]), ((4, 2, 1000), [8, 5, 5, 5]),
               ((2, 4, 1024), [4, 4, 4, 4, 4]), ((2, 4, 64), [4, 16]), ((8, 3, 96), [2, 3, 16]),
               ((6, 4, 143), [13, 11]), ((2, 2, 2048), [8, 8, 8, 4]), ((2, 8, 8), [2, 4]),
               ((16, 1000, 3), [5, 8, 5, 5])]


@pytest.mark.parametrize("shape,radices", RADIX_CASES)
def test_radix_sequence_option(shape, radices):
    """DFT3D_OPT_RADICES: the passes of the sequence's length run the
    mixed-radix kernel with those stages (powers of two included), forward
    and inverse against the oracle's direct sums, and against the default
    plan."""
    say("case radices", shape, radices)
    x = inputs.uniform_c64(shape, 50)
    xt = torch.from_numpy(x).cuda()
    t = tol_bl(shape) + 1e-6 / 18  # one more rounding level at most for the stage order
    for sign, inv in ((-1, False), (1, True)):
        p = dft3d.Plan(shape, "pencil", radices=radices)
        assert p.get_option(dft3d.OPT_RADICES) == dft3d.radix_code(radices)
        y = torch.empty_like(xt)
        p.execute(xt, y, inverse=inv)
        torch.cuda.synchronize()
        p.close()
        got = y.cpu().numpy()
        ref = direct_ref(x, sign)
        err = oracle.rel_l2(got, ref)
        say("  sign", sign, "rel_l2", err)
        assert err <= t, (shape, radices, sign, err)
        assert oracle.rel_l2(got, gpu_fftn(x, inv)) <= 2 * t


def test_autotune_other_lengths_radix_candidates(tmp_path, monkeypatch):
    """The autotuner on a shape with mixed-radix axes also times other radix
    sequences; the recorded choice (whatever wins) is written to the cache
    file with its radix code, and a later AUTO plan of the shape matches the
    oracle."""
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("DFT3D_TUNE_CACHE", str(cache))
    shape = (60, 100, 96)
    r = dft3d.autotune(shape)
    say("autotune", shape, r)
    assert r["ms"] > 0
    line = [l for l in cache.read_text().splitlines() if " 60 100 96 " in l]
    assert len(line) == 1 and len(line[0].split()) == 14, line
    x = inputs.uniform_c64(shape, 51)
    y = gpu_fftn(x, schedule="auto")
    assert oracle.rel_l2(y, direct_ref(x, -1)) <= tol_bl(shape) + 1e-6 / 18


RADER_PRIMES = [17, 19, 23, 29, 31, 37, 41, 43, 53, 61, 73, 97, 101, 109, 151, 181, 211, 241,
                271, 337, 401, 421, 449, 577, 601, 641, 673, 757, 769, 883, 1009, 1051, 1201,
                1297, 1459, 1601, 2003, 2017, 2161, 2593, 3001, 3137, 4001]


RADER_COMPILED = {197, 257, 281, 401, 577, 641, 769, 1009, 1201, 1601, 2017, 2593, 3001,
                  4001}


def run_plan(x, inverse, **kw):
    xt = torch.from_numpy(x).cuda()
    p = dft3d.Plan(x.shape, "pencil", **kw)
    y = torch.empty_like(xt)
    p.execute(xt, y, inverse=inverse)
    torch.cuda.synchronize()
    p.close()
    return y.cpu().numpy()


@pytest.mark.parametrize("n", sorted(set(RADER_PRIMES) | RADER_COMPILED))
def test_rader_lengths(n):
    """Primes n with n - 1 free of prime factors above 13 through the Rader
    pass (two mixed-radix FFTs of length n - 1 in LDS): the compiled-length
    kernel (the default for its primes) and the generic one
    (DFT3D_OPT_RADER = 2), forward and inverse against the oracle's direct
    sums, along a contiguous and a strided axis, and the Bluestein pass
    (DFT3D_OPT_RADER = 0) of the same plan."""
    for shape in ((3, 2, n), (n, 2, 3)):
        d = dft3d.describe(shape, "pencil")
        assert any(p["rader"] and p["rader_n"] == n for p in d["passes"]) == (n in RADER_COMPILED)
        say("case rader", shape)
        x = inputs.uniform_c64(shape, 60)
        for sign, inv in ((-1, False), (1, True)):
            ref = direct_ref(x, sign)
            for kw in ({}, {"rader": 2}, {"rader": 0}):
                err = oracle.rel_l2(run_plan(x, inv, **kw), ref)
                say("  sign", sign, kw, "rel_l2", err)
                assert err <= tol_bl(shape), (shape, sign, kw, err)
