"""CPU model of the planner's index arithmetic.

For every pass of every schedule the library plans, the kernel reads
element j of pencil b at
  (b >> s1) is2 + ((b >> s0) & m1) is1 + (b & m0) is0 + j ijs
and writes output k at the same form with the output strides.  These tests
check (a) that each pass's read and write maps are bijections onto
[0, N) -- so no kernel can touch memory outside its buffers -- and (b) that
running the pass list with a plain per-pencil DFT reproduces the oracle's 3D
DFT, which checks the schedules' index math without a GPU."""
import numpy as np
import pytest

import oracle
from paper_1904_10119_amd import dft3d

SCHEDULES = ["auto", "slab", "pencil", "volumetric"]
SHAPES = [(1, 1, 1), (2, 4, 8), (8, 2, 4), (16, 16, 16), (32, 4, 64), (4, 64, 2),
          (2, 256, 8), (64, 1, 32), (4096, 2, 1), (1, 2, 2048)]


def fields(args, b=None):
    """The pencil index split into its three fields: bit fields, or with
    s0 = -1 the general form b mod m0, (b div m0) mod m1, b div (m0 m1)."""
    if b is None:
        b = np.arange(args["B"], dtype=np.int64)
    if args["s0"] < 0:
        m0, m1 = args["m0"], args["m1"]
        return b % m0, (b // m0) % m1, b // (m0 * m1)
    return b & args["m0"], (b >> args["s0"]) & args["m1"], b >> args["s1"]


def addresses(args, n, inp):
    st = args["is"] if inp else args["os"]
    js = args["ijs"] if inp else args["oks"]
    f0, f1, f2 = fields(args)
    base = f2 * st[2] + f1 * st[1] + f0 * st[0]
    j = np.arange(n, dtype=np.int64)
    return base[:, None] + j[None, :] * js        # (B, n)


def pass_points(p):
    """Points one work item (pencil, or plane for fused plane passes) covers."""
    if p.get("bluestein"):
        return p["bl_n"]
    if p.get("mixed") or p.get("rader"):
        return p["args"]["res_mask"]
    return p["n"] * max(1, p.get("plane_rows", 0))


def fused_tiles(p):
    """(input, output) element addresses of a fused volumetric two-axis pass,
    shaped (tile, m, kk, c, l) and (tile, k2, kk, c, l') -- the kernel's
    documented argument fields read back literally."""
    a = p["args"]
    A, KC = p["n"], p["tile"]
    contig = p["load"] == "row"
    K, C = (KC, 1) if contig else (1, KC)
    t = np.arange(a["B"], dtype=np.int64)
    f0, f1, f2 = t & a["m0"], (t >> a["s0"]) & a["m1"], t >> a["s1"]
    ib = f0 * a["is"][0] + f1 * a["is"][1] + f2 * a["is"][2]
    ob = f0 * a["os"][0] + f1 * a["os"][1] + f2 * a["os"][2]
    RM, SD, b = a["ijs"], a["oks"], a["res_mask"]
    m = np.arange(A)[None, :, None, None, None]
    kk = np.arange(K)[None, None, :, None, None]
    c = np.arange(C)[None, None, None, :, None]
    l = np.arange(A)[None, None, None, None, :]
    ia = ib[:, None, None, None, None] + m * RM + (kk * A + l) * SD + c
    if p["fused_axes"] in (2, 3):   # shuffled order: in place
        oa = ob[:, None, None, None, None] + m * RM + (kk * A + l) * SD + c
    else:
        oa = ob[:, None, None, None, None] + m * RM + (kk + b * l) * SD + c
    if p["fused_axes"] == 3:        # the run index k' of the tile's runs kk
        run = (f0[:, None] * KC + np.arange(K)[None, :]) if contig else \
            np.broadcast_to(f2[:, None], (f2.size, K))
        return ia, oa, run
    return ia, oa, f1


def fused_model(bufs, p, sign, last):
    ia, oa, r = fused_tiles(p)
    v = bufs[p["src"]][ia]
    if sign == 1 and p["src"] == "in":
        v = np.conj(v)
    if p["fused_axes"] == 3:
        # inverse from the shuffled order: W2 of axis d-1 (DFT over the rows
        # m; with res_shift = 1 first the twiddle w^{r' m} of axis d-1's W1,
        # table length tw_len), then W1 of axis d (DFT over l' of run k',
        # times w_L^{k' a'})
        a = p["args"]
        if a["res_shift"]:
            Lr = a["tw_len"]
            m = np.arange(p["n"])
            r1 = fused_tiles(dict(p, fused_axes=2))[2]       # the residue r'
            pre = np.exp(-2j * np.pi * ((r1[:, None] * m[None, :]) % Lr) / Lr)
            v = v * pre[:, :, None, None, None]
        v = np.fft.fft(v, axis=1)
        v = np.fft.fft(v, axis=4)
        L = p["args"]["twp_len"]
        ap = np.arange(p["n"])
        tw = np.exp(-2j * np.pi * ((r[:, :, None] * ap[None, None, :]) % L) / L)
        v = v * tw[:, None, :, None, :]
        if sign == 1 and last:
            v = np.conj(v)
        bufs[p["dst"]][oa] = v
        return
    v = np.fft.fft(v, axis=4)            # V2 of axis d: DFT_a over l
    v = np.fft.fft(v, axis=1)            # V1 of axis d-1: DFT over the rows m
    L = p["args"]["twp_len"]
    k2 = np.arange(p["n"])
    tw = np.exp(-2j * np.pi * ((r[:, None] * k2[None, :]) % L) / L)
    v = v * tw[:, :, None, None, None]
    if sign == 1 and last:
        v = np.conj(v)
    bufs[p["dst"]][oa] = v


def bluestein_model(bufs, p, sign, last):
    """A one-pass Bluestein axis from its documented steps (chirp-z identity:
    w[j] = exp(-pi i j^2 / n); pad x w to length m, FFT_m, times H / m with
    H = FFT_m of the wrapped conj(w), FFT_m, read back at (m - k) mod m,
    times w[k]), computed in numpy independently of the library's tables."""
    a = p["args"]
    n, m = p["bl_n"], p["n"]
    ia = addresses(a, n, True)
    oa = addresses(a, n, False)
    v = bufs[p["src"]][ia + p["in_off"]]                   # (B, n)
    if sign == 1 and p["src"] == "in":
        v = np.conj(v)
    j = np.arange(n)
    w = np.exp(-1j * np.pi * ((j * j) % (2 * n)) / n)
    h = np.zeros(m, complex)
    h[:n] = np.conj(w)
    h[m - np.arange(1, n)] = np.conj(w[1:])
    H = np.fft.fft(h) / m
    pad = np.zeros((v.shape[0], m), complex)
    pad[:, :n] = v * w[None, :]
    c = np.fft.fft(np.fft.fft(pad, axis=1) * H[None, :], axis=1)
    y = c[:, (m - j) % m] * w[None, :]
    if sign == 1 and last:
        y = np.conj(y)
    bufs[p["dst"]][oa + p["out_off"]] = y


def run_model(x, d, sign, key=None):
    """Run a pass list; by default the one execute uses for `sign` (a
    shuffled plan's inverse runs its "inverse_passes")."""
    n_total = x.size
    n_ws = max(n_total, d["workspace_bytes"] // 8)
    bufs = {"in": x.reshape(-1).astype(np.complex128),
            "out": np.full(n_total, np.nan, np.complex128),
            "ws": np.full(n_ws, np.nan, np.complex128)}
    if key is None:
        key = "inverse_passes" if (sign == 1 and "inverse_passes" in d) else "passes"
    passes = d[key]
    for i, p in enumerate(passes):
        a = p["args"]
        if p.get("fused_axes"):
            fused_model(bufs, p, sign, i == len(passes) - 1)
            continue
        if p.get("bluestein"):
            bluestein_model(bufs, p, sign, i == len(passes) - 1)
            continue
        ia = addresses(a, pass_points(p), True)
        oa = addresses(a, pass_points(p), False)
        v = bufs[p["src"]][ia + p["in_off"]]
        if sign == 1 and p["src"] == "in":
            v = np.conj(v)
        if p.get("plane_rows", 0):   # fused 2D DFT of contiguous planes
            n1 = p["plane_rows"]
            y = np.fft.fft2(v.reshape(-1, n1, p["n"])).reshape(v.shape)
        else:
            y = np.fft.fft(v, axis=1)
        if p["post_twiddle"]:
            L = a["twp_len"]
            res = (np.arange(a["B"]) >> a["res_shift"]) & a["res_mask"]
            k = np.arange(p["n"])
            y = y * np.exp(-2j * np.pi * ((res[:, None] * k[None, :]) % L) / L)
        if sign == 1 and i == len(passes) - 1:
            y = np.conj(y)
        bufs[p["dst"]][oa + p["out_off"]] = y
    return bufs["out"].reshape(x.shape)


@pytest.mark.parametrize("shape", SHAPES + [(1024, 1024, 1024), (2048, 1024, 512),
                                            (4096, 4096, 4)])
@pytest.mark.parametrize("schedule", SCHEDULES + ["slab-grouped"])
def test_pass_maps_are_injective_and_in_bounds(shape, schedule):
    if schedule == "slab-grouped":
        d = dft3d.describe(shape, "slab", slab_group=max(1, shape[0] // 4))
    else:
        d = dft3d.describe(shape, schedule)
    check_pass_maps(d, shape[0] * shape[1] * shape[2])


def check_pass_maps(d, N):
    """Every pass reads and writes inside its N-point buffers, each point
    once (sampled for very large passes)."""
    for p in d["passes"]:
        a = p["args"]
        if p.get("fused_axes"):
            if a["B"] * p["n"] * p["n"] * p["tile"] <= (1 << 22):
                ia, oa, _ = fused_tiles(p)
                for addr in (ia.reshape(-1), oa.reshape(-1)):
                    assert addr.min() >= 0 and addr.max() < N, p["label"]
                    assert np.unique(addr).size == addr.size, p["label"]
            continue
        if a["B"] * pass_points(p) > (1 << 22):
            # sampled: the first, last and a middle block of pencils
            B = a["B"]
            for lo in (0, B // 2, B - 64):
                b = np.arange(lo, lo + 64, dtype=np.int64)
                for inp in (True, False):
                    st = a["is"] if inp else a["os"]
                    js = a["ijs"] if inp else a["oks"]
                    f0, f1, f2 = fields(a, b)
                    base = f2 * st[2] + f1 * st[1] + f0 * st[0]
                    off = p["in_off"] if inp else p["out_off"]
                    hi = base.max() + (pass_points(p) - 1) * js + off
                    assert base.min() + off >= 0 and hi < N, (p["label"], inp)
            continue
        for inp in (True, False):
            off = p["in_off"] if inp else p["out_off"]
            addr = addresses(a, pass_points(p), inp).reshape(-1) + off
            assert addr.min() >= 0 and addr.max() < N, (p["label"], inp)
            assert np.unique(addr).size == addr.size, (p["label"], inp)


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("schedule", SCHEDULES)
def test_pass_list_computes_the_dft(shape, schedule):
    g = np.random.default_rng(sum(shape))
    x = g.standard_normal(shape) + 1j * g.standard_normal(shape)
    d = dft3d.describe(shape, schedule)
    for sign in (-1, 1):
        got = run_model(x, d, sign)
        ref = oracle.dft3d(x, sign, "fft")
        assert oracle.rel_l2(got, ref) < 1e-13, (shape, schedule, sign)


OPTION_SETS = [dict(slab_group=1), dict(slab_group=2), dict(fused_plane=0), dict(tile=8), dict(tile=64),
               dict(split_max=4), dict(persistent=0), dict(nontemporal=1),
               dict(xcd_remap=0), dict(precision="bf16x6"), dict(precision="fp16x3"),
               dict(pencil_group=1), dict(pencil_group=2), dict(pencil_group=4),
               dict(pencil_group=3), dict(pencil_group=2, tile=8)]


@pytest.mark.parametrize("opts", OPTION_SETS)
@pytest.mark.parametrize("schedule", SCHEDULES)
def test_pass_list_with_options(opts, schedule):
    shape = (8, 16, 32)
    g = np.random.default_rng(7)
    x = g.standard_normal(shape) + 1j * g.standard_normal(shape)
    d = dft3d.describe(shape, schedule, **opts)
    for sign in (-1, 1):
        got = run_model(x, d, sign)
        assert oracle.rel_l2(got, oracle.dft3d(x, sign, "fft")) < 1e-13, (opts, sign)


SHUFFLED_SHAPES = [(1, 1, 1), (2, 4, 8), (8, 2, 4), (16, 16, 16), (32, 4, 64), (4, 64, 2),
                   (2, 256, 8), (64, 1, 32), (4096, 2, 1), (1, 2, 2048), (8, 16, 32)]


@pytest.mark.parametrize("shape", SHUFFLED_SHAPES + [(2, 256, 256), (256, 256, 32)])
@pytest.mark.parametrize("schedule", ["volumetric", "auto"])
def test_shuffled_pass_lists(shape, schedule):
    """Forward list: natural input to the documented shuffled order; inverse
    list: shuffled input to natural output (both within FP64 rounding)."""
    g = np.random.default_rng(sum(shape) + 1)
    x = g.standard_normal(shape) + 1j * g.standard_normal(shape)
    d = dft3d.describe(shape, schedule, "shuffled")
    assert d["schedule"] == "volumetric" and d["layout"] == "shuffled"
    f = dft3d.shuffle_factors(shape)
    fwd = run_model(x, d, -1)
    assert oracle.rel_l2(fwd, oracle.to_shuffled(oracle.dft3d(x, -1, "fft"), f)) < 1e-13
    s = oracle.to_shuffled(x, f)                 # any data in shuffled order
    inv = run_model(s, d, +1)
    assert oracle.rel_l2(inv, oracle.dft3d(x, +1, "fft")) < 1e-13
    # round trip through both lists
    back = run_model(fwd, d, +1)
    assert oracle.rel_l2(back, x.size * x) < 1e-13


@pytest.mark.parametrize("shape", SHUFFLED_SHAPES + [(1024, 1024, 1024), (4096, 4096, 4)])
def test_shuffled_pass_maps_in_bounds(shape):
    d = dft3d.describe(shape, "volumetric", "shuffled")
    N = shape[0] * shape[1] * shape[2]
    for key in ("passes", "inverse_passes"):
        for p in d[key]:
            a = p["args"]
            if a["B"] * p["n"] > (1 << 22):
                B = a["B"]
                for lo in (0, B // 2, B - 64):
                    b = np.arange(lo, lo + 64, dtype=np.int64)
                    for inp in (True, False):
                        st = a["is"] if inp else a["os"]
                        js = a["ijs"] if inp else a["oks"]
                        base = ((b >> a["s1"]) * st[2] + ((b >> a["s0"]) & a["m1"]) * st[1]
                                + (b & a["m0"]) * st[0])
                        assert base.min() >= 0 and base.max() + (p["n"] - 1) * js < N
                continue
            for inp in (True, False):
                addr = addresses(a, p["n"], inp).reshape(-1)
                assert addr.min() >= 0 and addr.max() < N, (key, p["label"], inp)
                assert np.unique(addr).size == addr.size, (key, p["label"], inp)


@pytest.mark.parametrize("shape,nfused", [
    ((2, 256, 256), 1), ((256, 256, 32), 1), ((2, 1024, 512), 1), ((1024, 512, 16), 1),
    ((64, 256, 256), 1), ((16, 256, 16), 0), ((4, 1024, 1024), 1),
    ((256, 256, 256), 2), ((1024, 1024, 1024), 2)])
def test_shuffled_inverse_fused(shape, nfused):
    """The inverse from the shuffled order fuses W2 of an axis with W1 of the
    next inner axis wherever the forward fuses the pair: as many passes as
    the forward, each fused pair one pass in place (the forward's transposed
    tiles); the list still maps shuffled input to the natural inverse DFT."""
    d = dft3d.describe(shape, "volumetric", "shuffled")
    fwd = [p["fused_axes"] for p in d["passes"]]
    inv = [p["fused_axes"] for p in d["inverse_passes"]]
    assert fwd.count(2) == nfused and inv.count(3) == nfused, (fwd, inv)
    assert len(d["inverse_passes"]) == len(d["passes"])
    for p in d["inverse_passes"]:
        if p["fused_axes"]:
            assert p["args"]["is"] == p["args"]["os"], p["label"]
    off = dft3d.describe(shape, "volumetric", "shuffled", fused_axes=0)
    assert not any(p["fused_axes"] for p in off["inverse_passes"])
    assert len(off["inverse_passes"]) == len(d["inverse_passes"]) + nfused
    if shape[0] * shape[1] * shape[2] <= (1 << 22):
        g = np.random.default_rng(sum(shape) + 7)
        x = g.standard_normal(shape) + 1j * g.standard_normal(shape)
        s = oracle.to_shuffled(x, dft3d.shuffle_factors(shape))
        assert oracle.rel_l2(run_model(s, d, +1), oracle.dft3d(x, +1, "fft")) < 1e-13


@pytest.mark.parametrize("schedule", ["pencil", "slab"])
def test_shuffled_rejected_by_other_schedules(schedule):
    with pytest.raises(dft3d.Dft3dError):
        dft3d.describe((8, 8, 8), schedule, "shuffled")


@pytest.mark.parametrize("shape", [(4, 16, 16), (2, 128, 128), (8, 32, 64), (16, 128, 16),
                                   (1, 64, 128), (32, 16, 8), (8, 256, 16)])
def test_slab_fused_plane_pass(shape):
    """Planes of 16..128 x 16..128 points go through one fused 2D pass;
    other planes keep the row and column passes."""
    d = dft3d.describe(shape, "slab")
    fused = 16 <= shape[1] <= 128 and 16 <= shape[2] <= 128
    planes = [p for p in d["passes"] if p["plane_rows"]]
    assert len(planes) == (1 if fused else 0)
    assert len(d["passes"]) == (2 if fused else 3)
    g = np.random.default_rng(5)
    x = g.standard_normal(shape) + 1j * g.standard_normal(shape)
    for sign in (-1, 1):
        assert oracle.rel_l2(run_model(x, d, sign), oracle.dft3d(x, sign, "fft")) < 1e-13
    off = dft3d.describe(shape, "slab", fused_plane=0)
    assert not any(p["plane_rows"] for p in off["passes"])


@pytest.mark.parametrize("shape,nfused", [
    ((2, 256, 256), 1),      # a = 16, V2 runs contiguous
    ((256, 256, 32), 1),     # a = 16, V2 runs strided
    ((2, 1024, 512), 1),     # a = 32, contiguous
    ((1024, 512, 16), 1),    # a = 32, strided
    ((256, 256, 256), 2),    # both pairs
    ((16, 256, 16), 0), ((256, 16, 256), 0), ((4, 1024, 1024), 1)])
def test_volumetric_fused_axes(shape, nfused):
    """Where the split factors match, V2 of an axis and V1 of the next run as
    one fused pass; the pass list still computes the DFT, and turning the
    option off restores the six separate halves."""
    d = dft3d.describe(shape, "volumetric")
    fused = [p for p in d["passes"] if p["fused_axes"]]
    assert len(fused) == nfused
    off = dft3d.describe(shape, "volumetric", fused_axes=0)
    assert not any(p["fused_axes"] for p in off["passes"])
    assert len(d["passes"]) == len(off["passes"]) - len(fused)
    if shape[0] * shape[1] * shape[2] <= (1 << 23):
        g = np.random.default_rng(9)
        x = g.standard_normal(shape) + 1j * g.standard_normal(shape)
        for sign in (-1, 1):
            ref = oracle.dft3d(x, sign, "fft")
            assert oracle.rel_l2(run_model(x, d, sign), ref) < 1e-13


def test_volumetric_1024_cubed_has_four_passes():
    d = dft3d.describe((1024, 1024, 1024), "volumetric")
    assert len(d["passes"]) == 4
    assert [p["fused_axes"] for p in d["passes"]] == [0, 1, 1, 0]


OTHER_SHAPES = [(3, 5, 7), (6, 10, 12), (1, 1, 3), (9, 1, 1), (2, 3, 4), (100, 30, 17),
                (64, 100, 64), (15, 8, 2048), (12, 7, 16), (19, 23, 4), (1009, 2, 3),
                (11, 13, 26), (2039, 3, 1), (4095, 2, 1), (4093, 2, 1), (2, 2062, 1)]


def is_smooth13(n):
    for f in (2, 3, 5, 7, 11, 13):
        while n % f == 0:
            n //= f
    return n == 1


@pytest.mark.parametrize("shape", OTHER_SHAPES)
def test_bluestein_pass_lists(shape):
    """Lengths that are not powers of two (pencil schedule, Bluestein steps):
    the pass list computes the DFT, forward and inverse."""
    d = dft3d.describe(shape, "auto")
    assert d["schedule"] == "pencil"
    assert any(p["bluestein"] or p["mixed"] or p["rader"] for p in d["passes"])
    g = np.random.default_rng(sum(shape))
    x = g.standard_normal(shape) + 1j * g.standard_normal(shape)
    for sign in (-1, 1):
        got = run_model(x, d, sign)
        ref = oracle.dft3d(x, sign, "direct")
        assert oracle.rel_l2(got, ref) < 1e-12, (shape, sign)


@pytest.mark.parametrize("shape", OTHER_SHAPES + [(2048, 1000, 3), (4096, 3, 5),
                                                  (1000, 1000, 1000)])
def test_bluestein_axis_passes(shape):
    """One pass per axis whose length is not a power of two (mixed radix
    when its prime factors are at most 13, else Bluestein with its
    convolution length), reading and writing N points of the chain's
    buffers (no region beyond N in the workspace)."""
    d = dft3d.describe(shape, "auto")
    N = shape[0] * shape[1] * shape[2]
    assert d["workspace_bytes"] <= 8 * N
    assert len(d["passes"]) == 3
    for p in d["passes"]:
        n = pass_points(p)
        assert p["args"]["B"] * n == N
        if n & (n - 1):
            assert bool(p["mixed"]) == is_smooth13(n)
            assert bool(p["rader"]) == is_rader(n)
            assert bool(p["bluestein"]) == (not is_smooth13(n) and not is_rader(n))
        if p["mixed"]:
            assert int(np.prod(p["radices"])) == n and p["n"] >= n
            # composite radices only in the kernel without 11 and 13, below 2048
            if {10, 16} & set(p["radices"]):
                assert n < 2048 and not {11, 13} & set(p["radices"]), n
            assert set(p["radices"]) <= {2, 3, 4, 5, 7, 8, 10, 11, 13, 16}
        if p["bluestein"]:
            m = p["n"]
            assert m & (m - 1) == 0 and 2 * n - 1 <= m < 4 * n - 2
            assert p["args"]["res_mask"] == n


@pytest.mark.parametrize("shape", OTHER_SHAPES + [(1000, 1000, 1000), (2047, 2047, 64)])
def test_bluestein_pass_maps_injective_and_in_bounds(shape):
    check_pass_maps(dft3d.describe(shape, "pencil"), shape[0] * shape[1] * shape[2])


@pytest.mark.parametrize("schedule,opts", [("pencil", {"precision": "bf16x6"}),
                                           ("slab", {"precision": "fp16x3"}),
                                           ("volumetric", {"move_only": 1})])
def test_bluestein_limits(schedule, opts):
    with pytest.raises(dft3d.Dft3dError):
        dft3d.describe((3, 4, 4), schedule, **opts)
    with pytest.raises(dft3d.Dft3dError):
        dft3d.describe((4097, 4, 4), "pencil")
    with pytest.raises(dft3d.Dft3dError):
        dft3d.describe((3, 4, 4), "auto", "shuffled")


@pytest.mark.parametrize("shape", OTHER_SHAPES + [(20, 3, 64), (64, 64, 1000), (17, 4, 19),
                                                  (1000, 64, 64), (64, 1000, 64)])
@pytest.mark.parametrize("schedule", ["slab", "volumetric"])
def test_other_lengths_on_slab_and_volumetric(shape, schedule):
    """The slab and volumetric schedules over lengths that are not powers of
    two: such axes run as one pass in layout (mixed radix or Bluestein);
    pencil counts that are not powers of two before the last field use the
    general index form (s0 = -1), which only those kernels read (a
    power-of-two axis whose pencils need it runs through the mixed-radix
    pass).  Every pass map is a bijection inside the buffers, and the pass
    list computes the DFT forward and inverse (direct sums as reference)."""
    d = dft3d.describe(shape, schedule)
    assert d["schedule"] == schedule
    N = shape[0] * shape[1] * shape[2]
    for p in d["passes"]:
        if p["args"]["s0"] < 0:
            assert p["mixed"] or p["bluestein"] or p["rader"], p["label"]
    if schedule == "volumetric":
        # axes that are powers of two with power-of-two axes after them are
        # still split four-step style
        for axis in range(3):
            inner = int(np.prod(shape[axis + 1:]))
            n = shape[axis]
            split = n >= 4 and n & (n - 1) == 0 and inner & (inner - 1) == 0
            labels = [p["label"] for p in d["passes"] if p["label"].startswith(f"vol{axis}")]
            assert any(".V1" in l for l in labels) == split, (axis, labels)
    check_pass_maps(d, N)
    if N <= 1 << 16:
        g = np.random.default_rng(sum(shape) + 5)
        x = g.standard_normal(shape) + 1j * g.standard_normal(shape)
        for sign in (-1, 1):
            got = run_model(x, d, sign)
            ref = oracle.dft3d(x, sign, "direct")
            assert oracle.rel_l2(got, ref) < 1e-12, (shape, schedule, sign)


def is_prime(n):
    return n >= 2 and all(n % f for f in range(2, int(n ** 0.5) + 1))


RADER_COMPILED = {197, 257, 281, 401, 577, 641, 769, 1009, 1201, 1601, 2017, 2593, 3001,
                  4001}


def is_rader(n, any_kernel=False):
    """A prime above 13 (smaller ones run mixed radix) with n - 1 free of
    prime factors above 13, within the Rader kernels' tile lengths (n + 1 <=
    4096); by default only the primes a Rader kernel is compiled for."""
    ok = is_prime(n) and n > 13 and is_smooth13(n - 1) and n + 1 <= 4096
    return ok and (any_kernel or n in RADER_COMPILED)


@pytest.mark.parametrize("tile", [1, 2, 4, 8, 16, 32, 64, 128, 256, 512, 1024, 2048, 4096])
def test_tile_option_keeps_pass_kinds(tile):
    """A tile option only picks among kernels of the pass's own kind: on
    power-of-two shapes no pass becomes a mixed-radix, Rader or Bluestein
    pass (a Rader kernel of 256 pencils of up to 32 points once matched a
    length-32 power-of-two pass by its tile alone), and on other shapes
    those passes carry their lengths."""
    for shape in [(64, 128, 32), (32, 32, 32), (4096, 2, 2), (2, 1024, 8), (16, 256, 512)]:
        for sched in ("pencil", "slab", "volumetric"):
            for p in dft3d.describe(shape, sched, tile=tile)["passes"]:
                assert not (p["mixed"] or p["rader"] or p["bluestein"]), (shape, sched, tile, p["label"])
    for shape in [(1009, 2, 3), (17, 19, 23), (1000, 4, 8)]:
        for p in dft3d.describe(shape, "pencil", tile=tile)["passes"]:
            if p["rader"]:
                assert p["rader_n"] >= 3
            if p["mixed"]:
                assert p["args"]["res_mask"] >= 2
            if p["bluestein"]:
                assert p["bl_n"] >= 1


def test_rader_option_levels():
    """DFT3D_OPT_RADER: 1 (default) Rader for the compiled primes only, 2 for
    every eligible prime, 0 Bluestein; other values rejected."""
    for n in range(14, 4097):
        if not is_prime(n):
            continue
        p1 = dft3d.describe((1, 1, n), "pencil")["passes"][0]
        p2 = dft3d.describe((1, 1, n), "pencil", rader=2)["passes"][0]
        p0 = dft3d.describe((1, 1, n), "pencil", rader=0)["passes"][0]
        assert bool(p1["rader"]) == is_rader(n), n
        assert bool(p2["rader"]) == is_rader(n, True), n
        assert not p0["rader"] and p0["bluestein"], n
        if p1["rader"]:
            assert p1["fixed_n"] == n and p1["radices"] == p2["radices"]
    for bad in (-1, 3):
        with pytest.raises(dft3d.Dft3dError):
            dft3d.describe((1, 1, 17), "pencil", rader=bad)


HALVES = {(2048, "row", "col"): 16, (2048, "col", "col"): 16, (1024, "col", "col"): 32}


def test_halves_option():
    """DFT3D_OPT_HALVES: the pencil schedule's rotate-on-write passes of
    length 2048 and the slab schedule's strided passes of lengths 1024 and
    2048 run as two halves in tiles of twice the pencils, persistent under
    the rule of the other passes except the strided 2048 pass (one form);
    with 0, or a tile option the
    halves kernel does not have, the whole-length kernels run.  Other
    lengths, orders, split precision and other values are untouched or
    rejected."""
    for shape in ((2048, 1024, 512), (1024, 1024, 1024), (2048, 3, 5), (4, 2048, 2),
                  (2, 2, 2048), (1024, 4, 2)):
        for sch in ("pencil", "slab", "volumetric"):
            for kw in ({}, {"persistent": 0}, {"nontemporal": 1}, {"nontemporal": 0},
                       {"fused_plane": 0}):
                d = dft3d.describe(shape, sch, **kw)
                for p in d["passes"]:
                    key = (p["n"], p["load"], p["store"])
                    want = key in HALVES and not p["post_twiddle"] and not p["mixed"] and \
                        not p["plane_rows"] and not p["fused_axes"]
                    assert p["halves"] == want, (shape, sch, kw, p)
                    if p["halves"]:
                        big = shape[0] * shape[1] * shape[2] * 8 >= 256 << 20
                        pers = kw.get("persistent", 1) and ("nontemporal" in kw or big) and \
                            key != (2048, "col", "col")
                        assert p["tile"] == HALVES[key] and p["persistent"] == pers
                        assert p["threads"] == p["tile"] * p["n"] // 64
                        assert p["radices"][0] == 2 and int(np.prod(p["radices"])) == p["n"]
                        if "nontemporal" in kw:
                            assert p["nontemporal"] == kw["nontemporal"]
            for kw in ({"halves": 0}, {"tile": 8}, {"precision": "bf16x6"}):
                if "precision" in kw and 3 in shape:
                    continue  # split precision is for powers of two
                d = dft3d.describe(shape, sch, **kw)
                assert not any(p["halves"] for p in d["passes"]), (shape, sch, kw)
    # automatic streaming and persistence on a streamed array
    d = dft3d.describe((2048, 1024, 512), "slab")
    assert [(p["n"], p["nontemporal"], p["persistent"]) for p in d["passes"] if p["halves"]] \
        == [(1024, 1, 1), (2048, 1, 0)]
    d = dft3d.describe((2048, 1024, 512), "pencil")
    assert [(p["n"], p["nontemporal"], p["persistent"]) for p in d["passes"] if p["halves"]] \
        == [(2048, 1, 1)]
    d = dft3d.describe((2048, 4, 8), "pencil")
    assert [(p["n"], p["nontemporal"], p["persistent"]) for p in d["passes"] if p["halves"]] \
        == [(2048, 0, 0)]
    for bad in (-1, 2):
        with pytest.raises(dft3d.Dft3dError):
            dft3d.describe((2048, 2, 2), "pencil", halves=bad)


def test_every_length_up_to_4096():
    """Each length 1..4096 is planned as a power-of-two pass, a mixed-radix
    pass (prime factors <= 13), a Rader pass (primes with n - 1 of prime
    factors <= 13) or a Bluestein pass (other lengths, with a convolution
    length up to 8192); 4097 is rejected."""
    with pytest.raises(dft3d.Dft3dError):
        dft3d.describe((4097, 1, 1), "pencil")
    for n in range(1, 4097):
        pow2 = n & (n - 1) == 0
        p = dft3d.describe((1, 1, n), "pencil")["passes"][0]
        if p["bluestein"]:
            assert p["n"] <= 8192 and p["n"] >= 2 * n - 1, n
        if n == 1:
            continue
        assert bool(p["mixed"]) == (not pow2 and is_smooth13(n)), n
        assert bool(p["rader"]) == (not pow2 and is_rader(n)), n
        assert bool(p["bluestein"]) == (not pow2 and not is_smooth13(n) and not is_rader(n)), n
        if p["rader"]:
            assert int(np.prod(p["radices"])) == n - 1 and p["n"] >= n + 1, n
        if p["mixed"]:
            assert int(np.prod(p["radices"])) == n and p["n"] >= n
            # composite radices only in the kernel without 11 and 13, below 2048
            if {10, 16} & set(p["radices"]):
                assert n < 2048 and not {11, 13} & set(p["radices"]), n


def stockham_mixed(x, radices):
    """The mixed-radix pass's stage formulas (index by index, as documented
    with the kernel) on one pencil, in FP64."""
    n = x.size
    buf = x.astype(complex).copy()
    ns = 1
    for R in radices:
        nr = n // R
        out = np.empty_like(buf)
        t = np.arange(nr)
        g, tm = t // ns, t % ns
        a = np.stack([buf[t + r * nr] for r in range(R)])              # (R, nr)
        w = np.exp(-2j * np.pi * ((tm[None, :] * np.arange(R)[:, None]) % (ns * R))
                   / (ns * R))
        a = np.fft.fft(a * w, axis=0)                                   # DFT_R
        for r in range(R):
            out[g * ns * R + tm + r * ns] = a[r]
        buf = out
        ns *= R
    return buf


@pytest.mark.parametrize("n", [3, 5, 6, 7, 9, 11, 12, 13, 15, 24, 45, 96, 100, 120, 143,
                               169, 243, 384, 768, 1000, 1001, 1144, 1250, 1920, 2000,
                               2310, 3000, 3072, 4095])
def test_mixed_stage_formulas(n):
    """The stage indexing and twiddles of the mixed-radix pass, with the
    radices the planner encodes, give the DFT of the pencil."""
    p = dft3d.describe((1, 1, n), "pencil")["passes"][0]
    assert p["mixed"]
    x = np.random.default_rng(n).standard_normal(n) + 1j * np.random.default_rng(n + 1).standard_normal(n)
    got = stockham_mixed(x, p["radices"])
    assert oracle.rel_l2(got, oracle.dft3d(x.reshape(n, 1, 1), -1, "direct").reshape(-1)) < 1e-12


def rader_steps(x):
    """Rader's identity written out step by step in numpy (the library's
    tables are not used): generator g by trial, a[j] = x[g^j], b[m] =
    w_n^(g^-m), cyclic convolution c = IFFT(FFT(a) FFT(b)), y[0] = sum x,
    y[g^-p] = x[0] + c[p]."""
    n = x.size
    L = n - 1
    g = next(c for c in range(2, n) if len({pow(c, j, n) for j in range(L)}) == L)
    pw = [pow(g, j, n) for j in range(L)]
    a = x[pw]
    b = np.exp(-2j * np.pi * np.array([pw[(-m) % L] for m in range(L)]) / n)
    c = np.fft.ifft(np.fft.fft(a) * np.fft.fft(b))
    y = np.empty(n, complex)
    y[0] = x.sum()
    for p_ in range(L):
        y[pw[(-p_) % L]] = x[0] + c[p_]
    return y


@pytest.mark.parametrize("n", [3, 5, 7, 17, 19, 23, 29, 31, 37, 41, 43, 53, 61, 97, 1009, 2003])
def test_rader_identity(n):
    """The steps of the Rader pass give the DFT (direct sums), and the
    permutation of the output is that of the input (y[g^j] = x[0] +
    FFT_L(FFT_L(a) B / L)[j], as the kernel stores it)."""
    g_ = np.random.default_rng(n)
    x = g_.standard_normal(n) + 1j * g_.standard_normal(n)
    ref = oracle.dft3d(x.reshape(n, 1, 1), -1, "direct").reshape(-1)
    assert oracle.rel_l2(rader_steps(x), ref) < 1e-12
    L = n - 1
    g = next(c for c in range(2, n) if len({pow(c, j, n) for j in range(L)}) == L)
    pw = np.array([pow(g, j, n) for j in range(L)])
    B = np.fft.fft(np.exp(-2j * np.pi * pw[(-np.arange(L)) % L] / n)) / L
    A = np.fft.fft(x[pw])
    D = np.fft.fft(A * B)
    y = np.empty(n, complex)
    y[pw] = x[0] + D
    y[0] = x[0] + A[0]
    assert oracle.rel_l2(y, ref) < 1e-12


RADIX_CASES = [((4, 2, 1000), [10, 10, 10]), ((4, 2, 1000), [8, 5, 5, 5]),
               ((2, 4, 1024), [4, 4, 4, 4, 4]), ((2, 4, 64), [4, 16]), ((8, 3, 96), [2, 3, 16]),
               ((6, 4, 143), [13, 11]), ((2, 2, 2048), [8, 8, 8, 4]), ((2, 8, 8), [2, 4])]


@pytest.mark.parametrize("shape,radices", RADIX_CASES)
def test_radices_option(shape, radices):
    """DFT3D_OPT_RADICES: the passes of the code's length run the mixed-radix
    kernel with those stages (powers of two too), other lengths keep their
    default; the stage formulas with that code give the DFT, and the pass
    list computes the 3D DFT."""
    n = int(np.prod(radices))
    d = dft3d.describe(shape, "pencil", radices=radices)
    hits = [p for p in d["passes"] if pass_points(p) == n]
    assert hits and all(p["mixed"] and p["radices"] == radices for p in hits)
    x1 = np.random.default_rng(n).standard_normal(n) + 1j * np.random.default_rng(n + 7).standard_normal(n)
    got = stockham_mixed(x1, radices)
    assert oracle.rel_l2(got, oracle.dft3d(x1.reshape(n, 1, 1), -1, "direct").reshape(-1)) < 1e-12
    check_pass_maps(d, int(np.prod(shape)))
    g = np.random.default_rng(3)
    x = g.standard_normal(shape) + 1j * g.standard_normal(shape)
    method = "fft" if all(m & (m - 1) == 0 for m in shape) else "direct"
    for sign in (-1, 1):
        assert oracle.rel_l2(run_model(x, d, sign), oracle.dft3d(x, sign, method)) < 1e-12


@pytest.mark.parametrize("radices", [[6, 5], [4, 0, 4], [16, 16, 16], [2] * 9, [1, 4], [17],
                                     [16, 16, 8], [11, 10], [13, 16]])
def test_radices_option_rejects(radices):
    """Radices outside the kernel's set, a zero stage inside the code, a
    product above 2048, more than 8 stages and composites the kernels do not
    run at that length (16 at 2048, 10 or 16 beside 11 or 13) are
    rejected."""
    with pytest.raises((dft3d.Dft3dError, ValueError)):
        dft3d.describe((4, 4, 64), "pencil", radices=radices)


try:
    from hypothesis import given, settings, strategies as st
except ImportError:  # pragma: no cover
    given = None

if given is not None:
    LENGTHS = st.integers(min_value=1, max_value=40)

    @settings(max_examples=40, deadline=None)
    @given(st.tuples(LENGTHS, LENGTHS, LENGTHS), st.integers(0, 2**31 - 1),
           st.sampled_from([-1, 1]))
    def test_any_small_shape_pass_list(shape, seed, sign):
        """Random shapes with lengths 1..40 (powers of two, mixed radix and
        Bluestein axes mixed): the auto plan's pass list, run by the model,
        gives the oracle's direct DFT, and its maps stay in bounds."""
        d = dft3d.describe(shape, "auto")
        N = shape[0] * shape[1] * shape[2]
        check_pass_maps(d, N)
        g = np.random.default_rng(seed)
        x = g.standard_normal(shape) + 1j * g.standard_normal(shape)
        got = run_model(x, d, sign)
        assert oracle.rel_l2(got, oracle.dft3d(x, sign, "direct")) < 1e-12


@pytest.mark.parametrize("tile", [0, 2, 4, 8, 16, 32, 64, 256])
def test_mixed_kernel_runs_its_radices(tile):
    """Whatever the tile option, the mixed-radix kernel a plan picks runs
    every stage radix of its length: composites (10, 16) only in the
    variant without 11 and 13 with a tile length of at most 2048; 11 and 13
    only in the other variant."""
    for n in list(range(3, 300)) + [500, 768, 1000, 1001, 1536, 2000, 2187, 3000, 4095]:
        if n & (n - 1) == 0 or not is_smooth13(n):
            continue
        kw = {"tile": tile} if tile else {}
        p = dft3d.describe((1, 1, n), "pencil", **kw)["passes"][0]
        assert p["mixed"], n
        r = set(p["radices"])
        if r & {10, 16}:
            assert p["mixed"] == 1 and p["n"] <= 2048, (n, tile, p["n"])
        if r & {11, 13}:
            assert p["mixed"] == 2, (n, tile)
        assert p["n"] > n


FIXED_LENGTHS = [48, 60, 72, 80, 96, 100, 120, 125, 144, 160, 192, 200, 240, 250, 300, 320,
                 384, 400, 480, 500, 600, 640, 768, 800, 960, 1000, 1200, 1536, 2000,
                 2400, 2500, 3000, 3072, 3200, 3600, 4000,
                 56, 112, 168, 224, 336, 448, 672, 896, 1008, 1344, 1792, 2016]


@pytest.mark.parametrize("n", FIXED_LENGTHS)
def test_fixed_length_kernels_are_picked(n):
    """Each length with a kernel compiled for it gets that kernel (its radix
    code matches the planner's packing), on every axis; the tile option
    falls back to the generic kernels."""
    d = dft3d.describe((n, n, n) if n <= 128 else (n, 4, 2), "pencil")
    picked = [p for p in d["passes"] if p.get("bl_n", 0) == 0 and p["mixed"]
              and pass_points(p) == n]
    assert picked and all(p["fixed_n"] == n for p in picked)
    p = dft3d.describe((1, 1, n), "pencil", tile=16)["passes"][0]
    assert p["fixed_n"] == 0


@pytest.mark.parametrize("shape,groups", [((1024, 1024, 1024), 32), ((64, 1024, 1024), 2),
                                          ((2048, 512, 512), 0), ((512, 512, 512), 0),
                                          ((128, 1024, 1024), 4), ((4096, 256, 256), 0)])
def test_grouped_pencil_plan(shape, groups):
    """Automatic group size for the pencil schedule's first two passes:
    groups of planes of at most 256 MB where both one-sided streaming
    kernels exist, the group's intermediate in OUT, the rotated second pass
    into WS at the group's columns, one pass along axis 0; every pass in
    bounds (sampled at full size).  Off unless asked for."""
    assert not any(" group " in p["label"] for p in dft3d.describe(shape, "auto")["passes"])
    d = dft3d.describe(shape, "auto", pencil_group=-1)
    ps = d["passes"]
    if not groups:
        assert not any("group" in p["label"] for p in ps)
        return
    n0, n1, n2 = shape
    G = n0 // groups
    assert len(ps) == 2 * groups + 1 and G * n1 * n2 * 8 <= (256 << 20)
    for g in range(groups):
        a, b = ps[2 * g], ps[2 * g + 1]
        assert (a["src"], a["dst"], a["nontemporal"]) == ("in", "out", 2)
        assert (b["src"], b["dst"], b["nontemporal"]) == ("out", "ws", 3)
        assert a["in_off"] == a["out_off"] == b["in_off"] == g * G * n1 * n2
        assert b["out_off"] == g * G
    assert (ps[-1]["src"], ps[-1]["dst"], ps[-1]["n"]) == ("ws", "out", n0)
    check_pass_maps(d, n0 * n1 * n2)


@pytest.mark.parametrize("shape", [(8, 16, 32), (4, 4, 4), (16, 2, 8), (2, 64, 1), (32, 8, 128)])
@pytest.mark.parametrize("group", [1, 2, 8])
def test_grouped_pencil_computes_the_dft(shape, group):
    g = np.random.default_rng(sum(shape) + group)
    x = g.standard_normal(shape) + 1j * g.standard_normal(shape)
    d = dft3d.describe(shape, "pencil", pencil_group=group)
    if group < shape[0]:
        assert any("group" in p["label"] for p in d["passes"])
    check_pass_maps(d, x.size)
    for sign in (-1, 1):
        assert oracle.rel_l2(run_model(x, d, sign), oracle.dft3d(x, sign, "fft")) < 1e-13


# ---------------------------------------------------------------------------
# Move-only plans (DFT3D_OPT_MOVE_ONLY): the passes' data movement alone.

def stockham_identity_perm(n, radices):
    """The Stockham stage maps of the pass kernels (input t + r n/R of the
    radix-R stage after ns goes to (t div ns) ns R + (t mod ns) + r ns) with
    every butterfly and twiddle removed: out[k] = in[perm[k]]."""
    src = np.arange(n)
    ns = 1
    for R in radices:
        nr = n // R
        out = np.empty_like(src)
        t = np.arange(nr)
        for r in range(R):
            out[(t // ns) * ns * R + (t % ns) + r * ns] = src[t + r * nr]
        src = out
        ns *= R
    assert ns == n
    return src


def halves_identity_perm(n, radices):
    """The two-halves pass of length n (radix 2, then the Stockham stages of
    radices[1:] on each half) with every butterfly and twiddle removed: half
    h of the input goes through the half-length maps to the outputs 2k + h."""
    assert radices[0] == 2
    half = stockham_identity_perm(n // 2, radices[1:])
    perm = np.empty(n, dtype=np.int64)
    for h in range(2):
        perm[h::2] = h * (n // 2) + half
    return perm


def halves_dft(x, radices):
    """The two-halves pass of length n with its arithmetic: the radix-2 split
    a = x[:n/2] + x[n/2:], b = (x[:n/2] - x[n/2:]) w_n^j, then the Stockham
    stages of radices[1:] on a (the even outputs) and on b (the odd ones)."""
    n = x.size
    assert radices[0] == 2
    lo, hi = x[:n // 2], x[n // 2:]
    w = np.exp(-2j * np.pi * np.arange(n // 2) / n)
    y = np.empty(n, dtype=complex)
    y[0::2] = stockham_mixed(lo + hi, radices[1:])
    y[1::2] = stockham_mixed((lo - hi) * w, radices[1:])
    return y


def run_move_model(x, d, sign=-1):
    """Run a move-only (1) or copy (2) pass list on x, as the kernels move
    data: per pencil the identity-butterfly permutation, or a flat copy."""
    n_total = x.size
    n_ws = max(n_total, d["workspace_bytes"] // 8)
    bufs = {"in": x.reshape(-1).copy(),
            "out": np.full(n_total, np.nan, x.dtype),
            "ws": np.full(n_ws, np.nan, x.dtype)}
    passes = d["passes"]
    for i, p in enumerate(passes):
        a = p["args"]
        if p["move_only"] == 2:
            m = a["B"] * p["n"]
            bufs[p["dst"]][p["out_off"]:p["out_off"] + m] = \
                bufs[p["src"]][p["in_off"]:p["in_off"] + m]
            continue
        assert p["move_only"] == 1
        ia = addresses(a, p["n"], True)
        oa = addresses(a, p["n"], False)
        v = bufs[p["src"]][ia + p["in_off"]]
        if sign == 1 and p["src"] == "in":
            v = np.conj(v)
        if p["halves"]:
            y = v[:, halves_identity_perm(p["n"], p["radices"])]
        else:
            y = v[:, stockham_identity_perm(p["n"], p["radices"])]
        if sign == 1 and i == len(passes) - 1:
            y = np.conj(y)
        bufs[p["dst"]][oa + p["out_off"]] = y
    return bufs["out"].reshape(x.shape)


def test_power_of_two_stage_radices_compute_the_dft():
    """The radix lists the FP32 pass kernels report, run through the same
    Stockham stage formulas with their butterflies and twiddles, give the
    DFT: the stage maps the move-only model uses are the kernels' own."""
    seen = set()
    for lg in range(1, 13):
        n = 1 << lg
        for shape in ((1, 1, n), (1, n, 2), (n, 2, 2)):
            for sch in ("pencil", "slab"):
                for p in dft3d.describe(shape, sch, fused_plane=0)["passes"]:
                    key = (p["n"], tuple(p["radices"]), p["halves"])
                    if p["n"] < 2 or key in seen:
                        continue
                    seen.add(key)
                    assert int(np.prod(p["radices"])) == p["n"], p
                    x = np.random.default_rng(p["n"]).standard_normal(p["n"]) * (1 + 1j)
                    if p["halves"]:
                        got = halves_dft(x, p["radices"])
                    else:
                        got = stockham_mixed(x, p["radices"])
                    assert oracle.rel_l2(got, np.fft.fft(x)) < 1e-12, key
    assert len(seen) >= 12


@pytest.mark.parametrize("shape", [(2, 4, 8), (16, 16, 16), (32, 4, 64), (4, 64, 2),
                                   (64, 32, 16), (2048, 2, 4), (1, 1, 1)])
@pytest.mark.parametrize("schedule", SCHEDULES)
@pytest.mark.parametrize("mode", [1, 2])
def test_move_only_plans(shape, schedule, mode):
    """Move-only plans: every pass has a move-only kernel, the maps stay in
    bounds, the output is a permutation of the input (mode 1) or the input
    itself (mode 2), forward and inverse alike."""
    d = dft3d.describe(shape, schedule, move_only=mode)
    assert all(p["move_only"] == mode for p in d["passes"])
    assert not any(p["plane_rows"] or p["fused_axes"] for p in d["passes"])
    N = shape[0] * shape[1] * shape[2]
    check_pass_maps(d, N)
    g = np.random.default_rng(N)
    x = (g.standard_normal(shape) + 1j * g.standard_normal(shape)).astype(np.complex64)
    for sign in (-1, 1):
        y = run_move_model(x, d, sign)
        if mode == 2:
            assert np.array_equal(y, x)
        else:
            assert np.array_equal(np.sort_complex(y.reshape(-1)), np.sort_complex(x.reshape(-1)))
    # the same passes as the full plan, in the same buffers
    full = dft3d.describe(shape, schedule, fused_plane=0, fused_axes=0)["passes"]
    assert [(p["src"], p["dst"], p["n"], p["args"]) for p in d["passes"]] == \
        [(p["src"], p["dst"], p["n"], p["args"]) for p in full]


def test_move_only_limits():
    for opts in ({"move_only": 1, "precision": "bf16x6"}, {"move_only": 3}):
        with pytest.raises(dft3d.Dft3dError):
            dft3d.describe((64, 64, 64), "pencil", **opts)
    with pytest.raises(dft3d.Dft3dError):
        dft3d.describe((100, 64, 64), "pencil", move_only=1)
    with pytest.raises(dft3d.Dft3dError):
        dft3d.describe((64, 64, 64), "volumetric", "shuffled", move_only=1)


# ---------------------------------------------------------------------------
# Pencil orders (DFT3D_OPT_PENCIL_ORDER): the intermediate layouts of the
# pencil schedule.

ORDER_SHAPES = [(8, 16, 32), (32, 4, 8), (2, 64, 4), (16, 16, 16), (1, 8, 4), (4, 1, 2),
                (2048, 2, 4), (4, 1024, 2)]


@pytest.mark.parametrize("shape", ORDER_SHAPES)
@pytest.mark.parametrize("order", [0, 1, 2])
def test_pencil_orders_compute_the_dft(shape, order):
    """Every order's pass list (fields, strides, buffers) computes the 3D
    DFT when each pass is run as the kernels address memory, forward and
    inverse, and its last pass writes the natural order."""
    d = dft3d.describe(shape, "pencil", pencil_order=order)
    assert len(d["passes"]) == 3
    tag = {0: "rot", 1: "swap", 2: "cyc"}[order]
    assert all(p["label"].split()[-1] in (tag, "rot") for p in d["passes"])
    check_pass_maps(d, int(np.prod(shape)))
    g = np.random.default_rng(int(np.prod(shape)) + order)
    x = g.standard_normal(shape) + 1j * g.standard_normal(shape)
    for sign in (-1, 1):
        assert oracle.rel_l2(run_model(x, d, sign), oracle.dft3d(x, sign, "fft")) < 1e-12


def test_pencil_order_default_and_values():
    """Automatic order: the cycle for split precision, for FP32 arrays of
    256 MiB and more and for arrays with an axis of 2048 or more, else the
    rotation; lengths that are not powers of two and split axes keep the
    rotation; values outside -1..2 are rejected.  In the cycle, FP32 passes
    of length up to 1024 take the one-tile kernels unless streaming is
    forced on."""
    def tags(shape, **kw):
        return [p["label"].split()[-1] for p in dft3d.describe(shape, "pencil", **kw)["passes"]]
    assert tags((1024, 1024, 1024)) == ["cyc"] * 3
    assert tags((256, 256, 256)) == ["rot"] * 3
    assert tags((512, 512, 256)) == ["cyc"] * 3           # 512 MiB
    assert tags((256, 256, 512)) == ["cyc"] * 3           # exactly 256 MiB
    assert tags((256, 128, 512)) == ["rot"] * 3           # 128 MiB
    assert tags((4096, 8, 8)) == ["cyc"] * 3
    assert tags((1024, 1024, 1024), precision="bf16x6") == ["cyc"] * 3
    d = dft3d.describe((1024, 1024, 1024), "pencil")
    assert [p["persistent"] for p in d["passes"]] == [0, 0, 0]
    d = dft3d.describe((1024, 1024, 1024), "pencil", nontemporal=1)
    assert [p["persistent"] for p in d["passes"]] == [1, 1, 1]
    d = dft3d.describe((2048, 1024, 512), "pencil")
    assert [(p["n"], p["persistent"]) for p in d["passes"]] == [(512, 0), (2048, 1), (1024, 0)]
    assert tags((1024, 1024, 1024), pencil_order=0) == ["rot"] * 3
    assert tags((2048, 1024, 512)) == ["cyc"] * 3
    assert tags((2048, 1024, 512), pencil_order=0) == ["rot"] * 3
    assert tags((1024, 1024, 1024), pencil_order=2) == ["cyc"] * 3
    assert tags((1024, 1024, 1024), pencil_order=1) == ["swap", "swap", "rot"]
    assert all(t in ("rot",) for t in tags((1000, 1000, 1000), pencil_order=2))
    assert tags((8, 8, 4096), pencil_order=2, split_max=2048)[-1] == "rot"
    for bad in (-2, 3):
        with pytest.raises(dft3d.Dft3dError):
            dft3d.describe((8, 8, 8), "pencil", pencil_order=bad)
