"""Full-size parity: every element of the 2^30-point transforms (1024^3 and
2048 x 1024 x 512, every schedule and split-precision form at 1024^3)
against the FP64 oracle O2 on the whole array.

Each result must meet rel_l2 <= tol(N) over the whole array and, element by
element, |y - ref| <= 10 tol(N) rms(ref): a single wrong element of the size
of a typical output would exceed that bound by five orders of magnitude.
The host needs about 50 GB for the input, the two FP64 references and one
result (the test prints the host's memory)."""
import os

import numpy as np
import pytest

import oracle
from paper_1904_10119_amd import dft3d, inputs

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

SEEDS = {(1024, 1024, 1024): 2, (2048, 1024, 512): 5}
_cache = {}


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    with open("/proc/meminfo") as f:
        say("host memory:", " ".join(f.readline().split()[1:]))
    dft3d.lib()
    yield
    _cache.clear()


def refs(shape):
    """Input and FP64 forward / inverse references of one shape (the
    previous shape's are dropped first)."""
    if shape not in _cache:
        _cache.clear()
        x = inputs.uniform_c64(shape, SEEDS[shape])
        say("oracle O2 forward", shape)
        fwd = oracle.dft3d_fft_c64(x, -1)
        say("oracle O2 inverse", shape)
        inv = oracle.dft3d_fft_c64(x, +1)
        _cache[shape] = (x, fwd, inv)
    return _cache[shape]


def run(shape, inverse=False, **kw):
    x, _, _ = refs(shape)
    xt = torch.from_numpy(x).cuda()
    y = torch.empty_like(xt)
    p = dft3d.Plan(shape, **kw)
    p.execute(xt, y, inverse=inverse)
    torch.cuda.synchronize()
    p.close()
    out = y.cpu().numpy()
    del xt, y
    torch.cuda.empty_cache()
    return out


def check(shape, got, ref, what):
    n = int(np.prod(shape))
    rel, worst, at = oracle.compare(got, ref, where=True)
    say(f"{what} {shape}: rel_l2 {rel:.3e} max element {worst:.3e} x rms at {at} "
        f"(tol {oracle.tol(n):.3e})")
    assert rel <= oracle.tol(n), (what, rel)
    assert worst <= 10 * oracle.tol(n), (what, worst)


CASES_1024 = [("pencil", {}), ("slab", {}), ("volumetric", {}),
              ("pencil", {"precision": "bf16x6"}), ("pencil", {"precision": "bf16x9"}),
              ("pencil", {"precision": "fp16x3"}),
              ("pencil", {"precision": "bf16x6", "mfma_leaf": 32}),
              ("pencil", {"precision": "fp16x3", "mfma_leaf": 32})]


def case_id(schedule, opts):
    leaf = f"-leaf{opts['mfma_leaf']}" if "mfma_leaf" in opts else ""
    return f"{schedule}-{opts.get('precision', 'fp32')}{leaf}"


@pytest.mark.parametrize("schedule,opts", CASES_1024,
                         ids=[case_id(s, o) for s, o in CASES_1024])
def test_1024_cubed_forward_every_element(schedule, opts):
    shape = (1024, 1024, 1024)
    say("case fullsize forward", shape, schedule, opts)
    _, fwd, _ = refs(shape)
    check(shape, run(shape, schedule=schedule, **opts), fwd, f"{schedule} {opts}")


@pytest.mark.parametrize("schedule", ["pencil", "slab", "volumetric"])
def test_1024_cubed_inverse_every_element(schedule):
    shape = (1024, 1024, 1024)
    say("case fullsize inverse", shape, schedule)
    _, _, inv = refs(shape)
    check(shape, run(shape, inverse=True, schedule=schedule), inv, f"{schedule} inverse")


def test_1024_cubed_shuffled_every_element():
    """The volumetric shuffled order: natural index k' + b l' of every axis
    sits at l' + a k'; each natural slab is gathered from the result."""
    shape = (1024, 1024, 1024)
    say("case fullsize shuffled", shape)
    _, fwd, _ = refs(shape)
    got = run(shape, schedule="volumetric", layout="shuffled")
    a = dft3d.shuffle_factors(shape)
    pos = []
    for n, ad in zip(shape, a):
        nat = oracle.shuffled_positions(n, ad)    # natural index at each position
        inv = np.empty_like(nat)
        inv[nat] = np.arange(n)                   # position of each natural index
        pos.append(inv)
    num = den = worst = 0.0
    for i in range(0, shape[0], 16):
        g = got[pos[0][i:i + 16]][:, pos[1]][:, :, pos[2]].astype(np.complex128)
        r = fwd[i:i + 16]
        d = g - r
        e2 = d.real ** 2 + d.imag ** 2
        num += float(e2.sum())
        worst = max(worst, float(e2.max()))
        den += float((r.real ** 2 + r.imag ** 2).sum())
    n = int(np.prod(shape))
    rel = np.sqrt(num / den)
    worst = np.sqrt(worst) / np.sqrt(den / n)
    say(f"shuffled {shape}: rel_l2 {rel:.3e} max element {worst:.3e} x rms")
    assert rel <= oracle.tol(n) and worst <= 10 * oracle.tol(n)


def test_1024_cubed_shuffled_inverse_every_element():
    """The inverse from the shuffled order (four passes, two of them the
    fused transposed passes): the input permuted into the shuffled order
    must come back as the natural inverse DFT of the input, every element."""
    shape = (1024, 1024, 1024)
    say("case fullsize shuffled inverse", shape)
    x, _, inv = refs(shape)
    d = dft3d.describe(shape, "volumetric", "shuffled")
    assert [p["fused_axes"] for p in d["inverse_passes"]] == [0, 3, 3, 0]
    xs = np.ascontiguousarray(oracle.to_shuffled(x, dft3d.shuffle_factors(shape)))
    xt = torch.from_numpy(xs).cuda()
    del xs
    y = torch.empty_like(xt)
    p = dft3d.Plan(shape, "volumetric", layout="shuffled")
    p.execute(xt, y, inverse=True)
    torch.cuda.synchronize()
    p.close()
    got = y.cpu().numpy()
    del xt, y
    torch.cuda.empty_cache()
    check(shape, got, inv, "volumetric shuffled inverse")


CASES_2048 = [("auto", {}, False), ("auto", {}, True), ("pencil", {}, False),
              ("auto", {"precision": "bf16x6"}, False),
              ("auto", {"precision": "bf16x6", "mfma_leaf": 32}, False)]


@pytest.mark.parametrize("schedule,opts,inverse", CASES_2048,
                         ids=["auto-fwd", "auto-inv", "pencil-fwd", "auto-bf16x6",
                              "auto-bf16x6-leaf32"])
def test_2048_1024_512_every_element(schedule, opts, inverse):
    shape = (2048, 1024, 512)
    say("case fullsize", shape, schedule, opts, "inverse" if inverse else "forward")
    _, fwd, inv = refs(shape)
    got = run(shape, inverse=inverse, schedule=schedule, **opts)
    check(shape, got, inv if inverse else fwd, f"{schedule} {opts} inv={inverse}")
