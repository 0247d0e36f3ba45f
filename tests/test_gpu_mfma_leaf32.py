"""GPU parity of the length-32 split-precision leaves (DFT3D_OPT_MFMA_LEAF
= 32): even and odd inputs through two 16-point products on the matrix
cores, the odd half's twiddles folded into its table, joined by one add and
one subtract.  Every compiled length, both kernel forms, forward and
inverse, element by element against the FP64 oracle; the split forms meet
the FP32 bar, the single-term forms a loose one."""
import numpy as np
import pytest

import oracle
from paper_1904_10119_amd import dft3d, inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SPLIT = ["bf16x6", "bf16x9", "fp16x3"]
SINGLE = {"bf16x1": 2e-2, "fp16x1": 3e-3}
LENGTHS = [32, 64, 128, 256, 1024, 2048, 4096]


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dft3d.lib()
    yield


def say(*a):
    print(*a, flush=True)


def execute(x, precision, inverse=False, **kw):
    xt = torch.from_numpy(x).cuda()
    y = torch.empty_like(xt)
    p = dft3d.Plan(x.shape, "pencil", precision=precision, mfma_leaf=32, **kw)
    p.execute(xt, y, inverse=inverse)
    torch.cuda.synchronize()
    p.close()
    return y.cpu().numpy()


def shape_for(n):
    """A pencil-schedule shape whose last axis has length n (the leaf-32
    pass) with fewer pencils than one tile of that pass (8192 / n, 4096 /
    n from 4096 on): a ragged tile."""
    return (2, max(2, 2048 // n), n) if n < 4096 else (1, 1, n)


@pytest.mark.parametrize("precision", SPLIT + list(SINGLE))
@pytest.mark.parametrize("n", LENGTHS)
def test_every_length_element_by_element(precision, n):
    shape = shape_for(n)
    say("case leaf32", precision, shape)
    x = inputs.uniform_c64(shape, 300 + n % 97)
    d = dft3d.describe(shape, "pencil", precision=precision, mfma_leaf=32)
    assert [p["mfma_leaf"] for p in d["passes"] if p["n"] == n] == [32]
    for sign, inv in ((-1, False), (1, True)):
        y = execute(x, precision, inverse=inv)
        ref = oracle.dft3d(x.astype(np.complex128), sign, "fft")
        rel, worst = oracle.compare(y, ref)
        say("  ", sign, rel, worst)
        if precision in SPLIT:
            assert rel <= oracle.tol(x.size), (precision, shape, sign, rel)
            assert worst <= 10 * oracle.tol(x.size), (precision, shape, sign, worst)
        else:
            assert rel <= SINGLE[precision], (precision, shape, sign, rel)


@pytest.mark.parametrize("precision", ["bf16x6", "fp16x3"])
@pytest.mark.parametrize("shape", [(16, 32, 64), (4, 1024, 2), (2, 2, 2048), (4096, 2, 2),
                                   (16, 2, 32), (8, 1024, 8)])
def test_one_tile_and_persistent_forms(precision, shape):
    """Both kernel forms on every axis position (ROW and COL loads), with
    ragged last tiles; the two agree to the tolerance."""
    say("case leaf32 forms", precision, shape)
    x = inputs.uniform_c64(shape, 35)
    for sign, inv in ((-1, False), (1, True)):
        ref = oracle.dft3d(x.astype(np.complex128), sign, "fft")
        outs = [execute(x, precision, inverse=inv, persistent=pers) for pers in (0, 1)]
        for pers, y in enumerate(outs):
            assert oracle.rel_l2(y, ref) <= oracle.tol(x.size), (pers, sign)
        assert oracle.rel_l2(outs[0], outs[1]) <= oracle.tol(x.size)


@pytest.mark.parametrize("precision", SPLIT)
@pytest.mark.parametrize("scale", [0.0, 1e-36, 1e30])
def test_extreme_magnitudes(precision, scale):
    """All-zero, tiny and huge inputs through the length-32 leaves: finite
    outputs, the FP32 bar relative to the exact transform of the input."""
    shape = (8, 8, 1024)
    x = (inputs.uniform_c64(shape, 36).astype(np.complex128) * scale).astype(np.complex64)
    y = execute(x, precision)
    assert np.isfinite(y.view(np.float32)).all()
    if scale == 0.0:
        assert not y.any()
        return
    ref = oracle.dft3d(x.astype(np.complex128), -1, "fft")
    assert oracle.rel_l2(y, ref) <= oracle.tol(x.size), (precision, scale)


def test_gaussian_plane_waves_256cubed():
    """256^3 N(0,1) plus 8 plane waves (the mixed-precision workload) with
    length-32 leaves on every axis (256 = 32 * 8): the split forms meet
    tol(2^24) over all bins and over the non-spike bins, the spikes (N
    times a unit phase) to 10 tol relative, and their largest non-spike
    element error is at most twice the FP32 path's on the same input (the
    plane waves' rounding errors are coherent and gather at a few bins: the
    FP32 path itself reaches about 1e-4 of the non-spike rms there, so an
    element bar tied to the rms does not apply to this input)."""
    shape = (256, 256, 256)
    x, freqs, _ = inputs.gaussian_waves_c64(shape, 3)
    ref = oracle.dft3d_fft_c64(x, -1)
    mask = np.ones(shape, dtype=bool)
    mask[tuple(freqs.T)] = False
    spikes = tuple(freqs.T)
    ns_rms = np.sqrt(np.mean(np.abs(ref[mask]) ** 2))

    def worst_non_spike(y):
        return np.max(np.abs(y[mask] - ref[mask])) / ns_rms

    xt = torch.from_numpy(x).cuda()
    y32 = dft3d.fftn(xt, schedule="pencil")
    torch.cuda.synchronize()
    fp32_worst = worst_non_spike(y32.cpu().numpy())
    say("fp32 256^3 worst non-spike", fp32_worst)
    for precision in SPLIT:
        y = execute(x, precision)
        rel = oracle.rel_l2(y, ref)
        rel_ns = oracle.rel_l2(y[mask], ref[mask])
        worst_ns = worst_non_spike(y)
        spike = np.max(np.abs(y[spikes] - ref[spikes]) / np.abs(ref[spikes]))
        say("leaf32 256^3", precision, rel, "non-spike", rel_ns, worst_ns, "spikes", spike)
        assert rel <= oracle.tol(x.size) and rel_ns <= oracle.tol(x.size), precision
        assert spike <= 10 * oracle.tol(x.size), precision
        assert worst_ns <= 2 * fp32_worst, (precision, worst_ns, fp32_worst)
