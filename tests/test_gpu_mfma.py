"""GPU parity of the split-precision MFMA leaves of length 16 (forced with
DFT3D_OPT_MFMA_LEAF = 16; the length-32 leaves have their own tests):
radix-16 stages as real GEMMs on the matrix cores with bf16 / fp16
operand splitting and FP32 accumulation.  The split forms (bf16x6,
bf16x9, fp16x3) meet the same tolerance as FP32; the single-term forms
(bf16x1, fp16x1) are reported and only checked against a loose bound."""
import sys

import numpy as np
import pytest

import oracle
from paper_1904_10119_amd import dft3d, inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SPLIT = ["bf16x6", "bf16x9", "fp16x3"]
SINGLE = {"bf16x1": 2e-2, "fp16x1": 3e-3}


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dft3d.lib()
    yield


def say(*a):
    print(*a, flush=True)


def run(x, precision, schedule="pencil", inverse=False):
    xt = torch.from_numpy(x).cuda()
    y = dft3d.fftn(xt, schedule=schedule, precision=precision, inverse=inverse,
                   mfma_leaf=0 if precision == "fp32" else 16)
    torch.cuda.synchronize()
    return y.cpu().numpy()


@pytest.mark.parametrize("precision", SPLIT + list(SINGLE))
@pytest.mark.parametrize("shape", [(16, 32, 64), (128, 2, 256), (512, 4, 2),
                                   (4, 1024, 2), (2, 2, 2048), (4096, 2, 2)])
def test_every_length_against_oracle(precision, shape):
    say("case", precision, shape)
    x = inputs.uniform_c64(shape, 31)
    for sign, inv in ((-1, False), (1, True)):
        y = run(x, precision, inverse=inv)
        ref = oracle.dft3d(x.astype(np.complex128), sign, "fft")
        err = oracle.rel_l2(y, ref)
        say("  ", sign, err)
        bound = oracle.tol(x.size) if precision in SPLIT else SINGLE[precision]
        assert err <= bound, (precision, shape, sign, err)


def test_256cubed_gaussian_plane_waves():
    """Mixed-precision 256^3 workload: N(0,1) plus 8 plane waves.  Reports
    the error of every form; the split forms meet tol(2^24) overall and on
    the non-spike bins.  At a plane-wave bin the transform is N e^{i phi}
    plus the noise's own transform there, a complex Gaussian of mean square
    2N; the oracle's spikes are checked against that closed form and the GPU
    spikes against the oracle point by point."""
    shape = (256, 256, 256)
    x, freqs, phases = inputs.gaussian_waves_c64(shape, 3)
    ref = oracle.dft3d(x.astype(np.complex128), -1, "fft")
    N = x.size
    spikes = tuple(freqs.T)
    mask = np.ones(shape, dtype=bool)
    mask[spikes] = False
    want = N * np.exp(1j * phases)
    assert np.max(np.abs(ref[spikes] - want)) <= 8 * np.sqrt(2 * N)
    errs = {}
    for prec in ["fp32"] + SPLIT + list(SINGLE):
        y = run(x, prec)
        errs[prec] = (oracle.rel_l2(y, ref), oracle.rel_l2(y[mask], ref[mask]))
        say("  256^3", prec, "rel_l2 all %.3e non-spike %.3e" % errs[prec])
        if prec in SPLIT + ["fp32"]:
            assert errs[prec][0] <= oracle.tol(N) and errs[prec][1] <= oracle.tol(N)
            spike_err = np.max(np.abs(y[spikes] - ref[spikes]) / np.abs(ref[spikes]))
            assert spike_err <= 10 * oracle.tol(N)
        else:
            assert errs[prec][0] <= SINGLE[prec]


@pytest.mark.parametrize("precision", SPLIT)
def test_round_trip_split(precision):
    shape = (64, 128, 32)
    x = inputs.uniform_c64(shape, 32)
    y = run(x, precision)
    back = run(y, precision, inverse=True) / x.size
    assert oracle.rel_l2(back, x) <= 2 * oracle.tol(x.size)


@pytest.mark.parametrize("schedule", ["slab", "volumetric", "auto"])
def test_split_on_other_schedules(schedule):
    shape = (64, 256, 32)
    x = inputs.uniform_c64(shape, 33)
    y = run(x, "bf16x6", schedule=schedule)
    ref = oracle.dft3d(x.astype(np.complex128), -1, "fft")
    assert oracle.rel_l2(y, ref) <= oracle.tol(x.size)


@pytest.mark.parametrize("precision", ["bf16x6", "fp16x3"])
@pytest.mark.parametrize("shape", [(16, 32, 64), (128, 2, 256), (4, 1024, 2),
                                   (2, 2, 2048), (4096, 2, 2), (16, 2, 16), (8, 512, 8)])
def test_one_tile_and_persistent_forms(precision, shape):
    """The one-tile-per-workgroup and the persistent (prefetching) MFMA
    kernels both meet the tolerance, also with ragged last tiles (shapes
    with fewer pencils than a tile), forward and inverse."""
    say("case mfma forms", precision, shape)
    x = inputs.uniform_c64(shape, 34)
    xt = torch.from_numpy(x).cuda()
    for sign, inv in ((-1, False), (1, True)):
        ref = oracle.dft3d(x.astype(np.complex128), sign, "fft")
        outs = []
        for pers in (0, 1):
            p = dft3d.Plan(shape, "pencil", precision=precision, persistent=pers,
                           mfma_leaf=16)
            y = torch.empty_like(xt)
            p.execute(xt, y, inverse=inv)
            torch.cuda.synchronize()
            outs.append(y.cpu().numpy())
            p.close()
            assert oracle.rel_l2(outs[-1], ref) <= oracle.tol(x.size), (pers, sign)
        assert oracle.rel_l2(outs[0], outs[1]) <= oracle.tol(x.size)


@pytest.mark.parametrize("precision", SPLIT)
@pytest.mark.parametrize("scale", [0.0, 1e-30, 1e-36, 1e-41, 1e30])
def test_split_extreme_magnitudes(precision, scale):
    """The splits at the ends of the FP32 range: all-zero input, tiny
    (1e-36 makes every 16-vector's largest component fall below 2^-101, where
    the per-vector power-of-two scale is capped; unscaled, the bf16 residuals
    of such inputs fell into the subnormal range: 4.6e-5 rel_l2 for bf16x6),
    subnormal (1e-41) and huge inputs.  Outputs
    are finite; down to 1e-36 they meet the FP32 tolerance relative to the
    exact transform of the same (rounded) input, and the subnormal case is
    checked against the output's size for fp16x3 (the input itself carries
    only a few significant bits there)."""
    shape = (8, 32, 64)
    say("case extreme", precision, scale)
    x = (inputs.uniform_c64(shape, 33).astype(np.complex128) * scale).astype(np.complex64)
    y = run(x, precision)
    assert np.isfinite(y.view(np.float32)).all(), (precision, scale)
    ref = oracle.dft3d(x.astype(np.complex128), -1, "fft")
    if scale == 0.0:
        assert not y.any()
        return
    if scale >= 1e-36:
        err = oracle.rel_l2(y, ref)
        say("  ", err)
        assert err <= oracle.tol(x.size), (precision, scale, err)
    elif precision == "fp16x3":
        # the scaled fp16 terms keep ~15 bits of these inputs
        err = np.max(np.abs(y - ref)) / np.max(np.abs(ref))
        say("  subnormal max error / max output", err)
        assert err <= 1e-3, (precision, scale, err)
    # bf16 terms of subnormal inputs may be flushed by the matrix cores:
    # only finiteness is required there


@pytest.mark.parametrize("precision", SPLIT)
def test_split_zero_pencils_among_data(precision):
    """Pencils that are exactly zero between ordinary ones (the fp16 scale's
    zero branch, per 16-vector)."""
    shape = (16, 16, 256)
    x = inputs.uniform_c64(shape, 34)
    x[:, ::3, :] = 0
    x[::5] = 0
    y = run(x, precision)
    ref = oracle.dft3d(x.astype(np.complex128), -1, "fft")
    assert np.isfinite(y.view(np.float32)).all()
    assert oracle.rel_l2(y, ref) <= oracle.tol(x.size)
