"""Pins for the FP64 oracle (O1 direct, O2 radix-2) against what the paper
and the mathematics fix -- never against the oracle itself.

* hand-written DFT_2 / DFT_4 / DFT_8 values (tests/golden/dft_small.txt),
  from the definition in Section 2.1, eqs. (1)-(2);
* closed forms: delta -> ones, shifted delta -> pure phase, constant ->
  scaled delta, single exponential -> scaled delta;
* brute-force triple sums in plain Python on tiny (also non power-of-two)
  shapes, which pins the axis order and the separability of Section 2.3;
* invariants: linearity, Parseval, F(F(x)) = N * index reversal, the shift
  theorem, Hermitian symmetry of real input, forward/inverse round trip;
* O1 == O2 and the numpy (pocketfft) library routine as a third witness.
"""
import cmath
import itertools

import numpy as np
import pytest

import oracle
from conftest import load_golden

METHODS = ("direct", "fft")


def rng_c128(shape, seed):
    g = np.random.default_rng(seed)
    return g.standard_normal(shape) + 1j * g.standard_normal(shape)


@pytest.mark.parametrize("method", METHODS)
def test_golden_small_dfts(method):
    for label, (n, x, y) in load_golden("dft_small.txt").items():
        got = oracle.dft1d(x, -1, method)
        assert np.allclose(got, y, rtol=0, atol=1e-13), label
        # the inverse undoes the forward up to the factor n (unnormalised)
        back = oracle.dft1d(y, +1, method)
        assert np.allclose(back, n * x, rtol=0, atol=1e-12), label


def brute_force_3d(x, sign):
    """The triple sum of the definition, literally, in Python."""
    n0, n1, n2 = x.shape
    y = np.zeros(x.shape, dtype=np.complex128)
    for k0, k1, k2 in itertools.product(range(n0), range(n1), range(n2)):
        s = 0j
        for i0, i1, i2 in itertools.product(range(n0), range(n1), range(n2)):
            ph = (i0 * k0 % n0) / n0 + (i1 * k1 % n1) / n1 + (i2 * k2 % n2) / n2
            s += x[i0, i1, i2] * cmath.exp(sign * 2j * cmath.pi * ph)
        y[k0, k1, k2] = s
    return y


@pytest.mark.parametrize("shape", [(2, 3, 5), (3, 1, 4), (1, 6, 2)])
@pytest.mark.parametrize("sign", [-1, 1])
def test_direct_equals_brute_force_any_size(shape, sign):
    x = rng_c128(shape, 11)
    ref = brute_force_3d(x, sign)
    assert oracle.rel_l2(oracle.dft3d(x, sign, "direct"), ref) < 1e-14


@pytest.mark.parametrize("shape", [(2, 4, 8), (8, 2, 4), (4, 8, 1)])
@pytest.mark.parametrize("method", METHODS)
def test_brute_force_pow2(shape, method):
    x = rng_c128(shape, 12)
    for sign in (-1, 1):
        ref = brute_force_3d(x, sign)
        assert oracle.rel_l2(oracle.dft3d(x, sign, method), ref) < 1e-14


@pytest.mark.parametrize("method", METHODS)
def test_delta_at_origin_gives_ones(method):
    x = np.zeros((8, 4, 16), dtype=np.complex128)
    x[0, 0, 0] = 1.0
    y = oracle.dft3d(x, -1, method)
    assert np.allclose(y, 1.0, rtol=0, atol=1e-14)


@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("pos", [(1, 0, 0), (0, 3, 0), (0, 0, 5), (5, 2, 9)])
def test_shifted_delta_gives_phase(method, pos):
    shape = (8, 4, 16)
    x = np.zeros(shape, dtype=np.complex128)
    x[pos] = 1.0
    y = oracle.dft3d(x, -1, method)
    k0, k1, k2 = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    a, b, c = pos
    phase = (a * k0 % 8) / 8 + (b * k1 % 4) / 4 + (c * k2 % 16) / 16
    expect = np.exp(-2j * np.pi * phase)
    assert np.max(np.abs(y - expect)) < 1e-13


@pytest.mark.parametrize("method", METHODS)
def test_constant_gives_scaled_delta(method):
    shape = (4, 16, 8)
    c = 0.75 - 1.25j
    y = oracle.dft3d(np.full(shape, c), -1, method)
    expect = np.zeros(shape, dtype=np.complex128)
    expect[0, 0, 0] = c * np.prod(shape)
    assert np.max(np.abs(y - expect)) < 1e-11


@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("freq", [(1, 2, 3), (7, 0, 15), (0, 3, 1)])
def test_single_exponential_gives_scaled_delta(method, freq):
    shape = (8, 4, 16)
    i0, i1, i2 = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    f0, f1, f2 = freq
    ph = (f0 * i0 % 8) / 8 + (f1 * i1 % 4) / 4 + (f2 * i2 % 16) / 16
    x = np.exp(2j * np.pi * ph)
    y = oracle.dft3d(x, -1, method)
    expect = np.zeros(shape, dtype=np.complex128)
    expect[freq] = np.prod(shape)
    assert np.max(np.abs(y - expect)) < 1e-10


@pytest.mark.parametrize("method", METHODS)
def test_linearity(method):
    shape = (4, 8, 16)
    a, b = rng_c128(shape, 1), rng_c128(shape, 2)
    alpha, beta = 0.3 - 2j, -1.7 + 0.5j
    lhs = oracle.dft3d(alpha * a + beta * b, -1, method)
    rhs = alpha * oracle.dft3d(a, -1, method) + beta * oracle.dft3d(b, -1, method)
    assert oracle.rel_l2(lhs, rhs) < 1e-14


@pytest.mark.parametrize("method", METHODS)
def test_parseval(method):
    shape = (16, 8, 32)
    x = rng_c128(shape, 3)
    y = oracle.dft3d(x, -1, method)
    n = x.size
    assert abs(np.vdot(y, y).real - n * np.vdot(x, x).real) < 1e-12 * n * np.vdot(x, x).real


@pytest.mark.parametrize("method", METHODS)
def test_double_forward_is_scaled_reversal(method):
    shape = (8, 16, 4)
    x = rng_c128(shape, 4)
    yy = oracle.dft3d(oracle.dft3d(x, -1, method), -1, method)
    rev = x[np.ix_(*[(-np.arange(n)) % n for n in shape])]
    assert oracle.rel_l2(yy, x.size * rev) < 1e-14


@pytest.mark.parametrize("method", METHODS)
def test_shift_theorem(method):
    shape = (8, 4, 16)
    x = rng_c128(shape, 5)
    s = (3, 1, 6)
    xs = np.roll(x, s, axis=(0, 1, 2))  # xs[i] = x[i - s]
    k0, k1, k2 = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    ph = (s[0] * k0 % 8) / 8 + (s[1] * k1 % 4) / 4 + (s[2] * k2 % 16) / 16
    lhs = oracle.dft3d(xs, -1, method)
    rhs = np.exp(-2j * np.pi * ph) * oracle.dft3d(x, -1, method)
    assert oracle.rel_l2(lhs, rhs) < 1e-14


@pytest.mark.parametrize("method", METHODS)
def test_real_input_hermitian(method):
    shape = (8, 16, 4)
    x = np.random.default_rng(6).standard_normal(shape).astype(np.complex128)
    y = oracle.dft3d(x, -1, method)
    yr = y[np.ix_(*[(-np.arange(n)) % n for n in shape])]
    assert oracle.rel_l2(y, np.conj(yr)) < 1e-14


@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("shape", [(64, 64, 64), (2, 128, 32)])
def test_round_trip(method, shape):
    x = rng_c128(shape, 7)
    back = oracle.dft3d(oracle.dft3d(x, -1, method), +1, method) / x.size
    assert oracle.rel_l2(back, x) < 1e-14


@pytest.mark.parametrize("shape", [(1, 1, 1), (2, 2, 2), (16, 8, 4),
                                   (4, 32, 64), (64, 64, 64), (128, 64, 32)])
def test_direct_equals_fft(shape):
    x = rng_c128(shape, 8)
    for sign in (-1, 1):
        a = oracle.dft3d(x, sign, "direct")
        b = oracle.dft3d(x, sign, "fft")
        assert oracle.rel_l2(a, b) < 1e-13


@pytest.mark.parametrize("shape", [(16, 8, 4), (64, 64, 64), (32, 128, 64)])
def test_numpy_library_witness(shape):
    x = rng_c128(shape, 9)
    assert oracle.rel_l2(oracle.dft3d(x, -1, "fft"), np.fft.fftn(x)) < 1e-12
    assert oracle.rel_l2(oracle.dft3d(x, +1, "fft"),
                         np.fft.ifftn(x) * x.size) < 1e-12


@pytest.mark.parametrize("n", [2, 16, 1024, 2048, 4096])
def test_1d_radix2_against_library(n):
    x = rng_c128((n,), 10)
    assert oracle.rel_l2(oracle.dft1d(x, -1, "fft"), np.fft.fft(x)) < 1e-13


def test_sample_pencils_match_full_transform():
    shape = (16, 32, 64)
    x = rng_c128(shape, 13).astype(np.complex64)
    k0 = [0, 5, 15, 7]
    k1 = [0, 31, 2, 16]
    for sign in (-1, 1):
        full = oracle.dft3d(x.astype(np.complex128), sign, "fft")
        s = oracle.sample_pencils(x, k0, k1, sign)
        assert oracle.rel_l2(s, full[k0, k1, :]) < 1e-13


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_fft_pencils_match_library(axis):
    shape = (8, 16, 32)
    x = rng_c128(shape, 14).astype(np.complex64)
    ref = np.moveaxis(np.fft.fft(x.astype(np.complex128), axis=axis), axis, -1)
    ref = ref.reshape(-1, shape[axis])
    got = oracle.fft_pencils(x, axis, 3, 20)
    assert oracle.rel_l2(got, ref[3:23]) < 1e-14


def test_bad_arguments_raise():
    with pytest.raises(oracle.OracleError):
        oracle.dft3d(np.zeros((3, 4, 4)), -1, "fft")  # not a power of two
    with pytest.raises(oracle.OracleError):
        oracle.dft3d(np.zeros((4, 4, 4)), 2, "direct")  # bad sign
    with pytest.raises(oracle.OracleError):
        oracle.sample_pencils(np.zeros((4, 4, 4), np.complex64), [4], [0])


def test_fft_c64_in_place_equals_o2_and_compare_matches_definitions():
    """dft3d_fft_c64 (O2 on one FP64 array, for 2^30-point inputs) is O2
    exactly; compare() gives rel_l2 and the largest element error relative
    to the reference's root mean square, also for a planted single-element
    error."""
    from paper_1904_10119_amd import inputs
    x = inputs.uniform_c64((16, 8, 32), 21)
    a = oracle.dft3d(x, -1, "fft")
    b = oracle.dft3d_fft_c64(x, -1)
    assert np.array_equal(a, b)
    a_inv = oracle.dft3d(x, +1, "fft")
    assert np.array_equal(a_inv, oracle.dft3d_fft_c64(x, +1))
    y = a.astype(np.complex64)
    rel, worst = oracle.compare(y, a, planes=3)
    assert rel == pytest.approx(oracle.rel_l2(y, a), rel=1e-12)
    rms = np.sqrt(np.mean(np.abs(a) ** 2))
    assert worst == pytest.approx(np.max(np.abs(y - a)) / rms, rel=1e-12)
    z = y.copy()
    z[5, 3, 7] += 0.5 * rms
    rel2, worst2, at = oracle.compare(z, a, planes=4, where=True)
    assert worst2 == pytest.approx(np.abs(z[5, 3, 7] - a[5, 3, 7]) / rms, rel=1e-6)
    assert at == (5, 3, 7)
    assert rel2 > rel


def test_thread_count_can_be_set():
    n = oracle.num_threads()
    oracle.set_num_threads(1)
    assert oracle.num_threads() == 1
    oracle.set_num_threads(n)
    assert oracle.num_threads() == n
