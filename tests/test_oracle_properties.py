"""Property tests of the FP64 oracle on random tiny shapes (hypothesis):
for any power-of-two shape up to 16 per axis and any seed, O1 (direct sums)
and O2 (radix-2) agree with each other and with numpy's pocketfft, and both
satisfy linearity, Parseval and the double-transform reversal identity.  The
shapes and values are drawn by hypothesis; nothing here comes from the GPU
library."""
import numpy as np
import pytest

hypothesis = pytest.importorskip("hypothesis")
from hypothesis import given, settings, strategies as st  # noqa: E402

import oracle  # noqa: E402

POW2 = st.sampled_from([1, 2, 4, 8, 16])
SHAPES = st.tuples(POW2, POW2, POW2)
SEEDS = st.integers(min_value=0, max_value=2**31 - 1)
SIGNS = st.sampled_from([-1, 1])


def draw(shape, seed):
    g = np.random.default_rng(seed)
    return g.standard_normal(shape) + 1j * g.standard_normal(shape)


@settings(max_examples=40, deadline=None)
@given(SHAPES, SEEDS, SIGNS)
def test_methods_agree_with_library(shape, seed, sign):
    x = draw(shape, seed)
    d = oracle.dft3d(x, sign, "direct")
    f = oracle.dft3d(x, sign, "fft")
    lib = np.fft.fftn(x) if sign == -1 else np.fft.ifftn(x) * x.size
    assert oracle.rel_l2(d, lib) < 1e-13
    assert oracle.rel_l2(f, lib) < 1e-13


@settings(max_examples=30, deadline=None)
@given(SHAPES, SEEDS, st.complex_numbers(max_magnitude=4, allow_nan=False,
                                         allow_infinity=False))
def test_linearity_and_parseval(shape, seed, alpha):
    x = draw(shape, seed)
    y = draw(shape, seed + 1)
    for method in ("direct", "fft"):
        lhs = oracle.dft3d(alpha * x + y, -1, method)
        rhs = alpha * oracle.dft3d(x, -1, method) + oracle.dft3d(y, -1, method)
        assert np.allclose(lhs, rhs, rtol=0, atol=1e-11 * (1 + abs(alpha)) * x.size)
        X = oracle.dft3d(x, -1, method)
        assert abs(np.sum(abs(X) ** 2) / (x.size * np.sum(abs(x) ** 2)) - 1) < 1e-12


@settings(max_examples=30, deadline=None)
@given(SHAPES, SEEDS)
def test_double_transform_reverses(shape, seed):
    x = draw(shape, seed)
    yy = oracle.dft3d(oracle.dft3d(x, -1, "fft"), -1, "fft")
    rev = x[np.ix_(*[(-np.arange(n)) % n for n in shape])]
    assert np.allclose(yy, x.size * rev, rtol=0, atol=1e-11 * x.size)
