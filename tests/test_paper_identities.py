"""The paper's decompositions, written as numpy models and checked against the
oracle's direct DFT.  These pin the readings the HIP schedules rely on:

* eq. (3) four-step Cooley-Tukey with the column-major views of Section 2.1
  (x~[l, k] = x[l + n0 k], y~[k', l'] = y[k' + n1 l']), on the Fig. 2 case
  16 = 4 * 4 and the Fig. 10 case 256 = 16 * 16;
* eq. (5) six-step, with the twiddle matrix read transposed so that the
  element-wise product is well defined (its entries are still w_n^{lk},
  eq. (4));
* eq. (6) slab (2D DFT of planes, then 1D) and eq. (8) pencil decomposition;
* the pencil rotation xyz -> yzx -> zxy of Section 2.4: three
  FFT-then-transpose passes return natural order;
* eqs. (13)-(17): the one-exchange parallel 1D DFT on p processors with
  rows dealt out cyclically, which keeps the cyclic distribution (Section 3.2);
* the 'shuffled' output order of a four-step transform without its final
  transposition (Section 2.4).
"""
import numpy as np
import pytest

import oracle


def dft_matrix(n, sign=-1):
    """DFT_n of eq. (2), each column taken from the oracle's direct DFT of a
    unit vector (so no root of unity is retyped here)."""
    eye = np.eye(n, dtype=np.complex128)
    return np.stack([oracle.dft1d(eye[:, k], sign, "direct") for k in range(n)],
                    axis=1)


def twiddle(n0, n1, sign=-1):
    """Twid_{n0 x n1}[l, k] = w_n^{l k} (eq. (4)), n = n0 n1, read off the
    DFT_n matrix so that no root of unity is retyped."""
    F = dft_matrix(n0 * n1, sign)
    l = np.arange(n0).reshape(n0, 1)
    k = np.arange(n1).reshape(1, n1)
    return F[1, (l * k) % (n0 * n1)]


def rng_vec(n, seed):
    g = np.random.default_rng(seed)
    return g.standard_normal(n) + 1j * g.standard_normal(n)


@pytest.mark.parametrize("n0,n1", [(4, 4), (16, 16), (4, 8), (8, 2)])
def test_eq3_four_step(n0, n1):
    n = n0 * n1
    x = rng_vec(n, n)
    xt = x.reshape(n1, n0).T                          # x~[l,k] = x[l + n0 k]
    yt = (twiddle(n0, n1) * (xt @ dft_matrix(n1))).T @ dft_matrix(n0)
    y = yt.T.reshape(n)                               # y[k' + n1 l'] = y~[k',l']
    assert oracle.rel_l2(y, oracle.dft1d(x, -1, "direct")) < 1e-14


@pytest.mark.parametrize("n0,n1", [(4, 4), (4, 8)])
def test_eq5_six_step_with_transposed_twiddle(n0, n1):
    n = n0 * n1
    x = rng_vec(n, 2 * n)
    xt = x.reshape(n1, n0).T
    inner = dft_matrix(n1) @ xt.T                     # n1 x n0
    yt = (dft_matrix(n0) @ (twiddle(n0, n1).T * inner).T).T
    assert oracle.rel_l2(yt.T.reshape(n), oracle.dft1d(x, -1, "direct")) < 1e-14


def test_eq6_slab_and_eq8_pencil():
    shape = (4, 8, 16)
    g = np.random.default_rng(3)
    x = g.standard_normal(shape) + 1j * g.standard_normal(shape)
    ref = oracle.dft3d(x, -1, "direct")
    F0, F1, F2 = (dft_matrix(n) for n in shape)
    # slab: 2D DFT of every (n1, n2) plane, then the 1D DFT across planes
    planes = np.einsum("ab,ibc,cd->iad", F1, x, F2)
    slab = np.einsum("ki,iad->kad", F0, planes)
    assert oracle.rel_l2(slab, ref) < 1e-14
    # pencil: three batches of 1D DFTs, one per dimension
    p = np.einsum("ijc,cd->ijd", x, F2)
    p = np.einsum("bj,ijd->ibd", F1, p)
    p = np.einsum("ai,ibd->abd", F0, p)
    assert oracle.rel_l2(p, ref) < 1e-14


def test_pencil_rotations_return_natural_order():
    """FFT along the contiguous axis of a (B, n) view, write (n, B): after
    three such passes (n0,n1,n2) -> (n2,n0,n1) -> (n1,n2,n0) -> (n0,n1,n2)."""
    shape = (8, 4, 16)
    g = np.random.default_rng(4)
    x = g.standard_normal(shape) + 1j * g.standard_normal(shape)
    buf, cur = x.reshape(-1), shape
    for _ in range(3):
        n = cur[2]
        rows = buf.reshape(-1, n)
        out = np.stack([oracle.dft1d(r, -1, "direct") for r in rows])
        buf = out.T.reshape(-1)                       # rotate-on-write
        cur = (cur[2], cur[0], cur[1])
    assert cur == shape
    assert oracle.rel_l2(buf.reshape(shape), oracle.dft3d(x, -1, "direct")) < 1e-14


@pytest.mark.parametrize("p", [2, 4])
def test_eq13_to_17_one_exchange_cyclic(p):
    """n = 256 = 16 * 16 on p processors (Fig. 10 uses p = 4): processor r
    owns rows l = r, r + p, ... of X~ (iota0 x iota1), does the local DFT_n1
    and twiddle (T0), one all-to-all (T1), a local transpose (T2) and the
    local DFT_n0; the output keeps the cyclic row distribution."""
    n0 = n1 = 16
    n = n0 * n1
    x = rng_vec(n, 5)
    X = x.reshape(n1, n0).T                           # X~[l, k] = x[l + n0 k]
    tw = twiddle(n0, n1)
    F1, F0 = dft_matrix(n1), dft_matrix(n0)
    local = [X[r::p, :] for r in range(p)]            # [(0)()] cyclic rows
    T0 = [(local[r] @ F1) * tw[r::p, :] for r in range(p)]
    # T1[()(0)]: processor r now owns columns k' = r, r + p, ... of T0
    T1 = [np.concatenate([T0[s] for s in range(p)], axis=0) for _ in range(p)]
    order = np.concatenate([np.arange(s, n0, p) for s in range(p)])
    T1 = [t[np.argsort(order), :][:, r::p] for r, t in enumerate(T1)]
    T2 = [t.T for t in T1]                            # local transpose
    Y = [t @ F0 for t in T2]                          # rows k' = r, r+p, ...
    y = np.empty((n1, n0), dtype=np.complex128)
    for r in range(p):
        y[r::p, :] = Y[r]
    ref = oracle.dft1d(x, -1, "direct")
    assert oracle.rel_l2(y.T.reshape(n), ref) < 1e-14


@pytest.mark.parametrize("a,b", [(4, 4), (16, 16), (4, 8)])
def test_shuffled_order_is_digit_transpose(a, b):
    """Without the final transposition, a four-step transform of n = a * b
    leaves natural entry y[k' + b l'] (k' < b, l' < a) at l' + a k'."""
    n = a * b
    x = rng_vec(n, 6)
    X = x.reshape(b, a).T                             # X[l, k] = x[l + a k]
    T = twiddle(a, b) * (X @ dft_matrix(b))           # a x b, stage I + II
    S = dft_matrix(a) @ T                             # stage IV, no transpose
    shuffled = S.T.reshape(n)                         # S[l', k'] at l' + a k'
    y = oracle.dft1d(x, -1, "direct")
    kp, lp = np.meshgrid(np.arange(b), np.arange(a), indexing="ij")
    assert np.allclose(shuffled[(lp + a * kp).ravel()], y[(kp + b * lp).ravel()],
                       rtol=0, atol=1e-12)
    # the oracle's shuffled order is exactly this four-step output order
    assert np.allclose(shuffled, y[oracle.shuffled_positions(n, a)], rtol=0, atol=1e-12)


def test_shuffle_helpers_are_inverse_permutations():
    g = np.random.default_rng(3)
    y = g.standard_normal((8, 16, 4)) + 1j * g.standard_normal((8, 16, 4))
    for factors in [(4, 4, 2), (1, 16, 4), (2, 8, 1)]:
        s = oracle.to_shuffled(y, factors)
        assert sorted(s.reshape(-1).tolist(), key=lambda c: (c.real, c.imag)) == \
            sorted(y.reshape(-1).tolist(), key=lambda c: (c.real, c.imag))
        assert np.array_equal(oracle.from_shuffled(s, factors), y)
    # a = 1 and a = n leave the order natural
    assert np.array_equal(oracle.shuffled_positions(16, 1), np.arange(16))
    assert np.array_equal(oracle.shuffled_positions(16, 16), np.arange(16))
    # n = 8 = 4 * 2: positions 0..7 hold 0, 2, 4, 6, 1, 3, 5, 7
    assert oracle.shuffled_positions(8, 4).tolist() == [0, 2, 4, 6, 1, 3, 5, 7]


def test_circular_convolution_by_transforms():
    """The use of the shuffled order: a pointwise product between a forward
    and an inverse transform is a circular convolution whatever the order
    of the transformed entries, as long as both factors share it."""
    g = np.random.default_rng(4)
    shape = (2, 4, 4)
    x = g.standard_normal(shape) + 1j * g.standard_normal(shape)
    h = g.standard_normal(shape) + 1j * g.standard_normal(shape)
    brute = np.zeros(shape, complex)
    for i in np.ndindex(shape):
        for j in np.ndindex(shape):
            brute[i] += x[j] * h[tuple((i[d] - j[d]) % shape[d] for d in range(3))]
    f = (2, 2, 2)
    X = oracle.to_shuffled(oracle.dft3d(x, -1), f)
    H = oracle.to_shuffled(oracle.dft3d(h, -1), f)
    got = oracle.dft3d(oracle.from_shuffled(X * H, f), +1) / x.size
    assert np.allclose(got, brute, rtol=0, atol=1e-12)
