"""CPU emulation of the distributed forms the single-GPU schedules would
shard into (Section 2.4, Figs. 5, 6 and 9): p simulated processes hold
array slices, local DFTs run per process, and every redistribution is an
explicit all-to-all of blocks.  Each emulation is checked against the FP64
oracle, and the exchange volumes against the figures used for the sharding
design (one GPU's share of the data crosses the links per exchange, minus
the block it keeps)."""
import numpy as np
import pytest

import oracle


def rand(shape, seed):
    g = np.random.default_rng(seed)
    return g.standard_normal(shape) + 1j * g.standard_normal(shape)


def all_to_all(blocks):
    """blocks[src][dst] -> received[dst][src]; returns (received, elements
    that crossed between distinct processes)."""
    p = len(blocks)
    moved = sum(blocks[s][d].size for s in range(p) for d in range(p) if s != d)
    return [[blocks[s][d] for s in range(p)] for d in range(p)], moved


@pytest.mark.parametrize("shape,p", [((8, 16, 4), 2), ((16, 8, 8), 4), ((32, 16, 16), 8)])
def test_slab_on_a_1d_grid(shape, p):
    """Slab (eq. (6), Fig. 5): each process transforms its n0 / p planes in
    2D, one all-to-all makes n0 local, the depth DFT finishes; the result is
    left distributed over n1 (the final exchange is optional, Section 2.4)."""
    n0, n1, n2 = shape
    x = rand(shape, 1)
    local = [np.fft.fft2(x[r * n0 // p:(r + 1) * n0 // p], axes=(1, 2)) for r in range(p)]
    blocks = [[loc[:, d * n1 // p:(d + 1) * n1 // p, :] for d in range(p)] for loc in local]
    recv, moved = all_to_all(blocks)
    out = [np.fft.fft(np.concatenate(recv[d], axis=0), axis=0) for d in range(p)]
    y = np.concatenate(out, axis=1)
    assert oracle.rel_l2(y, oracle.dft3d(x, -1, "fft")) < 1e-13
    # each process sends (p - 1) / p of its shard
    assert moved == x.size * (p - 1) // p


@pytest.mark.parametrize("shape,py,pz", [((8, 8, 8), 2, 2), ((16, 8, 16), 2, 4)])
def test_pencil_on_a_2d_mesh_with_rotation(shape, py, pz):
    """Pencil (eq. (8), Fig. 6) on a py x pz mesh: transform the local axis,
    exchange within mesh rows, transform, exchange within mesh columns,
    transform; the data ends rotated (zxy) and a last exchange would restore
    the natural distribution."""
    n0, n1, n2 = shape
    x = rand(shape, 2)
    # process (a, b) holds x[a-th n0 block, b-th n1 block, :] (n2 local)
    A0, B1 = n0 // py, n1 // pz
    P = {(a, b): np.fft.fft(x[a * A0:(a + 1) * A0, b * B1:(b + 1) * B1, :], axis=2)
         for a in range(py) for b in range(pz)}
    # exchange within rows (fixed a): make n1 local, split n2 over pz
    C2 = n2 // pz
    Q, moved1 = {}, 0
    for a in range(py):
        blocks = [[P[(a, b)][:, :, d * C2:(d + 1) * C2] for d in range(pz)] for b in range(pz)]
        recv, m = all_to_all(blocks)
        moved1 += m
        for d in range(pz):
            Q[(a, d)] = np.fft.fft(np.concatenate(recv[d], axis=1), axis=1)
    # exchange within columns (fixed d): make n0 local, split n1 over py
    D1 = n1 // py
    R, moved2 = {}, 0
    for d in range(pz):
        blocks = [[Q[(a, d)][:, e * D1:(e + 1) * D1, :] for e in range(py)] for a in range(py)]
        recv, m = all_to_all(blocks)
        moved2 += m
        for e in range(py):
            R[(e, d)] = np.fft.fft(np.concatenate(recv[e], axis=0), axis=0)
    y = np.empty(shape, complex)
    for (e, d), blk in R.items():
        y[:, e * D1:(e + 1) * D1, d * C2:(d + 1) * C2] = blk
    assert oracle.rel_l2(y, oracle.dft3d(x, -1, "fft")) < 1e-13
    assert moved1 == x.size * (pz - 1) // pz
    assert moved2 == x.size * (py - 1) // py


@pytest.mark.parametrize("n,p", [(16, 2), (256, 4), (64, 8)])
def test_volumetric_axis_on_p_processes(n, p):
    """One axis of the volumetric form (Fig. 9, Section 3.2) on p processes
    with the elemental-cyclic distribution (process r holds x[r + p k]):
    local DFT_{n/p}, twiddle, one all-to-all, local DFT_p; the output is
    again cyclic (process r' holds y[r' + p k'] after the local reorder)."""
    x = rand((n,), 3)
    m = n // p
    w = np.exp(-2j * np.pi / n)
    loc = []
    for r in range(p):
        z = np.fft.fft(x[r::p])                       # DFT_m over k, eq. (14)
        loc.append(z * w ** (r * np.arange(m)))       # twiddle w_n^{r k'}
    # process d receives k' in its cyclic share (k' = d + p j)
    blocks = [[loc[s][d::p] for d in range(p)] for s in range(p)]
    recv, moved = all_to_all(blocks)
    y = np.empty(n, complex)
    for d in range(p):
        T = np.stack(recv[d])                         # (s, j): residue s, k' = d + p j
        Y = np.fft.fft(T, axis=0)                     # DFT_p over s -> l'
        for lp in range(p):
            for j in range(m // p):
                kp = d + p * j
                y[kp + m * lp] = Y[lp, j]
    assert oracle.rel_l2(y, oracle.dft1d(x, -1, "direct")) < 1e-13
    assert moved == n * (p - 1) // p
