"""Seeded synthetic inputs for the 3D DFT workloads.

This module holds no DFT arithmetic: it only draws random numbers, so both
the oracle side (tests) and the HIP side (tests, bench) take their inputs from
here.  Importing it does not load the HIP library.

Recipes (each draw is reproducible from the seed alone, slab by slab, so a
2^30-point input can be produced in parallel chunks):

* ``uniform_c64(shape, seed)`` -- real and imaginary parts iid uniform on
  [-1, 1): for slab i0 a PCG64 stream seeded with SeedSequence([seed, i0])
  draws 2*n1*n2 doubles u in [0, 1) (re, im interleaved), mapped to 2u - 1
  and rounded once (round-to-nearest-even) to float32.
* ``gaussian_waves_c64(shape, seed, nwaves)`` -- real and imaginary parts iid
  N(0, 1) (same slab streams, standard normal) plus ``nwaves`` unit-amplitude
  complex exponentials exp(i(phi_j + 2 pi sum_d f_jd i_d / n_d)) with distinct
  integer frequency vectors f_j uniform on [0, n_d) and phases phi_j uniform
  on [0, 2 pi), summed in float64 then rounded once to float32.
* ``batch_shapes(count, seed, dims)`` -- ``count`` shapes with each dimension
  drawn iid uniformly from ``dims``.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np


def _slab_rng(seed: int, slab: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(
        [int(seed), int(slab)])))


def _workers() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def _fill_slabs(out: np.ndarray, seed: int, kind: str) -> None:
    """Fill out (n0, n1, n2) complex64 slab by slab."""
    n0 = out.shape[0]
    flat = out.reshape(n0, -1).view(np.float32)  # (n0, 2*n1*n2)

    def one(i0: int) -> None:
        g = _slab_rng(seed, i0)
        m = flat.shape[1]
        if kind == "uniform":
            u = g.random(m)
            flat[i0, :] = (2.0 * u - 1.0).astype(np.float32)
        else:
            flat[i0, :] = g.standard_normal(m).astype(np.float32)

    if n0 * flat.shape[1] < (1 << 22):
        for i0 in range(n0):
            one(i0)
    else:
        with ThreadPoolExecutor(_workers()) as ex:
            list(ex.map(one, range(n0)))


def uniform_c64(shape, seed: int) -> np.ndarray:
    """complex64 array of `shape` (3D, C order) with re, im iid U[-1, 1)."""
    n0, n1, n2 = (int(s) for s in shape)
    out = np.empty((n0, n1, n2), dtype=np.complex64)
    _fill_slabs(out, seed, "uniform")
    return out


def plane_wave_params(shape, seed: int, nwaves: int = 8):
    """Distinct integer frequency vectors and phases of the plane waves."""
    n0, n1, n2 = (int(s) for s in shape)
    g = np.random.Generator(np.random.PCG64(np.random.SeedSequence(
        [int(seed), 0x57A7E])))
    total = n0 * n1 * n2
    if nwaves > total:
        raise ValueError("more waves than frequencies")
    flat = g.choice(total, size=nwaves, replace=False)
    freqs = np.stack(np.unravel_index(flat, (n0, n1, n2)), axis=1)
    phases = g.random(nwaves) * 2.0 * np.pi
    return freqs.astype(np.int64), phases


def gaussian_waves_c64(shape, seed: int, nwaves: int = 8):
    """complex64 input N(0,1) + sum of `nwaves` plane waves.

    Returns (x, freqs, phases)."""
    n0, n1, n2 = (int(s) for s in shape)
    out = np.empty((n0, n1, n2), dtype=np.complex64)
    _fill_slabs(out, seed, "normal")
    freqs, phases = plane_wave_params((n0, n1, n2), seed, nwaves)
    i1 = np.arange(n1).reshape(n1, 1)
    i2 = np.arange(n2).reshape(1, n2)
    for i0 in range(n0):
        acc = out[i0].astype(np.complex128)
        for f, ph in zip(freqs, phases):
            theta = ph + 2.0 * np.pi * (
                (f[0] * i0 % n0) / n0 + (f[1] * i1 % n1) / n1
                + (f[2] * i2 % n2) / n2)
            acc += np.exp(1j * theta)
        out[i0] = acc.astype(np.complex64)
    return out, freqs, phases


def batch_shapes(count: int = 96, seed: int = 104, dims=(32, 64, 128)):
    """`count` 3D shapes, each dimension iid uniform over `dims`."""
    g = np.random.Generator(np.random.PCG64(np.random.SeedSequence(
        [int(seed), 0xBA7C])))
    d = np.asarray(dims, dtype=np.int64)
    return [tuple(int(v) for v in d[g.integers(0, d.size, size=3)])
            for _ in range(count)]
