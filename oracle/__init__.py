"""FP64 CPU oracle for the 3D complex DFT -- test infrastructure only.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the HIP
library in ``paper_1904_10119_amd/`` and never imports it.

Two independent FP64 methods (C, OpenMP), see ``oracle.h``:

* ``dft3d(x, sign, method="direct")`` -- O1, the 1D DFT of Section 2.1
  eqs. (1)-(2) as a direct matrix-vector sum, along every axis (Section 2.3).
* ``dft3d(x, sign, method="fft")`` -- O2, recursive radix-2 Cooley-Tukey
  (eq. (3) with n = 2 * n/2), along every axis.

Forward is ``sign=-1`` (w_n = exp(-2 pi i / n)); inverse ``sign=+1`` is
unnormalised, so ``dft3d(dft3d(x, -1), +1) == N * x``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SOURCES = ("dft_direct.c", "fft_radix2.c")
_lib = None


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (-O2, OpenMP).  Returns the path."""
    if not force and os.path.exists(_LIB_PATH):
        return _LIB_PATH
    srcs = [os.path.join(_HERE, s) for s in _SOURCES]
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared",
           "-Wall", "-Wextra", "-o", tmp] + srcs + ["-lm"]
    subprocess.run(cmd, check=True, cwd=_HERE)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    dp = ctypes.POINTER(ctypes.c_double)
    fp = ctypes.POINTER(ctypes.c_float)
    i64p = ctypes.POINTER(ctypes.c_int64)
    i64 = ctypes.c_int64
    ci = ctypes.c_int
    lib.oracle_dft1d_direct.argtypes = [dp, dp, i64, ci]
    lib.oracle_dft3d_direct.argtypes = [dp, dp, i64, i64, i64, ci]
    lib.oracle_dft3d_sample_pencils.argtypes = [fp, i64, i64, i64, ci, i64p,
                                                i64p, i64, dp]
    lib.oracle_fft1d_radix2.argtypes = [dp, dp, i64, ci]
    lib.oracle_fft3d_radix2.argtypes = [dp, dp, i64, i64, i64, ci]
    lib.oracle_fft_pencils_radix2.argtypes = [fp, i64, i64, i64, ci, ci, i64,
                                              i64, dp]
    lib.oracle_num_threads.argtypes = []
    lib.oracle_set_num_threads.argtypes = [ci]
    lib.oracle_set_num_threads.restype = None
    for f in ("oracle_dft1d_direct", "oracle_dft3d_direct",
              "oracle_dft3d_sample_pencils", "oracle_fft1d_radix2",
              "oracle_fft3d_radix2", "oracle_fft_pencils_radix2",
              "oracle_num_threads"):
        getattr(lib, f).restype = ctypes.c_int
    _lib = lib
    return lib


class OracleError(RuntimeError):
    pass


def _check(rc: int, what: str) -> None:
    if rc != 0:
        raise OracleError(f"{what} failed with status {rc}")


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _fptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def _as_c128(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x), dtype=np.complex128)


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def set_num_threads(n: int) -> None:
    """Threads the oracle uses from now on (timing on one core)."""
    _load().oracle_set_num_threads(int(n))


def dft1d(x, sign: int = -1, method: str = "direct") -> np.ndarray:
    """1D DFT of a vector (O1 direct sum or O2 radix-2)."""
    xv = _as_c128(x).reshape(-1)
    y = np.empty_like(xv)
    lib = _load()
    if method == "direct":
        _check(lib.oracle_dft1d_direct(_dptr(xv), _dptr(y), xv.size, sign),
               "oracle_dft1d_direct")
    elif method == "fft":
        _check(lib.oracle_fft1d_radix2(_dptr(xv), _dptr(y), xv.size, sign),
               "oracle_fft1d_radix2")
    else:
        raise ValueError(method)
    return y


def dft3d(x, sign: int = -1, method: str = "direct") -> np.ndarray:
    """3D DFT of a (n0, n1, n2) array in FP64 (C order, n2 contiguous)."""
    xa = _as_c128(x)
    if xa.ndim != 3:
        raise ValueError("expected a 3D array")
    n0, n1, n2 = xa.shape
    y = np.empty_like(xa)
    lib = _load()
    if method == "direct":
        _check(lib.oracle_dft3d_direct(_dptr(xa), _dptr(y), n0, n1, n2, sign),
               "oracle_dft3d_direct")
    elif method == "fft":
        _check(lib.oracle_fft3d_radix2(_dptr(xa), _dptr(y), n0, n1, n2, sign),
               "oracle_fft3d_radix2")
    else:
        raise ValueError(method)
    return y


def dft3d_fft_c64(x_c64: np.ndarray, sign: int = -1) -> np.ndarray:
    """O2 (recursive radix-2, FP64) of a complex64 (n0, n1, n2) array,
    widened exactly to complex128 and transformed in place: the same result
    as ``dft3d(x, sign, "fft")`` with one FP64 array instead of two (for
    2^30-point inputs)."""
    xa = np.asarray(x_c64)
    if xa.ndim != 3:
        raise ValueError("expected a 3D array")
    n0, n1, n2 = xa.shape
    y = np.empty(xa.shape, dtype=np.complex128)
    for i in range(0, n0, 16):  # widen slab by slab (no second full copy)
        y[i:i + 16] = xa[i:i + 16]
    _check(_load().oracle_fft3d_radix2(_dptr(y), _dptr(y), n0, n1, n2, sign),
           "oracle_fft3d_radix2")
    return y


def compare(a, ref, planes: int = 16, where: bool = False):
    """Errors of ``a`` against the FP64 ``ref`` over every element, taken
    slab by slab (no full-size temporaries): ``(rel_l2, max_rel)`` with
    rel_l2 = ||a - ref||_2 / ||ref||_2 and max_rel = max |a - ref| / rms(ref),
    the largest single-element error relative to the root mean square of the
    reference; with ``where`` also the index tuple of that element."""
    a = np.asarray(a)
    r = np.asarray(ref)
    if a.shape != r.shape:
        raise ValueError(f"shapes differ: {a.shape} vs {r.shape}")
    num = 0.0
    den = 0.0
    worst = 0.0
    at = (0,) * a.ndim
    for i in range(0, a.shape[0], planes):
        d = a[i:i + planes].astype(np.complex128) - r[i:i + planes]
        e2 = d.real * d.real + d.imag * d.imag
        num += float(e2.sum())
        if e2.size and float(e2.max()) > worst:
            worst = float(e2.max())
            loc = np.unravel_index(int(np.argmax(e2)), e2.shape)
            at = (i + int(loc[0]),) + tuple(int(v) for v in loc[1:])
        rr = r[i:i + planes]
        den += float((rr.real * rr.real + rr.imag * rr.imag).sum())
    rms = np.sqrt(den / max(1, a.size))
    rel = np.sqrt(num / den) if den > 0 else np.sqrt(num)
    wr = float(np.sqrt(worst) / rms) if rms > 0 else float(np.sqrt(worst))
    return (float(rel), wr, at) if where else (float(rel), wr)


def sample_pencils(x_c64: np.ndarray, k0, k1, sign: int = -1) -> np.ndarray:
    """Output pencils y[k0[s], k1[s], :] straight from the definition.

    ``x_c64`` is the complex64 input of shape (n0, n1, n2); the result is
    complex128 of shape (len(k0), n2)."""
    xa = np.ascontiguousarray(x_c64, dtype=np.complex64)
    n0, n1, n2 = xa.shape
    k0a = np.ascontiguousarray(k0, dtype=np.int64)
    k1a = np.ascontiguousarray(k1, dtype=np.int64)
    if k0a.shape != k1a.shape:
        raise ValueError("k0 and k1 must have the same length")
    out = np.empty((k0a.size, n2), dtype=np.complex128)
    _check(_load().oracle_dft3d_sample_pencils(
        _fptr(xa.view(np.float32)), n0, n1, n2, sign,
        k0a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
        k1a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), k0a.size,
        _dptr(out)), "oracle_dft3d_sample_pencils")
    return out


def fft_pencils(x_c64: np.ndarray, axis: int, first: int, count: int,
                sign: int = -1) -> np.ndarray:
    """O2 on ``count`` pencils along ``axis`` of a complex64 (n0,n1,n2)
    array, starting at pencil ``first`` (C order over the other two axes)."""
    xa = np.ascontiguousarray(x_c64, dtype=np.complex64)
    n0, n1, n2 = xa.shape
    n = (n0, n1, n2)[axis]
    out = np.empty((count, n), dtype=np.complex128)
    _check(_load().oracle_fft_pencils_radix2(
        _fptr(xa.view(np.float32)), n0, n1, n2, axis, sign, first, count,
        _dptr(out)), "oracle_fft_pencils_radix2")
    return out


def shuffled_positions(n: int, a: int) -> np.ndarray:
    """Natural index held at each position of the shuffled order of a
    length-n axis split n = a * b (Section 2.4; eq. (3) without its final
    transposition, as in Section 3.2): natural entry y[k' + b l'] (k' < b,
    l' < a) sits at position l' + a k'.  a = 1 or a = n is natural order."""
    if n % a:
        raise ValueError("a must divide n")
    b = n // a
    pos = np.arange(n, dtype=np.int64)
    lp, kp = pos % a, pos // a
    return kp + b * lp


def to_shuffled(y, factors) -> np.ndarray:
    """Rearrange a natural-order 3D array into the shuffled order with the
    per-axis split factors ``factors`` = (a0, a1, a2)."""
    y = np.asarray(y)
    for axis, a in enumerate(factors):
        idx = shuffled_positions(y.shape[axis], int(a))
        y = np.take(y, idx, axis=axis)
    return y


def from_shuffled(s, factors) -> np.ndarray:
    """Inverse of ``to_shuffled``."""
    s = np.asarray(s)
    for axis, a in enumerate(factors):
        idx = shuffled_positions(s.shape[axis], int(a))
        inv = np.empty_like(idx)
        inv[idx] = np.arange(idx.size)
        s = np.take(s, inv, axis=axis)
    return s


def rel_l2(a, ref) -> float:
    """||a - ref||_2 / ||ref||_2 over all complex entries, in FP64."""
    a = np.asarray(a).astype(np.complex128, copy=False).reshape(-1)
    r = np.asarray(ref).astype(np.complex128, copy=False).reshape(-1)
    den = np.linalg.norm(r)
    return float(np.linalg.norm(a - r) / den) if den > 0 else float(
        np.linalg.norm(a - r))


def tol(n_total: int) -> float:
    """Pass bar for an FP32 transform of N points: 1e-6 at 64^3 (N = 2^18),
    growing linearly in log2 N (1e-6 * log2(N) / 18)."""
    return 1e-6 * np.log2(max(int(n_total), 2)) / 18.0


def time_fft_pencils(x_c64: np.ndarray, axis: int, count: int,
                     sign: int = -1):
    """Wall-clock seconds of O2 on ``count`` pencils along ``axis``."""
    t0 = time.perf_counter()
    fft_pencils(x_c64, axis, 0, count, sign)
    return time.perf_counter() - t0
