"""ctypes binding of libdft3d.so (include/dft3d.h) -- argument marshalling
only.  Every step of the transform runs in the library's HIP kernels; torch
is used for device memory and the current stream.  There is no fallback: if
the library is missing, every call raises.
"""
from __future__ import annotations

import ctypes
import json
import os
from typing import Dict, List, Optional, Sequence, Tuple

_HERE = os.path.dirname(os.path.abspath(__file__))
# DFT3D_LIBRARY selects another build of the same library (the sanitizer
# build of build.py --sanitize); the default is the in-tree libdft3d.so.
LIB_PATH = os.environ.get("DFT3D_LIBRARY") or os.path.join(_HERE, "libdft3d.so")

SCHEDULES = {"auto": 0, "slab": 1, "pencil": 2, "volumetric": 3}
LAYOUTS = {"natural": 0, "shuffled": 1}
PRECISIONS = {"fp32": 0, "bf16x1": 1, "fp16x1": 2, "bf16x6": 3, "bf16x9": 4,
              "fp16x3": 5}
OPT_PRECISION, OPT_TILE, OPT_XCD_REMAP, OPT_SPLIT_MAX, OPT_NONTEMPORAL = 1, 2, 3, 4, 5
OPT_PERSISTENT, OPT_SLAB_GROUP, OPT_FUSED_PLANE, OPT_FUSED_AXES = 6, 7, 8, 9
OPT_PENCIL_GROUP, OPT_BATCH_LAUNCH, OPT_MOVE_ONLY, OPT_MFMA_LEAF = 10, 11, 12, 13
OPT_RADICES, OPT_RADER, OPT_HALVES, OPT_PENCIL_ORDER = 14, 15, 16, 17
OPT_NUM_PASSES = 100

OK = 0
ERR_INVALID_ARG = -1
ERR_UNSUPPORTED_SIZE = -2
ERR_UNSUPPORTED_SCHEDULE = -3
ERR_NO_DEVICE = -4
ERR_OUT_OF_MEMORY = -5
ERR_HIP = -6
ERR_WORKSPACE_TOO_SMALL = -7

# Every function include/dft3d.h declares.
EXPORTS = ("dft3d_status_string", "dft3d_plan", "dft3d_plan_describe",
           "dft3d_plan_set_option", "dft3d_plan_get_option",
           "dft3d_workspace_size", "dft3d_set_workspace", "dft3d_execute",
           "dft3d_execute_batched", "dft3d_autotune", "dft3d_destroy",
           "dft3d_execute_noalloc", "dft3d_batch_describe")

_lib = None


class Dft3dError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        msg = lib().dft3d_status_string(status).decode() if _lib else str(status)
        super().__init__(f"{what}: {msg} (status {status})" if what else msg)


def lib():
    """Load libdft3d.so (after torch, so that one HIP runtime serves both)."""
    global _lib
    if _lib is not None:
        return _lib
    try:  # torch ships the HIP runtime the library must share
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is not built; run `python -m paper_1904_10119_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, ci, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_size_t
    L.dft3d_status_string.argtypes = [ci]
    L.dft3d_status_string.restype = ctypes.c_char_p
    L.dft3d_plan.argtypes = [i64, i64, i64, ci, ci, ctypes.POINTER(vp)]
    L.dft3d_plan_describe.argtypes = [i64, i64, i64, ci, ci, ctypes.POINTER(ci),
                                      ctypes.POINTER(i64), ci, ctypes.c_char_p, sz,
                                      ctypes.POINTER(sz)]
    L.dft3d_plan_set_option.argtypes = [vp, ci, i64]
    L.dft3d_plan_get_option.argtypes = [vp, ci, ctypes.POINTER(i64)]
    L.dft3d_workspace_size.argtypes = [vp, ctypes.POINTER(sz)]
    L.dft3d_set_workspace.argtypes = [vp, vp, sz]
    L.dft3d_execute.argtypes = [vp, vp, vp, ci, vp]
    L.dft3d_execute_batched.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(vp),
                                        ctypes.POINTER(vp), ci, ci, vp]
    L.dft3d_autotune.argtypes = [i64, i64, i64, vp, vp, vp, ctypes.POINTER(ci),
                                 ctypes.POINTER(ctypes.c_double)]
    L.dft3d_destroy.argtypes = [vp]
    L.dft3d_execute_noalloc.argtypes = [vp, vp, vp, ci, vp]
    L.dft3d_batch_describe.argtypes = [ctypes.POINTER(i64), ci, ci, ci, ctypes.c_char_p,
                                       sz, ctypes.POINTER(sz)]
    for f in EXPORTS[1:]:
        getattr(L, f).restype = ci
    _lib = L
    return L


def _check(st: int, what: str) -> None:
    if st != OK:
        raise Dft3dError(st, what)


OPTION_KEYS = {"precision": OPT_PRECISION, "tile": OPT_TILE,
               "xcd_remap": OPT_XCD_REMAP, "split_max": OPT_SPLIT_MAX,
               "nontemporal": OPT_NONTEMPORAL, "persistent": OPT_PERSISTENT,
               "slab_group": OPT_SLAB_GROUP, "fused_plane": OPT_FUSED_PLANE,
               "fused_axes": OPT_FUSED_AXES, "pencil_group": OPT_PENCIL_GROUP,
               "batch_launch": OPT_BATCH_LAUNCH, "move_only": OPT_MOVE_ONLY,
               "mfma_leaf": OPT_MFMA_LEAF, "radices": OPT_RADICES, "rader": OPT_RADER,
               "halves": OPT_HALVES, "pencil_order": OPT_PENCIL_ORDER}


def radix_code(radices) -> int:
    """DFT3D_OPT_RADICES value of a radix sequence (first stage first), or
    the value itself if given as an int."""
    if isinstance(radices, int):
        return radices
    radices = [int(r) for r in radices]
    if len(radices) > 8 or any(not 0 < r < 256 for r in radices):
        raise ValueError(f"radix sequence {radices}: at most 8 stages of 1..255")
    code = 0
    for i, r in enumerate(radices):
        code |= r << (8 * i)
    return code


def _option_value(key, value) -> int:
    if key == "precision":
        return PRECISIONS[value]
    if key == "radices":
        return radix_code(value)
    return int(value)


def describe(shape: Sequence[int], schedule: str = "auto",
             layout: str = "natural", **opts) -> dict:
    """Pass list the library would run for `shape` (no device needed)."""
    n0, n1, n2 = (int(s) for s in shape)
    items = [(OPTION_KEYS[k], _option_value(k, v)) for k, v in opts.items()]
    keys = (ctypes.c_int * max(1, len(items)))(*[k for k, _ in items])
    vals = (ctypes.c_int64 * max(1, len(items)))(*[v for _, v in items])
    need = ctypes.c_size_t(0)
    L = lib()
    args = (n0, n1, n2, SCHEDULES[schedule], LAYOUTS[layout], keys, vals, len(items))
    _check(L.dft3d_plan_describe(*args, None, 0, ctypes.byref(need)), "describe")
    buf = ctypes.create_string_buffer(need.value)
    _check(L.dft3d_plan_describe(*args, buf, need.value, None), "describe")
    return json.loads(buf.value.decode())


BATCH_LAUNCHES = {"levels": 0, "persistent": 1}


def describe_batch(shapes, schedule: str = "auto", launch: str = "levels") -> dict:
    """Work items and launches of a batched call over `shapes` (no device)."""
    flat = [int(v) for s in shapes for v in s]
    arr = (ctypes.c_int64 * max(1, len(flat)))(*flat)
    need = ctypes.c_size_t(0)
    L = lib()
    args = (arr, len(shapes), SCHEDULES[schedule], BATCH_LAUNCHES[launch])
    _check(L.dft3d_batch_describe(*args, None, 0, ctypes.byref(need)), "batch_describe")
    buf = ctypes.create_string_buffer(need.value)
    _check(L.dft3d_batch_describe(*args, buf, need.value, None), "batch_describe")
    return json.loads(buf.value.decode())


class Plan:
    """Owns a dft3d_plan_t.  The workspace is a torch tensor on the plan's
    device, so torch's caching allocator owns that memory."""

    def __init__(self, shape: Sequence[int], schedule: str = "auto",
                 layout: str = "natural", precision: str = "fp32",
                 tile: int = 0, split_max: int = 0, xcd_remap: int = 1,
                 nontemporal: int = -1, persistent: int = -1,
                 slab_group: int = -2, fused_plane: int = -1, fused_axes: int = -1,
                 pencil_group: int = -2, batch_launch: int = -1, move_only: int = 0,
                 mfma_leaf: int = 0, radices=0, rader: int = -1, halves: int = -1,
                 pencil_order: int = -1):
        self.shape = tuple(int(s) for s in shape)
        self.schedule = schedule
        h = ctypes.c_void_p()
        L = lib()
        _check(L.dft3d_plan(*self.shape, SCHEDULES[schedule], LAYOUTS[layout],
                            ctypes.byref(h)), "dft3d_plan")
        self._h = h
        self._ws = None
        try:
            if precision != "fp32":
                self.set_option(OPT_PRECISION, PRECISIONS[precision])
            if tile:
                self.set_option(OPT_TILE, tile)
            if split_max:
                self.set_option(OPT_SPLIT_MAX, split_max)
            if xcd_remap != 1:
                self.set_option(OPT_XCD_REMAP, xcd_remap)
            if nontemporal >= 0:
                self.set_option(OPT_NONTEMPORAL, nontemporal)
            if persistent >= 0:
                self.set_option(OPT_PERSISTENT, persistent)
            if slab_group >= -1:
                self.set_option(OPT_SLAB_GROUP, slab_group)
            if fused_plane >= 0:
                self.set_option(OPT_FUSED_PLANE, fused_plane)
            if fused_axes >= 0:
                self.set_option(OPT_FUSED_AXES, fused_axes)
            if pencil_group >= -1:
                self.set_option(OPT_PENCIL_GROUP, pencil_group)
            if batch_launch >= 0:
                self.set_option(OPT_BATCH_LAUNCH, batch_launch)
            if move_only:
                self.set_option(OPT_MOVE_ONLY, move_only)
            if mfma_leaf:
                self.set_option(OPT_MFMA_LEAF, mfma_leaf)
            if radices:
                self.set_option(OPT_RADICES, radix_code(radices))
            if rader >= 0:
                self.set_option(OPT_RADER, rader)
            if halves >= 0:
                self.set_option(OPT_HALVES, halves)
            if pencil_order >= 0:
                self.set_option(OPT_PENCIL_ORDER, pencil_order)
        except Exception:
            self.close()
            raise

    @property
    def handle(self):
        return self._h

    def set_option(self, key: int, value: int) -> None:
        _check(lib().dft3d_plan_set_option(self._h, key, int(value)), "set_option")

    def get_option(self, key: int) -> int:
        v = ctypes.c_int64(0)
        _check(lib().dft3d_plan_get_option(self._h, key, ctypes.byref(v)),
               "get_option")
        return v.value

    @property
    def num_passes(self) -> int:
        return self.get_option(OPT_NUM_PASSES)

    def workspace_size(self) -> int:
        v = ctypes.c_size_t(0)
        _check(lib().dft3d_workspace_size(self._h, ctypes.byref(v)), "workspace_size")
        return v.value

    def bind_workspace(self, device) -> None:
        import torch
        need = self.workspace_size()
        if need == 0 or (self._ws is not None and self._ws.numel() >= need):
            return
        self._ws = torch.empty(need, dtype=torch.uint8, device=device)
        _check(lib().dft3d_set_workspace(self._h, self._ws.data_ptr(), need),
               "set_workspace")

    def execute(self, x, out, inverse: bool = False, stream=None) -> None:
        """x, out: contiguous complex64 CUDA tensors of the plan's shape."""
        import torch
        for t in (x, out):
            if t.dtype != torch.complex64 or not t.is_cuda or not t.is_contiguous():
                raise ValueError("expected contiguous complex64 CUDA tensors")
            if tuple(t.shape) != self.shape:
                raise ValueError(f"shape {tuple(t.shape)} != plan {self.shape}")
        self.bind_workspace(x.device)
        s = stream if stream is not None else torch.cuda.current_stream(x.device)
        _check(lib().dft3d_execute(self._h, x.data_ptr(), out.data_ptr(),
                                   1 if inverse else -1, s.cuda_stream),
               "dft3d_execute")

    def execute_noalloc(self, x, out, inverse: bool = False, stream=None) -> None:
        """As execute(), through dft3d_execute_noalloc: the workspace is the
        library's static per-device array (nothing is allocated)."""
        import torch
        for t in (x, out):
            if t.dtype != torch.complex64 or not t.is_cuda or not t.is_contiguous():
                raise ValueError("expected contiguous complex64 CUDA tensors")
            if tuple(t.shape) != self.shape:
                raise ValueError(f"shape {tuple(t.shape)} != plan {self.shape}")
        s = stream if stream is not None else torch.cuda.current_stream(x.device)
        _check(lib().dft3d_execute_noalloc(self._h, x.data_ptr(), out.data_ptr(),
                                           1 if inverse else -1, s.cuda_stream),
               "dft3d_execute_noalloc")

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().dft3d_destroy(self._h)
            self._h = ctypes.c_void_p()
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_plans: Dict[Tuple, Plan] = {}


def get_plan(shape, schedule="auto", precision="fp32", device_index=0, **opts) -> Plan:
    if "radices" in opts:
        opts["radices"] = radix_code(opts["radices"])
    key = (tuple(int(s) for s in shape), schedule, precision, device_index,
           tuple(sorted(opts.items())))
    p = _plans.get(key)
    if p is None:
        p = Plan(shape, schedule, precision=precision, **opts)
        _plans[key] = p
    return p


SCHEDULE_NAMES = {v: k for k, v in SCHEDULES.items()}


def shuffle_factors(shape) -> Tuple[int, int, int]:
    """Split factor a of every axis in the SHUFFLED layout: along an axis of
    length n = a * b, the transformed entry of natural index k' + b l' sits
    at position l' + a k'; a = 2^ceil(log2(n) / 2) for n >= 4, and axes
    shorter than 4 stay natural (a = 1)."""
    out = []
    for n in shape:
        n = int(n)
        if n < 4:
            out.append(1)
        else:
            lg = n.bit_length() - 1
            out.append(1 << ((lg + 1) // 2))
    return tuple(out)


def autotune(shape, device="cuda") -> dict:
    """Time candidate schedules for `shape` on the GPU and make the fastest
    the choice of later "auto" plans of that shape."""
    import torch
    from . import inputs
    shape = tuple(int(v) for v in shape)
    x = torch.from_numpy(inputs.uniform_c64(shape, 77)).to(device)
    out = torch.empty_like(x)
    best = ctypes.c_int(-1)
    ms = ctypes.c_double(0.0)
    _check(lib().dft3d_autotune(*shape, x.data_ptr(), out.data_ptr(),
                                torch.cuda.current_stream(x.device).cuda_stream,
                                ctypes.byref(best), ctypes.byref(ms)), "dft3d_autotune")
    for key in [k for k in _plans if k[0] == shape and k[1] == "auto"]:
        _plans.pop(key).close()
    return {"schedule": SCHEDULE_NAMES.get(best.value, str(best.value)), "ms": ms.value}


def fftn(x, schedule: str = "auto", precision: str = "fp32", inverse: bool = False,
         out=None, **opts):
    """3D DFT of a complex64 CUDA tensor of shape (n0, n1, n2); unnormalised.
    Extra keyword options go to the plan (e.g. layout="shuffled" with the
    volumetric schedule, tile=, persistent=)."""
    import torch
    if x.dim() != 3:
        raise ValueError("expected a 3D tensor")
    x = x.contiguous()
    if out is None:
        out = torch.empty_like(x)
    p = get_plan(x.shape, schedule, precision, x.device.index or 0, **opts)
    p.execute(x, out, inverse=inverse)
    return out


def ifftn(x, **kw):
    """Unnormalised inverse: ifftn(fftn(x)) == x.numel() * x."""
    return fftn(x, inverse=True, **kw)


def fftn_batched(xs: List, inverse: bool = False, outs: Optional[List] = None,
                 schedule: str = "auto", launch: str = "levels"):
    """Many 3D DFTs of possibly different shapes in one library call;
    launch="persistent" runs the whole batch as one persistent launch."""
    import torch
    n = len(xs)
    if outs is None:
        outs = [torch.empty_like(x) for x in xs]
    bl = BATCH_LAUNCHES[launch]
    plans = [get_plan(x.shape, schedule, "fp32", x.device.index or 0,
                      **({"batch_launch": bl} if bl else {})) for x in xs]
    for p, x in zip(plans, xs):
        p.bind_workspace(x.device)
    arr = ctypes.c_void_p * max(n, 1)
    hp = arr(*[p.handle.value for p in plans])
    ip = arr(*[x.data_ptr() for x in xs])
    op = arr(*[o.data_ptr() for o in outs])
    s = torch.cuda.current_stream(xs[0].device) if n else torch.cuda.current_stream()
    _check(lib().dft3d_execute_batched(hp, ip, op, n, 1 if inverse else -1,
                                       s.cuda_stream), "dft3d_execute_batched")
    return outs
