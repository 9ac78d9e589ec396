"""ctypes binding of libstencil.so (the C ABI in include/stencil.h).

Argument marshalling only: every step of a sweep runs in the library's HIP
kernels.  PyTorch supplies device memory (tensors) and streams.  There is no
fallback: if the library is missing the import of this module fails.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libstencil.so")

STENCIL_STAR, STENCIL_BOX = 0, 1
STENCIL_PERIODIC, STENCIL_DIRICHLET = 0, 1
STENCIL_F32, STENCIL_F64 = 0, 1
STENCIL_MODE_VECTOR, STENCIL_MODE_EXACT_ORDER, STENCIL_MODE_MFMA_BF16X3 = 0, 1, 2
STENCIL_MODE_SYMMETRIC = 3
STENCIL_MODE_SEPARABLE = 4
STENCIL_OK = 0
STENCIL_E_ARG = -1
STENCIL_E_UNSUPPORTED = -2
STENCIL_E_NOMEM = -3
STENCIL_E_DEVICE = -4
STENCIL_E_STATE = -5

# Symbols include/stencil.h declares.
EXPORTS = (
    "stencil_plan_create", "stencil_fold_weights", "stencil_fold_weights_f32",
    "stencil_plan_set_mode", "stencil_plan_set_fusion", "stencil_plan_set_graph",
    "stencil_plan_set_boundary_value",
    "stencil_plan_separable",
    "stencil_plan_set_floor", "stencil_life", "stencil_life_launches",
    "stencil_plan_info",
    "stencil_profitability", "stencil_run", "stencil_run_schedule", "stencil_run_batched", "stencil_residual",
    "stencil_residual_noalloc",
    "stencil_plan_destroy", "stencil_last_error", "stencil_version",
)


class stencil_grid(ctypes.Structure):
    _fields_ = [
        ("data", ctypes.c_void_p),
        ("scratch", ctypes.c_void_p),
        ("dtype", ctypes.c_int),
        ("dim", ctypes.c_int),
        ("shape", ctypes.c_int64 * 3),
        ("stream", ctypes.c_void_p),
    ]


class stencil_batch_opts(ctypes.Structure):
    _fields_ = [
        ("autotune", ctypes.c_int),
        ("tune_cache", ctypes.c_char_p),
        ("use_graph", ctypes.c_int),
        ("max_m", ctypes.c_int),
        ("chosen_m", ctypes.POINTER(ctypes.c_int)),
        ("passes", ctypes.POINTER(ctypes.c_int)),
    ]


class StencilError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("stencil error %d: %s" % (code, msg))
        self.code = code


def _load() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            "libstencil.so is not built (%s); run __graft_entry__.build() or "
            "python paper_2103_09235_amd/build_lib.py" % LIB_PATH)
    # torch first, so the HIP runtime it loads is the one the library binds to
    try:
        import torch  # noqa: F401
    except Exception:  # pragma: no cover - torch is always present here
        pass
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    i64p = ctypes.POINTER(ctypes.c_int64)
    ip = ctypes.POINTER(ctypes.c_int)
    dp = ctypes.POINTER(ctypes.c_double)
    fp = ctypes.POINTER(ctypes.c_float)
    lib.stencil_plan_create.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, dp,
                                        ctypes.c_int, ctypes.POINTER(P)]
    lib.stencil_fold_weights.argtypes = [P, ctypes.c_int, dp, i64p]
    lib.stencil_fold_weights_f32.argtypes = [P, fp, i64p]
    lib.stencil_plan_set_mode.argtypes = [P, ctypes.c_int]
    lib.stencil_plan_set_fusion.argtypes = [P, ctypes.c_int]
    lib.stencil_plan_set_graph.argtypes = [P, ctypes.c_int]
    lib.stencil_plan_set_boundary_value.argtypes = [P, ctypes.c_double]
    lib.stencil_plan_separable.argtypes = [P, ip, ip]
    lib.stencil_plan_set_floor.argtypes = [P, P, ctypes.c_int, ctypes.c_int64]
    lib.stencil_life.argtypes = [P, P, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, P]
    lib.stencil_life_launches.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, i64p]
    lib.stencil_plan_info.argtypes = [P, ip, ip, ip, ip, ip]
    lib.stencil_profitability.argtypes = [P, ctypes.c_int, i64p, i64p]
    lib.stencil_run.argtypes = [P, ctypes.POINTER(stencil_grid), ctypes.c_int64]
    lib.stencil_run_schedule.argtypes = [P, ctypes.POINTER(stencil_grid), ctypes.c_int64, i64p, ip]
    lib.stencil_run_batched.argtypes = [ctypes.POINTER(P), ctypes.POINTER(stencil_grid),
                                        ctypes.c_int, ctypes.c_int64,
                                        ctypes.POINTER(stencil_batch_opts)]
    lib.stencil_residual.argtypes = [P, P, ctypes.c_int, ctypes.c_int64, P, dp]
    lib.stencil_residual_noalloc.argtypes = [P, P, ctypes.c_int, ctypes.c_int64, P, P]
    lib.stencil_plan_destroy.argtypes = [P]
    lib.stencil_plan_destroy.restype = None
    lib.stencil_last_error.restype = ctypes.c_char_p
    lib.stencil_version.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name not in ("stencil_plan_destroy", "stencil_last_error", "stencil_version"):
            getattr(lib, name).restype = ctypes.c_int
    return lib


lib = _load()


def _check(rc: int) -> None:
    if rc != STENCIL_OK:
        raise StencilError(rc, stencil_last_error())


def stencil_last_error() -> str:
    return lib.stencil_last_error().decode()


def stencil_version() -> str:
    return lib.stencil_version().decode()


def stencil_plan_create(dim: int, radius: int, shape: int, weights, boundary: int = STENCIL_PERIODIC):
    w = np.ascontiguousarray(weights, dtype=np.float64).ravel()
    if w.size != (2 * radius + 1) ** dim:
        raise StencilError(STENCIL_E_ARG, "weights must hold (2r+1)^dim values")
    out = ctypes.c_void_p()
    _check(lib.stencil_plan_create(dim, radius, shape,
                                   w.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                   boundary, ctypes.byref(out)))
    return out


def stencil_fold_weights(plan, m: int) -> np.ndarray:
    n = ctypes.c_int64()
    _check(lib.stencil_fold_weights(plan, m, None, ctypes.byref(n)))
    out = np.empty(n.value, dtype=np.float64)
    _check(lib.stencil_fold_weights(plan, m, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                    None))
    return out


def stencil_fold_weights_f32(plan) -> np.ndarray:
    n = ctypes.c_int64()
    _check(lib.stencil_fold_weights_f32(plan, None, ctypes.byref(n)))
    out = np.empty(n.value, dtype=np.float32)
    _check(lib.stencil_fold_weights_f32(plan, out.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                        None))
    return out


def stencil_plan_set_mode(plan, mode: int) -> None:
    _check(lib.stencil_plan_set_mode(plan, mode))


def stencil_plan_set_fusion(plan, max_steps: int) -> None:
    _check(lib.stencil_plan_set_fusion(plan, max_steps))


def stencil_plan_set_graph(plan, on: bool) -> None:
    _check(lib.stencil_plan_set_graph(plan, int(bool(on))))


def stencil_plan_set_boundary_value(plan, value: float) -> None:
    _check(lib.stencil_plan_set_boundary_value(plan, float(value)))


def stencil_plan_separable(plan):
    """(rank of the current 2D operator, whether SEPARABLE mode applies it)."""
    rank, applies = ctypes.c_int(), ctypes.c_int()
    _check(lib.stencil_plan_separable(plan, ctypes.byref(rank), ctypes.byref(applies)))
    return rank.value, bool(applies.value)


def stencil_plan_set_floor(plan, floor) -> None:
    """Attach a device tensor as the plan's floor (None removes it).  The
    caller keeps the tensor alive while the plan may run."""
    if floor is None:
        _check(lib.stencil_plan_set_floor(plan, None, 0, 0))
        return
    if not floor.is_cuda or not floor.is_contiguous():
        raise StencilError(STENCIL_E_ARG, "floor must be a contiguous device tensor")
    _check(lib.stencil_plan_set_floor(plan, floor.data_ptr(), _dtype_code(floor), floor.numel()))


def stencil_life(cells, scratch, T: int, stream=None) -> None:
    """T generations of the Game of Life on a 2D uint8 device tensor."""
    import torch
    if cells.dtype != torch.uint8 or cells.dim() != 2 or not cells.is_contiguous():
        raise StencilError(STENCIL_E_ARG, "cells must be a contiguous 2D uint8 device tensor")
    if scratch.shape != cells.shape or scratch.dtype != torch.uint8:
        raise StencilError(STENCIL_E_ARG, "scratch must match cells")
    if stream is None:
        stream = torch.cuda.current_stream(cells.device)
    st = stream.cuda_stream if hasattr(stream, "cuda_stream") else stream
    _check(lib.stencil_life(cells.data_ptr(), scratch.data_ptr(), cells.shape[0], cells.shape[1],
                            int(T), st))


def stencil_life_launches(ny: int, nx: int, T: int) -> int:
    out = ctypes.c_int64()
    _check(lib.stencil_life_launches(ny, nx, T, ctypes.byref(out)))
    return out.value


def stencil_plan_info(plan) -> dict:
    v = [ctypes.c_int() for _ in range(5)]
    _check(lib.stencil_plan_info(plan, *[ctypes.byref(x) for x in v]))
    return dict(zip(("dim", "radius", "m", "folded_radius", "mode"), [x.value for x in v]))


def stencil_profitability(plan, m: int):
    a, b = ctypes.c_int64(), ctypes.c_int64()
    _check(lib.stencil_profitability(plan, m, ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def _dtype_code(t) -> int:
    import torch
    if t.dtype == torch.float32:
        return STENCIL_F32
    if t.dtype == torch.float64:
        return STENCIL_F64
    raise StencilError(STENCIL_E_ARG, "grid tensors must be float32 or float64")


def make_grid(data, scratch=None, stream=None) -> stencil_grid:
    """A stencil_grid describing a contiguous CUDA(HIP) tensor."""
    import torch
    if not data.is_cuda or not data.is_contiguous():
        raise StencilError(STENCIL_E_ARG, "data must be a contiguous device tensor")
    if scratch is not None and (scratch.shape != data.shape or scratch.dtype != data.dtype
                                or not scratch.is_contiguous()):
        raise StencilError(STENCIL_E_ARG, "scratch must match data")
    g = stencil_grid()
    g.data = data.data_ptr()
    g.scratch = scratch.data_ptr() if scratch is not None else None
    g.dtype = _dtype_code(data)
    g.dim = data.dim()
    for i, n in enumerate(data.shape):
        g.shape[i] = n
    if stream is None:
        stream = torch.cuda.current_stream(data.device)
    g.stream = stream.cuda_stream if hasattr(stream, "cuda_stream") else stream
    return g


def stencil_run(plan, data, T: int, scratch=None, stream=None) -> None:
    g = make_grid(data, scratch, stream)
    _check(lib.stencil_run(plan, ctypes.byref(g), int(T)))


def stencil_run_schedule(plan, shape, dtype: int, T: int, data_ptr: int,
                         scratch_ptr: int | None = None) -> dict:
    """Launch plan of a run on a grid of this shape and dtype whose buffers
    sit at these device addresses (compared only, never dereferenced)."""
    g = stencil_grid()
    g.data = data_ptr
    g.scratch = scratch_ptr
    g.dtype = dtype
    g.dim = len(shape)
    for i, n in enumerate(shape):
        g.shape[i] = int(n)
    out = (ctypes.c_int64 * 4)()
    copy = ctypes.c_int()
    _check(lib.stencil_run_schedule(plan, ctypes.byref(g), int(T),
                                    ctypes.cast(out, ctypes.POINTER(ctypes.c_int64)),
                                    ctypes.byref(copy)))
    return {"folded_apps": out[0], "folded_launches": out[1], "plain_apps": out[2],
            "plain_launches": out[3], "final_copy": bool(copy.value)}


class BatchedRun:
    """The arguments of stencil_run_batched marshalled once (plan handles,
    grid descriptors of the data and scratch tensors, stream) for repeated
    runs of one batch; the tensors are kept alive with it."""

    def __init__(self, plans, datas, scratches, stream=None):
        self.count = len(datas)
        self._tensors = (list(datas), list(scratches))
        self.parr = (ctypes.c_void_p * self.count)(
            *[p.value if isinstance(p, ctypes.c_void_p) else p for p in plans])
        self.garr = (stencil_grid * self.count)(
            *[make_grid(d, s, stream) for d, s in zip(datas, scratches)])
        self.chosen = (ctypes.c_int * self.count)()
        self.passes = (ctypes.c_int * self.count)()

    def run(self, T: int, autotune: bool = False, tune_cache: str | None = None,
            use_graph: bool = True, max_m: int = 1):
        """Advance every grid by T steps; returns the fold depth used per grid."""
        opts = stencil_batch_opts()
        opts.autotune = int(autotune)
        opts.tune_cache = tune_cache.encode() if tune_cache else None
        opts.use_graph = int(use_graph)
        opts.max_m = int(max_m)
        opts.chosen_m = ctypes.cast(self.chosen, ctypes.POINTER(ctypes.c_int))
        opts.passes = ctypes.cast(self.passes, ctypes.POINTER(ctypes.c_int))
        _check(lib.stencil_run_batched(self.parr, self.garr, self.count, int(T), ctypes.byref(opts)))
        return list(self.chosen)


def stencil_run_batched(plans, datas, scratches, T: int, autotune: bool = False,
                        tune_cache: str | None = None, use_graph: bool = True,
                        max_m: int = 1, stream=None, return_passes: bool = False):
    """Advance every grid by T steps; returns the fold depth used per grid
    (and, with return_passes, the launches that read and write each grid)."""
    br = BatchedRun(plans, datas, scratches, stream)
    chosen = br.run(T, autotune=autotune, tune_cache=tune_cache, use_graph=use_graph, max_m=max_m)
    if return_passes:
        return chosen, list(br.passes)
    return chosen


def stencil_residual(u, ref=None, stream=None):
    """(sum u, sum |u - ref|, max |u - ref|) in FP64 on the GPU."""
    import torch
    if ref is not None and (ref.shape != u.shape or ref.dtype != u.dtype):
        raise StencilError(STENCIL_E_ARG, "ref must match u")
    out = (ctypes.c_double * 3)()
    if stream is None:
        stream = torch.cuda.current_stream(u.device)
    s = stream.cuda_stream if hasattr(stream, "cuda_stream") else stream
    _check(lib.stencil_residual(u.data_ptr(), ref.data_ptr() if ref is not None else None,
                                _dtype_code(u), u.numel(), s, out))
    return out[0], out[1], out[2]


def stencil_residual_noalloc(u, out, ref=None, stream=None) -> None:
    """Enqueue (sum u, sum |u - ref|, max |u - ref|) into the device tensor
    out (3 float64) without any allocation by the library."""
    import torch
    if ref is not None and (ref.shape != u.shape or ref.dtype != u.dtype):
        raise StencilError(STENCIL_E_ARG, "ref must match u")
    if out.dtype != torch.float64 or out.numel() < 3 or not out.is_contiguous():
        raise StencilError(STENCIL_E_ARG, "out must be a contiguous float64 tensor of 3 values")
    if stream is None:
        stream = torch.cuda.current_stream(u.device)
    s = stream.cuda_stream if hasattr(stream, "cuda_stream") else stream
    _check(lib.stencil_residual_noalloc(u.data_ptr(), ref.data_ptr() if ref is not None else None,
                                        _dtype_code(u), u.numel(), s, out.data_ptr()))


def stencil_plan_destroy(plan) -> None:
    lib.stencil_plan_destroy(plan)


class Plan:
    """Owning wrapper of a stencil_plan."""

    def __init__(self, weights, shape: int = STENCIL_BOX, boundary: int = STENCIL_PERIODIC):
        w = np.asarray(weights, dtype=np.float64)
        self.dim = w.ndim
        self.radius = (w.shape[0] - 1) // 2
        self.handle = stencil_plan_create(self.dim, self.radius, shape, w, boundary)

    def fold(self, m: int) -> np.ndarray:
        W = stencil_fold_weights(self.handle, m)
        side = 2 * m * self.radius + 1
        return W.reshape((side,) * self.dim)

    def weights_f32(self) -> np.ndarray:
        W = stencil_fold_weights_f32(self.handle)
        side = round(W.size ** (1.0 / self.dim))
        while side ** self.dim < W.size:
            side += 1
        return W.reshape((side,) * self.dim)

    def set_mode(self, mode: int) -> None:
        stencil_plan_set_mode(self.handle, mode)

    def set_fusion(self, max_steps: int) -> None:
        stencil_plan_set_fusion(self.handle, max_steps)

    def set_graph(self, on: bool) -> None:
        stencil_plan_set_graph(self.handle, on)

    def set_boundary_value(self, value: float) -> None:
        stencil_plan_set_boundary_value(self.handle, value)

    def separable(self):
        return stencil_plan_separable(self.handle)

    def set_floor(self, floor) -> None:
        stencil_plan_set_floor(self.handle, floor)
        self._floor = floor  # keeps the tensor alive with the plan

    def info(self) -> dict:
        return stencil_plan_info(self.handle)

    def profitability(self, m: int):
        return stencil_profitability(self.handle, m)

    def run(self, data, T: int, scratch=None, stream=None) -> None:
        stencil_run(self.handle, data, T, scratch, stream)

    def schedule(self, data, T: int, scratch=None) -> dict:
        """stencil_run_schedule for a device tensor (and scratch tensor)."""
        return stencil_run_schedule(self.handle, tuple(data.shape), _dtype_code(data), T,
                                    data.data_ptr(),
                                    scratch.data_ptr() if scratch is not None else None)

    def close(self) -> None:
        if self.handle is not None:
            stencil_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
