"""MI355X (gfx950) Ahmad-Cohen regular force: Python binding of libnbreg.

Thin ctypes marshalling over the C ABI declared in ``include/nbreg.h``: every
step of the computation runs in the library's HIP kernels; PyTorch only
provides device memory and the stream.  If the library is missing this module
raises on first use -- there is no CPU fallback.

Arrays follow the ABI's structure-of-arrays layout: positions/velocities are
float64 tensors of shape (3, n) on the GPU, per-row outputs (3, n_i).

Physics: Wang et al. 2015 (NBODY6++GPU), section 2 (Ahmad-Cohen split of the
force into a regular part from bodies outside the neighbour radius and an
irregular part from neighbours), section 3.2.1 (regular force, its derivative
and the neighbour lists on the GPU in one pass) and section 3.3.3 (all-body
prediction for the regular force).
"""
from __future__ import annotations

import ctypes as C
import os
import threading

import torch

__all__ = [
    "NbError", "Context", "lib", "library_path", "context", "predict", "regular_force",
    "regular_force_adjoint", "regular_force_batched", "autotune", "autotune_batched",
    "regular_force_noalloc", "fixed_workspace_bytes", "RegularForce",
    "irregular_force", "hermite_correct", "potential", "sched_build", "sched_update",
    "sched_next", "radius_update", "regular_force_fit", "FP64", "MIXED", "STATUS_OVERFLOW", "STATUS_BAD_INDEX",
    "STATUS_NONFINITE", "STATUS_BAD_LEVEL",
]

FP64, MIXED = 0, 1
STATUS_OVERFLOW, STATUS_BAD_INDEX, STATUS_NONFINITE, STATUS_BAD_LEVEL = 1, 2, 4, 8
(CLASS_FORCE, CLASS_MERGE, CLASS_PREDICT, CLASS_ADJOINT, CLASS_BATCHED, CLASS_REDO,
 CLASS_STEP, CLASS_SCHED, CLASS_RADIUS) = range(9)

_HERE = os.path.dirname(os.path.abspath(__file__))
# NBREG_LIBRARY may point at another build of the same library (e.g. a
# variant built for a comparison); the default is the in-tree build.
_LIB_PATH = os.environ.get("NBREG_LIBRARY") or os.path.join(_HERE, "libnbreg.so")
_lib = None
_lock = threading.Lock()


class NbError(RuntimeError):
    """A negative return code from libnbreg."""

    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__(f"{what}: {lib().nb_error_string(code).decode()} ({code})")


def library_path() -> str:
    return _LIB_PATH


def lib() -> C.CDLL:
    """Loads libnbreg.so (built by ``python -m paper_1504_03687_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(_LIB_PATH):
            raise ImportError(f"libnbreg.so not found at {_LIB_PATH}; build it with "
                              "`python -m paper_1504_03687_amd.build`")
        L = C.CDLL(_LIB_PATH)
        vp, i64, i32, dbl, u32p = C.c_void_p, C.c_int64, C.c_int32, C.c_double, C.c_void_p
        sig = {
            "nb_version": ([], C.c_int),
            "nb_error_string": ([C.c_int], C.c_char_p),
            "nb_ctx_create": ([C.POINTER(vp), C.c_int, vp], C.c_int),
            "nb_ctx_set_stream": ([vp, vp], C.c_int),
            "nb_ctx_destroy": ([vp], C.c_int),
            "nb_ctx_set_plan": ([vp, C.c_int, C.c_int, C.c_int], C.c_int),
            "nb_ctx_last_plan": ([vp, C.c_char_p, C.c_int], C.c_int),
            "nb_ctx_set_scratch_limit": ([vp, i64], C.c_int),
            "nb_ctx_enable_timing": ([vp, C.c_int], C.c_int),
            "nb_ctx_kernel_time": ([vp, C.c_int, C.POINTER(dbl), C.POINTER(i64)], C.c_int),
            "nb_ctx_reset_timing": ([vp], C.c_int),
            "nb_ctx_set_mixed_tolerance": ([vp, dbl, dbl], C.c_int),
            "nb_ctx_set_refine_buffer_rows": ([vp, C.c_int32], C.c_int),
            "nb_ctx_last_refined_rows": ([vp, C.POINTER(i32)], C.c_int),
            "nb_predict": ([vp, i64, dbl, vp, vp, vp, vp, vp, vp, vp, vp, vp], C.c_int),
            "nb_regular_force": ([vp, i64, vp, vp, vp, i32, vp, vp, i32, C.c_int, vp, vp, vp,
                                  vp, vp, u32p], C.c_int),
            "nb_regular_force_noalloc": ([vp, i64, vp, vp, vp, i32, vp, vp, i32, C.c_int, vp,
                                          vp, vp, vp, vp, u32p], C.c_int),
            "nb_fixed_workspace_bytes": ([C.POINTER(i64)], C.c_int),
            "nb_regular_force_adjoint": ([vp, i64, vp, vp, vp, i32, vp, vp, vp, vp, vp, vp, vp,
                                          u32p], C.c_int),
            "nb_regular_force_batched": ([vp, i32, vp, vp, vp, vp, vp, vp, vp, i32, C.c_int, vp,
                                          vp, vp, vp, vp, u32p], C.c_int),
            "nb_autotune": ([vp, i64, C.c_char_p, C.c_int], C.c_int),
            "nb_ctx_set_batched_shape": ([vp, C.c_int, C.c_int, C.c_int, C.c_int], C.c_int),
            "nb_autotune_batched": ([vp, i32, vp, vp, vp, vp, vp, vp, vp, i32, C.c_int, vp, vp,
                                     vp, vp, vp, u32p, C.c_char_p, C.c_int], C.c_int),
            "nb_irregular_force": ([vp, i64, vp, vp, vp, i32, vp, i32, vp, vp, vp, vp, u32p],
                                   C.c_int),
            "nb_hermite_correct": ([vp, i64] + [vp] * 11, C.c_int),
            "nb_potential": ([vp, i64, vp, vp, vp, vp], C.c_int),
            "nb_sched_build": ([vp, i64, vp, i32, vp, vp, u32p], C.c_int),
            "nb_sched_update": ([vp, i64, i32, i32, vp, i32, vp, vp, u32p], C.c_int),
            "nb_sched_next": ([dbl, i32, vp, C.POINTER(dbl), C.POINTER(i32),
                               C.POINTER(i32)], C.c_int),
            "nb_radius_update": ([vp, i32, vp, vp, i32, dbl, dbl, vp], C.c_int),
            "nb_regular_force_fit": ([vp, i64, vp, vp, vp, i32, vp, vp, i32, C.c_int, i32, i32,
                                      vp, vp, vp, vp, vp, u32p, C.POINTER(i32)], C.c_int),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
        return _lib


def _check(rc: int, what: str):
    if rc != 0:
        raise NbError(rc, what)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _dev(t, name, dtype, shape=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return t


def _force_outputs(out, n_i: int, nb_cap: int, device):
    """The five output tensors of a regular-force call: new ones, or the
    caller's (acc, jerk, nb_count, nb_list, overflow), each checked for
    device, dtype, shape and contiguity before any pointer reaches the
    library (an undersized list would be written past its end)."""
    if nb_cap < 0:
        raise ValueError("nb_cap must be >= 0")
    shapes = (("acc", torch.float64, (3, n_i)), ("jerk", torch.float64, (3, n_i)),
              ("nb_count", torch.int32, (n_i,)), ("nb_list", torch.int32, (n_i, nb_cap)),
              ("overflow", torch.int32, (1,)))
    if out is None:
        return tuple(torch.empty(shape, dtype=dt, device=device) for _, dt, shape in shapes)
    if not isinstance(out, (tuple, list)) or len(out) != 5:
        raise ValueError("out must be (acc, jerk, nb_count, nb_list, overflow)")
    for t, (name, dt, shape) in zip(out, shapes):
        _dev(t, f"out {name}", dt, shape)
        if t.device != device:
            raise ValueError(f"out {name} is on {t.device}, the inputs on {device}")
    return tuple(out)


class Context:
    """One libnbreg context on one device.  Calls launch on torch's current
    stream of that device at the time of the call."""

    def __init__(self, device: int | None = None):
        L = lib()
        if device is None:
            device = torch.cuda.current_device()
        self.device = int(device)
        h = C.c_void_p()
        stream = torch.cuda.current_stream(self.device).cuda_stream
        _check(L.nb_ctx_create(C.byref(h), self.device, C.c_void_p(stream)), "nb_ctx_create")
        self._h = h

    @property
    def handle(self):
        return self._h

    def _bind_stream(self):
        s = torch.cuda.current_stream(self.device).cuda_stream
        _check(lib().nb_ctx_set_stream(self._h, C.c_void_p(s)), "nb_ctx_set_stream")

    def set_plan(self, mapping: int = 0, rows_per_lane: int = 0, splits: int = 0):
        _check(lib().nb_ctx_set_plan(self._h, mapping, rows_per_lane, splits), "nb_ctx_set_plan")

    def set_batched_shape(self, tile: int = 0, lanes: int = 0, rows_per_lane: int = 0,
                          items_per_cu: int = 0):
        """Forces the batched kernel shape (all zero: automatic)."""
        _check(lib().nb_ctx_set_batched_shape(self._h, tile, lanes, rows_per_lane, items_per_cu),
               "nb_ctx_set_batched_shape")

    def last_plan(self) -> str:
        buf = C.create_string_buffer(256)
        _check(lib().nb_ctx_last_plan(self._h, buf, 256), "nb_ctx_last_plan")
        return buf.value.decode()

    def set_scratch_limit(self, nbytes: int):
        _check(lib().nb_ctx_set_scratch_limit(self._h, int(nbytes)), "nb_ctx_set_scratch_limit")

    def enable_timing(self, on: bool = True):
        _check(lib().nb_ctx_enable_timing(self._h, int(bool(on))), "nb_ctx_enable_timing")

    def kernel_time(self, cls: int):
        ms = C.c_double()
        n = C.c_int64()
        _check(lib().nb_ctx_kernel_time(self._h, cls, C.byref(ms), C.byref(n)),
               "nb_ctx_kernel_time")
        return ms.value, n.value

    def reset_timing(self):
        _check(lib().nb_ctx_reset_timing(self._h), "nb_ctx_reset_timing")

    def set_mixed_tolerance(self, tol: float = 5e-6, safety: float = 32.0):
        """Target per-row relative error of NB_MIXED and the safety factor of
        its rounding-error estimate; rows above it are recomputed in FP64
        (tol = 0: never)."""
        _check(lib().nb_ctx_set_mixed_tolerance(self._h, float(tol), float(safety)),
               "nb_ctx_set_mixed_tolerance")

    def set_refine_buffer_rows(self, rows: int = 0):
        """Test override: at most `rows` refined rows of a single-block call
        keep chunk partials; the rest are refined one work-group per row, to
        the same bits (0 = automatic)."""
        _check(lib().nb_ctx_set_refine_buffer_rows(self._h, int(rows)),
               "nb_ctx_set_refine_buffer_rows")

    def last_refined_rows(self) -> int:
        """Rows the last mixed call recomputed in FP64 (synchronises)."""
        k = C.c_int32()
        _check(lib().nb_ctx_last_refined_rows(self._h, C.byref(k)), "nb_ctx_last_refined_rows")
        return k.value

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().nb_ctx_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_ctxs: dict[int, Context] = {}


def context(device: int | None = None) -> Context:
    """The shared per-device context used by the module-level functions."""
    if device is None:
        device = torch.cuda.current_device()
    ctx = _ctxs.get(device)
    if ctx is None:
        ctx = _ctxs[device] = Context(device)
    return ctx


def _prec(precision) -> int:
    if precision in (FP64, "fp64", "f64", "double"):
        return FP64
    if precision in (MIXED, "mixed", "fp32", "mp"):
        return MIXED
    raise ValueError(f"unknown precision {precision!r}")


def predict(x, v, a, jk, t0, t: float, m=None, out=None, ctx: Context | None = None):
    """Hermite predictor of all bodies to time t (FP64).  Returns (xp, vp, m32);
    m32 is None unless m is given."""
    n = t0.shape[0] if isinstance(t0, torch.Tensor) else 0
    for name, arr in (("x", x), ("v", v), ("a", a), ("jk", jk)):
        _dev(arr, name, torch.float64, (3, n))
    _dev(t0, "t0", torch.float64, (n,))
    ctx = ctx or context(x.device.index)
    if out is None:
        xp = torch.empty_like(x)
        vp = torch.empty_like(v)
    else:
        xp, vp = out
        _dev(xp, "xp", torch.float64, (3, n))
        _dev(vp, "vp", torch.float64, (3, n))
    m32 = None
    if m is not None:
        _dev(m, "m", torch.float64, (n,))
        m32 = torch.empty(n, dtype=torch.float32, device=x.device)
    ctx._bind_stream()
    _check(lib().nb_predict(ctx.handle, n, float(t), _ptr(x), _ptr(v), _ptr(a), _ptr(jk),
                            _ptr(t0), _ptr(m), _ptr(xp), _ptr(vp), _ptr(m32)), "nb_predict")
    return xp, vp, m32


def _regular_force_call(fn: str, xp, vp, m, i_block, rs2, nb_cap: int, precision, status,
                        out, ctx):
    n = m.shape[0]
    _dev(xp, "xp", torch.float64, (3, n))
    _dev(vp, "vp", torch.float64, (3, n))
    _dev(m, "m", torch.float64, (n,))
    n_i = i_block.shape[0]
    _dev(i_block, "i_block", torch.int32, (n_i,))
    _dev(rs2, "rs2", torch.float64, (n_i,))
    if nb_cap < 0:
        raise ValueError("nb_cap must be >= 0")
    dev = xp.device
    acc, jerk, cnt, lst, ovf = _force_outputs(out, n_i, nb_cap, dev)
    if status is not None:
        _dev(status, "status", torch.int32, (1,))
    ctx = ctx or context(dev.index)
    ctx._bind_stream()
    _check(getattr(lib(), fn)(ctx.handle, n, _ptr(xp), _ptr(vp), _ptr(m), n_i,
                              _ptr(i_block), _ptr(rs2), int(nb_cap), _prec(precision),
                              _ptr(acc), _ptr(jerk), _ptr(cnt),
                              _ptr(lst) if nb_cap > 0 else None, _ptr(ovf), _ptr(status)),
           fn)
    return acc, jerk, cnt, lst, ovf


def regular_force(xp, vp, m, i_block, rs2, nb_cap: int, precision="fp64", status=None,
                  out=None, ctx: Context | None = None):
    """Regular acc, jerk (3, n_i) float64, nb_count (n_i,) int32, nb_list
    (n_i, nb_cap) int32 and overflow (1,) int32 -- all on the GPU, no sync."""
    return _regular_force_call("nb_regular_force", xp, vp, m, i_block, rs2, nb_cap, precision,
                               status, out, ctx)


def regular_force_noalloc(xp, vp, m, i_block, rs2, nb_cap: int, precision, out,
                          status=None, ctx: Context | None = None):
    """nb_regular_force_noalloc: as regular_force, into the caller's `out`
    tensors (required, so nothing is allocated), with the library's fixed
    device workspace instead of context scratch."""
    if out is None:
        raise ValueError("regular_force_noalloc writes into the caller's out tensors")
    return _regular_force_call("nb_regular_force_noalloc", xp, vp, m, i_block, rs2, nb_cap,
                               precision, status, out, ctx)


def fixed_workspace_bytes() -> int:
    """Size of the fixed device workspace of regular_force_noalloc."""
    v = C.c_int64()
    _check(lib().nb_fixed_workspace_bytes(C.byref(v)), "nb_fixed_workspace_bytes")
    return v.value


def regular_force_adjoint(xp, vp, m, i_block, rs2, w_a, w_j, status=None,
                          ctx: Context | None = None):
    """dL/dxp, dL/dvp (3, n) and dL/dm (n,) for L = sum(w_a*acc + w_j*jerk),
    neighbour membership frozen."""
    n = m.shape[0]
    n_i = i_block.shape[0]
    _dev(xp, "xp", torch.float64, (3, n))
    _dev(vp, "vp", torch.float64, (3, n))
    _dev(m, "m", torch.float64, (n,))
    _dev(i_block, "i_block", torch.int32, (n_i,))
    _dev(rs2, "rs2", torch.float64, (n_i,))
    _dev(w_a, "w_a", torch.float64, (3, n_i))
    _dev(w_j, "w_j", torch.float64, (3, n_i))
    if status is not None:
        _dev(status, "status", torch.int32, (1,))
    gx = torch.empty_like(xp)
    gv = torch.empty_like(vp)
    gm = torch.empty_like(m)
    ctx = ctx or context(xp.device.index)
    ctx._bind_stream()
    _check(lib().nb_regular_force_adjoint(ctx.handle, n, _ptr(xp), _ptr(vp), _ptr(m), n_i,
                                          _ptr(i_block), _ptr(rs2), _ptr(w_a), _ptr(w_j),
                                          _ptr(gx), _ptr(gv), _ptr(gm), _ptr(status)),
           "nb_regular_force_adjoint")
    return gx, gv, gm


def _batched_call(fn: str, j_off, i_off, xp, vp, m, i_block, rs2, nb_cap: int, precision,
                  status, out, ctx, extra=()):
    import numpy as np
    j_off = np.ascontiguousarray(j_off, dtype=np.int64)
    i_off = np.ascontiguousarray(i_off, dtype=np.int64)
    if j_off.shape != i_off.shape or j_off.ndim != 1 or j_off.size < 1:
        raise ValueError("j_off and i_off must be 1-D of equal length n_clusters + 1")
    n = m.shape[0]
    n_rows = i_block.shape[0]
    _dev(xp, "xp", torch.float64, (3, n))
    _dev(vp, "vp", torch.float64, (3, n))
    _dev(m, "m", torch.float64, (n,))
    _dev(i_block, "i_block", torch.int32, (n_rows,))
    _dev(rs2, "rs2", torch.float64, (n_rows,))
    dev = xp.device
    acc, jerk, cnt, lst, ovf = _force_outputs(out, n_rows, nb_cap, dev)
    if status is not None:
        _dev(status, "status", torch.int32, (1,))
    ctx = ctx or context(dev.index)
    ctx._bind_stream()
    _check(getattr(lib(), fn)(
        ctx.handle, j_off.size - 1, j_off.ctypes.data_as(C.c_void_p),
        i_off.ctypes.data_as(C.c_void_p), _ptr(xp), _ptr(vp), _ptr(m), _ptr(i_block),
        _ptr(rs2), int(nb_cap), _prec(precision), _ptr(acc), _ptr(jerk), _ptr(cnt),
        _ptr(lst) if nb_cap > 0 else None, _ptr(ovf), _ptr(status), *extra), fn)
    return acc, jerk, cnt, lst, ovf


def regular_force_batched(j_off, i_off, xp, vp, m, i_block, rs2, nb_cap: int,
                          precision="mixed", status=None, out=None, ctx: Context | None = None):
    """Batched ensemble (see nbreg.h).  j_off, i_off: host int64 sequences of
    length n_clusters + 1.  Returns (acc, jerk, nb_count, nb_list, overflow)."""
    return _batched_call("nb_regular_force_batched", j_off, i_off, xp, vp, m, i_block, rs2,
                         nb_cap, precision, status, out, ctx)


def autotune_batched(j_off, i_off, xp, vp, m, i_block, rs2, nb_cap: int, precision="mixed",
                     status=None, out=None, cache_path: str | None = None, force: bool = False,
                     ctx: Context | None = None):
    """Times the batched kernel shapes on this ensemble and keeps the fastest
    for it (nb_autotune_batched); returns the outputs of the tuned shape."""
    return _batched_call("nb_autotune_batched", j_off, i_off, xp, vp, m, i_block, rs2, nb_cap,
                         precision, status, out, ctx,
                         extra=(cache_path.encode() if cache_path else None, int(bool(force))))


def autotune(n: int, cache_path: str | None = None, force: bool = False,
             ctx: Context | None = None):
    """Times candidate plans at n bodies and installs the fastest per block
    size bucket (see nb_autotune)."""
    ctx = ctx or context()
    ctx._bind_stream()
    _check(lib().nb_autotune(ctx.handle, int(n),
                             cache_path.encode() if cache_path else None, int(bool(force))),
           "nb_autotune")


def irregular_force(xp, vp, m, i_block, nb_cap, nb_count, nb_list, status=None,
                    ctx: Context | None = None):
    """Irregular acc, jerk (3, n_i) over the rows' neighbour lists (FP64)."""
    n = m.shape[0]
    n_i = i_block.shape[0]
    _dev(xp, "xp", torch.float64, (3, n))
    _dev(vp, "vp", torch.float64, (3, n))
    _dev(m, "m", torch.float64, (n,))
    _dev(i_block, "i_block", torch.int32, (n_i,))
    _dev(nb_count, "nb_count", torch.int32, (n_i,))
    _dev(nb_list, "nb_list", torch.int32, (n_i, nb_cap))
    if status is not None:
        _dev(status, "status", torch.int32, (1,))
    acc = torch.empty((3, n_i), dtype=torch.float64, device=xp.device)
    jerk = torch.empty_like(acc)
    ctx = ctx or context(xp.device.index)
    ctx._bind_stream()
    _check(lib().nb_irregular_force(ctx.handle, n, _ptr(xp), _ptr(vp), _ptr(m), n_i,
                                    _ptr(i_block), int(nb_cap), _ptr(nb_count),
                                    _ptr(nb_list) if nb_cap > 0 else None, _ptr(acc),
                                    _ptr(jerk), _ptr(status)), "nb_irregular_force")
    return acc, jerk


def hermite_correct(h, x0, v0, a0, j0, a1, j1, ctx: Context | None = None):
    """Fourth-order Hermite corrector: returns (x1, v1, a2, a3), each (3, n)."""
    n = h.shape[0]
    _dev(h, "h", torch.float64, (n,))
    for name, t in (("x0", x0), ("v0", v0), ("a0", a0), ("j0", j0), ("a1", a1), ("j1", j1)):
        _dev(t, name, torch.float64, (3, n))
    outs = [torch.empty_like(x0) for _ in range(4)]
    ctx = ctx or context(x0.device.index)
    ctx._bind_stream()
    _check(lib().nb_hermite_correct(ctx.handle, n, _ptr(h), _ptr(x0), _ptr(v0), _ptr(a0),
                                    _ptr(j0), _ptr(a1), _ptr(j1), *[_ptr(o) for o in outs]),
           "nb_hermite_correct")
    return tuple(outs)


def potential(x, m, ctx: Context | None = None):
    """(phi (n,), U (1,)): per-body potential and total potential energy (FP64)."""
    n = m.shape[0]
    _dev(x, "x", torch.float64, (3, n))
    _dev(m, "m", torch.float64, (n,))
    phi = torch.empty_like(m)
    U = torch.empty(1, dtype=torch.float64, device=x.device)
    ctx = ctx or context(x.device.index)
    ctx._bind_stream()
    _check(lib().nb_potential(ctx.handle, n, _ptr(x), _ptr(m), _ptr(phi), _ptr(U)),
           "nb_potential")
    return phi, U


def sched_build(level, k_max: int, order=None, level_end=None, status=None,
                ctx: Context | None = None):
    """Sorting list of the bodies by step (level descending, ties by index)
    and its offsets: returns (order (n,) int32, level_end (k_max+2,) int32),
    both on the GPU; level_end[L] = number of bodies with level >= L."""
    n = level.shape[0]
    _dev(level, "level", torch.int32, (n,))
    order = torch.empty(n, dtype=torch.int32, device=level.device) if order is None else \
        _dev(order, "order", torch.int32, (n,))
    level_end = torch.empty(k_max + 2, dtype=torch.int32, device=level.device) \
        if level_end is None else _dev(level_end, "level_end", torch.int32, (k_max + 2,))
    if status is not None:
        _dev(status, "status", torch.int32, (1,))
    ctx = ctx or context(level.device.index)
    ctx._bind_stream()
    _check(lib().nb_sched_build(ctx.handle, n, _ptr(level), int(k_max), _ptr(order),
                                _ptr(level_end), _ptr(status)), "nb_sched_build")
    return order, level_end


def sched_update(order, level_end, n_active: int, L: int, level, k_max: int, status=None,
                 ctx: Context | None = None):
    """In place: re-sorts the due prefix order[:n_active] (block level L) by
    the bodies' new levels and rewrites level_end[L:]."""
    n = level.shape[0]
    _dev(level, "level", torch.int32, (n,))
    _dev(order, "order", torch.int32, (n,))
    _dev(level_end, "level_end", torch.int32, (k_max + 2,))
    if status is not None:
        _dev(status, "status", torch.int32, (1,))
    ctx = ctx or context(level.device.index)
    ctx._bind_stream()
    _check(lib().nb_sched_update(ctx.handle, n, int(n_active), int(L), _ptr(level),
                                 int(k_max), _ptr(order), _ptr(level_end), _ptr(status)),
           "nb_sched_update")


def sched_next(t_now: float, k_max: int, level_end_host):
    """Host offset search: (t_new, L, n_active) of the next block from a host
    copy of level_end (sequence of k_max+2 ints)."""
    le = (C.c_int32 * (k_max + 2))(*[int(v) for v in level_end_host])
    t_new, L, n_a = C.c_double(), C.c_int32(), C.c_int32()
    _check(lib().nb_sched_next(float(t_now), int(k_max), C.cast(le, C.c_void_p),
                               C.byref(t_new), C.byref(L), C.byref(n_a)), "nb_sched_next")
    return t_new.value, L.value, n_a.value


def radius_update(nb_count, rs2, nnbopt: int, f_min: float = 0.5, f_max: float = 2.0,
                  out=None, ctx: Context | None = None):
    """Next-step squared neighbour radii toward nnbopt neighbours (see
    nb_radius_update); returns rs2_new (may be rs2 itself via out=rs2)."""
    n_i = rs2.shape[0]
    _dev(rs2, "rs2", torch.float64, (n_i,))
    _dev(nb_count, "nb_count", torch.int32, (n_i,))
    out = torch.empty_like(rs2) if out is None else _dev(out, "out", torch.float64, (n_i,))
    ctx = ctx or context(rs2.device.index)
    ctx._bind_stream()
    _check(lib().nb_radius_update(ctx.handle, n_i, _ptr(nb_count), _ptr(rs2), int(nnbopt),
                                  float(f_min), float(f_max), _ptr(out)), "nb_radius_update")
    return out


def regular_force_fit(xp, vp, m, i_block, rs2, nb_cap: int, nnbopt: int, max_rounds: int = 8,
                      precision="fp64", status=None, ctx: Context | None = None):
    """Regular force with overflowed rows shrunk toward min(nnbopt, nb_cap)
    neighbours and recomputed (see nb_regular_force_fit).  rs2 is updated in
    place.  Returns (acc, jerk, nb_count, nb_list, overflow, rounds)."""
    n = m.shape[0]
    n_i = i_block.shape[0]
    _dev(xp, "xp", torch.float64, (3, n))
    _dev(vp, "vp", torch.float64, (3, n))
    _dev(m, "m", torch.float64, (n,))
    _dev(i_block, "i_block", torch.int32, (n_i,))
    _dev(rs2, "rs2", torch.float64, (n_i,))
    if status is not None:
        _dev(status, "status", torch.int32, (1,))
    dv = xp.device
    acc = torch.empty((3, n_i), dtype=torch.float64, device=dv)
    jerk = torch.empty_like(acc)
    cnt = torch.empty(n_i, dtype=torch.int32, device=dv)
    lst = torch.empty((n_i, nb_cap), dtype=torch.int32, device=dv)
    ovf = torch.empty(1, dtype=torch.int32, device=dv)
    rounds = C.c_int32(0)
    ctx = ctx or context(dv.index)
    ctx._bind_stream()
    _check(lib().nb_regular_force_fit(ctx.handle, n, _ptr(xp), _ptr(vp), _ptr(m), n_i,
                                      _ptr(i_block), _ptr(rs2), int(nb_cap), _prec(precision),
                                      int(nnbopt), int(max_rounds), _ptr(acc), _ptr(jerk),
                                      _ptr(cnt), _ptr(lst), _ptr(ovf), _ptr(status),
                                      C.byref(rounds)), "nb_regular_force_fit")
    return acc, jerk, cnt, lst, ovf, rounds.value


class RegularForce(torch.autograd.Function):
    """(acc, jerk) = regular force of the block, differentiable with respect
    to xp, vp and m through the library's adjoint kernels (membership frozen)."""

    @staticmethod
    def forward(ctx, xp, vp, m, i_block, rs2, nb_cap, precision="fp64"):
        acc, jerk, cnt, lst, ovf = regular_force(xp, vp, m, i_block, rs2, nb_cap, precision)
        ctx.save_for_backward(xp, vp, m, i_block, rs2)
        ctx.mark_non_differentiable(cnt, lst, ovf)
        return acc, jerk, cnt, lst, ovf

    @staticmethod
    def backward(ctx, g_acc, g_jerk, *unused):
        xp, vp, m, i_block, rs2 = ctx.saved_tensors
        n_i = i_block.shape[0]
        z = torch.zeros((3, n_i), dtype=torch.float64, device=xp.device)
        w_a = z if g_acc is None else g_acc.contiguous()
        w_j = z if g_jerk is None else g_jerk.contiguous()
        gx, gv, gm = regular_force_adjoint(xp, vp, m, i_block, rs2, w_a, w_j)
        return gx, gv, gm, None, None, None, None
