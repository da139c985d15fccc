"""Plain FP64 CPU oracle for the Ahmad-Cohen regular-force step (ctypes wrapper
around ``oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``; nothing in the product path imports
it.  It shares no code with the HIP library.

Parity status per function (what pins it; see tests/test_oracle_pins.py):
  predict          -- exact rational Taylor polynomial, identity at dt = 0,
                      exact linear motion (pinned)
  regular          -- two-body closed forms, Decimal brute force, geometric
                      neighbour sets, momentum/jerk conservation, Plummer mean
                      field, power-of-two scaling, mass linearity, time
                      derivative of the force (pinned)
  irregular        -- regular + irregular = full force at rs2 = 0 (pinned)
  potential        -- two-body closed form, Plummer energy -1/2 (pinned)
  potential_rows   -- two-body and three-body closed forms (pinned)
  adjoint          -- central differences of local losses (pinned)
  local_loss       -- linear in m; equals the sum of pair losses (pinned)
  hermite_correct  -- exact for cubic force histories, two-body orbit
                      convergence at fourth order (pinned)
  sched.*          -- sorting-list selection of active bodies (oracle/sched.py):
                      hand-worked golden list, pairwise order, exact rational
                      block-step simulation (pinned)
  radius.*         -- neighbour-radius control toward NNBOPT (oracle/radius.py):
                      Decimal cube roots, clamp and fixed-point cases, uniform-
                      density counts, fit-loop invariants (pinned)
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_D = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_I = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (no fast-math, no fusion)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off",
                               "-fno-fast-math", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = C.CDLL(_LIB)
        i64, i32, dbl = C.c_int64, C.c_int32, C.c_double
        L.or_predict.argtypes = [i64, dbl, _D, _D, _D, _D, _D, _D, _D]
        L.or_predict.restype = None
        L.or_regular.argtypes = [i64, _D, _D, _D, i32, _I, _D, i32, _D, _D, _I, _I,
                                 C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.or_regular.restype = None
        L.or_irregular.argtypes = [i64, _D, _D, _D, i32, _I, i32, _I, _I, _D, _D]
        L.or_irregular.restype = None
        L.or_potential.argtypes = [i64, _D, _D, _D]
        L.or_potential.restype = dbl
        L.or_potential_rows.argtypes = [i64, _D, _D, i64, _I, _D]
        L.or_potential_rows.restype = None
        L.or_adjoint.argtypes = [i64, _D, _D, _D, _D, i32, _I, _D, _D, _D, _D, _D, _D]
        L.or_adjoint.restype = None
        L.or_local_loss.argtypes = [i64, _D, _D, _D, _D, i32, _I, _D, _D, _D, i64]
        L.or_local_loss.restype = dbl
        L.or_hermite_correct.argtypes = [i64, _D, _D, _D, _D, _D, _D, _D, _D, _D, _D, _D]
        L.or_hermite_correct.restype = None
        _lib = L
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def predict(t, x, v, a, jk, t0):
    """Hermite predictor of every body to time t.  Returns (xp, vp), [3][n]."""
    x, v, a, jk, t0 = map(_f64, (x, v, a, jk, t0))
    n = t0.size
    xp = np.empty((3, n))
    vp = np.empty((3, n))
    lib().or_predict(n, float(t), x, v, a, jk, t0, xp, vp)
    return xp, vp


def regular(xp, vp, m, i_block, rs2, nb_cap):
    """Regular acc/jerk [3][n_i], nb_count [n_i], nb_list [n_i][nb_cap],
    overflow flag and bad-index flag."""
    xp, vp, m, rs2 = map(_f64, (xp, vp, m, rs2))
    i_block = _i32(i_block)
    n, n_i = m.size, i_block.size
    acc = np.zeros((3, n_i))
    jerk = np.zeros((3, n_i))
    cnt = np.zeros(n_i, np.int32)
    lst = np.full((n_i, max(nb_cap, 0)), -1, np.int32)
    ovf = C.c_int32(0)
    bad = C.c_int32(0)
    lib().or_regular(n, xp, vp, m, n_i, i_block, rs2, int(nb_cap), acc, jerk, cnt,
                     lst if nb_cap > 0 else np.zeros((n_i, 1), np.int32),
                     C.byref(ovf), C.byref(bad))
    return acc, jerk, cnt, lst, int(ovf.value), int(bad.value)


def irregular(xp, vp, m, i_block, nb_cap, nb_count, nb_list):
    """Irregular acc/jerk [3][n_i] over the given neighbour lists."""
    xp, vp, m = map(_f64, (xp, vp, m))
    i_block, nb_count, nb_list = map(_i32, (i_block, nb_count, nb_list))
    n_i = i_block.size
    acc = np.zeros((3, n_i))
    jerk = np.zeros((3, n_i))
    lib().or_irregular(m.size, xp, vp, m, n_i, i_block, int(nb_cap), nb_count,
                       nb_list, acc, jerk)
    return acc, jerk


def potential(x, m):
    """(U, phi): total potential energy and per-body potential."""
    x, m = _f64(x), _f64(m)
    phi = np.empty(m.size)
    U = lib().or_potential(m.size, x, m, phi)
    return U, phi


def potential_rows(x, m, rows):
    """phi at the given bodies only (same sum as ``potential``)."""
    x, m, rows = _f64(x), _f64(m), _i32(rows)
    phi = np.empty(rows.size)
    lib().or_potential_rows(m.size, x, m, rows.size, rows, phi)
    return phi


def adjoint(xp, vp, m, i_block, rs2, w_a, w_j, xm=None):
    """dL/dxp, dL/dvp [3][n], dL/dm [n] for L = sum w_a.acc + w_j.jerk with
    membership frozen at positions ``xm`` (default xp)."""
    xp, vp, m, rs2, w_a, w_j = map(_f64, (xp, vp, m, rs2, w_a, w_j))
    xm = xp if xm is None else _f64(xm)
    i_block = _i32(i_block)
    n = m.size
    gx = np.empty((3, n))
    gv = np.empty((3, n))
    gm = np.empty(n)
    lib().or_adjoint(n, xp, vp, m, xm, i_block.size, i_block, rs2, w_a, w_j, gx, gv, gm)
    return gx, gv, gm


def local_loss(xp, vp, m, i_block, rs2, w_a, w_j, body, xm=None):
    """Sum of the regular pair losses that involve ``body`` (membership frozen
    at ``xm``)."""
    xp, vp, m, rs2, w_a, w_j = map(_f64, (xp, vp, m, rs2, w_a, w_j))
    xm = xp if xm is None else _f64(xm)
    i_block = _i32(i_block)
    return lib().or_local_loss(m.size, xp, vp, m, xm, i_block.size, i_block, rs2, w_a,
                               w_j, int(body))


def hermite_correct(h, x0, v0, a0, j0, a1, j1):
    """Fourth-order Hermite corrector: (x1, v1, a2 at the step end, a3)."""
    h, x0, v0, a0, j0, a1, j1 = map(_f64, (h, x0, v0, a0, j0, a1, j1))
    n = h.size
    out = [np.empty((3, n)) for _ in range(4)]
    lib().or_hermite_correct(n, h, x0, v0, a0, j0, a1, j1, *out)
    return tuple(out)
