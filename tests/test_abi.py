"""CPU-side checks of the C-ABI library: it loads, exports every function the
public header declares, and rejects bad arguments on the host before any GPU
work (using a host-only context, device -1, which launches nothing)."""
import ctypes as C
import os
import re

import pytest

import paper_1504_03687_amd as nb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    with open(os.path.join(ROOT, "include", "nbreg.h")) as f:
        src = f.read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(nb_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = nb.lib()
    names = _declared()
    assert "nb_regular_force" in names and "nb_predict" in names
    for name in names:
        assert hasattr(L, name), name
    assert L.nb_version() >= 10000
    assert nb.lib().nb_error_string(-1) == b"invalid argument"


@pytest.fixture
def host_ctx():
    L = nb.lib()
    h = C.c_void_p()
    assert L.nb_ctx_create(C.byref(h), -1, None) == 0
    yield h
    assert L.nb_ctx_destroy(h) == 0


def _fake(k):
    return C.c_void_p(0x1000 * k)   # never dereferenced: host-only context


def test_argument_validation(host_ctx):
    L = nb.lib()
    p = _fake
    ok = dict(n=100, n_i=10, cap=8)

    def reg(ctx=host_ctx, n=100, xp=p(1), vp=p(2), m=p(3), n_i=10, ib=p(4), rs2=p(5), cap=8,
            prec=0, acc=p(6), jerk=p(7), cnt=p(8), lst=p(9), ovf=p(10), st=None):
        return L.nb_regular_force(ctx, n, xp, vp, m, n_i, ib, rs2, cap, prec, acc, jerk, cnt,
                                  lst, ovf, st)

    E = -1
    assert reg(ctx=None) == E
    assert reg(n=0) == E and reg(n=-5) == E and reg(n=2 ** 31) == E
    assert reg(n_i=-1) == E and reg(cap=-1) == E and reg(prec=2) == E
    assert reg(xp=None) == E and reg(m=None) == E and reg(ovf=None) == E
    assert reg(ib=None) == E and reg(acc=None) == E and reg(cnt=None) == E
    assert reg(lst=None) == E                   # nb_cap > 0 needs a list
    assert reg(lst=None, cap=0) == -4           # valid; host-only context cannot launch
    assert reg(n_i=0, ib=None, rs2=None, acc=None, jerk=None, cnt=None, lst=None) == -4
    assert reg() == -4 and reg(prec=1) == -4
    # predictor
    pr = lambda **k: L.nb_predict(k.get("ctx", host_ctx), k.get("n", 10), k.get("t", 0.5),
                                  p(1), p(2), p(3), p(4), p(5), k.get("m", None), p(6), p(7),
                                  k.get("m32", None))
    assert pr(n=0) == E and pr(m=p(8)) == E and pr(t=float("nan")) == E
    assert pr() == -4 and pr(m=p(8), m32=p(9)) == -4
    # plan override
    assert L.nb_ctx_set_plan(host_ctx, 4, 0, 0) == E
    assert L.nb_ctx_set_plan(host_ctx, 3, 0, 0) == 0
    assert L.nb_ctx_set_plan(host_ctx, 1, 3, 0) == E
    assert L.nb_ctx_set_plan(host_ctx, 1, 2, 4) == 0
    assert L.nb_ctx_set_plan(host_ctx, 0, 0, 0) == 0
    assert L.nb_ctx_set_scratch_limit(host_ctx, -1) == E
    assert L.nb_ctx_set_refine_buffer_rows(host_ctx, -1) == E
    assert L.nb_ctx_set_refine_buffer_rows(host_ctx, 7) == 0
    assert L.nb_ctx_set_refine_buffer_rows(host_ctx, 0) == 0


def test_gpu_context_refused_without_gfx950():
    """Without an MI355X the library refuses a device context (no CPU fallback)."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = C.c_void_p()
    assert nb.lib().nb_ctx_create(C.byref(h), 0, None) == -4


def test_argument_validation_adjoint_batched_autotune(host_ctx):
    L = nb.lib()
    p = _fake
    E = -1

    def adj(ctx=host_ctx, n=50, n_i=5, ib=p(4), wa=p(6), gx=p(8)):
        return L.nb_regular_force_adjoint(ctx, n, p(1), p(2), p(3), n_i, ib, p(5), wa, p(7), gx,
                                          p(9), p(10), None)

    assert adj(ctx=None) == E and adj(n=0) == E and adj(n_i=-2) == E
    assert adj(ib=None) == E and adj(wa=None) == E and adj(gx=None) == E
    assert adj() == -4 and adj(n_i=0, ib=None, wa=None) == -4

    def bat(C=2, j=(0, 10, 30), i=(0, 3, 5), cap=4, prec=1, lst=p(9)):
        ja = (C_int64 * len(j))(*j)
        ia = (C_int64 * len(i))(*i)
        return L.nb_regular_force_batched(host_ctx, C, ja, ia, p(1), p(2), p(3), p(4), p(5), cap,
                                          prec, p(6), p(7), p(8), lst, p(10), None)

    C_int64 = C.c_int64
    assert bat() == -4
    assert bat(C=0) == E and bat(cap=-1) == E and bat(prec=3) == E
    assert bat(j=(1, 10, 30)) == E and bat(i=(0, 5, 3)) == E and bat(j=(0, 20, 10)) == E
    assert bat(j=(0, 0, 0)) == E                    # no bodies at all
    assert bat(lst=None) == E and bat(lst=None, cap=0) == -4
    assert L.nb_autotune(host_ctx, 10, None, 0) == E
    assert L.nb_autotune(host_ctx, 4096, None, 0) == -4


def test_argument_validation_scheduler(host_ctx):
    L = nb.lib()
    p = _fake
    E, U = -1, -4

    def build(ctx=host_ctx, n=100, lev=p(1), k_max=20, order=p(2), le=p(3)):
        return L.nb_sched_build(ctx, n, lev, k_max, order, le, None)

    def update(ctx=host_ctx, n=100, n_a=10, lvl=3, lev=p(1), k_max=20, order=p(2), le=p(3)):
        return L.nb_sched_update(ctx, n, n_a, lvl, lev, k_max, order, le, None)

    assert build(ctx=None) == E and build(n=0) == E and build(n=2 ** 31) == E
    assert build(k_max=-1) == E and build(k_max=64) == E
    assert build(lev=None) == E and build(order=None) == E and build(le=None) == E
    assert build() == U and build(k_max=63) == U          # valid; no device
    assert update(lvl=-1) == E and update(lvl=21) == E
    assert update(n_a=-1) == E and update(n_a=101) == E and update(k_max=64) == E
    assert update(order=None) == E and update(le=None) == E
    assert update() == U


def _next(t_now, k_max, le):
    t, lv, na = C.c_double(), C.c_int32(), C.c_int32()
    arr = (C.c_int32 * len(le))(*le)
    rc = nb.lib().nb_sched_next(float(t_now), k_max, C.cast(arr, C.c_void_p), C.byref(t),
                                C.byref(lv), C.byref(na))
    return rc, t.value, lv.value, na.value


def test_sched_next_rejects_bad_offsets():
    assert _next(0.0, 3, [5, 4, 2, 1, 0])[0] == 0
    assert _next(0.0, 3, [0, 0, 0, 0, 0])[0] == -1        # empty
    assert _next(0.0, 3, [5, 4, 2, 3, 0])[0] == -1        # not monotone
    assert _next(0.0, 3, [5, 4, 2, 1, 1])[0] == -1        # level_end[k_max+1] != 0
    assert _next(-1.0, 3, [5, 4, 2, 1, 0])[0] == -1
    assert _next(float("inf"), 3, [5, 4, 2, 1, 0])[0] == -1
    assert _next(0.0625, 3, [5, 4, 2, 1, 0])[0] == -1     # not a multiple of 2^-3
    assert _next(2.0 ** 60, 3, [5, 4, 2, 1, 0])[0] == -1  # step below resolution
    assert _next(0.0, -1, [0])[0] == -1 and _next(0.0, 64, [0] * 66)[0] == -1


def test_sched_next_matches_oracle_selection():
    """The host offset search (Figure 1) against the oracle's brute-force
    selection over all bodies, along a seeded synchronised block-step run."""
    import numpy as np
    import oracle.sched as S
    rng = np.random.default_rng(701)
    n, k_max = 500, 16
    lev = rng.integers(3, 12, n)
    t = np.zeros(n)
    t_now = 0.0
    for step in range(3000):
        _, le = S.sort_list(lev, k_max)
        rc, t_new, L, n_a = _next(t_now, k_max, le.tolist())
        assert rc == 0
        ot, act = S.next_block(t, np.ldexp(1.0, -lev))
        assert t_new == ot and L == S.due_level(ot, k_max) and n_a == act.size
        for i in act:
            lo = max(L, int(lev[i]) - 1)
            lev[i] = int(rng.integers(lo, min(k_max, int(lev[i]) + 2) + 1))
        t[act] = t_new
        t_now = t_new


def test_argument_validation_radius_control(host_ctx):
    L = nb.lib()
    p = _fake
    E, U = -1, -4

    def upd(ctx=host_ctx, n_i=10, cnt=p(1), rs2=p(2), nnb=64, lo=0.5, hi=2.0, out=p(3)):
        return L.nb_radius_update(ctx, n_i, cnt, rs2, nnb, lo, hi, out)

    assert upd(ctx=None) == E and upd(n_i=-1) == E and upd(nnb=0) == E
    assert upd(lo=0.0) == E and upd(lo=-1.0) == E and upd(hi=0.25) == E
    assert upd(hi=float("inf")) == E and upd(hi=float("nan")) == E
    assert upd(cnt=None) == E and upd(rs2=None) == E and upd(out=None) == E
    assert upd() == U and upd(n_i=0, cnt=None, rs2=None, out=None) == U

    def fit(ctx=host_ctx, n=100, n_i=10, rs2=p(5), cap=8, prec=0, nnb=64, rounds=4, lst=p(9)):
        return L.nb_regular_force_fit(ctx, n, p(1), p(2), p(3), n_i, p(4), rs2, cap, prec, nnb,
                                      rounds, p(6), p(7), p(8), lst, p(10), None, None)

    assert fit(ctx=None) == E and fit(cap=0) == E and fit(nnb=0) == E and fit(rounds=-1) == E
    assert fit(lst=None) == E and fit(rs2=None) == E and fit(n=0) == E and fit(prec=3) == E
    assert fit() == U
