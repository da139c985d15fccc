"""Pins of the CPU oracle against facts that do not come from the oracle itself:
closed forms, exact rational arithmetic, high-precision brute force, symmetry
and conservation laws, the Plummer mean field and finite differences.

Each pin is chosen so that a plausible slip in the oracle (a dropped term, a
wrong sign, power or index, a transposed operand, a wrong neighbour boundary)
fails at least one of them.
"""
import ctypes
import ctypes.util
import json
import math
import os
from decimal import Decimal, getcontext
from fractions import Fraction

import numpy as np
import pytest

import oracle
import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------- #
# predictor
# --------------------------------------------------------------------------- #
def test_predict_exact_rational_taylor():
    """xp = x + v dt + a dt^2/2 + j dt^3/6 and vp = v + a dt + j dt^2/2, checked
    against exact rational evaluation: the oracle may differ only by its own
    rounding (a few ulp of the largest term)."""
    rng = np.random.default_rng(7)
    n = 2000
    x, v, a, jk = (rng.standard_normal((3, n)) for _ in range(4))
    t0 = -rng.random(n) * 0.1
    t = 0.0625
    xp, vp = oracle.predict(t, x, v, a, jk, t0)
    for q in range(0, n, 37):
        for k in range(3):
            dt = Fraction(t) - Fraction(t0[q])
            X, V, A, J = (Fraction(float(arr[k, q])) for arr in (x, v, a, jk))
            ex = X + V * dt + A * dt ** 2 / 2 + J * dt ** 3 / 6
            ev = V + A * dt + J * dt ** 2 / 2
            scale_x = float(abs(X) + abs(V * dt) + abs(A * dt ** 2 / 2) + abs(J * dt ** 3 / 6))
            scale_v = float(abs(V) + abs(A * dt) + abs(J * dt ** 2 / 2))
            assert abs(Fraction(float(xp[k, q])) - ex) <= 4 * 2.0 ** -52 * scale_x
            assert abs(Fraction(float(vp[k, q])) - ev) <= 4 * 2.0 ** -52 * scale_v


def test_predict_identity_and_linear_motion():
    rng = np.random.default_rng(8)
    n = 257
    x, v, a, jk = (rng.standard_normal((3, n)) for _ in range(4))
    t0 = rng.random(n)
    # dt = 0: identity, bit for bit
    xp, vp = oracle.predict(0.5, x, v, a, jk, np.full(n, 0.5))
    assert np.array_equal(xp, x) and np.array_equal(vp, v)
    # a = j = 0 with short dyadic mantissas: xp = x + v dt exactly
    xi = np.round(rng.standard_normal((3, n)) * 64) / 64
    vi = np.round(rng.standard_normal((3, n)) * 64) / 64
    z = np.zeros((3, n))
    xp, vp = oracle.predict(0.25, xi, vi, z, z, np.full(n, -0.125))
    assert np.array_equal(xp, xi + vi * 0.375)
    assert np.array_equal(vp, vi)


# --------------------------------------------------------------------------- #
# two-body closed forms (golden fixture)
# --------------------------------------------------------------------------- #
def _golden_two_body():
    with open(os.path.join(GOLDEN, "two_body.json")) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("case", _golden_two_body(), ids=lambda c: c["name"])
def test_two_body_closed_form(case):
    x = np.array(case["x"], float).T.copy()
    v = np.array(case["v"], float).T.copy()
    m = np.array(case["m"], float)
    blk = np.array([0, 1], np.int32)
    acc, jerk, cnt, lst, ovf, bad = oracle.regular(x, v, m, blk, np.full(2, case["rs2"]), 4)
    ea = np.array(case["acc"], float).T
    ej = np.array(case["jerk"], float).T
    if case["exact"]:
        assert np.array_equal(acc, ea) and np.array_equal(jerk, ej)
    else:
        assert np.allclose(acc, ea, rtol=4e-16, atol=0) and np.allclose(jerk, ej, rtol=4e-16, atol=1e-300)
    for b in range(2):
        assert list(lst[b, :cnt[b]]) == case["nb"][b]
    assert ovf == 0 and bad == 0


# --------------------------------------------------------------------------- #
# brute force in independent arithmetic
# --------------------------------------------------------------------------- #
_libm = ctypes.CDLL(ctypes.util.find_library("m"))
_libm.fmaf.argtypes = [ctypes.c_float] * 3
_libm.fmaf.restype = ctypes.c_float


def _canonical_inside(dx, dy, dz, rs2):
    """The FP32-rounded r^2 < rs^2 test, from numpy float32 rounding and libm fmaf."""
    fx, fy, fz = (np.float32(d) for d in (dx, dy, dz))
    sq = np.float32(fx * fx)
    r2f = _libm.fmaf(float(fz), float(fz), _libm.fmaf(float(fy), float(fy), float(sq)))
    return np.float32(r2f) < np.float32(rs2)


def _decimal_row(x, v, m, i, members):
    getcontext().prec = 40
    A = [Decimal(0)] * 3
    J = [Decimal(0)] * 3
    for j in members:
        r = [Decimal(float(x[k, j])) - Decimal(float(x[k, i])) for k in range(3)]
        u = [Decimal(float(v[k, j])) - Decimal(float(v[k, i])) for k in range(3)]
        r2 = sum(c * c for c in r)
        rr = r2.sqrt()
        r3 = r2 * rr
        s = sum(r[k] * u[k] for k in range(3))
        mj = Decimal(float(m[j]))
        for k in range(3):
            A[k] += mj * r[k] / r3
            J[k] += mj * (u[k] / r3 - 3 * s * r[k] / (r3 * r2))
    return np.array([float(c) for c in A]), np.array([float(c) for c in J])


def test_bruteforce_tiny_n_decimal():
    rng = np.random.default_rng(11)
    n = 24
    x = rng.standard_normal((3, n))
    v = rng.standard_normal((3, n))
    m = rng.random(n) + 0.1
    blk = rng.permutation(n).astype(np.int32)
    rs2 = rng.random(n) * 1.5
    rs2[3] = 0.0
    rs2[5] = -1.0
    acc, jerk, cnt, lst, ovf, bad = oracle.regular(x, v, m, blk, rs2, n)
    for b in range(n):
        i = blk[b]
        nb = [j for j in range(n) if j != i and _canonical_inside(
            x[0, j] - x[0, i], x[1, j] - x[1, i], x[2, j] - x[2, i], rs2[b])]
        reg = [j for j in range(n) if j != i and j not in nb]
        assert list(lst[b, :cnt[b]]) == nb
        ea, ej = _decimal_row(x, v, m, i, reg)
        assert np.linalg.norm(acc[:, b] - ea) <= 1e-14 * np.linalg.norm(ea)
        assert np.linalg.norm(jerk[:, b] - ej) <= 1e-14 * np.linalg.norm(ej)


def test_neighbour_sets_match_geometry_away_from_boundary():
    """Inside the radius means |r|^2 < rs^2 (section 2).  Where the exact squared
    distance is not within 1e-6 (relative) of rs2, the canonical FP32 test must
    agree with exact geometry."""
    s = W.small_state(1, 700, k_nn=32)
    x = s["x"]
    blk = np.arange(700, dtype=np.int32)
    acc, jerk, cnt, lst, ovf, bad = oracle.regular(x, s["v"], s["m"], blk, s["rs2"], 700)
    for b in range(0, 700, 7):
        d = x - x[:, b:b + 1]
        r2 = [sum(Fraction(float(d[k, j])) ** 2 for k in range(3)) for j in range(700)]
        rs2 = Fraction(float(s["rs2"][b]))
        got = set(lst[b, :cnt[b]].tolist())
        for j in range(700):
            if j == b or abs(r2[j] - rs2) <= Fraction(1, 10 ** 6) * rs2:
                continue
            assert (j in got) == (r2[j] < rs2), (b, j)


def test_overflow_truncation_and_bad_index():
    s = W.small_state(2, 300, k_nn=40)
    blk = np.array([5, 17, 299, 300, -1, 5], np.int32)
    rs2 = s["rs2"][np.clip(blk, 0, 299)]
    full = oracle.regular(s["x"], s["v"], s["m"], blk, rs2, 300)
    cut = oracle.regular(s["x"], s["v"], s["m"], blk, rs2, 8)
    assert cut[4] == 1 and full[4] == 0          # overflow flag
    assert cut[5] == 1                           # bad-index flag
    assert np.array_equal(full[2], cut[2])       # true counts kept
    for b in (0, 1, 2, 5):
        c = full[2][b]
        assert np.all(np.diff(full[3][b, :c]) > 0)               # ascending j
        assert np.array_equal(cut[3][b, :min(c, 8)], full[3][b, :min(c, 8)])
    assert np.array_equal(full[0], cut[0]) and np.array_equal(full[1], cut[1])
    for b in (3, 4):
        assert full[2][b] == 0 and not full[0][:, b].any() and not full[1][:, b].any()
    for res, cap in ((full, 300), (cut, 8)):      # nothing written past min(count, cap)
        for b in range(blk.size):
            assert np.all(res[3][b, min(res[2][b], cap):] == -1)
    assert np.array_equal(full[0][:, 0], full[0][:, 5])          # duplicate rows


# --------------------------------------------------------------------------- #
# symmetries and conservation
# --------------------------------------------------------------------------- #
def test_power_of_two_scaling_and_mass_linearity_bitwise():
    s = W.small_state(3, 513, k_nn=24)
    blk = np.arange(513, dtype=np.int32)
    base = oracle.regular(s["x"], s["v"], s["m"], blk, s["rs2"], 64)
    sx = oracle.regular(2 * s["x"], s["v"], s["m"], blk, 4 * s["rs2"], 64)
    assert np.array_equal(base[3], sx[3]) and np.array_equal(base[2], sx[2])
    assert np.array_equal(sx[0], base[0] / 4)
    assert np.array_equal(sx[1], base[1] / 8)
    sv = oracle.regular(s["x"], 2 * s["v"], s["m"], blk, s["rs2"], 64)
    assert np.array_equal(sv[0], base[0]) and np.array_equal(sv[1], 2 * base[1])
    sm = oracle.regular(s["x"], s["v"], 2 * s["m"], blk, s["rs2"], 64)
    assert np.array_equal(sm[0], 2 * base[0]) and np.array_equal(sm[1], 2 * base[1])


def test_momentum_and_jerk_conservation_symmetric_membership():
    """With one radius for every body the membership is symmetric, so the
    regular forces of all bodies obey Newton's third law: sum m a = 0, and so
    does its time derivative.  Per-body radii break this for the regular part
    alone, but regular + irregular restores it."""
    s = W.small_state(4, 800, k_nn=32)
    x, v, m = s["x"], s["v"], s["m"]
    blk = np.arange(800, dtype=np.int32)
    for rs2 in (np.full(800, 0.02), np.zeros(800)):
        acc, jerk, cnt, lst, ovf, bad = oracle.regular(x, v, m, blk, rs2, 800)
        for q in (acc, jerk):
            tot = np.abs((q * m).sum(1)).max()
            assert tot <= 1e-13 * (np.abs(q) * m).sum()
    acc, jerk, cnt, lst, ovf, bad = oracle.regular(x, v, m, blk, s["rs2"], 800)
    assert np.abs((acc * m).sum(1)).max() > 1e-8          # regular part alone does not conserve
    ia, ij = oracle.irregular(x, v, m, blk, 800, cnt, lst)
    for q in (acc + ia, jerk + ij):
        assert np.abs((q * m).sum(1)).max() <= 1e-13 * (np.abs(q) * m).sum()


def test_regular_plus_irregular_is_full_force():
    s = W.small_state(5, 600, k_nn=48)
    x, v, m = s["x"], s["v"], s["m"]
    blk = np.arange(600, dtype=np.int32)
    fa, fj, *_ = oracle.regular(x, v, m, blk, np.zeros(600), 16)
    acc, jerk, cnt, lst, ovf, bad = oracle.regular(x, v, m, blk, s["rs2"], 600)
    ia, ij = oracle.irregular(x, v, m, blk, 600, cnt, lst)
    assert np.allclose(acc + ia, fa, rtol=0, atol=1e-12 * np.abs(fa).max())
    assert np.allclose(jerk + ij, fj, rtol=0, atol=1e-12 * np.abs(fj).max())


def test_jerk_is_time_derivative_of_force():
    """Move every body on a straight line x + v tau; the full force (rs2 = 0)
    then has d/dtau acc = jerk.  Central differences, h = 1e-4."""
    s = W.small_state(6, 200)
    x, v, m = s["x"], s["v"], s["m"]
    blk = np.arange(200, dtype=np.int32)
    z = np.zeros(200)
    h = 1e-4
    ap, *_ = oracle.regular(x + h * v, v, m, blk, z, 4)
    am, *_ = oracle.regular(x - h * v, v, m, blk, z, 4)
    _, jerk, *_ = oracle.regular(x, v, m, blk, z, 4)
    fd = (ap - am) / (2 * h)
    err = np.linalg.norm(fd - jerk, axis=0) / np.linalg.norm(jerk, axis=0)
    assert np.median(err) < 1e-6 and err.max() < 1e-3


def test_plummer_mean_field_convergence():
    """Full force of a Plummer sample approaches the analytic field
    -r / (r^2 + b^2)^(3/2) (b = 3 pi / 16 in Henon units); the median relative
    deviation shrinks roughly as N^-1/2."""
    dev = []
    for n in (2048, 8192, 32768):
        rng = np.random.Generator(np.random.PCG64(99 + n))
        x, v, m = W.plummer(rng, n, "equal")
        sel = np.arange(0, n, max(1, n // 2048), dtype=np.int32)
        acc, *_ = oracle.regular(x, v, m, sel, np.zeros(sel.size), 4)
        xs = x[:, sel]
        ana = -xs / ((xs * xs).sum(0) + W.PLUMMER_B ** 2) ** 1.5
        dev.append(np.median(np.linalg.norm(acc - ana, axis=0) / np.linalg.norm(ana, axis=0)))
    assert dev[0] < 0.2
    assert 0.3 < dev[1] / dev[0] < 0.75 and 0.3 < dev[2] / dev[1] < 0.75, dev


# --------------------------------------------------------------------------- #
# potential
# --------------------------------------------------------------------------- #
def test_potential_two_body_and_plummer_energy():
    x = np.array([[0.0, 3.0], [0.0, 4.0], [0.0, 0.0]])
    m = np.array([0.5, 0.25])
    U, phi = oracle.potential(x, m)
    assert phi[0] == -0.25 / 5 and phi[1] == -0.5 / 5 and U == -0.5 * 0.25 / 5
    rng = np.random.Generator(np.random.PCG64(4242))
    x, v, m = W.plummer(rng, 16384, "equal")
    U, phi = oracle.potential(x, m)
    assert abs(U + 0.5) < 0.02           # Henon units: E = -1/4, virial U = -1/2
    T = 0.5 * (m * (v * v).sum(0)).sum()
    assert abs(T - 0.25) < 0.02


def test_potential_rows_closed_forms():
    """phi at selected bodies: a 3-4-5 triangle (exact distances 3, 4, 5) and
    an equilateral triangle of side 2 (phi = -(sum of the other masses)/2)."""
    x = np.array([[0.0, 3.0, 0.0], [0.0, 0.0, 4.0], [0.0, 0.0, 0.0]])
    m = np.array([1.0, 0.5, 0.25])
    phi = oracle.potential_rows(x, m, np.array([2, 0, 1], np.int32))
    assert phi[0] == -(1.0 / 4 + 0.5 / 5)
    assert phi[1] == -(0.5 / 3 + 0.25 / 4)
    assert phi[2] == -(1.0 / 3 + 0.25 / 5)
    h = math.sqrt(3.0)
    x = np.array([[-1.0, 1.0, 0.0], [0.0, 0.0, h], [0.0, 0.0, 0.0]])
    m = np.array([0.125, 0.25, 0.5])
    phi = oracle.potential_rows(x, m, np.array([0, 1, 2], np.int32))
    want = -np.array([0.75, 0.625, 0.375]) / 2.0
    assert np.allclose(phi, want, rtol=4e-16, atol=0)


# --------------------------------------------------------------------------- #
# adjoint
# --------------------------------------------------------------------------- #
def test_adjoint_matches_local_finite_differences():
    s = W.small_state(7, 300, k_nn=20)
    x, v, m = s["x"], s["v"], s["m"]
    rng = np.random.default_rng(17)
    blk = rng.choice(300, 120, replace=False).astype(np.int32)
    rs2 = s["rs2"][blk]
    wa = rng.standard_normal((3, 120))
    wj = rng.standard_normal((3, 120))
    gx, gv, gm = oracle.adjoint(x, v, m, blk, rs2, wa, wj)
    h = 1e-6
    bodies = list(blk[:6]) + [k for k in range(300) if k not in set(blk.tolist())][:6]
    for k in bodies:
        for c in range(3):
            for arr, g in ((x, gx), (v, gv)):
                p = arr.copy(); p[c, k] += h
                q = arr.copy(); q[c, k] -= h
                if arr is x:
                    lp = oracle.local_loss(p, v, m, blk, rs2, wa, wj, k, xm=x)
                    lq = oracle.local_loss(q, v, m, blk, rs2, wa, wj, k, xm=x)
                else:
                    lp = oracle.local_loss(x, p, m, blk, rs2, wa, wj, k)
                    lq = oracle.local_loss(x, q, m, blk, rs2, wa, wj, k)
                fd = (lp - lq) / (2 * h)
                assert abs(fd - g[c, k]) <= 1e-6 * max(abs(g[c, k]), 1e-3 * np.abs(g).max()), (k, c)
        mp = m.copy(); mp[k] *= 1.5
        lp = oracle.local_loss(x, v, mp, blk, rs2, wa, wj, k)
        l0 = oracle.local_loss(x, v, m, blk, rs2, wa, wj, k)
        lj = lp - l0
        assert abs(lj / (0.5 * m[k]) - gm[k]) <= 1e-9 * max(abs(gm[k]), 1e-12)


def test_adjoint_is_linear_in_weights_and_matches_forward():
    """L is linear in the weights, and with w_a = e_c at one row, w_j = 0, the
    mass gradient times m reproduces the acc component (acc is linear in m)."""
    s = W.small_state(8, 200, k_nn=16)
    x, v, m = s["x"], s["v"], s["m"]
    blk = np.arange(200, dtype=np.int32)
    wa = np.zeros((3, 200)); wj = np.zeros((3, 200))
    wa[1, 37] = 1.0
    gx, gv, gm = oracle.adjoint(x, v, m, blk, s["rs2"], wa, wj)
    acc, jerk, *_ = oracle.regular(x, v, m, blk, s["rs2"], 200)
    assert abs((gm * m).sum() - acc[1, 37]) <= 1e-13 * np.abs(acc[:, 37]).sum()
    assert not gv.any()
    wa[:] = 0; wj[2, 11] = 1.0
    gx, gv, gm = oracle.adjoint(x, v, m, blk, s["rs2"], wa, wj)
    assert abs((gm * m).sum() - jerk[2, 11]) <= 1e-13 * np.abs(jerk[:, 11]).sum()


# --------------------------------------------------------------------------- #
# Hermite corrector
# --------------------------------------------------------------------------- #
def test_hermite_corrector_exact_for_cubic_force():
    """For a force history that is a cubic polynomial in time the corrector's
    velocity update (two-point Hermite quadrature) and the interpolated a2, a3
    are exact; the position update is exact when, in addition, a is at most
    quadratic (the velocity is then cubic)."""
    rng = np.random.default_rng(21)
    n = 50
    h = np.ldexp(1.0, -rng.integers(2, 8, n))
    x0, v0, A0, J0, S0 = (rng.standard_normal((3, n)) for _ in range(5))
    C0 = rng.standard_normal((3, n))
    for cubic in (C0, np.zeros((3, n))):
        a = lambda t: A0 + J0 * t + S0 * t ** 2 / 2 + cubic * t ** 3 / 6
        jd = lambda t: J0 + S0 * t + cubic * t ** 2 / 2
        vx = lambda t: v0 + A0 * t + J0 * t ** 2 / 2 + S0 * t ** 3 / 6 + cubic * t ** 4 / 24
        xx = lambda t: (x0 + v0 * t + A0 * t ** 2 / 2 + J0 * t ** 3 / 6 + S0 * t ** 4 / 24
                        + cubic * t ** 5 / 120)
        x1, v1, a2, a3 = oracle.hermite_correct(h, x0, v0, a(0), jd(0), a(h), jd(h))
        assert np.allclose(v1, vx(h), rtol=0, atol=1e-13)
        # a2, a3 divide differences of O(1) forces by h^2, h^3: allow that rounding
        assert np.all(np.abs(a3 - cubic) <= 64 * 2.0 ** -52 * 4 / h ** 3)
        assert np.all(np.abs(a2 - (S0 + cubic * h)) <= 64 * 2.0 ** -52 * 4 / h ** 2)
        if not cubic.any():
            assert np.allclose(x1, xx(h), rtol=0, atol=1e-13)


def test_hermite_two_body_orbit_fourth_order():
    """Integrate a circular two-body orbit for one period with predictor ->
    full force (rs2 = 0) -> corrector; the position error after one period
    falls by ~2^4 when the step halves."""
    def run(steps):
        m = np.array([0.5, 0.5])
        x = np.array([[0.5, -0.5], [0.0, 0.0], [0.0, 0.0]])
        v = np.array([[0.0, 0.0], [0.5, -0.5], [0.0, 0.0]])   # circular: v^2 = M/(4 r)
        blk = np.array([0, 1], np.int32)
        a, j, *_ = oracle.regular(x, v, m, blk, np.zeros(2), 2)
        period = 2 * np.pi * np.sqrt(1.0 / 1.0)            # a_rel = 1, M = 1
        h = period / steps
        for k in range(steps):
            xp, vp = oracle.predict(h, x, v, a, j, np.zeros(2))
            a1, j1, *_ = oracle.regular(xp, vp, m, blk, np.zeros(2), 2)
            x, v, _, _ = oracle.hermite_correct(np.full(2, h), x, v, a, j, a1, j1)
            a, j = a1, j1
        return np.abs(x - np.array([[0.5, -0.5], [0, 0], [0, 0]])).max()
    e1, e2 = run(200), run(400)
    assert e1 < 1e-5 and 12 < e1 / e2 < 20, (e1, e2)


# --------------------------------------------------------------------------- #
# sorting-list selection of active bodies (section 3.3.1)
# --------------------------------------------------------------------------- #
def _golden_sched():
    with open(os.path.join(GOLDEN, "sorting_list.json")) as f:
        return json.load(f)


def test_sorting_list_golden():
    """Hand-worked list, offsets, block sequence and post-update level sets."""
    import oracle.sched as S
    g = _golden_sched()
    lev = np.array(g["levels"])
    order, le = S.sort_list(lev, g["k_max"])
    assert order.tolist() == g["order"] and le.tolist() == g["level_end"]
    t = np.zeros(lev.size)
    dt = np.ldexp(1.0, -lev)
    t_now = 0.0
    for blk in g["blocks_from_t0"]:
        t_new, act = S.next_block(t, dt)
        assert t_new == blk["t_new"] and act.tolist() == blk["active"]
        L = S.due_level(t_new, g["k_max"])
        assert L == blk["level"]
        assert sorted(order[: le[L]].tolist()) == blk["active"]
        # the next block time is the current one plus the smallest step
        assert t_new == t_now + math.ldexp(1.0, -int(lev.max()))
        t[act] = t_new
        t_now = t_new
    assert t_now == g["update_at_t"] and S.due_level(t_now, g["k_max"]) == g["update_level"]
    new = np.array(g["new_levels"])
    order2, le2 = S.sort_list(new, g["k_max"])
    assert le2.tolist() == g["new_level_end"]
    for L, members in g["new_level_sets"].items():
        L = int(L)
        assert sorted(order2[le2[L + 1]: le2[L]].tolist()) == members
    t_new, act = S.next_block(t, np.ldexp(1.0, -new))
    nxt = g["next_after_update"]
    assert t_new == nxt["t_new"] and act.tolist() == nxt["active"]
    assert S.due_level(t_new, g["k_max"]) == nxt["level"]


@pytest.mark.parametrize("seed", range(6))
def test_sorting_list_pairwise_and_counts(seed):
    """Brute force on small random inputs: the list is a permutation, every
    pair of list positions is ordered by (level descending, index ascending),
    and every offset equals a direct count."""
    import oracle.sched as S
    rng = np.random.default_rng(600 + seed)
    n = [0, 1, 7, 64, 129, 300][seed]
    k_max = [0, 3, 5, 9, 20, 63][seed]
    lev = rng.integers(0, k_max + 1, n)
    order, le = S.sort_list(lev, k_max)
    assert sorted(order.tolist()) == list(range(n))
    for p in range(n):
        for q in range(p + 1, n):
            a, b = int(order[p]), int(order[q])
            assert lev[a] > lev[b] or (lev[a] == lev[b] and a < b)
    assert le.size == k_max + 2 and le[k_max + 1] == 0
    for L in range(k_max + 1):
        assert le[L] == sum(1 for v in lev.tolist() if v >= L)
    with pytest.raises(ValueError):
        S.sort_list(np.array([k_max + 1]), k_max)


def test_block_step_selection_exact_rational():
    """Synchronised block steps simulated in exact rationals: the brute-force
    next block time and active set agree with the exact ones, the active set is
    every body whose level is at least the coarsest level dividing the block
    time, and the block time advances by the smallest step."""
    import oracle.sched as S
    rng = np.random.default_rng(612)
    n, k_max = 97, 12
    lev = rng.integers(2, k_max + 1, n)
    t_ex = [Fraction(0)] * n
    t_now = Fraction(0)
    for step in range(400):
        dt_ex = [Fraction(1, 2 ** int(k)) for k in lev]
        nxt = [a + b for a, b in zip(t_ex, dt_ex)]
        T = min(nxt)
        act_ex = [i for i in range(n) if nxt[i] == T]
        t_new, act = S.next_block(np.array([float(a) for a in t_ex]),
                                  np.ldexp(1.0, -lev))
        assert Fraction(t_new) == T and act.tolist() == act_ex
        assert T == t_now + Fraction(1, 2 ** int(lev.max()))
        L = S.due_level(t_new, k_max)
        assert T.denominator == 2 ** L
        assert act_ex == [i for i in range(n) if lev[i] >= L]
        for i in act_ex:
            t_ex[i] = T
            # new level: commensurate with T (>= L), within [0, k_max]
            lo = max(L, int(lev[i]) - 1)
            hi = min(k_max, int(lev[i]) + 2)
            lev[i] = int(rng.integers(lo, hi + 1))
        t_now = T
    assert S.due_level(1.0, 8) == 0 and S.due_level(0.375, 8) == 3
    assert S.due_level(0.5, 8) == 1 and S.due_level(2.0 ** -9, 8) == -1


# --------------------------------------------------------------------------- #
# neighbour-radius control (Table A1, NNBOPT; uniform-density reading)
# --------------------------------------------------------------------------- #
def _ulp(x):
    return np.spacing(np.abs(x))


def test_pow23_against_decimal_cube_roots():
    """q^(2/3) by the fixed Newton steps is within 2 ulp of the 50-digit
    cube root of q*q, and exact where the root is a representable value."""
    import oracle.radius as R
    getcontext().prec = 50
    rng = np.random.default_rng(801)
    q = np.concatenate([np.exp(rng.uniform(np.log(1e-4), np.log(1e4), 4000)),
                        [1.0, 2.0, 0.5, 3.0, 64.0 / 63.0, 63.0 / 64.0, 1e-6, 1e6]])
    y = R.pow23(q)
    for qi, yi in zip(q.tolist(), y.tolist()):
        ex = (Decimal(qi) * Decimal(qi)) ** (Decimal(1) / Decimal(3))
        assert abs(Decimal(yi) - ex) <= 2 * Decimal(float(np.spacing(yi))), (qi, yi)
    for qi, exact in ((8.0, 4.0), (1.0, 1.0), (0.125, 0.25), (27.0, 9.0), (1 / 64, 1 / 16)):
        assert R.pow23(np.array([qi]))[0] == exact


def test_radius_update_rules():
    import oracle.radius as R
    rs2 = np.array([0.01, 0.02, 0.04, 0.0, -1.0, 0.03, 0.05])
    cnt = np.array([64, 512, 8, 10, 10, 0, 1], np.int64)
    out = R.radius_update(rs2, cnt, 64, 0.5, 2.0)
    assert out[0] == 0.01                      # at target: unchanged, bit for bit
    assert out[1] == 0.02 * 0.5                # (1/8)^(2/3) = 1/4, clamped to 0.5
    assert out[2] == 0.04 * 2.0                # 8^(2/3) = 4, clamped to 2
    assert out[3] == 0.0 and out[4] == -1.0    # no radius: kept
    assert out[5] == 0.03 * 2.0 and out[6] == 0.05 * 2.0   # empty sphere counts as one
    wide = R.radius_update(np.array([0.01, 0.01, 0.01]), np.array([512, 0, 1]), 64, 0.01, 100.0)
    assert wide[0] == 0.01 * 0.25 and wide[1] == wide[2] == 0.01 * 16.0
    # the shrink of an overflowed row never grows it and never cuts below 1/4
    s = R.overflow_shrink(np.full(5, 0.08), np.array([65, 100, 512, 4096, 10 ** 6]), 64)
    assert (s < 0.08).all() and (s >= 0.02).all()
    assert s[2] == 0.08 * 0.25 and s[4] == 0.02


def test_radius_update_reaches_target_in_uniform_density():
    """Uniform random bodies: from radii holding a wide spread of counts, one
    unclamped update brings the mean count of interior rows to NNBOPT within
    the Poisson scatter (counts by a KD-tree, independent of the oracle)."""
    from scipy.spatial import cKDTree
    import oracle.radius as R
    rng = np.random.default_rng(805)
    n, nnbopt = 200000, 64
    x = rng.random((n, 3))
    tree = cKDTree(x)
    rows = np.nonzero((np.abs(x - 0.5) < 0.3).all(axis=1))[0][:3000]
    r0 = np.exp(rng.uniform(np.log(0.008), np.log(0.03), rows.size))
    c0 = np.array([len(v) - 1 for v in tree.query_ball_point(x[rows], r0)])
    ok = c0 > 4
    rs2 = R.radius_update(r0[ok] ** 2, c0[ok], nnbopt, 1e-6, 1e6)
    c1 = np.array([len(v) - 1 for v in tree.query_ball_point(x[rows[ok]], np.sqrt(rs2))])
    assert abs(c1.mean() / nnbopt - 1) < 0.04, c1.mean()
    assert np.median(np.abs(c0[ok] / nnbopt - 1)) > 0.5      # the start was far off
    assert np.median(np.abs(c1 / nnbopt - 1)) < 0.2


def test_regular_fit_invariants():
    """Overflowed rows are shrunk and recomputed until none overflows; rows
    that never overflowed keep radius and results; the final block equals a
    direct regular-force call with the final radii."""
    import oracle.radius as R
    s = W.small_state(811, 2000, k_nn=40)
    blk = np.arange(0, 2000, 3, dtype=np.int32)
    rs2 = s["rs2"][blk]
    c_true = oracle.regular(s["x"], s["v"], s["m"], blk, rs2, 400)[2]
    cap = int(np.percentile(c_true, 60))
    a0, j0, c0, l0, ovf0, _ = oracle.regular(s["x"], s["v"], s["m"], blk, rs2, cap)
    assert ovf0 == 1 and (c0 > cap).sum() > 100 and (c0 == cap).sum() > 5
    acc, jerk, cnt, lst, ovf, rs2f, rounds = R.regular_fit(s["x"], s["v"], s["m"], blk, rs2,
                                                            cap, cap - 4, 8)
    assert ovf == 0 and rounds >= 1 and (cnt <= cap).all()
    keep = c0 <= cap
    assert np.array_equal(rs2f[keep], rs2[keep])
    assert (rs2f[~keep] < rs2[~keep]).all()
    assert np.array_equal(acc[:, keep], a0[:, keep]) and np.array_equal(cnt[keep], c0[keep])
    d = oracle.regular(s["x"], s["v"], s["m"], blk, rs2f, cap)
    for got, ref in zip((acc, jerk, cnt, lst), d[:4]):
        assert np.array_equal(got, ref)
    # a round limit of 0 leaves the overflowing result as is
    r0 = R.regular_fit(s["x"], s["v"], s["m"], blk, rs2, cap, cap - 4, 0)
    assert r0[4] == 1 and r0[6] == 0 and np.array_equal(r0[5], rs2)
