"""Plain CPU oracle of neighbour-radius control (numpy, FP64).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``; nothing in the product path
imports it.  It shares no code with the HIP library.

The paper states only that the neighbour number is steered toward the input
parameter NNBOPT (Table A1, "Neighbor criterion"), and that neighbour lists
are gathered by the GPU regular-force pass (section 3.2.1).  The rule written
out here is the uniform-density reading: a sphere holding `count` bodies
holds `target` bodies when its volume is scaled by target/count, so the
squared radius scales by (target/count)^(2/3).  The factor is clamped per
step; a row with no radius (rs2 <= 0) keeps it.

The 2/3 power is a cube root of q*q by a fixed number of Newton steps from a
power-of-two start, every operation an IEEE-rounded +, -, *, / or an exact
frexp/ldexp, in the order given below, so any implementation that follows the
same steps gets the same bits.

Functions:
  pow23(q)           -- q^(2/3) by the steps above
  radius_update      -- next-step squared radius toward NNBOPT
  overflow_shrink    -- squared radius of a row whose list overflowed
  regular_fit        -- regular force with overflowed rows shrunk and
                        recomputed until no row overflows (or a round limit)

Parity status (pinned in tests/test_oracle_pins.py): pow23 against 50-digit
Decimal cube roots (within 2 ulp); the update and shrink rules by their clamp
and fixed-point cases and by a uniform-density count test; regular_fit by its
invariants (no overflow left, untouched rows unchanged, recomputed rows equal
a direct regular-force call with the final radii).
"""
from __future__ import annotations

import numpy as np

NEWTON_STEPS = 8
SHRINK_MIN = 0.25     # largest per-round shrink of rs2 for an overflowed row


def pow23(q):
    """q^(2/3) for q > 0 (array), as cbrt(q*q): start from 2^floor(e/3) where
    q*q = f 2^e with f in [0.5, 1), then NEWTON_STEPS steps of
    y <- y - (y*y*y - x) / (3*y*y), evaluated as t = y*y; y - (t*y - x)/(3*t)."""
    q = np.asarray(q, np.float64)
    x = q * q
    _, e = np.frexp(x)
    k = np.floor_divide(e, 3)
    y = np.ldexp(np.ones_like(x), k)
    for _ in range(NEWTON_STEPS):
        t = y * y
        y = y - (t * y - x) / (3.0 * t)
    return y


def radius_update(rs2, count, nnbopt: int, f_min: float, f_max: float):
    """Squared radius for the next step: rs2 * clamp((nnbopt / max(count, 1))^(2/3),
    f_min, f_max); rows with rs2 <= 0 are returned unchanged."""
    rs2 = np.asarray(rs2, np.float64)
    c = np.maximum(np.asarray(count, np.int64), 1).astype(np.float64)
    f = np.minimum(np.maximum(pow23(float(nnbopt) / c), f_min), f_max)
    return np.where(rs2 > 0, rs2 * f, rs2)


def overflow_shrink(rs2, count, target: int):
    """Squared radius of a row with count > cap neighbours, aiming at target
    (= min(NNBOPT, cap)): rs2 * clamp((target / count)^(2/3), SHRINK_MIN, 1)."""
    rs2 = np.asarray(rs2, np.float64)
    c = np.asarray(count, np.int64).astype(np.float64)
    f = np.minimum(np.maximum(pow23(float(target) / c), SHRINK_MIN), 1.0)
    return rs2 * f


def regular_fit(xp, vp, m, i_block, rs2, nb_cap: int, nnbopt: int, max_rounds: int):
    """Regular force of the block; then, while some row has more than nb_cap
    neighbours and fewer than max_rounds rounds were made, shrink those rows'
    squared radii (overflow_shrink, target min(nnbopt, nb_cap)) and recompute
    them.  Returns (acc, jerk, count, list, overflow, rs2, rounds)."""
    from oracle import regular
    rs2 = np.array(rs2, np.float64, copy=True)
    i_block = np.asarray(i_block, np.int32)
    acc, jerk, cnt, lst, ovf, _ = regular(xp, vp, m, i_block, rs2, nb_cap)
    target = min(int(nnbopt), int(nb_cap))
    rounds = 0
    while ovf and rounds < max_rounds:
        rows = np.nonzero(cnt > nb_cap)[0]
        rs2[rows] = overflow_shrink(rs2[rows], cnt[rows], target)
        a2, j2, c2, l2, ovf, _ = regular(xp, vp, m, i_block[rows], rs2[rows], nb_cap)
        acc[:, rows] = a2
        jerk[:, rows] = j2
        cnt[rows] = c2
        lst[rows] = l2
        rounds += 1
    return acc, jerk, cnt, lst, int(ovf), rs2, rounds
