"""Plain CPU oracle of active-body selection for hierarchical block time steps.

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` and the CPU-baseline leg of
``bench.py``; nothing in the product path imports it.  It shares no code with
the HIP library.

Definitions followed (Wang et al. 2015, section 2 and section 3.3.1):
  * every body i has a time t_i and a step dt_i = 2^-level_i; the block time
    steps are synchronised, so t_i is a multiple of dt_i;
  * the next block time is the earliest t_i + dt_i over all bodies, and the
    active bodies are every body due at that time (``next_block``: the plain
    O(N) search over all bodies that the sorting list replaces);
  * the sorting list is the body index list ordered by step from the smallest
    step to the largest, with the boundary offset of each step block
    (``sort_list``); the paper's I_off(i), the last list position holding a
    body of step 0.5^i, is level_end[i] - 1 here;
  * the coarsest level whose step divides a block time (``due_level``) picks
    the offset: bodies of that level and every deeper one are due.

Parity status (pinned in tests/test_oracle_pins.py): sort_list by a hand-worked
golden list, pairwise order checks and bucket counts; next_block and
due_level by an exact rational block-step simulation.
"""
from __future__ import annotations

import math

import numpy as np


def sort_list(level, k_max: int):
    """(order, level_end): ``order`` lists body indices by step from smallest
    to largest (level descending), bodies of equal level by ascending index;
    ``level_end[L]`` (L = 0 .. k_max+1) = number of bodies with level >= L, so
    the bodies of level L sit at order[level_end[L+1] : level_end[L]]."""
    level = np.asarray(level, dtype=np.int64)
    if level.size and (level.min() < 0 or level.max() > k_max):
        raise ValueError("level outside [0, k_max]")
    idx = np.arange(level.size, dtype=np.int64)
    order = np.lexsort((idx, -level)).astype(np.int32)
    counts = np.bincount(level, minlength=k_max + 1)
    level_end = np.zeros(k_max + 2, np.int32)
    level_end[: k_max + 1] = np.cumsum(counts[::-1])[::-1]
    return order, level_end


def next_block(t, dt):
    """Earliest next update time over all bodies and the bodies due then
    (ascending index): T_new = min_i (t_i + dt_i), active = {i : t_i + dt_i ==
    T_new}.  Times and steps are dyadic, so the sums are exact in FP64."""
    nxt = np.asarray(t, np.float64) + np.asarray(dt, np.float64)
    t_new = float(nxt.min())
    return t_new, np.nonzero(nxt == t_new)[0].astype(np.int32)


def due_level(t: float, k_max: int) -> int:
    """Smallest L in [0, k_max] such that t is a whole multiple of 2^-L (t > 0);
    -1 if t is not a multiple of 2^-k_max."""
    for L in range(k_max + 1):
        q = math.ldexp(t, L)
        if q == math.floor(q):
            return L
    return -1
