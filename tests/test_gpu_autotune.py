"""Autotuner: tunes at a small n, writes and reloads its table, and the plans
it installs give the same (oracle-checked) results as the automatic ones."""
import os

import numpy as np
import pytest

import paper_1504_03687_amd as nb
import workloads as W
from gpu_util import TOL_FP64, TOL_MIXED, compare_force, dev, say

pytestmark = pytest.mark.gpu


def test_autotune_roundtrip_and_parity(tmp_path):
    ctx = nb.Context(0)
    try:
        path = str(tmp_path / "tune.txt")
        nb.autotune(8192, path, force=True, ctx=ctx)
        with open(path) as f:
            lines = f.read().splitlines()
        assert lines[0] == "nbreg-tune 2" and len(lines) > 4
        say(f"autotune table: {len(lines) - 1} entries")
        # a fresh context loads the table without re-timing
        ctx2 = nb.Context(0)
        nb.autotune(8192, path, ctx=ctx2)
        s = W.small_state(300, 8192, k_nn=48)
        for n_i in (1, 20, 300, 5000):
            ib = np.random.default_rng(n_i).choice(8192, n_i, replace=False).astype(np.int32)
            for prec, tol in (("fp64", TOL_FP64), ("mixed", TOL_MIXED)):
                res = nb.regular_force(dev(s["x"]), dev(s["v"]), dev(s["m"]), dev(ib),
                                       dev(s["rs2"][ib]), 64, prec, ctx=ctx2)
                compare_force(res, s["x"], s["v"], s["m"], ib, s["rs2"][ib], 64, tol)
                say(f"  n_i={n_i} {prec}: {ctx2.last_plan()}")
        ctx2.close()
    finally:
        ctx.close()
