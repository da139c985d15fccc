"""Runtime behaviour on the GPU: calls launch on torch's current stream (a
side stream works and is ordered by that stream alone), and the per-class
kernel timing counts the launches of each class."""
import numpy as np
import pytest
import torch

import paper_1504_03687_amd as nb
import workloads as W
from gpu_util import TOL_FP64, TOL_MIXED, compare_force, dev, host, say

pytestmark = pytest.mark.gpu


def test_side_stream():
    say("side stream")
    s = W.small_state(401, 4000, k_nn=32)
    ib = np.arange(0, 4000, 3, dtype=np.int32)
    c = nb.Context(0)
    side = torch.cuda.Stream()                    # default priority
    try:
        x, v, m, bd, r = dev(s["x"]), dev(s["v"]), dev(s["m"]), dev(ib), dev(s["rs2"][ib])
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            res = nb.regular_force(x, v, m, bd, r, 64, "mixed", ctx=c)
            irr = nb.irregular_force(x, v, m, bd, 64, res[2], res[3], ctx=c)
        side.synchronize()
        compare_force(res, s["x"], s["v"], s["m"], ib, s["rs2"][ib], 64, TOL_MIXED)
        # the same context back on the default stream
        res2 = nb.regular_force(x, v, m, bd, r, 64, "fp64", ctx=c)
        compare_force(res2, s["x"], s["v"], s["m"], ib, s["rs2"][ib], 64, TOL_FP64)
        assert np.isfinite(host(irr[0])).all()
    finally:
        c.close()


def test_kernel_timing_counts_launches():
    s = W.small_state(402, 3000, k_nn=32)
    ib = np.arange(3000, dtype=np.int32)
    c = nb.Context(0)
    try:
        x, v, m, bd, r = dev(s["x"]), dev(s["v"]), dev(s["m"]), dev(ib), dev(s["rs2"][ib])
        c.enable_timing(True)
        c.reset_timing()
        c.set_plan(1, 1, 3)                        # a split plan: force + merge
        for _ in range(3):
            nb.regular_force(x, v, m, bd, r, 64, "fp64", ctx=c)
        c.set_plan(0, 0, 0)
        nb.predict(x, v, x, v, dev(np.zeros(3000)), 0.0, ctx=c)
        nb.potential(x, m, ctx=c)
        ms, k = c.kernel_time(nb.CLASS_FORCE)
        assert k == 3 and ms > 0
        assert c.kernel_time(nb.CLASS_MERGE)[1] == 3
        assert c.kernel_time(nb.CLASS_PREDICT)[1] == 1
        assert c.kernel_time(nb.CLASS_STEP)[1] == 1
        assert c.kernel_time(nb.CLASS_BATCHED)[1] == 0
        c.reset_timing()
        assert c.kernel_time(nb.CLASS_FORCE) == (0.0, 0)
        c.enable_timing(False)
        nb.regular_force(x, v, m, bd, r, 64, "fp64", ctx=c)
        assert c.kernel_time(nb.CLASS_FORCE)[1] == 0
    finally:
        c.close()
