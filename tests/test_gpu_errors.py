"""Error paths on the GPU: scratch that may not grow is reported as an error
and the context keeps working; argument errors surface as exceptions from the
binding before anything is launched."""
import numpy as np
import pytest
import torch

import paper_1504_03687_amd as nb
import workloads as W
from gpu_util import TOL_FP64, compare_force, dev, host, say

pytestmark = pytest.mark.gpu


def test_scratch_limit_reports_oom_then_recovers():
    say("scratch limit")
    s = W.small_state(31, 3001, k_nn=40)
    rng = np.random.default_rng(31)
    ib = rng.integers(0, 3001, 777).astype(np.int32)
    rs2 = s["rs2"][ib].copy()
    c = nb.Context(0)
    try:
        c.set_plan(1, 1, 8)                  # eight j-splits need split scratch
        c.set_scratch_limit(64 * 1024)
        args = (dev(s["x"]), dev(s["v"]), dev(s["m"]), dev(ib), dev(rs2), 48, "fp64")
        with pytest.raises(nb.NbError) as err:
            nb.regular_force(*args, ctx=c)
        assert err.value.code == -3
        c.set_scratch_limit(0)
        res = nb.regular_force(*args, ctx=c)
        compare_force(res, s["x"], s["v"], s["m"], ib, rs2, 48, TOL_FP64)
    finally:
        c.close()


def test_binding_rejects_bad_tensors():
    c = nb.Context(0)
    try:
        s = W.small_state(32, 200)
        x, v, m = dev(s["x"]), dev(s["v"]), dev(s["m"])
        ib = dev(np.arange(10, dtype=np.int32))
        rs2 = dev(s["rs2"][:10])
        with pytest.raises(ValueError):          # host tensor
            nb.regular_force(x, v, m, torch.arange(10, dtype=torch.int32), rs2, 8, ctx=c)
        with pytest.raises(ValueError):          # wrong dtype
            nb.regular_force(x.float(), v, m, ib, rs2, 8, ctx=c)
        with pytest.raises(ValueError):          # not contiguous
            nb.regular_force(x.t().contiguous().t(), v, m, ib, rs2, 8, ctx=c)
        with pytest.raises(ValueError):          # wrong shape
            nb.regular_force(x[:2].contiguous(), v, m, ib, rs2, 8, ctx=c)
        with pytest.raises(ValueError):          # negative list capacity
            nb.regular_force(x, v, m, ib, rs2, -1, ctx=c)
        with pytest.raises(nb.NbError) as err:   # library argument check
            nb.sched_build(dev(np.zeros(5, np.int32)), 64, ctx=c)
        assert err.value.code == -1
        with pytest.raises(nb.NbError):
            nb.radius_update(dev(np.ones(10, np.int32)), rs2, 0, ctx=c)
        with pytest.raises(nb.NbError):
            nb.sched_next(0.0, 3, [0, 0, 0, 0, 0])
        # the context still works afterwards
        res = nb.regular_force(x, v, m, ib, rs2, 8, "fp64", ctx=c)
        compare_force(res, s["x"], s["v"], s["m"], host(ib), host(rs2), 8, TOL_FP64)
    finally:
        c.close()


@pytest.mark.parametrize("batched", [False, True], ids=["single", "batched"])
def test_bad_out_tensors_raise_before_launch(batched):
    """Every caller-supplied output of a regular-force call is checked for
    shape, dtype, device and contiguity: a wrong one raises ValueError and
    nothing is written (the sentinel in the other outputs survives)."""
    say(f"bad out tensors ({'batched' if batched else 'single'})")
    c = nb.Context(0)
    try:
        s = W.small_state(33, 300)
        x, v, m = dev(s["x"]), dev(s["v"]), dev(s["m"])
        n_i, cap = 40, 16
        ib = dev(np.arange(n_i, dtype=np.int32))
        rs2 = dev(s["rs2"][:n_i])

        def good():
            return [torch.full((3, n_i), 7.0, dtype=torch.float64, device="cuda"),
                    torch.full((3, n_i), 7.0, dtype=torch.float64, device="cuda"),
                    torch.full((n_i,), 7, dtype=torch.int32, device="cuda"),
                    torch.full((n_i, cap), 7, dtype=torch.int32, device="cuda"),
                    torch.full((1,), 7, dtype=torch.int32, device="cuda")]

        def call(out):
            if batched:
                return nb.regular_force_batched([0, 300], [0, n_i], x, v, m, ib, rs2, cap,
                                                "mixed", out=out, ctx=c)
            return nb.regular_force(x, v, m, ib, rs2, cap, "mixed", out=out, ctx=c)

        bad_cases = [
            (3, lambda t: t[:, : cap - 1].contiguous()),         # list one entry short
            (3, lambda t: t[: n_i - 1].contiguous()),            # list one row short
            (0, lambda t: t[:, :-1].contiguous()),               # acc one row short
            (1, lambda t: t.float()),                            # jerk in FP32
            (2, lambda t: t.to(torch.int64)),                    # count as int64
            (4, lambda t: torch.zeros(2, dtype=torch.int32, device="cuda")),
            (0, lambda t: t.cpu()),                              # host tensor
            (3, lambda t: t.t().contiguous().t()),               # transposed view
        ]
        for k, mutate in bad_cases:
            out = good()
            out[k] = mutate(out[k])
            with pytest.raises(ValueError):
                call(out)
            torch.cuda.synchronize()
            for q, t in enumerate(out):
                if q != k:
                    assert bool((t == 7).all()), f"output {q} written after a bad output {k}"
        with pytest.raises(ValueError):   # wrong number of outputs
            call(good()[:4])
        # the right outputs work
        out = good()
        res = call(out)
        torch.cuda.synchronize()
        assert res[0].data_ptr() == out[0].data_ptr()
        compare_force(res, s["x"], s["v"], s["m"], np.arange(n_i, dtype=np.int32),
                      s["rs2"][:n_i], cap, 5e-6)
    finally:
        c.close()
