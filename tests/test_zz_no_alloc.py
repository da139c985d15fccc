"""The allocation-free regular-force entry point (nb_regular_force_noalloc):
same outputs as nb_regular_force through the C ABI, with the library's fixed
device workspace instead of context scratch, on consecutive calls of
different sizes (the workspace keeps the previous call's contents)."""
import numpy as np
import pytest
import torch

import paper_1504_03687_amd as nb
import workloads as W
from gpu_util import TOL_FP64, TOL_MIXED, check_lists, compare_force, dev, host, say

pytestmark = pytest.mark.gpu


def _out(n_i, cap):
    return (torch.empty((3, n_i), dtype=torch.float64, device="cuda"),
            torch.empty((3, n_i), dtype=torch.float64, device="cuda"),
            torch.empty(n_i, dtype=torch.int32, device="cuda"),
            torch.empty((n_i, cap), dtype=torch.int32, device="cuda"),
            torch.empty(1, dtype=torch.int32, device="cuda"))


def _same(a, b, cap, tol, bitwise):
    """Outputs of the two entry points: counts, lists and overflow bit for
    bit; forces bit for bit when both ran the same plan, else within tol."""
    ha = [host(t) for t in a]
    hb = [host(t) for t in b]
    check_lists(ha[2], ha[3], hb[2], hb[3], cap)
    assert int(ha[4][0]) == int(hb[4][0])
    for k in (0, 1):
        if bitwise:
            assert np.array_equal(ha[k], hb[k])
        else:
            d = np.linalg.norm(ha[k] - hb[k], axis=0)
            r = np.linalg.norm(hb[k], axis=0)
            assert np.all(d <= tol * np.where(r > 0, r, 1.0))


@pytest.mark.parametrize("prec,tol", [("fp64", TOL_FP64), ("mixed", TOL_MIXED)])
def test_noalloc_matches_regular_force_on_two_calls(prec, tol):
    s = W.small_state(71, 3001, k_nn=40)
    xp, vp, m = dev(s["x"]), dev(s["v"]), dev(s["m"])
    rng = np.random.default_rng(71)
    cap = 48
    ctx = nb.Context(0)
    try:
        # the context may not allocate: every byte of workspace must come from
        # the library's fixed array
        ctx.set_scratch_limit(1)
        for n_i, splits in ((2000, 6), (700, 3)):   # second call smaller
            ib = rng.integers(0, 3001, n_i).astype(np.int32)
            rs2 = s["rs2"][ib].copy()
            rs2[::97] = 0.0                           # rows without neighbours
            say(f"noalloc {prec}: n_i={n_i} splits={splits}")
            ctx.set_plan(1, 1, splits)
            got = nb.regular_force_noalloc(xp, vp, m, dev(ib), dev(rs2), cap, prec,
                                           out=_out(n_i, cap), ctx=ctx)
            plan_fixed = ctx.last_plan()
            assert "workspace=fixed" in plan_fixed
            with pytest.raises(nb.NbError) as err:   # context scratch is capped
                nb.regular_force(xp, vp, m, dev(ib), dev(rs2), cap, prec, ctx=ctx)
            assert err.value.code == -3
            ref_ctx = nb.Context(0)
            try:
                ref_ctx.set_plan(1, 1, splits)
                ref = nb.regular_force(xp, vp, m, dev(ib), dev(rs2), cap, prec, ctx=ref_ctx)
                plan_ref = ref_ctx.last_plan()
            finally:
                ref_ctx.close()
            torch.cuda.synchronize()
            assert plan_fixed.replace(" workspace=fixed", "") == plan_ref
            _same(got, ref, cap, tol, bitwise=True)
            compare_force(got, s["x"], s["v"], s["m"], ib, rs2, cap, tol)
    finally:
        ctx.close()


@pytest.mark.parametrize("prec,tol", [("fp64", TOL_FP64), ("mixed", TOL_MIXED)])
def test_noalloc_lowers_splits_to_fit_the_workspace(prec, tol):
    """A block whose automatic plan needs far more split scratch than the
    fixed workspace holds: the call runs with fewer splits, and a smaller
    block right after it runs with its own plan."""
    s = W.small_state(72, 131072, k_nn=64)
    xp, vp, m = dev(s["x"]), dev(s["v"]), dev(s["m"])
    rng = np.random.default_rng(72)
    cap = 96
    ws = nb.fixed_workspace_bytes()
    assert ws >= 1 << 20
    ctx = nb.Context(0)
    try:
        ctx.set_scratch_limit(1)
        # wide tolerance band: many rows take the FP64 refinement path, whose
        # row lists and chunk partials then live in the workspace too
        if prec == "mixed":
            ctx.set_mixed_tolerance(5e-7, 32.0)
        for n_i in (16384, 1024):
            ib = rng.choice(131072, n_i, replace=False).astype(np.int32)
            rs2 = s["rs2"][ib].copy()
            say(f"noalloc fit {prec}: n_i={n_i}")
            got = nb.regular_force_noalloc(xp, vp, m, dev(ib), dev(rs2), cap, prec,
                                           out=_out(n_i, cap), ctx=ctx)
            plan = ctx.last_plan()
            splits = int(plan.split("splits=")[1].split()[0])
            assert splits * n_i * (64 + 4 + 4 * 96) <= ws, plan
            ref_ctx = nb.Context(0)
            try:
                if prec == "mixed":
                    ref_ctx.set_mixed_tolerance(5e-7, 32.0)
                ref = nb.regular_force(xp, vp, m, dev(ib), dev(rs2), cap, prec, ctx=ref_ctx)
                plan_ref = ref_ctx.last_plan()
            finally:
                ref_ctx.close()
            torch.cuda.synchronize()
            say(f"  fixed: {plan}; context scratch: {plan_ref}")
            # different split counts: each side is within tol of the exact
            # sums (checked against the oracle below), so within 2 tol of
            # each other
            _same(got, ref, cap, 2 * tol, bitwise=False)
            rows = rng.choice(n_i, 256, replace=False)
            compare_force(got, s["x"], s["v"], s["m"], ib, rs2, cap, tol, rows=rows)
    finally:
        ctx.close()


def test_noalloc_rejects_blocks_beyond_the_workspace():
    """Mixed blocks need 12 bytes of refinement bookkeeping per row in the
    workspace; a block of more rows than fit is refused before any launch."""
    ws = nb.fixed_workspace_bytes()
    n_i = ws // 12 + 4096
    s = W.small_state(73, 64, k_nn=8)
    xp, vp, m = dev(s["x"]), dev(s["v"]), dev(s["m"])
    ib = torch.zeros(n_i, dtype=torch.int32, device="cuda")
    rs2 = torch.zeros(n_i, dtype=torch.float64, device="cuda")
    out = _out(n_i, 0)
    out[4].fill_(7)
    ctx = nb.Context(0)
    try:
        with pytest.raises(nb.NbError) as err:
            nb.regular_force_noalloc(xp, vp, m, ib, rs2, 0, "mixed", out=out, ctx=ctx)
        assert err.value.code == -5
        torch.cuda.synchronize()
        assert int(out[4].item()) == 7          # nothing was launched
        # the same block in FP64 needs no workspace at one split
        ctx.set_plan(1, 1, 1)
        nb.regular_force_noalloc(xp, vp, m, ib, rs2, 0, "fp64", out=out, ctx=ctx)
        torch.cuda.synchronize()
        assert int(out[4].item()) == 0
        compare_force(out, s["x"], s["v"], s["m"], np.zeros(n_i, np.int32),
                      np.zeros(n_i), 0, TOL_FP64, rows=[0, n_i // 2, n_i - 1])
    finally:
        ctx.close()
