"""GPU parity of the sorting-list scheduler (section 3.3.1) against the CPU
oracle: the full build is compared bit for bit (list and offsets); after each
update the offsets and the set of bodies of every level are compared (the
order inside a level after an update is free), and the prefix selected for
every block equals the oracle's brute-force search over all bodies."""
import numpy as np
import pytest
import torch

import oracle
import oracle.sched as S
import paper_1504_03687_amd as nb
import workloads as W
from gpu_util import compare_force, dev, host, say, TOL_FP64

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = nb.Context(0)
    yield c
    c.close()


def _levels(seed, n, k_max):
    rng = np.random.default_rng(seed)
    if k_max < 4:
        return rng.integers(0, k_max + 1, n).astype(np.int32)
    return W.sample_levels(rng, n, 0, k_max, k_peak=min(10, k_max - 2))


def _segments_match(order, le, lev, k_max):
    """Offsets equal the oracle's, and every level block of the list holds
    exactly the bodies of that level."""
    o_order, o_le = S.sort_list(lev, k_max)
    assert np.array_equal(le, o_le), (le, o_le)
    assert np.array_equal(np.sort(order), np.arange(lev.size))
    # list position p lies in the block of level L iff le[L+1] <= p < le[L]
    pos_lev = np.empty(lev.size, np.int64)
    for L in range(k_max + 1):
        pos_lev[le[L + 1]: le[L]] = L
    assert np.array_equal(lev[order], pos_lev)


@pytest.mark.parametrize("n,k_max", [(1, 0), (1000, 5), (4095, 20), (4096, 20), (4097, 20),
                                     (8192, 20), (16384, 20), (16385, 20), (300001, 22), (1 << 20, 63)])
def test_build_bitwise(ctx, n, k_max):
    say(f"sched build n={n} k_max={k_max}")
    lev = _levels(900 + n, n, k_max)
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    order, le = nb.sched_build(dev(lev), k_max, status=st, ctx=ctx)
    torch.cuda.synchronize()
    o_order, o_le = S.sort_list(lev, k_max)
    assert int(st.item()) == 0
    assert np.array_equal(host(le), o_le)
    assert np.array_equal(host(order), o_order)


def test_build_single_level_and_all_distinct(ctx):
    n = 64 * 1024 + 7
    lev = np.full(n, 9, np.int32)
    order, le = nb.sched_build(dev(lev), 9, ctx=ctx)
    assert np.array_equal(host(order), np.arange(n))
    assert host(le).tolist() == [n] * 10 + [0]
    lev = (np.arange(64) % 64).astype(np.int32)[::-1].copy()
    order, le = nb.sched_build(dev(lev), 63, ctx=ctx)
    o_order, o_le = S.sort_list(lev, 63)
    assert np.array_equal(host(order), o_order) and np.array_equal(host(le), o_le)


def test_build_bad_level_leaves_list(ctx):
    n, k_max = 5000, 10
    lev = _levels(931, n, k_max)
    lev[4321] = k_max + 1
    order = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    le = torch.full((k_max + 2,), -7, dtype=torch.int32, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    nb.sched_build(dev(lev), k_max, order=order, level_end=le, status=st, ctx=ctx)
    torch.cuda.synchronize()
    assert int(st.item()) & nb.STATUS_BAD_LEVEL
    assert (host(order) == -7).all() and (host(le) == -7).all()
    lev[4321] = -1
    st.zero_()
    nb.sched_build(dev(lev), k_max, order=order, level_end=le, status=st, ctx=ctx)
    torch.cuda.synchronize()
    assert int(st.item()) & nb.STATUS_BAD_LEVEL and (host(order) == -7).all()


@pytest.mark.parametrize("n,k_lo,k_max,steps", [(50000, 2, 9, 260), (3001, 4, 20, 400)])
def test_block_step_sequence(ctx, n, k_lo, k_max, steps):
    """A synchronised block-step run: at every block the host offset search
    picks the prefix, which must equal the oracle's brute-force active set;
    then the active bodies get new levels and the list is updated on the GPU."""
    say(f"sched sequence n={n} levels {k_lo}..{k_max}")
    rng = np.random.default_rng(950 + n)
    lev = W.sample_levels(rng, n, k_lo, k_max, k_peak=k_lo + 3)
    t = np.zeros(n)
    t_now = 0.0
    g_lev = dev(lev)
    order, le = nb.sched_build(g_lev, k_max, ctx=ctx)
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    sizes = []
    for step in range(steps):
        le_h = host(le)
        t_new, L, n_a = nb.sched_next(t_now, k_max, le_h)
        ot, act = S.next_block(t, np.ldexp(1.0, -lev.astype(np.int64)))
        assert t_new == ot and L == S.due_level(ot, k_max) and n_a == act.size, step
        pre = host(order[:n_a])
        assert np.array_equal(np.sort(pre), act), f"step {step}: active set differs"
        sizes.append(n_a)
        new = W.next_levels(rng, lev[act], L, k_max)
        lev[act] = new
        g_lev[torch.from_numpy(act.astype(np.int64)).cuda()] = torch.from_numpy(new).cuda()
        nb.sched_update(order, le, n_a, L, g_lev, k_max, status=st, ctx=ctx)
        t[act] = t_new
        t_now = t_new
        if step % 16 == 0 or n_a > 4096:
            _segments_match(host(order), host(le), lev, k_max)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    _segments_match(host(order), host(le), lev, k_max)
    say(f"  blocks: {len(sizes)}, n_active min {min(sizes)} max {max(sizes)}")
    assert max(sizes) > 4096 or n < 4096


@pytest.mark.parametrize("L", [5, 8])
def test_update_rejects_bad_input(ctx, L):
    """Both the one-work-group path (block <= 16384) and the multi-work-group
    path leave the list untouched on bad input."""
    n, k_max = 20000, 12
    rng = np.random.default_rng(977)
    lev = W.sample_levels(rng, n, 3, k_max, k_peak=6)
    g_lev = dev(lev)
    order, le = nb.sched_build(g_lev, k_max, ctx=ctx)
    o0, l0 = host(order), host(le)
    n_a = int(l0[L])
    assert (n_a > 16384) == (L == 5), n_a
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    # a new level coarser than the block level
    bad = g_lev.clone()
    bad[int(o0[n_a // 2])] = L - 1
    nb.sched_update(order, le, n_a, L, bad, k_max, status=st, ctx=ctx)
    torch.cuda.synchronize()
    assert int(st.item()) & nb.STATUS_BAD_LEVEL
    assert np.array_equal(host(order), o0) and np.array_equal(host(le), l0)
    # a prefix that is not the due block
    st.zero_()
    nb.sched_update(order, le, n_a - 1, L, g_lev, k_max, status=st, ctx=ctx)
    torch.cuda.synchronize()
    assert int(st.item()) & nb.STATUS_BAD_LEVEL
    assert np.array_equal(host(order), o0) and np.array_equal(host(le), l0)
    # the valid call still works afterwards
    st.zero_()
    nb.sched_update(order, le, n_a, L, g_lev, k_max, status=st, ctx=ctx)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    _segments_match(host(order), host(le), lev, k_max)


def test_prefix_is_the_force_block(ctx):
    """The selected prefix is passed to the regular force as i_block as is."""
    s = W.small_state(985, 3000, k_nn=24)
    rng = np.random.default_rng(986)
    lev = W.sample_levels(rng, 3000, 3, 12, k_peak=6)
    order, le = nb.sched_build(dev(lev), 12, ctx=ctx)
    kd = int(lev.max())
    t_new, L, n_a = nb.sched_next(0.09375 - 2.0 ** -kd, 12, host(le))   # next block 3/32
    assert t_new == 0.09375 and L == 5 and 0 < n_a < 3000
    blk = order[:n_a]
    xp, vp, m = dev(s["x"]), dev(s["v"]), dev(s["m"])
    rs2 = dev(s["rs2"])[blk.long()].contiguous()
    res = nb.regular_force(xp, vp, m, blk, rs2, 64, "fp64", ctx=ctx)
    compare_force(res, s["x"], s["v"], s["m"], host(blk), host(rs2), 64, TOL_FP64)
    assert np.array_equal(np.sort(host(blk)), np.nonzero(lev >= L)[0])


def test_bench_configuration_levels(ctx):
    """The scheduler as the benchmark runs it: the N = 2^20 binary cluster's own step levels
    (2^20 bodies, levels 3..20, k_max 20): the build is the oracle's list bit
    for bit, and each level's update keeps every level block's members."""
    s = W.binary_cluster_n1m()
    lev = s["levels"].astype(np.int32)
    k_max = 20
    g_lev = dev(lev)
    order, le = nb.sched_build(g_lev, k_max, ctx=ctx)
    o_order, o_le = S.sort_list(lev, k_max)
    assert np.array_equal(host(order), o_order) and np.array_equal(host(le), o_le)
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    for L in (20, 14, 5, 3):
        nb.sched_update(order, le, int(o_le[L]), L, g_lev, k_max, status=st, ctx=ctx)
        _segments_match(host(order), host(le), lev, k_max)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
