"""GPU parity of the predictor and the regular-force kernels against the CPU
oracle, through the C ABI (via the ctypes binding).

Bars: predictor and neighbour lists/counts bit-exact; acc/jerk per-row
relative error <= 1e-12 (FP64 kernels) and <= 5e-6 (mixed kernels).
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1504_03687_amd as nb
import workloads as W
from gpu_util import (TOL_FP64, TOL_MIXED, oracle_rows, check_lists, compare_force, dev, host, row_rel_err,
                      say)

pytestmark = pytest.mark.gpu

TOL = {"fp64": TOL_FP64, "mixed": TOL_MIXED}


@pytest.fixture(scope="module")
def ctx():
    c = nb.Context(0)
    yield c
    c.close()


def _predict_dev(ctx, s):
    xp, vp, m32 = nb.predict(dev(s["x"]), dev(s["v"]), dev(s["a"]), dev(s["jk"]), dev(s["t0"]),
                             s["t"], m=dev(s["m"]), ctx=ctx)
    return xp, vp, m32


@pytest.mark.parametrize("n", [1, 257, 4099])
def test_predict_bitwise(ctx, n):
    say(f"predict n={n}")
    rng = np.random.default_rng(n)
    x, v, a, jk = (rng.standard_normal((3, n)) for _ in range(4))
    t0 = -np.ldexp(1.0, -rng.integers(3, 20, n))
    m = rng.random(n)
    s = dict(x=x, v=v, a=a, jk=jk, t0=t0, t=0.375, m=m)
    xp, vp, m32 = _predict_dev(ctx, s)
    torch.cuda.synchronize()
    ox, ov = oracle.predict(0.375, x, v, a, jk, t0)
    assert np.array_equal(host(xp), ox) and np.array_equal(host(vp), ov)
    assert np.array_equal(host(m32), m.astype(np.float32))
    # in place
    xd, vd = dev(x), dev(v)
    nb.predict(xd, vd, dev(a), dev(jk), dev(t0), 0.375, out=(xd, vd), ctx=ctx)
    torch.cuda.synchronize()
    assert np.array_equal(host(xd), ox) and np.array_equal(host(vd), ov)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_plummer_n1024_all_active(ctx, prec):
    """N = 1024 equal-mass Plummer, every body active, nb_cap 256."""
    say(f"plummer N=1024 {prec}")
    s = W.plummer_equal_n1024()
    xp, vp, _ = _predict_dev(ctx, s)
    ox, ov = oracle.predict(s["t"], s["x"], s["v"], s["a"], s["jk"], s["t0"])
    assert np.array_equal(host(xp), ox) and np.array_equal(host(vp), ov)
    res = nb.regular_force(xp, vp, dev(s["m"]), dev(s["i_block"]), dev(s["rs2"]), s["nb_cap"],
                           prec, ctx=ctx)
    ea, ej = compare_force(res, ox, ov, s["m"], s["i_block"], s["rs2"], s["nb_cap"], TOL[prec])
    say(f"  plan {ctx.last_plan()}  max err acc {ea:.2e} jerk {ej:.2e}")


PLANS = [(1, 1, 1), (1, 2, 1), (1, 4, 1), (1, 1, 3), (1, 2, 5), (1, 4, 2),
         (2, 1, 1), (2, 2, 4), (2, 4, 7), (2, 4, 1), (2, 1, 13), (3, 1, 1), (3, 1, 5),
         (3, 1, 40)]


def _ragged_case(seed=31, n=3001, n_i=777):
    s = W.small_state(seed, n, k_nn=40)
    rng = np.random.default_rng(seed)
    ib = rng.integers(0, n, n_i).astype(np.int32)     # duplicates allowed
    ib[5] = ib[6]
    rs2 = s["rs2"][ib].copy()
    rs2[10] = 0.0
    rs2[11] = -1.0
    rs2[12] = s["rs2"].max() * 6                      # many neighbours
    return s, ib, rs2


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("plan", PLANS, ids=lambda p: "m%d-r%d-s%d" % p)
def test_plans_ragged(ctx, plan, prec):
    say(f"plan {plan} {prec}")
    s, ib, rs2 = _ragged_case()
    ctx.set_plan(*plan)
    try:
        for cap in (48, 0):
            res = nb.regular_force(dev(s["x"]), dev(s["v"]), dev(s["m"]), dev(ib), dev(rs2), cap,
                                   prec, ctx=ctx)
            compare_force(res, s["x"], s["v"], s["m"], ib, rs2, cap, TOL[prec])
    finally:
        ctx.set_plan(0, 0, 0)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_merge_group_widths(ctx, prec):
    """Split counts on both sides of the merge's lane-group widths (4, 16 and
    64 lanes per row, and more splits than lanes), a ragged block of 777 rows
    (partial groups and waves) and a cap small enough to truncate lists."""
    n = 17308   # 68 tiles of 256: the requests below land on distinct counts
    s = W.small_state(41, n, k_nn=40)
    rng = np.random.default_rng(41)
    ib = rng.integers(0, n, 777).astype(np.int32)
    rs2 = s["rs2"][ib].copy()
    seen = set()
    try:
        for req in (2, 4, 5, 16, 17, 64, 68):
            ctx.set_plan(1, 1, req)
            say(f"merge widths {prec} splits requested {req}")
            for cap in (64, 8):
                res = nb.regular_force(dev(s["x"]), dev(s["v"]), dev(s["m"]), dev(ib), dev(rs2),
                                       cap, prec, ctx=ctx)
                compare_force(res, s["x"], s["v"], s["m"], ib, rs2, cap, TOL[prec])
            seen.add(int(ctx.last_plan().split("splits=")[1].split()[0]))
    finally:
        ctx.set_plan(0, 0, 0)
    assert {2, 4, 5, 14, 17, 34, 68} <= seen, seen


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_bad_rows_in_merge_groups(ctx, prec):
    """Rows with out-of-range body indices next to valid rows, merged by 4-,
    16- and 64-lane groups: the bad rows get zero acc/jerk, count 0 and the
    status bit; the valid rows match the oracle."""
    n = 17308
    s = W.small_state(43, n, k_nn=32)
    rng = np.random.default_rng(43)
    ib = rng.integers(0, n, 300).astype(np.int32)
    bad = np.array([0, 1, 17, 64, 65, 299])
    ib[bad[::2]] = -1
    ib[bad[1::2]] = n + 3
    rs2 = s["rs2"][np.clip(ib, 0, n - 1)]
    good = np.setdiff1d(np.arange(ib.size), bad)
    try:
        for req in (3, 12, 40):
            ctx.set_plan(1, 1, req)
            say(f"bad rows {prec} splits requested {req}")
            st = torch.zeros(1, dtype=torch.int32, device="cuda")
            res = nb.regular_force(dev(s["x"]), dev(s["v"]), dev(s["m"]), dev(ib), dev(rs2), 32,
                                   prec, status=st, ctx=ctx)
            torch.cuda.synchronize()
            assert int(st.item()) & nb.STATUS_BAD_INDEX
            acc, jerk, cnt = host(res[0]), host(res[1]), host(res[2])
            assert not acc[:, bad].any() and not jerk[:, bad].any() and not cnt[bad].any()
            compare_force(res, s["x"], s["v"], s["m"], ib, rs2, 32, TOL[prec], rows=good)
    finally:
        ctx.set_plan(0, 0, 0)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_segment_rebuild(ctx, prec):
    """Rows with hundreds of neighbours per j-range overflow the per-split
    scratch segments; the merge must rebuild them in ascending order."""
    say(f"segment rebuild {prec}")
    s = W.small_state(41, 5000, k_nn=32)
    ib = np.arange(0, 5000, 9, dtype=np.int32)
    rs2 = np.full(ib.size, np.quantile(s["rs2"], 0.5) * 8)
    for plan in ((1, 1, 2), (1, 2, 3), (2, 4, 3), (2, 1, 5)):
        ctx.set_plan(*plan)
        try:
            for cap in (150, 2000):
                res = nb.regular_force(dev(s["x"]), dev(s["v"]), dev(s["m"]), dev(ib), dev(rs2),
                                       cap, prec, ctx=ctx)
                compare_force(res, s["x"], s["v"], s["m"], ib, rs2, cap, TOL[prec])
        finally:
            ctx.set_plan(0, 0, 0)
    assert host(res[2]).max() > 200


def test_edge_cases(ctx):
    say("edge cases")
    s = W.small_state(51, 600)
    x, v, m = dev(s["x"]), dev(s["v"]), dev(s["m"])
    # bad indices give zero rows, count 0 and the status bit
    ib = np.array([3, 600, -1, 599, 3], np.int32)
    rs2 = s["rs2"][np.clip(ib, 0, 599)]
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    acc, jerk, cnt, lst, ovf = nb.regular_force(x, v, m, dev(ib), dev(rs2), 16, "fp64", status=st,
                                                ctx=ctx)
    torch.cuda.synchronize()
    assert int(st.item()) & nb.STATUS_BAD_INDEX
    assert not host(acc)[:, 1:3].any() and not host(jerk)[:, 1:3].any()
    assert host(cnt)[1] == 0 and host(cnt)[2] == 0
    assert np.array_equal(host(acc)[:, 0], host(acc)[:, 4])
    # empty block
    e = nb.regular_force(x, v, m, dev(np.zeros(0, np.int32)), dev(np.zeros(0)), 8, "mixed",
                         ctx=ctx)
    assert int(e[4].item()) == 0
    # a single body: no pairs at all
    one = nb.regular_force(dev(s["x"][:, :1]), dev(s["v"][:, :1]), dev(s["m"][:1]),
                           dev(np.zeros(1, np.int32)), dev(np.ones(1)), 4, "fp64", ctx=ctx)
    assert not host(one[0]).any() and host(one[2])[0] == 0
    # coincident distinct bodies outside each other's radius: non-finite flag
    x2 = s["x"][:, :4].copy()
    x2[:, 1] = x2[:, 0]
    st.zero_()
    bad = nb.regular_force(dev(x2), dev(s["v"][:, :4]), dev(s["m"][:4]),
                           dev(np.array([0], np.int32)), dev(np.zeros(1)), 4, "mixed",
                           status=st, ctx=ctx)
    torch.cuda.synchronize()
    assert int(st.item()) & nb.STATUS_NONFINITE


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_huge_and_infinite_radius(ctx, prec):
    """rs2 at or beyond the FP32 range (infinite after rounding): every other
    body is a neighbour and the force is exactly zero.  Padding bodies of a
    partial j-tile or past the end of a wave's j-range (far away, mass 0)
    must not enter the lists, for any plan."""
    say(f"huge radius {prec}")
    n = 1000   # partial 256-body tiles and partial 64-body wave ranges
    s = W.small_state(53, n, k_nn=16)
    ib = np.array([0, 17, 999, 500, 3, 3], np.int32)
    rs2 = np.array([np.inf, 1e300, 1e37, 3.5e38, s["rs2"][500], 0.0])
    try:
        for plan in ((1, 1, 1), (1, 2, 3), (2, 1, 1), (2, 4, 5), (0, 0, 0)):
            ctx.set_plan(*plan)
            for cap in (n, 100):
                res = nb.regular_force(dev(s["x"]), dev(s["v"]), dev(s["m"]), dev(ib), dev(rs2),
                                       cap, prec, ctx=ctx)
                compare_force(res, s["x"], s["v"], s["m"], ib, rs2, cap, TOL[prec])
                cnt = host(res[2])
                assert list(cnt[:4]) == [n - 1] * 4, (plan, cnt)
                assert not host(res[0])[:, :4].any() and not host(res[1])[:, :4].any()
    finally:
        ctx.set_plan(0, 0, 0)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_determinism_and_block_independence(ctx, prec):
    """A fixed plan gives bitwise-identical rows whatever else is in the block,
    and identical results on a re-run."""
    say(f"determinism {prec}")
    s = W.small_state(61, 4096, k_nn=48)
    x, v, m = dev(s["x"]), dev(s["v"]), dev(s["m"])
    full = np.arange(4096, dtype=np.int32)
    for plan in ((1, 1, 4), (2, 2, 8)):
        ctx.set_plan(*plan)
        try:
            a0 = [host(t) for t in nb.regular_force(x, v, m, dev(full), dev(s["rs2"]), 128, prec,
                                                   ctx=ctx)]
            a1 = [host(t) for t in nb.regular_force(x, v, m, dev(full), dev(s["rs2"]), 128, prec,
                                                   ctx=ctx)]
            for p, q in zip(a0, a1):
                assert np.array_equal(p, q)
            for sub in (np.array([1234], np.int32), np.arange(100, 132, dtype=np.int32)):
                r = [host(t) for t in nb.regular_force(x, v, m, dev(sub), dev(s["rs2"][sub]),
                                                      128, prec, ctx=ctx)]
                assert np.array_equal(r[0], a0[0][:, sub]) and np.array_equal(r[1], a0[1][:, sub])
                assert np.array_equal(r[2], a0[2][sub])
        finally:
            ctx.set_plan(0, 0, 0)


def test_power_of_two_scaling_fp64(ctx):
    """x -> 2x, rs2 -> 4 rs2 leaves the lists unchanged and scales acc by 1/4
    and jerk by 1/8 exactly in the FP64 kernels."""
    say("scaling")
    s = W.small_state(71, 2048, k_nn=32)
    ib = np.arange(2048, dtype=np.int32)
    base = [host(t) for t in nb.regular_force(dev(s["x"]), dev(s["v"]), dev(s["m"]), dev(ib),
                                              dev(s["rs2"]), 64, "fp64", ctx=ctx)]
    sc = [host(t) for t in nb.regular_force(dev(2 * s["x"]), dev(s["v"]), dev(s["m"]), dev(ib),
                                            dev(4 * s["rs2"]), 64, "fp64", ctx=ctx)]
    assert np.array_equal(base[2], sc[2]) and np.array_equal(base[3], sc[3])
    assert np.array_equal(sc[0], base[0] / 4) and np.array_equal(sc[1], base[1] / 8)


def test_plummer_kroupa_n131072_blocks(ctx):
    """N = 131072 Plummer + Kroupa: random blocks of 1, 32, 1024, 16384 rows
    and the all-active block, every row of each against the oracle, in both
    precisions (one oracle run per block)."""
    s = W.plummer_kroupa_n131072()
    xp, vp, _ = _predict_dev(ctx, s)
    ox, ov = oracle.predict(s["t"], s["x"], s["v"], s["a"], s["jk"], s["t0"])
    assert np.array_equal(host(xp), ox)
    m = dev(s["m"])
    for size, blk in s["blocks"].items():
        rs2 = s["rs2"][blk]
        say(f"plummer-kroupa N=131072 n_i={size}: oracle on all {blk.size} rows")
        ref = oracle_rows(ox, ov, s["m"], blk, rs2, s["nb_cap"])
        for prec in ("mixed", "fp64"):
            res = nb.regular_force(xp, vp, m, dev(blk), dev(rs2), s["nb_cap"], prec, ctx=ctx)
            ea, ej = compare_force(res, ox, ov, s["m"], blk, rs2, s["nb_cap"], TOL[prec],
                                   ref=ref)
            say(f"  {prec} plan {ctx.last_plan()}  err acc {ea:.2e} jerk {ej:.2e}")
            del res


def _million_body_sample_rows(s, blk, k=4096):
    """Rows of block blk to check against the oracle: the 64 most central
    bodies, up to 1024 binary components, and a random remainder up to k."""
    r = np.sqrt((s["x"] ** 2).sum(0))[blk]
    central = np.argsort(r)[:64]
    comp = np.nonzero(blk < 2 * s["n_bin"])[0]
    rng = np.random.default_rng(3)
    binaries = rng.choice(comp, min(1024, comp.size), replace=False)
    chosen = np.unique(np.concatenate([central, binaries]))
    rest = np.setdiff1d(np.arange(blk.size), chosen)
    extra = rng.choice(rest, max(0, min(k - chosen.size, rest.size)), replace=False)
    return np.unique(np.concatenate([chosen, extra]))


@pytest.mark.parametrize("level", [3, 12])
def test_million_body_cluster(ctx, level):
    """N = 2^20 Plummer + Kroupa with 5% binaries, both precisions, at the full
    block (level 3) and a deep block level: 4096 rows against the oracle (the
    64 most central bodies, 1024 binary components, random others), counts
    and lists of every row equal across the two precisions."""
    s = W.binary_cluster_n1m()
    t, t0, blk = W.binary_cluster_level(s, level)
    say(f"N=2^20 cluster level {level}: n_i={blk.size}")
    xp, vp, _ = nb.predict(dev(s["x"]), dev(s["v"]), dev(s["a"]), dev(s["jk"]), dev(t0), t,
                           ctx=ctx)
    ox, ov = oracle.predict(t, s["x"], s["v"], s["a"], s["jk"], t0)
    assert np.array_equal(host(xp), ox) and np.array_equal(host(vp), ov)
    rows = _million_body_sample_rows(s, blk)
    n_bin_rows = int((blk[rows] < 2 * s["n_bin"]).sum())
    say(f"  oracle on {rows.size} rows ({n_bin_rows} binary components)")
    assert rows.size >= min(4096, blk.size) and n_bin_rows >= min(1024, int(
        (blk < 2 * s["n_bin"]).sum()))
    m = dev(s["m"])
    rs2 = s["rs2"][blk]
    ref = oracle_rows(ox, ov, s["m"], blk, rs2, s["nb_cap"], rows)
    keep = {}
    for prec in ("mixed", "fp64"):
        res = nb.regular_force(xp, vp, m, dev(blk), dev(rs2), s["nb_cap"], prec, ctx=ctx)
        ea, ej = compare_force(res, ox, ov, s["m"], blk, rs2, s["nb_cap"], TOL[prec], ref=ref)
        say(f"  {prec} plan {ctx.last_plan()}  err acc {ea:.2e} jerk {ej:.2e}")
        keep[prec] = res
    # every row: counts and lists are the same in both precisions (the lists
    # of the sampled rows are the oracle's, above); forces of the two
    # precisions agree within the mixed bar on every row
    mx, fp = keep["mixed"], keep["fp64"]
    assert torch.equal(mx[2], fp[2])
    cap = s["nb_cap"]
    defined = torch.arange(cap, device=mx[3].device)[None, :] < mx[2][:, None].clamp(max=cap)
    assert bool(((mx[3] == fp[3]) | ~defined).all())
    for k in (0, 1):
        d = torch.linalg.vector_norm(mx[k] - fp[k], dim=0)
        r = torch.linalg.vector_norm(fp[k], dim=0)
        e = float((d / r).max())
        say(f"  all {blk.size} rows, mixed vs fp64 {'acc' if k == 0 else 'jerk'}: max {e:.2e}")
        assert e <= TOL_MIXED - TOL_FP64
    del keep, mx, fp
    torch.cuda.empty_cache()


def _uniform_cube(seed, n):
    rng = np.random.default_rng(seed)
    x = rng.uniform(-1.0, 1.0, (3, n))
    v = rng.standard_normal((3, n)) * 0.3
    m = rng.uniform(0.5, 1.5, n) / n
    return x, v, m


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_many_splits_workgroup_merge(ctx, prec):
    """Plans with >= 256 j-splits merge each row with a whole work-group:
    sums over the splits in fixed order, segments placed by a prefix scan,
    overflowed segments (> 96 neighbours in one split) rebuilt in order."""
    say(f"work-group merge {prec}")
    n = 40000
    x, v, m = _uniform_cube(901, n)
    centre = int(np.argmin((x ** 2).sum(axis=0)))
    ib = np.array([centre, 17, 39999, 12345, 12345, 20000, 777], np.int32)
    # row 0 (the body nearest the centre) holds > 90% of the bodies: more than
    # 96 in every 128-body split
    rs2 = np.array([1.5 ** 2, 0.05 ** 2, 0.6 ** 2, 0.01 ** 2, 0.01 ** 2, 0.0, 0.45 ** 2])
    try:
        for plan in ((2, 1, 400), (2, 4, 320), (2, 2, 625)):   # 313, 313, 625 splits
            ctx.set_plan(*plan)
            for cap in (5000, 64):
                res = nb.regular_force(dev(x), dev(v), dev(m), dev(ib), dev(rs2), cap, prec,
                                       ctx=ctx)
                compare_force(res, x, v, m, ib, rs2, cap, TOL[prec])
            assert "splits=" in ctx.last_plan()
            assert int(ctx.last_plan().split("splits=")[1].split()[0]) >= 256
        assert host(res[2])[0] > 0.9 * n
    finally:
        ctx.set_plan(0, 0, 0)


def test_more_than_64_splits_per_merge_lane(ctx):
    """Over 16384 splits (N > 2^20 bodies in 64-body splits) each merge lane
    owns more than 64 segments and walks them all."""
    say("merge with > 64 splits per lane")
    n = (1 << 21) + 4097
    x, v, m = _uniform_cube(902, n)
    ib = np.array([5, n - 1, 1 << 20, 31337], np.int32)
    rs2 = np.full(ib.size, 0.03 ** 2)
    try:
        ctx.set_plan(2, 1, 40000)
        res = nb.regular_force(dev(x), dev(v), dev(m), dev(ib), dev(rs2), 256, "fp64", ctx=ctx)
        assert int(ctx.last_plan().split("splits=")[1].split()[0]) > 64 * 256
        compare_force(res, x, v, m, ib, rs2, 256, TOL_FP64)
        assert host(res[2]).min() > 10
    finally:
        ctx.set_plan(0, 0, 0)


def _same_result(got, want, cap, what):
    """Two results of one call are the same bits (list entries past a row's
    count are undefined and not compared)."""
    for k, name in ((0, "acc"), (1, "jerk"), (2, "nb_count"), (4, "overflow")):
        assert np.array_equal(got[k], want[k]), f"{name} differs: {what}"
    check_lists(got[2], got[3], want[2], want[3], cap)


@pytest.mark.parametrize("plan,rows", [((0, 0, 0), 300), ((1, 1, 1), 300), ((1, 1, 6), 300),
                                       ((2, 1, 400), 300), ((0, 0, 0), 1500), ((1, 1, 6), 1500)])
def test_refinement_of_every_flagged_row(plan, rows):
    """A mixed-precision tolerance so small that every row is flagged: every
    row is recomputed in FP64 by the refinement (chunk partials, added by the
    work-group that finishes last in blocks of up to 1024 rows, by a launch of
    their own, a wave per row, in larger ones), so the mixed call meets the
    FP64 bar.  Calls in between that flag nothing, and repeated calls, leave
    the refinement's arrival word ready: the flagged call gives the same bits
    every time.  Plans: automatic, one split (rows flagged by the force
    kernel), a few splits (lane-group merge), 313 splits (work-group merge)."""
    say(f"refinement of every row, plan {plan}, {rows} rows")
    c = nb.Context(0)
    try:
        n = 20000
        x, v, m = _uniform_cube(911, n)
        ib = np.random.default_rng(912).choice(n, rows, replace=False).astype(np.int32)
        rs2 = np.full(ib.size, 0.08 ** 2)
        cap = 256
        X, V, M, IB, RS = dev(x), dev(v), dev(m), dev(ib), dev(rs2)
        if plan != (0, 0, 0):
            c.set_plan(*plan)
        ref = oracle_rows(x, v, m, ib, rs2, cap)
        runs = []
        for k in range(3):
            c.set_mixed_tolerance(1e-30, 32.0)
            res = nb.regular_force(X, V, M, IB, RS, cap, "mixed", ctx=c)
            assert c.last_refined_rows() == ib.size
            compare_force(res, x, v, m, ib, rs2, cap, TOL_FP64, ref=ref)
            runs.append([host(t) for t in res])
            c.set_mixed_tolerance()   # the default: few rows, or none, flagged
            res = nb.regular_force(X, V, M, IB, RS, cap, "mixed", ctx=c)
            compare_force(res, x, v, m, ib, rs2, cap, TOL_MIXED, ref=ref)
        for r in runs[1:]:
            _same_result(r, runs[0], cap, "repeated flagged call")
    finally:
        c.close()


def test_refined_rows_independent_of_route():
    """A refined row's FP64 result depends only on the row and its j-range:
    rows refined in a 300-row call (pass 2 in the same launch), in a 1500-row
    call that contains them (pass 2 in a launch of its own), and with the
    partials buffer capped at 1 or 7 rows (the others refined one work-group
    per row, chunk after chunk), in regular and allocation-free calls, are
    the same bits."""
    say("refined rows independent of route")
    c = nb.Context(0)
    try:
        n = 20000
        x, v, m = _uniform_cube(931, n)
        rng = np.random.default_rng(932)
        big = rng.choice(n, 1500, replace=False).astype(np.int32)
        small = big[:300].copy()
        X, V, M = dev(x), dev(v), dev(m)
        rs_small, rs_big = dev(np.full(300, 0.08 ** 2)), dev(np.full(1500, 0.08 ** 2))
        c.set_mixed_tolerance(1e-30, 32.0)
        ref = nb.regular_force(X, V, M, dev(small), rs_small, 256, "mixed", ctx=c)
        assert c.last_refined_rows() == 300
        want = [host(ref[0]), host(ref[1])]
        res = nb.regular_force(X, V, M, dev(big), rs_big, 256, "mixed", ctx=c)
        assert c.last_refined_rows() == 1500
        for k in (0, 1):
            assert np.array_equal(host(res[k])[:, :300], want[k]), "fused vs separate final launch"
        for cap in (1, 7):
            c.set_refine_buffer_rows(cap)
            res = nb.regular_force(X, V, M, dev(small), rs_small, 256, "mixed", ctx=c)
            out = tuple(torch.empty_like(t) for t in res)
            nb.regular_force_noalloc(X, V, M, dev(small), rs_small, 256, "mixed", out=out, ctx=c)
            for k in (0, 1):
                assert np.array_equal(host(res[k]), want[k]), f"buffer of {cap} rows"
                assert np.array_equal(host(out[k]), want[k]), f"buffer of {cap} rows, no-alloc"
        compare_force(ref, x, v, m, small, np.full(300, 0.08 ** 2), 256, TOL_FP64)
    finally:
        c.close()


def test_graph_replay_of_small_blocks(ctx):
    """A stepping loop may capture its block calls in a graph: replays of a
    captured small-block call (split force launch, merge and refinement, no
    host work) reproduce the eager call bit for bit, replay after replay,
    with eager calls and synchronisations in between."""
    say("graph replay of small blocks")
    n = 1 << 16
    x, v, m = _uniform_cube(913, n)
    X, V, M = dev(x), dev(v), dev(m)
    rng = np.random.default_rng(914)
    for size in (1, 32):
        for prec in ("mixed", "fp64"):
            IB = dev(rng.choice(n, size, replace=False).astype(np.int32))
            RS = dev(np.full(size, 0.05 ** 2))
            eager = [host(t) for t in nb.regular_force(X, V, M, IB, RS, 128, prec, ctx=ctx)]
            out = tuple(torch.empty_like(torch.from_numpy(e)).cuda() for e in eager)
            side = torch.cuda.Stream()
            side.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(side):
                nb.regular_force(X, V, M, IB, RS, 128, prec, out=out, ctx=ctx)
            torch.cuda.current_stream().wait_stream(side)
            torch.cuda.synchronize()
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, capture_error_mode="thread_local"):
                nb.regular_force(X, V, M, IB, RS, 128, prec, out=out, ctx=ctx)
            for rep in range(3):
                for t in out:
                    t.fill_(-1)
                g.replay()
                torch.cuda.synchronize()
                _same_result([host(t) for t in out], eager, 128, f"replay {rep}, {size} rows, {prec}")
                again = [host(t) for t in nb.regular_force(X, V, M, IB, RS, 128, prec, ctx=ctx)]
                _same_result(again, eager, 128, f"eager call after replay {rep}")
            del g


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_workgroup_merge_many_rows_and_row_independence(ctx, prec):
    """100 rows with 313 j-splits each (work-group merge, many work-groups
    resident per CU; wave force kernel with four rows per wave, the row
    groups of a split on consecutive waves): parity with the oracle, and each
    row's results are the same bits as a call with that row alone under the
    same split plan (a row's sums depend only on the row and the splits)."""
    say(f"work-group merge of 100 rows {prec}")
    n = 40000
    x, v, m = _uniform_cube(915, n)
    ib = np.random.default_rng(916).choice(n, 100, replace=False).astype(np.int32)
    rs2 = np.random.default_rng(917).uniform(0.02, 0.12, ib.size) ** 2
    cap = 200
    X, V, M = dev(x), dev(v), dev(m)
    try:
        for plan in ((2, 4, 400), (2, 1, 400)):
            ctx.set_plan(*plan)
            res = nb.regular_force(X, V, M, dev(ib), dev(rs2), cap, prec, ctx=ctx)
            assert int(ctx.last_plan().split("splits=")[1].split()[0]) == 313
            compare_force(res, x, v, m, ib, rs2, cap, TOL[prec])
            full = [host(t) for t in res]
            for b in (0, 37, 99):
                one = [host(t) for t in nb.regular_force(X, V, M, dev(ib[b:b + 1]),
                                                          dev(rs2[b:b + 1]), cap, prec, ctx=ctx)]
                assert np.array_equal(one[0][:, 0], full[0][:, b])
                assert np.array_equal(one[1][:, 0], full[1][:, b])
                assert one[2][0] == full[2][b]
                k = min(int(full[2][b]), cap)
                assert np.array_equal(one[3][0, :k], full[3][b, :k])
    finally:
        ctx.set_plan(0, 0, 0)


def test_small_mixed_blocks_run_fp64_kernels(ctx):
    """Under automatic plans a mixed-precision request on a block of at most
    40 rows runs the FP64 kernels (latency-bound there) and meets the FP64
    bar; 41, 128 and 320 rows run the mixed kernels in one-wave row-per-lane
    work-groups (64-row tiles fill their lanes more than 1.2 times better
    than 256-row ones), 193 and 640 rows in 256-lane ones; a forced plan
    keeps the mixed kernels too."""
    say("small mixed blocks on FP64 kernels")
    n = 30000
    x, v, m = _uniform_cube(918, n)
    rng = np.random.default_rng(919)
    X, V, M = dev(x), dev(v), dev(m)
    for n_i, want in ((1, "prec=fp64 requested=mixed"), (40, "prec=fp64 requested=mixed"),
                      (41, "mapping=3 rows_per_lane=1"), (128, "mapping=3 rows_per_lane=1"),
                      (193, "mapping=1 rows_per_lane=1"), (320, "mapping=3 rows_per_lane=1"),
                      (640, "mapping=1 rows_per_lane=1")):
        ib = rng.choice(n, n_i, replace=False).astype(np.int32)
        rs2 = np.full(n_i, 0.07 ** 2)
        res = nb.regular_force(X, V, M, dev(ib), dev(rs2), 128, "mixed", ctx=ctx)
        assert want in ctx.last_plan(), ctx.last_plan()
        assert ("fp64" in want) == ("prec=fp64" in ctx.last_plan())
        tol = TOL_FP64 if "fp64" in want else TOL_MIXED
        compare_force(res, x, v, m, ib, rs2, 128, tol)
        if "fp64" in want:
            f = nb.regular_force(X, V, M, dev(ib), dev(rs2), 128, "fp64", ctx=ctx)
            _same_result([host(t) for t in res], [host(t) for t in f], 128, f"{n_i} rows")
    try:
        ctx.set_plan(2, 1, 0)
        ib = rng.choice(n, 8, replace=False).astype(np.int32)
        nb.regular_force(X, V, M, dev(ib), dev(np.full(8, 0.07 ** 2)), 128, "mixed", ctx=ctx)
        assert "prec=mixed" in ctx.last_plan()
    finally:
        ctx.set_plan(0, 0, 0)
