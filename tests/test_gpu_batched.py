"""Batched ensemble (one persistent launch over many uneven clusters, replayed
from a captured HIP graph) against the oracle run cluster by cluster, and
against single-block launches of the library itself."""
import numpy as np
import pytest
import torch

import oracle
import paper_1504_03687_amd as nb
import workloads as W
from gpu_util import TOL_FP64, TOL_MIXED, check_lists, dev, host, row_rel_err, say

pytestmark = pytest.mark.gpu
TOL = {"fp64": TOL_FP64, "mixed": TOL_MIXED}


@pytest.fixture(scope="module")
def ctx():
    c = nb.Context(0)
    yield c
    c.close()


def _ensemble(seed=7, sizes=(1, 64, 300, 1000, 2500, 777, 40, 4096, 513, 2, 9000, 130)):
    rng = np.random.default_rng(seed)
    xs, vs, ms, blocks, rs2s = [], [], [], [], []
    j_off, i_off = [0], [0]
    for c, n in enumerate(sizes):
        s = W.small_state(200 + c, n, k_nn=min(24, max(n - 1, 1)))
        ni = 0 if c == 6 else int(rng.integers(1, n + 1))   # one cluster without rows
        blk = rng.choice(n, ni, replace=False).astype(np.int32)
        xs.append(s["x"]); vs.append(s["v"]); ms.append(s["m"])
        blocks.append(blk + j_off[-1]); rs2s.append(s["rs2"][blk])
        j_off.append(j_off[-1] + n); i_off.append(i_off[-1] + ni)
    return dict(x=np.concatenate(xs, 1), v=np.concatenate(vs, 1), m=np.concatenate(ms),
                ib=np.concatenate(blocks).astype(np.int32), rs2=np.concatenate(rs2s),
                j_off=np.array(j_off), i_off=np.array(i_off))


def _oracle_cluster(E, c, cap, rows=None):
    j0, j1 = E["j_off"][c], E["j_off"][c + 1]
    r0, r1 = E["i_off"][c], E["i_off"][c + 1]
    sel = np.arange(r0, r1) if rows is None else rows
    res = oracle.regular(E["x"][:, j0:j1], E["v"][:, j0:j1], E["m"][j0:j1], E["ib"][sel] - j0,
                         E["rs2"][sel], cap)
    lst = np.where(res[3] >= 0, res[3] + j0, res[3])
    return sel, res[0], res[1], res[2], lst


def _check(E, out, cap, tol, rows_per_cluster=None):
    acc, jerk, cnt, lst, ovf = (host(t) for t in out)
    worst = 0.0
    any_ovf = 0
    for c in range(len(E["j_off"]) - 1):
        r0, r1 = E["i_off"][c], E["i_off"][c + 1]
        if r1 == r0:
            continue
        rows = None
        if rows_per_cluster is not None and r1 - r0 > rows_per_cluster:
            rows = np.random.default_rng(c).choice(np.arange(r0, r1), rows_per_cluster,
                                                   replace=False)
        sel, oa, oj, oc, ol = _oracle_cluster(E, c, cap, rows)
        check_lists(cnt[sel], lst[sel], oc, ol, cap)
        ea, ej = row_rel_err(acc[:, sel], oa), row_rel_err(jerk[:, sel], oj)
        worst = max(worst, ea.max(), ej.max())
        any_ovf |= int((oc > cap).any())
    assert worst <= tol, worst
    if rows_per_cluster is None:
        assert int(ovf[0]) == any_ovf
    return worst


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("splits", [0, 3])
def test_batched_small_ensemble(ctx, prec, splits):
    say(f"batched small {prec} splits={splits}")
    E = _ensemble()
    ctx.set_plan(0, 0, splits)
    try:
        args = (E["j_off"], E["i_off"], dev(E["x"]), dev(E["v"]), dev(E["m"]), dev(E["ib"]),
                dev(E["rs2"]))
        out = nb.regular_force_batched(*args, 20, prec, ctx=ctx)
        w = _check(E, out, 20, TOL[prec])
        say(f"  {ctx.last_plan()}  worst err {w:.2e}")
        # replay of the cached graph gives identical results
        first = [host(t).copy() for t in out]
        out2 = nb.regular_force_batched(*args, 20, prec, out=out, ctx=ctx)
        for p, q in zip(first, out2):
            assert np.array_equal(p, host(q))
    finally:
        ctx.set_plan(0, 0, 0)


def test_batched_graph_replay_sees_new_data(ctx):
    """The graph captures pointers, not values: new positions in the same
    buffers give the new forces on replay."""
    say("batched replay with new data")
    E = _ensemble(seed=9)
    x, v, m = dev(E["x"]), dev(E["v"]), dev(E["m"])
    ib, rs2 = dev(E["ib"]), dev(E["rs2"])
    out = nb.regular_force_batched(E["j_off"], E["i_off"], x, v, m, ib, rs2, 16, "fp64", ctx=ctx)
    torch.cuda.synchronize()
    x.mul_(2.0)
    rs2.mul_(4.0)
    out = nb.regular_force_batched(E["j_off"], E["i_off"], x, v, m, ib, rs2, 16, "fp64",
                                   out=out, ctx=ctx)
    E2 = dict(E, x=2 * E["x"], rs2=4 * E["rs2"])
    _check(E2, out, 16, TOL_FP64)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("splits", [1, 3, 7, 16])
def test_batched_equals_single_launches(ctx, prec, splits):
    """Each cluster of the batch gives bit-identical rows to a single-block
    launch of the same plan on that cluster alone.  At 7 and 16 requested
    splits the clusters get 1 to 12 splits, so the batched merge runs 16-lane
    row groups on clusters whose own launch merges with 4-lane groups."""
    say(f"batched vs single {prec} splits={splits}")
    E = _ensemble(seed=11)
    ctx.set_plan(1, 1, splits)
    try:
        out = [host(t) for t in nb.regular_force_batched(
            E["j_off"], E["i_off"], dev(E["x"]), dev(E["v"]), dev(E["m"]), dev(E["ib"]),
            dev(E["rs2"]), 32, prec, ctx=ctx)]
        for c in range(len(E["j_off"]) - 1):
            j0, j1 = E["j_off"][c], E["j_off"][c + 1]
            r0, r1 = E["i_off"][c], E["i_off"][c + 1]
            if r1 == r0:
                continue
            single = [host(t) for t in nb.regular_force(
                dev(E["x"][:, j0:j1]), dev(E["v"][:, j0:j1]), dev(E["m"][j0:j1]),
                dev((E["ib"][r0:r1] - j0).astype(np.int32)), dev(E["rs2"][r0:r1]), 32, prec, ctx=ctx)]
            assert np.array_equal(out[0][:, r0:r1], single[0])
            assert np.array_equal(out[1][:, r0:r1], single[1])
            assert np.array_equal(out[2][r0:r1], single[2])
            for b in range(r1 - r0):
                k = min(int(single[2][b]), 32)
                assert np.array_equal(out[3][r0 + b, :k], single[3][b, :k] + j0)
    finally:
        ctx.set_plan(0, 0, 0)


def test_cluster_ensemble_256(ctx):
    """256 Plummer + Kroupa clusters, N log-uniform in [1024, 32768], active
    fractions U[0.01, 1]: one persistent launch, sampled rows of every cluster
    against the oracle."""
    s = W.cluster_ensemble_256()
    say(f"ensemble: {s['n']} bodies, {s['i_block'].size} rows")
    xp, vp, _ = nb.predict(dev(s["x"]), dev(s["v"]), dev(s["a"]), dev(s["jk"]), dev(s["t0"]),
                           s["t"], ctx=ctx)
    ox, ov = oracle.predict(s["t"], s["x"], s["v"], s["a"], s["jk"], s["t0"])
    E = dict(x=ox, v=ov, m=s["m"], ib=s["i_block"], rs2=s["rs2"], j_off=s["j_off"],
             i_off=s["i_off"])
    for prec in ("mixed", "fp64"):
        out = nb.regular_force_batched(s["j_off"], s["i_off"], xp, vp, dev(s["m"]),
                                       dev(s["i_block"]), dev(s["rs2"]), s["nb_cap"], prec,
                                       ctx=ctx)
        w = _check(E, out, s["nb_cap"], TOL[prec], rows_per_cluster=12)
        say(f"  {prec}: {ctx.last_plan()}  worst err {w:.2e}")


SHAPES = [(256, 256, 1), (256, 256, 2), (128, 128, 1), (64, 64, 1), (512, 512, 1), (256, 512, 1)]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_batched_shapes_equal_single_launches(ctx, prec):
    """Every built kernel shape of the batched ensemble (LDS tile length,
    work-group width, rows per lane) and work cap gives rows bit-identical to
    single-block launches with the same split count on each cluster alone."""
    E = _ensemble(seed=13)
    args = (E["j_off"], E["i_off"], dev(E["x"]), dev(E["v"]), dev(E["m"]), dev(E["ib"]),
            dev(E["rs2"]))
    try:
        for splits in (1, 3):
            ctx.set_batched_shape()
            ctx.set_plan(1, 1, splits)
            singles = []
            for c in range(len(E["j_off"]) - 1):
                j0, j1 = E["j_off"][c], E["j_off"][c + 1]
                r0, r1 = E["i_off"][c], E["i_off"][c + 1]
                if r1 == r0:
                    singles.append(None)
                    continue
                singles.append([host(t) for t in nb.regular_force(
                    dev(E["x"][:, j0:j1]), dev(E["v"][:, j0:j1]), dev(E["m"][j0:j1]),
                    dev((E["ib"][r0:r1] - j0).astype(np.int32)), dev(E["rs2"][r0:r1]), 32,
                    prec, ctx=ctx)])
            for shape in SHAPES:
                for ipc in (16, 256):
                    ctx.set_batched_shape(*shape, ipc)
                    out = [host(t) for t in nb.regular_force_batched(*args, 32, prec, ctx=ctx)]
                    plan = ctx.last_plan()
                    say(f"  {prec} splits={splits}: {plan}")
                    assert f"tile={shape[0]} lanes={shape[1]} rows_per_lane={shape[2]}" in plan
                    assert f"items_per_cu={ipc}" in plan and "shape=forced" in plan
                    for c, single in enumerate(singles):
                        if single is None:
                            continue
                        j0 = E["j_off"][c]
                        r0, r1 = E["i_off"][c], E["i_off"][c + 1]
                        assert np.array_equal(out[0][:, r0:r1], single[0]), (shape, c)
                        assert np.array_equal(out[1][:, r0:r1], single[1]), (shape, c)
                        assert np.array_equal(out[2][r0:r1], single[2]), (shape, c)
                        for b in range(r1 - r0):
                            k = min(int(single[2][b]), 32)
                            assert np.array_equal(out[3][r0 + b, :k], single[3][b, :k] + j0)
    finally:
        ctx.set_batched_shape()
        ctx.set_plan(0, 0, 0)


def test_batched_shape_override_rejects_unbuilt_shapes(ctx):
    with pytest.raises(nb.NbError) as err:
        ctx.set_batched_shape(192, 256, 1, 64)
    assert err.value.code == -4
    with pytest.raises(nb.NbError) as err:
        ctx.set_batched_shape(256, 256, 1, 5000)
    assert err.value.code == -1
    ctx.set_batched_shape()


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_batched_autotune(tmp_path, prec):
    """The batched tuner picks a shape for this ensemble; its outputs match
    the oracle, later calls use the tuned shape with the same bits, and a
    fresh context loads the choice from the cache file without re-timing."""
    E = _ensemble(seed=17)
    args = (E["j_off"], E["i_off"], dev(E["x"]), dev(E["v"]), dev(E["m"]), dev(E["ib"]),
            dev(E["rs2"]))
    path = str(tmp_path / "batched.txt")
    c1 = nb.Context(0)
    try:
        tuned = nb.autotune_batched(*args, 24, prec, cache_path=path, force=True, ctx=c1)
        plan = c1.last_plan()
        say(f"  tuned {prec}: {plan}")
        assert "shape=tuned" in plan
        _check(E, tuned, 24, TOL[prec])
        first = [host(t).copy() for t in tuned]

        def same(out):
            got = [host(t) for t in out]
            for k in (0, 1, 2, 4):
                assert np.array_equal(first[k], got[k])
            check_lists(got[2], got[3], first[2], first[3], 24)   # defined entries only

        same(nb.regular_force_batched(*args, 24, prec, ctx=c1))
        assert c1.last_plan() == plan
        with open(path) as f:
            lines = f.read().splitlines()
        assert lines[0] == "nbreg-batched-tune 1" and len(lines) == 2
        c2 = nb.Context(0)
        try:
            nb.autotune_batched(*args, 24, prec, cache_path=path, ctx=c2)
            same(nb.regular_force_batched(*args, 24, prec, ctx=c2))
            assert c2.last_plan() == plan
        finally:
            c2.close()
    finally:
        c1.close()
