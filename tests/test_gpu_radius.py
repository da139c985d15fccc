"""GPU parity of neighbour-radius control (Table A1, NNBOPT) against the CPU
oracle: next-step radii bit for bit; the overflow shrink-and-recompute loop
with the same rounds, final radii, counts and lists bit for bit, and forces
within the precision's bar."""
import numpy as np
import pytest
import torch

import oracle
import oracle.radius as R
import paper_1504_03687_amd as nb
import workloads as W
from gpu_util import TOL_FP64, TOL_MIXED, check_lists, dev, host, row_rel_err, say

pytestmark = pytest.mark.gpu
TOL = {"fp64": TOL_FP64, "mixed": TOL_MIXED}


@pytest.fixture(scope="module")
def ctx():
    c = nb.Context(0)
    yield c
    c.set_plan(0, 0, 0)
    c.close()


@pytest.mark.parametrize("clamp", [(0.5, 2.0), (1e-3, 1e3)])
def test_radius_update_bitwise(ctx, clamp):
    rng = np.random.default_rng(830)
    n_i = 50001
    cnt = rng.integers(0, 600, n_i).astype(np.int32)
    rs2 = np.exp(rng.uniform(np.log(1e-6), np.log(1e-1), n_i))
    rs2[::97] = 0.0
    rs2[::89] = -0.5
    ref = R.radius_update(rs2, cnt, 64, *clamp)
    got = nb.radius_update(dev(cnt), dev(rs2), 64, *clamp, ctx=ctx)
    assert np.array_equal(host(got), ref)
    g = dev(rs2)
    nb.radius_update(dev(cnt), g, 64, *clamp, out=g, ctx=ctx)      # in place
    assert np.array_equal(host(g), ref)


def _fit_case(seed, n, k_nn, stride, pct):
    s = W.small_state(seed, n, k_nn=k_nn)
    blk = np.arange(0, n, stride, dtype=np.int32)
    rs2 = s["rs2"][blk].copy()
    c_true = oracle.regular(s["x"], s["v"], s["m"], blk, rs2, 1000)[2]
    cap = int(np.percentile(c_true, pct))
    return s, blk, rs2, cap


def _compare_fit(got, ref, cap, tol):
    acc, jerk, cnt, lst, ovf, rounds = got
    oa, oj, oc, ol, oo, ors2, orounds = ref
    assert rounds == orounds and int(host(ovf)[0]) == oo
    check_lists(host(cnt), host(lst), oc, ol, cap)
    ea, ej = row_rel_err(host(acc), oa), row_rel_err(host(jerk), oj)
    assert ea.max() <= tol and ej.max() <= tol, (ea.max(), ej.max())
    return ea.max(), ej.max()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("plan", [(0, 0, 0), (2, 1, 3), (1, 2, 2)])
def test_fit_matches_oracle(ctx, prec, plan):
    say(f"fit prec={prec} plan={plan}")
    s, blk, rs2, cap = _fit_case(840, 3001, 48, 2, 55)
    nnbopt = cap - 6
    ref = R.regular_fit(s["x"], s["v"], s["m"], blk, rs2, cap, nnbopt, 8)
    assert ref[6] >= 1 and ref[4] == 0
    ctx.set_plan(*plan)
    g_rs2 = dev(rs2)
    got = nb.regular_force_fit(dev(s["x"]), dev(s["v"]), dev(s["m"]), dev(blk), g_rs2, cap,
                               nnbopt, 8, prec, ctx=ctx)
    ctx.set_plan(0, 0, 0)
    assert np.array_equal(host(g_rs2), ref[5])
    ea, ej = _compare_fit(got, ref, cap, TOL[prec])
    say(f"  rounds {got[5]}, max err acc {ea:.2e} jerk {ej:.2e}")


def test_fit_round_limit_and_no_overflow(ctx):
    s, blk, rs2, cap = _fit_case(850, 2000, 64, 1, 50)
    cap = max(cap // 8, 1)                          # needs several rounds at 1/4 per round
    for rounds in (1, 2):
        ref = R.regular_fit(s["x"], s["v"], s["m"], blk, rs2, cap, 64, rounds)
        g_rs2 = dev(rs2)
        got = nb.regular_force_fit(dev(s["x"]), dev(s["v"]), dev(s["m"]), dev(blk), g_rs2,
                                   cap, 64, rounds, "fp64", ctx=ctx)
        assert got[5] == rounds and np.array_equal(host(g_rs2), ref[5])
        _compare_fit(got, ref, cap, TOL_FP64)
    # nothing overflows: zero rounds, same as the plain regular force
    big = 1000
    ref = R.regular_fit(s["x"], s["v"], s["m"], blk, rs2, big, 64, 8)
    g_rs2 = dev(rs2)
    got = nb.regular_force_fit(dev(s["x"]), dev(s["v"]), dev(s["m"]), dev(blk), g_rs2, big,
                               64, 8, "fp64", ctx=ctx)
    assert got[5] == 0 and ref[6] == 0 and np.array_equal(host(g_rs2), rs2)
    _compare_fit(got, ref, big, TOL_FP64)


def test_fit_n131072_block(ctx):
    """N = 131072 Plummer + Kroupa, a random block of 4096 rows with radii
    from the 64th neighbour and a list cap of 56: most rows overflow."""
    say("fit N=131072")
    s = W.plummer_kroupa_n131072()
    rng = np.random.default_rng(860)
    blk = np.sort(rng.choice(s["n"], 4096, replace=False)).astype(np.int32)
    rs2 = s["rs2"][blk].copy()
    cap, nnbopt = 56, 48
    xp, vp, _ = nb.predict(dev(s["x"]), dev(s["v"]), dev(s["a"]), dev(s["jk"]), dev(s["t0"]),
                           s["t"], ctx=ctx)
    ox, ov = oracle.predict(s["t"], s["x"], s["v"], s["a"], s["jk"], s["t0"])
    assert np.array_equal(host(xp), ox)
    ref = R.regular_fit(ox, ov, s["m"], blk, rs2, cap, nnbopt, 8)
    for prec in ("fp64", "mixed"):
        g_rs2 = dev(rs2)
        got = nb.regular_force_fit(xp, vp, dev(s["m"]), dev(blk), g_rs2, cap, nnbopt, 8, prec,
                                   ctx=ctx)
        assert np.array_equal(host(g_rs2), ref[5])
        ea, ej = _compare_fit(got, ref, cap, TOL[prec])
        say(f"  {prec}: rounds {got[5]}, rows shrunk {(ref[5] < rs2).sum()}, "
            f"err {ea:.2e} {ej:.2e}")


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_fit_bench_configuration_sampled(ctx, prec):
    """The fit as the benchmark runs it: the N = 2^20 binary cluster, the level-10
    block (51374 rows), radii from the 64th neighbour, nb_cap 48, NNBOPT 40.
    Rows are independent in the fit, so the oracle's fit of 256 sampled rows
    alone must give those rows' radii, counts and lists bit for bit."""
    say(f"fit at the benchmark configuration {prec}")
    s = W.binary_cluster_n1m()
    t, t0, blk = W.binary_cluster_level(s, 10)
    xp, vp, _ = nb.predict(dev(s["x"]), dev(s["v"]), dev(s["a"]), dev(s["jk"]), dev(t0), t,
                           ctx=ctx)
    ox, ov = oracle.predict(t, s["x"], s["v"], s["a"], s["jk"], t0)
    rs2 = s["rs2"][blk].copy()
    g_rs2 = dev(rs2)
    got = nb.regular_force_fit(xp, vp, dev(s["m"]), dev(blk), g_rs2, 48, 40, 8, prec, ctx=ctx)
    assert int(host(got[4])[0]) == 0
    rows = np.sort(np.random.default_rng(870).choice(blk.size, 256, replace=False))
    ref = R.regular_fit(ox, ov, s["m"], blk[rows], rs2[rows], 48, 40, 8)
    assert np.array_equal(host(g_rs2)[rows], ref[5])
    check_lists(host(got[2])[rows], host(got[3])[rows], ref[2], ref[3], 48)
    ea = row_rel_err(host(got[0])[:, rows], ref[0])
    ej = row_rel_err(host(got[1])[:, rows], ref[1])
    say(f"  rounds {got[5]}, sampled err acc {ea.max():.2e} jerk {ej.max():.2e}")
    assert ea.max() <= TOL[prec] and ej.max() <= TOL[prec]
