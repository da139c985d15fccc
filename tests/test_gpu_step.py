"""GPU irregular force, Hermite corrector and potential against the oracle,
and a short shared-step Hermite integration driven by the library's kernels
against the same integration driven by the oracle."""
import numpy as np
import pytest
import torch

import oracle
import paper_1504_03687_amd as nb
import workloads as W
from gpu_util import dev, host, row_rel_err, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = nb.Context(0)
    yield c
    c.close()


def test_irregular_force_and_full_force(ctx):
    say("irregular force")
    s = W.config2()
    xp, vp, m = dev(s["x"]), dev(s["v"]), dev(s["m"])
    blk = s["blocks"][16384]
    cap = 128
    reg = nb.regular_force(xp, vp, m, dev(blk), dev(s["rs2"][blk]), cap, "fp64", ctx=ctx)
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    ia, ij = nb.irregular_force(xp, vp, m, dev(blk), cap, reg[2], reg[3], status=st, ctx=ctx)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    cnt, lst = host(reg[2]), host(reg[3])
    oa, oj = oracle.irregular(s["x"], s["v"], s["m"], blk, cap, cnt, lst)
    ea, ej = row_rel_err(host(ia), oa), row_rel_err(host(ij), oj)
    say(f"  irregular max err acc {ea.max():.2e} jerk {ej.max():.2e}")
    assert ea.max() <= 1e-12 and ej.max() <= 1e-12
    # regular + irregular = full force (rs2 = 0), rows without list overflow
    full = nb.regular_force(xp, vp, m, dev(blk), dev(np.zeros(blk.size)), 1, "fp64", ctx=ctx)
    ok = cnt <= cap
    for part_r, part_i, f in ((reg[0], ia, full[0]), (reg[1], ij, full[1])):
        e = row_rel_err(host(part_r + part_i)[:, ok], host(f)[:, ok])
        assert e.max() <= 1e-11, e.max()


def test_irregular_bad_list_entry(ctx):
    s = W.small_state(91, 300)
    ib = np.array([3, 4], np.int32)
    cnt = np.array([2, 2], np.int32)
    lst = np.array([[5, 700], [4, 6]], np.int32)     # 700 out of range, 4 is the row itself
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    ia, ij = nb.irregular_force(dev(s["x"]), dev(s["v"]), dev(s["m"]), dev(ib), 2, dev(cnt),
                                dev(lst), status=st, ctx=ctx)
    torch.cuda.synchronize()
    assert int(st.item()) & nb.STATUS_BAD_INDEX
    oa, oj = oracle.irregular(s["x"], s["v"], s["m"], ib, 1, np.array([1, 1], np.int32),
                              np.array([[5], [6]], np.int32))
    assert np.allclose(host(ia), oa, rtol=1e-13, atol=0)


def test_hermite_corrector_bitwise(ctx):
    say("corrector")
    rng = np.random.default_rng(31)
    n = 4099
    h = np.ldexp(1.0, -rng.integers(3, 20, n))
    arrs = [rng.standard_normal((3, n)) for _ in range(6)]
    got = nb.hermite_correct(dev(h), *[dev(a) for a in arrs], ctx=ctx)
    ref = oracle.hermite_correct(h, *arrs)
    for g, r in zip(got, ref):
        assert np.array_equal(host(g), r)


@pytest.mark.parametrize("n", [1, 3001, 16384])
def test_potential(ctx, n):
    say(f"potential n={n}")
    rng = np.random.Generator(np.random.PCG64(77 + n))
    x, v, m = W.plummer(rng, n, "kroupa") if n > 1 else (np.zeros((3, 1)), None, np.ones(1))
    phi, U = nb.potential(dev(x), dev(m), ctx=ctx)
    oU, ophi = oracle.potential(x, m)
    if n == 1:
        assert host(phi)[0] == 0 and host(U)[0] == 0
        return
    e = np.abs(host(phi) - ophi) / np.abs(ophi)
    assert e.max() <= 1e-12
    assert abs(host(U)[0] - oU) <= 1e-12 * abs(oU)


def test_shared_step_integration_matches_oracle(ctx):
    """Eight shared Hermite steps of a 512-body cluster: predict -> regular +
    irregular force -> corrector, all on the GPU, against the same loop on the
    oracle.  Trajectories agree to ~1e-12 over the run."""
    say("integration")
    s = W.small_state(95, 512, k_nn=24)
    n = 512
    blk = np.arange(n, dtype=np.int32)
    h = 2.0 ** -7
    cap = 128
    # oracle loop
    ox, ov = s["x"].copy(), s["v"].copy()
    ra, rj, rc, rl, *_ = oracle.regular(ox, ov, s["m"], blk, s["rs2"], cap)
    ia, ij = oracle.irregular(ox, ov, s["m"], blk, cap, rc, rl)
    oa, oj = ra + ia, rj + ij
    # GPU loop
    gx, gv, gm = dev(s["x"]), dev(s["v"]), dev(s["m"])
    grs2, gblk = dev(s["rs2"]), dev(blk)
    r = nb.regular_force(gx, gv, gm, gblk, grs2, cap, "fp64", ctx=ctx)
    i2 = nb.irregular_force(gx, gv, gm, gblk, cap, r[2], r[3], ctx=ctx)
    ga, gj = r[0] + i2[0], r[1] + i2[1]
    hh = dev(np.full(n, h))
    for step in range(8):
        xp, vp = oracle.predict(h, ox, ov, oa, oj, np.zeros(n))
        ra, rj, rc, rl, *_ = oracle.regular(xp, vp, s["m"], blk, s["rs2"], cap)
        ia, ij = oracle.irregular(xp, vp, s["m"], blk, cap, rc, rl)
        ox, ov, _, _ = oracle.hermite_correct(np.full(n, h), ox, ov, oa, oj, ra + ia, rj + ij)
        oa, oj = ra + ia, rj + ij

        gxp, gvp, _ = nb.predict(gx, gv, ga, gj, dev(np.zeros(n)), h, ctx=ctx)
        r = nb.regular_force(gxp, gvp, gm, gblk, grs2, cap, "fp64", ctx=ctx)
        i2 = nb.irregular_force(gxp, gvp, gm, gblk, cap, r[2], r[3], ctx=ctx)
        a1, j1 = r[0] + i2[0], r[1] + i2[1]
        gx, gv, _, _ = nb.hermite_correct(hh, gx, gv, ga, gj, a1, j1, ctx=ctx)
        ga, gj = a1, j1
    dx = np.abs(host(gx) - ox).max()
    dv = np.abs(host(gv) - ov).max()
    say(f"  after 8 steps: max |dx| {dx:.2e}  max |dv| {dv:.2e}")
    assert dx <= 1e-12 and dv <= 1e-11
