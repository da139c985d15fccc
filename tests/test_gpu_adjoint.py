"""GPU adjoint of the regular force (frozen neighbour sets) against the
oracle's analytic gradient and against central differences of local losses,
through the C ABI; plus the torch.autograd wrapper."""
import numpy as np
import pytest
import torch

import oracle
import paper_1504_03687_amd as nb
import workloads as W
from gpu_util import dev, host, say

pytestmark = pytest.mark.gpu
TOL_ADJ = 1e-10   # per-body norm-wise relative error vs the oracle gradient


@pytest.fixture(scope="module")
def ctx():
    c = nb.Context(0)
    yield c
    c.close()


def _body_err(got, ref):
    d = np.linalg.norm(got - ref, axis=0) if got.ndim == 2 else np.abs(got - ref)
    r = np.linalg.norm(ref, axis=0) if ref.ndim == 2 else np.abs(ref)
    scale = np.maximum(r, 1e-3 * r.max())
    return (d / scale).max()


def _check_vs_oracle(ctx, x, v, m, ib, rs2, wa, wj, tol=TOL_ADJ):
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    gx, gv, gm = (host(t) for t in nb.regular_force_adjoint(
        dev(x), dev(v), dev(m), dev(ib), dev(rs2), dev(wa), dev(wj), status=st, ctx=ctx))
    ox, ov, om = oracle.adjoint(x, v, m, ib, rs2, wa, wj)
    errs = (_body_err(gx, ox), _body_err(gv, ov), _body_err(gm, om))
    say(f"  adjoint err x {errs[0]:.2e} v {errs[1]:.2e} m {errs[2]:.2e}")
    assert max(errs) <= tol, errs
    return int(st.item())


def test_adjoint_ragged_small(ctx):
    say("adjoint ragged")
    s = W.small_state(81, 3001, k_nn=40)
    rng = np.random.default_rng(81)
    ib = rng.integers(0, 3001, 900).astype(np.int32)
    ib[7] = ib[8]                                 # duplicate rows
    rs2 = s["rs2"][ib].copy()
    rs2[3] = 0.0
    wa = rng.standard_normal((3, 900))
    wj = rng.standard_normal((3, 900))
    assert _check_vs_oracle(ctx, s["x"], s["v"], s["m"], ib, rs2, wa, wj) == 0


def test_adjoint_bad_index_and_empty(ctx):
    s = W.small_state(82, 500)
    ib = np.array([1, 700, 5], np.int32)
    rs2 = s["rs2"][[1, 0, 5]]
    rng = np.random.default_rng(1)
    wa, wj = rng.standard_normal((3, 3)), rng.standard_normal((3, 3))
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    gx, gv, gm = nb.regular_force_adjoint(dev(s["x"]), dev(s["v"]), dev(s["m"]), dev(ib),
                                          dev(rs2), dev(wa), dev(wj), status=st, ctx=ctx)
    torch.cuda.synchronize()
    assert int(st.item()) & nb.STATUS_BAD_INDEX
    keep = np.array([0, 2])
    ox, ov, om = oracle.adjoint(s["x"], s["v"], s["m"], ib[keep], rs2[keep], wa[:, keep],
                                wj[:, keep])
    assert _body_err(host(gx), ox) <= TOL_ADJ and _body_err(host(gm), om) <= TOL_ADJ
    e = nb.regular_force_adjoint(dev(s["x"]), dev(s["v"]), dev(s["m"]),
                                 dev(np.zeros(0, np.int32)), dev(np.zeros(0)),
                                 dev(np.zeros((3, 0))), dev(np.zeros((3, 0))), ctx=ctx)
    assert not any(host(t).any() for t in e)


def test_adjoint_n65536(ctx):
    """N = 65536 Plummer + Kroupa, all bodies active: the whole gradient
    against the oracle's, body by body; a 1024-row subset the same way; and
    the all-active gradient against central differences (h = 1e-6) of local
    losses at 256 bodies (the 32 most central and 224 random ones)."""
    s = W.adjoint_plummer_n65536()
    x, v, m = s["x"], s["v"], s["m"]
    ib, rs2, wa, wj = s["i_block"], s["rs2"], s["w_a"], s["w_j"]
    say("adjoint N=65536 full block vs the oracle gradient")
    _check_vs_oracle(ctx, x, v, m, ib, rs2, wa, wj)
    say("adjoint N=65536 subset")
    sub = np.random.default_rng(5).choice(s["n"], 1024, replace=False).astype(np.int32)
    _check_vs_oracle(ctx, x, v, m, sub, s["rs2"][sub], s["w_a"][:, sub], s["w_j"][:, sub])
    say("adjoint N=65536 full block vs finite differences")
    gx, gv, gm = (host(t) for t in nb.regular_force_adjoint(
        dev(x), dev(v), dev(m), dev(ib), dev(rs2), dev(wa), dev(wj), ctx=ctx))
    r = np.sqrt((x ** 2).sum(0))
    rng = np.random.default_rng(55)
    central = np.argsort(r)[:32]
    others = rng.choice(np.setdiff1d(np.arange(s["n"]), central), 224, replace=False)
    bodies = np.concatenate([central, others])
    assert np.unique(bodies).size == 256
    h = 1e-6
    worst = 0.0
    for k in bodies:
        for arr, g in ((x, gx), (v, gv)):
            for c in range(3):
                p = arr.copy(); p[c, k] += h
                q = arr.copy(); q[c, k] -= h
                if arr is x:
                    lp = oracle.local_loss(p, v, m, ib, rs2, wa, wj, k, xm=x)
                    lq = oracle.local_loss(q, v, m, ib, rs2, wa, wj, k, xm=x)
                else:
                    lp = oracle.local_loss(x, p, m, ib, rs2, wa, wj, k)
                    lq = oracle.local_loss(x, q, m, ib, rs2, wa, wj, k)
                fd = (lp - lq) / (2 * h)
                scale = max(np.linalg.norm(g[:, k]), 1e-12)
                worst = max(worst, abs(fd - g[c, k]) / scale)
        mp = m.copy(); mp[k] *= 1.5
        dl = oracle.local_loss(x, v, mp, ib, rs2, wa, wj, k) - oracle.local_loss(x, v, m, ib, rs2,
                                                                               wa, wj, k)
        worst = max(worst, abs(dl / (0.5 * m[k]) - gm[k]) / max(abs(gm[k]), 1e-12))
    say(f"  worst FD relative deviation {worst:.2e} over {bodies.size} bodies")
    assert worst <= 1e-6


def test_autograd_function(ctx):
    say("autograd")
    s = W.small_state(83, 2000, k_nn=32)
    ib = np.random.default_rng(3).choice(2000, 500, replace=False).astype(np.int32)
    rs2 = s["rs2"][ib]
    xp = dev(s["x"]).requires_grad_(True)
    vp = dev(s["v"]).requires_grad_(True)
    m = dev(s["m"]).requires_grad_(True)
    acc, jerk, cnt, lst, ovf = nb.RegularForce.apply(xp, vp, m, dev(ib), dev(rs2), 64, "fp64")
    rng = np.random.default_rng(4)
    wa, wj = rng.standard_normal((3, 500)), rng.standard_normal((3, 500))
    loss = (acc * dev(wa)).sum() + (jerk * dev(wj)).sum()
    loss.backward()
    ox, ov, om = oracle.adjoint(s["x"], s["v"], s["m"], ib, rs2, wa, wj)
    assert _body_err(host(xp.grad), ox) <= TOL_ADJ
    assert _body_err(host(vp.grad), ov) <= TOL_ADJ
    assert _body_err(host(m.grad), om) <= TOL_ADJ
    # the forward values are the library's regular force
    oa, oj, *_ = oracle.regular(s["x"], s["v"], s["m"], ib, rs2, 64)
    assert np.abs(host(acc) - oa).max() <= 1e-12 * np.abs(oa).max()
