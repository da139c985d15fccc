"""Benchmark of the Ahmad-Cohen regular-force step on one MI355X.

Workload: the million-body cluster -- N = 2^20 Plummer sphere, Kroupa (2001)
IMF, 5% of bodies in primordial binaries, Hermite step levels 2^-3..2^-20 --
at its full block (all N bodies active), the shape of the paper's
million-body runs (section 4.2, section 5).  One step = predict all N bodies
to the block time + regular force, jerk and neighbour lists of the full block
(nb_cap 1024).  Inputs are generated on the host and resident in HBM before
timing starts.

Printed: ONE JSON line with the mixed-precision pair-interaction rate as
`value` (G pairs/s), the FP64 rate beside it, the dominant kernel's roofline
(ALU-bound: algorithmic flops per pair x pairs / kernel time, timed with HIP
events on the library's stream), the per-level aggregate, and the CPU oracle
timed on a bounded row sample on the host cores.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic floating-point operations per regular pair interaction
# (acc + jerk, FMA counted as 2): r = xj - xi (3), u = vj - vi (3), r.r (5),
# r.u (5), 1/sqrt (1), r^-2 (1), m r^-3 (2), 3 (r.u) r^-2 (2), acc += m r^-3 r
# (6), jerk += m r^-3 (u - alpha r) (12).
FLOPS_PER_PAIR = 40
# Algorithmic floating-point operations per pair of the adjoint's two FP64
# recompute passes (FMA = 2), counted from the gradient formulas with the
# row-constant weights A = w_a, B = w_j factored out of the pair loops:
#  row pass: r, u differences 6, |r|^2 5, 1/sqrt 1, |r|^-2, |r|^-3, |r|^-5 3,
#    r.u, A.r, B.r, B.u 20, m |r|^-5 and its (B.r) product 2, the r
#    coefficient 6, sum m |r|^-3 2, sum m |r|^-5 (r.u) 2, the u and r sums
#    of H 12, sum (B.r) r 6 -> 65;
#  body pass: the same geometry 35, A.r + B.u and s (B.r) 2, the two mass
#    sums 4, |r|^-5 s and |r|^-5 (B.r) 2, the r coefficient 4, the A, B and
#    u/r sums 36 -> 83.
ADJ_FLOPS_ROWS = 65
ADJ_FLOPS_BODIES = 83

# MI355X published vector peaks (TFLOP/s): FP32 157.3, FP64 78.6.  Plain
# (unpacked) FP32 instructions issue in 2 cycles per wave64 on gfx950 and
# FP64 ones in 4, which are these two rates on 256 CUs x 4 SIMDs at 2.4 GHz.
PEAK_FP32 = 157.3
PEAK_FP64 = 78.6


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# the kernels and the plan rules that shape their launches
KERNEL_SOURCES = ("nb_internal.h", "nb_pair.h", "nb_rows.h", "nb_force.hip", "nb_plan.hip")


def kernel_src_hash() -> str:
    """SHA-1 over the sources of the regular-force kernels and their plans."""
    import hashlib
    h = hashlib.sha1()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1504_03687_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def profiled(prec: str, key: str):
    """A figure of the full-block force kernel from the committed rocprofv3
    counter summary (HBM bytes per launch from FETCH_SIZE / WRITE_SIZE, the
    fraction of the instruction issue model), or None when that summary was
    taken on different kernel sources (or does not exist)."""
    path = os.path.join(ROOT, "profiles", "force_rows_kernel_full_block_n1048576.traffic.json")
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("kernel_src_sha1") != kernel_src_hash():
        return None
    return d.get(prec, {}).get(key)


def steady_ms(call, warm_ms=30.0, time_ms=50.0, min_reps=3):
    """Mean wall time of one call in steady state.  The calls first run back
    to back, untimed, for at least warm_ms (the GPU clock ramps up under
    load: a few calls after an idle gap read up to 20% slow on the small
    step levels); then at least min_reps calls and time_ms are timed."""
    import torch
    call()
    torch.cuda.synchronize()
    t = time.perf_counter()
    k = 0
    while True:
        call()
        k += 1
        torch.cuda.synchronize()
        if (time.perf_counter() - t) * 1e3 >= warm_ms:
            break
    est = (time.perf_counter() - t) * 1e3 / k
    reps = max(min_reps, int(math.ceil(time_ms / max(est, 1e-3))))
    c1 = time.perf_counter()
    for _ in range(reps):
        call()
    torch.cuda.synchronize()
    return (time.perf_counter() - c1) * 1e3 / reps


def graph_ms(call, per_graph=10):
    """Mean time of one call replayed from a captured graph of per_graph
    back-to-back calls: the GPU time of the call's launch chain without the
    host's per-call work (argument checks, plan lookup, launches)."""
    import torch
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        call()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, capture_error_mode="thread_local"):
        for _ in range(per_graph):
            call()
    ms = steady_ms(g.replay) / per_graph
    del g
    return ms


def cpu_model() -> str:
    """Host CPU model name (lscpu, else /proc/cpuinfo)."""
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def small_blocks_leg(nb, ctx, dev, s, xp, vp, m, cap, precs):
    """Blocks of 1, 32, 1024 and 320 random rows of the 2^20 cluster (HBM-
    and launch-bound; 320 rows run one-wave work-groups), in steady state with
    outputs reused across calls, as in a stepping loop: per call from the host
    (us) and replayed from a captured graph (graph_us, the launch chain
    alone)."""
    n = s["n"]
    small = {}
    rng = np.random.default_rng(1)
    for size in (1, 32, 1024, 320):
        sb = rng.choice(n, size, replace=False).astype(np.int32)
        bd, rd = dev(sb), dev(s["rs2"][sb])
        ent = {}
        for prec in precs:
            o = nb.regular_force(xp, vp, m, bd, rd, cap, prec, ctx=ctx)
            call = lambda: nb.regular_force(xp, vp, m, bd, rd, cap, prec, out=o, ctx=ctx)
            us = 1e3 * steady_ms(call)
            gus = 1e3 * graph_ms(call)
            ent[prec] = {"us": round(us, 1), "graph_us": round(gus, 1),
                         "gpairs_per_s": round(size * (n - 1) / us * 1e-3, 2),
                         "jset_GB_per_s": round(56.0 * n / us * 1e-3, 1),
                         "plan": ctx.last_plan()}
        small[str(size)] = ent
        log(f"small block n_i={size}: " + " ".join(
            f"{pp}={ent[pp]['us']} us (graph {ent[pp]['graph_us']} us)" for pp in precs))
    return small


def adjoint_leg(nb, W, ctx, dev):
    """Adjoint of the regular force at N = 65536 Plummer + Kroupa, all bodies
    active, FP64, in steady state; roofline by the algorithmic flops of both
    passes over the whole call's time."""
    s5 = W.adjoint_plummer_n65536()
    n5 = s5["n"]
    a5 = [dev(s5[k]) for k in ("x", "v", "m", "i_block", "rs2", "w_a", "w_j")]
    ms = steady_ms(lambda: nb.regular_force_adjoint(*a5, ctx=ctx))
    pp = float(n5) * (n5 - 1)
    ach = (ADJ_FLOPS_ROWS + ADJ_FLOPS_BODIES) * pp / ms * 1e-9
    log(f"adjoint: {ms:.2f} ms, {ach:.1f} TFLOP/s")
    return {"workload": f"N={n5} Plummer+Kroupa, all active, FP64",
            "ms": round(ms, 3), "gpairs_per_s_per_pass": round(pp / ms * 1e-6, 2),
            "roofline": {"bound": "alu", "achieved": round(ach, 2), "peak": PEAK_FP64,
                         "unit": "TFLOP/s", "frac": round(ach / PEAK_FP64, 4),
                         "flops_per_pair": {"row_pass": ADJ_FLOPS_ROWS,
                                            "body_pass": ADJ_FLOPS_BODIES},
                         "time": "whole call (both passes and their reductions)"}}


def small_configs_leg(nb, W, ctx, dev, precs):
    """GPU rates of the smaller workloads, in steady state (predict + regular
    force per call): N = 1024 equal-mass Plummer, all active, nb_cap 256; and
    N = 131072 Plummer + Kroupa with random blocks of 1, 32, 1024, 16384 and
    131072 rows, nb_cap 512."""
    import torch
    out = {}
    s1 = W.plummer_equal_n1024()
    s2 = W.plummer_kroupa_n131072()
    for name, s, blocks in (("plummer_equal_n1024", s1, {1024: s1["i_block"]}),
                            ("plummer_kroupa_n131072", s2, s2["blocks"])):
        x, v, a, jk, t0 = (dev(s[k]) for k in ("x", "v", "a", "jk", "t0"))
        m = dev(s["m"])
        xp = torch.empty_like(x)
        vp = torch.empty_like(v)
        n = s["n"]
        ent = {}
        for size, blk in blocks.items():
            bd, rd = dev(blk), dev(s["rs2"][blk])
            row = {}
            for prec in precs:
                o = nb.regular_force(x, v, m, bd, rd, s["nb_cap"], prec, ctx=ctx)

                def call():
                    nb.predict(x, v, a, jk, t0, s["t"], out=(xp, vp), ctx=ctx)
                    nb.regular_force(xp, vp, m, bd, rd, s["nb_cap"], prec, out=o, ctx=ctx)
                ms = steady_ms(call)
                row[prec] = {"ms": round(ms, 4),
                             "gpairs_per_s": round(blk.size * (n - 1) / ms * 1e-6, 2),
                             "plan": ctx.last_plan()}
                del o
            ent[str(size)] = row
            log(f"{name} n_i={size}: " + " ".join(
                f"{p}={row[p]['gpairs_per_s']} G/s" for p in precs))
        out[name] = ent
    return out


def oracle_leg(W, threads):
    """The CPU oracle (plain FP64 C, OpenMP over rows) on the other workloads,
    in full: N = 1024 all active; N = 131072 blocks of 1 .. 131072 rows; the
    256-cluster ensemble cluster by cluster; the N = 65536 adjoint."""
    import oracle
    res = {}

    def timed(fn):
        c1 = time.perf_counter()
        fn()
        return time.perf_counter() - c1

    s1 = W.plummer_equal_n1024()
    ox, ov = oracle.predict(s1["t"], s1["x"], s1["v"], s1["a"], s1["jk"], s1["t0"])
    p1 = 1024.0 * 1023
    dt = timed(lambda: oracle.regular(ox, ov, s1["m"], s1["i_block"], s1["rs2"], 256))
    res["plummer_equal_n1024"] = {"pairs": p1, "s": round(dt, 3),
                                  "gpairs_per_s": round(p1 / dt * 1e-9, 4)}
    s2 = W.plummer_kroupa_n131072()
    ox, ov = oracle.predict(s2["t"], s2["x"], s2["v"], s2["a"], s2["jk"], s2["t0"])
    n2 = s2["n"]
    p2, dt = 0.0, 0.0
    for blk in s2["blocks"].values():
        dt += timed(lambda: oracle.regular(ox, ov, s2["m"], blk, s2["rs2"][blk], 512))
        p2 += blk.size * (n2 - 1.0)
    res["plummer_kroupa_n131072_all_blocks"] = {"pairs": p2, "s": round(dt, 3),
                                                "gpairs_per_s": round(p2 / dt * 1e-9, 4)}
    log(f"oracle: N=131072 blocks {p2:.3g} pairs in {dt:.1f}s")
    s4 = W.cluster_ensemble_256()
    ox, ov = oracle.predict(s4["t"], s4["x"], s4["v"], s4["a"], s4["jk"], s4["t0"])
    p4, dt = 0.0, 0.0
    for c in range(len(s4["j_off"]) - 1):
        j0, j1 = s4["j_off"][c], s4["j_off"][c + 1]
        r0, r1 = s4["i_off"][c], s4["i_off"][c + 1]
        ib = (s4["i_block"][r0:r1] - j0).astype(np.int32)
        dt += timed(lambda: oracle.regular(ox[:, j0:j1], ov[:, j0:j1], s4["m"][j0:j1], ib,
                                           s4["rs2"][r0:r1], s4["nb_cap"]))
        p4 += (r1 - r0) * float(j1 - j0)
    res["cluster_ensemble_256"] = {"pairs": p4, "s": round(dt, 3),
                                   "gpairs_per_s": round(p4 / dt * 1e-9, 4)}
    log(f"oracle: ensemble {p4:.3g} pairs in {dt:.1f}s")
    s5 = W.adjoint_plummer_n65536()
    n5 = s5["n"]
    dt = timed(lambda: oracle.adjoint(s5["x"], s5["v"], s5["m"], s5["i_block"], s5["rs2"],
                                      s5["w_a"], s5["w_j"]))
    p5 = float(n5) * (n5 - 1)
    res["adjoint_plummer_n65536"] = {"pairs_per_pass": p5, "s": round(dt, 3),
                                     "gpairs_per_s_per_pass": round(p5 / dt * 1e-9, 4)}
    log(f"oracle: adjoint {dt:.1f}s")
    res["threads"] = threads
    return res


def sched_leg(nb, W, s, ctx, dev, reps=20):
    """Sorting-list scheduler (section 3.3.1) on the cluster's step levels:
    full build, then the O(N_i) update of each level's block, weighted by how
    often each level is due in one 2^-3 cycle of the hierarchy."""
    import torch
    n = s["n"]
    k_max = 20
    lev_h = s["levels"].astype(np.int32)
    lev_d = dev(lev_h)
    order_d, le_d = nb.sched_build(lev_d, k_max, ctx=ctx)
    torch.cuda.synchronize()
    ctx.reset_timing()
    ctx.enable_timing(True)
    c1 = time.perf_counter()
    for _ in range(10):
        nb.sched_build(lev_d, k_max, order=order_d, level_end=le_d, ctx=ctx)
    torch.cuda.synchronize()
    b_wall = (time.perf_counter() - c1) * 1e6 / 10
    bms, bl = ctx.kernel_time(nb.CLASS_SCHED)
    b_us = bms * 1e3 / max(bl, 1)
    le_h = le_d.cpu().numpy()
    per_level, cyc_us, cyc_bodies = {}, 0.0, 0
    for L in range(3, k_max + 1):
        n_a = int(le_h[L])
        if n_a == 0:
            continue
        ctx.reset_timing()
        c1 = time.perf_counter()
        for _ in range(reps):
            nb.sched_update(order_d, le_d, n_a, L, lev_d, k_max, ctx=ctx)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - c1) * 1e6 / reps
        ums, ul = ctx.kernel_time(nb.CLASS_SCHED)
        us = ums * 1e3 / max(ul, 1)
        per_level[str(L)] = {"n_active": n_a, "update_us": round(us, 2),
                             "wall_us": round(wall, 2),
                             "GB_per_s": round(28.0 * n_a / us * 1e-3, 1)}
        cyc_us += W.level_weight(L) * us
        cyc_bodies += W.level_weight(L) * n_a
    ctx.enable_timing(False)
    blocks = sum(W.level_weight(L) for L in range(3, k_max + 1) if str(L) in per_level)
    log(f"sched: build {b_us:.1f} us, cycle of {blocks} blocks: update "
        f"{cyc_us * 1e-3:.2f} ms ({cyc_us / max(blocks, 1):.1f} us/block)")
    return {
        "workload": f"N={n} step levels 3..20 of the same cluster, k_max {k_max}",
        "build_us": round(b_us, 2), "build_wall_us": round(b_wall, 2),
        "build_GB_per_s": round(12.0 * n / b_us * 1e-3, 1),
        "update_per_level": per_level,
        "cycle": {"blocks": blocks, "active_bodies": cyc_bodies,
                  "update_ms": round(cyc_us * 1e-3, 3),
                  "mean_update_us": round(cyc_us / max(blocks, 1), 2)}}


def radius_leg(nb, W, s, ctx, dev, x, v, a, jk, m, precs, L=10, cap=48, nnbopt=40):
    """Neighbour-radius control on one step level's block of the same cluster:
    the next-step radius update of the full block, and the regular force with
    overflowed rows shrunk and recomputed, against the plain regular force of
    the same block and cap."""
    import torch
    n = s["n"]
    tl, t0l, bl = W.binary_cluster_level(s, L)
    xp, vp, _ = nb.predict(x, v, a, jk, dev(t0l), tl, ctx=ctx)
    bd = dev(bl)
    rs2_0 = dev(s["rs2"][bl])
    out = {"workload": f"N={n}, level {L} block ({bl.size} rows), nb_cap {cap}, "
                       f"NNBOPT {nnbopt}, radii from the 64th neighbour"}
    for prec in precs:
        plain = nb.regular_force(xp, vp, m, bd, rs2_0, cap, prec, ctx=ctx)
        over = int((plain[2] > cap).sum().item())
        torch.cuda.synchronize()
        c1 = time.perf_counter()
        nb.regular_force(xp, vp, m, bd, rs2_0, cap, prec, ctx=ctx)
        torch.cuda.synchronize()
        t_plain = (time.perf_counter() - c1) * 1e3
        rs2 = rs2_0.clone()
        torch.cuda.synchronize()
        c1 = time.perf_counter()
        res = nb.regular_force_fit(xp, vp, m, bd, rs2, cap, nnbopt, 8, prec, ctx=ctx)
        torch.cuda.synchronize()
        t_fit = (time.perf_counter() - c1) * 1e3
        out[prec] = {"plain_ms": round(t_plain, 3), "fit_ms": round(t_fit, 3),
                     "rounds": res[5], "rows_overflowing_before": over,
                     "overflow_after": int(res[4].item())}
        log(f"radius fit {prec}: plain {t_plain:.2f} ms, fit {t_fit:.2f} ms, "
            f"{over} rows overflowed, {res[5]} rounds")
    # next-step radius update of the full 2^20 block (HBM-bound, 20 B per row)
    full = dev(s["rs2"])
    cnt = torch.full((n,), 70, dtype=torch.int32, device="cuda")
    nb.radius_update(cnt, full, 64, ctx=ctx)
    torch.cuda.synchronize()
    ctx.reset_timing()
    ctx.enable_timing(True)
    for _ in range(20):
        nb.radius_update(cnt, full, 64, ctx=ctx)
    ums, ul = ctx.kernel_time(nb.CLASS_RADIUS)
    ctx.enable_timing(False)
    us = ums * 1e3 / max(ul, 1)
    out["update_full_block_us"] = round(us, 2)
    out["update_GB_per_s"] = round(20.0 * n / us * 1e-3, 1)
    log(f"radius update, {n} rows: {us:.1f} us ({20.0 * n / us * 1e-3:.0f} GB/s)")
    return out


def step_leg(nb, s, ctx, x, v, a, jk, m, xp, vp, ibd, out, t, t0d):
    """The rest of the Ahmad-Cohen block step at the full 2^20 block: the
    irregular force over the lists of the regular pass just timed (gathers),
    the Hermite corrector (streaming) and the O(N^2) potential (FP64 ALU).
    Each figure is the library's own HIP-event time of that kernel class."""
    import torch
    n = s["n"]
    cap = s["nb_cap"]

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        ctx.reset_timing()
        ctx.enable_timing(True)
        for _ in range(reps):
            fn()
        ms, calls = ctx.kernel_time(nb.CLASS_STEP)
        ctx.enable_timing(False)
        return ms / max(calls, 1)

    # the lists in `out` belong to the full block at time t: predict to t again
    nb.predict(x, v, a, jk, t0d, t, out=(xp, vp), ctx=ctx)
    res = {}
    pairs = float(out[2].clamp(max=cap).sum().item())
    ms = timed(lambda: nb.irregular_force(xp, vp, m, ibd, cap, out[2], out[3], ctx=ctx), 5)
    # algorithmic bytes per neighbour pair: the neighbour's xp, vp, m (56 B) and its
    # list entry (4 B); the rows' own state is negligible
    res["irregular"] = {"ms": round(ms, 4), "pairs": pairs,
                        "gpairs_per_s": round(pairs / ms * 1e-6, 2),
                        "roofline": {"bound": "hbm", "achieved": round(60.0 * pairs / ms * 1e-6, 1),
                                     "peak": 8000.0, "unit": "GB/s",
                                     "frac": round(60.0 * pairs / ms * 1e-6 / 8000.0, 4)}}
    h = torch.full((n,), 2.0 ** -10, dtype=torch.float64, device="cuda")
    ms = timed(lambda: nb.hermite_correct(h, x, v, a, jk, out[0], out[1], ctx=ctx), 10)
    # 1 + 6 x 3 doubles read, 4 x 3 written per entry
    res["corrector"] = {"ms": round(ms, 4), "entries": n,
                        "roofline": {"bound": "hbm", "achieved": round(248.0 * n / ms * 1e-6, 1),
                                     "peak": 8000.0, "unit": "GB/s",
                                     "frac": round(248.0 * n / ms * 1e-6 / 8000.0, 4)}}
    ms = timed(lambda: nb.potential(x, m, ctx=ctx), 1)
    pp = float(n) * (n - 1)
    # 11 flops per pair: 3 differences, r2 5, rsqrt 1, the m/r accumulation 2
    res["potential"] = {"ms": round(ms, 3), "gpairs_per_s": round(pp / ms * 1e-6, 2),
                        "roofline": {"bound": "alu", "achieved": round(11.0 * pp / ms * 1e-9, 2),
                                     "peak": PEAK_FP64, "unit": "TFLOP/s",
                                     "frac": round(11.0 * pp / ms * 1e-9 / PEAK_FP64, 4)}}
    log(f"step: irregular {res['irregular']['ms']:.3f} ms ({res['irregular']['gpairs_per_s']} G pairs/s), "
        f"corrector {res['corrector']['ms']:.3f} ms, potential {res['potential']['ms']:.1f} ms")
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=1 << 20)
    ap.add_argument("--cpu-rows", type=int, default=16384,
                    help="rows of the full block timed on the CPU oracle (0 = skip)")
    ap.add_argument("--no-oracle-configs", action="store_true",
                    help="skip timing the CPU oracle on the other workloads")
    ap.add_argument("--no-levels", action="store_true")
    ap.add_argument("--only", choices=["both", "mixed", "fp64"], default="both")
    ap.add_argument("--step-only", action="store_true",
                    help="only time the rest of the block step (irregular force, corrector, "
                         "potential) at the full block and print its figures")
    ap.add_argument("--sched-only", action="store_true",
                    help="only time the block-step scheduler on the same cluster's levels "
                         "and print its figures (used for kernel profiles)")
    ap.add_argument("--small-only", action="store_true",
                    help="only time the small blocks (1, 32, 1024, 320 random rows of the 2^20 "
                         "cluster) and print their figures (used for kernel profiles)")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="only time the adjoint at N = 65536 (all active, FP64) and print "
                         "its figures (used for kernel profiles)")
    ap.add_argument("--batched-profile", action="store_true",
                    help="only replay the 256-cluster batched call three times in mixed "
                         "precision and three times in FP64, at the default shape (used for "
                         "kernel profiles)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (FP64 elementwise kernel) "
                         "and print its bandwidth; used to scale rocprofv3 byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_probe:
        n = args.copy_probe * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        reps = 5
        t1 = time.perf_counter()
        for _ in range(reps):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t1) / reps
        print(json.dumps({"copy_probe_bytes_read": n * 8, "copy_probe_bytes_written": n * 8,
                          "launches": reps + 1, "GB_per_s": round(2 * n * 8 / dt * 1e-9, 1)}))
        return

    import paper_1504_03687_amd as nb
    import workloads as W

    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    if args.adjoint_only:
        ctx = nb.Context(0)
        print(json.dumps({"adjoint": adjoint_leg(nb, W, ctx, dev)}), flush=True)
        return
    if args.batched_profile:
        ctx = nb.Context(0)
        s4 = W.cluster_ensemble_256()
        xp4, vp4, _ = nb.predict(dev(s4["x"]), dev(s4["v"]), dev(s4["a"]), dev(s4["jk"]),
                                 dev(s4["t0"]), s4["t"], ctx=ctx)
        b4 = (s4["j_off"], s4["i_off"], xp4, vp4, dev(s4["m"]), dev(s4["i_block"]),
              dev(s4["rs2"]))
        plans = {}
        for prec in ("mixed", "fp64"):
            o4 = nb.regular_force_batched(*b4, s4["nb_cap"], prec, ctx=ctx)
            for _ in range(2):
                nb.regular_force_batched(*b4, s4["nb_cap"], prec, out=o4, ctx=ctx)
            torch.cuda.synchronize()
            plans[prec] = ctx.last_plan()
        print(json.dumps({"batched_profile": plans}), flush=True)
        return
    t_gen = time.time()
    s = W.binary_cluster_n1m(args.n)
    n = s["n"]
    t, t0, blk = W.binary_cluster_level(s, 3)
    log(f"workload generated in {time.time() - t_gen:.1f}s: n={n} full block={blk.size}")
    x, v, a, jk, m = dev(s["x"]), dev(s["v"]), dev(s["a"]), dev(s["jk"]), dev(s["m"])
    t0d, ibd, rs2d = dev(t0), dev(blk), dev(s["rs2"][blk])
    cap = s["nb_cap"]
    n_i = blk.size
    pairs = float(n_i) * float(n - 1)
    xp = torch.empty_like(x)
    vp = torch.empty_like(v)
    out = (torch.empty((3, n_i), dtype=torch.float64, device="cuda"),
           torch.empty((3, n_i), dtype=torch.float64, device="cuda"),
           torch.empty(n_i, dtype=torch.int32, device="cuda"),
           torch.empty((n_i, cap), dtype=torch.int32, device="cuda"),
           torch.empty(1, dtype=torch.int32, device="cuda"))
    ctx = nb.Context(0)
    if args.step_only:
        nb.predict(x, v, a, jk, t0d, t, out=(xp, vp), ctx=ctx)
        nb.regular_force(xp, vp, m, ibd, rs2d, cap, "mixed", out=out, ctx=ctx)
        print(json.dumps({"step": step_leg(nb, s, ctx, x, v, a, jk, m, xp, vp, ibd, out, t,
                                           t0d)}), flush=True)
        return
    if args.sched_only:
        print(json.dumps({"sched": sched_leg(nb, W, s, ctx, dev)}), flush=True)
        return
    if args.small_only:
        nb.predict(x, v, a, jk, t0d, t, out=(xp, vp), ctx=ctx)
        precs = ["mixed", "fp64"] if args.only == "both" else [args.only]
        print(json.dumps({"small_blocks": small_blocks_leg(nb, ctx, dev, s, xp, vp, m, cap,
                                                           precs)}), flush=True)
        return

    def step(prec):
        nb.predict(x, v, a, jk, t0d, t, out=(xp, vp), ctx=ctx)
        nb.regular_force(xp, vp, m, ibd, rs2d, cap, prec, out=out, ctx=ctx)

    res = {}
    precs = ["mixed", "fp64"] if args.only == "both" else [args.only]
    for prec in precs:
        for _ in range(args.warmup):
            step(prec)
        torch.cuda.synchronize()
        ctx.reset_timing()
        ctx.enable_timing(True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.steps):
            step(prec)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        kms, kl = ctx.kernel_time(nb.CLASS_FORCE)
        mms, ml = ctx.kernel_time(nb.CLASS_MERGE)
        pms, pl = ctx.kernel_time(nb.CLASS_PREDICT)
        rms, rl = ctx.kernel_time(nb.CLASS_REDO)
        ctx.enable_timing(False)
        refined = ctx.last_refined_rows() if prec == "mixed" else 0
        ms_step = (t2 - t1) * 1e3 / args.steps
        res[prec] = dict(ms_per_step=ms_step, pairs_per_s=pairs / (ms_step * 1e-3),
                         force_kernel_ms=kms / max(kl, 1), merge_kernel_ms=mms / max(ml, 1),
                         predict_kernel_ms=pms / max(pl, 1), refine_kernel_ms=rms / max(rl, 1),
                         refined_rows=refined, plan=ctx.last_plan(),
                         overflow=int(out[4].item()))
        log(f"{prec}: {ms_step:.2f} ms/step, {pairs / ms_step * 1e-6:.1f} G pairs/s, "
            f"force kernel {res[prec]['force_kernel_ms']:.2f} ms, plan {ctx.last_plan()}")

    # per-level blocks of the step hierarchy (occurrence-weighted aggregate)
    levels = None
    if not args.no_levels:
        levels = {}
        tot_pairs = {p: 0.0 for p in precs}
        tot_time = {p: 0.0 for p in precs}
        for L in range(3, 21):
            tl, t0l, bl = W.binary_cluster_level(s, L)
            if bl.size == 0:
                continue
            w = W.level_weight(L)
            bd, rd, t0ld = dev(bl), dev(s["rs2"][bl]), dev(t0l)
            ent = {"n_i": int(bl.size), "weight": w}
            for prec in precs:
                def level_call():
                    nb.predict(x, v, a, jk, t0ld, tl, out=(xp, vp), ctx=ctx)
                    nb.regular_force(xp, vp, m, bd, rd, cap, prec, ctx=ctx)
                ms = steady_ms(level_call)
                p = float(bl.size) * (n - 1)
                ent[prec] = {"ms": round(ms, 4), "gpairs_per_s": round(p / ms * 1e-6, 2)}
                tot_pairs[prec] += w * p
                tot_time[prec] += w * ms
            levels[str(L)] = ent
            log(f"level {L}: n_i={bl.size} " + " ".join(
                f"{pp}={ent[pp]['gpairs_per_s']} G/s" for pp in precs))
        levels["aggregate_gpairs_per_s"] = {
            p: round(tot_pairs[p] / tot_time[p] * 1e-6, 2) for p in precs}

    # small blocks (HBM / latency bound): random rows of the same cluster
    small = {}
    if not args.no_levels:
        small = small_blocks_leg(nb, ctx, dev, s, xp, vp, m, cap, precs)

    # adjoint (N = 65536 all active, FP64) and the batched ensemble
    # (256 clusters, one graph launch), each timed in steady state
    extras = {}
    if not args.no_levels:
        extras["adjoint"] = adjoint_leg(nb, W, ctx, dev)
        s4 = W.cluster_ensemble_256()
        xp4, vp4, _ = nb.predict(dev(s4["x"]), dev(s4["v"]), dev(s4["a"]), dev(s4["jk"]),
                                 dev(s4["t0"]), s4["t"], ctx=ctx)
        b4 = (s4["j_off"], s4["i_off"], xp4, vp4, dev(s4["m"]), dev(s4["i_block"]),
              dev(s4["rs2"]))
        sizes = np.diff(s4["j_off"])
        rows = np.diff(s4["i_off"])
        pairs4 = float((sizes * rows).sum())
        for prec in precs:
            # the default shape rule first, then the shape the batched tuner
            # picks for this ensemble
            o4 = nb.regular_force_batched(*b4, s4["nb_cap"], prec, ctx=ctx)
            ms = steady_ms(
                lambda: nb.regular_force_batched(*b4, s4["nb_cap"], prec, out=o4, ctx=ctx))
            ent = {"workload": "256 clusters, N log-uniform [1024, 32768], active 1-100%",
                   "default": {"ms": round(ms, 3), "gpairs_per_s": round(pairs4 / ms * 1e-6, 2),
                               "plan": ctx.last_plan()}}
            log(f"batched {prec} (default shape): {ms:.2f} ms, "
                f"{pairs4 / ms * 1e-6:.1f} G pairs/s")
            c1 = time.perf_counter()
            nb.autotune_batched(*b4, s4["nb_cap"], prec, out=o4, force=True, ctx=ctx)
            torch.cuda.synchronize()
            tune_s = time.perf_counter() - c1
            ms = steady_ms(
                lambda: nb.regular_force_batched(*b4, s4["nb_cap"], prec, out=o4, ctx=ctx))
            ent.update({"ms": round(ms, 3), "gpairs_per_s": round(pairs4 / ms * 1e-6, 2),
                        "plan": ctx.last_plan(), "tuning_s": round(tune_s, 2)})
            extras[f"batched_{prec}"] = ent
            log(f"batched {prec} (tuned, {tune_s:.1f}s to tune): {ms:.2f} ms, "
                f"{pairs4 / ms * 1e-6:.1f} G pairs/s, {ctx.last_plan()}")
            del o4

    if not args.no_levels:
        extras["step"] = step_leg(nb, s, ctx, x, v, a, jk, m, xp, vp, ibd, out, t, t0d)
        extras["sched"] = sched_leg(nb, W, s, ctx, dev)
        extras["radius"] = radius_leg(nb, W, s, ctx, dev, x, v, a, jk, m, precs)
        extras["small_configs"] = small_configs_leg(nb, W, ctx, dev, precs)

    # CPU oracle on a bounded sample of the same full block, then the other
    # workloads in full
    cpu = None
    if args.cpu_rows > 0:
        import oracle
        rng = np.random.default_rng(0)
        rows = rng.choice(n_i, min(args.cpu_rows, n_i), replace=False)
        ox, ov = oracle.predict(t, s["x"], s["v"], s["a"], s["jk"], t0)
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        c1 = time.perf_counter()
        oracle.regular(ox, ov, s["m"], blk[rows], s["rs2"][blk][rows], cap)
        dt = time.perf_counter() - c1
        cpu = {"value": round(rows.size * (n - 1) / dt * 1e-9, 4), "unit": "G pairs/s",
               "cores": threads, "kind": "oracle", "cpu_model": cpu_model(),
               "sample": f"{rows.size} random rows of the N=2^20 full block against all "
                         f"{n} bodies ({rows.size * (n - 1):.3g} pairs, {dt:.1f}s, FP64)"}
        log(f"cpu oracle: {cpu['value']} G pairs/s on {threads} threads ({cpu['cpu_model']})")
        if "sched" in extras:
            # the oracle's plain O(N) search for the next block over all bodies
            import oracle.sched as osched
            tt = np.zeros(n)
            dts = np.ldexp(1.0, -s["levels"].astype(np.int64))
            c1 = time.perf_counter()
            for _ in range(5):
                osched.next_block(tt, dts)
            extras["sched"]["cpu_oracle_full_search_ms"] = round(
                (time.perf_counter() - c1) * 1e3 / 5, 3)
        if not args.no_levels and not args.no_oracle_configs:
            extras["cpu_oracle_other_workloads"] = oracle_leg(W, threads)

    head = res.get("mixed") or res["fp64"]
    dom = "mixed" if "mixed" in res else "fp64"
    kernel_s = res[dom]["force_kernel_ms"] * 1e-3
    achieved = FLOPS_PER_PAIR * pairs / kernel_s * 1e-12
    peak = PEAK_FP32 if dom == "mixed" else PEAK_FP64
    line = {
        "metric": "regular force+jerk pair interactions/s (G/s) & % VALU peak, N=2^20, "
                  "mixed vs FP64",
        "value": round(head["pairs_per_s"] * 1e-9, 3),
        "unit": "G pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if dom == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": "N=2^20 Plummer + Kroupa IMF, 5% primordial binaries, full "
                               "block (all bodies active), predict + regular force, nb_cap 1024",
                   "n": n, "n_i": n_i, "pairs_per_step": pairs},
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": peak,
                     "unit": "TFLOP/s", "frac": round(achieved / peak, 4),
                     "traffic": profiled(dom, "hbm_bytes_per_launch"),
                     "kernel": f"force_rows_kernel ({dom})",
                     "flops_per_pair": FLOPS_PER_PAIR,
                     "issue_model_frac": profiled(dom, "issue_model_frac")},
        "cpu_baseline": cpu,
        "precisions": {p: {"gpairs_per_s": round(r["pairs_per_s"] * 1e-9, 3),
                           "ms_per_step": round(r["ms_per_step"], 3),
                           "force_kernel_ms": round(r["force_kernel_ms"], 3),
                           "merge_kernel_ms": round(r["merge_kernel_ms"], 3),
                           "predict_kernel_ms": round(r["predict_kernel_ms"], 4),
                           "refine_kernel_ms": round(r["refine_kernel_ms"], 3),
                           "refined_rows": r["refined_rows"],
                           "plan": r["plan"], "overflow": r["overflow"]}
                       for p, r in res.items()},
        "levels": levels,
        "small_blocks": small or None,
        "extras": extras or None,
    }
    if "mixed" in res and "fp64" in res:
        line["mixed_over_fp64"] = round(res["mixed"]["pairs_per_s"] / res["fp64"]["pairs_per_s"], 3)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
