"""Helpers shared by the GPU parity tests: moving seeded numpy inputs to the
GPU, and comparing the library's outputs with the oracle's."""
import sys

import numpy as np
import torch

import oracle

TOL_FP64 = 1e-12   # max per-row relative error (norm-wise), FP64 kernels
TOL_MIXED = 5e-6   # max per-row relative error (norm-wise), mixed kernels


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    return t.detach().cpu().numpy()


def row_rel_err(got, ref):
    """Per-row norm-wise relative error ||got - ref|| / ||ref||; rows whose
    reference is exactly zero must be exactly zero (error 0 or inf)."""
    d = np.linalg.norm(got - ref, axis=0)
    r = np.linalg.norm(ref, axis=0)
    out = np.where(r > 0, d / np.where(r > 0, r, 1.0), np.where(d == 0, 0.0, np.inf))
    return out


def check_lists(cnt, lst, ocnt, olst, cap):
    """Neighbour counts and the defined part of every list are bit-identical."""
    assert np.array_equal(cnt, ocnt), f"counts differ at rows {np.nonzero(cnt != ocnt)[0][:10]}"
    for b in np.nonzero(ocnt > 0)[0]:
        k = min(int(ocnt[b]), cap)
        if not np.array_equal(lst[b, :k], olst[b, :k]):
            raise AssertionError(f"list of row {b} differs: {lst[b, :k][:8]} vs {olst[b, :k][:8]}")


def oracle_rows(xp, vp, m, i_block, rs2, cap, rows=None):
    """The oracle's regular force for all rows of a block (or a subset);
    pass the result to compare_force(ref=...) to check several GPU results
    against one oracle run."""
    ib = np.asarray(i_block)
    r2 = np.asarray(rs2)
    sel = np.arange(ib.size) if rows is None else np.asarray(rows)
    return sel, oracle.regular(xp, vp, m, ib[sel], r2[sel], cap)


def compare_force(res, xp, vp, m, i_block, rs2, cap, tol, rows=None, ref=None):
    """res: tuple from paper_1504_03687_amd.regular_force (GPU tensors).
    Compares all rows (or the given subset) with the oracle; returns max errors.
    ref: a precomputed oracle_rows(...) result for the same rows."""
    acc, jerk, cnt, lst, ovf = (host(t) for t in res)
    sel, (oa, oj, oc, ol, oo, obad) = (
        ref if ref is not None else oracle_rows(xp, vp, m, i_block, rs2, cap, rows))
    check_lists(cnt[sel], lst[sel] if cap > 0 else lst, oc, ol, cap)
    ea = row_rel_err(acc[:, sel], oa)
    ej = row_rel_err(jerk[:, sel], oj)
    assert ea.max() <= tol, f"acc error {ea.max():.3e} > {tol} at row {sel[ea.argmax()]}"
    assert ej.max() <= tol, f"jerk error {ej.max():.3e} > {tol} at row {sel[ej.argmax()]}"
    if sel.size == acc.shape[1] and np.array_equal(sel, np.arange(sel.size)):
        assert int(ovf[0]) == int(oo)   # every row checked: the overflow word too
    return float(ea.max()), float(ej.max())
