"""Writes henon_scale.json: the exact Henon-unit corrections of the named
workloads.

Each named workload is sampled as in workloads/__init__.py (Plummer sphere at
the analytic scale length 3 pi / 16, masses normalised to 1, centre of mass at
rest at the origin; for the binary cluster, its centre-of-mass system).  The
oracle's O(N^2) FP64 potential gives its potential energy U, and
T = 1/2 sum m v^2 its kinetic energy; the stored factors cx = -2 U and
cv = 1 / (2 sqrt(T)) then scale positions and velocities so that U = -1/2 and
T = 1/4: E = -1/4 and virial ratio 1/2 exactly (up to rounding) in
G = M = 1 units, the N-body units the paper's runs use.

    python -m workloads.henon_scale [--only PREFIX]

The million-body entry takes about ten minutes on eight cores.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402


def _samples():
    """(key, x, v, m) of every named workload before the correction."""
    x, v, m = W.plummer(W.rng_for(1), 1024, "equal")
    yield "plummer_equal_n1024", x, v, m
    x, v, m = W.plummer(W.rng_for(2), 131072, "kroupa")
    yield "plummer_kroupa_n131072", x, v, m
    x, v, m = W.plummer(W.rng_for(5), 65536, "kroupa")
    yield "adjoint_plummer_n65536", x, v, m
    rng = W.rng_for(4)
    ns = np.exp(rng.uniform(math.log(1024), math.log(32768), 256)).round().astype(np.int64)
    for c in range(256):
        x, v, m = W.plummer(W.rng_for(4, c), int(ns[c]), "kroupa")
        yield f"cluster_ensemble_256/{c}", x, v, m
    n = 1 << 20
    x, v, m = W.plummer_with_binaries(W.rng_for(3), n, n // 40, cm_only=True)
    yield "binary_cluster_n1m", x, v, m


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", default="", help="recompute only keys with this prefix")
    args = ap.parse_args()
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "henon_scale.json")
    table = {}
    if os.path.exists(path):
        with open(path) as f:
            table = json.load(f)
    for key, x, v, m in _samples():
        if not key.startswith(args.only):
            continue
        t0 = time.time()
        U, _ = oracle.potential(x, m)
        T = 0.5 * float((m * (v * v).sum(0)).sum())
        table[key] = {"n": int(m.size), "U": U, "T": T, "cx": -2.0 * U,
                      "cv": 1.0 / (2.0 * math.sqrt(T))}
        print(f"{key}: n={m.size} U={U:.12f} T={T:.12f} ({time.time() - t0:.1f}s)",
              flush=True)
        with open(path + ".tmp", "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
        os.replace(path + ".tmp", path)


if __name__ == "__main__":
    main()
