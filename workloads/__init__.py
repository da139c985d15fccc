"""Seeded synthetic star-cluster inputs shared by the oracle tests, the GPU tests
and the benchmark.

This module only *draws inputs*: Plummer spheres in Henon (N-body) units, Kroupa
(2001) initial masses, primordial binaries, Hermite power-of-two step levels,
neighbour radii from the 64th-nearest body, active i-blocks and cluster
ensembles.  It contains none of the regular-force arithmetic (no pair force,
jerk, neighbour test or predictor); those live in the oracle and, separately, in
the HIP library.

Recipes follow the workloads the paper runs (Plummer models with a Kroupa IMF,
optionally 5% primordial binaries; sections 4.1, 4.2 and 4.4) and the paper's
description of block time steps as powers of 0.5 (section 2, section 3.3.1).
Every array is float64 SoA: positions ``x`` have shape ``(3, n)``.
"""
from __future__ import annotations

import functools
import json
import math
import os

import numpy as np
from scipy.spatial import cKDTree

SEED_BASE = 1504036870

#: Henon units: G = M = 1, E = -1/4.  A Plummer sphere of scale length b has
#: E = -3 pi / (64 b) at G = M = 1, so E = -1/4 needs b = 3 pi / 16.  Samples
#: are drawn at this scale; the named workloads below are then rescaled
#: exactly (see henon_correction).
PLUMMER_B = 3.0 * math.pi / 16.0

_HENON_TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "henon_scale.json")


@functools.lru_cache(maxsize=1)
def _henon_table() -> dict:
    with open(_HENON_TABLE) as f:
        return json.load(f)


def henon_correction(key: str):
    """(cx, cv): the factors that take the sampled (analytically scaled) state
    of a named workload to exact Henon units.  With U the potential energy and
    T the kinetic energy of the sampled state (total mass 1), x -> cx x and
    v -> cv v with cx = -2 U and cv = 1 / (2 sqrt(T)) give U = -1/2 and
    T = 1/4, so E = -1/4 and 2T = -U.  The factors are computed once, with the
    oracle's O(N^2) potential, by workloads/henon_scale.py and stored in
    henon_scale.json."""
    e = _henon_table()[key]
    return float(e["cx"]), float(e["cv"])


def rng_for(k: int, *spawn) -> np.random.Generator:
    """Generator for workload number ``k`` (1..5: the five workload builders
    below, in order); ``spawn`` selects a child stream."""
    if spawn:
        ss = np.random.SeedSequence(SEED_BASE + k)
        child = ss.spawn(spawn[0] + 1)[spawn[0]]
        return np.random.Generator(np.random.PCG64(child))
    return np.random.Generator(np.random.PCG64(SEED_BASE + k))


# --------------------------------------------------------------------------- #
# masses
# --------------------------------------------------------------------------- #
def kroupa_masses(rng: np.random.Generator, n: int, m_lo=0.08, m_br=0.5, m_hi=100.0,
                  a1=1.3, a2=2.3) -> np.ndarray:
    """Kroupa (2001) two-segment power law dN/dm ~ m^-a1 on [m_lo, m_br),
    m^-a2 on [m_br, m_hi], continuous at m_br; drawn by segment-wise inverse CDF.
    Returned in solar masses (not normalised)."""

    def seg_int(a, lo, hi):  # integral of m^-a dm
        return (hi ** (1 - a) - lo ** (1 - a)) / (1 - a)

    c2 = m_br ** (a2 - a1)  # continuity factor for the upper segment
    w1 = seg_int(a1, m_lo, m_br)
    w2 = c2 * seg_int(a2, m_br, m_hi)
    u_seg = rng.random(n)
    u = rng.random(n)
    lower = u_seg < w1 / (w1 + w2)

    def inv(a, lo, hi, uu):
        e = 1 - a
        return (lo ** e + uu * (hi ** e - lo ** e)) ** (1 / e)

    return np.where(lower, inv(a1, m_lo, m_br, u), inv(a2, m_br, m_hi, u))


# --------------------------------------------------------------------------- #
# Plummer sphere
# --------------------------------------------------------------------------- #
def _isotropic(rng, n):
    cth = rng.uniform(-1.0, 1.0, n)
    phi = rng.uniform(0.0, 2.0 * math.pi, n)
    sth = np.sqrt(1.0 - cth * cth)
    return np.stack([sth * np.cos(phi), sth * np.sin(phi), cth])


def plummer_positions_velocities(rng: np.random.Generator, n: int, x_max=0.999):
    """Aarseth, Henon & Wielen (1974) sampling at G = M = b = 1, truncated at
    mass fraction ``x_max``; then scaled to Henon units (b = 3 pi / 16)."""
    X = rng.uniform(0.0, x_max, n)
    X = np.maximum(X, 1e-300)
    r = 1.0 / np.sqrt(X ** (-2.0 / 3.0) - 1.0)
    pos = _isotropic(rng, n) * r
    # speed fraction q by von Neumann rejection on g(q) = q^2 (1 - q^2)^(7/2)
    q = np.empty(n)
    todo = np.arange(n)
    while todo.size:
        qq = rng.random(todo.size)
        yy = rng.random(todo.size) * 0.1
        ok = yy < qq * qq * (1.0 - qq * qq) ** 3.5
        q[todo[ok]] = qq[ok]
        todo = todo[~ok]
    speed = q * math.sqrt(2.0) * (1.0 + r * r) ** (-0.25)
    vel = _isotropic(rng, n) * speed
    pos *= PLUMMER_B
    vel /= math.sqrt(PLUMMER_B)
    return pos, vel


def _centre(x, v, m):
    x -= (x @ m)[:, None] / m.sum()
    v -= (v @ m)[:, None] / m.sum()


def plummer(rng: np.random.Generator, n: int, imf: str = "equal", henon_key: str | None = None):
    """Plummer sphere of ``n`` bodies, total mass 1, centre of mass at rest at 0.
    With ``henon_key`` the state is rescaled to exact Henon units by the stored
    factors of that workload (henon_correction)."""
    x, v = plummer_positions_velocities(rng, n)
    if imf == "equal":
        m = np.full(n, 1.0 / n)
    elif imf == "kroupa":
        m = kroupa_masses(rng, n)
        m /= m.sum()
    else:
        raise ValueError(imf)
    _centre(x, v, m)
    if henon_key is not None:
        cx, cv = henon_correction(henon_key)
        x *= cx
        v *= cv
    return np.ascontiguousarray(x), np.ascontiguousarray(v), m


# --------------------------------------------------------------------------- #
# primordial binaries
# --------------------------------------------------------------------------- #
def _kepler_E(M, e, iters=40):
    E = np.where(e < 0.8, M, np.pi * np.ones_like(M))
    for _ in range(iters):
        f = E - e * np.sin(E) - M
        E = E - f / (1.0 - e * np.cos(E))
    return E


def plummer_with_binaries(rng: np.random.Generator, n: int, n_bin: int,
                          a_lo=1e-5, a_hi=1e-3, henon_key: str | None = None,
                          cm_only: bool = False):
    """``n`` bodies of which ``2*n_bin`` are components of primordial binaries.

    Centres of mass (n - n_bin of them) follow a Plummer sphere; every component
    mass is an independent Kroupa draw; total mass is 1.  Binary orbits: semi-major
    axis log-uniform in [a_lo, a_hi], thermal eccentricity (e = sqrt(U)),
    isotropic orientation, uniform mean anomaly.  Binary components occupy
    indices 0 .. 2*n_bin-1, pairs adjacent (2k, 2k+1).
    With ``henon_key`` the centre-of-mass system is rescaled to exact Henon
    units (henon_correction) before the binary orbits are added.
    Returns x, v, m and the per-body orbital period (0 for single stars); with
    ``cm_only`` the centre-of-mass system (xc, vc, mc) right before that
    rescaling instead.
    """
    n_cm = n - n_bin
    xc, vc = plummer_positions_velocities(rng, n_cm)
    m1 = kroupa_masses(rng, n_bin)
    m2 = kroupa_masses(rng, n_bin)
    ms = kroupa_masses(rng, n_cm - n_bin)
    tot = m1.sum() + m2.sum() + ms.sum()
    m1, m2, ms = m1 / tot, m2 / tot, ms / tot
    mc = np.concatenate([m1 + m2, ms])
    _centre(xc, vc, mc)
    if cm_only:
        return xc, vc, mc
    if henon_key is not None:
        cx, cv = henon_correction(henon_key)
        xc *= cx
        vc *= cv

    a = np.exp(rng.uniform(math.log(a_lo), math.log(a_hi), n_bin))
    e = np.sqrt(rng.random(n_bin))
    Mmean = rng.uniform(0.0, 2.0 * math.pi, n_bin)
    E = _kepler_E(Mmean, e)
    mb = m1 + m2
    # relative orbit in its own plane (P along x, Q along y)
    cosE, sinE = np.cos(E), np.sin(E)
    sq = np.sqrt(1.0 - e * e)
    rx = a * (cosE - e)
    ry = a * sq * sinE
    rdot = np.sqrt(mb / a) / (1.0 - e * cosE)
    vx = -rdot * sinE
    vy = rdot * sq * cosE
    # random orientation: orthonormal frame from two isotropic draws
    P = _isotropic(rng, n_bin)
    t = _isotropic(rng, n_bin)
    Q = t - (t * P).sum(0) * P
    Q /= np.linalg.norm(Q, axis=0)
    rel_x = P * rx + Q * ry
    rel_v = P * vx + Q * vy

    x = np.empty((3, n))
    v = np.empty((3, n))
    m = np.empty(n)
    period = np.zeros(n)
    f1 = m2 / mb  # component 1 sits at +m2/M of the relative vector
    f2 = m1 / mb
    x[:, 0:2 * n_bin:2] = xc[:, :n_bin] + f1 * rel_x
    x[:, 1:2 * n_bin:2] = xc[:, :n_bin] - f2 * rel_x
    v[:, 0:2 * n_bin:2] = vc[:, :n_bin] + f1 * rel_v
    v[:, 1:2 * n_bin:2] = vc[:, :n_bin] - f2 * rel_v
    m[0:2 * n_bin:2] = m1
    m[1:2 * n_bin:2] = m2
    x[:, 2 * n_bin:] = xc[:, n_bin:]
    v[:, 2 * n_bin:] = vc[:, n_bin:]
    m[2 * n_bin:] = ms
    P_orb = 2.0 * math.pi * np.sqrt(a ** 3 / mb)
    period[0:2 * n_bin:2] = P_orb
    period[1:2 * n_bin:2] = P_orb
    return np.ascontiguousarray(x), np.ascontiguousarray(v), m, period


# --------------------------------------------------------------------------- #
# neighbour radii, blocks, predictor inputs
# --------------------------------------------------------------------------- #
def knn_rs2(x: np.ndarray, k: int = 64, workers: int = -1) -> np.ndarray:
    """Squared distance to the k-th nearest other body (float64)."""
    tree = cKDTree(x.T)
    d, _ = tree.query(x.T, k=k + 1, workers=workers)
    return d[:, k] ** 2


def random_block(rng: np.random.Generator, n: int, n_i: int) -> np.ndarray:
    """``n_i`` distinct body indices in random (unsorted) order, int32."""
    return rng.choice(n, size=n_i, replace=False).astype(np.int32)


def plummer_field(x, v, b=PLUMMER_B):
    """Analytic Plummer acceleration at x and its time derivative along v
    (G = M = 1); used only to give the predictor plausible a and da/dt inputs."""
    r2 = (x * x).sum(0) + b * b
    r3 = r2 ** 1.5
    rv = (x * v).sum(0)
    a = -x / r3
    jk = -v / r3 + 3.0 * rv * x / (r3 * r2)
    return a, jk


def binary_companion_field(x, v, m, n_bin):
    """Two-body acceleration and its derivative between binary components."""
    a = np.zeros_like(x)
    jk = np.zeros_like(x)
    if n_bin == 0:
        return a, jk
    i1 = np.arange(0, 2 * n_bin, 2)
    i2 = i1 + 1
    r = x[:, i2] - x[:, i1]
    u = v[:, i2] - v[:, i1]
    r2 = (r * r).sum(0)
    r3 = r2 ** 1.5
    s = (r * u).sum(0)
    g = r / r3
    dg = u / r3 - 3.0 * s * r / (r3 * r2)
    a[:, i1] = m[i2] * g
    a[:, i2] = -m[i1] * g
    jk[:, i1] = m[i2] * dg
    jk[:, i2] = -m[i1] * dg
    return a, jk


def step_levels(x, m, rs2, period=None, eta=0.1, k_min=3, k_max=20):
    """Hermite block-step level k (step 2^-k) per body: singles use
    eta * (G rho)^-1/2 with rho from the mass inside the neighbour sphere,
    binary components P_orb / 100; rounded down to a power of two and clamped."""
    n = m.size
    mbar = m.mean()
    rs3 = rs2 ** 1.5
    rho = 64.0 * mbar / (4.0 * math.pi * rs3 / 3.0)
    dt = eta / np.sqrt(rho)
    if period is not None:
        b = period > 0
        dt[b] = period[b] / 100.0
    k = np.ceil(-np.log2(dt)).astype(np.int64)
    return np.clip(k, k_min, k_max).astype(np.int32)


def level_time(L: int) -> float:
    """Block time at which level L and all deeper levels are active: 5/8 + 2^-L."""
    return 5.0 * 2.0 ** -3 + 2.0 ** -L


def level_t0(levels: np.ndarray, t: float) -> np.ndarray:
    """Start of each body's current step at block time t: for dt = 2^-k,
    t0 = (ceil(t/dt) - 1) * dt (all exact dyadics)."""
    dt = np.ldexp(1.0, -levels.astype(np.int64))
    return (np.ceil(t / dt) - 1.0) * dt


def level_block(levels: np.ndarray, L: int) -> np.ndarray:
    """Active block at level L: every body with step level >= L, ascending."""
    return np.nonzero(levels >= L)[0].astype(np.int32)


def level_weight(L: int, k_min: int = 3) -> int:
    """Occurrences of level L per 2^-k_min cycle of the block-step hierarchy."""
    return 1 if L == k_min else 2 ** (L - k_min - 1)


def sample_levels(rng: np.random.Generator, n: int, k_lo: int, k_hi: int, k_peak: float,
                  width: float = 1.5, deep_frac: float = 0.05) -> np.ndarray:
    """Synthetic step levels in [k_lo, k_hi]: a bulk around k_peak (rounded
    normal of the given width) plus a fraction deep_frac spread uniformly over
    the deeper levels, the shape of a cluster's step distribution with a tail of
    close pairs and binaries."""
    k = np.rint(rng.normal(k_peak, width, n))
    deep = rng.random(n) < deep_frac
    k[deep] = rng.integers(int(k_peak) + 1, k_hi + 1, int(deep.sum()))
    return np.clip(k, k_lo, k_hi).astype(np.int32)


def next_levels(rng: np.random.Generator, lev: np.ndarray, L: int, k_max: int,
                p_keep: float = 0.7) -> np.ndarray:
    """New levels for bodies of a block of level L: kept with probability
    p_keep, else one coarser or one to three finer, clamped to [L, k_max] (a new
    step must divide the block time)."""
    lev = np.asarray(lev, np.int64)
    u = rng.random(lev.size)
    d = np.where(u < p_keep, 0, np.where(u < p_keep + (1 - p_keep) / 2, -1,
                                         rng.integers(1, 4, lev.size)))
    return np.clip(lev + d, L, k_max).astype(np.int32)


# --------------------------------------------------------------------------- #
# named workloads
# --------------------------------------------------------------------------- #
def _state(x, v, m, a, jk, t0, t, rs2):
    return dict(x=x, v=v, m=m, a=np.ascontiguousarray(a), jk=np.ascontiguousarray(jk),
                t0=t0, t=float(t), rs2=rs2, n=int(m.size))


def uniform_step_state(rng, n, imf, dt_k=8, k_nn=64, henon_key: str | None = None):
    """Plummer state where every body has step 2^-dt_k, t0 = 0, t = 2^-dt_k."""
    x, v, m = plummer(rng, n, imf, henon_key)
    b = PLUMMER_B * (henon_correction(henon_key)[0] if henon_key is not None else 1.0)
    a, jk = plummer_field(x, v, b)
    rs2 = knn_rs2(x, k_nn) if n > k_nn else np.full(n, 0.0)
    t = 2.0 ** -dt_k
    return _state(x, v, m, a, jk, np.zeros(n), t, rs2)


@functools.lru_cache(maxsize=4)
def plummer_equal_n1024():
    """N = 1024 equal-mass Plummer, all active, nb_cap 256, FP64."""
    s = uniform_step_state(rng_for(1), 1024, "equal", henon_key="plummer_equal_n1024")
    s["i_block"] = np.arange(1024, dtype=np.int32)
    s["nb_cap"] = 256
    return s


@functools.lru_cache(maxsize=4)
def plummer_kroupa_n131072(n: int = 131072):
    """N = 131072 Plummer + Kroupa; random blocks of 1, 32, 1024, 16384, N."""
    rng = rng_for(2)
    s = uniform_step_state(rng, n, "kroupa",
                           henon_key="plummer_kroupa_n131072" if n == 131072 else None)
    sizes = [sz for sz in (1, 32, 1024, 16384, n) if sz <= n]
    s["blocks"] = {sz: random_block(rng, n, sz) for sz in sizes}
    s["nb_cap"] = 512
    return s


@functools.lru_cache(maxsize=2)
def binary_cluster_n1m(n: int = 1 << 20):
    """N = 2^20 Plummer + Kroupa with n/40 primordial binaries (5% of bodies in
    binaries); Hermite step levels 3..20; nb_cap 1024."""
    rng = rng_for(3)
    n_bin = n // 40
    key = "binary_cluster_n1m" if n == 1 << 20 else None
    x, v, m, period = plummer_with_binaries(rng, n, n_bin, henon_key=key)
    rs2 = knn_rs2(x, 64)
    a, jk = plummer_field(x, v, PLUMMER_B * (henon_correction(key)[0] if key else 1.0))
    ab, jb = binary_companion_field(x, v, m, n_bin)
    a += ab
    jk += jb
    lev = step_levels(x, m, rs2, period)
    s = _state(x, v, m, a, jk, np.zeros(n), 0.0, rs2)
    s["levels"] = lev
    s["n_bin"] = n_bin
    s["nb_cap"] = 1024
    return s


def binary_cluster_level(s: dict, L: int):
    """(t, t0, i_block) for block level L of a binary_cluster_n1m state; L = 3 is the full
    block only if every body sits at level >= 3, which the clamp guarantees."""
    t = level_time(L)
    return t, level_t0(s["levels"], t), level_block(s["levels"], L)


@functools.lru_cache(maxsize=2)
def cluster_ensemble_256(n_clusters: int = 256, n_lo: int = 1024, n_hi: int = 32768):
    """Ensemble of independent Plummer + Kroupa clusters, N log-uniform in
    [n_lo, n_hi], active fraction U[0.01, 1]; concatenated SoA with offsets."""
    rng = rng_for(4)
    ns = np.exp(rng.uniform(math.log(n_lo), math.log(n_hi), n_clusters)).round().astype(np.int64)
    fr = rng.uniform(0.01, 1.0, n_clusters)
    xs, vs, ms, as_, js, rss, blocks = [], [], [], [], [], [], []
    j_off = [0]
    i_off = [0]
    for c in range(n_clusters):
        rc = rng_for(4, c)
        nc = int(ns[c])
        key = f"cluster_ensemble_256/{c}" if (n_clusters, n_lo, n_hi) == (256, 1024, 32768) else None
        st = uniform_step_state(rc, nc, "kroupa", henon_key=key)
        ni = max(1, int(round(fr[c] * nc)))
        blk = random_block(rc, nc, ni) + j_off[-1]
        xs.append(st["x"]); vs.append(st["v"]); ms.append(st["m"])
        as_.append(st["a"]); js.append(st["jk"]); rss.append(st["rs2"][blk - j_off[-1]])
        blocks.append(blk)
        j_off.append(j_off[-1] + nc)
        i_off.append(i_off[-1] + ni)
    x = np.ascontiguousarray(np.concatenate(xs, axis=1))
    v = np.ascontiguousarray(np.concatenate(vs, axis=1))
    a = np.ascontiguousarray(np.concatenate(as_, axis=1))
    jk = np.ascontiguousarray(np.concatenate(js, axis=1))
    m = np.concatenate(ms)
    n = m.size
    return dict(x=x, v=v, m=m, a=a, jk=jk, t0=np.zeros(n), t=2.0 ** -8, n=n,
                j_off=np.array(j_off, np.int64), i_off=np.array(i_off, np.int64),
                i_block=np.concatenate(blocks).astype(np.int32),
                rs2=np.concatenate(rss), nb_cap=256, sizes=ns, fractions=fr)


@functools.lru_cache(maxsize=2)
def adjoint_plummer_n65536(n: int = 65536):
    """N = 65536 Plummer + Kroupa, all active; random upstream weights."""
    rng = rng_for(5)
    s = uniform_step_state(rng, n, "kroupa",
                           henon_key="adjoint_plummer_n65536" if n == 65536 else None)
    s["i_block"] = np.arange(n, dtype=np.int32)
    s["w_a"] = rng.standard_normal((3, n))
    s["w_j"] = rng.standard_normal((3, n))
    s["nb_cap"] = 512
    return s


def small_state(seed: int, n: int, imf: str = "kroupa", k_nn: int = 16, dt_k: int = 8):
    """Small Plummer state for parity tests (seeded, ragged sizes welcome)."""
    rng = np.random.Generator(np.random.PCG64(SEED_BASE + 100 + seed))
    s = uniform_step_state(rng, n, imf, dt_k=dt_k, k_nn=min(k_nn, max(n - 1, 1)))
    s["rng"] = rng
    return s
