// Device building blocks of the regular-force kernels (gfx950): the
// row-per-lane tile pass and the per-row merge of split partials.  Shared by
// the single-block launch (nb_force.hip) and the batched ensemble
// (nb_batched.hip).
//
// Slot layout of split partials (both launch kinds): a (row, split) pair owns
// one slot, and a row's slots are consecutive (slot = row's first slot +
// split).  part[slot * kSlotComp + k] holds component k of its FP64 sums
// (acc x,y,z, jerk x,y,z, then the mixed plan's two error-scale sums: one
// 64-byte record per slot), seg_cnt[slot] its neighbour count and
// seg_list[slot * kSegCap ...] the first kSegCap neighbours in ascending j.
// The force kernels write whole records; the merge reads a row's records as
// one contiguous run.
#pragma once

#include "nb_internal.h"
#include "nb_pair.h"

namespace nb {

struct alignas(16) JBody {
    double x, y, z, m;
    double vx, vy, vz;
    float m32;
    int32_t pad;
};

template <bool MIXED>
struct Row {
    double x, y, z, vx, vy, vz;
    double hi;      // FP64 candidate bound (FP64 plan)
    float rs2f;     // canonical radius
    float candf;    // FP32 candidate bound (mixed plan)
    int32_t i;      // body index, -1 when the lane has no row
    int32_t jend;   // end of the j-range: staged bodies at or past it are padding
    int32_t cnt;    // neighbours found so far (true count)
    int32_t *lst;   // where this row's neighbours go
    int32_t lcap;   // capacity of lst
    Sums<MIXED> S;
};

// Where the rows of one pass write: straight to the caller's outputs, or to
// the slots of one split (slot of row b = slot_base + (b - row_origin) *
// slot_stride, where slot_stride is the split count).
struct Dest {
    bool direct;
    int64_t slot_base;
    int64_t row_origin;
    int64_t slot_stride;
};

__device__ __forceinline__ int64_t dest_slot(const Dest &d, int64_t b)
{
    return d.slot_base + (b - d.row_origin) * d.slot_stride;
}

// The 64-byte partial-sum record of one slot.
__device__ __forceinline__ double2 *slot_rec(const ForceArgs &a, int64_t slot)
{
    return reinterpret_cast<double2 *>(a.part + slot * kSlotComp);
}

template <bool MIXED>
__device__ __forceinline__ void row_init(Row<MIXED> &R, const ForceArgs &a, int64_t b,
                                         int64_t row_end, const Dest &d, float near)
{
    R.S.zero();
    R.cnt = 0;
    R.i = -1;
    R.x = R.y = R.z = kFar * 0.5;   // inert placeholder
    R.vx = R.vy = R.vz = 0.0;
    R.rs2f = -1.0f;
    R.hi = -1.0;
    R.candf = -1.0f;
    R.lst = nullptr;
    R.lcap = 0;
    R.jend = 0;
    if (b >= row_end) return;
    const int64_t i = a.i_block[b];
    if (i < 0 || i >= a.n) return;   // bad index: handled in the epilogue / merge
    R.i = (int32_t)i;
    R.x = a.xp[i];
    R.y = a.xp[a.n + i];
    R.z = a.xp[2 * a.n + i];
    R.vx = a.vp[i];
    R.vy = a.vp[a.n + i];
    R.vz = a.vp[2 * a.n + i];
    R.rs2f = (float)a.rs2[b];
    R.hi = cand_bound_f64(R.rs2f);
    R.candf = cand_bound_f32(R.rs2f, near);
    if (d.direct) {
        R.lst = a.nb_list + b * (int64_t)a.cap;
        R.lcap = a.cap;
    } else {
        R.lst = a.seg_list + dest_slot(d, b) * kSegCap;
        R.lcap = kSegCap;
    }
}

// Row-per-lane mapping: each lane appends to its own row's list (in j order).
// Rare branch of a mixed pair (neighbour, self or near pair): appends a
// neighbour, or adds a near pair's term in FP64.
template <bool MIXED>
__device__ __forceinline__ void rare_mixed(Row<MIXED> &R, const JBody &J, int32_t jidx, float r2f,
                                           double dx, double dy, double dz)
{
    double ex = dx, ey = dy, ez = dz;
    int32_t jj = jidx;
    opaque(ex, ey, ez);
    opaque(jj);
    // padding past the j-range (far away, mass 0) passes the test only for a
    // huge or infinite radius; it is never a neighbour and adds nothing
    if (jj >= R.jend) return;
    const bool self = jj == R.i;
    const bool nbr = (r2f < R.rs2f) && !self;
    if (nbr) {
        if (R.cnt < R.lcap) R.lst[R.cnt] = jidx;
        ++R.cnt;
    } else if (!self) {
        add_term_f64(R.S.ax, R.S.ay, R.S.az, R.S.jx, R.S.jy, R.S.jz, ex, ey, ez,
                     J.vx - R.vx, J.vy - R.vy, J.vz - R.vz, J.m);
    }
}

// Exact canonical test of an FP64 candidate pair; appends a neighbour.
// Returns true if the pair is excluded (neighbour or self).
template <bool MIXED>
__device__ __forceinline__ bool rare_f64(Row<MIXED> &R, int32_t jidx, double dx, double dy,
                                         double dz)
{
    double ex = dx, ey = dy, ez = dz;
    int32_t jj = jidx;
    opaque(ex, ey, ez);
    opaque(jj);
    if (jj >= R.jend) return false;   // padding: mass 0, its term is exactly zero
    const bool self = jj == R.i;
    const bool nbr = (canon_r2f(ex, ey, ez) < R.rs2f) && !self;
    if (nbr) {
        if (R.cnt < R.lcap) R.lst[R.cnt] = jidx;
        ++R.cnt;
    }
    return nbr || self;
}

// One row against two consecutive j, with a single branch for the rare cases
// (one exec-mask change per two j).  Mixed: FP64 differences, canonical FP32
// r2f (the neighbour test itself), FP32 terms; pairs with r2f below the
// near bound (neighbours, self, near pairs) take the rare branch.  FP64: FP64
// r2 against the candidate bound, the exact canonical test only for
// candidates.  Every accumulator receives the terms of j and then j+1, as a
// loop over single j would give them.
template <bool MIXED>
__device__ __forceinline__ void pair_rows2(Row<MIXED> &R, const JBody &J0, const JBody &J1,
                                           int32_t jidx0)
{
    if constexpr (MIXED) {
        const double dx0 = J0.x - R.x, dy0 = J0.y - R.y, dz0 = J0.z - R.z;
        const double dx1 = J1.x - R.x, dy1 = J1.y - R.y, dz1 = J1.z - R.z;
        const float fx0 = (float)dx0, fy0 = (float)dy0, fz0 = (float)dz0;
        const float fx1 = (float)dx1, fy1 = (float)dy1, fz1 = (float)dz1;
        const float r0 = __builtin_fmaf(fz0, fz0, __builtin_fmaf(fy0, fy0, fx0 * fx0));
        const float r1 = __builtin_fmaf(fz1, fz1, __builtin_fmaf(fy1, fy1, fx1 * fx1));
        const bool c0 = r0 < R.candf, c1 = r1 < R.candf;
        // the FP32 terms first, the rare cases after them: every LDS read of
        // the two bodies can then be issued before the first arithmetic (the
        // rare cases touch only the FP64 sums and the list, so the order of
        // the two changes no result)
        accum_mixed(R.S, fx0, fy0, fz0, r0, J0.vx - R.vx, J0.vy - R.vy, J0.vz - R.vz, J0.m32, c0);
        accum_mixed(R.S, fx1, fy1, fz1, r1, J1.vx - R.vx, J1.vy - R.vy, J1.vz - R.vz, J1.m32, c1);
        if (c0 || c1) {
            if (c0) rare_mixed<MIXED>(R, J0, jidx0, r0, dx0, dy0, dz0);
            if (c1) rare_mixed<MIXED>(R, J1, jidx0 + 1, r1, dx1, dy1, dz1);
        }
    } else {
        const double dx0 = J0.x - R.x, dy0 = J0.y - R.y, dz0 = J0.z - R.z;
        const double dx1 = J1.x - R.x, dy1 = J1.y - R.y, dz1 = J1.z - R.z;
        const double r0 = __builtin_fma(dz0, dz0, __builtin_fma(dy0, dy0, dx0 * dx0));
        const double r1 = __builtin_fma(dz1, dz1, __builtin_fma(dy1, dy1, dx1 * dx1));
        const bool c0 = r0 < R.hi, c1 = r1 < R.hi;
        bool e0 = false, e1 = false;
        if (c0 || c1) {
            if (c0) e0 = rare_f64<MIXED>(R, jidx0, dx0, dy0, dz0);
            if (c1) e1 = rare_f64<MIXED>(R, jidx0 + 1, dx1, dy1, dz1);
        }
        accum_f64(R.S, dx0, dy0, dz0, r0, J0.vx - R.vx, J0.vy - R.vy, J0.vz - R.vz, J0.m, e0);
        accum_f64(R.S, dx1, dy1, dz1, r1, J1.vx - R.vx, J1.vy - R.vy, J1.vz - R.vz, J1.m, e1);
    }
}

__device__ __forceinline__ void load_body(JBody &J, const ForceArgs &a, int64_t j, int64_t j1)
{
    if (j < j1) {
        J.x = a.xp[j];
        J.y = a.xp[a.n + j];
        J.z = a.xp[2 * a.n + j];
        J.vx = a.vp[j];
        J.vy = a.vp[a.n + j];
        J.vz = a.vp[2 * a.n + j];
        J.m = a.m[j];
    } else {
        J.x = J.y = J.z = kFar;
        J.vx = J.vy = J.vz = 0.0;
        J.m = 0.0;
    }
    J.m32 = (float)J.m;
    J.pad = 0;
}

// Appends row b (with its j-range) to the FP64 redo list.
__device__ __forceinline__ void redo_push(const ForceArgs &a, int64_t b, int64_t j0, int64_t j1)
{
    const int32_t q = atomicAdd(a.redo_count, 1);
    a.redo_rows[q] = (int32_t)b;
    a.redo_j0[q] = (int32_t)j0;
    a.redo_j1[q] = (int32_t)j1;
}

// One row's final sums and count: to the outputs, or to its split slot.
// [j0, j1) is the row's whole j-range when the destination is direct.
template <bool MIXED>
__device__ __forceinline__ void row_store(const ForceArgs &a, int64_t b, const Dest &d,
                                          bool valid, const Sums<MIXED> &S, int32_t cnt,
                                          bool &ovf, bool &bad, bool &nonfin, int64_t j0,
                                          int64_t j1)
{
    if (d.direct) {
        if (!valid) {
            a.acc[b] = a.acc[a.n_i + b] = a.acc[2 * (int64_t)a.n_i + b] = 0.0;
            a.jerk[b] = a.jerk[a.n_i + b] = a.jerk[2 * (int64_t)a.n_i + b] = 0.0;
            a.nb_count[b] = 0;
            bad = true;
            return;
        }
        a.acc[b] = S.ax;
        a.acc[a.n_i + b] = S.ay;
        a.acc[2 * (int64_t)a.n_i + b] = S.az;
        a.jerk[b] = S.jx;
        a.jerk[a.n_i + b] = S.jy;
        a.jerk[2 * (int64_t)a.n_i + b] = S.jz;
        a.nb_count[b] = cnt;
        ovf = cnt > a.cap;
        nonfin = !finite6(S.ax, S.ay, S.az, S.jx, S.jy, S.jz);
        if (MIXED && a.redo_k > 0.0 &&
            needs_redo(a.redo_k, S.ax, S.ay, S.az, S.jx, S.jy, S.jz, S.va, S.vj))
            redo_push(a, b, j0, j1);
    } else {
        const int64_t slot = dest_slot(d, b);
        double2 *p = slot_rec(a, slot);
        p[0] = make_double2(S.ax, S.ay);
        p[1] = make_double2(S.az, S.jx);
        p[2] = make_double2(S.jy, S.jz);
        p[3] = make_double2(S.va, S.vj);
        a.seg_cnt[slot] = cnt;
    }
}

__device__ __forceinline__ void flush_flags(const ForceArgs &a, bool ovf, bool bad, bool nonfin)
{
    // called in uniform control flow by every lane of the wave
    const uint64_t o = __ballot(ovf), b = __ballot(bad), f = __ballot(nonfin);
    if ((threadIdx.x & (kWave - 1)) == 0 && (o | b | f)) {
        const uint32_t st =
            (o ? kStOverflow : 0u) | (b ? kStBadIndex : 0u) | (f ? kStNonFinite : 0u);
        if (o) atomicOr(a.overflow, 1);
        if (a.status) atomicOr(a.status, st);
    }
}

// Rows [row0 + r*NB + tid] (r < IR, < row_end) of one work-group of NB
// lanes against bodies [j0, j1), staged through a double-buffered LDS tile
// of T bodies.  With T == NB every lane loads one body of the next tile
// into registers while the current tile is computed (one barrier per tile);
// otherwise each lane loads its T/NB bodies (or one, for T < NB) straight
// into the free buffer when the work-group reaches the tile, so no registers
// are held across the pair loop.  The j order, the FP32 fold points (every
// kFold bodies from j0) and all sums are the same for every T and NB, so
// results do not depend on the tile or work-group shape.  Must be called by
// the whole work-group (it contains barriers).
template <bool MIXED, int IR, int T, int NB>
__device__ __forceinline__ void rows_pass(const ForceArgs &a, JBody (*tile)[T], int64_t row0,
                                          int64_t row_end, int64_t j0, int64_t j1,
                                          const Dest &d, float near)
{
    static_assert(T % kFold == 0 && NB % kWave == 0, "tile and work-group shape");
    constexpr bool kPrefetch = T == NB;
    const int tid = threadIdx.x;
    Row<MIXED> R[IR];
#pragma unroll
    for (int r = 0; r < IR; ++r) {
        row_init(R[r], a, row0 + r * NB + tid, row_end, d, near);
        R[r].jend = (int32_t)j1;
    }

    // a wave none of whose lanes holds a valid row (the tail of a cluster's
    // last row tile) skips the pair loop; it still stages its share of every
    // tile and meets every barrier
    bool mine = false;
#pragma unroll
    for (int r = 0; r < IR; ++r) mine = mine || R[r].i >= 0;
    const bool wave_busy = __ballot(mine) != 0;

    const int64_t ntiles = j1 > j0 ? (j1 - j0 + T - 1) / T : 0;
    JBody nxt;
    if constexpr (kPrefetch) {
        if (ntiles > 0) {
            load_body(nxt, a, j0 + tid, j1);
            tile[0][tid] = nxt;
        }
        __syncthreads();
    }
    for (int64_t t = 0; t < ntiles; ++t) {
        const int cur = (int)(t & 1);
        const int64_t tbase = j0 + t * T;
        if constexpr (kPrefetch) {
            if (t + 1 < ntiles) load_body(nxt, a, tbase + T + tid, j1);
        } else {
            // buffer cur was last read for tile t-2, and every wave has
            // passed the barrier of tile t-1 since
            for (int k = tid; k < T; k += NB) {
                JBody J;
                load_body(J, a, tbase + k, j1);
                tile[cur][k] = J;
            }
            __syncthreads();
        }
        const JBody *buf = tile[cur];
        for (int jj = 0; jj < (wave_busy ? T : 0); jj += kFold) {
            for (int q = 0; q < kFold; q += 2) {
                const int32_t jidx = (int32_t)(tbase + jj + q);
#pragma unroll
                for (int r = 0; r < IR; ++r)
                    pair_rows2<MIXED>(R[r], buf[jj + q], buf[jj + q + 1], jidx);
            }
            if constexpr (MIXED) {
#pragma unroll
                for (int r = 0; r < IR; ++r) R[r].S.fold();
            } else if (((t * T + jj + kFold) & (kFoldF64 - 1)) == 0) {
#pragma unroll
                for (int r = 0; r < IR; ++r) R[r].S.fold();
            }
        }
        if constexpr (kPrefetch) {
            if (t + 1 < ntiles) tile[cur ^ 1][tid] = nxt;
            __syncthreads();
        }
    }
    if constexpr (!kPrefetch) __syncthreads();   // the tile may be reused by the caller

    bool ovf = false, bad = false, nonfin = false;
#pragma unroll
    for (int r = 0; r < IR; ++r) {
        if constexpr (!MIXED) R[r].S.fold();
        const int64_t b = row0 + r * NB + tid;
        if (b < row_end) {
            bool o = false, bd = false, f = false;
            row_store<MIXED>(a, b, d, R[r].i >= 0, R[r].S, R[r].cnt, o, bd, f, j0, j1);
            ovf |= o;
            bad |= bd;
            nonfin |= f;
        }
    }
    flush_flags(a, ovf, bad, nonfin);
}

// Geometry of one row's splits for the merge.
struct MergeGeom {
    int32_t splits;
    int64_t slot0;        // slot of split 0
    int64_t slot_step;    // slot(s) = slot0 + s * slot_step
    int64_t j_begin, j_end, split_len;
};

// Sums of K values over the W aligned lanes of a lane group (butterfly,
// largest offset first; every lane of the group gets the results).  The
// butterflies run level by level across the K values, so the K shuffles of a
// level are issued together and a level waits on one cross-lane permute
// latency instead of K (value after value, eight values took about 2 us).
// Each value gets the pairs and order of its own butterfly.
template <int W, int K>
__device__ __forceinline__ void group_sums(double (&v)[K])
{
#pragma unroll
    for (int o = W / 2; o > 0; o >>= 1) {
        double t[K];
#pragma unroll
        for (int k = 0; k < K; ++k) t[k] = __shfl_xor(v[k], o, kWave);
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] += t[k];
    }
}

// A word written by an earlier launch (a counter), read at a uniform address
// through the scalar cache: many work-groups reading one word this way do
// not queue on one memory channel, as uncached vector loads of it do.
__device__ __forceinline__ int32_t load_word_uniform(const int32_t *p)
{
    return *(const __attribute__((address_space(4))) int32_t *)p;
}

// The same for a double that no lane writes during the kernel (an input, or
// data of an earlier kernel): it lands in scalar registers.
__device__ __forceinline__ double load_f64_uniform(const double *p)
{
    return *(const __attribute__((address_space(4))) double *)p;
}

// Lanes per row of the single-wave merge for a given split count: the next of
// 4, 16, 64 at or above it.  For S <= W each lane holds at most one partial
// and the lanes past S hold exact zeros, which the butterfly adds before any
// two partials meet, so every W >= S gives the same bits (and the same as one
// whole wave per row).
__host__ __device__ constexpr int merge_width(int64_t splits)
{
    return splits <= 4 ? 4 : (splits <= 16 ? 16 : 64);
}

// Merge of one row by a group of W lanes (W = 64: one whole wave; smaller W:
// 64/W rows per wave): sums the split partials in a fixed order, concatenates
// neighbour segments in split order (ascending j), writes the true count, and
// rebuilds any segment that overflowed its scratch capacity by re-running the
// canonical test over that split's j-range.  has_row = false for a group past
// the last row; every lane of the wave must call this (it ends in a ballot).
template <int W>
__device__ __forceinline__ void merge_row(const ForceArgs &a, int64_t b, bool has_row,
                                          const MergeGeom &g)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int l = lane & (W - 1);       // lane within the row's group
    const int gbase = lane - l;         // first lane of the group
    const uint64_t gmask = W == kWave ? ~0ull : (((1ull << W) - 1) << gbase);
    const int64_t i = has_row ? a.i_block[b] : -1;
    const bool bad = has_row && (i < 0 || i >= a.n);
    const int32_t S = has_row ? g.splits : 0;

    double v[kSlotComp] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int32_t s = l; s < S; s += W) {
        const double2 *p = slot_rec(a, g.slot0 + (int64_t)s * g.slot_step);
#pragma unroll
        for (int k = 0; k < kSlotComp / 2; ++k) {
            const double2 t = p[k];
            v[2 * k] += t.x;
            v[2 * k + 1] += t.y;
        }
    }
    group_sums<W, kSlotComp>(v);

    bool ovf = false, nonfin = false;
    if (bad) {
        if (l == 0) {
            for (int k = 0; k < 3; ++k) {
                a.acc[(int64_t)k * a.n_i + b] = 0.0;
                a.jerk[(int64_t)k * a.n_i + b] = 0.0;
            }
            a.nb_count[b] = 0;
        }
    } else if (has_row) {
        const double xi = a.xp[i], yi = a.xp[a.n + i], zi = a.xp[2 * a.n + i];
        const float rs2f = (float)a.rs2[b];
        int64_t off = 0;   // uniform in the group: neighbours placed so far (true count)
        for (int32_t s0 = 0; s0 < S; s0 += W) {
            const int32_t s = s0 + l;
            const int64_t slot = g.slot0 + (int64_t)s * g.slot_step;
            const int32_t c = s < S ? a.seg_cnt[slot] : 0;
            int64_t inc = c;   // inclusive scan of c over the group
#pragma unroll
            for (int o = 1; o < W; o <<= 1) {
                const int64_t t = __shfl_up(inc, o, W);
                if (l >= o) inc += t;
            }
            const int64_t start = off + inc - c;
            const bool room = c > 0 && start < a.cap;
            const bool rebuild = room && c > kSegCap;
            // segments that fit.  Short ones (at most kLaneCopy entries, the
            // usual case with many splits): each lane copies its own in
            // 16-byte loads (a segment's storage holds kSegCap entries, a
            // multiple of 8, so the loads stay inside it), all segments of the
            // group in flight together.  Longer ones: the whole group copies
            // each in turn (coalesced).
            static_assert(kSegCap % 8 == 0, "segment storage in 8-entry rounds");
            constexpr int64_t kLaneCopy = 16;
            const int64_t take = room ? ((int64_t)c < a.cap - start ? c : a.cap - start) : 0;
            if (room && !rebuild && take <= kLaneCopy) {
                const int4 *src = reinterpret_cast<const int4 *>(a.seg_list + slot * kSegCap);
                int32_t *dst = a.nb_list + b * (int64_t)a.cap + start;
                for (int64_t e = 0; e < take; e += 8) {
                    const int4 u0 = src[e / 4], u1 = src[e / 4 + 1];
                    const int32_t t[8] = {u0.x, u0.y, u0.z, u0.w, u1.x, u1.y, u1.z, u1.w};
#pragma unroll
                    for (int k = 0; k < 8; ++k)
                        if (e + k < take) dst[e + k] = t[k];
                }
            }
            uint64_t cp = __ballot(room && !rebuild && take > kLaneCopy) & gmask;
            while (cp) {
                const int q = __builtin_ctzll(cp);
                cp &= cp - 1;
                const int64_t sl = __shfl(slot, q, kWave);
                const int64_t st = __shfl(start, q, kWave);
                const int64_t tk = __shfl(take, q, kWave);
                const int32_t *src = a.seg_list + sl * kSegCap;
                int32_t *dst = a.nb_list + b * (int64_t)a.cap + st;
                for (int64_t e = l; e < tk; e += W) dst[e] = src[e];
            }
            uint64_t rb = __ballot(rebuild) & gmask;
            while (rb) {   // overflowed segments: the group rescans them one by one
                const int q = __builtin_ctzll(rb);
                rb &= rb - 1;
                const int32_t sq = __shfl(s, q, kWave);
                const int64_t st = __shfl(start, q, kWave);
                const int64_t lim = a.cap - st;
                const int64_t jb = g.j_begin + (int64_t)sq * g.split_len;
                const int64_t je = jb + g.split_len < g.j_end ? jb + g.split_len : g.j_end;
                int64_t placed = 0;
                for (int64_t base = jb; base < je && placed < lim; base += W) {
                    const int64_t j = base + l;
                    bool nbr = false;
                    if (j < je && j != i) {
                        const double dx = a.xp[j] - xi, dy = a.xp[a.n + j] - yi,
                                     dz = a.xp[2 * a.n + j] - zi;
                        nbr = canon_r2f(dx, dy, dz) < rs2f;
                    }
                    const uint64_t nm = __ballot(nbr) & gmask;
                    if (nbr) {
                        const int64_t p = placed + lanes_below(nm);
                        if (p < lim) a.nb_list[b * (int64_t)a.cap + st + p] = (int32_t)j;
                    }
                    placed += __popcll(nm);
                }
            }
            off += __shfl(inc, gbase + W - 1, kWave);
        }
        if (l == 0) {
            a.acc[b] = v[0];
            a.acc[a.n_i + b] = v[1];
            a.acc[2 * (int64_t)a.n_i + b] = v[2];
            a.jerk[b] = v[3];
            a.jerk[a.n_i + b] = v[4];
            a.jerk[2 * (int64_t)a.n_i + b] = v[5];
            a.nb_count[b] = (int32_t)off;
            ovf = off > a.cap;
            nonfin = !finite6(v[0], v[1], v[2], v[3], v[4], v[5]);
            if (a.redo_k > 0.0 && needs_redo(a.redo_k, v[0], v[1], v[2], v[3], v[4], v[5], v[6], v[7]))
                redo_push(a, b, g.j_begin, g.j_end);
        }
    }
    flush_flags(a, ovf, bad && l == 0, nonfin);
}

// Fixed-order sums of K values over the 256 lanes of a work-group (all lanes
// must call it): each value is summed over its wave by a butterfly, then the
// four wave sums are added in wave order; every lane gets the results.
template <int K>
__device__ __forceinline__ void block_sums(double (&v)[K], double (*lds)[kBlock / kWave])
{
    group_sums<kWave, K>(v);
    const int w = threadIdx.x / kWave;
    __syncthreads();   // earlier readers of lds are done
    if ((threadIdx.x & (kWave - 1)) == 0)
#pragma unroll
        for (int k = 0; k < K; ++k) lds[k][w] = v[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double t = 0.0;
#pragma unroll
        for (int q = 0; q < kBlock / kWave; ++q) t += lds[k][q];
        v[k] = t;
    }
}

// Chunks of refined row q: its j-range cut into kRedoChunk bodies.
__device__ __forceinline__ int32_t redo_row_chunks(const ForceArgs &a, int32_t q)
{
    const int64_t len = (int64_t)a.redo_j1[q] - a.redo_j0[q];
    return len > 0 ? (int32_t)((len + kRedoChunk - 1) / kRedoChunk) : 0;
}

// FP64 sums over chunk c [j0 + c*kRedoChunk, ...) of refined row q, by a whole
// work-group in a fixed pattern; every lane gets the six sums (acc, jerk).
// The chunk must lie inside the row's j-range (c < redo_row_chunks).
__device__ __forceinline__ void redo_chunk(const ForceArgs &a, int32_t q, int32_t c,
                                          double (*lds)[kBlock / kWave], double (&out)[6])
{
    // q is uniform: the row's data go to scalar registers
    const int64_t b = load_word_uniform(a.redo_rows + q);
    const int64_t j0 = load_word_uniform(a.redo_j0 + q), j1 = load_word_uniform(a.redo_j1 + q);
    const int64_t cj0 = j0 + (int64_t)c * kRedoChunk;
    const int64_t cj1 = cj0 + kRedoChunk < j1 ? cj0 + kRedoChunk : j1;
    const int64_t i = load_word_uniform(a.i_block + b);
    const double xi = load_f64_uniform(a.xp + i), yi = load_f64_uniform(a.xp + a.n + i),
                 zi = load_f64_uniform(a.xp + 2 * a.n + i);
    const double vxi = load_f64_uniform(a.vp + i), vyi = load_f64_uniform(a.vp + a.n + i),
                 vzi = load_f64_uniform(a.vp + 2 * a.n + i);
    const float rs2f = (float)load_f64_uniform(a.rs2 + b);
    const double hi = cand_bound_f64(rs2f);
    Sums<false> S;
    S.zero();
    for (int64_t j = cj0 + threadIdx.x; j < cj1; j += kBlock) {
        JBody J;
        load_body(J, a, j, cj1);
        const double dx = J.x - xi, dy = J.y - yi, dz = J.z - zi;
        const double r2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
        bool excl = false;
        if (r2 < hi) {
            double ex = dx, ey = dy, ez = dz;
            opaque(ex, ey, ez);
            excl = j == i || canon_r2f(ex, ey, ez) < rs2f;
        }
        accum_f64(S, dx, dy, dz, r2, J.vx - vxi, J.vy - vyi, J.vz - vzi, J.m, excl);
    }
    S.fold();
    out[0] = S.ax;
    out[1] = S.ay;
    out[2] = S.az;
    out[3] = S.jx;
    out[4] = S.jy;
    out[5] = S.jz;
    block_sums<6>(out, lds);
}

// Refined rows sharing one j-range are summed kRedoRows at a time: each lane
// loads a body once for all of them.  Per row the lane order and the
// reduction are those of redo_chunk, so every row gets the same bits.
constexpr int kRedoRows = 2;

// Chunk c of refined rows q0 .. q0+nr-1 (nr <= kRedoRows), which all have
// the j-range of row q0 and c < its chunk count; out[r][k] for row q0 + r.
__device__ __forceinline__ void redo_chunk_rows(const ForceArgs &a, int32_t q0, int nr, int32_t c,
                                               double (*lds)[kBlock / kWave],
                                               double (&out)[kRedoRows * 6])
{
    const int64_t j0 = load_word_uniform(a.redo_j0 + q0), j1 = load_word_uniform(a.redo_j1 + q0);
    const int64_t cj0 = j0 + (int64_t)c * kRedoChunk;
    const int64_t cj1 = cj0 + kRedoChunk < j1 ? cj0 + kRedoChunk : j1;
    double xi[kRedoRows], yi[kRedoRows], zi[kRedoRows], vxi[kRedoRows], vyi[kRedoRows],
        vzi[kRedoRows], hi[kRedoRows];
    float rs2f[kRedoRows];
    int64_t ii[kRedoRows];
    Sums<false> S[kRedoRows];
#pragma unroll
    for (int r = 0; r < kRedoRows; ++r) {
        S[r].zero();
        const int32_t q = q0 + (r < nr ? r : 0);   // uniform: scalar registers
        const int64_t b = load_word_uniform(a.redo_rows + q);
        const int64_t i = load_word_uniform(a.i_block + b);
        ii[r] = i;
        xi[r] = load_f64_uniform(a.xp + i);
        yi[r] = load_f64_uniform(a.xp + a.n + i);
        zi[r] = load_f64_uniform(a.xp + 2 * a.n + i);
        vxi[r] = load_f64_uniform(a.vp + i);
        vyi[r] = load_f64_uniform(a.vp + a.n + i);
        vzi[r] = load_f64_uniform(a.vp + 2 * a.n + i);
        rs2f[r] = (float)load_f64_uniform(a.rs2 + b);
        hi[r] = cand_bound_f64(rs2f[r]);
    }
    for (int64_t j = cj0 + threadIdx.x; j < cj1; j += kBlock) {
        JBody J;
        load_body(J, a, j, cj1);
#pragma unroll
        for (int r = 0; r < kRedoRows; ++r) {
            if (r >= nr) break;
            const double dx = J.x - xi[r], dy = J.y - yi[r], dz = J.z - zi[r];
            const double r2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
            bool excl = false;
            if (r2 < hi[r]) {
                double ex = dx, ey = dy, ez = dz;
                opaque(ex, ey, ez);
                excl = j == ii[r] || canon_r2f(ex, ey, ez) < rs2f[r];
            }
            accum_f64(S[r], dx, dy, dz, r2, J.vx - vxi[r], J.vy - vyi[r], J.vz - vzi[r], J.m,
                      excl);
        }
    }
#pragma unroll
    for (int r = 0; r < kRedoRows; ++r) {
        S[r].fold();
        out[r * 6 + 0] = S[r].ax;
        out[r * 6 + 1] = S[r].ay;
        out[r * 6 + 2] = S[r].az;
        out[r * 6 + 3] = S[r].jx;
        out[r * 6 + 4] = S[r].jy;
        out[r * 6 + 5] = S[r].jz;
    }
    block_sums<kRedoRows * 6>(out, lds);
}

constexpr int kMergeBatch = 8;    // strides of split partials loaded per batch
constexpr int kCountBatch = 8;    // segment counts loaded per batch

// Copies entries [from, take) of the neighbour segment of split s (count c)
// to dst: from its slot, or, for an overflowed segment, by rescanning the
// split's j-range in order.
__device__ __forceinline__ void copy_segment(const ForceArgs &a, const MergeGeom &g, int64_t b,
                                             int64_t i, int32_t s, int32_t c, int64_t from,
                                             int64_t take, int32_t *dst)
{
    const int64_t slot = g.slot0 + (int64_t)s * g.slot_step;
    if (c <= kSegCap) {
        const int32_t *src = a.seg_list + slot * kSegCap;
        for (int64_t q = from; q < take; ++q) dst[q] = src[q];
        return;
    }
    const double xi = a.xp[i], yi = a.xp[a.n + i], zi = a.xp[2 * a.n + i];
    const float rs2f = (float)a.rs2[b];
    const int64_t jb = g.j_begin + (int64_t)s * g.split_len;
    const int64_t je = jb + g.split_len < g.j_end ? jb + g.split_len : g.j_end;
    int64_t placed = 0;
    for (int64_t j = jb; j < je && placed < take; ++j) {
        if (j == i) continue;
        const double dx = a.xp[j] - xi, dy = a.xp[a.n + j] - yi, dz = a.xp[2 * a.n + j] - zi;
        if (canon_r2f(dx, dy, dz) < rs2f) {
            if (placed >= from) dst[placed] = (int32_t)j;
            ++placed;
        }
    }
}

// Partial records of splits sb + u * kBlock (u < kMergeBatch) of one row;
// past the last split, split 0's record is loaded (and not added).
__device__ __forceinline__ void merge_load_batch(const ForceArgs &a, const MergeGeom &g,
                                                 int32_t sb, double (&t)[kMergeBatch][kSlotComp])
{
#pragma unroll
    for (int u = 0; u < kMergeBatch; ++u) {
        const int32_t s = sb + u * kBlock;
        const double2 *p = slot_rec(a, g.slot0 + (int64_t)(s < g.splits ? s : 0) * g.slot_step);
#pragma unroll
        for (int k = 0; k < kSlotComp / 2; ++k) {
            const double2 q = p[k];
            t[u][2 * k] = q.x;
            t[u][2 * k + 1] = q.y;
        }
    }
}

__device__ __forceinline__ void merge_add_batch(int32_t S, int32_t sb,
                                                const double (&t)[kMergeBatch][kSlotComp],
                                                double (&v)[kSlotComp])
{
#pragma unroll
    for (int u = 0; u < kMergeBatch; ++u)
        if (sb + u * kBlock < S) {
#pragma unroll
            for (int k = 0; k < kSlotComp; ++k) v[k] += t[u][k];
        }
}

// Merge of one row by a whole work-group, for plans with many splits.  The
// sums stride the splits over the lanes (fixed order: a lane adds its splits
// in increasing order, then the wave butterfly, then the four wave sums in
// wave order).  For the list, lane t owns the contiguous splits [t*K,
// (t+1)*K), and a work-group prefix scan of the lanes' counts places its
// segments, so the list stays in split order.  The work is laid out for few
// memory round trips: a lane's counts are loaded with its partials, and the
// first two entries of all its segments are loaded before any is stored.
// Called once per work-group (its LDS arrays are not reused).
__device__ __forceinline__ void merge_row_wg(const ForceArgs &a, int64_t b, const MergeGeom &g,
                                             double (*lds)[kBlock / kWave], int64_t *scan)
{
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1), w = tid / kWave;
    const int64_t i = a.i_block[b];
    const bool bad = i < 0 || i >= a.n;
    const int32_t S = g.splits;
    const int32_t K = (S + kBlock - 1) / kBlock;
    const int32_t s0 = tid * K;
    const int32_t nmine = s0 < S ? (S - s0 < K ? S - s0 : K) : 0;

    // sums: the loads of kMergeBatch strides are issued before any is added,
    // so a lane waits on one memory latency per batch, not per split.  The
    // first batch is issued ahead of the lane's first kCountBatch counts (the
    // memory counter waits in issue order), so both arrive in one round trip.
    double v[kSlotComp] = {0, 0, 0, 0, 0, 0, 0, 0};
    double t[kMergeBatch][kSlotComp];
    merge_load_batch(a, g, tid, t);
    int32_t ck[kCountBatch];
#pragma unroll
    for (int u = 0; u < kCountBatch; ++u) {
        const int32_t s = s0 + u < S ? s0 + u : S - 1;   // in range; unused past nmine
        const int32_t c = a.seg_cnt[g.slot0 + (int64_t)s * g.slot_step];
        ck[u] = u < nmine ? c : 0;
    }
    merge_add_batch(S, tid, t, v);
    for (int32_t sb = tid + kBlock * kMergeBatch; sb < S; sb += kBlock * kMergeBatch) {
        merge_load_batch(a, g, sb, t);
        merge_add_batch(S, sb, t, v);
    }
    int64_t mine = 0;
#pragma unroll
    for (int u = 0; u < kCountBatch; ++u) mine += ck[u];
    for (int32_t sb = kCountBatch; sb < nmine; sb += kCountBatch) {   // K > kCountBatch
        int32_t c[kCountBatch];
#pragma unroll
        for (int u = 0; u < kCountBatch; ++u) {
            const int32_t s = sb + u < nmine ? s0 + sb + u : s0;
            c[u] = a.seg_cnt[g.slot0 + (int64_t)s * g.slot_step];
        }
#pragma unroll
        for (int u = 0; u < kCountBatch; ++u) mine += sb + u < nmine ? c[u] : 0;
    }

    // one barrier for both reductions: wave butterflies of the sums and a
    // wave scan of the counts, then the four waves' values from LDS
    group_sums<kWave, kSlotComp>(v);
    int64_t inc = mine;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const int64_t t = __shfl_up(inc, o, kWave);
        if (lane >= o) inc += t;
    }
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < kSlotComp; ++k) lds[k][w] = v[k];
    if (lane == kWave - 1) scan[w] = inc;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kSlotComp; ++k) {
        double t = 0.0;
#pragma unroll
        for (int q = 0; q < kBlock / kWave; ++q) t += lds[k][q];
        v[k] = t;
    }
    int64_t before = 0, total = 0;
#pragma unroll
    for (int q = 0; q < kBlock / kWave; ++q) {
        const int64_t t = scan[q];
        total += t;
        before += q < w ? t : 0;
    }
    const int64_t start = before + inc - mine;

    bool ovf = false, nonfin = false;
    if (!bad) {
        // the lane's segments in batches of kCountBatch: the first two
        // entries of every segment of a batch are loaded before any is stored
        int32_t *row = a.nb_list + b * (int64_t)a.cap;
        int64_t at = start;
        for (int32_t sb = 0; sb < nmine && at < a.cap; sb += kCountBatch) {
            if (sb > 0) {
#pragma unroll
                for (int u = 0; u < kCountBatch; ++u) {
                    const int32_t s = sb + u < nmine ? s0 + sb + u : s0;
                    const int32_t c = a.seg_cnt[g.slot0 + (int64_t)s * g.slot_step];
                    ck[u] = sb + u < nmine ? c : 0;
                }
            }
            int32_t e0[kCountBatch], e1[kCountBatch];
            int64_t p = at;
#pragma unroll
            for (int u = 0; u < kCountBatch; ++u) {
                const int32_t *src =
                    a.seg_list + (g.slot0 + (int64_t)(s0 + sb + u) * g.slot_step) * kSegCap;
                const bool ok = ck[u] > 0 && ck[u] <= kSegCap && p < a.cap;
                e0[u] = ok ? src[0] : 0;
                e1[u] = ok && ck[u] > 1 && p + 1 < a.cap ? src[1] : 0;
                p += ck[u];
            }
#pragma unroll
            for (int u = 0; u < kCountBatch; ++u) {
                const int32_t c = ck[u];
                if (c > 0 && at < a.cap) {
                    const int64_t take = (int64_t)c < a.cap - at ? c : a.cap - at;
                    if (c <= kSegCap) {
                        row[at] = e0[u];
                        if (take > 1) row[at + 1] = e1[u];
                        if (take > 2) copy_segment(a, g, b, i, s0 + sb + u, c, 2, take, row + at);
                    } else {
                        copy_segment(a, g, b, i, s0 + sb + u, c, 0, take, row + at);
                    }
                }
                at += c;
            }
        }
        if (tid == 0) {
            a.acc[b] = v[0];
            a.acc[a.n_i + b] = v[1];
            a.acc[2 * (int64_t)a.n_i + b] = v[2];
            a.jerk[b] = v[3];
            a.jerk[a.n_i + b] = v[4];
            a.jerk[2 * (int64_t)a.n_i + b] = v[5];
            a.nb_count[b] = (int32_t)total;
            ovf = total > a.cap;
            nonfin = !finite6(v[0], v[1], v[2], v[3], v[4], v[5]);
            if (a.redo_k > 0.0 &&
                needs_redo(a.redo_k, v[0], v[1], v[2], v[3], v[4], v[5], v[6], v[7]))
                redo_push(a, b, g.j_begin, g.j_end);
        }
    } else if (tid == 0) {
        for (int k = 0; k < 3; ++k) {
            a.acc[(int64_t)k * a.n_i + b] = 0.0;
            a.jerk[(int64_t)k * a.n_i + b] = 0.0;
        }
        a.nb_count[b] = 0;
    }
    flush_flags(a, ovf, bad && tid == 0, nonfin);
}

}  // namespace nb
