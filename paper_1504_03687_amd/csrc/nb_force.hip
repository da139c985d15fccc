// Regular force + jerk + neighbour lists of one active block on gfx950
// (Wang et al. 2015, section 2 and section 3.2.1: the GPU computes the regular
// force and its derivative and builds the neighbour lists in the same pass;
// Table 1 "Reg.").
//
// Two mappings of the O(N_i N) pair loop onto CDNA4:
//
//  * row-per-lane (large blocks): every lane owns 1, 2 or 4 rows in
//    registers; the work-group streams its j-range through LDS in tiles of
//    kTile bodies (coalesced SoA global loads, double-buffered, one barrier per
//    tile) and every lane reads each staged body by LDS broadcast.  Neighbour
//    appends are lane-private (see nb_rows.h).
//
//  * row-group-per-wave (small blocks): the 64 lanes of a wavefront take 64
//    consecutive j while 1, 2 or 4 rows sit in scalar registers; sums are
//    reduced across the wave with butterfly shuffles and neighbour appends are
//    ordered by a ballot + lane prefix count, so lists come out in ascending j.
//
// Either mapping may split the j-set into contiguous ranges ("splits") to put
// enough waves on the 256 CUs; the per-split FP64 partial sums and neighbour
// segments are combined by the merge kernel in split order, which keeps every
// list in ascending j.  No floating-point atomics are used anywhere, so each
// plan is bitwise deterministic and a row's result does not depend on the
// other rows of the block.
#include <algorithm>

#include "nb_rows.h"

namespace nb {

namespace {

// A split launch zeroes the call's overflow word and refinement counter
// itself (its rows go to split slots, so nothing in it touches those words;
// the merge launch after it is the first to write them).
__device__ __forceinline__ void clear_call_words(const ForceArgs &a)
{
    if (a.clear0 && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) {
        *a.clear0 = 0;
        if (a.clear1) *a.clear1 = 0;
    }
}

// grid = (ceil(n_i / (IR * kBlock)), splits)
template <bool MIXED, int IR>
__global__ __launch_bounds__(kBlock) void force_rows_kernel(ForceArgs a)
{
    __shared__ JBody tile[2][kTile];
    clear_call_words(a);
    const int32_t split = blockIdx.y;
    const int64_t j0 = (int64_t)split * a.split_len;
    const int64_t j1 = j0 + a.split_len < a.n ? j0 + a.split_len : a.n;
    const Dest d{a.splits == 1, (int64_t)split, 0, (int64_t)a.splits};
    rows_pass<MIXED, IR, kTile, kBlock>(a, tile, (int64_t)blockIdx.x * IR * kBlock, a.n_i, j0, j1, d,
                         a.near_factor);
}

// One-wave work-groups of the row-per-lane pass (64 rows, a 64-body LDS tile):
// blocks of a few row tiles fill the lanes of 64-row groups instead of
// leaving most of a 256-lane work-group idle.  grid = (ceil(n_i / 64), splits).
// Held to four waves per SIMD (128 VGPRs, no spill): the plan puts about 16
// work-groups on each CU, and at the compiler's 130 VGPRs only 12 fit at
// once (64 rows took 95 us instead of 87).
template <bool MIXED>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(4))) void force_rows_wave_kernel(ForceArgs a)
{
    __shared__ JBody tile[2][kWave];
    clear_call_words(a);
    const int32_t split = blockIdx.y;
    const int64_t j0 = (int64_t)split * a.split_len;
    const int64_t j1 = j0 + a.split_len < a.n ? j0 + a.split_len : a.n;
    const Dest d{a.splits == 1, (int64_t)split, 0, (int64_t)a.splits};
    rows_pass<MIXED, 1, kWave, kWave>(a, tile, (int64_t)blockIdx.x * kWave, a.n_i, j0, j1, d,
                                      a.near_factor);
}

// Wave w (global) handles row group w % ngroups (rows G*(w%ngroups) + g) over
// j-range w / ngroups.  The row groups of one j-range are consecutive waves,
// mostly of one work-group, so the groups after the first read that range
// from cache, not from memory.  grid = ceil(waves / 4).
template <bool MIXED, int G>
__global__ __launch_bounds__(kBlock) void force_wave_kernel(ForceArgs a)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t gw = (int64_t)blockIdx.x * (kBlock / kWave) +
                       __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    clear_call_words(a);
    const int64_t ngroups = (a.n_i + G - 1) / G;
    if (gw >= ngroups * a.splits) return;   // whole wave leaves together
    const int32_t split = (int32_t)(gw / ngroups);
    const int64_t group = gw - (int64_t)split * ngroups;
    const int64_t j0 = (int64_t)split * a.split_len;
    const int64_t j1 = j0 + a.split_len < a.n ? j0 + a.split_len : a.n;
    const Dest d{a.splits == 1, (int64_t)split, 0, (int64_t)a.splits};

    // Row data is uniform across the wave (scalar registers).  The loads of
    // all G rows are issued together, at in-range indices, and invalid rows
    // are masked afterwards: every wave starts at the same time, so the
    // round trips of this setup add directly to the launch (with a branch per
    // row the G rows took 2 G dependent round trips).
    double rx[G], ry[G], rz[G], rvx[G], rvy[G], rvz[G], hi[G];
    float rs2f[G], candf[G];
    int32_t ri[G], cnt[G], lcap[G];
    int32_t *lst[G];
    Sums<MIXED> S[G];
    int64_t iraw[G];
    double rsv[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const int64_t b = group * G + g;
        const int64_t bc = b < a.n_i ? b : a.n_i - 1;
        iraw[g] = a.i_block[bc];
        rsv[g] = a.rs2[bc];
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const int64_t b = group * G + g;
        const bool ok = b < a.n_i && iraw[g] >= 0 && iraw[g] < a.n;
        const int64_t i = ok ? iraw[g] : 0;
        S[g].zero();
        cnt[g] = 0;
        ri[g] = ok ? (int32_t)i : -1;
        rx[g] = a.xp[i];
        ry[g] = a.xp[a.n + i];
        rz[g] = a.xp[2 * a.n + i];
        rvx[g] = a.vp[i];
        rvy[g] = a.vp[a.n + i];
        rvz[g] = a.vp[2 * a.n + i];
        rs2f[g] = (float)rsv[g];
        hi[g] = cand_bound_f64(rs2f[g]);
        candf[g] = cand_bound_f32(rs2f[g], a.near_factor);
        if (d.direct) {
            lst[g] = a.nb_list + b * (int64_t)a.cap;
            lcap[g] = a.cap;
        } else {
            lst[g] = a.seg_list + dest_slot(d, b) * kSegCap;
            lcap[g] = kSegCap;
        }
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
        if (ri[g] >= 0) continue;
        // no row (past n_i, or a bad index): far away, never a neighbour
        rx[g] = ry[g] = rz[g] = kFar * 0.5;
        rvx[g] = rvy[g] = rvz[g] = 0.0;
        rs2f[g] = -1.0f;
        hi[g] = -1.0;
        candf[g] = -1.0f;
        lst[g] = nullptr;
        lcap[g] = 0;
    }

    // the bodies of the next D iterations are loaded ahead (a ring of D
    // registers), so D loads per lane are in flight while one is computed:
    // with few rows per wave the loop is bound by memory latency
    constexpr int D = G == 1 ? 4 : 2;
    int iter = 0;
    JBody Jq[D];
#pragma unroll
    for (int u = 0; u < D; ++u) load_body(Jq[u], a, j0 + u * kWave + lane, j1);
    for (int64_t base0 = j0; base0 < j1; base0 += D * kWave) {
#pragma unroll
    for (int u = 0; u < D; ++u) {
        const int64_t base = base0 + u * kWave;
        if (base >= j1) break;   // uniform
        const int64_t j = base + lane;
        const JBody J = Jq[u];
        if (base + D * kWave < j1) load_body(Jq[u], a, j + D * kWave, j1);
        const int32_t jidx = (int32_t)j;
        // differences and the candidate test of every row first, then one
        // branch for the rare cases of all rows (one exec-mask change per
        // iteration instead of one per row); operands and sums unchanged
        double dx[G], dy[G], dz[G];
        bool cand[G];
        bool any = false;
#pragma unroll
        for (int g = 0; g < G; ++g) {
            dx[g] = J.x - rx[g];
            dy[g] = J.y - ry[g];
            dz[g] = J.z - rz[g];
        }
        if constexpr (MIXED) {
            float fx[G], fy[G], fz[G], r2f[G];
#pragma unroll
            for (int g = 0; g < G; ++g) {
                fx[g] = (float)dx[g];
                fy[g] = (float)dy[g];
                fz[g] = (float)dz[g];
                r2f[g] = __builtin_fmaf(fz[g], fz[g], __builtin_fmaf(fy[g], fy[g], fx[g] * fx[g]));
                cand[g] = r2f[g] < candf[g];
                any = any || cand[g];
            }
            if (__ballot(any)) {   // neighbours, self, near pairs (FP64 terms)
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    // lanes past j1 hold padding (mass 0): never a neighbour
                    const bool self = cand[g] && jidx == ri[g];
                    const bool nbr = cand[g] && (r2f[g] < rs2f[g]) && !self && j < j1;
                    const uint64_t nm = __ballot(nbr);
                    if (nbr) {
                        const int p = cnt[g] + lanes_below(nm);
                        if (p < lcap[g]) lst[g][p] = jidx;
                    }
                    cnt[g] += __popcll(nm);
                    if (cand[g] && !nbr && !self)
                        add_term_f64(S[g].ax, S[g].ay, S[g].az, S[g].jx, S[g].jy, S[g].jz,
                                     dx[g], dy[g], dz[g], J.vx - rvx[g], J.vy - rvy[g],
                                     J.vz - rvz[g], J.m);
                }
            }
#pragma unroll
            for (int g = 0; g < G; ++g)
                accum_mixed(S[g], fx[g], fy[g], fz[g], r2f[g], J.vx - rvx[g], J.vy - rvy[g],
                            J.vz - rvz[g], J.m32, cand[g]);
        } else {
            double r2[G];
            bool excl[G];
#pragma unroll
            for (int g = 0; g < G; ++g) {
                r2[g] = __builtin_fma(dz[g], dz[g], __builtin_fma(dy[g], dy[g], dx[g] * dx[g]));
                cand[g] = r2[g] < hi[g];
                excl[g] = false;
                any = any || cand[g];
            }
            if (__ballot(any)) {
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    const bool self = cand[g] && jidx == ri[g];
                    const bool nbr = cand[g] && (canon_r2f(dx[g], dy[g], dz[g]) < rs2f[g]) &&
                                     !self && j < j1;
                    const uint64_t nm = __ballot(nbr);
                    if (nbr) {
                        const int p = cnt[g] + lanes_below(nm);
                        if (p < lcap[g]) lst[g][p] = jidx;
                    }
                    cnt[g] += __popcll(nm);
                    excl[g] = nbr || self;
                }
            }
#pragma unroll
            for (int g = 0; g < G; ++g)
                accum_f64(S[g], dx[g], dy[g], dz[g], r2[g], J.vx - rvx[g], J.vy - rvy[g],
                          J.vz - rvz[g], J.m, excl[g]);
        }
        if constexpr (MIXED) {
            if (++iter == kFold) {
                iter = 0;
#pragma unroll
                for (int g = 0; g < G; ++g) S[g].fold();
            }
        }
    }
    }
    // the wave sums of all rows' eight components in one butterfly pass
    double r[G * 8];
#pragma unroll
    for (int g = 0; g < G; ++g) {
        S[g].fold();
        r[g * 8 + 0] = S[g].ax;
        r[g * 8 + 1] = S[g].ay;
        r[g * 8 + 2] = S[g].az;
        r[g * 8 + 3] = S[g].jx;
        r[g * 8 + 4] = S[g].jy;
        r[g * 8 + 5] = S[g].jz;
        r[g * 8 + 6] = S[g].va;
        r[g * 8 + 7] = S[g].vj;
    }
    group_sums<kWave, G * 8>(r);
    bool ovf = false, bad = false, nonfin = false;
#pragma unroll
    for (int g = 0; g < G; ++g) {
        Sums<MIXED> T = S[g];
        T.ax = r[g * 8 + 0];
        T.ay = r[g * 8 + 1];
        T.az = r[g * 8 + 2];
        T.jx = r[g * 8 + 3];
        T.jy = r[g * 8 + 4];
        T.jz = r[g * 8 + 5];
        T.va = r[g * 8 + 6];
        T.vj = r[g * 8 + 7];
        const int64_t b = group * G + g;
        if (lane == 0 && b < a.n_i) {
            bool o = false, bd = false, f = false;
            row_store<MIXED>(a, b, d, ri[g] >= 0, T, cnt[g], o, bd, f, j0, j1);
            ovf |= o;
            bad |= bd;
            nonfin |= f;
        }
    }
    flush_flags(a, ovf, bad, nonfin);
}

// W lanes per row (W = merge_width(splits)), kBlock / W rows per work-group.
template <int W>
__global__ __launch_bounds__(kBlock) void merge_kernel(ForceArgs a)
{
    const int64_t wave_row0 = (int64_t)blockIdx.x * (kBlock / W) +
                              __builtin_amdgcn_readfirstlane(threadIdx.x / kWave) * (kWave / W);
    if (wave_row0 >= a.n_i) return;   // whole wave past the last row
    const int64_t b = (int64_t)blockIdx.x * (kBlock / W) + threadIdx.x / W;
    const MergeGeom g{a.splits, b * a.splits, 1, 0, a.n, a.split_len};
    merge_row<W>(a, b, b < a.n_i, g);
}

// One work-group per row for plans with many splits.
__global__ __launch_bounds__(kBlock) void merge_wg_kernel(ForceArgs a)
{
    __shared__ double lds[kSlotComp][kBlock / kWave];
    __shared__ int64_t scan[kBlock / kWave];
    const int64_t b = blockIdx.x;
    const MergeGeom g{a.splits, b * a.splits, 1, 0, a.n, a.split_len};
    merge_row_wg(a, b, g, lds, scan);
}

__device__ __forceinline__ void write_forces(const ForceArgs &a, int64_t b, const double v[6])
{
    a.acc[b] = v[0];
    a.acc[a.n_i + b] = v[1];
    a.acc[2 * (int64_t)a.n_i + b] = v[2];
    a.jerk[b] = v[3];
    a.jerk[a.n_i + b] = v[4];
    a.jerk[2 * (int64_t)a.n_i + b] = v[5];
}

// Final sums of the buffered rows: six lanes per row, a lane per force
// component, each adding the row's chunk partials of its component in chunk
// order (kFinalBatch of them loaded before any is added).  Starting from zero
// in chunk order, this is the sum of the unbuffered route.  slot / slots: this
// lane's row slot and the number of slots (rows q = slot, slot + slots, ...).
constexpr int kFinalBatch = 32;
constexpr int kFinalRowsPerGroup = kBlock / 6;

__device__ __forceinline__ void redo_final_rows(const ForceArgs &a, int32_t par, int32_t slot,
                                                int32_t slots)
{
    const int k = (int)(threadIdx.x % 6);
    if (threadIdx.x >= kFinalRowsPerGroup * 6) return;
    for (int32_t q = slot; q < par; q += slots) {
        const int32_t nc = redo_row_chunks(a, q);
        const int64_t row = a.redo_rows[q];
        const double *p = a.redo_part + (int64_t)q * a.redo_chunks * 6 + k;
        double s = 0.0;
        for (int32_t c0 = 0; c0 < nc; c0 += kFinalBatch) {
            double t[kFinalBatch];
#pragma unroll
            for (int u = 0; u < kFinalBatch; ++u) t[u] = c0 + u < nc ? p[(int64_t)(c0 + u) * 6] : 0.0;
#pragma unroll
            for (int u = 0; u < kFinalBatch; ++u)
                if (c0 + u < nc) s += t[u];
        }
        double *dst = k < 3 ? a.acc + (int64_t)k * a.n_i : a.jerk + (int64_t)(k - 3) * a.n_i;
        dst[row] = s;
    }
}

// Refinement of the listed rows.  Pass 1: the first redo_rcap listed rows as
// (row group, chunk) items over the whole grid (chunk partials to scratch);
// any further rows one work-group each, chunks in order.  Pass 2 adds each
// buffered row's chunk partials in chunk order and overwrites its forces:
// with FUSED, the work-group that finishes pass 1 last does it (one launch,
// for calls that can list few rows); otherwise redo_final_kernel, launched
// next, spreads it over the GPU.  Both routes give the same chunk-ordered
// sum.  A group is kRedoRows consecutive listed rows: when they share one
// j-range (always in a single-block call) they are summed together, each body
// loaded once; otherwise row by row.  Chunks past a row's own range are
// skipped.  With no listed row every work-group leaves at once (no fence, no
// atomic), which is the common case of small blocks.
template <bool FUSED>
__global__ __launch_bounds__(kBlock) void redo_kernel(ForceArgs a)
{
    __shared__ double lds[kRedoRows * 6][kBlock / kWave];
    __shared__ int32_t last;
    const int32_t count = load_word_uniform(a.redo_count);
    if (count == 0) return;
    const int32_t par = count < a.redo_rcap ? count : a.redo_rcap;
    const int32_t C = a.redo_chunks;
    const int32_t G = (par + kRedoRows - 1) / kRedoRows;
    const int64_t items = (int64_t)G * C;
    double v[kRedoRows * 6], v1[6];
    // chunk-major order: work-groups running at the same time share a chunk
    // of bodies (L2 reuse across the refined rows)
    for (int64_t it = blockIdx.x; it < items; it += gridDim.x) {
        const int32_t c = (int32_t)(it / G), q0 = (int32_t)(it % G) * kRedoRows;
        const int nr = par - q0 < kRedoRows ? par - q0 : kRedoRows;
        bool same = true;   // uniform over the work-group
        for (int r = 1; r < nr; ++r)
            same = same && a.redo_j0[q0 + r] == a.redo_j0[q0] && a.redo_j1[q0 + r] == a.redo_j1[q0];
        if (same) {
            if (c >= redo_row_chunks(a, q0)) continue;
            redo_chunk_rows(a, q0, nr, c, lds, v);
            if (threadIdx.x == 0)
                for (int r = 0; r < nr; ++r)
#pragma unroll
                    for (int k = 0; k < 6; ++k)
                        a.redo_part[((int64_t)(q0 + r) * C + c) * 6 + k] = v[r * 6 + k];
        } else {
            for (int r = 0; r < nr; ++r) {
                const int32_t q = q0 + r;
                if (c >= redo_row_chunks(a, q)) continue;
                redo_chunk(a, q, c, lds, v1);
                if (threadIdx.x == 0)
#pragma unroll
                    for (int k = 0; k < 6; ++k) a.redo_part[((int64_t)q * C + c) * 6 + k] = v1[k];
            }
        }
    }
    for (int64_t q = (int64_t)par + blockIdx.x; q < count; q += gridDim.x) {
        double acc[6] = {0, 0, 0, 0, 0, 0};
        const int32_t nc = redo_row_chunks(a, (int32_t)q);
        for (int32_t c = 0; c < nc; ++c) {
            redo_chunk(a, (int32_t)q, c, lds, v1);
#pragma unroll
            for (int k = 0; k < 6; ++k) acc[k] += v1[k];
        }
        if (threadIdx.x == 0) write_forces(a, a.redo_rows[q], acc);
    }
    if (!FUSED || par == 0) return;   // par == 0: nothing buffered (uniform over the grid)

    // arrival: the chunk partials were written by lane 0, which publishes
    // them device-wide before it counts this work-group in
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        last = atomicAdd(a.redo_arrive, 1) == (int32_t)gridDim.x - 1;
    }
    __syncthreads();
    if (!last) return;
    __threadfence();   // every work-group's partials are visible from here
    if (threadIdx.x == 0) *a.redo_arrive = 0;   // every work-group has arrived
    redo_final_rows(a, par, (int32_t)(threadIdx.x / 6), kFinalRowsPerGroup);
}

// Pass 2 of the refinement as a launch of its own, spread over the grid: for
// calls that can list many rows, where one work-group adding them all would
// take longer than the rest of the refinement.
__global__ __launch_bounds__(kBlock) void redo_final_kernel(ForceArgs a)
{
    const int32_t count = load_word_uniform(a.redo_count);
    const int32_t par = count < a.redo_rcap ? count : a.redo_rcap;
    redo_final_rows(a, par, (int32_t)(blockIdx.x * kFinalRowsPerGroup + threadIdx.x / 6),
                    (int32_t)(gridDim.x * kFinalRowsPerGroup));
}

__global__ void fill_i32_kernel(int32_t *p, int32_t value, int64_t count)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < count) p[k] = value;
}

// Zeroes one or two words in a single launch (the overflow word and the
// refinement counter of a force call).
__global__ void clear_words_kernel(int32_t *a, int32_t *b)
{
    if (threadIdx.x == 0) {
        *a = 0;
        if (b) *b = 0;
    }
}

}  // namespace

static size_t round256(size_t b) { return (b + 255) / 256 * 256; }

size_t slot_scratch_bytes(int64_t slots)
{
    if (slots <= 0) return 0;
    const size_t s = (size_t)slots;
    return round256(s * kSlotComp * sizeof(double)) + round256(s * sizeof(int32_t)) +
           round256(s * kSegCap * sizeof(int32_t));
}

// Calls that can buffer at most this many refined rows add them up in the
// work-group that finishes pass 1 last (42 rows at a time); larger ones
// launch redo_final_kernel.  The 256-cluster ensemble
// (about 1.2e4 buffered rows) took 0.25 ms longer per call with one
// work-group adding them all.
constexpr int64_t kFusedRedoRows = 1024;

int32_t redo_groups_for(int cu_count) { return (cu_count > 0 ? cu_count : 256) * 4; }

static int32_t redo_chunks_for(int64_t max_len)
{
    const int64_t c = (max_len + kRedoChunk - 1) / kRedoChunk;
    return (int32_t)(c > 0 ? c : 1);
}

static int32_t redo_rcap_for(int32_t n_i, int32_t chunks, int32_t limit)
{
    int64_t r = kRedoPartItems / chunks;
    if (limit > 0 && r > limit) r = limit;
    if (r < 1) r = 1;
    if (r > n_i) r = n_i > 0 ? n_i : 1;
    return (int32_t)r;
}

size_t redo_scratch_bytes(int32_t n_i, int64_t max_len, int32_t rcap_limit)
{
    const int64_t rows = n_i > 0 ? n_i : 1;
    const int32_t C = redo_chunks_for(max_len);
    const int64_t parts = (int64_t)redo_rcap_for(n_i, C, rcap_limit) * C;
    return 3 * round256((size_t)rows * sizeof(int32_t)) +
           round256((size_t)parts * 6 * sizeof(double));
}

void bind_redo_scratch(ForceArgs &a, void *base, int32_t *counter, int32_t groups,
                       int64_t max_len, int32_t rcap_limit)
{
    char *p = (char *)base;
    const size_t arr = round256((size_t)(a.n_i > 0 ? a.n_i : 1) * sizeof(int32_t));
    a.redo_count = counter;
    a.redo_arrive = counter + 16;   // its own 64 bytes; zero when the words are created
    a.redo_rows = (int32_t *)p;
    a.redo_j0 = (int32_t *)(p + arr);
    a.redo_j1 = (int32_t *)(p + 2 * arr);
    a.redo_part = (double *)(p + 3 * arr);
    a.redo_groups = groups;
    a.redo_chunks = redo_chunks_for(max_len);
    a.redo_rcap = redo_rcap_for(a.n_i, a.redo_chunks, rcap_limit);
}

hipError_t launch_redo(const ForceArgs &a, hipStream_t s)
{
    // no more work-groups than the most items a call of n_i rows can list
    const int64_t rows = std::max<int64_t>(a.n_i, 1);
    const int64_t par = std::min<int64_t>(rows, a.redo_rcap);
    const int64_t items = (par + kRedoRows - 1) / kRedoRows * a.redo_chunks + (rows - par);
    const int64_t grid = std::max<int64_t>(1, std::min<int64_t>(a.redo_groups, items));
    if (par <= kFusedRedoRows) {
        hipLaunchKernelGGL(redo_kernel<true>, dim3((unsigned)grid), dim3(kBlock), 0, s, a);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(redo_kernel<false>, dim3((unsigned)grid), dim3(kBlock), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t fgrid = std::min<int64_t>(a.redo_groups, (par + kFinalRowsPerGroup - 1) / kFinalRowsPerGroup);
    hipLaunchKernelGGL(redo_final_kernel, dim3((unsigned)fgrid), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

void bind_slot_scratch(ForceArgs &a, int64_t slots, void *base)
{
    a.total_slots = slots;
    if (slots <= 0) {
        a.part = nullptr;
        a.seg_cnt = nullptr;
        a.seg_list = nullptr;
        return;
    }
    const size_t s = (size_t)slots;
    char *p = (char *)base;
    a.part = (double *)p;
    p += round256(s * kSlotComp * sizeof(double));
    a.seg_cnt = (int32_t *)p;
    p += round256(s * sizeof(int32_t));
    a.seg_list = (int32_t *)p;
}

size_t force_scratch_bytes(const Plan &p, int32_t n_i)
{
    return p.splits > 1 ? slot_scratch_bytes((int64_t)p.splits * n_i) : 0;
}

void force_bind_scratch(ForceArgs &a, void *base)
{
    bind_slot_scratch(a, a.splits > 1 ? (int64_t)a.splits * a.n_i : 0, base);
}

template <bool MIXED>
static hipError_t launch_force_t(const Plan &p, const ForceArgs &a, hipStream_t s)
{
    if (p.mapping == 1) {
        const int per = p.rows_per_lane * kBlock;
        dim3 grid((unsigned)((a.n_i + per - 1) / per), (unsigned)p.splits);
        switch (p.rows_per_lane) {
        case 1: hipLaunchKernelGGL((force_rows_kernel<MIXED, 1>), grid, dim3(kBlock), 0, s, a); break;
        case 2: hipLaunchKernelGGL((force_rows_kernel<MIXED, 2>), grid, dim3(kBlock), 0, s, a); break;
        case 4: hipLaunchKernelGGL((force_rows_kernel<MIXED, 4>), grid, dim3(kBlock), 0, s, a); break;
        default: return hipErrorInvalidValue;
        }
    } else if (p.mapping == 3) {
        dim3 grid((unsigned)((a.n_i + kWave - 1) / kWave), (unsigned)p.splits);
        hipLaunchKernelGGL((force_rows_wave_kernel<MIXED>), grid, dim3(kWave), 0, s, a);
    } else {
        const int G = p.rows_per_lane;
        const int64_t waves = ((a.n_i + G - 1) / G) * (int64_t)p.splits;
        const int64_t per = kBlock / kWave;
        dim3 grid((unsigned)((waves + per - 1) / per));
        switch (G) {
        case 1: hipLaunchKernelGGL((force_wave_kernel<MIXED, 1>), grid, dim3(kBlock), 0, s, a); break;
        case 2: hipLaunchKernelGGL((force_wave_kernel<MIXED, 2>), grid, dim3(kBlock), 0, s, a); break;
        case 4: hipLaunchKernelGGL((force_wave_kernel<MIXED, 4>), grid, dim3(kBlock), 0, s, a); break;
        default: return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

hipError_t launch_force(const Plan &p, bool mixed, const ForceArgs &a, hipStream_t s)
{
    return mixed ? launch_force_t<true>(p, a, s) : launch_force_t<false>(p, a, s);
}

hipError_t launch_merge(bool mixed, const ForceArgs &a, hipStream_t s)
{
    (void)mixed;
    if (a.splits >= 256) {   // few rows, many splits: one work-group per row
        hipLaunchKernelGGL(merge_wg_kernel, dim3((unsigned)a.n_i), dim3(kBlock), 0, s, a);
    } else {
        const int w = merge_width(a.splits);
        const int per = kBlock / w;
        dim3 grid((unsigned)((a.n_i + per - 1) / per));
        if (w == 4)
            hipLaunchKernelGGL(merge_kernel<4>, grid, dim3(kBlock), 0, s, a);
        else if (w == 16)
            hipLaunchKernelGGL(merge_kernel<16>, grid, dim3(kBlock), 0, s, a);
        else
            hipLaunchKernelGGL(merge_kernel<64>, grid, dim3(kBlock), 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_clear_words(int32_t *a, int32_t *b, hipStream_t s)
{
    hipLaunchKernelGGL(clear_words_kernel, dim3(1), dim3(64), 0, s, a, b);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t *p, int32_t value, int64_t count, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    dim3 grid((unsigned)((count + 255) / 256));
    hipLaunchKernelGGL(fill_i32_kernel, grid, dim3(256), 0, s, p, value, count);
    return hipGetLastError();
}

}  // namespace nb
