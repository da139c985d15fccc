// Sorting-list selection of active bodies for hierarchical block time steps
// (Wang et al. 2015, section 3.3.1 and Figures 1-2).
//
// The body indices are kept in a list ordered by step, smallest step (deepest
// level, step 2^-level) first, with boundary offsets level_end[L] = number of
// bodies with level >= L.  With synchronised block steps every body's time is
// a multiple of its step, so at a block time whose coarsest dividing step is
// 2^-L the due bodies are exactly those with level >= L: the list prefix
// order[0 : level_end[L]].  Selecting the block costs nothing, and the prefix
// is directly the i_block argument of the force entry points.
//
// After the block is integrated only the active bodies change step, and a new
// step must divide the block time, so every new level is again >= L: the
// update re-sorts the active prefix alone by its new levels and rewrites
// level_end[L..].  That is O(N_i), never O(N).  Within one level the order
// after an update follows the counting sort of the prefix (the paper allows
// giving up stability); the full build is stable (ties by ascending index).
//
// GPU shape: a counting sort by level, deterministic.  Each wave owns a
// contiguous run of items and walks it in rounds of 64: per round, one ballot
// per distinct level gives every item its rank among the wave's earlier items
// of that level (a running per-wave count in LDS); the per-level wave counts
// are then scanned across waves (and work-groups) in item order, so the
// build is stable.  All rounds' gathers are issued before any is used.
//   <= 16384 items: one work-group of 1024 threads does the whole sort in one
//            launch, in place (every read of the list precedes the first
//            write);
//   larger:  two launches: count (4096 items per work-group: per-level
//            counts stored level-major [K][blocks], a per-block range flag,
//            and for an update a copy of the prefix), then scatter (each
//            work-group sums the count rows it needs for its own offsets, so
//            no scan kernel and no cleared counters are needed).
// Out-of-range input turns the sort into a no-op that sets a status bit.
#include <cmath>

#include "nbreg.h"
#include "nb_internal.h"
#include "nb_runtime.h"

namespace nb {
namespace {

constexpr int kMaxLevels = 64;
constexpr int kRounds = 16;   // rounds of 64 items per wave
// multi-work-group path
constexpr int kMwThreads = 256;
constexpr int kMwItems = kMwThreads * kRounds;
// single-work-group path
constexpr int kSwThreads = 1024;
constexpr int kSwItems = kSwThreads * kRounds;

__device__ __forceinline__ uint32_t lane_rank(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Item of round r of this lane: with reff rounds per wave, wave w owns items
// [w*64*reff, (w+1)*64*reff) of the work-group's range, so item order is
// (wave, round, lane) order.
__device__ __forceinline__ int64_t item_index(int64_t base, int r, int reff)
{
    return base + (int64_t)(threadIdx.x / kWave) * (kWave * reff) + r * kWave +
           (threadIdx.x & (kWave - 1));
}

// Body index (src[k], or k) and level of this lane's items (rounds r < reff);
// lv = -1 for missing items.  Returns true if an item has a body index outside
// [0, n) or a level outside [lmin, K).  Loads use clamped indices so all of a
// kind are in flight together.  copy (optional) receives src[k] per item.
template <int R>
__device__ __forceinline__ bool load_items(int64_t n, const int32_t *src, int32_t n_items,
                                           const int32_t *level, int32_t lmin, int32_t K,
                                           int64_t base, int reff, int32_t (&body)[R],
                                           int32_t (&lv)[R], int32_t *copy)
{
    int32_t raw[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        body[r] = -1;
        if (r < reff) {
            int64_t k = item_index(base, r, reff);
            k = k < n_items ? k : n_items - 1;
            body[r] = src ? src[k] : (int32_t)k;
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int32_t i = body[r];
        raw[r] = -1;
        if (r < reff) raw[r] = level[(i >= 0 && i < n) ? i : 0];
    }
    bool bad = false;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t k = item_index(base, r, reff);
        lv[r] = -1;
        if (r < reff && k < n_items) {
            if (copy) copy[k] = body[r];
            const int32_t i = body[r], L = raw[r];
            if (i < 0 || i >= n || L < lmin || L >= K)
                bad = true;
            else
                lv[r] = L;
        }
    }
    return bad;
}

// Ranks within the wave: rk[r] = number of the wave's earlier items with the
// same level.  Returns the wave's count of level L in lane L (the running
// counts live in that VGPR and are read back with readlane, so the loop has no
// memory round trip).
template <int R>
__device__ __forceinline__ int32_t wave_rank(const int32_t (&lv)[R], int32_t (&rk)[R])
{
    const int lane = threadIdx.x & (kWave - 1);
    int32_t runv = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        rk[r] = 0;
        uint64_t todo = __ballot(lv[r] >= 0);
        while (todo) {
            const int first = __builtin_ctzll(todo);
            const int32_t val = __builtin_amdgcn_readlane(lv[r], first);
            const uint64_t m = __ballot(lv[r] == val);
            const int32_t before = __builtin_amdgcn_readlane(runv, val);
            if (lv[r] == val) rk[r] = before + (int32_t)lane_rank(m);
            if (lane == val) runv += (int32_t)__popcll(m);
            todo &= ~m;
        }
    }
    return runv;
}

// Exclusive scan of the per-wave level counts across the W waves, in wave
// order, for every level: thread (L = tid / W, w = tid % W) with T = 64 W.
// Replaces run[w][L] by start[L] + (count of level L in waves < w) and returns
// the level total in *total (valid in the thread with w == W-1).
template <int W>
__device__ __forceinline__ int32_t wave_scan_first(int32_t (*run)[kMaxLevels], int32_t K,
                                                   int32_t *excl_out)
{
    const int L = threadIdx.x / W, w = threadIdx.x % W;
    const int32_t v = L < K ? run[w][L] : 0;
    int32_t incl = v;
    for (int d = 1; d < W; d <<= 1) {
        const int32_t t = __shfl_up(incl, d, W);
        if (w >= d) incl += t;
    }
    *excl_out = incl - v;
    return incl;
}

// above[L] = number of items with level > L from per-level totals tot[]
// (LDS), computed by wave 0; also writes level_end[L] (L >= lmin) and
// level_end[K] = 0 when level_end is given.
__device__ __forceinline__ void level_offsets(const int32_t *tot, int32_t K, int32_t lmin,
                                              int32_t *above, int32_t *level_end)
{
    if (threadIdx.x >= kWave) return;
    const int lane = threadIdx.x;
    const int Ll = K - 1 - lane;   // lane l holds level K-1-l
    const int32_t v = Ll >= 0 ? tot[Ll] : 0;
    int32_t s = v;
    for (int d = 1; d < kWave; d <<= 1) {
        const int32_t t = __shfl_up(s, d);
        if (lane >= d) s += t;
    }
    if (Ll >= 0) {
        above[Ll] = s - v;
        if (level_end && Ll >= lmin) level_end[Ll] = s;
    }
    if (level_end && lane == 0) level_end[K] = 0;
}

// Whole sort of 1 <= n_items <= kSwItems items in one work-group, written to
// dst (which may be src).
__global__ __launch_bounds__(kSwThreads) void sched_single_kernel(
    int64_t n, const int32_t *src, int32_t n_items, const int32_t *level, int32_t lmin,
    int32_t K, const int32_t *level_end_old, int32_t *dst, int32_t *level_end,
    uint32_t *status)
{
    constexpr int W = kSwThreads / kWave;
    __shared__ int32_t run[W][kMaxLevels];
    __shared__ int32_t tot[kMaxLevels], above[kMaxLevels];
    __shared__ int32_t bad_any;
    const int w = threadIdx.x / kWave;
    if (threadIdx.x == 0) bad_any = 0;
    __syncthreads();
    // spread the items evenly: reff rounds per wave
    const int reff = (n_items + kSwThreads - 1) / kSwThreads;
    int32_t body[kRounds], lv[kRounds], rk[kRounds];
    bool bad = load_items<kRounds>(n, src, n_items, level, lmin, K, 0, reff, body, lv, nullptr);
    // an update's prefix must be exactly the bodies of level >= lmin
    if (level_end_old && threadIdx.x == 0 && level_end_old[lmin] != n_items) bad = true;
    if (bad) atomicOr(&bad_any, 1);
    run[w][threadIdx.x & (kWave - 1)] = wave_rank<kRounds>(lv, rk);
    __syncthreads();
    if (bad_any) {
        if (threadIdx.x == 0 && status) atomicOr(status, (uint32_t)NB_STATUS_BAD_LEVEL);
        return;
    }
    int32_t excl;
    const int32_t incl = wave_scan_first<W>(run, K, &excl);
    const int Ls = threadIdx.x / W, ws = threadIdx.x % W;
    if (Ls < K && ws == W - 1) tot[Ls] = incl;
    __syncthreads();
    level_offsets(tot, K, lmin, above, level_end);
    __syncthreads();
    if (Ls < K) run[ws][Ls] = above[Ls] + excl;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kRounds; ++r)
        if (lv[r] >= 0) dst[run[w][lv[r]] + rk[r]] = body[r];
}

// Multi-work-group pass 1: per-block level counts into hist[L][b], the block's
// range flag into bad_blk[b], and (update) the prefix copied to copy[].
__global__ __launch_bounds__(kMwThreads) void sched_count_kernel(
    int64_t n, const int32_t *src, int32_t n_items, const int32_t *level, int32_t lmin,
    int32_t K, const int32_t *level_end_old, int32_t nblk, int32_t *hist, int32_t *bad_blk,
    int32_t *copy)
{
    __shared__ int32_t h[kMaxLevels];
    __shared__ int32_t bad_any;
    if (threadIdx.x < kMaxLevels) h[threadIdx.x] = 0;
    if (threadIdx.x == 0) bad_any = 0;
    __syncthreads();
    const int lane = threadIdx.x & (kWave - 1);
    int32_t body[kRounds], lv[kRounds];
    bool bad = load_items<kRounds>(n, src, n_items, level, lmin, K,
                                   (int64_t)blockIdx.x * kMwItems, kRounds, body, lv, copy);
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
        uint64_t todo = __ballot(lv[r] >= 0);
        while (todo) {
            const int first = __builtin_ctzll(todo);
            const int32_t val = __builtin_amdgcn_readlane(lv[r], first);
            const uint64_t m = __ballot(lv[r] == val);
            if (lane == first) atomicAdd(&h[val], (int32_t)__popcll(m));
            todo &= ~m;
        }
    }
    if (level_end_old && blockIdx.x == 0 && threadIdx.x == 0 && level_end_old[lmin] != n_items)
        bad = true;
    if (bad) atomicOr(&bad_any, 1);
    __syncthreads();
    if (threadIdx.x < K) hist[(int64_t)threadIdx.x * nblk + blockIdx.x] = h[threadIdx.x];
    if (threadIdx.x == 0) bad_blk[blockIdx.x] = bad_any;
}

// Multi-work-group pass 2: offsets of this block from the count rows, then the
// scatter.  Block 0 writes level_end and the status bit.
__global__ __launch_bounds__(kMwThreads) void sched_scatter_kernel(
    int64_t n, const int32_t *src, int32_t n_items, const int32_t *level, int32_t lmin,
    int32_t K, int32_t nblk, const int32_t *hist, const int32_t *bad_blk, int32_t *dst,
    int32_t *level_end, uint32_t *status)
{
    constexpr int W = kMwThreads / kWave;   // 4 threads per level slot below
    __shared__ int32_t run[W][kMaxLevels];
    __shared__ int32_t tot[kMaxLevels], above[kMaxLevels], before[kMaxLevels];
    int bad = 0;
    for (int32_t b = threadIdx.x; b < nblk; b += kMwThreads) bad |= bad_blk[b];
    if (__syncthreads_or(bad)) {
        if (blockIdx.x == 0 && threadIdx.x == 0 && status)
            atomicOr(status, (uint32_t)NB_STATUS_BAD_LEVEL);
        return;
    }
    const int w = threadIdx.x / kWave;
    {
        // level totals and the counts of blocks before this one: thread
        // (L = tid / W, part = tid % W) sums a quarter of row L
        const int L = threadIdx.x / W, part = threadIdx.x % W;
        int32_t all = 0, bef = 0;
        if (L < K) {
            const int32_t *row = hist + (int64_t)L * nblk;
            for (int32_t b = part; b < nblk; b += W) {
                const int32_t c = row[b];
                all += c;
                bef += b < (int32_t)blockIdx.x ? c : 0;
            }
        }
        for (int d = 1; d < W; d <<= 1) {
            all += __shfl_xor(all, d, W);
            bef += __shfl_xor(bef, d, W);
        }
        if (L < K && part == 0) {
            tot[L] = all;
            before[L] = bef;
        }
    }
    __syncthreads();
    level_offsets(tot, K, lmin, above, blockIdx.x == 0 ? level_end : nullptr);
    int32_t body[kRounds], lv[kRounds], rk[kRounds];
    (void)load_items<kRounds>(n, src, n_items, level, lmin, K, (int64_t)blockIdx.x * kMwItems,
                              kRounds, body, lv, nullptr);
    run[w][threadIdx.x & (kWave - 1)] = wave_rank<kRounds>(lv, rk);
    __syncthreads();
    int32_t excl;
    (void)wave_scan_first<W>(run, K, &excl);
    const int Ls = threadIdx.x / W, ws = threadIdx.x % W;
    __syncthreads();
    if (Ls < K) run[ws][Ls] = above[Ls] + before[Ls] + excl;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kRounds; ++r)
        if (lv[r] >= 0) dst[run[w][lv[r]] + rk[r]] = body[r];
}

struct SchedScratch {
    int32_t *hist, *bad_blk, *copy;
};

// Scratch of the multi-work-group path: hist [K][nblk], bad_blk [nblk] and
// (update) a copy of the prefix.
int sched_prepare(nb_ctx *ctx, int32_t n_items, int32_t K, bool in_place, SchedScratch &s)
{
    s = SchedScratch{};
    if (n_items <= kSwItems) return NB_OK;
    const int32_t nblk = (n_items + kMwItems - 1) / kMwItems;
    auto up = [](size_t b) { return (b + 255) / 256 * 256; };
    const size_t h = up(sizeof(int32_t) * (size_t)nblk * K);
    const size_t f = up(sizeof(int32_t) * (size_t)nblk);
    const size_t c = in_place ? up(sizeof(int32_t) * (size_t)n_items) : 0;
    const int rc = nbrt::ensure_scratch(ctx, h + f + c);
    if (rc != NB_OK) return rc;
    char *p = (char *)ctx->scratch;
    s.hist = (int32_t *)p;
    s.bad_blk = (int32_t *)(p + h);
    s.copy = in_place ? (int32_t *)(p + h + f) : nullptr;
    return NB_OK;
}

// Counting sort of n_items items (body src[k], or k) by level into dst (dst
// may be src; then the multi-work-group path reads the copy made by pass 1).
hipError_t sched_sort(nb_ctx *ctx, int64_t n, const int32_t *src, int32_t n_items,
                      const int32_t *level, int32_t lmin, int32_t K, const int32_t *check_le,
                      const SchedScratch &s, int32_t *dst, int32_t *level_end, uint32_t *status)
{
    if (n_items <= kSwItems) {
        hipLaunchKernelGGL(sched_single_kernel, dim3(1), dim3(kSwThreads), 0, ctx->stream, n,
                           src, n_items, level, lmin, K, check_le, dst, level_end, status);
        return hipGetLastError();
    }
    const int32_t nblk = (n_items + kMwItems - 1) / kMwItems;
    hipLaunchKernelGGL(sched_count_kernel, dim3((unsigned)nblk), dim3(kMwThreads), 0,
                       ctx->stream, n, src, n_items, level, lmin, K, check_le, nblk, s.hist,
                       s.bad_blk, s.copy);
    hipLaunchKernelGGL(sched_scatter_kernel, dim3((unsigned)nblk), dim3(kMwThreads), 0,
                       ctx->stream, n, s.copy ? s.copy : src, n_items, level, lmin, K, nblk,
                       s.hist, s.bad_blk, dst, level_end, status);
    return hipGetLastError();
}

}  // namespace
}  // namespace nb

using namespace nbrt;

extern "C" {

int nb_sched_build(nb_ctx *ctx, int64_t n, const int32_t *level, int32_t k_max, int32_t *order,
                   int32_t *level_end, uint32_t *status)
{
    if (!ctx || n <= 0 || n > INT32_MAX || k_max < 0 || k_max >= nb::kMaxLevels || !level ||
        !order || !level_end)
        return NB_ERR_INVALID_ARG;
    if (!ctx->usable) return NB_ERR_UNSUPPORTED;
    const int32_t K = k_max + 1;
    nb::SchedScratch s;
    int rc = nb::sched_prepare(ctx, (int32_t)n, K, false, s);
    if (rc != NB_OK) return rc;
    hipEvent_t ev[2];
    hipError_t e = timed_begin(ctx, NB_CLASS_SCHED, ev);
    if (e == hipSuccess)
        e = nb::sched_sort(ctx, n, nullptr, (int32_t)n, level, 0, K, nullptr, s, order,
                           level_end, status);
    if (e == hipSuccess) e = timed_end(ctx, NB_CLASS_SCHED, ev);
    return e == hipSuccess ? NB_OK : hip_fail(ctx, e);
}

int nb_sched_update(nb_ctx *ctx, int64_t n, int32_t n_active, int32_t L, const int32_t *level,
                    int32_t k_max, int32_t *order, int32_t *level_end, uint32_t *status)
{
    if (!ctx || n <= 0 || n > INT32_MAX || k_max < 0 || k_max >= nb::kMaxLevels || L < 0 ||
        L > k_max || n_active < 0 || n_active > n || !level || !order || !level_end)
        return NB_ERR_INVALID_ARG;
    if (!ctx->usable) return NB_ERR_UNSUPPORTED;
    if (n_active == 0) return NB_OK;
    const int32_t K = k_max + 1;
    nb::SchedScratch s;
    int rc = nb::sched_prepare(ctx, n_active, K, true, s);
    if (rc != NB_OK) return rc;
    hipEvent_t ev[2];
    hipError_t e = timed_begin(ctx, NB_CLASS_SCHED, ev);
    if (e == hipSuccess)
        e = nb::sched_sort(ctx, n, order, n_active, level, L, K, level_end, s, order,
                           level_end, status);
    if (e == hipSuccess) e = timed_end(ctx, NB_CLASS_SCHED, ev);
    return e == hipSuccess ? NB_OK : hip_fail(ctx, e);
}

int nb_sched_next(double t_now, int32_t k_max, const int32_t *level_end_host, double *t_new,
                  int32_t *level, int32_t *n_active)
{
    if (k_max < 0 || k_max >= nb::kMaxLevels || !level_end_host || !t_new || !level ||
        !n_active || !(t_now >= 0.0) || !std::isfinite(t_now))
        return NB_ERR_INVALID_ARG;
    const int32_t *le = level_end_host;
    if (le[0] <= 0 || le[k_max + 1] != 0) return NB_ERR_INVALID_ARG;
    for (int32_t k = 0; k <= k_max; ++k)
        if (le[k] < le[k + 1]) return NB_ERR_INVALID_ARG;
    // the smallest step is that of the first body of the list (deepest level)
    int32_t kd = k_max;
    while (le[kd] == 0) --kd;
    const double dt_min = std::ldexp(1.0, -kd);
    const double q = std::ldexp(t_now, kd);
    if (q != std::floor(q)) return NB_ERR_INVALID_ARG;   // steps not synchronised
    const double tn = t_now + dt_min;
    if (tn - t_now != dt_min) return NB_ERR_INVALID_ARG;   // time no longer resolves the step
    // coarsest level whose step divides the new block time
    int32_t L = 0;
    while (L < kd) {
        const double r = std::ldexp(tn, L);
        if (r == std::floor(r)) break;
        ++L;
    }
    *t_new = tn;
    *level = L;
    *n_active = le[L];
    return NB_OK;
}

}  // extern "C"
