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
// GPU shape (both entries): a counting sort by level.
//   count:   4096 items per work-group; wave-aggregated LDS histogram per
//            work-group, stored level-major [K][blocks], plus global totals;
//            range checks raise a flag that makes the later kernels no-ops;
//   offsets: one wave per level; exclusive scan of its row of block counts
//            plus the count of all deeper levels; writes level_end;
//   scatter: ranks within a work-group from per-wave ballots, combined in LDS
//            over (round, wave) in item order, so the result is deterministic
//            and, for the build, stable;
//   copy:    (update only) the re-sorted prefix back into the list.
#include <cmath>

#include "nbreg.h"
#include "nb_internal.h"
#include "nb_runtime.h"

namespace nb {
namespace {

constexpr int kSchedThreads = 256;
constexpr int kSchedRounds = 16;                          // items per thread
constexpr int kSchedItems = kSchedThreads * kSchedRounds;  // items per work-group
constexpr int kSchedWaves = kSchedThreads / kWave;
constexpr int kMaxLevels = 64;

__device__ __forceinline__ uint32_t lane_rank(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Level of item k, or -1 (with bad set) if the body index or the level is out
// of range.  src == nullptr: item k is body k.
__device__ __forceinline__ int32_t item_level(int64_t n, const int32_t *src, int64_t k,
                                              const int32_t *level, int32_t lmin, int32_t K,
                                              int32_t &body, bool &bad)
{
    const int64_t i = src ? (int64_t)src[k] : k;
    if (i < 0 || i >= n) {
        bad = true;
        return -1;
    }
    body = (int32_t)i;
    const int32_t L = level[i];
    if (L < lmin || L >= K) {
        bad = true;
        return -1;
    }
    return L;
}

__global__ __launch_bounds__(kSchedThreads) void sched_count_kernel(
    int64_t n, const int32_t *src, int32_t n_items, const int32_t *level, int32_t lmin,
    int32_t K, const int32_t *level_end_old, int32_t nblk, int32_t *hist, int32_t *totals,
    int32_t *flag)
{
    __shared__ int32_t h[kMaxLevels];
    for (int k = threadIdx.x; k < K; k += kSchedThreads) h[k] = 0;
    __syncthreads();
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t base = (int64_t)blockIdx.x * kSchedItems;
    bool bad = false;
    for (int r = 0; r < kSchedRounds; ++r) {
        const int64_t k = base + r * kSchedThreads + threadIdx.x;
        int32_t body = 0;
        const int32_t L = k < n_items ? item_level(n, src, k, level, lmin, K, body, bad) : -1;
        uint64_t todo = __ballot(L >= 0);
        while (todo) {
            const int first = __builtin_ctzll(todo);
            const int32_t val = __shfl(L, first);
            const uint64_t m = __ballot(L == val);
            if (lane == first) atomicAdd(&h[val], (int32_t)__popcll(m));
            todo &= ~m;
        }
    }
    // an update's prefix must be exactly the bodies of level >= lmin
    if (level_end_old && blockIdx.x == 0 && threadIdx.x == 0 && level_end_old[lmin] != n_items)
        bad = true;
    if (bad) atomicOr(flag, 1);
    __syncthreads();
    for (int k = threadIdx.x; k < K; k += kSchedThreads) {
        hist[(int64_t)k * nblk + blockIdx.x] = h[k];
        if (h[k]) atomicAdd(&totals[k], h[k]);
    }
}

// One wave per level L = blockIdx.x.
__global__ __launch_bounds__(kWave) void sched_offsets_kernel(int32_t nblk, int32_t lmin,
                                                              int32_t K, const int32_t *hist,
                                                              const int32_t *totals,
                                                              const int32_t *flag, int32_t *offs,
                                                              int32_t *level_end,
                                                              uint32_t *status)
{
    const int L = blockIdx.x;
    const int lane = threadIdx.x;
    if (*flag) {
        if (L == 0 && lane == 0 && status) atomicOr(status, (uint32_t)NB_STATUS_BAD_LEVEL);
        return;
    }
    int32_t above = 0;
    for (int k = L + 1; k < K; ++k) above += totals[k];
    int32_t run = above;
    const int32_t *row = hist + (int64_t)L * nblk;
    for (int32_t b0 = 0; b0 < nblk; b0 += kWave) {
        const int32_t b = b0 + lane;
        const int32_t c = b < nblk ? row[b] : 0;
        int32_t s = c;
        for (int d = 1; d < kWave; d <<= 1) {
            const int32_t t = __shfl_up(s, d);
            if (lane >= d) s += t;
        }
        if (b < nblk) offs[(int64_t)L * nblk + b] = run + s - c;
        run += __shfl(s, kWave - 1);
    }
    if (lane == 0) {
        if (L >= lmin) level_end[L] = above + totals[L];
        if (L == K - 1) level_end[K] = 0;
    }
}

__global__ __launch_bounds__(kSchedThreads) void sched_scatter_kernel(
    int64_t n, const int32_t *src, int32_t n_items, const int32_t *level, int32_t lmin,
    int32_t K, int32_t nblk, const int32_t *offs, const int32_t *flag, int32_t *dst)
{
    constexpr int kQ = kSchedRounds * kSchedWaves;   // (round, wave) groups, in item order
    __shared__ int32_t cnt[kQ][kMaxLevels];
    if (*flag) return;
    for (int e = threadIdx.x; e < kQ * kMaxLevels; e += kSchedThreads) (&cnt[0][0])[e] = 0;
    __syncthreads();
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const int64_t base = (int64_t)blockIdx.x * kSchedItems;
    int32_t lv[kSchedRounds], rk[kSchedRounds], body[kSchedRounds];
#pragma unroll
    for (int r = 0; r < kSchedRounds; ++r) {
        const int64_t k = base + r * kSchedThreads + threadIdx.x;
        bool bad = false;
        body[r] = 0;
        lv[r] = k < n_items ? item_level(n, src, k, level, lmin, K, body[r], bad) : -1;
        rk[r] = 0;
        uint64_t todo = __ballot(lv[r] >= 0);
        while (todo) {
            const int first = __builtin_ctzll(todo);
            const int32_t val = __shfl(lv[r], first);
            const uint64_t m = __ballot(lv[r] == val);
            if (lv[r] == val) rk[r] = (int32_t)lane_rank(m);
            if (lane == first) cnt[r * kSchedWaves + w][val] = (int32_t)__popcll(m);
            todo &= ~m;
        }
    }
    __syncthreads();
    for (int L = threadIdx.x; L < K; L += kSchedThreads) {
        int32_t run = offs[(int64_t)L * nblk + blockIdx.x];
        for (int q = 0; q < kQ; ++q) {
            const int32_t c = cnt[q][L];
            cnt[q][L] = run;
            run += c;
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kSchedRounds; ++r)
        if (lv[r] >= 0) dst[cnt[r * kSchedWaves + w][lv[r]] + rk[r]] = body[r];
}

__global__ __launch_bounds__(256) void sched_copy_kernel(const int32_t *flag, const int32_t *tmp,
                                                         int32_t n_items, int32_t *order)
{
    if (*flag) return;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n_items;
         k += (int64_t)gridDim.x * blockDim.x)
        order[k] = tmp[k];
}

struct SchedScratch {
    int32_t *hist, *offs, *totals, *flag, *tmp;
};

// Scratch: hist and offs [K][nblk], totals [64] + flag (cleared together),
// and (update) the re-sorted prefix.
int sched_scratch(nb_ctx *ctx, int32_t nblk, int32_t K, int32_t n_tmp, SchedScratch &s)
{
    auto up = [](size_t b) { return (b + 255) / 256 * 256; };
    const size_t grid = up(sizeof(int32_t) * (size_t)nblk * K);
    const size_t small = up(sizeof(int32_t) * (kMaxLevels + 64));
    const size_t bytes = 2 * grid + small + up(sizeof(int32_t) * (size_t)n_tmp);
    const int rc = nbrt::ensure_scratch(ctx, bytes);
    if (rc != NB_OK) return rc;
    char *p = (char *)ctx->scratch;
    s.hist = (int32_t *)p;
    s.offs = (int32_t *)(p + grid);
    s.totals = (int32_t *)(p + 2 * grid);
    s.flag = s.totals + kMaxLevels;
    s.tmp = (int32_t *)(p + 2 * grid + small);
    return NB_OK;
}

// Counting sort of n_items items (body src[k], or k) by level into dst.
hipError_t sched_sort(nb_ctx *ctx, int64_t n, const int32_t *src, int32_t n_items,
                      const int32_t *level, int32_t lmin, int32_t K, const int32_t *check_le,
                      const SchedScratch &s, int32_t nblk, int32_t *dst, int32_t *level_end,
                      uint32_t *status)
{
    hipError_t e = launch_fill_i32(s.totals, 0, kMaxLevels + 64, ctx->stream);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(sched_count_kernel, dim3((unsigned)nblk), dim3(kSchedThreads), 0,
                       ctx->stream, n, src, n_items, level, lmin, K, check_le, nblk, s.hist,
                       s.totals, s.flag);
    hipLaunchKernelGGL(sched_offsets_kernel, dim3((unsigned)K), dim3(kWave), 0, ctx->stream,
                       nblk, lmin, K, s.hist, s.totals, s.flag, s.offs, level_end, status);
    hipLaunchKernelGGL(sched_scatter_kernel, dim3((unsigned)nblk), dim3(kSchedThreads), 0,
                       ctx->stream, n, src, n_items, level, lmin, K, nblk, s.offs, s.flag, dst);
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
    const int32_t nblk = (int32_t)((n + nb::kSchedItems - 1) / nb::kSchedItems);
    nb::SchedScratch s;
    int rc = nb::sched_scratch(ctx, nblk, K, 0, s);
    if (rc != NB_OK) return rc;
    hipEvent_t ev[2];
    hipError_t e = timed_begin(ctx, NB_CLASS_SCHED, ev);
    if (e == hipSuccess)
        e = nb::sched_sort(ctx, n, nullptr, (int32_t)n, level, 0, K, nullptr, s, nblk, order,
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
    const int32_t nblk = (n_active + nb::kSchedItems - 1) / nb::kSchedItems;
    nb::SchedScratch s;
    int rc = nb::sched_scratch(ctx, nblk, K, n_active, s);
    if (rc != NB_OK) return rc;
    hipEvent_t ev[2];
    hipError_t e = timed_begin(ctx, NB_CLASS_SCHED, ev);
    if (e == hipSuccess)
        e = nb::sched_sort(ctx, n, order, n_active, level, L, K, level_end, s, nblk, s.tmp,
                           level_end, status);
    if (e == hipSuccess) {
        const unsigned g = (unsigned)std::min<int64_t>(1024, (n_active + 255) / 256);
        hipLaunchKernelGGL(nb::sched_copy_kernel, dim3(g), dim3(256), 0, ctx->stream, s.flag,
                           s.tmp, n_active, order);
        e = hipGetLastError();
    }
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
