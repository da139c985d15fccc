// Batched ensemble of independent clusters in one persistent launch.
//
// The paper integrates one cluster at a time; running many uneven clusters
// (an ensemble of star-cluster models) through one launch is this library's
// own extension of the regular-force step of section 3.2.1.  Each cluster's
// rows are cut into row tiles of kBlock rows (one work-group) and, for large
// clusters, its bodies into j-splits; every (cluster, row tile, split) is one
// work item.  Items are sorted longest-first on the host; a persistent grid
// of (CUs x resident work-groups) pulls them from an atomic counter, so short
// and long clusters share the chip without per-cluster launches.  Clusters
// with one split write their outputs directly; the others go through split
// slots and the same merge as the single-block launch.  The launch sequence
// (counter reset, overflow reset, persistent kernel, merge) is captured once
// per shape into a HIP graph and replayed.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <vector>

#include "nbreg.h"
#include "nb_pair.h"
#include "nb_rows.h"
#include "nb_runtime.h"

namespace nb {
namespace {

// The one-row shapes with 256-body tiles are held to four waves per SIMD
// (the mixed 256-lane one needed 129 VGPRs, one too many: 21.9 ms per call
// on the 256-cluster ensemble against 20.7 at 128, no spill); the other
// shapes would spill.
template <bool MIXED, int IR, int T, int NB>
__global__ __launch_bounds__(NB) __attribute__((amdgpu_waves_per_eu(IR == 1 && T == 256 ? 4 : 1))) void batched_kernel(BatchArgs A)
{
    __shared__ JBody tile[2][T];
    __shared__ int32_t s_item;
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(A.queue, 1);
        __syncthreads();
        const int32_t it = __builtin_amdgcn_readfirstlane(s_item);
        __syncthreads();   // every lane has read s_item before it is replaced
        if (it >= A.n_items) break;
        const BItem I = A.items[it];
        const BCluster C = A.clusters[I.cluster];
        const int64_t j0 = C.j_begin + (int64_t)I.split * C.split_len;
        const int64_t j1 = j0 + C.split_len < C.j_end ? j0 + C.split_len : C.j_end;
        const Dest d{C.splits == 1, C.slot_base + (int64_t)I.split, (int64_t)C.row_begin,
                     (int64_t)C.splits};
        rows_pass<MIXED, IR, T, NB>(A.f, tile, I.row0, (int64_t)C.row_begin + C.n_rows, j0, j1,
                                    d, C.near);
    }
}

// W lanes per merged row (W = merge_width of the largest split count among
// the split clusters), kBlock / W rows per work-group.
template <int W>
__global__ __launch_bounds__(kBlock) void batched_merge_kernel(BatchArgs A)
{
    const int64_t wave_q0 = (int64_t)blockIdx.x * (kBlock / W) +
                            __builtin_amdgcn_readfirstlane(threadIdx.x / kWave) * (kWave / W);
    if (wave_q0 >= A.n_merge_rows) return;   // whole wave past the last row
    const int64_t q = (int64_t)blockIdx.x * (kBlock / W) + threadIdx.x / W;
    const bool has = q < A.n_merge_rows;
    int64_t b = 0;
    MergeGeom g{0, 0, 1, 0, 0, 0};
    if (has) {
        b = A.merge_rows[q];
        const BCluster C = A.clusters[A.row_cluster[q]];
        g = MergeGeom{C.splits, C.slot_base + (b - C.row_begin) * C.splits, 1, C.j_begin,
                      C.j_end, C.split_len};
    }
    merge_row<W>(A.f, b, has, g);
}

template <bool MIXED, int S>
const void *batched_fn_t()
{
    constexpr BShape sh = kBatchedShape[S];
    return (const void *)&batched_kernel<MIXED, sh.rows_per_lane, sh.tile, sh.lanes>;
}

template <bool MIXED>
const void *batched_fn(int shape)
{
    static_assert(kBatchedShapes == 6, "one case per shape");
    switch (shape) {
    case 0: return batched_fn_t<MIXED, 0>();
    case 1: return batched_fn_t<MIXED, 1>();
    case 2: return batched_fn_t<MIXED, 2>();
    case 3: return batched_fn_t<MIXED, 3>();
    case 4: return batched_fn_t<MIXED, 4>();
    case 5: return batched_fn_t<MIXED, 5>();
    default: return nullptr;
    }
}

}  // namespace

int batched_shape_index(int tile, int lanes, int rows_per_lane)
{
    for (int k = 0; k < kBatchedShapes; ++k)
        if (kBatchedShape[k].tile == tile && kBatchedShape[k].lanes == lanes &&
            kBatchedShape[k].rows_per_lane == rows_per_lane)
            return k;
    return -1;
}

int batched_max_blocks_per_cu(bool mixed, int shape)
{
    const void *fn = mixed ? batched_fn<true>(shape) : batched_fn<false>(shape);
    int blocks = 0;
    if (!fn || hipOccupancyMaxActiveBlocksPerMultiprocessor(
                   &blocks, fn, kBatchedShape[shape].lanes, 0) != hipSuccess) {
        (void)hipGetLastError();
        return 1;
    }
    return blocks > 0 ? blocks : 1;
}

hipError_t launch_batched(bool mixed, int shape, int grid, const BatchArgs &a, hipStream_t s)
{
    const void *fn = mixed ? batched_fn<true>(shape) : batched_fn<false>(shape);
    if (!fn) return hipErrorInvalidValue;
    BatchArgs arg = a;
    void *args[] = {&arg};
    return hipLaunchKernel(fn, dim3((unsigned)grid), dim3((unsigned)kBatchedShape[shape].lanes),
                           args, 0, s);
}

hipError_t launch_batched_merge(const BatchArgs &a, hipStream_t s)
{
    if (a.n_merge_rows <= 0) return hipSuccess;
    const int w = merge_width(a.max_splits);
    const dim3 grid((unsigned)((a.n_merge_rows + kBlock / w - 1) / (kBlock / w)));
    if (w == 4)
        hipLaunchKernelGGL(batched_merge_kernel<4>, grid, dim3(kBlock), 0, s, a);
    else if (w == 16)
        hipLaunchKernelGGL(batched_merge_kernel<16>, grid, dim3(kBlock), 0, s, a);
    else
        hipLaunchKernelGGL(batched_merge_kernel<64>, grid, dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

}  // namespace nb

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
namespace nbrt {

struct BatchedCache {
    // key
    std::vector<int64_t> j_off, i_off;
    int32_t cap = 0;
    int prec = 0;
    int shape = 0;            // index into nb::kBatchedShape
    int items_per_cu = 64;    // work cap: items of ~1/(items_per_cu x CUs) of the pairs
    int forced_splits = 0;
    double redo_k = 0.0;
    const void *ptrs[11] = {};
    // device state
    void *dmem = nullptr;
    nb::BatchArgs args{};
    int grid = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint64_t last_use = 0;
};

static uint64_t g_use_clock = 0;

static void release_one(nb_ctx *ctx, BatchedCache *c)
{
    // the refinement counter of the last call may live in this cache
    if (ctx && c->args.f.redo_count && ctx->last_redo_counter == c->args.f.redo_count)
        ctx->last_redo_counter = nullptr;
    if (c->exec) (void)hipGraphExecDestroy(c->exec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    if (c->dmem) (void)hipFree(c->dmem);
    delete c;
}

void batched_release(nb_ctx *ctx)
{
    for (auto *c : ctx->batched) release_one(ctx, c);
    ctx->batched.clear();
}

static size_t r256(size_t b) { return (b + 255) / 256 * 256; }

// Builds the work list, uploads metadata, and captures the launch graph.
static int build_cache(nb_ctx *ctx, BatchedCache *c, const nb::ForceArgs &f, bool mixed)
{
    const int32_t C = (int32_t)c->j_off.size() - 1;
    std::vector<nb::BCluster> cl((size_t)C);
    int64_t slots = 0;
    // automatic splits: items of at most ~1/(items_per_cu per CU) of the
    // total pair work, so the queue's tail is short (as for single blocks),
    // with splits of at least 8 split units
    double total_work = 0.0;
    for (int32_t k = 0; k < C; ++k)
        total_work += (double)(c->i_off[k + 1] - c->i_off[k]) * (double)(c->j_off[k + 1] - c->j_off[k]);
    const double item_work =
        std::max(1.0, total_work / ((ctx->cu_count > 0 ? ctx->cu_count : 256) *
                                    (double)c->items_per_cu));
    const nb::BShape sh = nb::kBatchedShape[c->shape];
    const int64_t rows_per_item = (int64_t)sh.rows_per_lane * sh.lanes;
    constexpr int64_t U = nb::kSplitUnit;
    for (int32_t k = 0; k < C; ++k) {
        const int64_t nc = c->j_off[k + 1] - c->j_off[k];
        const int64_t rc = c->i_off[k + 1] - c->i_off[k];
        int64_t S;
        if (nc <= 0) {
            S = 1;
        } else if (c->forced_splits > 0) {
            S = std::min<int64_t>(c->forced_splits, (nc + U - 1) / U);
        } else {
            const double rows = (double)std::min<int64_t>(rc, rows_per_item);
            S = (int64_t)std::ceil(rows * (double)nc / item_work);
            S = std::max<int64_t>(1, std::min<int64_t>(S, nc / (8 * U)));
        }
        const int64_t tiles = std::max<int64_t>(1, (nc + U - 1) / U);
        const int64_t per = (tiles + S - 1) / S;
        const int64_t split_len = per * U;
        S = nc > 0 ? (nc + split_len - 1) / split_len : 1;
        nb::BCluster &b = cl[(size_t)k];
        b.j_begin = c->j_off[k];
        b.j_end = c->j_off[k + 1];
        b.split_len = split_len;
        b.row_begin = (int32_t)c->i_off[k];
        b.n_rows = (int32_t)rc;
        b.splits = (int32_t)S;
        b.near = nc >= nb::kNearMinBodies ? nb::kNearFactor : 1.0f;
        b.slot_base = 0;
        if (S > 1) {
            b.slot_base = slots;
            slots += S * rc;
        }
    }
    // work items, longest first
    struct W {
        int64_t work;
        nb::BItem it;
    };
    std::vector<W> items;
    std::vector<int32_t> merge_rows, row_cluster;
    for (int32_t k = 0; k < C; ++k) {
        const nb::BCluster &b = cl[(size_t)k];
        for (int64_t r = 0; r < b.n_rows; r += rows_per_item) {
            const int64_t nr = std::min<int64_t>(rows_per_item, b.n_rows - r);
            for (int32_t s = 0; s < b.splits; ++s) {
                const int64_t j0 = b.j_begin + s * b.split_len;
                const int64_t j1 = std::min<int64_t>(b.j_end, j0 + b.split_len);
                items.push_back({nr * std::max<int64_t>(j1 - j0, 1),
                                 nb::BItem{k, (int32_t)(b.row_begin + r), s, 0}});
            }
        }
        if (b.splits > 1)
            for (int32_t r = 0; r < b.n_rows; ++r) {
                merge_rows.push_back(b.row_begin + r);
                row_cluster.push_back(k);
            }
    }
    std::stable_sort(items.begin(), items.end(),
                     [](const W &x, const W &y) { return x.work > y.work; });
    std::vector<nb::BItem> it_dev(items.size());
    for (size_t q = 0; q < items.size(); ++q) it_dev[q] = items[q].it;

    // one device allocation: queue | clusters | items | merge rows | row cluster | slots
    const size_t b_queue = 256;
    const size_t b_cl = r256(cl.size() * sizeof(nb::BCluster));
    const size_t b_it = r256(std::max<size_t>(1, it_dev.size()) * sizeof(nb::BItem));
    const size_t b_mr = r256(std::max<size_t>(1, merge_rows.size()) * sizeof(int32_t));
    const size_t b_slots = nb::slot_scratch_bytes(slots);
    const int32_t groups = nb::redo_groups_for(ctx->cu_count);
    int64_t max_len = 1;
    for (int32_t k = 0; k < C; ++k) max_len = std::max<int64_t>(max_len, c->j_off[k + 1] - c->j_off[k]);
    const size_t b_redo = c->redo_k > 0.0 ? nb::redo_scratch_bytes(f.n_i, max_len) : 0;
    const size_t total = b_queue + b_cl + 2 * b_mr + b_it + b_slots + b_redo;
    if (ctx->scratch_limit && total > ctx->scratch_limit) return NB_ERR_OOM;
    hipError_t e = hipMalloc(&c->dmem, total);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        c->dmem = nullptr;
        return NB_ERR_OOM;
    }
    char *p = (char *)c->dmem;
    int32_t *queue = (int32_t *)p;
    p += b_queue;
    nb::BCluster *dcl = (nb::BCluster *)p;
    p += b_cl;
    nb::BItem *dit = (nb::BItem *)p;
    p += b_it;
    int32_t *dmr = (int32_t *)p;
    p += b_mr;
    int32_t *drc = (int32_t *)p;
    p += b_mr;
    void *dslots = p;
    p += b_slots;
    void *dredo = p;

    e = hipMemcpy(dcl, cl.data(), cl.size() * sizeof(nb::BCluster), hipMemcpyHostToDevice);
    if (e == hipSuccess && !it_dev.empty())
        e = hipMemcpy(dit, it_dev.data(), it_dev.size() * sizeof(nb::BItem),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess && !merge_rows.empty()) {
        e = hipMemcpy(dmr, merge_rows.data(), merge_rows.size() * sizeof(int32_t),
                      hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(drc, row_cluster.data(), row_cluster.size() * sizeof(int32_t),
                          hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) return hip_fail(ctx, e);

    nb::BatchArgs &A = c->args;
    A.f = f;
    nb::bind_slot_scratch(A.f, slots, dslots);
    A.f.redo_k = c->redo_k;
    // the refinement counter sits in the queue's 256-byte block, away from the
    // work counter's word
    if (c->redo_k > 0.0) nb::bind_redo_scratch(A.f, dredo, queue + 32, groups, max_len);
    A.f.splits = 0;          // per-cluster
    A.f.split_len = 0;
    A.clusters = dcl;
    A.items = dit;
    A.n_items = (int32_t)it_dev.size();
    A.queue = queue;
    A.merge_rows = dmr;
    A.row_cluster = drc;
    A.n_merge_rows = (int32_t)merge_rows.size();
    A.max_splits = 1;
    for (int32_t k = 0; k < C; ++k) A.max_splits = std::max(A.max_splits, cl[(size_t)k].splits);
    const int cus = ctx->cu_count > 0 ? ctx->cu_count : 256;
    c->grid = cus * nb::batched_max_blocks_per_cu(mixed, c->shape);
    if (A.n_items < c->grid) c->grid = std::max(1, A.n_items);

    // capture the launch sequence on a private stream (default priority)
    hipStream_t cs = nullptr;
    e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(ctx, e);
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        // the queue's block holds the work counter, the refinement counter
        // and the refinement's arrival word (which also resets itself)
        hipError_t le = nb::launch_fill_i32(queue, 0, 64, cs);
        if (le == hipSuccess) le = nb::launch_fill_i32(f.overflow, 0, 1, cs);
        if (le == hipSuccess) le = nb::launch_batched(mixed, c->shape, c->grid, A, cs);
        if (le == hipSuccess) le = nb::launch_batched_merge(A, cs);
        if (le == hipSuccess && c->redo_k > 0.0)
            le = nb::launch_redo(A.f, cs);
        e = hipStreamEndCapture(cs, &c->graph);
        if (e == hipSuccess) e = le;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&c->exec, c->graph, nullptr, nullptr, 0);
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess) return hip_fail(ctx, e);
    return NB_OK;
}

}  // namespace nbrt

using namespace nbrt;

namespace nbrt {

// Key of an ensemble shape for the tuned-shape table: FNV-1a over the
// precision, list capacity and both offset arrays.
static uint64_t ensemble_key(int prec, int32_t cap, int32_t C, const int64_t *j_off,
                             const int64_t *i_off)
{
    uint64_t h = 1469598103934665603ull;
    auto mix = [&h](uint64_t v) {
        for (int k = 0; k < 8; ++k) {
            h ^= (v >> (8 * k)) & 0xff;
            h *= 1099511628211ull;
        }
    };
    mix((uint64_t)prec);
    mix((uint64_t)(uint32_t)cap);
    mix((uint64_t)(uint32_t)C);
    for (int32_t k = 0; k <= C; ++k) {
        mix((uint64_t)j_off[k]);
        mix((uint64_t)i_off[k]);
    }
    return h;
}

// Host-side argument checks shared by the batched call and its tuner.
static int batched_check(const nb_ctx *ctx, int32_t n_clusters, const int64_t *j_off_host,
                         const int64_t *i_off_host, const double *xp, const double *vp,
                         const double *m, const int32_t *i_block, const double *rs2,
                         int32_t nb_cap, nb_precision prec, const double *acc,
                         const double *jerk, const int32_t *nb_count, const int32_t *nb_list,
                         const int32_t *overflow)
{
    if (!ctx || n_clusters < 1 || !j_off_host || !i_off_host || nb_cap < 0)
        return NB_ERR_INVALID_ARG;
    if (prec != NB_FP64 && prec != NB_MIXED) return NB_ERR_INVALID_ARG;
    if (j_off_host[0] != 0 || i_off_host[0] != 0) return NB_ERR_INVALID_ARG;
    for (int32_t k = 0; k < n_clusters; ++k)
        if (j_off_host[k + 1] < j_off_host[k] || i_off_host[k + 1] < i_off_host[k])
            return NB_ERR_INVALID_ARG;
    const int64_t n = j_off_host[n_clusters];
    const int64_t n_rows = i_off_host[n_clusters];
    if (n <= 0 || n > INT32_MAX || n_rows > INT32_MAX) return NB_ERR_INVALID_ARG;
    if (!xp || !vp || !m || !overflow) return NB_ERR_INVALID_ARG;
    if (n_rows > 0 && (!i_block || !rs2 || !acc || !jerk || !nb_count)) return NB_ERR_INVALID_ARG;
    if (n_rows > 0 && nb_cap > 0 && !nb_list) return NB_ERR_INVALID_ARG;
    if (!ctx->usable) return NB_ERR_UNSUPPORTED;
    return NB_OK;
}

}  // namespace nbrt

extern "C" int nb_regular_force_batched(nb_ctx *ctx, int32_t n_clusters, const int64_t *j_off_host,
                                        const int64_t *i_off_host, const double *xp,
                                        const double *vp, const double *m,
                                        const int32_t *i_block, const double *rs2,
                                        int32_t nb_cap, nb_precision prec, double *acc,
                                        double *jerk, int32_t *nb_count, int32_t *nb_list,
                                        int32_t *overflow, uint32_t *status)
{
    int rc = batched_check(ctx, n_clusters, j_off_host, i_off_host, xp, vp, m, i_block, rs2,
                           nb_cap, prec, acc, jerk, nb_count, nb_list, overflow);
    if (rc != NB_OK) return rc;
    const int64_t n = j_off_host[n_clusters];
    const int64_t n_rows = i_off_host[n_clusters];

    const bool mixed = prec == NB_MIXED;
    // shape: a forced one, else the tuned one for this ensemble, else the
    // default (256-body tiles, 256 lanes, one row per lane; two rows per lane
    // if the single-block plan override asks for them)
    BatchedChoice ch{(ctx->has_forced && ctx->forced.rows_per_lane == 2) ? 1 : 0, 64};
    const char *origin = "default";
    if (ctx->has_batched_forced) {
        ch = ctx->batched_forced;
        origin = "forced";
    } else {
        auto it = ctx->batched_tuned.find(
            ensemble_key((int)prec, nb_cap, n_clusters, j_off_host, i_off_host));
        if (it != ctx->batched_tuned.end()) {
            ch = it->second;
            origin = "tuned";
        }
    }
    const int fsplits = ctx->has_forced ? ctx->forced.splits : 0;
    const double rk = mixed ? redo_k(ctx) : 0.0;
    const void *ptrs[11] = {xp, vp, m, i_block, rs2, acc, jerk, nb_count, nb_list, overflow,
                            status};
    BatchedCache *hit = nullptr;
    for (auto *c : ctx->batched) {
        if (c->cap == nb_cap && c->prec == (int)prec && c->shape == ch.shape &&
            c->items_per_cu == ch.items_per_cu && c->forced_splits == fsplits &&
            c->redo_k == rk && (int32_t)c->j_off.size() == n_clusters + 1 &&
            std::memcmp(c->ptrs, ptrs, sizeof ptrs) == 0 &&
            std::equal(c->j_off.begin(), c->j_off.end(), j_off_host) &&
            std::equal(c->i_off.begin(), c->i_off.end(), i_off_host)) {
            hit = c;
            break;
        }
    }
    if (!hit) {
        if (ctx->batched.size() >= 4) {   // evict the least recently used shape
            auto old = std::min_element(ctx->batched.begin(), ctx->batched.end(),
                                        [](const BatchedCache *x, const BatchedCache *y) {
                                            return x->last_use < y->last_use;
                                        });
            hipError_t e = hipStreamSynchronize(ctx->stream);
            if (e != hipSuccess) return hip_fail(ctx, e);
            release_one(ctx, *old);
            ctx->batched.erase(old);
        }
        auto *c = new BatchedCache();
        c->j_off.assign(j_off_host, j_off_host + n_clusters + 1);
        c->i_off.assign(i_off_host, i_off_host + n_clusters + 1);
        c->cap = nb_cap;
        c->prec = (int)prec;
        c->shape = ch.shape;
        c->items_per_cu = ch.items_per_cu;
        c->forced_splits = fsplits;
        c->redo_k = rk;
        std::memcpy(c->ptrs, ptrs, sizeof ptrs);
        nb::ForceArgs f{};
        f.n = n;
        f.xp = xp;
        f.vp = vp;
        f.m = m;
        f.n_i = (int32_t)n_rows;
        f.i_block = i_block;
        f.rs2 = rs2;
        f.cap = nb_cap;
        f.acc = acc;
        f.jerk = jerk;
        f.nb_count = nb_count;
        f.nb_list = nb_list;
        f.overflow = overflow;
        f.status = status;
        rc = build_cache(ctx, c, f, mixed);
        if (rc != NB_OK) {
            release_one(ctx, c);
            return rc;
        }
        ctx->batched.push_back(c);
        hit = c;
    }
    hit->last_use = ++g_use_clock;
    ctx->last_redo_counter = hit->redo_k > 0.0 ? hit->args.f.redo_count : nullptr;
    const nb::BShape &sh = nb::kBatchedShape[hit->shape];
    std::snprintf(ctx->last_plan, sizeof ctx->last_plan,
                  "batched clusters=%d items=%d grid=%d tile=%d lanes=%d rows_per_lane=%d "
                  "items_per_cu=%d merge_rows=%d shape=%s prec=%s",
                  n_clusters, hit->args.n_items, hit->grid, sh.tile, sh.lanes, sh.rows_per_lane,
                  hit->items_per_cu, hit->args.n_merge_rows, origin, mixed ? "mixed" : "fp64");
    hipEvent_t ev[2];
    hipError_t e = timed_begin(ctx, NB_CLASS_BATCHED, ev);
    if (e == hipSuccess) e = hipGraphLaunch(hit->exec, ctx->stream);
    if (e == hipSuccess) e = timed_end(ctx, NB_CLASS_BATCHED, ev);
    return e == hipSuccess ? NB_OK : hip_fail(ctx, e);
}

extern "C" int nb_ctx_set_batched_shape(nb_ctx *ctx, int tile, int lanes, int rows_per_lane,
                                        int items_per_cu)
{
    if (!ctx) return NB_ERR_INVALID_ARG;
    if (tile == 0 && lanes == 0 && rows_per_lane == 0 && items_per_cu == 0) {
        ctx->has_batched_forced = false;
        return NB_OK;
    }
    if (items_per_cu < 0 || items_per_cu > 4096) return NB_ERR_INVALID_ARG;
    const int k = nb::batched_shape_index(tile, lanes, rows_per_lane);
    if (k < 0) return NB_ERR_UNSUPPORTED;
    ctx->batched_forced = BatchedChoice{k, items_per_cu > 0 ? items_per_cu : 64};
    ctx->has_batched_forced = true;
    return NB_OK;
}

// Candidate work caps of the batched tuner (items per CU).
static const int kTuneItemsPerCu[] = {16, 64, 256};

extern "C" int nb_autotune_batched(nb_ctx *ctx, int32_t n_clusters, const int64_t *j_off_host,
                                   const int64_t *i_off_host, const double *xp, const double *vp,
                                   const double *m, const int32_t *i_block, const double *rs2,
                                   int32_t nb_cap, nb_precision prec, double *acc, double *jerk,
                                   int32_t *nb_count, int32_t *nb_list, int32_t *overflow,
                                   uint32_t *status, const char *cache_path, int flags)
{
    int rc = batched_check(ctx, n_clusters, j_off_host, i_off_host, xp, vp, m, i_block, rs2,
                           nb_cap, prec, acc, jerk, nb_count, nb_list, overflow);
    if (rc != NB_OK) return rc;
    const uint64_t key = ensemble_key((int)prec, nb_cap, n_clusters, j_off_host, i_off_host);
    if (cache_path && !(flags & 1)) {
        FILE *f = std::fopen(cache_path, "r");
        if (f) {
            char head[64] = {0};
            bool found = false;
            if (std::fgets(head, sizeof head, f) &&
                std::strncmp(head, "nbreg-batched-tune 1", 20) == 0) {
                unsigned long long kk;
                int tile, lanes, rows, ipc;
                while (std::fscanf(f, "%llx %d %d %d %d", &kk, &tile, &lanes, &rows, &ipc) == 5) {
                    const int sh = nb::batched_shape_index(tile, lanes, rows);
                    if (sh < 0 || ipc < 1 || ipc > 4096) continue;
                    ctx->batched_tuned[(uint64_t)kk] = BatchedChoice{sh, ipc};
                    found |= (uint64_t)kk == key;
                }
            }
            std::fclose(f);
            if (found) return NB_OK;
        }
    }
    const bool saved_has = ctx->has_batched_forced;
    const BatchedChoice saved = ctx->batched_forced;
    const bool saved_timing = ctx->timing;
    ctx->timing = false;
    hipEvent_t t0 = nullptr, t1 = nullptr;
    hipError_t e = hipEventCreate(&t0);
    if (e == hipSuccess) e = hipEventCreate(&t1);
    float best_ms = 1e30f;
    BatchedChoice best{0, 64};
    for (int shape = 0; shape < nb::kBatchedShapes && rc == NB_OK && e == hipSuccess; ++shape)
        for (int ipc : kTuneItemsPerCu) {
            ctx->batched_forced = BatchedChoice{shape, ipc};
            ctx->has_batched_forced = true;
            // first call builds and captures; then the best of three replays
            rc = nb_regular_force_batched(ctx, n_clusters, j_off_host, i_off_host, xp, vp, m,
                                          i_block, rs2, nb_cap, prec, acc, jerk, nb_count,
                                          nb_list, overflow, status);
            float ms_min = 1e30f;
            for (int rep = 0; rep < 3 && rc == NB_OK && e == hipSuccess; ++rep) {
                e = hipEventRecord(t0, ctx->stream);
                if (e != hipSuccess) break;
                rc = nb_regular_force_batched(ctx, n_clusters, j_off_host, i_off_host, xp, vp,
                                              m, i_block, rs2, nb_cap, prec, acc, jerk,
                                              nb_count, nb_list, overflow, status);
                if (e == hipSuccess) e = hipEventRecord(t1, ctx->stream);
                if (e == hipSuccess) e = hipEventSynchronize(t1);
                float ms = 0.f;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
                ms_min = std::min(ms_min, ms);
            }
            if (rc != NB_OK || e != hipSuccess) break;
            if (ms_min < best_ms) {
                best_ms = ms_min;
                best = ctx->batched_forced;
            }
            // keep only the cached graph of the best shape so far
            if (!(best.shape == shape && best.items_per_cu == ipc)) {
                e = hipStreamSynchronize(ctx->stream);
                for (auto it = ctx->batched.begin(); it != ctx->batched.end(); ++it)
                    if ((*it)->shape == shape && (*it)->items_per_cu == ipc &&
                        (*it)->prec == (int)prec && (*it)->cap == nb_cap) {
                        release_one(ctx, *it);
                        ctx->batched.erase(it);
                        break;
                    }
            }
        }
    ctx->has_batched_forced = saved_has;
    ctx->batched_forced = saved;
    ctx->timing = saved_timing;
    if (t0) (void)hipEventDestroy(t0);
    if (t1) (void)hipEventDestroy(t1);
    if (rc != NB_OK) return rc;
    if (e != hipSuccess) return hip_fail(ctx, e);
    ctx->batched_tuned[key] = best;
    // the caller's outputs end with the tuned shape's results
    rc = nb_regular_force_batched(ctx, n_clusters, j_off_host, i_off_host, xp, vp, m, i_block,
                                  rs2, nb_cap, prec, acc, jerk, nb_count, nb_list, overflow,
                                  status);
    if (rc != NB_OK) return rc;
    if (cache_path) {
        FILE *f = std::fopen(cache_path, "w");
        if (f) {
            std::fprintf(f, "nbreg-batched-tune 1\n");
            for (auto &kv : ctx->batched_tuned) {
                const nb::BShape &sh = nb::kBatchedShape[kv.second.shape];
                std::fprintf(f, "%llx %d %d %d %d\n", (unsigned long long)kv.first, sh.tile,
                             sh.lanes, sh.rows_per_lane, kv.second.items_per_cu);
            }
            std::fclose(f);
        }
    }
    return NB_OK;
}
