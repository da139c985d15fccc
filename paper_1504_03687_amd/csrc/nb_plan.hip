// Launch plans of the regular-force kernels: which mapping, how many rows
// per lane or per wave, and how many contiguous j-splits.  These rules shape
// every force launch (and so its memory traffic); the rest of the runtime is
// in nb_runtime.hip.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "nbreg.h"
#include "nb_internal.h"
#include "nb_runtime.h"

using nb::Plan;

namespace nbrt {

int64_t bucket_log2(int64_t v)
{
    int64_t b = 0;
    while ((int64_t(1) << (b + 1)) <= v) ++b;
    return b;
}

// Largest useful split count: splits of about 4 waves' worth of bodies in the
// wave mapping, 2 tiles in the row-per-lane mapping.  With a row's split
// partials contiguous the merge stays cheap at high split counts.  At
// N = 2^20: the 1272-row block ran 14% faster (mixed) with 3-tile splits
// (1366) than with the earlier 8-tile floor (512), and 2-tile splits (2048)
// tie with 3-tile ones there; a single row tile (255 rows) took 308 us with
// 2048 splits, 339 us with 1366 and 318 us with 1024 (mixed; FP64 353 / 387 /
// 362 us): 2048 work-groups spread evenly over 256 CUs.
int64_t max_splits(int64_t n, int mapping)
{
    const int64_t unit = mapping == 2 ? 4 * nb::kWave : mapping == 3 ? 2 * nb::kWave : 2 * nb::kTile;
    return std::max<int64_t>(1, (n + unit - 1) / unit);
}

// Split count of the automatic plan for a given mapping and rows per lane
// (or per wave).
//  * mapping 2 (small blocks stream the j-set): about 2 waves per SIMD in
//    total, and at most kWaveMaxSplits splits per row; more splits only add
//    merge work (measured at N = 2^20, n_i = 1 .. 255).
//  * mapping 3 (one-wave work-groups, 64 rows each): about 16 work-groups
//    per CU in total (a 64-row block at N = 2^20: 4096 splits 104.7 us,
//    2048 108.4, 1024 149.9, FP64).
//  * mapping 1: many short work-groups even out their run-time differences;
//    a split sweep over the step-level blocks at N = 2^20 was best near 64
//    work-groups per CU in total (full block: 4 splits, +3-4%; 52428 rows:
//    80 splits instead of 10, +25%).
constexpr int64_t kWaveMaxSplits = 1024;

int64_t default_splits(const nb_ctx *ctx, int64_t n, int32_t n_i, int mapping, int rows)
{
    const int64_t cus = ctx->cu_count > 0 ? ctx->cu_count : 256;
    int64_t units, target;
    if (mapping == 2) {
        units = (n_i + rows - 1) / rows;                       // row groups, one wave each
        target = cus * 8;
    } else if (mapping == 3) {
        units = (n_i + nb::kWave - 1) / nb::kWave;             // one-wave work-groups
        target = cus * 16;
    } else {
        units = (n_i + (int64_t)rows * nb::kBlock - 1) / ((int64_t)rows * nb::kBlock);
        target = cus * 64;                                      // work-groups
    }
    // mapping 2 rounds down: with only ~2 work-groups per CU, one wave group
    // past the target puts a third work-group on some CU and stretches the
    // whole launch by half (72 rows at N = 2^20: 2052 waves took 257 us,
    // against 152 us for 64 rows in 2048 waves).  finish_plan can only lower
    // the count further.  Mapping 1 rounds up: at ~64 work-groups per CU one
    // extra costs little.
    const int64_t u = std::max<int64_t>(units, 1);
    int64_t s = mapping == 2 ? std::max<int64_t>(1, target / u) : (target + u - 1) / u;
    // mapping 2 with few row groups: at most kWaveMaxSplits splits.  Each
    // split adds a partial to every row's merge, which one work-group reads;
    // with bodies loaded four iterations ahead, one wave per SIMD streams the
    // j-set as fast as two.  FP64, N = 2^20, forced plans: 1 row 20.6 us at
    // 2048 splits, 19.7 at 1024, 21.1 at 512; 4 rows 29.1 / 25.6 / 31.9 us.
    if (mapping == 2) s = std::min(s, kWaveMaxSplits);
    return std::max<int64_t>(1, std::min(s, max_splits(n, mapping)));
}

// Mappings of the automatic plan by block size, from steady-state calls at
// N = 2^20 (mixed / FP64 kernels, whole call):
//  * wave mapping (rows in scalar registers, lanes over j) up to
//    kWaveMaxRows: 32 rows 67.6 us FP64, against 104.7 us with one-wave
//    row-per-lane work-groups (half their lanes idle) and more than that with
//    256-lane work-groups;
//  * above that, one-wave row-per-lane work-groups (mapping 3) when the
//    256-row tiles of mapping 1 would hold more than 1.2 times the rows of
//    64-row tiles, else mapping 1.  Per filled lane mapping 1 is the faster
//    one (256 rows 255 / 350 us against 268 / 362 with mapping 3, 512 rows
//    512 / 669 against 559 / 714), so it needs a clear lane advantage:
//    64 rows 87 us mixed against 136 (wave), 192 rows 207 / 276 against
//    226 / 285, 320 rows 379 / 451 against 508 / 598, 832 rows 896 / 1179
//    against 939 / 1268; at 448 rows (ratio 1.14) the two tie, at 640 (1.2)
//    mapping 1 leads by 4%, at 1088 (1.18) by 21%.  The largest block this
//    picks mapping 3 for is 832 rows.
constexpr int32_t kWaveMaxRows = 40;

// Largest block whose mixed-precision request runs the FP64 kernels in the
// automatic plan: the wave mapping, which is bound by memory latency, so its
// FP64 kernel is no slower than the mixed one, and it needs no refinement
// launch (nor, for a flagged row, the refinement itself).  N = 2^20, mixed vs
// FP64 wave kernels: 1 row 22.7 vs 20.4 us, 8 rows 36.7 vs 31.4, 32 rows
// 124.7 (one row refined) vs 67.3.  From 64 rows up the mixed one-wave
// row-per-lane kernel is ahead (87 against the FP64 wave kernel's 137 us).
// The results of such a call meet the FP64 bar.
constexpr int32_t kMixedAsF64MaxRows = kWaveMaxRows;

// Automatic plan for a block of n_i rows against n bodies: the autotuned
// entry for the size buckets if there is one, else the mapping for its size
// (above).
Plan auto_plan(const nb_ctx *ctx, int64_t n, int32_t n_i, bool mixed)
{
    auto it = ctx->tuned.find(std::make_tuple((int)mixed, bucket_log2(n), bucket_log2(n_i)));
    if (it != ctx->tuned.end()) return it->second;
    if (mixed && n_i <= kMixedAsF64MaxRows) {
        Plan p = auto_plan(ctx, n, n_i, false);
        p.f64 = 1;
        return p;
    }
    Plan p{};
    p.rows_per_lane = 1;
    if (n_i <= kWaveMaxRows) {
        p.mapping = 2;
        p.rows_per_lane = n_i >= 4 ? 4 : (n_i >= 2 ? 2 : 1);
    } else {
        const int64_t pad1 = ((int64_t)n_i + nb::kBlock - 1) / nb::kBlock * nb::kBlock;
        const int64_t pad3 = ((int64_t)n_i + nb::kWave - 1) / nb::kWave * nb::kWave;
        p.mapping = pad1 * 5 > pad3 * 6 ? 3 : 1;
    }
    p.splits = (int)default_splits(ctx, n, n_i, p.mapping, p.rows_per_lane);
    return p;
}

// Normalises a plan for (n, n_i): fills zero fields, rounds split lengths.
void finish_plan(Plan &p, int64_t n, int32_t n_i, int64_t *split_len)
{
    if (p.splits < 1) p.splits = 1;
    const int64_t unit = p.mapping == 1 ? nb::kTile : nb::kWave;
    const int64_t units = (n + unit - 1) / unit;
    int64_t per = (units + p.splits - 1) / p.splits;
    if (per < 1) per = 1;
    *split_len = per * unit;
    p.splits = (int)((n + *split_len - 1) / *split_len);
    if (p.splits < 1) p.splits = 1;
    if (p.mapping == 1 && p.splits > 65535) {   // grid.y limit
        *split_len = ((n + 65534) / 65535 + unit - 1) / unit * unit;
        p.splits = (int)((n + *split_len - 1) / *split_len);
    }
    (void)n_i;
}

}  // namespace nbrt
