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

// Automatic plan for a block of n_i rows against n bodies.
Plan auto_plan(const nb_ctx *ctx, int64_t n, int32_t n_i, bool mixed)
{
    auto it = ctx->tuned.find(std::make_tuple((int)mixed, bucket_log2(n), bucket_log2(n_i)));
    if (it != ctx->tuned.end()) return it->second;
    Plan p{};
    const int cus = ctx->cu_count > 0 ? ctx->cu_count : 256;
    if (n_i < 256) {
        // small blocks stream the j-set: ~2 waves per SIMD in total; more
        // splits only add merge work (measured at N = 2^20, n_i = 1 .. 255)
        p.mapping = 2;
        p.rows_per_lane = n_i >= 4 ? 4 : (n_i >= 2 ? 2 : 1);
        const int64_t groups = (n_i + p.rows_per_lane - 1) / p.rows_per_lane;
        const int64_t target = (int64_t)cus * 8;
        int64_t s = (target + groups - 1) / groups;
        const int64_t max_s = std::max<int64_t>(1, n / (4 * nb::kWave));
        p.splits = (int)std::max<int64_t>(1, std::min(s, max_s));
    } else {
        // many short work-groups even out their run-time differences: a
        // split sweep over the step-level blocks at N = 2^20 was best near
        // 64 work-groups per CU in total (full block: 4 splits, +3-4%;
        // 52428 rows: 80 splits instead of 10, +25%)
        p.mapping = 1;
        p.rows_per_lane = 1;
        const int64_t wgs = (n_i + p.rows_per_lane * nb::kBlock - 1) / (p.rows_per_lane * nb::kBlock);
        const int64_t target = (int64_t)cus * 64;
        int64_t s = (target + wgs - 1) / wgs;
        const int64_t max_s = std::max<int64_t>(1, n / (8 * nb::kTile));   // >= 8 tiles a split
        p.splits = (int)std::max<int64_t>(1, std::min(s, max_s));
    }
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
