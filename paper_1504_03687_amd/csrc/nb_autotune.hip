// Autotuner for the single-block regular-force launch: times candidate plans
// (mapping, rows per lane or per wave, number of j-splits) on a synthetic
// Plummer cluster for a ladder of block sizes at the caller's n, in both
// precisions, and installs the fastest plan per (precision, log2 n, log2 n_i)
// bucket in the context.  The table can be saved to and loaded from a small
// text file.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <vector>

#include "nbreg.h"
#include "nb_runtime.h"

namespace nbrt {
namespace {

// xorshift64* generator: deterministic synthetic input for timing only.
struct Rng {
    uint64_t s;
    double uniform()
    {
        s ^= s >> 12;
        s ^= s << 25;
        s ^= s >> 27;
        return (double)((s * 2685821657736338717ull) >> 11) * 0x1p-53;
    }
};

// Plummer sphere (scale length 3 pi / 16, total mass 1) with a neighbour
// radius from the local density so that a row has ~64 neighbours.
void synth(int64_t n, std::vector<double> &x, std::vector<double> &v, std::vector<double> &m,
           std::vector<double> &rs2)
{
    const double b = 3.0 * M_PI / 16.0;
    Rng r{0x9E3779B97F4A7C15ull};
    x.resize(3 * n);
    v.resize(3 * n);
    m.assign(n, 1.0 / (double)n);
    rs2.resize(n);
    for (int64_t i = 0; i < n; ++i) {
        const double X = std::max(r.uniform() * 0.999, 1e-12);
        const double rad = b / std::sqrt(std::pow(X, -2.0 / 3.0) - 1.0);
        const double ct = 2.0 * r.uniform() - 1.0, ph = 2.0 * M_PI * r.uniform();
        const double st = std::sqrt(1.0 - ct * ct);
        x[i] = rad * st * std::cos(ph);
        x[n + i] = rad * st * std::sin(ph);
        x[2 * n + i] = rad * ct;
        for (int k = 0; k < 3; ++k) v[k * n + i] = 0.4 * (r.uniform() - 0.5);
        const double rho = (double)n * 3.0 / (4.0 * M_PI * b * b * b) *
                           std::pow(1.0 + rad * rad / (b * b), -2.5);
        const double rs = std::cbrt(64.0 * 3.0 / (4.0 * M_PI * rho));
        rs2[i] = rs * rs;
    }
}

}  // namespace
}  // namespace nbrt

using namespace nbrt;

static int load_table(nb_ctx *ctx, const char *path, int64_t n_bucket, bool *found)
{
    *found = false;
    FILE *f = std::fopen(path, "r");
    if (!f) return NB_OK;
    char head[64] = {0};
    if (!std::fgets(head, sizeof head, f) || std::strncmp(head, "nbreg-tune 2", 12) != 0) {
        std::fclose(f);
        return NB_OK;
    }
    int prec, mapping, rows, splits, f64;
    long long nb, nib;
    while (std::fscanf(f, "%d %lld %lld %d %d %d %d", &prec, &nb, &nib, &mapping, &rows, &splits,
                       &f64) == 7) {
        if (mapping < 1 || mapping > 3 || splits < 1 ||
            !(rows == 1 || rows == 2 || rows == 4) || f64 < 0 || f64 > 1)
            continue;
        ctx->tuned[std::make_tuple(prec, (int64_t)nb, (int64_t)nib)] =
            nb::Plan{mapping, rows, splits, prec == 1 ? f64 : 0};
        if (nb == n_bucket) *found = true;
    }
    std::fclose(f);
    return NB_OK;
}

extern "C" int nb_autotune(nb_ctx *ctx, int64_t n, const char *cache_path, int flags)
{
    if (!ctx || n < 64 || n > INT32_MAX) return NB_ERR_INVALID_ARG;
    if (!ctx->usable) return NB_ERR_UNSUPPORTED;
    const int64_t nbk = bucket_log2(n);
    if (cache_path && !(flags & 1)) {
        bool found = false;
        load_table(ctx, cache_path, nbk, &found);
        if (found) return NB_OK;
    }

    std::vector<double> hx, hv, hm, hrs2;
    synth(n, hx, hv, hm, hrs2);
    const int32_t max_ni = (int32_t)std::min<int64_t>(n, 65536);
    const int32_t cap = 128;
    // device buffers
    const size_t bytes = sizeof(double) * (3 * n + 3 * n + n + max_ni + 6 * (size_t)max_ni) +
                         sizeof(int32_t) * ((size_t)max_ni * (cap + 2) + 4);
    char *buf = nullptr;
    hipError_t e = hipMalloc(&buf, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return NB_ERR_OOM;
    }
    double *dx = (double *)buf, *dv = dx + 3 * n, *dm = dv + 3 * n, *drs2 = dm + n;
    double *dacc = drs2 + max_ni, *djerk = dacc + 3 * (size_t)max_ni;
    int32_t *dib = (int32_t *)(djerk + 3 * (size_t)max_ni);
    int32_t *dcnt = dib + max_ni, *dlist = dcnt + max_ni, *dovf = dlist + (size_t)max_ni * cap;
    // rows: a fixed stride permutation of the bodies
    std::vector<int32_t> ib(max_ni);
    std::vector<double> rrs2(max_ni);
    // i -> i * stride mod n is a bijection when gcd(stride, n) = 1
    int64_t stride = 40503;
    while (std::gcd(stride, n) != 1) stride += 2;
    for (int32_t k = 0; k < max_ni; ++k) {
        ib[k] = (int32_t)(((int64_t)k * stride) % n);
        rrs2[k] = hrs2[ib[k]];
    }
    e = hipMemcpy(dx, hx.data(), 3 * n * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dv, hv.data(), 3 * n * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dm, hm.data(), n * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(drs2, rrs2.data(), max_ni * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dib, ib.data(), max_ni * sizeof(int32_t), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(buf);
        return hip_fail(ctx, e);
    }

    const nb::Plan saved = ctx->forced;
    const bool saved_has = ctx->has_forced;
    const bool saved_timing = ctx->timing;
    ctx->timing = false;
    hipEvent_t t0, t1;
    (void)hipEventCreate(&t0);
    (void)hipEventCreate(&t1);
    int rc = NB_OK;
    std::vector<int32_t> ladder;
    for (int32_t ni = 1; ni <= max_ni; ni *= 4) ladder.push_back(ni);
    if (ladder.back() != max_ni) ladder.push_back(max_ni);

    for (int prec = 0; prec < 2 && rc == NB_OK; ++prec) {
        std::vector<std::pair<int64_t, nb::Plan>> best_at;
        for (int32_t ni : ladder) {
            // candidates around the automatic plan of each mapping
            ctx->has_forced = false;
            std::vector<nb::Plan> cands;
            for (int mapping = 1; mapping <= 3; ++mapping) {
                if (mapping == 1 && ni < 64) continue;
                if (mapping == 3 && (ni < 16 || ni > 1024)) continue;
                const int rows_opts[3] = {1, 2, 4};
                for (int rows : rows_opts) {
                    if (mapping == 1 && rows == 4) continue;
                    if (mapping == 2 && rows > ni) continue;
                    if (mapping == 3 && rows != 1) continue;
                    // the automatic split count of this mapping, halved and doubled
                    const int64_t base = default_splits(ctx, n, ni, mapping, rows);
                    for (int64_t sc : {base / 2, base, base * 2}) {
                        const int64_t maxs = max_splits(n, mapping);
                        const int s = (int)std::max<int64_t>(1, std::min<int64_t>(sc, maxs));
                        nb::Plan p{mapping, rows, s, 0};
                        bool dup = false;
                        for (auto &q : cands)
                            dup |= q.mapping == p.mapping && q.rows_per_lane == p.rows_per_lane &&
                                   q.splits == p.splits;
                        if (!dup) cands.push_back(p);
                    }
                }
            }
            // a mixed request on a small block may be served faster by the
            // FP64 kernels (latency-bound, and no refinement)
            if (prec == 1 && ni <= 256) {
                const size_t k = cands.size();
                for (size_t q = 0; q < k; ++q) {
                    nb::Plan p = cands[q];
                    p.f64 = 1;
                    cands.push_back(p);
                }
            }
            float best_ms = 1e30f;
            nb::Plan best{};
            for (const nb::Plan &p : cands) {
                ctx->forced = p;
                ctx->has_forced = true;
                float ms_min = 1e30f;
                for (int rep = 0; rep < 4 && rc == NB_OK; ++rep) {
                    (void)hipEventRecord(t0, ctx->stream);
                    rc = nb_regular_force(ctx, n, dx, dv, dm, ni, dib, drs2, cap,
                                          prec ? NB_MIXED : NB_FP64, dacc, djerk, dcnt, dlist,
                                          dovf, nullptr);
                    (void)hipEventRecord(t1, ctx->stream);
                    (void)hipEventSynchronize(t1);
                    float ms = 0.f;
                    (void)hipEventElapsedTime(&ms, t0, t1);
                    if (rep > 0) ms_min = std::min(ms_min, ms);
                }
                if (rc != NB_OK) break;
                if (ms_min < best_ms) {
                    best_ms = ms_min;
                    best = p;
                }
            }
            if (rc != NB_OK) break;
            best_at.push_back({bucket_log2(ni), best});
        }
        // fill the n_i buckets up to the largest tuned size from the nearest
        // tuned size below; larger blocks keep the automatic plan
        for (int64_t bk = 0; !best_at.empty() && bk <= best_at.back().first; ++bk) {
            nb::Plan p = best_at.front().second;
            for (auto &q : best_at)
                if (q.first <= bk) p = q.second;
            ctx->tuned[std::make_tuple(prec, nbk, bk)] = p;
        }
    }
    ctx->forced = saved;
    ctx->has_forced = saved_has;
    ctx->timing = saved_timing;
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    (void)hipStreamSynchronize(ctx->stream);
    (void)hipFree(buf);
    if (rc != NB_OK) return rc;

    if (cache_path) {
        FILE *f = std::fopen(cache_path, "w");
        if (f) {
            std::fprintf(f, "nbreg-tune 2\n");
            for (auto &kv : ctx->tuned)
                std::fprintf(f, "%d %lld %lld %d %d %d %d\n", std::get<0>(kv.first),
                             (long long)std::get<1>(kv.first), (long long)std::get<2>(kv.first),
                             kv.second.mapping, kv.second.rows_per_lane, kv.second.splits,
                             kv.second.f64);
            std::fclose(f);
        }
    }
    return NB_OK;
}
