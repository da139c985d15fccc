// Host runtime and C ABI of libnbreg (see include/nbreg.h for the contract).
//
// The context owns only its scratch memory (grown on demand, bounded by a
// limit), timing events, the autotuned plan table and the cached HIP graphs of
// the batched entry point.  Every entry point validates its arguments on the
// host, picks a plan and enqueues kernels on the context's stream; nothing
// synchronises except nb_autotune, nb_ctx_kernel_time and nb_ctx_destroy.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "nbreg.h"
#include "nb_internal.h"
#include "nb_pair.h"
#include "nb_runtime.h"

using nb::Plan;

// ---------------------------------------------------------------------------
// fixed workspace of the allocation-free entry point
// ---------------------------------------------------------------------------
// One copy per GPU, part of the library's code object: it exists from the
// moment the library's kernels are loaded on a device until the process ends.
// Host code never uses this name as a device address (on the host it is only
// a stand-in); the address comes from hipGetSymbolAddress, looked up once per
// device when the first context on that device is created.
static constexpr size_t kFixedScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kFixedScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_fixed_mu;
void *g_fixed_ptr[kMaxDevices] = {};

// Device address of 'scratch' on the current device (which must be
// 'device'), looked up on first use and kept.
hipError_t fixed_scratch_of(int device, void **out)
{
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_fixed_mu);
    if (!g_fixed_ptr[device]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_fixed_ptr[device] = p;
    }
    *out = g_fixed_ptr[device];
    return hipSuccess;
}
}  // namespace

// ---------------------------------------------------------------------------
// context helpers
// ---------------------------------------------------------------------------
namespace nbrt {

int hip_fail(nb_ctx *ctx, hipError_t e)
{
    if (ctx) ctx->last_hip_error = e;
    return NB_ERR_HIP;
}

// Grows a context-owned device buffer to at least 'bytes' (contents are not
// kept); the scratch limit bounds each buffer.
static int ensure_buffer(nb_ctx *ctx, void **buf, size_t *have, size_t bytes)
{
    if (bytes <= *have) return NB_OK;
    if (ctx->scratch_limit && bytes > ctx->scratch_limit) return NB_ERR_OOM;
    if (*buf) {
        // the old buffer may still be in use by queued work on the stream
        hipError_t e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess) return hip_fail(ctx, e);
        (void)hipFree(*buf);
        *buf = nullptr;
        *have = 0;
    }
    size_t want = std::max(bytes, (size_t)1 << 20);
    want = (want + ((size_t)1 << 20) - 1) & ~(((size_t)1 << 20) - 1);
    if (ctx->scratch_limit && want > ctx->scratch_limit) want = bytes;
    hipError_t e = hipMalloc(buf, want);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *buf = nullptr;
        return NB_ERR_OOM;
    }
    *have = want;
    return NB_OK;
}

int ensure_scratch(nb_ctx *ctx, size_t bytes)
{
    return ensure_buffer(ctx, &ctx->scratch, &ctx->scratch_bytes, bytes);
}

int ensure_aux(nb_ctx *ctx, size_t bytes)
{
    return ensure_buffer(ctx, &ctx->aux, &ctx->aux_bytes, bytes);
}

hipError_t timed_begin(nb_ctx *ctx, int cls, hipEvent_t *ev)
{
    ev[0] = ev[1] = nullptr;
    if (!ctx->timing) return hipSuccess;
    for (int k = 0; k < 2; ++k) {
        if (!ctx->free_events.empty()) {
            ev[k] = ctx->free_events.back();
            ctx->free_events.pop_back();
        } else {
            hipError_t e = hipEventCreate(&ev[k]);
            if (e != hipSuccess) return e;
        }
    }
    (void)cls;
    return hipEventRecord(ev[0], ctx->stream);
}

hipError_t timed_end(nb_ctx *ctx, int cls, hipEvent_t *ev)
{
    if (!ctx->timing || !ev[0]) return hipSuccess;
    hipError_t e = hipEventRecord(ev[1], ctx->stream);
    if (e != hipSuccess) return e;
    ctx->pending.push_back({cls, ev[0], ev[1]});
    return hipSuccess;
}

double redo_k(const nb_ctx *ctx)
{
    if (!(ctx->mixed_tol > 0.0)) return 0.0;
    return 0x1p-24 * ctx->mixed_safety / ctx->mixed_tol;
}

}  // namespace nbrt

using namespace nbrt;

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

int nb_version(void) { return 10000; }   // 1.0.0

const char *nb_error_string(int code)
{
    switch (code) {
    case NB_OK: return "ok";
    case NB_ERR_INVALID_ARG: return "invalid argument";
    case NB_ERR_HIP: return "HIP runtime error";
    case NB_ERR_OOM: return "out of device memory or over the scratch limit";
    case NB_ERR_UNSUPPORTED: return "unsupported device or plan";
    case NB_ERR_TOO_LARGE:
        return "block too large for the fixed workspace of the allocation-free entry point";
    default: return "unknown error";
    }
}

int nb_ctx_create(nb_ctx **out, int device, void *hip_stream)
{
    if (!out) return NB_ERR_INVALID_ARG;
    *out = nullptr;
    nb_ctx *ctx = new (std::nothrow) nb_ctx();
    if (!ctx) return NB_ERR_OOM;
    ctx->device = device;
    ctx->stream = (hipStream_t)hip_stream;
    if (device >= 0) {
        int count = 0;
        if (hipGetDeviceCount(&count) != hipSuccess || device >= count) {
            (void)hipGetLastError();
            delete ctx;
            return NB_ERR_UNSUPPORTED;
        }
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
            delete ctx;
            return NB_ERR_HIP;
        }
        if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
            delete ctx;
            return NB_ERR_UNSUPPORTED;
        }
        ctx->cu_count = prop.multiProcessorCount;
        // the context's own device words, allocated on its device
        int prev = 0;
        (void)hipGetDevice(&prev);
        hipError_t e = hipSetDevice(device);
        if (e == hipSuccess) e = hipMalloc((void **)&ctx->words, 256);
        // the refinement's arrival word must start at zero (it resets itself)
        if (e == hipSuccess) e = hipMemset(ctx->words, 0, 256);
        if (e == hipSuccess) e = fixed_scratch_of(device, &ctx->fixed_scratch);
        (void)hipSetDevice(prev);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            delete ctx;
            return NB_ERR_OOM;
        }
        ctx->usable = true;
    }
    // device < 0: a host-only context that validates arguments and launches
    // nothing (every compute call returns NB_ERR_UNSUPPORTED after checks).
    *out = ctx;
    return NB_OK;
}

int nb_ctx_set_stream(nb_ctx *ctx, void *hip_stream)
{
    if (!ctx) return NB_ERR_INVALID_ARG;
    ctx->stream = (hipStream_t)hip_stream;
    return NB_OK;
}

int nb_ctx_destroy(nb_ctx *ctx)
{
    if (!ctx) return NB_ERR_INVALID_ARG;
    if (ctx->usable) {
        (void)hipSetDevice(ctx->device);
        (void)hipStreamSynchronize(ctx->stream);
        nbrt::batched_release(ctx);
        if (ctx->scratch) (void)hipFree(ctx->scratch);
        if (ctx->aux) (void)hipFree(ctx->aux);
        if (ctx->words) (void)hipFree(ctx->words);
        for (auto &p : ctx->pending) {
            (void)hipEventDestroy(p.start);
            (void)hipEventDestroy(p.stop);
        }
        for (auto e : ctx->free_events) (void)hipEventDestroy(e);
    }
    delete ctx;
    return NB_OK;
}

int nb_ctx_set_plan(nb_ctx *ctx, int mapping, int rows_per_lane, int splits)
{
    if (!ctx) return NB_ERR_INVALID_ARG;
    if (mapping < 0 || mapping > 3 || splits < 0) return NB_ERR_INVALID_ARG;
    if (!(rows_per_lane == 0 || rows_per_lane == 1 || rows_per_lane == 2 || rows_per_lane == 4))
        return NB_ERR_INVALID_ARG;
    ctx->forced = Plan{mapping, rows_per_lane, splits};
    ctx->has_forced = mapping != 0 || rows_per_lane != 0 || splits != 0;
    return NB_OK;
}

int nb_ctx_last_plan(nb_ctx *ctx, char *buf, int len)
{
    if (!ctx || !buf || len <= 0) return NB_ERR_INVALID_ARG;
    std::snprintf(buf, (size_t)len, "%s", ctx->last_plan);
    return NB_OK;
}

int nb_ctx_set_scratch_limit(nb_ctx *ctx, int64_t bytes)
{
    if (!ctx || bytes < 0) return NB_ERR_INVALID_ARG;
    ctx->scratch_limit = (size_t)bytes;
    return NB_OK;
}

int nb_ctx_enable_timing(nb_ctx *ctx, int on)
{
    if (!ctx) return NB_ERR_INVALID_ARG;
    ctx->timing = on != 0;
    return NB_OK;
}

int nb_ctx_kernel_time(nb_ctx *ctx, int kernel_class, double *ms, int64_t *launches)
{
    if (!ctx || kernel_class < 0 || kernel_class >= NB_NCLASS || !ms || !launches)
        return NB_ERR_INVALID_ARG;
    if (ctx->usable) {
        for (auto &p : ctx->pending) {
            hipError_t e = hipEventSynchronize(p.stop);
            if (e != hipSuccess) return hip_fail(ctx, e);
            float t = 0.f;
            e = hipEventElapsedTime(&t, p.start, p.stop);
            if (e != hipSuccess) return hip_fail(ctx, e);
            ctx->ms[p.cls] += t;
            ctx->launches[p.cls] += 1;
            ctx->free_events.push_back(p.start);
            ctx->free_events.push_back(p.stop);
        }
        ctx->pending.clear();
    }
    *ms = ctx->ms[kernel_class];
    *launches = ctx->launches[kernel_class];
    return NB_OK;
}

int nb_ctx_reset_timing(nb_ctx *ctx)
{
    if (!ctx) return NB_ERR_INVALID_ARG;
    double ms;
    int64_t l;
    int rc = nb_ctx_kernel_time(ctx, 0, &ms, &l);   // drains pending events
    if (rc != NB_OK) return rc;
    for (int k = 0; k < NB_NCLASS; ++k) {
        ctx->ms[k] = 0.0;
        ctx->launches[k] = 0;
    }
    return NB_OK;
}

int nb_predict(nb_ctx *ctx, int64_t n, double t, const double *x, const double *v,
               const double *a, const double *jrk, const double *t0, const double *m,
               double *xp, double *vp, float *m32)
{
    if (!ctx || n <= 0 || n > INT32_MAX) return NB_ERR_INVALID_ARG;
    if (!x || !v || !a || !jrk || !t0 || !xp || !vp) return NB_ERR_INVALID_ARG;
    if ((m == nullptr) != (m32 == nullptr)) return NB_ERR_INVALID_ARG;
    if (!std::isfinite(t)) return NB_ERR_INVALID_ARG;
    if (!ctx->usable) return NB_ERR_UNSUPPORTED;
    hipEvent_t ev[2];
    hipError_t e = timed_begin(ctx, NB_CLASS_PREDICT, ev);
    if (e == hipSuccess) e = nb::launch_predict(n, t, x, v, a, jrk, t0, m, xp, vp, m32, ctx->stream);
    if (e == hipSuccess) e = timed_end(ctx, NB_CLASS_PREDICT, ev);
    return e == hipSuccess ? NB_OK : hip_fail(ctx, e);
}

}  // extern "C"

namespace nbrt {

// Shared body of nb_regular_force and nb_regular_force_noalloc.  With
// fixed == nullptr the scratch comes from the context (grown on demand);
// otherwise it is the caller-supplied device workspace of fixed_bytes, no
// allocation and no event creation happens, and the plan's split count is
// lowered until its scratch fits (NB_ERR_TOO_LARGE when even one split does
// not).
static int regular_force_impl(nb_ctx *ctx, int64_t n, const double *xp, const double *vp,
                              const double *m, int32_t n_i, const int32_t *i_block,
                              const double *rs2, int32_t nb_cap, nb_precision prec,
                              double *acc, double *jerk, int32_t *nb_count, int32_t *nb_list,
                              int32_t *overflow, uint32_t *status, void *fixed,
                              size_t fixed_bytes)
{
    if (!ctx || n <= 0 || n > INT32_MAX || n_i < 0 || nb_cap < 0) return NB_ERR_INVALID_ARG;
    if (prec != NB_FP64 && prec != NB_MIXED) return NB_ERR_INVALID_ARG;
    if (!xp || !vp || !m || !overflow) return NB_ERR_INVALID_ARG;
    if (n_i > 0 && (!i_block || !rs2 || !acc || !jerk || !nb_count)) return NB_ERR_INVALID_ARG;
    if (n_i > 0 && nb_cap > 0 && !nb_list) return NB_ERR_INVALID_ARG;
    if (!ctx->usable) return NB_ERR_UNSUPPORTED;

    hipError_t e = hipSuccess;
    if (n_i == 0) {
        e = nb::launch_clear_words(overflow, nullptr, ctx->stream);
        if (e != hipSuccess) return hip_fail(ctx, e);
        std::snprintf(ctx->last_plan, sizeof ctx->last_plan, "empty");
        return NB_OK;
    }
    Plan p = auto_plan(ctx, n, n_i, prec == NB_MIXED);
    if (ctx->has_forced) {
        if (ctx->forced.mapping) p.mapping = ctx->forced.mapping;
        if (ctx->forced.rows_per_lane) p.rows_per_lane = ctx->forced.rows_per_lane;
        if (ctx->forced.splits) p.splits = ctx->forced.splits;
        p.f64 = ctx->forced.f64;   // a forced plan runs the requested kernels
    }
    const bool mixed = prec == NB_MIXED && !p.f64;
    int64_t split_len = 0;
    finish_plan(p, n, n_i, &split_len);

    nb::ForceArgs fa{};
    fa.n = n;
    fa.xp = xp;
    fa.vp = vp;
    fa.m = m;
    fa.n_i = n_i;
    fa.i_block = i_block;
    fa.rs2 = rs2;
    fa.cap = nb_cap;
    fa.acc = acc;
    fa.jerk = jerk;
    fa.nb_count = nb_count;
    fa.nb_list = nb_list;
    fa.overflow = overflow;
    fa.status = status;
    fa.redo_k = mixed ? redo_k(ctx) : 0.0;
    fa.near_factor = n >= nb::kNearMinBodies ? nb::kNearFactor : 1.0f;
    const int32_t groups = nb::redo_groups_for(ctx->cu_count);
    void *base = nullptr;
    int32_t rcap_limit = ctx->redo_rows_limit;   // 0: automatic
    size_t redo_bytes = fa.redo_k > 0.0 ? nb::redo_scratch_bytes(n_i, n, rcap_limit) : 0;
    if (fixed) {
        // the refinement's chunk partials shrink first (rows past them are
        // summed one work-group each, to the same bits), then the splits
        for (rcap_limit = rcap_limit > 0 ? rcap_limit : (int32_t)nb::kRedoPartItems;
             redo_bytes > fixed_bytes / 2 && rcap_limit > 1; rcap_limit /= 2)
            redo_bytes = nb::redo_scratch_bytes(n_i, n, rcap_limit / 2);
        if (redo_bytes > fixed_bytes) return NB_ERR_TOO_LARGE;
        const size_t room = fixed_bytes - redo_bytes;
        while (p.splits > 1 && nb::force_scratch_bytes(p, n_i) > room) {
            // largest split count whose slots fit, then re-normalised
            const size_t per_slot = nb::kSlotComp * sizeof(double) + sizeof(int32_t) +
                                    nb::kSegCap * sizeof(int32_t);
            const int64_t fit = (int64_t)(room / per_slot) / std::max<int32_t>(n_i, 1);
            p.splits = (int)std::max<int64_t>(1, std::min<int64_t>(fit, p.splits - 1));
            finish_plan(p, n, n_i, &split_len);
        }
        base = fixed;
    }
    fa.splits = p.splits;
    fa.split_len = split_len;
    const size_t slot_bytes = nb::force_scratch_bytes(p, n_i);
    if (!fixed && redo_bytes + slot_bytes > 0) {
        int rc = ensure_scratch(ctx, redo_bytes + slot_bytes);
        if (rc != NB_OK) return rc;
        base = ctx->scratch;
    }
    if (redo_bytes) nb::bind_redo_scratch(fa, base, ctx->words, groups, n, rcap_limit);
    // the overflow word and the refinement counter start at zero: zeroed by
    // the force kernel of a split launch, else by one small launch first
    if (p.splits > 1) {
        fa.clear0 = overflow;
        fa.clear1 = redo_bytes ? fa.redo_count : nullptr;
    } else {
        e = nb::launch_clear_words(overflow, redo_bytes ? fa.redo_count : nullptr, ctx->stream);
        if (e != hipSuccess) return hip_fail(ctx, e);
    }
    nb::force_bind_scratch(fa, (char *)base + redo_bytes);
    std::snprintf(ctx->last_plan, sizeof ctx->last_plan,
                  "mapping=%d rows_per_lane=%d splits=%d split_len=%lld prec=%s%s%s", p.mapping,
                  p.rows_per_lane, p.splits, (long long)split_len, mixed ? "mixed" : "fp64",
                  p.f64 && prec == NB_MIXED ? " requested=mixed" : "",
                  fixed ? " workspace=fixed" : "");

    // timing events are created on demand, so the allocation-free path is
    // never timed
    const bool timed = !fixed;
    hipEvent_t ev[2] = {nullptr, nullptr};
    if (timed) e = timed_begin(ctx, NB_CLASS_FORCE, ev);
    if (e == hipSuccess) e = nb::launch_force(p, mixed, fa, ctx->stream);
    if (e == hipSuccess && timed) e = timed_end(ctx, NB_CLASS_FORCE, ev);
    if (e != hipSuccess) return hip_fail(ctx, e);
    if (p.splits > 1) {
        if (timed) e = timed_begin(ctx, NB_CLASS_MERGE, ev);
        if (e == hipSuccess) e = nb::launch_merge(mixed, fa, ctx->stream);
        if (e == hipSuccess && timed) e = timed_end(ctx, NB_CLASS_MERGE, ev);
        if (e != hipSuccess) return hip_fail(ctx, e);
    }
    if (redo_bytes) {
        if (timed) e = timed_begin(ctx, NB_CLASS_REDO, ev);
        if (e == hipSuccess) e = nb::launch_redo(fa, ctx->stream);
        if (e == hipSuccess && timed) e = timed_end(ctx, NB_CLASS_REDO, ev);
        if (e != hipSuccess) return hip_fail(ctx, e);
        ctx->last_redo_counter = fa.redo_count;
    } else {
        ctx->last_redo_counter = nullptr;
    }
    return NB_OK;
}

}  // namespace nbrt

extern "C" {

int nb_regular_force(nb_ctx *ctx, int64_t n, const double *xp, const double *vp,
                     const double *m, int32_t n_i, const int32_t *i_block, const double *rs2,
                     int32_t nb_cap, nb_precision prec, double *acc, double *jerk,
                     int32_t *nb_count, int32_t *nb_list, int32_t *overflow, uint32_t *status)
{
    return regular_force_impl(ctx, n, xp, vp, m, n_i, i_block, rs2, nb_cap, prec, acc, jerk,
                              nb_count, nb_list, overflow, status, nullptr, 0);
}

int nb_regular_force_noalloc(nb_ctx *ctx, int64_t n, const double *xp, const double *vp,
                             const double *m, int32_t n_i, const int32_t *i_block,
                             const double *rs2, int32_t nb_cap, nb_precision prec, double *acc,
                             double *jerk, int32_t *nb_count, int32_t *nb_list,
                             int32_t *overflow, uint32_t *status)
{
    if (ctx && ctx->usable && !ctx->fixed_scratch) return NB_ERR_UNSUPPORTED;
    return regular_force_impl(ctx, n, xp, vp, m, n_i, i_block, rs2, nb_cap, prec, acc, jerk,
                              nb_count, nb_list, overflow, status,
                              ctx ? ctx->fixed_scratch : nullptr, kFixedScratchBytes);
}

int nb_fixed_workspace_bytes(int64_t *bytes)
{
    if (!bytes) return NB_ERR_INVALID_ARG;
    *bytes = (int64_t)kFixedScratchBytes;
    return NB_OK;
}

int nb_ctx_set_mixed_tolerance(nb_ctx *ctx, double tol, double safety)
{
    if (!ctx || !(tol >= 0.0) || !(safety > 0.0)) return NB_ERR_INVALID_ARG;
    ctx->mixed_tol = tol;
    ctx->mixed_safety = safety;
    return NB_OK;
}

int nb_ctx_set_refine_buffer_rows(nb_ctx *ctx, int32_t rows)
{
    if (!ctx || rows < 0) return NB_ERR_INVALID_ARG;
    ctx->redo_rows_limit = rows;
    return NB_OK;
}

int nb_ctx_last_refined_rows(nb_ctx *ctx, int32_t *rows)
{
    if (!ctx || !rows) return NB_ERR_INVALID_ARG;
    *rows = 0;
    if (!ctx->usable || !ctx->last_redo_counter) return NB_OK;
    hipError_t e = hipMemcpyAsync(rows, ctx->last_redo_counter, sizeof(int32_t),
                                  hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    return e == hipSuccess ? NB_OK : hip_fail(ctx, e);
}

int nb_regular_force_adjoint(nb_ctx *ctx, int64_t n, const double *xp, const double *vp,
                             const double *m, int32_t n_i, const int32_t *i_block,
                             const double *rs2, const double *w_a, const double *w_j,
                             double *gx, double *gv, double *gm, uint32_t *status)
{
    if (!ctx || n <= 0 || n > INT32_MAX || n_i < 0) return NB_ERR_INVALID_ARG;
    if (!xp || !vp || !m || !gx || !gv || !gm) return NB_ERR_INVALID_ARG;
    if (n_i > 0 && (!i_block || !rs2 || !w_a || !w_j)) return NB_ERR_INVALID_ARG;
    if (!ctx->usable) return NB_ERR_UNSUPPORTED;
    const int cus = ctx->cu_count > 0 ? ctx->cu_count : 256;
    // as for the forward pass: many short work-groups (~64 per CU in total),
    // with at least 2048 bodies (row pass) or 512 rows (body pass) per split
    const int64_t target = (int64_t)cus * 64;
    const int64_t row_wgs = std::max<int64_t>(1, (n_i + nb::kBlock - 1) / nb::kBlock);
    const int64_t body_wgs = (n + nb::kBlock - 1) / nb::kBlock;
    int row_splits = (int)std::max<int64_t>(
        1, std::min<int64_t>((target + row_wgs - 1) / row_wgs, std::max<int64_t>(1, n / 2048)));
    int body_splits = (int)std::max<int64_t>(
        1, std::min<int64_t>((target + body_wgs - 1) / body_wgs,
                             std::max<int64_t>(1, (n_i + 511) / 512)));
    int rc = ensure_scratch(ctx, nb::adjoint_scratch_bytes(n, n_i, row_splits, body_splits));
    if (rc != NB_OK) return rc;
    nb::AdjointArgs aa{};
    aa.n = n;
    aa.xp = xp;
    aa.vp = vp;
    aa.m = m;
    aa.n_i = n_i;
    aa.i_block = i_block;
    aa.rs2 = rs2;
    aa.w_a = w_a;
    aa.w_j = w_j;
    aa.gx = gx;
    aa.gv = gv;
    aa.gm = gm;
    aa.status = status;
    hipEvent_t ev[2];
    hipError_t e = timed_begin(ctx, NB_CLASS_ADJOINT, ev);
    if (e == hipSuccess)
        e = nb::launch_adjoint_plan(aa, row_splits, body_splits, ctx->scratch, ctx->stream);
    if (e == hipSuccess) e = timed_end(ctx, NB_CLASS_ADJOINT, ev);
    return e == hipSuccess ? NB_OK : hip_fail(ctx, e);
}

}  // extern "C"
