// Neighbour-radius control (Wang et al. 2015, Table A1: the neighbour number
// is steered toward the input parameter NNBOPT; the lists come from the GPU
// regular-force pass of section 3.2.1).
//
// The rule is the uniform-density one: a sphere holding `count` bodies holds
// `target` when its volume is scaled by target/count, so rs2 scales by
// (target/count)^(2/3), clamped per step.  The 2/3 power is the cube root of
// q*q by eight Newton steps from a power-of-two start, using only IEEE-rounded
// + - * / and exact frexp/ldexp in a fixed order (the library is built without
// contraction), so the radii are reproducible bit for bit.
//
//  * nb_radius_update: next-step radii of a block from its neighbour counts
//    (one thread per row).
//  * nb_regular_force_fit: the regular force, then, while some row overflows
//    its list, those rows' radii are shrunk toward min(NNBOPT, nb_cap) and the
//    rows are recomputed: an ordered compaction of the overflowed rows (which
//    also rewrites their rs2 in place), a regular-force call on that sub-block,
//    and a scatter of its results back into the caller's outputs.
#include <cmath>

#include "nbreg.h"
#include "nb_internal.h"
#include "nb_runtime.h"

namespace nb {
namespace {

constexpr double kShrinkMin = 0.25;   // largest per-round shrink of an overflowed rs2
constexpr int kFitRows = 1024;        // rows per compaction work-group
constexpr int kFitRounds = kFitRows / kBlock;

__device__ __forceinline__ double pow23(double q)
{
    const double x = q * q;
    int e = 0;
    (void)frexp(x, &e);
    const int k = e >= 0 ? e / 3 : -((-e + 2) / 3);   // floor(e / 3)
    double y = ldexp(1.0, k);
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        const double t = y * y;
        y = y - (t * y - x) / (3.0 * t);
    }
    return y;
}

__global__ __launch_bounds__(kBlock) void radius_update_kernel(int32_t n_i,
                                                               const int32_t *count,
                                                               const double *rs2,
                                                               double nnbopt, double f_min,
                                                               double f_max, double *out)
{
    const int64_t b = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (b >= n_i) return;
    const double r = rs2[b];
    const int32_t c = count[b] > 1 ? count[b] : 1;
    const double f = fmin(fmax(pow23(nnbopt / (double)c), f_min), f_max);
    out[b] = r > 0.0 ? r * f : r;
}

// Per-work-group number of rows with count > cap; total accumulated.
__global__ __launch_bounds__(kBlock) void fit_count_kernel(int32_t n_i, const int32_t *count,
                                                           int32_t cap, int32_t *wgcnt,
                                                           int32_t *total)
{
    __shared__ int32_t part[kBlock / kWave];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    int32_t c = 0;
    for (int r = 0; r < kFitRounds; ++r) {
        const int64_t b = (int64_t)blockIdx.x * kFitRows + r * kBlock + threadIdx.x;
        c += __popcll(__ballot(b < n_i && count[b] > cap));
    }
    if (lane == 0) part[w] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t s = 0;
        for (int k = 0; k < kBlock / kWave; ++k) s += part[k];
        wgcnt[blockIdx.x] = s;
        if (s) atomicAdd(total, s);
    }
}

// Ordered compaction of the overflowed rows (ascending row index): sub-block
// rows, bodies and shrunk radii; the caller's rs2 of those rows is rewritten.
__global__ __launch_bounds__(kBlock) void fit_gather_kernel(
    int32_t n_i, const int32_t *count, int32_t cap, const int32_t *i_block, double *rs2,
    double target, const int32_t *wgcnt, int32_t *sub_rows, int32_t *sub_ib, double *sub_rs2)
{
    constexpr int W = kBlock / kWave;
    __shared__ int32_t grp[kFitRounds * W];
    __shared__ int32_t red[W];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    // rows in earlier work-groups
    int32_t before = 0;
    for (int32_t q = threadIdx.x; q < (int32_t)blockIdx.x; q += kBlock) before += wgcnt[q];
    for (int d = kWave / 2; d >= 1; d >>= 1) before += __shfl_xor(before, d);
    if (lane == 0) red[w] = before;
    bool flag[kFitRounds];
    int32_t rank[kFitRounds];
    for (int r = 0; r < kFitRounds; ++r) {
        const int64_t b = (int64_t)blockIdx.x * kFitRows + r * kBlock + threadIdx.x;
        flag[r] = b < n_i && count[b] > cap;
        const uint64_t m = __ballot(flag[r]);
        rank[r] = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                            __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
        if (lane == 0) grp[r * W + w] = __popcll(m);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t run = 0;
        for (int k = 0; k < W; ++k) run += red[k];
        for (int g = 0; g < kFitRounds * W; ++g) {
            const int32_t c = grp[g];
            grp[g] = run;
            run += c;
        }
    }
    __syncthreads();
    for (int r = 0; r < kFitRounds; ++r) {
        if (!flag[r]) continue;
        const int64_t b = (int64_t)blockIdx.x * kFitRows + r * kBlock + threadIdx.x;
        const int32_t k = grp[r * W + w] + rank[r];
        const double f = fmin(fmax(pow23(target / (double)count[b]), kShrinkMin), 1.0);
        const double nr = rs2[b] * f;
        rs2[b] = nr;
        sub_rows[k] = (int32_t)b;
        sub_ib[k] = i_block[b];
        sub_rs2[k] = nr;
    }
}

// One wave per sub-block row: results back into the block's rows.
__global__ __launch_bounds__(kBlock) void fit_scatter_kernel(
    int32_t n_sub, int32_t n_i, int32_t cap, const int32_t *sub_rows, const double *sub_acc,
    const double *sub_jerk, const int32_t *sub_cnt, const int32_t *sub_list,
    const int32_t *sub_ovf, double *acc, double *jerk, int32_t *nb_count, int32_t *nb_list,
    int32_t *overflow)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t k = (int64_t)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
    if (blockIdx.x == 0 && threadIdx.x == 0) *overflow = *sub_ovf;
    if (k >= n_sub) return;
    const int64_t b = sub_rows[k];
    const int32_t c = sub_cnt[k];
    const int32_t len = c < cap ? c : cap;
    for (int32_t q = lane; q < len; q += kWave) nb_list[b * cap + q] = sub_list[k * cap + q];
    if (lane < 3) {
        acc[lane * (int64_t)n_i + b] = sub_acc[lane * (int64_t)n_sub + k];
        jerk[lane * (int64_t)n_i + b] = sub_jerk[lane * (int64_t)n_sub + k];
    }
    if (lane == 0) nb_count[b] = c;
}

}  // namespace
}  // namespace nb

using namespace nbrt;

extern "C" {

int nb_radius_update(nb_ctx *ctx, int32_t n_i, const int32_t *nb_count, const double *rs2,
                     int32_t nnbopt, double f_min, double f_max, double *rs2_new)
{
    if (!ctx || n_i < 0 || nnbopt < 1 || !(f_min > 0.0) || !(f_max >= f_min) ||
        !std::isfinite(f_max))
        return NB_ERR_INVALID_ARG;
    if (n_i > 0 && (!nb_count || !rs2 || !rs2_new)) return NB_ERR_INVALID_ARG;
    if (!ctx->usable) return NB_ERR_UNSUPPORTED;
    if (n_i == 0) return NB_OK;
    hipEvent_t ev[2];
    hipError_t e = timed_begin(ctx, NB_CLASS_RADIUS, ev);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(nb::radius_update_kernel, dim3((unsigned)((n_i + nb::kBlock - 1) /
                                                                     nb::kBlock)),
                           dim3(nb::kBlock), 0, ctx->stream, n_i, nb_count, rs2,
                           (double)nnbopt, f_min, f_max, rs2_new);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = timed_end(ctx, NB_CLASS_RADIUS, ev);
    return e == hipSuccess ? NB_OK : hip_fail(ctx, e);
}

int nb_regular_force_fit(nb_ctx *ctx, int64_t n, const double *xp, const double *vp,
                         const double *m, int32_t n_i, const int32_t *i_block, double *rs2,
                         int32_t nb_cap, nb_precision prec, int32_t nnbopt, int32_t max_rounds,
                         double *acc, double *jerk, int32_t *nb_count, int32_t *nb_list,
                         int32_t *overflow, uint32_t *status, int32_t *rounds_host)
{
    if (!ctx || nb_cap < 1 || nnbopt < 1 || max_rounds < 0) return NB_ERR_INVALID_ARG;
    if (n_i > 0 && !nb_list) return NB_ERR_INVALID_ARG;
    int rc = nb_regular_force(ctx, n, xp, vp, m, n_i, i_block, rs2, nb_cap, prec, acc, jerk,
                              nb_count, nb_list, overflow, status);
    if (rc != NB_OK) return rc;
    int32_t rounds = 0;
    const double target = (double)std::min(nnbopt, nb_cap);
    const int32_t nblk = (n_i + nb::kFitRows - 1) / nb::kFitRows;
    while (n_i > 0 && rounds < max_rounds) {
        int32_t h_ovf = 0;
        hipError_t e = hipMemcpyAsync(&h_ovf, overflow, sizeof h_ovf, hipMemcpyDeviceToHost,
                                      ctx->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess) return hip_fail(ctx, e);
        if (!h_ovf) break;
        // 1. count the overflowed rows (per work-group, in scratch)
        rc = ensure_scratch(ctx, sizeof(int32_t) * ((size_t)nblk + 64));
        if (rc != NB_OK) return rc;
        int32_t *wgcnt = (int32_t *)ctx->scratch;
        int32_t *total = wgcnt + nblk;
        hipEvent_t ev[2];
        e = timed_begin(ctx, NB_CLASS_RADIUS, ev);
        if (e == hipSuccess) e = nb::launch_fill_i32(total, 0, 1, ctx->stream);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(nb::fit_count_kernel, dim3((unsigned)nblk), dim3(nb::kBlock), 0,
                               ctx->stream, n_i, nb_count, nb_cap, wgcnt, total);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = timed_end(ctx, NB_CLASS_RADIUS, ev);
        int32_t n_sub = 0;
        if (e == hipSuccess)
            e = hipMemcpyAsync(&n_sub, total, sizeof n_sub, hipMemcpyDeviceToHost, ctx->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess) return hip_fail(ctx, e);
        if (n_sub <= 0) break;
        // 2. sub-block arrays (aux) and the ordered compaction
        auto up = [](size_t b) { return (b + 255) / 256 * 256; };
        const size_t ns = (size_t)n_sub;
        const size_t o_rows = 0, o_ib = up(4 * ns), o_rs2 = o_ib + up(4 * ns);
        const size_t o_acc = o_rs2 + up(8 * ns), o_jerk = o_acc + up(24 * ns);
        const size_t o_cnt = o_jerk + up(24 * ns), o_ovf = o_cnt + up(4 * ns);
        const size_t o_list = o_ovf + 256, end = o_list + up(4 * ns * (size_t)nb_cap);
        rc = ensure_aux(ctx, end);
        if (rc != NB_OK) return rc;
        char *A = (char *)ctx->aux;
        int32_t *sub_rows = (int32_t *)(A + o_rows), *sub_ib = (int32_t *)(A + o_ib);
        double *sub_rs2 = (double *)(A + o_rs2), *sub_acc = (double *)(A + o_acc);
        double *sub_jerk = (double *)(A + o_jerk);
        int32_t *sub_cnt = (int32_t *)(A + o_cnt), *sub_ovf = (int32_t *)(A + o_ovf);
        int32_t *sub_list = (int32_t *)(A + o_list);
        e = timed_begin(ctx, NB_CLASS_RADIUS, ev);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(nb::fit_gather_kernel, dim3((unsigned)nblk), dim3(nb::kBlock), 0,
                               ctx->stream, n_i, nb_count, nb_cap, i_block, rs2, target, wgcnt,
                               sub_rows, sub_ib, sub_rs2);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = timed_end(ctx, NB_CLASS_RADIUS, ev);
        if (e != hipSuccess) return hip_fail(ctx, e);
        // 3. recompute the sub-block (may regrow scratch: wgcnt is consumed)
        rc = nb_regular_force(ctx, n, xp, vp, m, n_sub, sub_ib, sub_rs2, nb_cap, prec, sub_acc,
                              sub_jerk, sub_cnt, sub_list, sub_ovf, status);
        if (rc != NB_OK) return rc;
        // 4. results back into the block
        e = timed_begin(ctx, NB_CLASS_RADIUS, ev);
        if (e == hipSuccess) {
            const unsigned g = (unsigned)((n_sub + nb::kBlock / nb::kWave - 1) /
                                          (nb::kBlock / nb::kWave));
            hipLaunchKernelGGL(nb::fit_scatter_kernel, dim3(g), dim3(nb::kBlock), 0,
                               ctx->stream, n_sub, n_i, nb_cap, sub_rows, sub_acc, sub_jerk,
                               sub_cnt, sub_list, sub_ovf, acc, jerk, nb_count, nb_list,
                               overflow);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = timed_end(ctx, NB_CLASS_RADIUS, ev);
        if (e != hipSuccess) return hip_fail(ctx, e);
        ++rounds;
    }
    if (rounds_host) *rounds_host = rounds;
    return NB_OK;
}

}  // extern "C"
