// The rest of an Ahmad-Cohen block step around the regular force (Wang et al.
// 2015, section 2; Table 1 "Irr." and "Adjust"):
//  * irregular force + jerk over each row's neighbour list (the bodies inside
//    the neighbour radius, section 2), FP64, one wave per row with the list
//    spread over the lanes; gathers from the SoA planes, or for large blocks
//    from a packed copy of the bodies (one cache line per neighbour);
//  * the fourth-order Hermite corrector of the integrator (section 2), FP64,
//    one thread per entry, with the second and third force derivatives from
//    the cubic Hermite interpolant (used by step-size criteria);
//  * the O(N^2) potential (section 3.2.1 and the energy check / scaling of
//    section 3.3.2), FP64, one body per lane with j-tiles in LDS, and a
//    fixed-order reduction of the total potential energy.
#include "nbreg.h"
#include "nb_rows.h"
#include "nb_runtime.h"

namespace nb {
namespace {

// Where the irregular force reads neighbour bodies from: the SoA planes
// (seven cache lines per neighbour) or a packed copy with one 64-byte record
// per body {x, y, z, m | vx, vy, vz, 0} (one line per neighbour).
struct SoaBodies {
    const double *xp, *vp, *m;
    int64_t n;
    __device__ __forceinline__ void load(int64_t j, double &x, double &y, double &z, double &vx,
                                         double &vy, double &vz, double &mj) const
    {
        x = xp[j];
        y = xp[n + j];
        z = xp[2 * n + j];
        vx = vp[j];
        vy = vp[n + j];
        vz = vp[2 * n + j];
        mj = m[j];
    }
};

struct PackedBodies {
    const double4 *p;
    __device__ __forceinline__ void load(int64_t j, double &x, double &y, double &z, double &vx,
                                         double &vy, double &vz, double &mj) const
    {
        const double4 a = p[2 * j], b = p[2 * j + 1];
        x = a.x;
        y = a.y;
        z = a.z;
        mj = a.w;
        vx = b.x;
        vy = b.y;
        vz = b.z;
    }
};

__global__ __launch_bounds__(256) void pack_bodies_kernel(int64_t n, const double *xp,
                                                          const double *vp, const double *m,
                                                          double4 *out)
{
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * blockDim.x) {
        out[2 * j] = make_double4(xp[j], xp[n + j], xp[2 * n + j], m[j]);
        out[2 * j + 1] = make_double4(vp[j], vp[n + j], vp[2 * n + j], 0.0);
    }
}

// r^-1 for the potential: the hardware estimate (measured 2^-24.2 relative
// error on gfx950) and one Newton step (measured 2^-47.8, 4.2e-15).  The
// potential's terms all have one sign, so this bound carries over to the sum;
// the force and jerk sums, whose terms cancel, keep the third-order step of
// rsqrt_f64.
__device__ __forceinline__ double rsqrt_newton_f64(double r2)
{
    const double y = __builtin_amdgcn_rsq(r2);
    const double t = r2 * y;
    const double e = __builtin_fma(-t, y, 1.0);
    return __builtin_fma(y * e, 0.5, y);
}

template <class Bodies>
__global__ __launch_bounds__(kBlock) void irregular_kernel(int64_t n, const double *xp,
                                                           const double *vp, Bodies B,
                                                           int32_t n_i, const int32_t *i_block,
                                                           int32_t cap, const int32_t *nb_count,
                                                           const int32_t *nb_list, double *acc,
                                                           double *jerk, uint32_t *status)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t b = (int64_t)blockIdx.x * (kBlock / kWave) +
                      __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    if (b >= n_i) return;
    const int64_t i = i_block[b];
    bool bad = i < 0 || i >= n;
    double ax = 0, ay = 0, az = 0, jx = 0, jy = 0, jz = 0;
    if (!bad) {
        const double xi = xp[i], yi = xp[n + i], zi = xp[2 * n + i];
        const double vxi = vp[i], vyi = vp[n + i], vzi = vp[2 * n + i];
        const int32_t c = nb_count[b];
        const int32_t k = c < cap ? c : cap;
        for (int32_t q = lane; q < k; q += kWave) {
            const int64_t j = nb_list[b * (int64_t)cap + q];
            if (j < 0 || j >= n || j == i) {
                bad = true;
                continue;
            }
            double x, y, z, vx, vy, vz, mj;
            B.load(j, x, y, z, vx, vy, vz, mj);
            add_term_f64(ax, ay, az, jx, jy, jz, x - xi, y - yi, z - zi, vx - vxi, vy - vyi,
                         vz - vzi, mj);
        }
    }
    double r[6] = {ax, ay, az, jx, jy, jz};
    group_sums<kWave, 6>(r);
    ax = r[0];
    ay = r[1];
    az = r[2];
    jx = r[3];
    jy = r[4];
    jz = r[5];
    const bool nonfin = !finite6(ax, ay, az, jx, jy, jz);
    const uint64_t bb = __ballot(bad);
    if (lane == 0) {
        acc[b] = ax;
        acc[n_i + b] = ay;
        acc[2 * (int64_t)n_i + b] = az;
        jerk[b] = jx;
        jerk[n_i + b] = jy;
        jerk[2 * (int64_t)n_i + b] = jz;
        if (status && (bb || nonfin))
            atomicOr(status, (bb ? kStBadIndex : 0u) | (nonfin ? kStNonFinite : 0u));
    }
}

// Fourth-order Hermite corrector, the textbook two-point form, evaluated in
// the same operation order as its plain definition:
//   v1 = v0 + h/2 (a0 + a1) + h^2/12 (j0 - j1)
//   x1 = x0 + h/2 (v0 + v1) + h^2/12 (a0 - a1)
//   a3 = (12 (a0 - a1) + 6 h (j0 + j1)) / h^3
//   a2 = (-6 (a0 - a1) - h (4 j0 + 2 j1)) / h^2 + h a3     (at the step end)
__global__ __launch_bounds__(256) void corrector_kernel(int64_t n, const double *h,
                                                       const double *x0, const double *v0,
                                                       const double *a0, const double *j0,
                                                       const double *a1, const double *j1,
                                                       double *x1, double *v1, double *a2,
                                                       double *a3)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double dt = h[i];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int64_t q = (int64_t)k * n + i;
            const double A0 = a0[q], A1 = a1[q], J0 = j0[q], J1 = j1[q], V0 = v0[q];
            const double vn = V0 + dt / 2 * (A0 + A1) + dt * dt / 12 * (J0 - J1);
            const double xn = x0[q] + dt / 2 * (V0 + vn) + dt * dt / 12 * (A0 - A1);
            const double s0 = (-6 * (A0 - A1) - dt * (4 * J0 + 2 * J1)) / (dt * dt);
            const double c = (12 * (A0 - A1) + 6 * dt * (J0 + J1)) / (dt * dt * dt);
            v1[q] = vn;
            x1[q] = xn;
            a2[q] = s0 + dt * c;
            a3[q] = c;
        }
    }
}

struct alignas(16) PBody {
    double x, y, z, m;
};

// phi_i = -sum_{j != i} m_j / |x_j - x_i|.  grid = (ceil(n / kBlock), splits);
// split s writes partial phi to part[s][n] (or phi directly when splits == 1).
__global__ __launch_bounds__(kBlock) void potential_kernel(int64_t n, const double *x,
                                                           const double *m, int32_t splits,
                                                           int64_t split_len, double *out)
{
    __shared__ PBody tile[2][kTile];
    const int tid = threadIdx.x;
    const int32_t split = blockIdx.y;
    const int64_t j0 = (int64_t)split * split_len;
    const int64_t j1 = j0 + split_len < n ? j0 + split_len : n;
    const int64_t i = (int64_t)blockIdx.x * kBlock + tid;
    double xi = kFar * 0.5, yi = kFar * 0.5, zi = kFar * 0.5;
    if (i < n) {
        xi = x[i];
        yi = x[n + i];
        zi = x[2 * n + i];
    }
    double phi = 0.0;
    const int64_t ntiles = j1 > j0 ? (j1 - j0 + kTile - 1) / kTile : 0;
    PBody nxt;
    auto load = [&](int64_t j) {
        if (j < j1) {
            nxt.x = x[j];
            nxt.y = x[n + j];
            nxt.z = x[2 * n + j];
            nxt.m = m[j];
        } else {
            nxt.x = nxt.y = nxt.z = kFar;
            nxt.m = 0.0;
        }
    };
    if (ntiles > 0) {
        load(j0 + tid);
        tile[0][tid] = nxt;
    }
    __syncthreads();
    for (int64_t t = 0; t < ntiles; ++t) {
        const int cur = (int)(t & 1);
        const int64_t tbase = j0 + t * kTile;
        if (t + 1 < ntiles) load(tbase + kTile + tid);
        const PBody *buf = tile[cur];
        // only a tile that overlaps this work-group's own rows can hold a
        // lane's self pair (uniform per work-group)
        const int64_t row0 = (int64_t)blockIdx.x * kBlock;
        if (tbase < row0 + kBlock && row0 < tbase + kTile) {
#pragma unroll 4
            for (int jj = 0; jj < kTile; ++jj) {
                const PBody &J = buf[jj];
                const double dx = J.x - xi, dy = J.y - yi, dz = J.z - zi;
                const double r2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
                double y = rsqrt_newton_f64(r2);
                y = (tbase + jj == i) ? 0.0 : y;
                phi = __builtin_fma(-J.m, y, phi);
            }
        } else {
#pragma unroll 4
            for (int jj = 0; jj < kTile; ++jj) {
                const PBody &J = buf[jj];
                const double dx = J.x - xi, dy = J.y - yi, dz = J.z - zi;
                const double r2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
                phi = __builtin_fma(-J.m, rsqrt_newton_f64(r2), phi);
            }
        }
        if (t + 1 < ntiles) tile[cur ^ 1][tid] = nxt;
        __syncthreads();
    }
    if (i < n) out[(int64_t)split * n + i] = phi;
}

// Sums split partials (fixed order) into phi and forms m_i phi_i / 2 per
// body; then a fixed-shape tree reduction of those into one value per
// work-group, and a final single-work-group pass.
__global__ __launch_bounds__(256) void potential_reduce(int64_t n, const double *m,
                                                        int32_t splits, const double *part,
                                                        double *phi, double *wg_sum)
{
    __shared__ double red[256];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double e = 0.0;
    if (i < n) {
        double p = 0.0;
        for (int32_t s = 0; s < splits; ++s) p += part[(int64_t)s * n + i];
        phi[i] = p;
        e = 0.5 * m[i] * p;
    }
    red[threadIdx.x] = e;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) wg_sum[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void sum_kernel(int64_t count, const double *v, double *out)
{
    __shared__ double red[256];
    double s = 0.0;
    for (int64_t k = threadIdx.x; k < count; k += 256) s += v[k];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

}  // namespace
}  // namespace nb

using namespace nbrt;

extern "C" {

int nb_irregular_force(nb_ctx *ctx, int64_t n, const double *xp, const double *vp,
                       const double *m, int32_t n_i, const int32_t *i_block, int32_t nb_cap,
                       const int32_t *nb_count, const int32_t *nb_list, double *acc,
                       double *jerk, uint32_t *status)
{
    if (!ctx || n <= 0 || n > INT32_MAX || n_i < 0 || nb_cap < 0) return NB_ERR_INVALID_ARG;
    if (!xp || !vp || !m) return NB_ERR_INVALID_ARG;
    if (n_i > 0 && (!i_block || !nb_count || !acc || !jerk)) return NB_ERR_INVALID_ARG;
    if (n_i > 0 && nb_cap > 0 && !nb_list) return NB_ERR_INVALID_ARG;
    if (!ctx->usable) return NB_ERR_UNSUPPORTED;
    if (n_i == 0) return NB_OK;
    const int per = nb::kBlock / nb::kWave;
    const dim3 grid((unsigned)((n_i + per - 1) / per));
    // large blocks gather many neighbours per body: pack the bodies once into
    // 64-byte records (one cache line per gather instead of seven)
    const bool pack = (int64_t)n_i * 128 >= n;
    if (pack) {
        const int rc = ensure_scratch(ctx, (size_t)n * 2 * sizeof(double4));
        if (rc != NB_OK) return rc;
    }
    hipEvent_t ev[2];
    hipError_t e = timed_begin(ctx, NB_CLASS_STEP, ev);
    if (e == hipSuccess && pack) {
        double4 *packed = (double4 *)ctx->scratch;
        const unsigned pg = (unsigned)std::min<int64_t>(8192, (n + 255) / 256);
        hipLaunchKernelGGL(nb::pack_bodies_kernel, dim3(pg), dim3(256), 0, ctx->stream, n, xp, vp,
                           m, packed);
        hipLaunchKernelGGL(nb::irregular_kernel<nb::PackedBodies>, grid, dim3(nb::kBlock), 0,
                           ctx->stream, n, xp, vp, nb::PackedBodies{packed}, n_i, i_block,
                           nb_cap, nb_count, nb_list, acc, jerk, status);
        e = hipGetLastError();
    } else if (e == hipSuccess) {
        hipLaunchKernelGGL(nb::irregular_kernel<nb::SoaBodies>, grid, dim3(nb::kBlock), 0,
                           ctx->stream, n, xp, vp, nb::SoaBodies{xp, vp, m, n}, n_i, i_block,
                           nb_cap, nb_count, nb_list, acc, jerk, status);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = timed_end(ctx, NB_CLASS_STEP, ev);
    return e == hipSuccess ? NB_OK : hip_fail(ctx, e);
}

int nb_hermite_correct(nb_ctx *ctx, int64_t n, const double *h, const double *x0,
                       const double *v0, const double *a0, const double *j0, const double *a1,
                       const double *j1, double *x1, double *v1, double *a2, double *a3)
{
    if (!ctx || n <= 0 || n > INT32_MAX) return NB_ERR_INVALID_ARG;
    if (!h || !x0 || !v0 || !a0 || !j0 || !a1 || !j1 || !x1 || !v1 || !a2 || !a3)
        return NB_ERR_INVALID_ARG;
    if (!ctx->usable) return NB_ERR_UNSUPPORTED;
    const int64_t want = (n + 255) / 256;
    const unsigned grid = (unsigned)(want < 65536 ? want : 65536);
    hipEvent_t ev[2];
    hipError_t e = timed_begin(ctx, NB_CLASS_STEP, ev);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(nb::corrector_kernel, dim3(grid), dim3(256), 0, ctx->stream, n, h, x0,
                           v0, a0, j0, a1, j1, x1, v1, a2, a3);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = timed_end(ctx, NB_CLASS_STEP, ev);
    return e == hipSuccess ? NB_OK : hip_fail(ctx, e);
}

int nb_potential(nb_ctx *ctx, int64_t n, const double *x, const double *m, double *phi,
                 double *energy)
{
    if (!ctx || n <= 0 || n > INT32_MAX || !x || !m || !phi) return NB_ERR_INVALID_ARG;
    if (!ctx->usable) return NB_ERR_UNSUPPORTED;
    const int cus = ctx->cu_count > 0 ? ctx->cu_count : 256;
    const int64_t wgs = (n + nb::kBlock - 1) / nb::kBlock;
    int64_t splits = std::max<int64_t>(1, std::min<int64_t>((cus * 64 + wgs - 1) / wgs,
                                                             std::max<int64_t>(1, n / 2048)));
    const int64_t tiles = (n + nb::kTile - 1) / nb::kTile;
    const int64_t split_len = (tiles + splits - 1) / splits * nb::kTile;
    splits = (n + split_len - 1) / split_len;
    const int64_t red_wgs = (n + 255) / 256;
    const size_t bytes = (size_t)(splits * n + red_wgs + 1) * sizeof(double) + 512;
    int rc = ensure_scratch(ctx, bytes);
    if (rc != NB_OK) return rc;
    double *part = (double *)ctx->scratch;
    double *wg = part + splits * n;
    double *tot = wg + red_wgs;
    hipEvent_t ev[2];
    hipError_t e = timed_begin(ctx, NB_CLASS_STEP, ev);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(nb::potential_kernel, dim3((unsigned)wgs, (unsigned)splits),
                           dim3(nb::kBlock), 0, ctx->stream, n, x, m, (int32_t)splits, split_len,
                           part);
        hipLaunchKernelGGL(nb::potential_reduce, dim3((unsigned)red_wgs), dim3(256), 0,
                           ctx->stream, n, m, (int32_t)splits, part, phi, wg);
        hipLaunchKernelGGL(nb::sum_kernel, dim3(1), dim3(256), 0, ctx->stream, red_wgs, wg,
                           energy ? energy : tot);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = timed_end(ctx, NB_CLASS_STEP, ev);
    return e == hipSuccess ? NB_OK : hip_fail(ctx, e);
}

}  // extern "C"
