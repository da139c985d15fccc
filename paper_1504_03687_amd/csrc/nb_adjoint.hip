// Adjoint of the regular force (no counterpart in the paper; it differentiates
// the regular force of section 2 / section 3.2.1 with the neighbour sets held
// fixed).
//
//   L = sum_b  w_a[:,b] . acc_b + w_j[:,b] . jerk_b
//
// For a regular pair (row b with body i, source j), with A = w_a[:,b],
// B = w_j[:,b], r = x_j - x_i, u = v_j - v_i, s = r.u, R3 = |r|^-3,
// R5 = |r|^-5, R7 = |r|^-7:
//   dL/dm_j += (A.r) R3 + (B.u) R3 - 3 s (B.r) R5
//   g_r      = m_j [ A R3 - 3 R5 (s B + (B.r) u) + r (15 s (B.r) R7 - 3 R5 (A.r + B.u)) ]
//   g_u      = m_j [ B R3 - 3 (B.r) R5 r ]
//   dL/dx_j += g_r,  dL/dx_i -= g_r,  dL/dv_j += g_u,  dL/dv_i -= g_u.
//
// Two recompute passes, FP64, no per-pair storage and no atomics:
//  * row pass: one row per lane, j-tiles through LDS; sums g_r and g_u over j
//    (the per-row "-" terms).  The row-constant factors A and B are applied
//    once at the end: sum_j g_r = A sum(m R3) - 3 B sum(m R5 s) + ...
//  * body pass: one body j per lane, row tiles through LDS; sums the "+"
//    terms and dL/dm_j over all rows, and subtracts the row pass result of
//    every row whose body is j, in row order.
// Both passes may split their loop range; partials are reduced in a fixed
// order, so results are bitwise deterministic.
#include "nb_internal.h"
#include "nb_pair.h"

namespace nb {
namespace {

constexpr int kRowTile = 128;   // rows staged per LDS tile in the body pass

struct alignas(16) JB {
    double x, y, z, m;
    double vx, vy, vz, pad;
};

struct alignas(16) RB {
    double x, y, z, vx, vy, vz;
    double ax, ay, az, bx, by, bz;
    double hi;
    float rs2f;
    int32_t i;
    int32_t b;
    int32_t pad;
};

struct AdjPlan {
    int32_t row_splits;
    int64_t row_split_len;   // j per split in the row pass
    int32_t body_splits;
    int64_t body_split_len;  // rows per split in the body pass
    double *row_partial;     // [row_splits][6][n_i]
    double *body_partial;    // [body_splits][7][n]
};

__device__ __forceinline__ void load_jb(JB &J, const AdjointArgs &a, int64_t j, int64_t j1)
{
    if (j < j1) {
        J.x = a.xp[j];
        J.y = a.xp[a.n + j];
        J.z = a.xp[2 * a.n + j];
        J.vx = a.vp[j];
        J.vy = a.vp[a.n + j];
        J.vz = a.vp[2 * a.n + j];
        J.m = a.m[j];
    } else {
        J.x = J.y = J.z = kFar;
        J.vx = J.vy = J.vz = 0.0;
        J.m = 0.0;
    }
    J.pad = 0.0;
}

// Exclusion (self pair or neighbour) by the canonical test, run only for
// candidates below the FP64 bound hi.
__device__ __forceinline__ bool excluded(double dx, double dy, double dz, double r2, double hi,
                                         float rs2f, int32_t jidx, int32_t i)
{
    bool excl = false;
    if (r2 < hi) {
        double ex = dx, ey = dy, ez = dz;
        int32_t jj = jidx;
        opaque(ex, ey, ez);
        opaque(jj);
        excl = jj == i || canon_r2f(ex, ey, ez) < rs2f;
    }
    return excl;
}

// ---------------------------------------------------------------------------
// Row pass.  grid = (ceil(n_i / kBlock), row_splits).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void adj_rows_kernel(AdjointArgs a, AdjPlan p)
{
    __shared__ JB tile[2][kTile];
    const int tid = threadIdx.x;
    const int32_t split = blockIdx.y;
    const int64_t j0 = (int64_t)split * p.row_split_len;
    const int64_t j1 = j0 + p.row_split_len < a.n ? j0 + p.row_split_len : a.n;
    const int64_t b = (int64_t)blockIdx.x * kBlock + tid;

    double xi = kFar * 0.5, yi = kFar * 0.5, zi = kFar * 0.5, vxi = 0, vyi = 0, vzi = 0;
    double Ax = 0, Ay = 0, Az = 0, Bx = 0, By = 0, Bz = 0, hi = -1.0;
    float rs2f = -1.0f;
    int32_t i = -1;
    if (b < a.n_i) {
        const int64_t ii = a.i_block[b];
        if (ii >= 0 && ii < a.n) {
            i = (int32_t)ii;
            xi = a.xp[ii];
            yi = a.xp[a.n + ii];
            zi = a.xp[2 * a.n + ii];
            vxi = a.vp[ii];
            vyi = a.vp[a.n + ii];
            vzi = a.vp[2 * a.n + ii];
            Ax = a.w_a[b];
            Ay = a.w_a[a.n_i + b];
            Az = a.w_a[2 * (int64_t)a.n_i + b];
            Bx = a.w_j[b];
            By = a.w_j[a.n_i + b];
            Bz = a.w_j[2 * (int64_t)a.n_i + b];
            rs2f = (float)a.rs2[b];
            hi = cand_bound_f64(rs2f);
        }
    }
    // With k5 = m R5 and t = k5 (B.r):
    //   sum_j g_r = A C1 - 3 (B C2 + H),  sum_j g_u = B C1 - 3 U,
    //   C1 = sum m R3,  C2 = sum k5 s,  U = sum t r,
    //   H = sum [t u + k5 ((A.r + B.u) - 5 s (B.r) |r|^-2) r];
    // the factor -3 is applied once per row.
    double C1 = 0, C2 = 0, Hx = 0, Hy = 0, Hz = 0, Ux = 0, Uy = 0, Uz = 0;

    // Each tile is loaded when the work-group reaches it, into the buffer
    // last read for tile t-2 (every wave has passed tile t-1's barrier since):
    // one barrier per tile and no registers held across the pair loop.
    const int64_t ntiles = j1 > j0 ? (j1 - j0 + kTile - 1) / kTile : 0;
    for (int64_t t = 0; t < ntiles; ++t) {
        const int cur = (int)(t & 1);
        const int64_t tbase = j0 + t * kTile;
        {
            JB J;
            load_jb(J, a, tbase + tid, j1);
            tile[cur][tid] = J;
        }
        __syncthreads();
        const JB *buf = tile[cur];
#pragma unroll 2
        for (int jj = 0; jj < kTile; ++jj) {
            const JB &J = buf[jj];
            const double dx = J.x - xi, dy = J.y - yi, dz = J.z - zi;
            const double r2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
            const bool excl = excluded(dx, dy, dz, r2, hi, rs2f, (int32_t)(tbase + jj), i);
            const double ux = J.vx - vxi, uy = J.vy - vyi, uz = J.vz - vzi;
            double y = rsqrt_f64(r2);
            y = excl ? 0.0 : y;
            const double y2 = y * y;
            const double R3 = y * y2, R5 = R3 * y2;
            const double s = __builtin_fma(dz, uz, __builtin_fma(dy, uy, dx * ux));
            const double Ar = __builtin_fma(Az, dz, __builtin_fma(Ay, dy, Ax * dx));
            const double Br = __builtin_fma(Bz, dz, __builtin_fma(By, dy, Bx * dx));
            const double Bu = __builtin_fma(Bz, uz, __builtin_fma(By, uy, Bx * ux));
            const double m = J.m;
            const double k5 = m * R5;
            const double tb = k5 * Br;
            const double c = k5 * __builtin_fma(-5.0 * (s * Br), y2, Ar + Bu);
            C1 = __builtin_fma(m, R3, C1);
            C2 = __builtin_fma(k5, s, C2);
            Hx = __builtin_fma(tb, ux, __builtin_fma(c, dx, Hx));
            Hy = __builtin_fma(tb, uy, __builtin_fma(c, dy, Hy));
            Hz = __builtin_fma(tb, uz, __builtin_fma(c, dz, Hz));
            Ux = __builtin_fma(tb, dx, Ux);
            Uy = __builtin_fma(tb, dy, Uy);
            Uz = __builtin_fma(tb, dz, Uz);
        }
    }
    if (b < a.n_i) {
        double *o = p.row_partial + (int64_t)split * 6 * a.n_i + b;
        o[0] = __builtin_fma(Ax, C1, -3.0 * __builtin_fma(Bx, C2, Hx));
        o[a.n_i] = __builtin_fma(Ay, C1, -3.0 * __builtin_fma(By, C2, Hy));
        o[2 * (int64_t)a.n_i] = __builtin_fma(Az, C1, -3.0 * __builtin_fma(Bz, C2, Hz));
        o[3 * (int64_t)a.n_i] = __builtin_fma(Bx, C1, -3.0 * Ux);
        o[4 * (int64_t)a.n_i] = __builtin_fma(By, C1, -3.0 * Uy);
        o[5 * (int64_t)a.n_i] = __builtin_fma(Bz, C1, -3.0 * Uz);
    }
}

// Sums the row-pass partials over splits (fixed order) into row_part[6][n_i].
__global__ void adj_rows_reduce(AdjointArgs a, AdjPlan p)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = 6 * (int64_t)a.n_i;
    if (k >= total) return;
    double s = 0.0;
    for (int32_t q = 0; q < p.row_splits; ++q) s += p.row_partial[(int64_t)q * total + k];
    a.row_part[k] = s;
}

// ---------------------------------------------------------------------------
// Body pass.  grid = (ceil(n / kBlock), body_splits); split q covers rows
// [q * body_split_len, ...).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void load_rb(RB &R, const AdjointArgs &a, int64_t b, int64_t b1)
{
    R.x = R.y = R.z = kFar * 0.5;
    R.vx = R.vy = R.vz = 0.0;
    R.ax = R.ay = R.az = R.bx = R.by = R.bz = 0.0;
    R.hi = -1.0;
    R.rs2f = -1.0f;
    R.i = -1;
    R.b = (int32_t)b;
    R.pad = 0;
    if (b >= b1) return;
    const int64_t i = a.i_block[b];
    if (i < 0 || i >= a.n) return;
    R.i = (int32_t)i;
    R.x = a.xp[i];
    R.y = a.xp[a.n + i];
    R.z = a.xp[2 * a.n + i];
    R.vx = a.vp[i];
    R.vy = a.vp[a.n + i];
    R.vz = a.vp[2 * a.n + i];
    R.ax = a.w_a[b];
    R.ay = a.w_a[a.n_i + b];
    R.az = a.w_a[2 * (int64_t)a.n_i + b];
    R.bx = a.w_j[b];
    R.by = a.w_j[a.n_i + b];
    R.bz = a.w_j[2 * (int64_t)a.n_i + b];
    R.rs2f = (float)a.rs2[b];
    R.hi = cand_bound_f64(R.rs2f);
}

__global__ __launch_bounds__(kBlock) void adj_bodies_kernel(AdjointArgs a, AdjPlan p)
{
    __shared__ RB tile[2][kRowTile];
    const int tid = threadIdx.x;
    const int32_t split = blockIdx.y;
    const int64_t b0 = (int64_t)split * p.body_split_len;
    const int64_t b1 = b0 + p.body_split_len < a.n_i ? b0 + p.body_split_len : a.n_i;
    const int64_t j = (int64_t)blockIdx.x * kBlock + tid;
    const bool live = j < a.n;

    double xj = kFar, yj = kFar, zj = kFar, vxj = 0, vyj = 0, vzj = 0, mj = 0;
    if (live) {
        xj = a.xp[j];
        yj = a.xp[a.n + j];
        zj = a.xp[2 * a.n + j];
        vxj = a.vp[j];
        vyj = a.vp[a.n + j];
        vzj = a.vp[2 * a.n + j];
        mj = a.m[j];
    }
    const int32_t jidx = live ? (int32_t)j : -2;
    // The body's own mass and the factor -3 are applied once per body:
    //   dL/dx_j = m_j (GA - 3 GB) - D_x,  dL/dv_j = m_j (UA - 3 UB) - D_v,
    //   dL/dm_j = MA - 3 MB,
    // GA = sum R3 A, GB = sum [R5 s B + R5 (B.r) u + R5 ((A.r + B.u) - 5 s (B.r) |r|^-2) r],
    // UA = sum R3 B, UB = sum R5 (B.r) r, MA = sum (A.r + B.u) R3, MB = sum s (B.r) R5,
    // and D the row-pass sums of the rows whose body is j (in row order).
    double GAx = 0, GAy = 0, GAz = 0, GBx = 0, GBy = 0, GBz = 0;
    double UAx = 0, UAy = 0, UAz = 0, UBx = 0, UBy = 0, UBz = 0, MA = 0, MB = 0;
    double Dx = 0, Dy = 0, Dz = 0, Dux = 0, Duy = 0, Duz = 0;

    // row tiles are loaded as in the row pass: when reached, into the buffer
    // last read two tiles ago, one barrier per tile
    const int64_t ntiles = b1 > b0 ? (b1 - b0 + kRowTile - 1) / kRowTile : 0;
    for (int64_t t = 0; t < ntiles; ++t) {
        const int cur = (int)(t & 1);
        const int64_t tbase = b0 + t * kRowTile;
        if (tid < kRowTile) {
            RB R;
            load_rb(R, a, tbase + tid, b1);
            tile[cur][tid] = R;
        }
        __syncthreads();
        const RB *buf = tile[cur];
#pragma unroll 1
        for (int q = 0; q < kRowTile; ++q) {
            const RB &R = buf[q];
            const double dx = xj - R.x, dy = yj - R.y, dz = zj - R.z;
            const double r2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
            const bool excl = excluded(dx, dy, dz, r2, R.hi, R.rs2f, jidx, R.i);
            const double ux = vxj - R.vx, uy = vyj - R.vy, uz = vzj - R.vz;
            double y = rsqrt_f64(r2);
            y = excl ? 0.0 : y;
            const double y2 = y * y;
            const double R3 = y * y2, R5 = R3 * y2;
            const double s = __builtin_fma(dz, uz, __builtin_fma(dy, uy, dx * ux));
            const double Ar = __builtin_fma(R.az, dz, __builtin_fma(R.ay, dy, R.ax * dx));
            const double Br = __builtin_fma(R.bz, dz, __builtin_fma(R.by, dy, R.bx * dx));
            const double Bu = __builtin_fma(R.bz, uz, __builtin_fma(R.by, uy, R.bx * ux));
            const double AB = Ar + Bu;
            const double sBr = s * Br;
            MA = __builtin_fma(AB, R3, MA);
            MB = __builtin_fma(sBr, R5, MB);
            const double R5s = R5 * s;
            const double R5Br = R5 * Br;
            const double cr = R5 * __builtin_fma(-5.0 * sBr, y2, AB);
            GAx = __builtin_fma(R3, R.ax, GAx);
            GAy = __builtin_fma(R3, R.ay, GAy);
            GAz = __builtin_fma(R3, R.az, GAz);
            GBx = __builtin_fma(R5s, R.bx, __builtin_fma(R5Br, ux, __builtin_fma(cr, dx, GBx)));
            GBy = __builtin_fma(R5s, R.by, __builtin_fma(R5Br, uy, __builtin_fma(cr, dy, GBy)));
            GBz = __builtin_fma(R5s, R.bz, __builtin_fma(R5Br, uz, __builtin_fma(cr, dz, GBz)));
            UAx = __builtin_fma(R3, R.bx, UAx);
            UAy = __builtin_fma(R3, R.by, UAy);
            UAz = __builtin_fma(R3, R.bz, UAz);
            UBx = __builtin_fma(R5Br, dx, UBx);
            UBy = __builtin_fma(R5Br, dy, UBy);
            UBz = __builtin_fma(R5Br, dz, UBz);
            // this body is the row's own body: subtract the row pass sum
            int32_t ri = R.i;
            if (ri == jidx) {
                opaque(ri);
                const double *rp = a.row_part + R.b;
                Dx += rp[0];
                Dy += rp[a.n_i];
                Dz += rp[2 * (int64_t)a.n_i];
                Dux += rp[3 * (int64_t)a.n_i];
                Duy += rp[4 * (int64_t)a.n_i];
                Duz += rp[5 * (int64_t)a.n_i];
            }
        }
    }
    if (live) {
        double *o = p.body_partial + (int64_t)split * 7 * a.n + j;
        o[0] = mj * __builtin_fma(-3.0, GBx, GAx) - Dx;
        o[a.n] = mj * __builtin_fma(-3.0, GBy, GAy) - Dy;
        o[2 * a.n] = mj * __builtin_fma(-3.0, GBz, GAz) - Dz;
        o[3 * a.n] = mj * __builtin_fma(-3.0, UBx, UAx) - Dux;
        o[4 * a.n] = mj * __builtin_fma(-3.0, UBy, UAy) - Duy;
        o[5 * a.n] = mj * __builtin_fma(-3.0, UBz, UAz) - Duz;
        o[6 * a.n] = __builtin_fma(-3.0, MB, MA);
    }
}

// Sums the body-pass partials (fixed order) into gx, gv, gm; flags bad
// indices and non-finite results.
__global__ void adj_bodies_reduce(AdjointArgs a, AdjPlan p)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool nonfin = false;
    if (j < a.n) {
        double v[7] = {0, 0, 0, 0, 0, 0, 0};
        for (int32_t q = 0; q < p.body_splits; ++q) {
            const double *src = p.body_partial + (int64_t)q * 7 * a.n + j;
#pragma unroll
            for (int k = 0; k < 7; ++k) v[k] += src[(int64_t)k * a.n];
        }
        a.gx[j] = v[0];
        a.gx[a.n + j] = v[1];
        a.gx[2 * a.n + j] = v[2];
        a.gv[j] = v[3];
        a.gv[a.n + j] = v[4];
        a.gv[2 * a.n + j] = v[5];
        a.gm[j] = v[6];
        nonfin = !finite6(v[0], v[1], v[2], v[3], v[4], v[5]) || !__builtin_isfinite(v[6]);
    }
    bool bad = false;
    for (int64_t b = j; b < a.n_i; b += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = a.i_block[b];
        bad |= i < 0 || i >= a.n;
    }
    const uint64_t f = __ballot(nonfin), bb = __ballot(bad);
    if ((threadIdx.x & (kWave - 1)) == 0 && (f | bb) && a.status)
        atomicOr(a.status, (f ? kStNonFinite : 0u) | (bb ? kStBadIndex : 0u));
}

}  // namespace

size_t adjoint_scratch_bytes(int64_t n, int32_t n_i, int row_splits, int body_splits)
{
    return (size_t)row_splits * 6 * n_i * sizeof(double) + 6 * (size_t)n_i * sizeof(double) +
           (size_t)body_splits * 7 * n * sizeof(double) + 3 * 256;
}

hipError_t launch_adjoint_plan(const AdjointArgs &a0, int row_splits, int body_splits,
                               void *scratch, hipStream_t s)
{
    AdjointArgs a = a0;
    AdjPlan p{};
    // row pass: split j
    const int64_t tiles = (a.n + kTile - 1) / kTile;
    const int64_t per_t = (tiles + row_splits - 1) / row_splits;
    p.row_split_len = per_t * kTile;
    p.row_splits = (int32_t)((a.n + p.row_split_len - 1) / p.row_split_len);
    // body pass: split rows
    const int64_t rt = (a.n_i + kRowTile - 1) / kRowTile;
    const int64_t per_r = (rt + body_splits - 1) / body_splits;
    p.body_split_len = (per_r > 0 ? per_r : 1) * kRowTile;
    p.body_splits = (int32_t)((a.n_i + p.body_split_len - 1) / p.body_split_len);
    if (p.body_splits < 1) p.body_splits = 1;
    char *c = (char *)scratch;
    auto take = [&c](size_t bytes) {
        char *r = c;
        c += (bytes + 255) / 256 * 256;
        return r;
    };
    p.row_partial = (double *)take((size_t)p.row_splits * 6 * a.n_i * sizeof(double));
    a.row_part = (double *)take(6 * (size_t)a.n_i * sizeof(double));
    p.body_partial = (double *)take((size_t)p.body_splits * 7 * a.n * sizeof(double));

    if (a.n_i > 0) {
        dim3 g1((unsigned)((a.n_i + kBlock - 1) / kBlock), (unsigned)p.row_splits);
        hipLaunchKernelGGL(adj_rows_kernel, g1, dim3(kBlock), 0, s, a, p);
        const int64_t tot = 6 * (int64_t)a.n_i;
        hipLaunchKernelGGL(adj_rows_reduce, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s,
                           a, p);
    }
    dim3 g2((unsigned)((a.n + kBlock - 1) / kBlock), (unsigned)p.body_splits);
    hipLaunchKernelGGL(adj_bodies_kernel, g2, dim3(kBlock), 0, s, a, p);
    hipLaunchKernelGGL(adj_bodies_reduce, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, s,
                       a, p);
    return hipGetLastError();
}

}  // namespace nb
