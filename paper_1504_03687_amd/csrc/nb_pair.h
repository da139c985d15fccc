// Device-side pair arithmetic shared by the force, merge, batched and adjoint
// kernels of libnbreg (gfx950).
//
// Physics (Wang et al. 2015, section 2; fourth-order Hermite with the
// Ahmad-Cohen neighbour scheme): for a row body i and a source body j with
// r = x_j - x_i, u = v_j - v_i (G = 1, no softening) the regular force term is
// m_j r / |r|^3 and its time derivative m_j [u / |r|^3 - 3 (r.u) r / |r|^5].
// j is a neighbour of i (and contributes nothing to the regular force) iff it
// lies inside i's neighbour radius, decided by one canonical single-precision
// test shared by every kernel so that lists are bit-identical across kernels,
// precisions and plans.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nb {

// Canonical squared distance for the neighbour test: each FP64 difference is
// rounded to FP32 (round-to-nearest-even), then r2f = fz*fz + (fy*fy + fx*fx)
// with two fused multiply-adds.  The whole file is compiled without
// floating-point contraction, so the plain product fx*fx stays a product.
__device__ __forceinline__ float canon_r2f(double dx, double dy, double dz)
{
    const float fx = (float)dx, fy = (float)dy, fz = (float)dz;
    return __builtin_fmaf(fz, fz, __builtin_fmaf(fy, fy, fx * fx));
}

// 1/sqrt(r2) in FP64: hardware estimate, then one third-order correction
// y <- y (1 + e/2 + 3 e^2 / 8) with e = 1 - r2 y^2 (the Taylor series of
// (1 - e)^-1/2).  From an estimate good to ~2^-22 this lands within an ulp or
// two.  r2 = 0 gives NaN, which the callers mask by selection.
__device__ __forceinline__ double rsqrt_f64(double r2)
{
    double y = __builtin_amdgcn_rsq(r2);
    const double t = r2 * y;
    const double e = __builtin_fma(-t, y, 1.0);
    const double c = __builtin_fma(0.375, e, 0.5);
    return __builtin_fma(y * e, c, y);
}

// Running sums of one row.  FP64 plan: FP64 sums.  Mixed plan: FP32 partial
// sums over short runs of j, folded into FP64 running sums.
template <bool MIXED>
struct Sums;

// FP64: pair terms go into partial sums over runs of j, which fold() adds
// into the running sums (ax..jz).  Summing a long j-range in runs keeps the
// rounding of the running sums from growing with the whole range: a row of
// 2^18 terms sums 2^10 runs of 2^8 instead of 2^18 single terms, so its
// error stays far below 1e-12 even where the jerk cancels strongly.  The
// jerk partial is kept as two parts, sum m r^-3 u (pjx..) and
// sum m (r.u) r^-5 r (prx..), combined at the fold as pj - 3 pr, so the
// factor -3 is not multiplied in for every pair.  fold() must run before
// the sums are read; it is idempotent.
template <>
struct Sums<false> {
    double ax, ay, az, jx, jy, jz;
    double va, vj;   // unused in FP64 (kept for a common slot layout)
    double pax, pay, paz, pjx, pjy, pjz, prx, pry, prz;
    __device__ __forceinline__ void zero()
    {
        ax = ay = az = jx = jy = jz = va = vj = 0.0;
        pax = pay = paz = pjx = pjy = pjz = prx = pry = prz = 0.0;
    }
    __device__ __forceinline__ void fold()
    {
        ax += pax;
        ay += pay;
        az += paz;
        jx += __builtin_fma(-3.0, prx, pjx);
        jy += __builtin_fma(-3.0, pry, pjy);
        jz += __builtin_fma(-3.0, prz, pjz);
        pax = pay = paz = pjx = pjy = pjz = prx = pry = prz = 0.0;
    }
};

// The FP64 row kernels fold their partial sums every kFoldF64 bodies from
// the start of the j-range (at the same positions for every tile length).
constexpr int kFoldF64 = 256;

// va, vj: sums of the squared norms of the folded FP32 partials.  For terms of
// varying sign this estimates sum |term|^2, the scale of the accumulated FP32
// rounding error of the row (which grows like its square root); rows whose
// estimated relative error is too large are recomputed in FP64.
// The jerk partial is kept as two parts, sum m r^-3 u and sum m r^-3 (r.u)
// r^-2 r, combined as (first - 3 * second) at the fold, so the factor -3 is
// applied once per run instead of once per pair.
template <>
struct Sums<true> {
    double ax, ay, az, jx, jy, jz;
    double va, vj;
    float pax, pay, paz, pjx, pjy, pjz, prx, pry, prz;
    __device__ __forceinline__ void zero()
    {
        ax = ay = az = jx = jy = jz = va = vj = 0.0;
        pax = pay = paz = pjx = pjy = pjz = prx = pry = prz = 0.0f;
    }
    __device__ __forceinline__ void fold()
    {
        const float qx = __builtin_fmaf(-3.0f, prx, pjx);
        const float qy = __builtin_fmaf(-3.0f, pry, pjy);
        const float qz = __builtin_fmaf(-3.0f, prz, pjz);
        ax += (double)pax; ay += (double)pay; az += (double)paz;
        jx += (double)qx; jy += (double)qy; jz += (double)qz;
        va += (double)__builtin_fmaf(paz, paz, __builtin_fmaf(pay, pay, pax * pax));
        vj += (double)__builtin_fmaf(qz, qz, __builtin_fmaf(qy, qy, qx * qx));
        pax = pay = paz = pjx = pjy = pjz = prx = pry = prz = 0.0f;
    }
};

// True when a mixed row should be recomputed in FP64: the rounding-error
// estimate k * sqrt(v) exceeds |sum| for acc or jerk (k = 2^-24 * safety / tol).
__device__ __forceinline__ bool needs_redo(double k, double ax, double ay, double az, double jx,
                                           double jy, double jz, double va, double vj)
{
    const double na2 = ax * ax + ay * ay + az * az;
    const double nj2 = jx * jx + jy * jy + jz * jz;
    return k * k * va > na2 || k * k * vj > nj2;
}

// FP64 regular term.  r2 is the FP64 squared distance; 'excl' marks the self
// pair or a neighbour (the term is then exactly zero: r^-1 is selected to 0).
__device__ __forceinline__ void accum_f64(Sums<false> &S, double dx, double dy, double dz,
                                          double r2, double ux, double uy, double uz,
                                          double mj, bool excl)
{
    double y = rsqrt_f64(r2);
    y = excl ? 0.0 : y;
    const double y2 = y * y;
    const double mr3 = (mj * y) * y2;               // m / r^3
    const double s = __builtin_fma(dz, uz, __builtin_fma(dy, uy, dx * ux));
    const double q = (s * y2) * mr3;                // m (r.u) / r^5; -3 applied by fold()
    S.pax = __builtin_fma(mr3, dx, S.pax);
    S.pay = __builtin_fma(mr3, dy, S.pay);
    S.paz = __builtin_fma(mr3, dz, S.paz);
    S.pjx = __builtin_fma(mr3, ux, S.pjx);
    S.pjy = __builtin_fma(mr3, uy, S.pjy);
    S.pjz = __builtin_fma(mr3, uz, S.pjz);
    S.prx = __builtin_fma(q, dx, S.prx);
    S.pry = __builtin_fma(q, dy, S.pry);
    S.prz = __builtin_fma(q, dz, S.prz);
}

// Mixed regular term: FP32 arithmetic on the FP32-rounded FP64 differences.
__device__ __forceinline__ void accum_mixed(Sums<true> &S, float fx, float fy, float fz,
                                            float r2f, double ux, double uy, double uz,
                                            float mj, bool excl)
{
    const float gx = (float)ux, gy = (float)uy, gz = (float)uz;
    float y = __builtin_amdgcn_rsqf(r2f);
    y = excl ? 0.0f : y;
    const float y2 = y * y;
    const float mr3 = (mj * y) * y2;
    const float s = __builtin_fmaf(fz, gz, __builtin_fmaf(fy, gy, fx * gx));
    const float q = (s * y2) * mr3;                 // m (r.u) / r^5; -3 applied at the fold
    S.pax = __builtin_fmaf(mr3, fx, S.pax);
    S.pay = __builtin_fmaf(mr3, fy, S.pay);
    S.paz = __builtin_fmaf(mr3, fz, S.paz);
    S.pjx = __builtin_fmaf(mr3, gx, S.pjx);
    S.pjy = __builtin_fmaf(mr3, gy, S.pjy);
    S.pjz = __builtin_fmaf(mr3, gz, S.pjz);
    S.prx = __builtin_fmaf(q, fx, S.prx);
    S.pry = __builtin_fmaf(q, fy, S.pry);
    S.prz = __builtin_fmaf(q, fz, S.prz);
}

// FP64 regular term added straight into FP64 running sums (used by the mixed
// kernels for near pairs, where FP32 rounding would dominate the error).
__device__ __forceinline__ void add_term_f64(double &ax, double &ay, double &az, double &jx,
                                             double &jy, double &jz, double dx, double dy,
                                             double dz, double ux, double uy, double uz,
                                             double mj)
{
    const double r2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
    const double y = rsqrt_f64(r2);
    const double y2 = y * y;
    const double mr3 = (mj * y) * y2;
    const double s = __builtin_fma(dz, uz, __builtin_fma(dy, uy, dx * ux));
    const double q = (s * y2) * (-3.0 * mr3);
    ax = __builtin_fma(mr3, dx, ax);
    ay = __builtin_fma(mr3, dy, ay);
    az = __builtin_fma(mr3, dz, az);
    jx = __builtin_fma(q, dx, __builtin_fma(mr3, ux, jx));
    jy = __builtin_fma(q, dy, __builtin_fma(mr3, uy, jy));
    jz = __builtin_fma(q, dz, __builtin_fma(mr3, uz, jz));
}

// Mixed kernels evaluate pairs closer than sqrt(near) neighbour radii in FP64
// (near = kNearFactor for large j-ranges, 1 otherwise: in a small cluster the
// near pairs are a large share of all pairs and the FP64 branch would be taken
// in most wave iterations).  Those few pairs carry the largest terms, so their
// FP32 rounding would dominate the error of a row whose sum cancels.
constexpr float kNearFactor = 4.0f;
constexpr int64_t kNearMinBodies = int64_t(1) << 18;

// Candidate bound for the FP64 plans: every canonical neighbour (and the self
// pair, r2 = 0) has FP64 r2 < hi, so the exact canonical test only runs for
// the rare pairs below hi.  The FP32 roundings in r2f change r2 by less than
// 3.3e-7 relative; the margin 2^-20 (9.5e-7) covers that.
__device__ __forceinline__ double cand_bound_f64(float rs2f)
{
    const double h = (double)rs2f * (1.0 + 0x1p-20);
    return h > 1e-300 ? h : 1e-300;
}

// Candidate bound for the mixed plans, on r2f itself: the near-field bound
// (neighbours included), or the smallest normal float when rs2 <= 0 so that
// the self pair still enters.
__device__ __forceinline__ float cand_bound_f32(float rs2f, float near)
{
    const float h = rs2f * near;
    return h > 1.17549435e-38f ? h : 1.17549435e-38f;
}

// Keeps the compiler from hoisting the rare exact-test path above its branch
// (the test is cheap enough that it would otherwise be evaluated for every
// pair).  Emits no instruction.
__device__ __forceinline__ void opaque(double &a, double &b, double &c)
{
    __asm__ volatile("" : "+v"(a), "+v"(b), "+v"(c));
}
__device__ __forceinline__ void opaque(int32_t &a)
{
    __asm__ volatile("" : "+v"(a));
}

__device__ __forceinline__ bool finite6(double a, double b, double c, double d, double e,
                                        double f)
{
    return __builtin_isfinite(a) && __builtin_isfinite(b) && __builtin_isfinite(c) &&
           __builtin_isfinite(d) && __builtin_isfinite(e) && __builtin_isfinite(f);
}

__device__ __forceinline__ int lanes_below(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

}  // namespace nb
