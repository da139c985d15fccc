// Regular force + jerk + neighbour lists on gfx950 (Wang et al. 2015, section
// 2 and section 3.2.1: the GPU computes the regular force and its derivative
// and builds the neighbour lists in the same pass; Table 1 "Reg.").
//
// Two mappings of the O(N_i N) pair loop onto CDNA4:
//
//  * row-per-lane ("rows" kernel, large blocks): every lane owns 1, 2 or 4
//    rows in registers; the work-group streams its j-range through LDS in
//    tiles of kTile bodies (coalesced SoA global loads, double-buffered, one
//    barrier per tile) and every lane reads each staged body by LDS broadcast.
//    Neighbour appends are lane-private: a lane writes its own row's list.
//
//  * row-group-per-wave ("wave" kernel, small blocks): the 64 lanes of a
//    wavefront take 64 consecutive j while 1, 2 or 4 rows sit in scalar
//    registers; sums are reduced across the wave with butterfly shuffles and
//    neighbour appends are ordered by a ballot + lane prefix count, so lists
//    come out in ascending j.
//
// Either mapping may split the j-set into contiguous ranges ("splits") to put
// enough waves on the 256 CUs; the per-split FP64 partial sums and neighbour
// segments are combined by the merge kernel in split order, which keeps every
// list in ascending j.  No floating-point atomics are used anywhere, so each
// plan is bitwise deterministic and a row's result does not depend on the
// other rows of the block.
#include "nb_internal.h"
#include "nb_pair.h"

namespace nb {

namespace {

struct alignas(16) JBody {
    double x, y, z, m;
    double vx, vy, vz;
    float m32;
    int32_t pad;
};

template <bool MIXED>
struct Row {
    double x, y, z, vx, vy, vz;
    double hi;      // FP64 candidate bound (FP64 plan)
    float rs2f;     // canonical radius
    float candf;    // FP32 candidate bound (mixed plan)
    int32_t i;      // body index, -1 when the lane has no row
    int32_t cnt;    // neighbours found so far (true count)
    int32_t *lst;   // where this row's neighbours go
    int32_t lcap;   // capacity of lst
    Sums<MIXED> S;
};

template <bool MIXED>
__device__ __forceinline__ void row_init(Row<MIXED> &R, const ForceArgs &a, int64_t b,
                                         int32_t split)
{
    R.S.zero();
    R.cnt = 0;
    R.i = -1;
    R.x = R.y = R.z = kFar * 0.5;   // inert placeholder
    R.vx = R.vy = R.vz = 0.0;
    R.rs2f = -1.0f;
    R.hi = -1.0;
    R.candf = -1.0f;
    R.lst = nullptr;
    R.lcap = 0;
    if (b >= a.n_i) return;
    const int64_t i = a.i_block[b];
    if (i < 0 || i >= a.n) return;   // bad index: handled in the epilogue / merge
    R.i = (int32_t)i;
    R.x = a.xp[i];
    R.y = a.xp[a.n + i];
    R.z = a.xp[2 * a.n + i];
    R.vx = a.vp[i];
    R.vy = a.vp[a.n + i];
    R.vz = a.vp[2 * a.n + i];
    R.rs2f = (float)a.rs2[b];
    R.hi = cand_bound_f64(R.rs2f);
    R.candf = cand_bound_f32(R.rs2f);
    if (a.splits == 1) {
        R.lst = a.nb_list + b * (int64_t)a.cap;
        R.lcap = a.cap;
    } else {
        R.lst = a.seg_list + ((int64_t)split * a.n_i + b) * kSegCap;
        R.lcap = kSegCap;
    }
}

// One (row, body) pair in the row-per-lane kernel: lane-private append.
template <bool MIXED>
__device__ __forceinline__ void pair_rows(Row<MIXED> &R, const JBody &J, int32_t jidx)
{
    const double dx = J.x - R.x, dy = J.y - R.y, dz = J.z - R.z;
    if constexpr (MIXED) {
        const float fx = (float)dx, fy = (float)dy, fz = (float)dz;
        const float r2f = __builtin_fmaf(fz, fz, __builtin_fmaf(fy, fy, fx * fx));
        bool excl = false;
        if (r2f < R.candf) {
            int32_t jj = jidx;
            opaque(jj);
            const bool self = jj == R.i;
            const bool nbr = (r2f < R.rs2f) && !self;
            if (nbr) {
                if (R.cnt < R.lcap) R.lst[R.cnt] = jidx;
                ++R.cnt;
            }
            excl = nbr || self;
        }
        accum_mixed(R.S, fx, fy, fz, r2f, J.vx - R.vx, J.vy - R.vy, J.vz - R.vz, J.m32, excl);
    } else {
        const double r2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
        bool excl = false;
        if (r2 < R.hi) {
            double ex = dx, ey = dy, ez = dz;
            int32_t jj = jidx;
            opaque(ex, ey, ez);
            opaque(jj);
            const bool self = jj == R.i;
            const bool nbr = (canon_r2f(ex, ey, ez) < R.rs2f) && !self;
            if (nbr) {
                if (R.cnt < R.lcap) R.lst[R.cnt] = jidx;
                ++R.cnt;
            }
            excl = nbr || self;
        }
        accum_f64(R.S, dx, dy, dz, r2, J.vx - R.vx, J.vy - R.vy, J.vz - R.vz, J.m, excl);
    }
}

__device__ __forceinline__ void load_body(JBody &J, const ForceArgs &a, int64_t j, int64_t j1)
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
    J.m32 = (float)J.m;
    J.pad = 0;
}

// Epilogue shared by both kernels: one row's final sums and count.
template <bool MIXED>
__device__ __forceinline__ void row_store(const ForceArgs &a, int64_t b, int32_t split,
                                          int32_t i_raw_valid, const Sums<MIXED> &S,
                                          int32_t cnt, bool &ovf, bool &bad, bool &nonfin)
{
    if (a.splits == 1) {
        if (!i_raw_valid) {
            a.acc[b] = a.acc[a.n_i + b] = a.acc[2 * (int64_t)a.n_i + b] = 0.0;
            a.jerk[b] = a.jerk[a.n_i + b] = a.jerk[2 * (int64_t)a.n_i + b] = 0.0;
            a.nb_count[b] = 0;
            bad = true;
            return;
        }
        a.acc[b] = S.ax;
        a.acc[a.n_i + b] = S.ay;
        a.acc[2 * (int64_t)a.n_i + b] = S.az;
        a.jerk[b] = S.jx;
        a.jerk[a.n_i + b] = S.jy;
        a.jerk[2 * (int64_t)a.n_i + b] = S.jz;
        a.nb_count[b] = cnt;
        ovf = cnt > a.cap;
        nonfin = !finite6(S.ax, S.ay, S.az, S.jx, S.jy, S.jz);
    } else {
        double *p = a.part + (int64_t)split * 6 * a.n_i + b;
        p[0] = S.ax;
        p[a.n_i] = S.ay;
        p[2 * (int64_t)a.n_i] = S.az;
        p[3 * (int64_t)a.n_i] = S.jx;
        p[4 * (int64_t)a.n_i] = S.jy;
        p[5 * (int64_t)a.n_i] = S.jz;
        a.seg_cnt[(int64_t)split * a.n_i + b] = cnt;
    }
}

__device__ __forceinline__ void flush_flags(const ForceArgs &a, bool ovf, bool bad, bool nonfin)
{
    // called in uniform control flow by every lane of the wave
    const uint64_t o = __ballot(ovf), b = __ballot(bad), f = __ballot(nonfin);
    if ((threadIdx.x & (kWave - 1)) == 0 && (o | b | f)) {
        uint32_t st = (o ? kStOverflow : 0u) | (b ? kStBadIndex : 0u) | (f ? kStNonFinite : 0u);
        if (o) atomicOr(a.overflow, 1);
        if (a.status) atomicOr(a.status, st);
    }
}

// --------------------------------------------------------------------------
// Row-per-lane kernel.  grid = (ceil(n_i / (IR * kBlock)), splits).
// Lane t of work-group g owns rows g*IR*kBlock + r*kBlock + t, r < IR.
// --------------------------------------------------------------------------
template <bool MIXED, int IR>
__global__ __launch_bounds__(kBlock) void force_rows_kernel(ForceArgs a)
{
    __shared__ JBody tile[2][kTile];
    const int tid = threadIdx.x;
    const int32_t split = blockIdx.y;
    const int64_t j0 = (int64_t)split * a.split_len;
    const int64_t j1 = j0 + a.split_len < a.n ? j0 + a.split_len : a.n;
    const int64_t row0 = (int64_t)blockIdx.x * IR * kBlock;

    Row<MIXED> R[IR];
#pragma unroll
    for (int r = 0; r < IR; ++r) row_init(R[r], a, row0 + r * kBlock + tid, split);

    const int64_t ntiles = j1 > j0 ? (j1 - j0 + kTile - 1) / kTile : 0;
    JBody nxt;
    if (ntiles > 0) {
        load_body(nxt, a, j0 + tid, j1);
        tile[0][tid] = nxt;
    }
    __syncthreads();
    for (int64_t t = 0; t < ntiles; ++t) {
        const int cur = (int)(t & 1);
        const int64_t tbase = j0 + t * kTile;
        if (t + 1 < ntiles) load_body(nxt, a, tbase + kTile + tid, j1);
        const JBody *buf = tile[cur];
        for (int jj = 0; jj < kTile; jj += kFold) {
#pragma unroll 4
            for (int q = 0; q < kFold; ++q) {
                const JBody &J = buf[jj + q];
                const int32_t jidx = (int32_t)(tbase + jj + q);
#pragma unroll
                for (int r = 0; r < IR; ++r) pair_rows<MIXED>(R[r], J, jidx);
            }
            if constexpr (MIXED) {
#pragma unroll
                for (int r = 0; r < IR; ++r) R[r].S.fold();
            }
        }
        if (t + 1 < ntiles) tile[cur ^ 1][tid] = nxt;
        __syncthreads();
    }

    bool ovf = false, bad = false, nonfin = false;
#pragma unroll
    for (int r = 0; r < IR; ++r) {
        const int64_t b = row0 + r * kBlock + tid;
        if (b < a.n_i) {
            bool o = false, bd = false, f = false;
            row_store<MIXED>(a, b, split, R[r].i >= 0, R[r].S, R[r].cnt, o, bd, f);
            ovf |= o;
            bad |= bd;
            nonfin |= f;
        }
    }
    flush_flags(a, ovf, bad, nonfin);
}

// --------------------------------------------------------------------------
// Row-group-per-wave kernel.  Wave w (global) handles row group w / splits
// (rows G*(w/splits) + g) over j-range w % splits.  grid = ceil(waves / 4).
// --------------------------------------------------------------------------
template <int G>
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

template <bool MIXED, int G>
__global__ __launch_bounds__(kBlock) void force_wave_kernel(ForceArgs a)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t gw = (int64_t)blockIdx.x * (kBlock / kWave) +
                       __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int64_t ngroups = (a.n_i + G - 1) / G;
    if (gw >= ngroups * a.splits) return;   // whole wave leaves together
    const int64_t group = gw / a.splits;
    const int32_t split = (int32_t)(gw - group * a.splits);
    const int64_t j0 = (int64_t)split * a.split_len;
    const int64_t j1 = j0 + a.split_len < a.n ? j0 + a.split_len : a.n;

    // Row data is uniform across the wave.
    double rx[G], ry[G], rz[G], rvx[G], rvy[G], rvz[G], hi[G];
    float rs2f[G], candf[G];
    int32_t ri[G], cnt[G], lcap[G];
    int32_t *lst[G];
    Sums<MIXED> S[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const int64_t b = group * G + g;
        S[g].zero();
        cnt[g] = 0;
        ri[g] = -1;
        rx[g] = ry[g] = rz[g] = kFar * 0.5;
        rvx[g] = rvy[g] = rvz[g] = 0.0;
        rs2f[g] = -1.0f;
        hi[g] = -1.0;
        candf[g] = -1.0f;
        lst[g] = nullptr;
        lcap[g] = 0;
        if (b < a.n_i) {
            const int64_t i = a.i_block[b];
            if (i >= 0 && i < a.n) {
                ri[g] = (int32_t)i;
                rx[g] = a.xp[i];
                ry[g] = a.xp[a.n + i];
                rz[g] = a.xp[2 * a.n + i];
                rvx[g] = a.vp[i];
                rvy[g] = a.vp[a.n + i];
                rvz[g] = a.vp[2 * a.n + i];
                rs2f[g] = (float)a.rs2[b];
                hi[g] = cand_bound_f64(rs2f[g]);
                candf[g] = cand_bound_f32(rs2f[g]);
                if (a.splits == 1) {
                    lst[g] = a.nb_list + b * (int64_t)a.cap;
                    lcap[g] = a.cap;
                } else {
                    lst[g] = a.seg_list + ((int64_t)split * a.n_i + b) * kSegCap;
                    lcap[g] = kSegCap;
                }
            }
        }
    }

    int iter = 0;
    for (int64_t base = j0; base < j1; base += kWave) {
        const int64_t j = base + lane;
        JBody J;
        load_body(J, a, j, j1);
        const int32_t jidx = (int32_t)j;
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const double dx = J.x - rx[g], dy = J.y - ry[g], dz = J.z - rz[g];
            if constexpr (MIXED) {
                const float fx = (float)dx, fy = (float)dy, fz = (float)dz;
                const float r2f = __builtin_fmaf(fz, fz, __builtin_fmaf(fy, fy, fx * fx));
                const bool cand = r2f < candf[g];
                bool excl = false;
                if (__ballot(cand)) {
                    const bool self = cand && jidx == ri[g];
                    const bool nbr = cand && (r2f < rs2f[g]) && !self;
                    const uint64_t nm = __ballot(nbr);
                    if (nbr) {
                        const int p = cnt[g] + lanes_below(nm);
                        if (p < lcap[g]) lst[g][p] = jidx;
                    }
                    cnt[g] += __popcll(nm);
                    excl = nbr || self;
                }
                accum_mixed(S[g], fx, fy, fz, r2f, J.vx - rvx[g], J.vy - rvy[g], J.vz - rvz[g],
                            J.m32, excl);
            } else {
                const double r2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
                const bool cand = r2 < hi[g];
                bool excl = false;
                if (__ballot(cand)) {
                    const bool self = cand && jidx == ri[g];
                    const bool nbr = cand && (canon_r2f(dx, dy, dz) < rs2f[g]) && !self;
                    const uint64_t nm = __ballot(nbr);
                    if (nbr) {
                        const int p = cnt[g] + lanes_below(nm);
                        if (p < lcap[g]) lst[g][p] = jidx;
                    }
                    cnt[g] += __popcll(nm);
                    excl = nbr || self;
                }
                accum_f64(S[g], dx, dy, dz, r2, J.vx - rvx[g], J.vy - rvy[g], J.vz - rvz[g],
                          J.m, excl);
            }
        }
        if constexpr (MIXED) {
            if (++iter == kFold) {
                iter = 0;
#pragma unroll
                for (int g = 0; g < G; ++g) S[g].fold();
            }
        }
    }
    bool ovf = false, bad = false, nonfin = false;
#pragma unroll
    for (int g = 0; g < G; ++g) {
        S[g].fold();
        Sums<MIXED> T = S[g];
        T.ax = wave_sum<G>(T.ax);
        T.ay = wave_sum<G>(T.ay);
        T.az = wave_sum<G>(T.az);
        T.jx = wave_sum<G>(T.jx);
        T.jy = wave_sum<G>(T.jy);
        T.jz = wave_sum<G>(T.jz);
        const int64_t b = group * G + g;
        if (lane == 0 && b < a.n_i) {
            bool o = false, bd = false, f = false;
            row_store<MIXED>(a, b, split, ri[g] >= 0, T, cnt[g], o, bd, f);
            ovf |= o;
            bad |= bd;
            nonfin |= f;
        }
    }
    flush_flags(a, ovf, bad, nonfin);
}

// --------------------------------------------------------------------------
// Merge: one wave per row.  Sums the split partials in a fixed order,
// concatenates neighbour segments in split order (ascending j), writes the
// true count, and rebuilds any segment that overflowed its scratch capacity
// by re-running the canonical test over that split's j-range.
// --------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void merge_kernel(ForceArgs a)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t b = (int64_t)blockIdx.x * (kBlock / kWave) +
                      __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    if (b >= a.n_i) return;
    const int64_t i = a.i_block[b];
    const bool bad = i < 0 || i >= a.n;
    const int32_t S = a.splits;

    double v[6] = {0, 0, 0, 0, 0, 0};
    for (int32_t s = lane; s < S; s += kWave) {
        const double *p = a.part + (int64_t)s * 6 * a.n_i + b;
#pragma unroll
        for (int k = 0; k < 6; ++k) v[k] += p[(int64_t)k * a.n_i];
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) v[k] = wave_sum<1>(v[k]);

    bool ovf = false, nonfin = false;
    if (bad) {
        if (lane == 0) {
            for (int k = 0; k < 3; ++k) {
                a.acc[(int64_t)k * a.n_i + b] = 0.0;
                a.jerk[(int64_t)k * a.n_i + b] = 0.0;
            }
            a.nb_count[b] = 0;
        }
    } else {
        const double xi = a.xp[i], yi = a.xp[a.n + i], zi = a.xp[2 * a.n + i];
        const float rs2f = (float)a.rs2[b];
        int64_t off = 0;   // uniform: entries placed so far (true count)
        for (int32_t s0 = 0; s0 < S; s0 += kWave) {
            const int32_t s = s0 + lane;
            const int32_t c = s < S ? a.seg_cnt[(int64_t)s * a.n_i + b] : 0;
            // inclusive scan of c over lanes
            int64_t inc = c;
#pragma unroll
            for (int o = 1; o < kWave; o <<= 1) {
                const int64_t t = __shfl_up(inc, o, kWave);
                if (lane >= o) inc += t;
            }
            const int64_t start = off + inc - c;
            const bool room = c > 0 && start < a.cap;
            const bool rebuild = room && c > kSegCap;
            if (room && !rebuild) {
                const int64_t take = (int64_t)c < a.cap - start ? c : a.cap - start;
                const int32_t *src = a.seg_list + ((int64_t)s * a.n_i + b) * kSegCap;
                int32_t *dst = a.nb_list + b * (int64_t)a.cap + start;
                for (int64_t q = 0; q < take; ++q) dst[q] = src[q];
            }
            // segments that overflowed scratch: the wave rescans them one by one
            uint64_t rb = __ballot(rebuild);
            while (rb) {
                const int q = __builtin_ctzll(rb);
                rb &= rb - 1;
                const int32_t sq = __shfl(s, q, kWave);
                const int64_t st = __shfl(start, q, kWave);
                const int64_t lim = a.cap - st;   // entries this segment may place
                const int64_t jb = (int64_t)sq * a.split_len;
                const int64_t je = jb + a.split_len < a.n ? jb + a.split_len : a.n;
                int64_t placed = 0;
                for (int64_t base = jb; base < je && placed < lim; base += kWave) {
                    const int64_t j = base + lane;
                    bool nbr = false;
                    if (j < je && j != i) {
                        const double dx = a.xp[j] - xi, dy = a.xp[a.n + j] - yi,
                                     dz = a.xp[2 * a.n + j] - zi;
                        nbr = canon_r2f(dx, dy, dz) < rs2f;
                    }
                    const uint64_t nm = __ballot(nbr);
                    if (nbr) {
                        const int64_t p = placed + lanes_below(nm);
                        if (p < lim) a.nb_list[b * (int64_t)a.cap + st + p] = (int32_t)j;
                    }
                    placed += __popcll(nm);
                }
            }
            off += __shfl(inc, kWave - 1, kWave);
        }
        if (lane == 0) {
            a.acc[b] = v[0];
            a.acc[a.n_i + b] = v[1];
            a.acc[2 * (int64_t)a.n_i + b] = v[2];
            a.jerk[b] = v[3];
            a.jerk[a.n_i + b] = v[4];
            a.jerk[2 * (int64_t)a.n_i + b] = v[5];
            a.nb_count[b] = (int32_t)off;
            ovf = off > a.cap;
            nonfin = !finite6(v[0], v[1], v[2], v[3], v[4], v[5]);
        }
    }
    flush_flags(a, ovf, bad && lane == 0, nonfin);
}

__global__ void fill_i32_kernel(int32_t *p, int32_t value, int64_t count)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < count) p[k] = value;
}

}  // namespace

size_t force_scratch_bytes(const Plan &p, int32_t n_i)
{
    if (p.splits <= 1) return 0;
    const size_t rows = (size_t)p.splits * (size_t)n_i;
    return rows * (6 * sizeof(double) + sizeof(int32_t) + kSegCap * sizeof(int32_t)) + 1024;
}

void force_bind_scratch(ForceArgs &a, void *base)
{
    if (a.splits <= 1) {
        a.part = nullptr;
        a.seg_cnt = nullptr;
        a.seg_list = nullptr;
        return;
    }
    const size_t rows = (size_t)a.splits * (size_t)a.n_i;
    char *p = (char *)base;
    a.part = (double *)p;
    p += rows * 6 * sizeof(double);
    a.seg_cnt = (int32_t *)p;
    p += ((rows * sizeof(int32_t) + 255) / 256) * 256;
    a.seg_list = (int32_t *)p;
}

template <bool MIXED>
static hipError_t launch_force_t(const Plan &p, const ForceArgs &a, hipStream_t s)
{
    if (p.mapping == 1) {
        const int per = p.rows_per_lane * kBlock;
        dim3 grid((unsigned)((a.n_i + per - 1) / per), (unsigned)p.splits);
        switch (p.rows_per_lane) {
        case 1: hipLaunchKernelGGL((force_rows_kernel<MIXED, 1>), grid, dim3(kBlock), 0, s, a); break;
        case 2: hipLaunchKernelGGL((force_rows_kernel<MIXED, 2>), grid, dim3(kBlock), 0, s, a); break;
        case 4: hipLaunchKernelGGL((force_rows_kernel<MIXED, 4>), grid, dim3(kBlock), 0, s, a); break;
        default: return hipErrorInvalidValue;
        }
    } else {
        const int G = p.rows_per_lane;
        const int64_t waves = ((a.n_i + G - 1) / G) * (int64_t)p.splits;
        const int64_t per = kBlock / kWave;
        dim3 grid((unsigned)((waves + per - 1) / per));
        switch (G) {
        case 1: hipLaunchKernelGGL((force_wave_kernel<MIXED, 1>), grid, dim3(kBlock), 0, s, a); break;
        case 2: hipLaunchKernelGGL((force_wave_kernel<MIXED, 2>), grid, dim3(kBlock), 0, s, a); break;
        case 4: hipLaunchKernelGGL((force_wave_kernel<MIXED, 4>), grid, dim3(kBlock), 0, s, a); break;
        default: return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

hipError_t launch_force(const Plan &p, bool mixed, const ForceArgs &a, hipStream_t s)
{
    return mixed ? launch_force_t<true>(p, a, s) : launch_force_t<false>(p, a, s);
}

hipError_t launch_merge(bool mixed, const ForceArgs &a, hipStream_t s)
{
    (void)mixed;
    const int per = kBlock / kWave;
    dim3 grid((unsigned)((a.n_i + per - 1) / per));
    hipLaunchKernelGGL(merge_kernel, grid, dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t *p, int32_t value, int64_t count, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    dim3 grid((unsigned)((count + 255) / 256));
    hipLaunchKernelGGL(fill_i32_kernel, grid, dim3(256), 0, s, p, value, count);
    return hipGetLastError();
}

}  // namespace nb
