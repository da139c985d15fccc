// All-particle Hermite predictor (Wang et al. 2015, section 3.3.3 and Table 1
// "Pred.": every body is predicted once to the block time before the regular
// force; section 2: the force and its first derivative kept from the body's
// last step drive the prediction).  FP64, fixed operation order:
//   dt = t - t0;  xp = fma(dt, fma(dt, fma(dt, jrk*C6, a*0.5), v), x)
//                 vp = fma(dt, fma(dt, jrk*0.5, a), v)
// with C6 the FP64 value nearest 1/6.  A pure HBM stream: 13 FP64 in, 6 out
// (+ the optional FP32 mass copy) per body.
#include "nb_internal.h"

namespace nb {
namespace {

__global__ __launch_bounds__(256) void predict_kernel(int64_t n, double t, const double *x,
                                                      const double *v, const double *a,
                                                      const double *jrk, const double *t0,
                                                      const double *m, double *xp, double *vp,
                                                      float *m32)
{
    const double c6 = 0x1.5555555555555p-3;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double dt = t - t0[i];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int64_t q = (int64_t)k * n + i;
            const double xq = x[q], vq = v[q], aq = a[q], jq = jrk[q];
            const double px = __builtin_fma(dt, __builtin_fma(dt, __builtin_fma(dt, jq * c6, aq * 0.5), vq), xq);
            const double pv = __builtin_fma(dt, __builtin_fma(dt, jq * 0.5, aq), vq);
            xp[q] = px;
            vp[q] = pv;
        }
        if (m32) m32[i] = (float)m[i];
    }
}

}  // namespace

hipError_t launch_predict(int64_t n, double t, const double *x, const double *v, const double *a,
                          const double *jrk, const double *t0, const double *m, double *xp,
                          double *vp, float *m32, hipStream_t s)
{
    const int64_t want = (n + 255) / 256;
    const unsigned grid = (unsigned)(want < 65536 ? want : 65536);
    hipLaunchKernelGGL(predict_kernel, dim3(grid), dim3(256), 0, s, n, t, x, v, a, jrk, t0, m,
                       xp, vp, m32);
    return hipGetLastError();
}

}  // namespace nb
