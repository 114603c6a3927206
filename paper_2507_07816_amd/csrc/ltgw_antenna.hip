// Antenna-pattern weight tables for the lattice evaluation (one row of
// segment weights per sky point of the grid).
#include "ltgw_antenna.h"

#pragma clang fp contract(off)

namespace ltgw {

__global__ __launch_bounds__(256) void antenna_weights_kernel(const Arms A, const double *__restrict__ era,
                                                              int32_t n_seg, const double *__restrict__ sky,
                                                              int32_t n_sky,
                                                              const float *__restrict__ w,
                                                              const float *__restrict__ scale,
                                                              float *__restrict__ w_sky,
                                                              float *__restrict__ wq_sky) {
    const int32_t j = blockIdx.x * 256 + threadIdx.x;
    if (j >= n_seg) return;
    for (int32_t k = blockIdx.y; k < n_sky; k += gridDim.y) {
        const double *n = sky + 3 * (int64_t)k;
        float wo, wqo;
        antenna_weights(A, era[j], n[0], n[1], n[2], w[j], scale[j], wo, wqo);
        w_sky[(int64_t)k * n_seg + j] = wo;
        wq_sky[(int64_t)k * n_seg + j] = wqo;
    }
}

hipError_t launch_antenna_weights(const Arms &A, const double *era, int32_t n_seg, const double *sky,
                                  int32_t n_sky, const float *w, const float *scale, float *w_sky,
                                  float *wq_sky, hipStream_t st) {
    if (n_seg < 1 || n_sky < 1) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((n_seg + 255) / 256), (unsigned)(n_sky < 65535 ? n_sky : 65535)), block(256);
    hipLaunchKernelGGL(antenna_weights_kernel, grid, block, 0, st, A, era, n_seg, sky, n_sky, w, scale, w_sky,
                       wq_sky);
    return hipGetLastError();
}

}  // namespace ltgw
