// Antenna-pattern weights (the weighting of Sec. 2): the response
// F+^2 + Fx^2 of an interferometer to a wave from direction n, used as a
// factor on the per-segment weights.  Internal to the library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#pragma clang fp contract(off)

namespace ltgw {

// Arms a, b: unit vectors in the Earth-fixed frame (z on the rotation axis).
struct Arms {
    double a[3], b[3];
};

// With the detector tensor Dt = (a a^T - b b^T)/2, the responses to the two
// polarisations come from the part of Dt transverse to n, and their squares
// summed are basis-free:
//   F+^2 + Fx^2 = 2 tr(Dt^2) - 4 |Dt n|^2 + (n^T Dt n)^2,
//   tr(Dt^2) = (|a|^4 - 2 (a.b)^2 + |b|^4)/4.
// The Earth's rotation by era turns the arms into the frame of n; the same
// value follows from turning n back instead: m = R_z(-era) n.  Rounding can
// leave a value just below 0 near a null of the response; it is clamped.
__host__ __device__ inline double antenna_response(const Arms &A, double era, double nx, double ny, double nz) {
    const double ce = cos(era), se = sin(era);
    const double mx = ce * nx + se * ny;
    const double my = ce * ny - se * nx;
    const double mz = nz;
    const double pa = (A.a[0] * mx + A.a[1] * my) + A.a[2] * mz;
    const double pb = (A.b[0] * mx + A.b[1] * my) + A.b[2] * mz;
    const double dx = 0.5 * (A.a[0] * pa - A.b[0] * pb);
    const double dy = 0.5 * (A.a[1] * pa - A.b[1] * pb);
    const double dz = 0.5 * (A.a[2] * pa - A.b[2] * pb);
    const double aa = (A.a[0] * A.a[0] + A.a[1] * A.a[1]) + A.a[2] * A.a[2];
    const double bb = (A.b[0] * A.b[0] + A.b[1] * A.b[1]) + A.b[2] * A.b[2];
    const double ab = (A.a[0] * A.b[0] + A.a[1] * A.b[1]) + A.a[2] * A.b[2];
    const double tr2 = 0.25 * ((aa * aa - 2.0 * (ab * ab)) + bb * bb);
    const double dn2 = (dx * dx + dy * dy) + dz * dz;
    const double ndn = 0.5 * (pa * pa - pb * pb);
    const double r = (2.0 * tr2 - 4.0 * dn2) + ndn * ndn;
    return r > 0.0 ? r : 0.0;
}

// The weights of one (detector, sky point, segment): the segment weight times
// the response, rounded once to FP32, and that times the store's row scale
// (the form the statistic takes for its FMA).
__device__ inline void antenna_weights(const Arms &A, double era, double nx, double ny, double nz, float w,
                                       float scale, float &w_out, float &wq_out) {
    const double r = antenna_response(A, era, nx, ny, nz);
    w_out = (float)((double)w * r);
    wq_out = w_out * scale;
}

// w_sky[k][j], wq_sky[k][j] for every sky point k of sky[n_sky][3] and segment j.
hipError_t launch_antenna_weights(const Arms &A, const double *era, int32_t n_seg, const double *sky,
                                  int32_t n_sky, const float *w, const float *scale, float *w_sky,
                                  float *wq_sky, hipStream_t st);

}  // namespace ltgw
