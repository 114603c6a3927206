// HIP kernels (gfx950) for the template-bank detection statistic.
//
// Data layout in HBM
//   store   per detector, [n_seg][pitch] elements of 4/2/1 bytes (FP32, BF16,
//           OCP E4M3).  Element 0 and element n_bins+1 of every row are 0
//           guards; element b+1 holds column b.  The sign bit of each element
//           is the number-count bit (rho > rho_th, decided on the FP32 input):
//           normalised power is non-negative, so the bit is free and one
//           gather serves both statistics (Sec. 2: power and number count).
//   H       per detector, [n_sky][n_brake][n_tau][n_seg] FP64,
//           H = RN(RN(g*D)*T_sft), the bin-scaled ratio f^/f0 of Eqs. 1-2.
//   results per template: s (FP64), c, N (int32), W1, W2 (FP64).
//
// Evaluation kernel: one lane per template, 256 consecutive f0 per block,
// one (sky, n, tau) group per block row.  Per segment a lane does
//   x = f0*H (FP64)  v = x + (1.5 - k_lo)  i = (unsigned)trunc(v)
// and gathers element i of the segment's row with a structured buffer load
// (idxen; stride = element size; the row as the scalar byte offset).  The
// resource holds n_bins + 2 records, so the hardware range check returns 0
// for every index past the upper guard, including negative ones (large as
// unsigned).  Neighbouring f0 lanes read neighbouring
// columns, so a wavefront's 64 gathers fall in a few cache lines.  The
// per-segment H, weight and row address are wavefront-uniform (SGPRs).
// trunc(v) - 1 equals floor(RN(x + 0.5)) - k_lo whenever the latter is in
// band, for k_lo >= 2 and x < 2^30 (both checked by the host): x + 1.5 - k_lo
// is exact in FP64 whenever its magnitude is at most x, and every other case
// lands on the lower guard or out of range.
#include "ltgw_internal.h"
#include "ddpow.h"

#pragma clang fp contract(off)

namespace ltgw {

extern "C" __device__ float ltgw_sbuf_f32(__amdgpu_buffer_rsrc_t, int vindex, int voffset,
                                          int soffset, int aux)
    __asm("llvm.amdgcn.struct.ptr.buffer.load.f32");
extern "C" __device__ unsigned short ltgw_sbuf_u16(__amdgpu_buffer_rsrc_t, int vindex, int voffset,
                                                   int soffset, int aux)
    __asm("llvm.amdgcn.struct.ptr.buffer.load.i16");
extern "C" __device__ unsigned char ltgw_sbuf_u8(__amdgpu_buffer_rsrc_t, int vindex, int voffset,
                                                 int soffset, int aux)
    __asm("llvm.amdgcn.struct.ptr.buffer.load.i8");

// Word 3 of a gfx9 buffer resource: 32-bit data format, no swizzle.
constexpr int kBufDword3 = 0x00020000;

template <int STORE>
struct Store;
template <>
struct Store<LTGW_STORE_F32> {
    static constexpr int kBytes = 4;
    // returns |value| and adds the count bit
    __device__ static float get(__amdgpu_buffer_rsrc_t r, int i, int soff, int &cnt) {
        float p = ltgw_sbuf_f32(r, i, 0, soff, 0);
        cnt += (int)(__float_as_uint(p) >> 31);
        return __builtin_fabsf(p);
    }
};
template <>
struct Store<LTGW_STORE_BF16> {
    static constexpr int kBytes = 2;
    __device__ static float get(__amdgpu_buffer_rsrc_t r, int i, int soff, int &cnt) {
        unsigned u = ltgw_sbuf_u16(r, i, 0, soff, 0);
        cnt += (int)(u >> 15);
        return __builtin_fabsf(__uint_as_float(u << 16));
    }
};
template <>
struct Store<LTGW_STORE_FP8> {
    static constexpr int kBytes = 1;
    __device__ static float get(__amdgpu_buffer_rsrc_t r, int i, int soff, int &cnt) {
        unsigned u = ltgw_sbuf_u8(r, i, 0, soff, 0);
        cnt += (int)(u >> 7);
        return __builtin_fabsf(__builtin_amdgcn_cvt_f32_fp8((int)u, 0));
    }
};

// ---------------------------------------------------------------------------
// Ingest: FP32 power -> store with guards and the count bit.
__device__ inline unsigned bf16_rne_bits(float x) {  // finite x >= 0
    unsigned u = __float_as_uint(x);
    return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}
__device__ inline unsigned e4m3_rne_sat_bits(float a) {  // finite a >= 0
    if (!(a < 448.0f)) return 0x7eu;
    unsigned u = __float_as_uint(a);
    int ex = (int)(u >> 23) - 127;
    if (ex < -6) return (unsigned)__builtin_rintf(a * 512.0f);  // m * 2^-9, m <= 8
    unsigned keep = (u >> 20) & 7u, rem = u & 0xfffffu;
    if (rem > 0x80000u || (rem == 0x80000u && (keep & 1u))) keep += 1u;
    return ((unsigned)(ex + 7) << 3) + keep;
}

__device__ inline float block_max_256(float v, float *sh) {
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    float m = fmaxf(fmaxf(sh[0], sh[1]), fmaxf(sh[2], sh[3]));
    __syncthreads();
    return m;
}

template <int STORE>
__global__ __launch_bounds__(256) void ingest_kernel(const float *__restrict__ in, int n_bins,
                                                     int64_t pitch, void *__restrict__ out,
                                                     float *__restrict__ scale,
                                                     const float *__restrict__ w,
                                                     float *__restrict__ wq, float th,
                                                     unsigned long long *bad) {
    __shared__ float sh[4];
    const int64_t j = blockIdx.x;
    const float *row = in + j * (int64_t)n_bins;
    float sc = 1.0f;
    if (STORE == LTGW_STORE_FP8) {
        float m = 0.0f;
        for (int b = threadIdx.x; b < n_bins; b += 256) {
            float x = row[b];
            if (x >= 0.0f && x <= 3.402823466e38f) m = fmaxf(m, x);
        }
        m = block_max_256(m, sh);
        sc = (m == 0.0f) ? 1.0f : m / 448.0f;
    }
    unsigned nbad = 0;
    for (int64_t b = threadIdx.x; b < pitch; b += 256) {
        unsigned code = 0;
        if (b >= 1 && b <= n_bins) {
            float x = row[b - 1];
            if (!(x >= 0.0f && x <= 3.402823466e38f)) {
                ++nbad;
                x = 0.0f;
            }
            x = __builtin_fabsf(x);  // -0 -> +0
            unsigned bit = x > th ? 1u : 0u;
            if (STORE == LTGW_STORE_F32) code = __float_as_uint(x) | (bit << 31);
            if (STORE == LTGW_STORE_BF16) code = bf16_rne_bits(x) | (bit << 15);
            if (STORE == LTGW_STORE_FP8) code = e4m3_rne_sat_bits(x / sc) | (bit << 7);
        }
        if (STORE == LTGW_STORE_F32) ((unsigned *)out)[j * pitch + b] = code;
        if (STORE == LTGW_STORE_BF16) ((unsigned short *)out)[j * pitch + b] = (unsigned short)code;
        if (STORE == LTGW_STORE_FP8) ((unsigned char *)out)[j * pitch + b] = (unsigned char)code;
    }
    if (nbad) atomicAdd(bad, (unsigned long long)nbad);
    if (threadIdx.x == 0) {
        scale[j] = sc;
        wq[j] = w[j] * sc;
    }
}

hipError_t launch_ingest(int store, const float *power, int32_t n_seg, int32_t n_bins,
                         int64_t pitch, void *out, float *scale, const float *w, float *wq,
                         float rho_th, unsigned long long *bad, hipStream_t st) {
    dim3 grid(n_seg), block(256);
    if (store == LTGW_STORE_F32)
        hipLaunchKernelGGL(ingest_kernel<LTGW_STORE_F32>, grid, block, 0, st, power, n_bins, pitch,
                           out, scale, w, wq, rho_th, bad);
    else if (store == LTGW_STORE_BF16)
        hipLaunchKernelGGL(ingest_kernel<LTGW_STORE_BF16>, grid, block, 0, st, power, n_bins, pitch,
                           out, scale, w, wq, rho_th, bad);
    else
        hipLaunchKernelGGL(ingest_kernel<LTGW_STORE_FP8>, grid, block, 0, st, power, n_bins, pitch,
                           out, scale, w, wq, rho_th, bad);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Eq. 1: g[(i_n*n_tau + i_tau)][j] = RN(u^e), 0 where t_j < T0.
__global__ __launch_bounds__(256) void spin_factor_kernel(const double *__restrict__ t_seg,
                                                          int n_seg, double t0,
                                                          const double *__restrict__ tau,
                                                          int n_tau,
                                                          const double *__restrict__ brake,
                                                          double *__restrict__ g,
                                                          unsigned long long *undecided) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    const int grp = blockIdx.y;
    if (j >= n_seg) return;
    const double t = t_seg[j];
    double out = 0.0;
    if (!(t < t0)) {
        const double ta = tau[grp % n_tau];
        const double n = brake[grp / n_tau];
        const double d = t - t0;
        const double q = d / ta;
        const double u = 1.0 + q;
        const double e = 1.0 / (1.0 - n);
        int und = 0;
        out = pow_cr(u, e, &und);
        if (und) atomicAdd(undecided, 1ull);
    }
    g[(int64_t)grp * n_seg + j] = out;
}

hipError_t launch_spin_factor(const double *t_seg, int32_t n_seg, double t0, const double *tau,
                              int32_t n_tau, const double *brake, int32_t n_brake, double *g,
                              unsigned long long *undecided, hipStream_t st) {
    dim3 grid((n_seg + 255) / 256, n_tau * n_brake), block(256);
    hipLaunchKernelGGL(spin_factor_kernel, grid, block, 0, st, t_seg, n_seg, t0, tau, n_tau, brake,
                       g, undecided);
    return hipGetLastError();
}

// Eq. 2 and the bin scale: H[(sky*n_tn + tn)][j] = RN(RN(g*D)*T_sft),
// D = 1 + ((vx nx + vy ny) + vz nz)/c.
__global__ __launch_bounds__(256) void track_factor_kernel(const double *__restrict__ g,
                                                           int n_tn,
                                                           const double *__restrict__ v,
                                                           int n_seg,
                                                           const double *__restrict__ sky,
                                                           double t_sft, double *__restrict__ H) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    const int row = blockIdx.y;  // sky * n_tn + tn
    if (j >= n_seg) return;
    const int s = row / n_tn, tn = row % n_tn;
    const double a = v[3 * j + 0] * sky[3 * s + 0];
    const double b = v[3 * j + 1] * sky[3 * s + 1];
    const double z = v[3 * j + 2] * sky[3 * s + 2];
    const double vn = (a + b) + z;
    const double r = vn / kC;
    const double D = 1.0 + r;
    const double h = g[(int64_t)tn * n_seg + j] * D;
    H[(int64_t)row * n_seg + j] = h * t_sft;
}

hipError_t launch_track_factor(const double *g, int32_t n_tn, const double *v, int32_t n_seg,
                               const double *sky, int32_t n_sky, double t_sft, double *H,
                               hipStream_t st) {
    dim3 grid((n_seg + 255) / 256, n_sky * n_tn), block(256);
    hipLaunchKernelGGL(track_factor_kernel, grid, block, 0, st, g, n_tn, v, n_seg, sky, t_sft, H);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Statistic (Sec. 2).  A lane carries TPL templates (f0 256 apart, so each
// of them is a coalesced wavefront access); segments go in batches of U so
// that U*TPL independent gathers are in flight per wavefront.  FP32 partial
// sums over chunks of 32 segments are carried in FP64.
constexpr int kChunk = 32;

// Bin-scaled track factor H_j of one (detector, group): from a table, or
// formed on the fly as RN(RN(g_j D_j) T_sft) (batched searches, whose sky
// patches would make a full table too large).  Both are wavefront-uniform.
struct HTable {
    const double *H;
    __device__ double operator()(int j) const { return H[j]; }
};
struct HFromGD {
    const double *g;  // [n_seg] of the group's (n, tau)
    const double *D;  // [n_seg] of the group's sky direction
    double t_sft;
    __device__ double operator()(int j) const {
        const double h = g[j] * D[j];
        return h * t_sft;
    }
};

template <int TPL>
struct Acc {
    double s[TPL], w1[TPL], w2[TPL];
    int cnt[TPL], nin[TPL];
    __device__ void zero() {
        for (int t = 0; t < TPL; ++t) {
            s[t] = w1[t] = w2[t] = 0.0;
            cnt[t] = nin[t] = 0;
        }
    }
};

// SHIFT = 1 reads a 2x2-coarsened store (pairs of segments and of bins; the
// caller passes cshift + 1 and the pair's first-segment track factor): the
// coarse column of fine column b is b >> 1, i.e. index trunc(v) >> 1.
template <int STORE, bool MOMENTS, int TPL, int U, class HS, int SHIFT = 0>
__device__ __forceinline__ void seg_batch(const DetView &D, __amdgpu_buffer_rsrc_t rs, const HS &hs,
                                          int j, const double (&f0)[TPL], float (&sc)[TPL],
                                          float (&w1c)[TPL], float (&w2c)[TPL], Acc<TPL> &acc) {
    const unsigned nb = (unsigned)D.n_bins;
    double h[U];
#pragma unroll
    for (int k = 0; k < U; ++k) h[k] = hs(j + k);
    unsigned idx[TPL][U];
#pragma unroll
    for (int t = 0; t < TPL; ++t)
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const double x = f0[t] * h[k];
            const double vv = x + D.cshift;
            // a negative index wraps to a large unsigned value: out of range, reads 0
            idx[t][k] = (unsigned)__double2int_rz(vv) >> SHIFT;
        }
    float p[TPL][U];
#pragma unroll
    for (int k = 0; k < U; ++k)
#pragma unroll
        for (int t = 0; t < TPL; ++t)
            p[t][k] = Store<STORE>::get(rs, (int)idx[t][k], (j + k) * D.pitch_bytes, acc.cnt[t]);
#pragma unroll
    for (int k = 0; k < U; ++k) {
        const float wq = D.wq[j + k];
#pragma unroll
        for (int t = 0; t < TPL; ++t) {
            sc[t] = __builtin_fmaf(wq, p[t][k], sc[t]);
            if (MOMENTS) {
                const bool inb = (idx[t][k] - 1u) < nb;
                acc.nin[t] += inb ? 1 : 0;
                const float wj = inb ? D.w[j + k] : 0.0f;
                w1c[t] += wj;
                w2c[t] = __builtin_fmaf(wj, wj, w2c[t]);
            }
        }
    }
}

// All segments of one detector.
// Segments [jb, je) of detector D to visit for the runs [blk0, blk1) of 64 f0
// of group grp: the in-band window widened to whole chunks (chunks outside
// add exact zeros, so skipping them leaves every sum bit-identical); all
// segments when D has no windows.  Wave-uniform.
__device__ __forceinline__ void seg_window(const DetView &D, int grp, int blk0, int blk1, int &jb, int &je) {
    jb = 0;
    je = D.n_seg;
    if (!D.win) return;
    int lo = D.n_seg, hi = -1;
    const int end = blk1 < D.win_blocks ? blk1 : D.win_blocks;
    for (int b = blk0; b < end; ++b) {
        const int2 w = D.win[(int64_t)grp * D.win_blocks + b];
        lo = min(lo, w.x);
        hi = max(hi, w.y);
    }
    lo = __builtin_amdgcn_readfirstlane(lo);
    hi = __builtin_amdgcn_readfirstlane(hi);
    if (hi < lo) {
        je = 0;
        return;
    }
    jb = (lo / kChunk) * kChunk;
    je = min(D.n_seg, (hi / kChunk + 1) * kChunk);
}

template <int STORE, bool MOMENTS, int TPL, int U, class HS, int SHIFT = 0>
__device__ __forceinline__ void accumulate_det(const DetView &D, const HS &hs,
                                               const double (&f0)[TPL], Acc<TPL> &acc, int jb = 0,
                                               int je = -1) {
    if (je < 0) je = D.n_seg;
    // one resource per detector, n_bins + 2 records (a row with its guards);
    // the row is the instruction's scalar byte offset
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        (void *)D.store, Store<STORE>::kBytes, D.n_bins + 2, kBufDword3);
    int j = jb;
    for (; j + kChunk <= je; j += kChunk) {
        float sc[TPL], w1c[TPL], w2c[TPL];
        for (int t = 0; t < TPL; ++t) sc[t] = w1c[t] = w2c[t] = 0.0f;
#pragma unroll 1
        for (int b = 0; b < kChunk; b += U)
            seg_batch<STORE, MOMENTS, TPL, U, HS, SHIFT>(D, rs, hs, j + b, f0, sc, w1c, w2c, acc);
        for (int t = 0; t < TPL; ++t) {
            acc.s[t] += (double)sc[t];
            if (MOMENTS) {
                acc.w1[t] += (double)w1c[t];
                acc.w2[t] += (double)w2c[t];
            }
        }
    }
    if (j < je) {
        float sc[TPL], w1c[TPL], w2c[TPL];
        for (int t = 0; t < TPL; ++t) sc[t] = w1c[t] = w2c[t] = 0.0f;
        for (; j < je; ++j)
            seg_batch<STORE, MOMENTS, TPL, 1, HS, SHIFT>(D, rs, hs, j, f0, sc, w1c, w2c, acc);
        for (int t = 0; t < TPL; ++t) {
            acc.s[t] += (double)sc[t];
            if (MOMENTS) {
                acc.w1[t] += (double)w1c[t];
                acc.w2[t] += (double)w2c[t];
            }
        }
    }
}

// Results of a lane's templates; template index grp*n_f0 + i.
template <bool MOMENTS, int TPL>
__device__ __forceinline__ void store_results(const Acc<TPL> &acc, const int (&i)[TPL], int grp,
                                              int n_f0, double *s, int32_t *c, int32_t *n,
                                              double *w1, double *w2, float *out_s, int32_t *out_c,
                                              int32_t *out_n, unsigned long long *in_band_total) {
    if (MOMENTS) {
        // in-band total for the roofline's algorithmic bytes (one atomic per wave)
        unsigned long long nw = 0;
        for (int t = 0; t < TPL; ++t) nw += (i[t] < n_f0) ? (unsigned long long)acc.nin[t] : 0ull;
        for (int o = 32; o > 0; o >>= 1) nw += __shfl_xor(nw, o, 64);
        if (in_band_total) atomicAdd(in_band_total, (threadIdx.x & 63) == 0 ? nw : 0ull);
    }
    for (int t = 0; t < TPL; ++t) {
        if (i[t] >= n_f0) continue;
        const int64_t q = (int64_t)grp * n_f0 + i[t];
        s[q] = acc.s[t];
        c[q] = acc.cnt[t];
        if (out_s) out_s[q] = (float)acc.s[t];
        if (out_c) out_c[q] = acc.cnt[t];
        if (MOMENTS) {
            n[q] = acc.nin[t];
            w1[q] = acc.w1[t];
            w2[q] = acc.w2[t];
            if (out_n) out_n[q] = acc.nin[t];
        }
    }
}

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2).  Block w runs on XCD w % 8; it is given the (f0 tile, group) pair
// number start(x) + w / 8 in tile-major order (group fastest), where XCD x
// owns a contiguous range of pairs.  So the blocks resident on one XCD at a
// time cover one f0 tile of many neighbouring (tau, n, sky) groups: their
// tracks start at the same bins and stay close for similar tau and n, so
// their reads of each row overlap in that XCD's L2.  (Group-major order, one
// group's successive f0 tiles side by side, reads disjoint bins and measured
// slower.)
// A launch may cover a slice [first, first + gridDim.x) of the pairs (a
// generation of the grid); the XCD ranges are taken within the slice.
constexpr int kXcds = 8;
__device__ inline void xcd_tile_group(int w, int n_blocks, int n_tiles, int &tile, int &grp,
                                      int first = 0, int total = -1) {
    const int x = w % kXcds, k = w / kXcds;
    const int base = n_blocks / kXcds, extra = n_blocks % kXcds;
    const int start = x * base + (x < extra ? x : extra);
    const int p = first + start + k;
    const int n_groups = (total < 0 ? n_blocks : total) / n_tiles;
    tile = p / n_groups;
    grp = p % n_groups;
}

// A launch covers the segments [j_lo, j_hi) (a slab; multiples of the chunk
// except a final j_hi = n_seg): a slab after the first resumes from the sums
// the previous slab stored (the same operations in the same order as one
// pass), and only the last slab writes the caller's outputs.
template <int STORE, bool MOMENTS, int TPL, int U>
__global__ __launch_bounds__(256) void eval_kernel(const EvalArgs a, int first, int total, int j_lo, int j_hi,
                                                   int last) {
    const int n_tiles = (a.n_f0 + 256 * TPL - 1) / (256 * TPL);
    int tile, grp;
    xcd_tile_group(blockIdx.x, gridDim.x, n_tiles, tile, grp, first, total);
    int i[TPL];
    double f0[TPL];
    for (int t = 0; t < TPL; ++t) {
        i[t] = tile * 256 * TPL + t * 256 + threadIdx.x;
        f0[t] = a.f0_min + (double)i[t] * a.f0_step;
    }
    Acc<TPL> acc;
    acc.zero();
    if (j_lo > 0)
        for (int t = 0; t < TPL; ++t) {
            if (i[t] >= a.n_f0) continue;
            const int64_t q = (int64_t)grp * a.n_f0 + i[t];
            acc.s[t] = a.s[q];
            acc.cnt[t] = a.c[q];
            if (MOMENTS) {
                acc.nin[t] = a.n[q];
                acc.w1[t] = a.w1[q];
                acc.w2[t] = a.w2[q];
            }
        }
    for (int d = 0; d < a.n_det; ++d) {
        const DetView D = a.det[d];
        int jb, je;
        const int runs = D.win ? 256 * TPL / D.win_run : 1;
        seg_window(D, grp, tile * runs, (tile + 1) * runs, jb, je);
        jb = jb > j_lo ? jb : j_lo;
        je = je < j_hi ? je : j_hi;
        if (jb < je)
            accumulate_det<STORE, MOMENTS, TPL, U>(D, HTable{D.H + (int64_t)grp * D.n_seg}, f0, acc, jb, je);
    }
    store_results<MOMENTS, TPL>(acc, i, grp, a.n_f0, a.s, a.c, a.n, a.w1, a.w2, last ? a.out_s : nullptr,
                                last ? a.out_c : nullptr, last ? a.out_n : nullptr,
                                last ? a.in_band_total : nullptr);
}

// Tile shapes: (templates per lane, segments per gather batch).
constexpr int kVariantTpl[kNumShapes] = {1, 1, 2, 2};

int variant_templates_per_block(int variant) { return 256 * kVariantTpl[variant & 3]; }

// Segments per slab (variant & 8); a multiple of the chunk.
constexpr int kSlab = 1024;

template <int STORE, bool MOMENTS, int TPL, int U>
static hipError_t launch_eval_v(const EvalArgs &a, bool generations, bool slabs, int cu_count, hipStream_t st) {
    const int64_t blocks = (int64_t)((a.n_f0 + 256 * TPL - 1) / (256 * TPL)) * a.n_groups;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    int64_t step = blocks;
    if (generations) {
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, eval_kernel<STORE, MOMENTS, TPL, U>, 256, 0) !=
                hipSuccess || per_cu < 1) {
            (void)hipGetLastError();
            per_cu = 1;
        }
        step = (int64_t)cu_count * per_cu;
    }
    // slabs only for one detector (one segment axis)
    const int n_seg = a.det[0].n_seg;
    const int slab = (slabs && a.n_det == 1) ? kSlab : 0x7fffffff;
    for (int j_lo = 0; j_lo == 0 || j_lo < n_seg; j_lo += slab) {
        const int j_hi = (a.n_det > 1 || slab == 0x7fffffff || j_lo + slab >= n_seg) ? 0x7fffffff : j_lo + slab;
        const int last = j_hi == 0x7fffffff ? 1 : 0;
        for (int64_t first = 0; first < blocks; first += step) {
            const int64_t n = blocks - first < step ? blocks - first : step;
            hipLaunchKernelGGL((eval_kernel<STORE, MOMENTS, TPL, U>), dim3((unsigned)n), dim3(256), 0, st, a,
                               (int)first, (int)blocks, j_lo, j_hi, last);
            const hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        if (last) break;
    }
    return hipSuccess;
}

template <int STORE, bool MOMENTS>
static hipError_t launch_eval_m(int variant, const EvalArgs &a, int cu_count, hipStream_t st) {
    const bool gen = (variant & 4) != 0, slabs = (variant & 8) != 0;
    switch (variant & 3) {
        case 0: return launch_eval_v<STORE, MOMENTS, 1, 8>(a, gen, slabs, cu_count, st);
        case 1: return launch_eval_v<STORE, MOMENTS, 1, 16>(a, gen, slabs, cu_count, st);
        case 2: return launch_eval_v<STORE, MOMENTS, 2, 8>(a, gen, slabs, cu_count, st);
        default: return launch_eval_v<STORE, MOMENTS, 2, 16>(a, gen, slabs, cu_count, st);
    }
}

template <int STORE>
static hipError_t launch_eval_s(bool moments, int variant, const EvalArgs &a, int cu_count, hipStream_t st) {
    return moments ? launch_eval_m<STORE, true>(variant, a, cu_count, st)
                   : launch_eval_m<STORE, false>(variant, a, cu_count, st);
}

hipError_t launch_eval(int store, bool moments, int variant, const EvalArgs &a, int cu_count, hipStream_t st) {
    if (variant < 0 || variant >= kNumVariants) return hipErrorInvalidValue;
    if (store == LTGW_STORE_F32) return launch_eval_s<LTGW_STORE_F32>(moments, variant, a, cu_count, st);
    if (store == LTGW_STORE_BF16) return launch_eval_s<LTGW_STORE_BF16>(moments, variant, a, cu_count, st);
    return launch_eval_s<LTGW_STORE_FP8>(moments, variant, a, cu_count, st);
}

// A value that is the same in every lane, moved to scalar registers word by
// word (lets the compiler treat descriptors read from memory as uniform).
template <class T>
__device__ __forceinline__ T uniform(const T &x) {
    static_assert(sizeof(T) % 4 == 0, "whole words only");
    int w[sizeof(T) / 4];
    __builtin_memcpy(w, &x, sizeof(T));
#pragma unroll
    for (unsigned k = 0; k < sizeof(T) / 4; ++k) w[k] = __builtin_amdgcn_readfirstlane(w[k]);
    T y;
    __builtin_memcpy(&y, w, sizeof(T));
    return y;
}

// ---------------------------------------------------------------------------
// Many searches in one persistent launch.  Tiles (search, group, 64 x TPL
// consecutive f0) are listed largest search first; every resident wavefront
// takes the next tile from an atomic counter until the list is exhausted (the
// loop ends for every wave once the counter passes the tile count).  The wave
// that finishes a search's last tile stamps the search's completion time.
template <int STORE, bool MOMENTS, int TPL, int U>
__global__ __launch_bounds__(256) void batch_kernel(const BatchArgs a) {
    // Work is pulled per wavefront.  The loop body has no lane-divergent
    // branch around the tile hand-out: every lane issues the atomic (lane 0
    // adds 1, the others 0) and the wave takes lane 0's ticket as a scalar, so
    // the compiler keeps one wave-uniform loop (a lane-0-only branch there let
    // it split the loop, parking lane 0 while the other lanes re-read a stale
    // ticket forever).  No barrier is used.
    const int lane = threadIdx.x & 63;
    if (threadIdx.x == 0 && a.t_start) atomicMin(a.t_start, (unsigned long long)wall_clock64());
    for (;;) {
        const unsigned ticket = atomicAdd(a.counter, lane == 0 ? 1u : 0u);
        const int tt = __builtin_amdgcn_readfirstlane((int)ticket);
        if (tt >= a.n_tiles) break;
        // descriptors are read into scalar registers (uniform loop bounds, buffer
        // resources and table pointers)
        const BatchTile T = uniform(a.tiles[tt]);
        const BatchSearch *Sp = a.searches + T.search;
        const int n_det = uniform(Sp->n_det), n_f0 = uniform(Sp->n_f0), n_tn = uniform(Sp->n_tn);
        const double f0_min = uniform(Sp->f0_min), f0_step = uniform(Sp->f0_step);
        int i[TPL];
        double f0[TPL];
        for (int t = 0; t < TPL; ++t) {
            i[t] = T.tile * 64 * TPL + t * 64 + lane;
            f0[t] = f0_min + (double)i[t] * f0_step;
        }
        const int tn = T.grp % n_tn, sky = T.grp / n_tn;
        Acc<TPL> acc;
        acc.zero();
        for (int d = 0; d < n_det; ++d) {
            const DetView D = uniform(Sp->det[d]);
            const HFromGD hs{D.g + (int64_t)tn * D.n_seg, D.D + (int64_t)sky * D.n_seg, D.t_sft};
            int jb, je;
            const int runs = D.win ? 64 * TPL / D.win_run : 1;  // the batch's windows are per 64 f0
            seg_window(D, T.grp, T.tile * runs, (T.tile + 1) * runs, jb, je);
            accumulate_det<STORE, MOMENTS, TPL, U>(D, hs, f0, acc, jb, je);
        }
        store_results<MOMENTS, TPL>(acc, i, T.grp, n_f0, uniform(Sp->s), uniform(Sp->c), uniform(Sp->n),
                                    uniform(Sp->w1), uniform(Sp->w2), nullptr, nullptr, nullptr,
                                    a.in_band_total);
        __threadfence();
        unsigned *const tiles_done = uniform(Sp->tiles_done);
        unsigned long long *const t_done = uniform(Sp->t_done);
        const unsigned done = (unsigned)__builtin_amdgcn_readfirstlane(
                                  (int)atomicAdd(tiles_done, lane == 0 ? 1u : 0u)) + 1u;
        if (done == (unsigned)uniform(Sp->n_tiles) && t_done) *t_done = wall_clock64();  // same value, every lane
    }
}

template <int STORE, bool MOMENTS, int TPL, int U>
static hipError_t launch_batch_v(const BatchArgs &a, int grid, hipStream_t st) {
    hipLaunchKernelGGL((batch_kernel<STORE, MOMENTS, TPL, U>), dim3(grid), dim3(256), 0, st, a);
    return hipGetLastError();
}

template <int STORE, bool MOMENTS>
static hipError_t launch_batch_m(int variant, const BatchArgs &a, int grid, hipStream_t st) {
    switch (variant & 3) {
        case 0: return launch_batch_v<STORE, MOMENTS, 1, 8>(a, grid, st);
        case 1: return launch_batch_v<STORE, MOMENTS, 1, 16>(a, grid, st);
        case 2: return launch_batch_v<STORE, MOMENTS, 2, 8>(a, grid, st);
        default: return launch_batch_v<STORE, MOMENTS, 2, 16>(a, grid, st);
    }
}

hipError_t launch_batch(int store, bool moments, int variant, const BatchArgs &a, int grid,
                        hipStream_t st) {
    if (store == LTGW_STORE_F32)
        return moments ? launch_batch_m<LTGW_STORE_F32, true>(variant, a, grid, st)
                       : launch_batch_m<LTGW_STORE_F32, false>(variant, a, grid, st);
    if (store == LTGW_STORE_BF16)
        return moments ? launch_batch_m<LTGW_STORE_BF16, true>(variant, a, grid, st)
                       : launch_batch_m<LTGW_STORE_BF16, false>(variant, a, grid, st);
    return moments ? launch_batch_m<LTGW_STORE_FP8, true>(variant, a, grid, st)
                   : launch_batch_m<LTGW_STORE_FP8, false>(variant, a, grid, st);
}

int batch_blocks_per_cu(int store, bool moments, int variant) {
    int n = 0;
    hipError_t e = hipSuccess;
#define LTGW_OCC(S, M, T, U)                                                                    \
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, batch_kernel<S, M, T, U>, 256, 0)
#define LTGW_OCC_V(S, M)                            \
    switch (variant & 3) {                          \
        case 0: LTGW_OCC(S, M, 1, 8); break;        \
        case 1: LTGW_OCC(S, M, 1, 16); break;       \
        case 2: LTGW_OCC(S, M, 2, 8); break;        \
        default: LTGW_OCC(S, M, 2, 16); break;      \
    }
    if (store == LTGW_STORE_F32) {
        if (moments) { LTGW_OCC_V(LTGW_STORE_F32, true) } else { LTGW_OCC_V(LTGW_STORE_F32, false) }
    } else if (store == LTGW_STORE_BF16) {
        if (moments) { LTGW_OCC_V(LTGW_STORE_BF16, true) } else { LTGW_OCC_V(LTGW_STORE_BF16, false) }
    } else {
        if (moments) { LTGW_OCC_V(LTGW_STORE_FP8, true) } else { LTGW_OCC_V(LTGW_STORE_FP8, false) }
    }
#undef LTGW_OCC_V
#undef LTGW_OCC
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return 1;
    }
    return n < 1 ? 1 : n;
}

// Eq. 2 table for batched searches: D[sky][j] = 1 + ((vx nx + vy ny) + vz nz)/c.
__global__ __launch_bounds__(256) void doppler_kernel(const double *__restrict__ v, int n_seg,
                                                      const double *__restrict__ sky,
                                                      double *__restrict__ D) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    const int s = blockIdx.y;
    if (j >= n_seg) return;
    const double a = v[3 * j + 0] * sky[3 * s + 0];
    const double b = v[3 * j + 1] * sky[3 * s + 1];
    const double z = v[3 * j + 2] * sky[3 * s + 2];
    const double vn = (a + b) + z;
    const double r = vn / kC;
    D[(int64_t)s * n_seg + j] = 1.0 + r;
}

// In-band segment windows.  For a segment, the column index trunc(f0 h +
// 1.5 - k_lo) is non-decreasing in f0, so a run of consecutive f0 has a lane
// in band exactly when its last f0 reaches column 1 and its first f0 is at
// most column n_bins (the statistic kernel's arithmetic).  One wavefront per
// (group, run): lanes stride over the segments, then min / max.
__global__ __launch_bounds__(256) void window_kernel(const DetView D, int n_groups, int n_tn, double f0_min,
                                                     double f0_step, int n_f0, int2 *__restrict__ win) {
    const int lane = threadIdx.x & 63;
    const int per_group = (D.win_blocks + 3) / 4;
    const int grp = blockIdx.x / per_group;
    const int blk = (blockIdx.x % per_group) * 4 + (threadIdx.x >> 6);
    if (blk >= D.win_blocks) return;
    const int ia = blk * D.win_run;
    const int ib = min(ia + D.win_run - 1, n_f0 - 1);
    const double fa = f0_min + (double)ia * f0_step;
    const double fb = f0_min + (double)ib * f0_step;
    const int tn = grp % n_tn, sky = grp / n_tn;
    int lo = D.n_seg, hi = -1;
    for (int j = lane; j < D.n_seg; j += 64) {
        double h;
        if (D.H) {
            h = D.H[(int64_t)grp * D.n_seg + j];
        } else {
            const double hg = D.g[(int64_t)tn * D.n_seg + j] * D.D[(int64_t)sky * D.n_seg + j];
            h = hg * D.t_sft;
        }
        const double xa = fa * h, xb = fb * h;
        const int ca = __double2int_rz(xa + D.cshift), cb = __double2int_rz(xb + D.cshift);
        if (cb >= 1 && ca <= D.n_bins) {
            lo = min(lo, j);
            hi = max(hi, j);
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        lo = min(lo, __shfl_xor(lo, o, 64));
        hi = max(hi, __shfl_xor(hi, o, 64));
    }
    if (lane == 0) win[(int64_t)grp * D.win_blocks + blk] = make_int2(lo, hi);
}

hipError_t launch_windows(const DetView &D, int n_groups, int n_tn, double f0_min, double f0_step, int n_f0,
                          int2 *win, hipStream_t st) {
    const int64_t blocks = (int64_t)((D.win_blocks + 3) / 4) * n_groups;
    if (n_groups < 1 || D.win_blocks < 1 || blocks > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(window_kernel, dim3((unsigned)blocks), dim3(256), 0, st, D, n_groups, n_tn, f0_min, f0_step,
                       n_f0, win);
    return hipGetLastError();
}

hipError_t launch_doppler(const double *v, int32_t n_seg, const double *sky, int32_t n_sky,
                          double *D, hipStream_t st) {
    hipLaunchKernelGGL(doppler_kernel, dim3((n_seg + 255) / 256, n_sky), dim3(256), 0, st, v, n_seg,
                       sky, D);
    return hipGetLastError();
}

__global__ void fill_u32_kernel(unsigned *p, int n, unsigned v) {
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) p[i] = v;
}
__global__ void fill_u64_kernel(unsigned long long *p, int n, unsigned long long v) {
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) p[i] = v;
}

hipError_t launch_fill_u32(unsigned *p, int n, unsigned v, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_u32_kernel, dim3((n + 255) / 256 < 1024 ? (n + 255) / 256 : 1024), dim3(256),
                       0, st, p, n, v);
    return hipGetLastError();
}
__global__ void f64_to_f32_kernel(const double *in, float *out, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        out[i] = (float)in[i];
}

hipError_t launch_f64_to_f32(const double *in, float *out, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(f64_to_f32_kernel, dim3((unsigned)(blocks < 4096 ? blocks : 4096)), dim3(256), 0, st,
                       in, out, n);
    return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long *p, int n, unsigned long long v, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_u64_kernel, dim3((n + 255) / 256 < 1024 ? (n + 255) / 256 : 1024), dim3(256),
                       0, st, p, n, v);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Stacks of realisations (the learned proposer's data): R spectrograms of one
// geometry, realisation r at byte offset r * stack_bytes of the store and
// r * stack_rows of the per-row weights.  One launch evaluates every template
// of a grid on every realisation and writes the power critical ratio
//     Psi = (s - mu W1) / sqrt(var W2)
// with the per-pixel noise mean mu and variance var of the store (Exp(1):
// 1, 1; a 2x2 sum of Exp(1): 4, 4), NaN (or 0 with nan_to_zero) for N = 0.
template <int STORE, int SHIFT>
__global__ __launch_bounds__(256) void stack_eval_kernel(const EvalArgs a, int64_t stack_bytes,
                                                         int64_t stack_rows, double mu, double var,
                                                         int nan_to_zero, double *__restrict__ out_psi,
                                                         int32_t *__restrict__ out_c) {
    const int n_tiles = (a.n_f0 + 255) / 256;
    int tile, grp;
    xcd_tile_group(blockIdx.x, gridDim.x, n_tiles, tile, grp);
    const int r = blockIdx.y;
    int i[1] = {tile * 256 + (int)threadIdx.x};
    double f0[1] = {a.f0_min + (double)i[0] * a.f0_step};
    DetView D = a.det[0];
    D.store = (const char *)D.store + (int64_t)r * stack_bytes;
    D.wq += (int64_t)r * stack_rows;
    D.w += (int64_t)r * stack_rows;
    Acc<1> acc;
    acc.zero();
    accumulate_det<STORE, true, 1, 16, HTable, SHIFT>(D, HTable{D.H + (int64_t)grp * D.n_seg}, f0, acc);
    if (i[0] >= a.n_f0) return;
    const int64_t t = (int64_t)r * ((int64_t)a.n_groups * a.n_f0) + (int64_t)grp * a.n_f0 + i[0];
    double psi;
    if (acc.nin[0] == 0) {
        psi = nan_to_zero ? 0.0 : __builtin_nan("");
    } else {
        const double num = acc.s[0] - mu * acc.w1[0];
        psi = num / sqrt(var * acc.w2[0]);
    }
    out_psi[t] = psi;
    if (out_c) out_c[t] = acc.cnt[0];
}

hipError_t launch_stack_eval(int store, int shift, const EvalArgs &a, int R, int64_t stack_bytes,
                             int64_t stack_rows, double mu, double var, int nan_to_zero,
                             double *out_psi, int32_t *out_c, hipStream_t st) {
    const int64_t blocks = (int64_t)((a.n_f0 + 255) / 256) * a.n_groups;
    if (blocks > 0x7fffffff || R > 65535 || R < 1) return hipErrorInvalidValue;
    dim3 grid((unsigned)blocks, (unsigned)R), block(256);
    if (store == LTGW_STORE_F32 && shift == 0)
        hipLaunchKernelGGL((stack_eval_kernel<LTGW_STORE_F32, 0>), grid, block, 0, st, a, stack_bytes, stack_rows, mu, var, nan_to_zero, out_psi, out_c);
    else if (store == LTGW_STORE_BF16 && shift == 0)
        hipLaunchKernelGGL((stack_eval_kernel<LTGW_STORE_BF16, 0>), grid, block, 0, st, a, stack_bytes, stack_rows, mu, var, nan_to_zero, out_psi, out_c);
    else if (store == LTGW_STORE_BF16 && shift == 1)
        hipLaunchKernelGGL((stack_eval_kernel<LTGW_STORE_BF16, 1>), grid, block, 0, st, a, stack_bytes, stack_rows, mu, var, nan_to_zero, out_psi, out_c);
    else if (store == LTGW_STORE_FP8 && shift == 0)
        hipLaunchKernelGGL((stack_eval_kernel<LTGW_STORE_FP8, 0>), grid, block, 0, st, a, stack_bytes, stack_rows, mu, var, nan_to_zero, out_psi, out_c);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

// Explicit template lists: lane q of realisation r evaluates template
// idx[r][q] of the grid (any order; each lane reads its own group's track
// factors).  Writes the power critical ratio (mu = var = 1) or NaN.
template <int STORE>
__global__ __launch_bounds__(256) void list_eval_kernel(const EvalArgs a, int64_t stack_bytes,
                                                        int64_t stack_rows, const int32_t *__restrict__ idx,
                                                        int m, const int32_t *__restrict__ rmap,
                                                        double *__restrict__ out_psi) {
    const int q = blockIdx.x * 256 + threadIdx.x;
    const int rr = blockIdx.y;                  // row of idx and out_psi
    const int r = rmap ? rmap[rr] : rr;         // realisation of the stack
    DetView D = a.det[0];
    D.store = (const char *)D.store + (int64_t)r * stack_bytes;
    D.wq += (int64_t)r * stack_rows;
    D.w += (int64_t)r * stack_rows;
    const int64_t n_tpl = (int64_t)a.n_groups * a.n_f0;
    int t = q < m ? idx[(int64_t)rr * m + q] : 0;
    const bool bad = t < 0 || t >= n_tpl;  // not a template of the grid: NaN
    if (bad) t = 0;
    const int i_f0 = t % a.n_f0, grp = t / a.n_f0;
    const double f0 = a.f0_min + (double)i_f0 * a.f0_step;
    const double *__restrict__ H = D.H + (int64_t)grp * D.n_seg;
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        (void *)D.store, Store<STORE>::kBytes, D.n_bins + 2, kBufDword3);
    const unsigned nb = (unsigned)D.n_bins;
    double s = 0.0, w1 = 0.0, w2 = 0.0;
    int cnt = 0, nin = 0;
    for (int j0 = 0; j0 < D.n_seg; j0 += kChunk) {
        const int je = min(j0 + kChunk, D.n_seg);
        float sc = 0.0f, w1c = 0.0f, w2c = 0.0f;
        int j = j0;
        // batches of 8 segments: the track factors, then the gathers, then the
        // sums in segment order (the same sums as one segment at a time)
        for (; j + 8 <= je; j += 8) {
            unsigned ix[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const double x = f0 * H[j + k];
                const double vv = x + D.cshift;
                ix[k] = (unsigned)__double2int_rz(vv);
            }
            float p[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) p[k] = Store<STORE>::get(rs, (int)ix[k], (j + k) * D.pitch_bytes, cnt);
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                sc = __builtin_fmaf(D.wq[j + k], p[k], sc);
                const bool inb = (ix[k] - 1u) < nb;
                nin += inb ? 1 : 0;
                const float wj = inb ? D.w[j + k] : 0.0f;
                w1c += wj;
                w2c = __builtin_fmaf(wj, wj, w2c);
            }
        }
        for (; j < je; ++j) {
            const double x = f0 * H[j];
            const double vv = x + D.cshift;
            const unsigned ix = (unsigned)__double2int_rz(vv);
            const float p = Store<STORE>::get(rs, (int)ix, j * D.pitch_bytes, cnt);
            sc = __builtin_fmaf(D.wq[j], p, sc);
            const bool inb = (ix - 1u) < nb;
            nin += inb ? 1 : 0;
            const float wj = inb ? D.w[j] : 0.0f;
            w1c += wj;
            w2c = __builtin_fmaf(wj, wj, w2c);
        }
        s += (double)sc;
        w1 += (double)w1c;
        w2 += (double)w2c;
    }
    if (q >= m) return;
    out_psi[(int64_t)rr * m + q] = (nin && !bad) ? (s - w1) / sqrt(w2) : __builtin_nan("");
}

hipError_t launch_list_eval(int store, const EvalArgs &a, int R, int64_t stack_bytes, int64_t stack_rows,
                            const int32_t *idx, int m, const int32_t *rmap, double *out_psi, hipStream_t st) {
    if (R > 65535 || R < 1 || m < 1) return hipErrorInvalidValue;
    dim3 grid((unsigned)((m + 255) / 256), (unsigned)R), block(256);
    if (store == LTGW_STORE_F32)
        hipLaunchKernelGGL(list_eval_kernel<LTGW_STORE_F32>, grid, block, 0, st, a, stack_bytes, stack_rows, idx, m, rmap, out_psi);
    else if (store == LTGW_STORE_BF16)
        hipLaunchKernelGGL(list_eval_kernel<LTGW_STORE_BF16>, grid, block, 0, st, a, stack_bytes, stack_rows, idx, m, rmap, out_psi);
    else
        hipLaunchKernelGGL(list_eval_kernel<LTGW_STORE_FP8>, grid, block, 0, st, a, stack_bytes, stack_rows, idx, m, rmap, out_psi);
    return hipGetLastError();
}

// Cells of the network's output (channel ch, position l of L) to fine
// templates: group ch / 2, f0 index 2 l + ch % 2 (fine n_f0 = 2 L).
__global__ void cells_to_templates_kernel(const int32_t *cells, int64_t n, int L, int32_t *tpl) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int cell = cells[i];
    const int ch = cell / L, l = cell % L;
    tpl[i] = (ch / 2) * (2 * L) + 2 * l + (ch % 2);
}

hipError_t launch_cells_to_templates(const int32_t *cells, int64_t n, int L, int32_t *tpl, hipStream_t st) {
    hipLaunchKernelGGL(cells_to_templates_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, cells,
                       n, L, tpl);
    return hipGetLastError();
}

// Proposal blocks: runs of W consecutive fine f0 of one fine group (block k
// of group g covers f0 indices [k W, k W + W) of the 2 L).  The score of a
// block is the largest network logit of its cells (cell of fine (g, i):
// (2 g + i % 2) L + i / 2).  One thread per (realisation, block).
__global__ void block_scores_kernel(const float *logits, int64_t total, int c_out, int L, int W, int nbg,
                                    float *score) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= total) return;
    const int G = c_out / 2;
    const int64_t r = e / ((int64_t)G * nbg);
    const int rem = (int)(e % ((int64_t)G * nbg));
    const int g = rem / nbg, k = rem % nbg;
    const float *z = logits + r * (int64_t)c_out * L;
    float m = -__builtin_inff();
    for (int j = 0; j < W; ++j) {
        const int i = k * W + j;
        if (i >= 2 * L) break;
        const float v = z[(2 * g + (i & 1)) * L + (i >> 1)];
        m = v > m ? v : m;
    }
    score[e] = m;
}

hipError_t launch_block_scores(const float *logits, int R, int c_out, int L, int W, int nbg, float *score,
                               hipStream_t st) {
    const int64_t total = (int64_t)R * (c_out / 2) * nbg;
    hipLaunchKernelGGL(block_scores_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, logits, total,
                       c_out, L, W, nbg, score);
    return hipGetLastError();
}

// Scores of the blocks already taken (blk[r][0..K)) become NaN, which ranks last.
__global__ void mask_blocks_kernel(float *score, const int32_t *blk, int64_t total, int K, int nb) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= total) return;
    const int64_t r = e / K;
    const int b = blk[e];
    if (b >= 0 && b < nb) score[r * nb + b] = __builtin_nanf("");
}

hipError_t launch_mask_blocks(float *score, const int32_t *blk, int R, int K, int nb, hipStream_t st) {
    const int64_t total = (int64_t)R * K;
    hipLaunchKernelGGL(mask_blocks_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, score, blk, total,
                       K, nb);
    return hipGetLastError();
}

// Templates of the selected blocks: row q (realisation rmap[q], or q)
// lists blk[r][0..K) expanded to W consecutive f0 each (-1 past the grid).
__global__ void expand_blocks_kernel(const int32_t *blk, int K, int W, int two_L, int nbg, const int32_t *rmap,
                                     int64_t total, int32_t *tpl) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= total) return;
    const int64_t row = e / ((int64_t)K * W);
    const int rem = (int)(e % ((int64_t)K * W));
    const int q = rem / W, j = rem % W;
    const int64_t r = rmap ? rmap[row] : row;
    const int b = blk[r * K + q];
    const int g = b / nbg, i = (b % nbg) * W + j;
    tpl[e] = (b >= 0 && i < two_L) ? g * two_L + i : -1;
}

hipError_t launch_expand_blocks(const int32_t *blk, int K, int W, int two_L, int nbg, const int32_t *rmap, int rows,
                                int32_t *tpl, hipStream_t st) {
    const int64_t total = (int64_t)rows * K * W;
    hipLaunchKernelGGL(expand_blocks_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, blk, K, W,
                       two_L, nbg, rmap, total, tpl);
    return hipGetLastError();
}

// Each row of m template indices into ascending order (bitonic sort in LDS,
// one workgroup per row): neighbouring lanes of the listed evaluation then
// take neighbouring f0 wherever the selection is contiguous, so their gathers
// share cache lines.
constexpr int kSortMax = 8192;
__global__ __launch_bounds__(256) void sort_rows_kernel(int32_t *idx, int m) {
    __shared__ int32_t v[kSortMax];
    int32_t *row = idx + (int64_t)blockIdx.x * m;
    int P = 1;
    while (P < m) P <<= 1;
    for (int i = threadIdx.x; i < P; i += 256) v[i] = i < m ? row[i] : 0x7fffffff;
    __syncthreads();
    for (int size = 2; size <= P; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = threadIdx.x; i < P; i += 256) {
                const int j = i ^ stride;
                if (j > i) {
                    const bool up = (i & size) == 0;
                    const int32_t a = v[i], b = v[j];
                    if (up ? a > b : a < b) {
                        v[i] = b;
                        v[j] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int i = threadIdx.x; i < m; i += 256) row[i] = v[i];
}

hipError_t launch_sort_rows(int32_t *idx, int rows, int m, hipStream_t st) {
    if (rows < 1 || m < 1 || m > kSortMax) return hipErrorInvalidValue;
    hipLaunchKernelGGL(sort_rows_kernel, dim3(rows), dim3(256), 0, st, idx, m);
    return hipGetLastError();
}

// The fallback rule per realisation (one workgroup per row): the largest
// coarse ratio above cthr while the best listed fine ratio does not pass thr.
__global__ __launch_bounds__(256) void fallback_kernel(const double *psi_coarse, int nc, const double *best_psi,
                                                       double thr, double cthr, int32_t *fallback) {
    __shared__ double sh[4];
    const int64_t r = blockIdx.x;
    double cm = -__builtin_inf();
    for (int q = threadIdx.x; q < nc; q += 256) {
        const double v = psi_coarse[r * nc + q];
        if (v == v && v > cm) cm = v;
    }
    for (int o = 32; o > 0; o >>= 1) cm = fmax(cm, __shfl_xor(cm, o, 64));
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = cm;
    __syncthreads();
    if (threadIdx.x == 0) {
        cm = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
        const double b = best_psi[r];
        fallback[r] = (cm > cthr && !(b > thr)) ? 1 : 0;
    }
}

hipError_t launch_fallback(int R, const double *psi_coarse, int nc, const double *best_psi, double thr,
                           double cthr, int32_t *fallback, hipStream_t st) {
    if (R < 1 || nc < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(fallback_kernel, dim3(R), dim3(256), 0, st, psi_coarse, nc, best_psi, thr, cthr, fallback);
    return hipGetLastError();
}

// Best entry of each row of psi[rows][n] (largest finite value, ties to the
// lowest index; index = position, or idx[row][position] when idx is given):
// one block per row, strided scan and an LDS tree.  No finite value: -1, -inf.
__device__ inline bool best_before(double a, int ia, double b, int ib) {
    return a > b || (a == b && (unsigned)ia < (unsigned)ib);
}

__global__ __launch_bounds__(256) void row_best_kernel(const double *psi, int64_t n, const int32_t *idx,
                                                       int32_t *best_idx, double *best_psi) {
    __shared__ double sv[256];
    __shared__ int si[256];
    const int64_t row = blockIdx.x;
    double b = -__builtin_inf();
    int bi = -1;
    for (int64_t q = threadIdx.x; q < n; q += 256) {
        const double v = psi[row * n + q];
        const int t = idx ? idx[row * n + q] : (int)q;
        if (v == v && (bi < 0 || best_before(v, t, b, bi))) {
            b = v;
            bi = t;
        }
    }
    sv[threadIdx.x] = b;
    si[threadIdx.x] = bi;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            const double v = sv[threadIdx.x + w];
            const int t = si[threadIdx.x + w];
            if (t >= 0 && (si[threadIdx.x] < 0 || best_before(v, t, sv[threadIdx.x], si[threadIdx.x]))) {
                sv[threadIdx.x] = v;
                si[threadIdx.x] = t;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        best_idx[row] = si[0];
        best_psi[row] = si[0] < 0 ? -__builtin_inf() : sv[0];
    }
}

hipError_t launch_row_best(const double *psi, int rows, int64_t n, const int32_t *idx, int32_t *best_idx,
                           double *best_psi, hipStream_t st) {
    if (rows < 1 || n < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(row_best_kernel, dim3(rows), dim3(256), 0, st, psi, n, idx, best_idx, best_psi);
    return hipGetLastError();
}

// Fine templates to network cells (fine n_f0 = 2 L): template (group g, f0
// index i) is cell (2 g + i % 2) L + i / 2; -1 where mask[r] == 0, tpl < 0,
// or psi (when given) is not above min_psi.
__global__ void templates_to_cells_kernel(const int32_t *tpl, int n, int L, const int32_t *mask,
                                          const double *psi, double min_psi, int32_t *cells) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int t = tpl[i];
    if (t < 0 || (mask && mask[i] == 0) || (psi && !(psi[i] > min_psi))) {
        cells[i] = -1;
        return;
    }
    const int g = t / (2 * L), f = t % (2 * L);
    cells[i] = (2 * g + (f & 1)) * L + (f >> 1);
}

hipError_t launch_templates_to_cells(const int32_t *tpl, int n, int L, const int32_t *mask, const double *psi,
                                     double min_psi, int32_t *cells, hipStream_t st) {
    hipLaunchKernelGGL(templates_to_cells_kernel, dim3((n + 255) / 256), dim3(256), 0, st, tpl, n, L, mask, psi,
                       min_psi, cells);
    return hipGetLastError();
}

// Every template index of a grid, once per listed realisation.
__global__ void iota_rows_kernel(int32_t *idx, int rows, int n) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < (int64_t)rows * n) idx[i] = (int32_t)(i % n);
}

hipError_t launch_iota_rows(int32_t *idx, int rows, int n, hipStream_t st) {
    const int64_t t = (int64_t)rows * n;
    hipLaunchKernelGGL(iota_rows_kernel, dim3((unsigned)((t + 255) / 256)), dim3(256), 0, st, idx, rows, n);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// In-band moments (N, W1, W2) without touching the spectrogram.  For a fixed
// (group, segment) the column index trunc(f0_i*H + 1.5 - k_lo) is a
// non-decreasing function of i (every step is monotone), so the in-band
// templates are the contiguous range [lo, hi) with lo the first i whose
// index reaches 1 and hi the first whose index passes n_bins.  Both are
// found by binary search with exactly the statistic kernel's arithmetic.
__device__ inline int col_index(double f0_min, double f0_step, int i, double H, double cshift) {
    const double f0 = f0_min + (double)i * f0_step;
    const double x = f0 * H;
    const double vv = x + cshift;
    return __double2int_rz(vv);
}

// first i in [0, n] with col_index(i) >= target (n if none)
__device__ inline int first_at_least(double f0_min, double f0_step, int n, double H,
                                     double cshift, int target) {
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = lo + ((hi - lo) >> 1);
        if (col_index(f0_min, f0_step, mid, H, cshift) >= target)
            hi = mid;
        else
            lo = mid + 1;
    }
    return lo;
}

// Each lane takes kMomSeg consecutive segments of one group and merges
// consecutive equal range ends before adding them, so the many segments that
// share an end (every template in band: lo = 0, hi = n_f0) cost one atomic
// per lane instead of one per segment.
constexpr int kMomSeg = 32;

struct RangeRun {
    int key = -1;
    unsigned long long v[4] = {0, 0, 0, 0};
};

__device__ inline void flush_run(RangeRun &r, unsigned long long *base, int64_t stride, int na,
                                 bool negate) {
    if (r.key < 0) return;
    for (int q = 0; q < na; ++q)
        if (r.v[q]) atomicAdd(base + q * stride + r.key, negate ? (unsigned long long)(-(long long)r.v[q]) : r.v[q]);
    r.key = -1;
    for (int q = 0; q < 4; ++q) r.v[q] = 0;
}

__device__ inline void add_run(RangeRun &r, int key, const unsigned long long *val, int na,
                               unsigned long long *base, int64_t stride, bool negate) {
    if (key != r.key) {
        flush_run(r, base, stride, na, negate);
        r.key = key;
    }
    for (int q = 0; q < na; ++q) r.v[q] += val[q];
}

__global__ __launch_bounds__(256) void moments_ranges_kernel(const EvalArgs a, int weights,
                                                             int64_t *__restrict__ diff) {
    const int d = blockIdx.z;
    const DetView D = a.det[d];
    const int row = blockIdx.y;
    const int j0 = (blockIdx.x * 256 + threadIdx.x) * kMomSeg;
    const int64_t stride = (int64_t)a.n_groups * (a.n_f0 + 1);
    unsigned long long *base = (unsigned long long *)diff + (int64_t)row * (a.n_f0 + 1);
    const int na = weights ? 4 : 1;
    RangeRun rlo, rhi;
    unsigned long long inb = 0;
    const int j1 = min(j0 + kMomSeg, D.n_seg);
    const int tn = row % a.n_tn, sky = row / a.n_tn;
    for (int j = j0; j < j1; ++j) {
        double H;
        if (D.H) {
            H = D.H[(int64_t)row * D.n_seg + j];
        } else {
            const double h = D.g[(int64_t)tn * D.n_seg + j] * D.D[(int64_t)sky * D.n_seg + j];
            H = h * D.t_sft;
        }
        const int lo = first_at_least(a.f0_min, a.f0_step, a.n_f0, H, D.cshift, 1);
        const int hi = first_at_least(a.f0_min, a.f0_step, a.n_f0, H, D.cshift, D.n_bins + 1);
        if (lo >= hi) continue;
        inb += (unsigned long long)(hi - lo);
        unsigned long long val[4] = {1ull, 0ull, 0ull, 0ull};
        if (weights)
            for (int q = 0; q < 3; ++q) val[q + 1] = (unsigned long long)D.wfix[3 * j + q];
        add_run(rlo, lo, val, na, base, stride, false);
        add_run(rhi, hi, val, na, base, stride, true);
    }
    flush_run(rlo, base, stride, na, false);
    flush_run(rhi, base, stride, na, true);
    for (int o = 32; o > 0; o >>= 1) inb += __shfl_xor(inb, o, 64);
    if ((threadIdx.x & 63) == 0 && inb && a.in_band_total) atomicAdd(a.in_band_total, inb);
}

// One block per group: prefix sums of the difference arrays over f0, in tiles
// of 256 consecutive positions (coalesced), with a running carry.
__device__ inline int64_t block_inclusive_scan_256(int64_t v, int64_t *sh, int64_t &total) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int o = 1; o < 64; o <<= 1) {
        const int64_t u = __shfl_up(v, o, 64);
        if (lane >= o) v += u;
    }
    if (lane == 63) sh[wv] = v;
    __syncthreads();
    int64_t off = 0;
    for (int k = 0; k < wv; ++k) off += sh[k];
    total = sh[0] + sh[1] + sh[2] + sh[3];
    __syncthreads();
    return v + off;
}

__global__ __launch_bounds__(256) void moments_scan_kernel(const EvalArgs a, int weights, int e0,
                                                           const int64_t *__restrict__ diff) {
    __shared__ int64_t sh[4];
    const int row = blockIdx.x;
    const int n = a.n_f0;
    const int64_t stride = (int64_t)a.n_groups * (n + 1);
    const int64_t *base = diff + (int64_t)row * (n + 1);
    const int na = weights ? 4 : 1;
    int64_t carry[4] = {0, 0, 0, 0};
    const double wu = (double)a.w_uniform;
    for (int i0 = 0; i0 < n; i0 += 256) {
        const int i = i0 + threadIdx.x;
        int64_t run[4] = {0, 0, 0, 0};
        for (int q = 0; q < na; ++q) {
            const int64_t v = i < n ? base[q * stride + i] : 0;
            int64_t tot;
            run[q] = block_inclusive_scan_256(v, sh, tot) + carry[q];
            carry[q] += tot;
        }
        if (i < n) {
            const int64_t t = (int64_t)row * n + i;
            const int nin = (int)run[0];
            double w1, w2;
            if (weights) {
                w1 = ldexp((double)run[1], e0);
                w2 = ldexp((double)run[2] * 4294967296.0 + (double)run[3], 2 * e0);
            } else {
                w1 = (double)nin * wu;
                w2 = (double)nin * (wu * wu);
            }
            a.n[t] = nin;
            a.w1[t] = w1;
            a.w2[t] = w2;
            if (a.out_n) a.out_n[t] = nin;
        }
    }
}

__global__ void zero_i64_kernel(int64_t *p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        p[i] = 0;
}

hipError_t launch_moments(const EvalArgs &a, int weights, int e0, int64_t *diff, hipStream_t st) {
    const int64_t n_entries = (int64_t)(weights ? 4 : 1) * a.n_groups * (a.n_f0 + 1);
    hipLaunchKernelGGL(zero_i64_kernel, dim3(1024), dim3(256), 0, st, diff, n_entries);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    int max_seg = 0;
    for (int d = 0; d < a.n_det; ++d) max_seg = a.det[d].n_seg > max_seg ? a.det[d].n_seg : max_seg;
    const int lanes = (max_seg + kMomSeg - 1) / kMomSeg;
    hipLaunchKernelGGL(moments_ranges_kernel, dim3((lanes + 255) / 256, a.n_groups, a.n_det),
                       dim3(256), 0, st, a, weights, diff);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(moments_scan_kernel, dim3(a.n_groups), dim3(256), 0, st, a, weights, e0,
                       (const int64_t *)diff);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Eq. 4 critical ratios.
__device__ inline double psi_of(uint32_t stat, int64_t t, const double *s, const int32_t *c,
                                const int32_t *N, const double *w1, const double *w2, double q) {
    const int32_t nn = N[t];
    if (nn == 0) return __builtin_nan("");
    if (stat == LTGW_STAT_POWER) {
        const double num = s[t] - w1[t];
        return num / sqrt(w2[t]);
    }
    const double Nq = (double)nn * q;
    const double num = (double)c[t] - Nq;
    const double var = Nq * (1.0 - q);
    return num / sqrt(var);
}

__global__ __launch_bounds__(256) void psi_kernel(uint32_t stat, int64_t n, const double *s,
                                                  const int32_t *c, const int32_t *N,
                                                  const double *w1, const double *w2, double q,
                                                  double *out) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t < n) out[t] = psi_of(stat, t, s, c, N, w1, w2, q);
}

hipError_t launch_psi(uint32_t stat, int64_t n, const double *s, const int32_t *c,
                      const int32_t *N, const double *w1, const double *w2, double q,
                      double *out, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(psi_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, stat, n, s,
                       c, N, w1, w2, q, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Top-k by (psi desc, index asc).  A block takes 4096 items into registers
// (16 per lane) and extracts its k best by k rounds of a block-wide arg-max;
// levels repeat over the per-block winners until one block remains.
constexpr int kTopkIpt = 16;
constexpr int kTopkChunk = 256 * kTopkIpt;
constexpr int64_t kNoIndex = 0x7fffffffffffffffll;

__device__ inline bool better(double pa, int64_t ia, double pb, int64_t ib) {
    return pa > pb || (pa == pb && ia < ib);
}

template <bool FROM_RESULTS>
__global__ __launch_bounds__(256) void topk_level_kernel(
    int64_t n, int32_t k, uint32_t stat, const double *s, const int32_t *c, const int32_t *N,
    const double *w1, const double *w2, double q, const double *in_psi, const int64_t *in_idx,
    double *out_psi, int64_t *out_idx) {
    __shared__ double sp[4];
    __shared__ int64_t si[4];
    double pv[kTopkIpt];
    int64_t iv[kTopkIpt];
    const int64_t base = (int64_t)blockIdx.x * kTopkChunk;
#pragma unroll
    for (int u = 0; u < kTopkIpt; ++u) {
        const int64_t t = base + (int64_t)u * 256 + threadIdx.x;
        double p = -__builtin_inf();
        int64_t id = kNoIndex;
        if (t < n) {
            if (FROM_RESULTS) {
                p = psi_of(stat, t, s, c, N, w1, w2, q);
                id = t;
            } else {
                p = in_psi[t];
                id = in_idx[t];
            }
            if (!(p == p) || id == kNoIndex) {  // NaN: never ranks
                p = -__builtin_inf();
                id = kNoIndex;
            }
        }
        pv[u] = p;
        iv[u] = id;
    }
    for (int r = 0; r < k; ++r) {
        double bp = -__builtin_inf();
        int64_t bi = kNoIndex;
#pragma unroll
        for (int u = 0; u < kTopkIpt; ++u)
            if (iv[u] != kNoIndex && better(pv[u], iv[u], bp, bi)) {
                bp = pv[u];
                bi = iv[u];
            }
        for (int o = 32; o > 0; o >>= 1) {
            const double op = __shfl_xor(bp, o, 64);
            const int64_t oi = __shfl_xor(bi, o, 64);
            if (oi != kNoIndex && (bi == kNoIndex || better(op, oi, bp, bi))) {
                bp = op;
                bi = oi;
            }
        }
        if ((threadIdx.x & 63) == 0) {
            sp[threadIdx.x >> 6] = bp;
            si[threadIdx.x >> 6] = bi;
        }
        __syncthreads();
        bp = sp[0];
        bi = si[0];
        for (int wv = 1; wv < 4; ++wv)
            if (si[wv] != kNoIndex && (bi == kNoIndex || better(sp[wv], si[wv], bp, bi))) {
                bp = sp[wv];
                bi = si[wv];
            }
        // block-uniform values from LDS, made scalar so the early exit below
        // is a uniform branch (barriers inside the loop)
        bi = ((int64_t)__builtin_amdgcn_readfirstlane((int)(bi >> 32)) << 32) |
             (int64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)bi);
        __syncthreads();
        if (threadIdx.x == 0) {
            out_psi[(int64_t)blockIdx.x * k + r] = bp;
            out_idx[(int64_t)blockIdx.x * k + r] = bi;
        }
        if (bi == kNoIndex) {
            // no valid item left: pad the rest
            for (int r2 = r + 1 + (int)threadIdx.x; r2 < k; r2 += 256) {
                out_psi[(int64_t)blockIdx.x * k + r2] = -__builtin_inf();
                out_idx[(int64_t)blockIdx.x * k + r2] = kNoIndex;
            }
            break;
        }
#pragma unroll
        for (int u = 0; u < kTopkIpt; ++u)
            if (iv[u] == bi) {
                iv[u] = kNoIndex;
                pv[u] = -__builtin_inf();
            }
    }
}

__global__ void topk_records_kernel(int32_t k, uint32_t stat, const double *s, const int32_t *c,
                                    const int32_t *N, const double *psi, const int64_t *idx,
                                    TopkDecode dec, ltgw_candidate *out, int32_t *n_out) {
    const int r = threadIdx.x;
    if (r == 0) {
        int cntv = 0;
        for (int u = 0; u < k; ++u)
            if (idx[u] != kNoIndex) ++cntv;
        *n_out = cntv;
    }
    if (r >= k) return;
    const int64_t t = idx[r];
    ltgw_candidate rec;
    if (t == kNoIndex) {
        rec.index = -1;
        rec.f0 = rec.tau = rec.brake = rec.stat = rec.psi = 0.0;
        rec.sky = -1;
        rec.n_valid = 0;
    } else {
        const int64_t i_f0 = t % dec.n_f0;
        const int64_t grp = t / dec.n_f0;
        const int64_t i_tau = grp % dec.n_tau;
        const int64_t rr = grp / dec.n_tau;
        rec.index = t;
        rec.f0 = dec.f0_min + (double)i_f0 * dec.f0_step;
        rec.tau = dec.tau[i_tau];
        rec.brake = dec.brake[rr % dec.n_brake];
        rec.sky = (int32_t)(rr / dec.n_brake);
        rec.n_valid = N[t];
        rec.stat = stat == LTGW_STAT_POWER ? s[t] : (double)c[t];
        rec.psi = psi[r];
    }
    out[r] = rec;
}

int64_t topk_scratch_entries(int64_t n, int32_t k) {
    return ((n + kTopkChunk - 1) / kTopkChunk) * (int64_t)k + k;
}

hipError_t launch_topk(uint32_t stat, int64_t n, const double *s, const int32_t *c,
                       const int32_t *N, const double *w1, const double *w2, double q, int32_t k,
                       double *pa, int64_t *ia, double *pb, int64_t *ib, int64_t cand_cap,
                       const TopkDecode &dec, ltgw_candidate *out_dev, int32_t *n_out_dev,
                       hipStream_t st) {
    int64_t blocks = (n + kTopkChunk - 1) / kTopkChunk;
    if (blocks < 1) blocks = 1;
    if (blocks * k > cand_cap) return hipErrorInvalidValue;
    hipLaunchKernelGGL(topk_level_kernel<true>, dim3((unsigned)blocks), dim3(256), 0, st, n, k, stat,
                       s, c, N, w1, w2, q, (const double *)nullptr, (const int64_t *)nullptr, pa, ia);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    int64_t m = blocks * k;
    while (blocks > 1) {
        blocks = (m + kTopkChunk - 1) / kTopkChunk;
        hipLaunchKernelGGL(topk_level_kernel<false>, dim3((unsigned)blocks), dim3(256), 0, st, m, k,
                           stat, s, c, N, w1, w2, q, pa, ia, pb, ib);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        m = blocks * k;
        double *tp = pa;
        pa = pb;
        pb = tp;
        int64_t *ti = ia;
        ia = ib;
        ib = ti;
    }
    hipLaunchKernelGGL(topk_records_kernel, dim3(1), dim3(256), 0, st, k, stat, s, c, N, pa, ia, dec,
                       out_dev, n_out_dev);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Synthetic injection (Sec. 3): add amp*w_j at the template's bin, one thread
// per segment, same arithmetic as the evaluation.
__global__ __launch_bounds__(256) void inject_kernel(float *power, int n_seg, int n_bins,
                                                     int64_t k_lo, double t_sft,
                                                     const double *t_seg, const double *v,
                                                     const float *w, double f0, double tau,
                                                     double brake, double sx, double sy, double sz,
                                                     double t0, float amp,
                                                     unsigned long long *undecided) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= n_seg) return;
    const double t = t_seg[j];
    if (t < t0) return;
    const double d = t - t0;
    const double qq = d / tau;
    const double u = 1.0 + qq;
    const double e = 1.0 / (1.0 - brake);
    int und = 0;
    const double g = pow_cr(u, e, &und);
    if (und) atomicAdd(undecided, 1ull);
    const double a = v[3 * j + 0] * sx;
    const double b = v[3 * j + 1] * sy;
    const double z = v[3 * j + 2] * sz;
    const double vn = (a + b) + z;
    const double D = 1.0 + vn / kC;
    const double h = g * D;
    const double H = h * t_sft;
    const double x = f0 * H;
    const double y = x + 0.5;
    const int64_t bin = (int64_t)floor(y) - k_lo;
    if (bin < 0 || bin >= n_bins) return;
    float *px = power + (int64_t)j * n_bins + bin;
    *px = *px + amp * w[j];
}

hipError_t launch_inject(float *power, int32_t n_seg, int32_t n_bins, int64_t k_lo,
                         double t_sft, const double *t_seg, const double *v, const float *w,
                         double f0, double tau, double brake, double sx, double sy, double sz,
                         double t0, float amp, unsigned long long *undecided, hipStream_t st) {
    hipLaunchKernelGGL(inject_kernel, dim3((n_seg + 255) / 256), dim3(256), 0, st, power, n_seg,
                       n_bins, k_lo, t_sft, t_seg, v, w, f0, tau, brake, sx, sy, sz, t0, amp,
                       undecided);
    return hipGetLastError();
}

}  // namespace ltgw
