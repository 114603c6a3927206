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
#include "ltgw_gather.h"
#include "ltgw_internal.h"
#include "ddpow.h"

#pragma clang fp contract(off)

namespace ltgw {

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

// Stack ingest with the proposer's coarse store in the same pass: workgroup
// (j2, r) reads the S fine rows S j2 .. S j2 + S - 1 of realisation r once and
//  - writes them to the fine store: the codes, count bits and FP8 scales of
//    ingest_kernel, bit for bit;
//  - writes coarse pixel m of coarse row j2 (column m + 1; columns 0 and
//    nb2 + 1 .. pitch2 - 1 are 0 guards): the FP32 sum, segment by segment in
//    order, of the pair sums P[2m] + P[2m+1], rounded to bfloat16, in the
//    upper half of a 32-bit word whose low byte counts the 2 S pixels of the
//    block above rho_th (the fine count bits; at most 16).
// With crs NULL only the fine store is written (S rows per workgroup).
template <int STORE>
__global__ __launch_bounds__(256) void stack_ingest_kernel(const float *__restrict__ in, int n_seg, int n_bins,
                                                           int S, int64_t pitch, void *__restrict__ out,
                                                           float *__restrict__ scale, const float *__restrict__ w,
                                                           float *__restrict__ wq, float th, int64_t pitch2,
                                                           unsigned *__restrict__ crs, unsigned long long *bad) {
    __shared__ float sh[4];
    __shared__ float ssc[8];
    const int j2 = blockIdx.x, r = blockIdx.y;
    const int ns2 = n_seg / S, nb2 = n_bins / 2;
    const int64_t row0 = (int64_t)r * n_seg + (int64_t)S * j2;  // first fine row of the block
    for (int k = 0; k < S; ++k) {
        float sc = 1.0f;
        if (STORE == LTGW_STORE_FP8) {
            const float *row = in + (row0 + k) * n_bins;
            float m = 0.0f;
            for (int b = threadIdx.x; b < n_bins; b += 256) {
                const float x = row[b];
                if (x >= 0.0f && x <= 3.402823466e38f) m = fmaxf(m, x);
            }
            m = block_max_256(m, sh);
            sc = (m == 0.0f) ? 1.0f : m / 448.0f;
        }
        if (threadIdx.x == 0) {
            ssc[k] = sc;
            scale[row0 + k] = sc;
            wq[row0 + k] = w[row0 + k] * sc;
        }
    }
    __syncthreads();
    unsigned nbad = 0;
    unsigned *co = crs ? crs + ((int64_t)r * ns2 + j2) * pitch2 : nullptr;
    for (int m = threadIdx.x; m < nb2; m += 256) {
        float acc = 0.0f;
        unsigned cnt = 0;
        for (int k = 0; k < S; ++k) {
            const float *src = in + (row0 + k) * n_bins + 2 * m;
            float x[2] = {src[0], src[1]};
            unsigned code[2];
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                if (!(x[e] >= 0.0f && x[e] <= 3.402823466e38f)) {
                    ++nbad;
                    x[e] = 0.0f;
                }
                x[e] = __builtin_fabsf(x[e]);  // -0 -> +0
                const unsigned bit = x[e] > th ? 1u : 0u;
                cnt += bit;
                if (STORE == LTGW_STORE_F32) code[e] = __float_as_uint(x[e]) | (bit << 31);
                if (STORE == LTGW_STORE_BF16) code[e] = bf16_rne_bits(x[e]) | (bit << 15);
                if (STORE == LTGW_STORE_FP8) code[e] = e4m3_rne_sat_bits(x[e] / ssc[k]) | (bit << 7);
            }
            const float pair = x[0] + x[1];
            acc = k == 0 ? pair : acc + pair;
            const int64_t o = (row0 + k) * pitch + 2 * m + 1;
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                if (STORE == LTGW_STORE_F32) ((unsigned *)out)[o + e] = code[e];
                if (STORE == LTGW_STORE_BF16) ((unsigned short *)out)[o + e] = (unsigned short)code[e];
                if (STORE == LTGW_STORE_FP8) ((unsigned char *)out)[o + e] = (unsigned char)code[e];
            }
        }
        if (co) co[m + 1] = (bf16_rne_bits(acc) << 16) | cnt;
    }
    // the guards: fine columns 0 and n_bins + 1 .. pitch - 1 of the S rows,
    // coarse columns 0 and nb2 + 1 .. pitch2 - 1
    const int64_t gf = pitch - n_bins;  // guard columns per fine row
    for (int64_t e = threadIdx.x; e < (int64_t)S * gf; e += 256) {
        const int64_t k = e / gf, q = e % gf;
        const int64_t o = (row0 + k) * pitch + (q == 0 ? 0 : n_bins + q);
        if (STORE == LTGW_STORE_F32) ((unsigned *)out)[o] = 0u;
        if (STORE == LTGW_STORE_BF16) ((unsigned short *)out)[o] = 0;
        if (STORE == LTGW_STORE_FP8) ((unsigned char *)out)[o] = 0;
    }
    if (co)
        for (int64_t q = threadIdx.x; q < pitch2 - nb2; q += 256) co[q == 0 ? 0 : nb2 + q] = 0u;
    if (nbad) atomicAdd(bad, (unsigned long long)nbad);
}

hipError_t launch_stack_ingest(int store, const float *power, int R, int32_t n_seg, int32_t n_bins, int S,
                               int64_t pitch, void *out, float *scale, const float *w, float *wq, float rho_th,
                               int64_t pitch2, unsigned *crs, unsigned long long *bad, hipStream_t st) {
    if (R < 1 || R > 65535 || S < 1 || S > 8 || n_seg % S || (n_bins & 1) || pitch < n_bins + 2 ||
        (crs && pitch2 < n_bins / 2 + 2))
        return hipErrorInvalidValue;
    const dim3 grid((unsigned)(n_seg / S), (unsigned)R), block(256);
#define LTGW_STACK_INGEST(ST)                                                                                   \
    hipLaunchKernelGGL(stack_ingest_kernel<ST>, grid, block, 0, st, power, n_seg, n_bins, S, pitch, out, scale, \
                       w, wq, rho_th, pitch2, crs, bad)
    if (store == LTGW_STORE_F32)
        LTGW_STACK_INGEST(LTGW_STORE_F32);
    else if (store == LTGW_STORE_BF16)
        LTGW_STACK_INGEST(LTGW_STORE_BF16);
    else
        LTGW_STACK_INGEST(LTGW_STORE_FP8);
#undef LTGW_STACK_INGEST
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
                                                          unsigned long long *pow_counts) {
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
        int slow = 0;
        out = pow_cr(u, e, &und, &slow);
        if (und) atomicAdd(pow_counts, 1ull);
        if (slow) atomicAdd(pow_counts + 1, 1ull);
    }
    g[(int64_t)grp * n_seg + j] = out;
}

hipError_t launch_spin_factor(const double *t_seg, int32_t n_seg, double t0, const double *tau,
                              int32_t n_tau, const double *brake, int32_t n_brake, double *g,
                              unsigned long long *pow_counts, hipStream_t st) {
    dim3 grid((n_seg + 255) / 256, n_tau * n_brake), block(256);
    hipLaunchKernelGGL(spin_factor_kernel, grid, block, 0, st, t_seg, n_seg, t0, tau, n_tau, brake,
                       g, pow_counts);
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
        DetView D = a.det[d];
        if (D.w_sky_stride) {  // antenna-pattern weights: the row of this group's sky point
            const int64_t off = (int64_t)(grp / a.n_tn) * D.w_sky_stride;
            D.wq += off;
            D.w += off;
        }
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
static hipError_t launch_eval_v(const EvalArgs &a, bool generations, bool slabs, int cu_count, hipStream_t st,
                                int *launches) {
    *launches = 0;
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
            ++*launches;
        }
        if (last) break;
    }
    return hipSuccess;
}

template <int STORE, bool MOMENTS>
static hipError_t launch_eval_m(int variant, const EvalArgs &a, int cu_count, hipStream_t st, int *launches) {
    const bool gen = (variant & 4) != 0, slabs = (variant & 8) != 0;
    switch (variant & 3) {
        case 0: return launch_eval_v<STORE, MOMENTS, 1, 8>(a, gen, slabs, cu_count, st, launches);
        case 1: return launch_eval_v<STORE, MOMENTS, 1, 16>(a, gen, slabs, cu_count, st, launches);
        case 2: return launch_eval_v<STORE, MOMENTS, 2, 8>(a, gen, slabs, cu_count, st, launches);
        default: return launch_eval_v<STORE, MOMENTS, 2, 16>(a, gen, slabs, cu_count, st, launches);
    }
}

template <int STORE>
static hipError_t launch_eval_s(bool moments, int variant, const EvalArgs &a, int cu_count, hipStream_t st,
                                int *launches) {
    return moments ? launch_eval_m<STORE, true>(variant, a, cu_count, st, launches)
                   : launch_eval_m<STORE, false>(variant, a, cu_count, st, launches);
}

hipError_t launch_eval(int store, bool moments, int variant, const EvalArgs &a, int cu_count, hipStream_t st,
                       int *launches) {
    if (variant < 0 || variant >= kNumVariants) return hipErrorInvalidValue;
    if (store == LTGW_STORE_F32) return launch_eval_s<LTGW_STORE_F32>(moments, variant, a, cu_count, st, launches);
    if (store == LTGW_STORE_BF16) return launch_eval_s<LTGW_STORE_BF16>(moments, variant, a, cu_count, st, launches);
    return launch_eval_s<LTGW_STORE_FP8>(moments, variant, a, cu_count, st, launches);
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
// most column n_bins (the statistic kernel's arithmetic).
// One wavefront per (group, kWinRuns consecutive runs of f0): each lane takes
// segments lane, lane + 64, ... and tests every run of the wavefront against
// its track factor, so the group's row of track factors is read once per
// kWinRuns runs; each run's first and last in-band segment are then reduced
// across the wavefront.
constexpr int kWinRuns = 8;
__global__ __launch_bounds__(256) void window_kernel(const DetView D, int n_groups, int n_tn, double f0_min,
                                                     double f0_step, int n_f0, int2 *__restrict__ win) {
    const int lane = threadIdx.x & 63;
    const int per_group = (D.win_blocks + 4 * kWinRuns - 1) / (4 * kWinRuns);
    const int grp = blockIdx.x / per_group;
    const int blk0 = ((blockIdx.x % per_group) * 4 + (threadIdx.x >> 6)) * kWinRuns;
    if (blk0 >= D.win_blocks) return;
    double fa[kWinRuns], fb[kWinRuns];
    int lo[kWinRuns], hi[kWinRuns];
#pragma unroll
    for (int r = 0; r < kWinRuns; ++r) {
        const int ia = (blk0 + r) * D.win_run;
        const int ib = min(ia + D.win_run - 1, n_f0 - 1);
        fa[r] = f0_min + (double)ia * f0_step;
        fb[r] = f0_min + (double)ib * f0_step;
        lo[r] = D.n_seg;
        hi[r] = -1;
    }
    const int tn = grp % n_tn, sky = grp / n_tn;
    for (int j = lane; j < D.n_seg; j += 64) {
        double h;
        if (D.H) {
            h = D.H[(int64_t)grp * D.n_seg + j];
        } else {
            const double hg = D.g[(int64_t)tn * D.n_seg + j] * D.D[(int64_t)sky * D.n_seg + j];
            h = hg * D.t_sft;
        }
#pragma unroll
        for (int r = 0; r < kWinRuns; ++r) {
            const double xa = fa[r] * h, xb = fb[r] * h;
            const int ca = __double2int_rz(xa + D.cshift), cb = __double2int_rz(xb + D.cshift);
            if (cb >= 1 && ca <= D.n_bins) {
                lo[r] = min(lo[r], j);
                hi[r] = max(hi[r], j);
            }
        }
    }
#pragma unroll
    for (int r = 0; r < kWinRuns; ++r) {
        int l = lo[r], u = hi[r];
        for (int o = 32; o > 0; o >>= 1) {
            l = min(l, __shfl_xor(l, o, 64));
            u = max(u, __shfl_xor(u, o, 64));
        }
        if (lane == 0 && blk0 + r < D.win_blocks) win[(int64_t)grp * D.win_blocks + blk0 + r] = make_int2(l, u);
    }
}

hipError_t launch_windows(const DetView &D, int n_groups, int n_tn, double f0_min, double f0_step, int n_f0,
                          int2 *win, hipStream_t st) {
    const int64_t blocks = (int64_t)((D.win_blocks + 4 * kWinRuns - 1) / (4 * kWinRuns)) * n_groups;
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
        if (dec.list) {
            const ltgw_template &T = dec.list[t];
            rec.f0 = T.f0;
            rec.tau = T.tau;
            rec.brake = T.brake;
            rec.sky = -1;
        } else {
            const int64_t i_f0 = t % dec.n_f0;
            const int64_t grp = t / dec.n_f0;
            const int64_t i_tau = grp % dec.n_tau;
            const int64_t rr = grp / dec.n_tau;
            rec.f0 = dec.f0_min + (double)i_f0 * dec.f0_step;
            rec.tau = dec.tau[i_tau];
            rec.brake = dec.brake[rr % dec.n_brake];
            rec.sky = (int32_t)(rr / dec.n_brake);
        }
        rec.index = t;
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
