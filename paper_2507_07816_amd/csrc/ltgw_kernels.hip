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
//   x = f0*H (FP64)  v = x + (1.5 - k_lo)  i = min((unsigned)trunc(v), n_bins+1)
// and gathers element i of the segment's row with a structured buffer load
// (idxen; stride = element size).  Neighbouring f0 lanes read neighbouring
// columns, so a wavefront's 64 gathers fall in a few cache lines.  The
// per-segment H, weight and row address are wavefront-uniform (SGPRs).
// trunc(v) - 1 equals floor(RN(x + 0.5)) - k_lo whenever the latter is in
// band, for k_lo >= 2 and x < 2^30 (both checked by the host): x + 1.5 - k_lo
// is exact in FP64 whenever its magnitude is at most x, and every other case
// lands on a guard (a negative trunc(v) wraps to a large unsigned value and is
// clamped onto the upper guard).
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
// Statistic (Sec. 2): one lane per template.  FP32 partial sums over chunks
// of 32 segments, carried in FP64.  Segments are processed in batches of 8
// so that 8 independent gathers are in flight per wavefront.
constexpr int kChunk = 32;
constexpr int kBatch = 8;

template <int STORE, bool WEIGHTED, int U>
__device__ __forceinline__ void seg_batch(const DetView &D, __amdgpu_buffer_rsrc_t rs,
                                          const double *__restrict__ H, int j, double f0,
                                          float &sc, float &w1c, float &w2c, int &cnt, int &nin) {
    const unsigned nb = (unsigned)D.n_bins;
    const unsigned hi = nb + 1u;
    unsigned idx[U];
#pragma unroll
    for (int k = 0; k < U; ++k) {
        const double x = f0 * H[j + k];
        const double vv = x + D.cshift;
        // negative values wrap to large unsigned and clamp onto the upper guard
        const unsigned u = (unsigned)__double2int_rz(vv);
        idx[k] = u < hi ? u : hi;
    }
    float p[U];
#pragma unroll
    for (int k = 0; k < U; ++k)
        p[k] = Store<STORE>::get(rs, (int)idx[k], (j + k) * D.pitch_bytes, cnt);
#pragma unroll
    for (int k = 0; k < U; ++k) {
        sc = __builtin_fmaf(D.wq[j + k], p[k], sc);
        const bool inb = (idx[k] - 1u) < nb;
        nin += inb ? 1 : 0;
        if (WEIGHTED) {
            const float wj = inb ? D.w[j + k] : 0.0f;
            w1c += wj;
            w2c = __builtin_fmaf(wj, wj, w2c);
        }
    }
}

template <int STORE, bool WEIGHTED>
__global__ __launch_bounds__(256) void eval_kernel(const EvalArgs a) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int grp = blockIdx.y;
    const double f0 = a.f0_min + (double)i * a.f0_step;
    double s = 0.0, w1 = 0.0, w2 = 0.0;
    int cnt = 0, nin = 0;
    for (int d = 0; d < a.n_det; ++d) {
        const DetView D = a.det[d];
        const double *__restrict__ H = D.H + (int64_t)grp * D.n_seg;
        // one resource for the whole store; the row is the instruction's scalar offset
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            (void *)D.store, Store<STORE>::kBytes, D.store_elems, kBufDword3);
        int j = 0;
        for (; j + kChunk <= D.n_seg; j += kChunk) {
            float sc = 0.0f, w1c = 0.0f, w2c = 0.0f;
#pragma unroll 1
            for (int b = 0; b < kChunk; b += kBatch)
                seg_batch<STORE, WEIGHTED, kBatch>(D, rs, H, j + b, f0, sc, w1c, w2c, cnt, nin);
            s += (double)sc;
            if (WEIGHTED) {
                w1 += (double)w1c;
                w2 += (double)w2c;
            }
        }
        if (j < D.n_seg) {
            float sc = 0.0f, w1c = 0.0f, w2c = 0.0f;
            for (; j < D.n_seg; ++j) seg_batch<STORE, WEIGHTED, 1>(D, rs, H, j, f0, sc, w1c, w2c, cnt, nin);
            s += (double)sc;
            if (WEIGHTED) {
                w1 += (double)w1c;
                w2 += (double)w2c;
            }
        }
    }
    if (!WEIGHTED) {
        const double wu = (double)a.w_uniform;
        w1 = (double)nin * wu;
        w2 = (double)nin * (wu * wu);
    }
    // in-band total for the roofline's algorithmic bytes (one atomic per wave)
    unsigned long long nw = (i < a.n_f0) ? (unsigned long long)nin : 0ull;
    for (int o = 32; o > 0; o >>= 1) nw += __shfl_xor(nw, o, 64);
    if ((threadIdx.x & 63) == 0 && a.in_band_total) atomicAdd(a.in_band_total, nw);
    if (i >= a.n_f0) return;
    const int64_t t = (int64_t)grp * a.n_f0 + i;
    a.s[t] = s;
    a.c[t] = cnt;
    a.n[t] = nin;
    a.w1[t] = w1;
    a.w2[t] = w2;
    if (a.out_s) a.out_s[t] = (float)s;
    if (a.out_c) a.out_c[t] = cnt;
    if (a.out_n) a.out_n[t] = nin;
}

template <int STORE>
static hipError_t launch_eval_s(bool weighted, const EvalArgs &a, hipStream_t st) {
    dim3 grid((a.n_f0 + 255) / 256, a.n_groups), block(256);
    if (weighted)
        hipLaunchKernelGGL((eval_kernel<STORE, true>), grid, block, 0, st, a);
    else
        hipLaunchKernelGGL((eval_kernel<STORE, false>), grid, block, 0, st, a);
    return hipGetLastError();
}

hipError_t launch_eval(int store, bool weighted, const EvalArgs &a, hipStream_t st) {
    if (store == LTGW_STORE_F32) return launch_eval_s<LTGW_STORE_F32>(weighted, a, st);
    if (store == LTGW_STORE_BF16) return launch_eval_s<LTGW_STORE_BF16>(weighted, a, st);
    return launch_eval_s<LTGW_STORE_FP8>(weighted, a, st);
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
