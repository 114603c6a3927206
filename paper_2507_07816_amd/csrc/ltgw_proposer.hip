// Kernels of the learned proposer: synthetic training data (counter-based
// Exp(1) noise, injected tracks), the ranking network (BF16 MFMA, FP32
// accumulation) with its backward pass, loss and Adam, and the per-row top-M
// selection of fine cells.  (The stores, fine and coarse, are written by
// launch_stack_ingest beside the single-detector ingest.)
#include "ltgw_proposer.h"
#include "ddpow.h"

#pragma clang fp contract(off)

namespace ltgw {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC11): ten rounds of
//   (c0, c1, c2, c3) -> (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0))
// with the key advanced by the Weyl constants W0, W1 between rounds.
constexpr uint32_t kPhM0 = 0xD2511F53u, kPhM1 = 0xCD9E8D57u;
constexpr uint32_t kPhW0 = 0x9E3779B9u, kPhW1 = 0xBB67AE85u;

__device__ inline void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)kPhM0 * c[0];
        const uint64_t p1 = (uint64_t)kPhM1 * c[2];
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
        const uint32_t n1 = (uint32_t)p1;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
        const uint32_t n3 = (uint32_t)p0;
        c[0] = n0;
        c[1] = n1;
        c[2] = n2;
        c[3] = n3;
        k0 += kPhW0;
        k1 += kPhW1;
    }
}

// Exp(1) noise: element e of realisation r takes word e % 4 of
// Philox(counter = (e/4 low, e/4 high, r, stream), key = seed);
// u = (word + 1/2) 2^-32 in (0, 1) exactly; value RN_32(-log(u)) (FP64 log).
__global__ __launch_bounds__(256) void noise_kernel(uint64_t seed, uint32_t stream, int r0,
                                                    int64_t n_per, float *__restrict__ out) {
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int r = blockIdx.y;
    if (q * 4 >= n_per) return;
    uint32_t c[4] = {(uint32_t)q, (uint32_t)((uint64_t)q >> 32), (uint32_t)(r0 + r), stream};
    philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    float *o = out + (int64_t)r * n_per;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int64_t e = q * 4 + i;
        if (e < n_per) {
            const double u = ((double)c[i] + 0.5) * 0x1p-32;
            o[e] = (float)(-log(u));
        }
    }
}

hipError_t launch_noise(uint64_t seed, uint32_t stream, int r0, int R, int64_t n_per, float *out,
                        hipStream_t st) {
    if (R < 1 || R > 65535 || n_per < 1) return hipErrorInvalidValue;
    const int64_t blocks = ((n_per + 3) / 4 + 255) / 256;
    hipLaunchKernelGGL(noise_kernel, dim3((unsigned)blocks, (unsigned)R), dim3(256), 0, st, seed, stream,
                       r0, n_per, out);
    return hipGetLastError();
}

// Injected tracks into a stack: realisation r gets amp_r * w_j at the bin of
// template params[r] = (f0, tau, brake, amp) in every in-band segment (amp 0:
// none); the bin arithmetic is the statistic's.
__global__ __launch_bounds__(256) void inject_stack_kernel(
    float *power, int n_seg, int n_bins, int64_t k_lo, double t_sft, const double *t_seg,
    const double *v, const float *w, const double *params, double sx, double sy, double sz,
    double t0, unsigned long long *undecided) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    const int r = blockIdx.y;
    if (j >= n_seg) return;
    const double f0 = params[4 * r + 0], tau = params[4 * r + 1], brake = params[4 * r + 2];
    const float amp = (float)params[4 * r + 3];
    if (amp == 0.0f) return;
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
    float *px = power + ((int64_t)r * n_seg + j) * n_bins + bin;
    *px = *px + amp * w[j];
}

hipError_t launch_inject_stack(float *power, int R, int32_t n_seg, int32_t n_bins, int64_t k_lo,
                               double t_sft, const double *t_seg, const double *v, const float *w,
                               const double *params, double sx, double sy, double sz, double t0,
                               unsigned long long *undecided, hipStream_t st) {
    if (R < 1 || R > 65535) return hipErrorInvalidValue;
    hipLaunchKernelGGL(inject_stack_kernel, dim3((n_seg + 255) / 256, R), dim3(256), 0, st, power,
                       n_seg, n_bins, k_lo, t_sft, t_seg, v, w, params, sx, sy, sz, t0, undecided);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Ranking network.  Layers (width 32, kernel 5, zero padding 2):
//   h1 = relu(conv(x; W1, b1)), h2 = relu(conv(h1; W2, b2)), h3 = relu(conv(h2; W3, b3)),
//   z = conv1(h3; W4, b4)
// conv(x; W, b)[b][o][l] = b[o] + sum_{c,t} W[o][c][t] x[b][c][l + t - p].
// Every contraction is a GEMM on v_mfma_f32_16x16x16_bf16 (operands rounded
// to bfloat16, FP32 accumulation): a wavefront owns a 16 x 16 output tile
// and walks K in steps of 16.  Lane l of the wavefront holds A[l % 16][4 (l/16) + i],
// B[4 (l/16) + i][l % 16] (i < 4) and receives C[4 (l/16) + i][l % 16].
constexpr int kWidth = 32;
constexpr int kTaps = 5;

typedef __attribute__((__vector_size__(4 * sizeof(short)))) short bf16x4;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

__device__ inline short to_bf16(float x) {
    unsigned u = __float_as_uint(x);
    if ((u & 0x7f800000u) == 0x7f800000u) return (short)(u >> 16);  // inf/nan kept
    return (short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

struct ConvDims {
    int B, C, L, O, k, p;
};

// Offsets of W1 b1 W2 b2 W3 b3 W4 b4 in the flat parameter vector.
struct CnnOffsets {
    int64_t o[8];
};

// Y = conv(X; W, b) (+ relu).  GEMM rows o, columns n = (b, l), K = (c, t).
template <int KT>  // taps (1 or 5), zero padding KT / 2
__global__ __launch_bounds__(256) void conv_fwd_kernel(ConvDims d, const float *__restrict__ X,
                                                       const float *__restrict__ W,
                                                       const float *__restrict__ bias, int relu,
                                                       float *__restrict__ Y) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t N = (int64_t)d.B * d.L;
    const int64_t n0 = ((int64_t)blockIdx.x * 4 + wv) * 16;
    const int m0 = blockIdx.y * 16;
    const int K = d.C * KT;
    const int row = lane & 15, kq = (lane >> 4) * 4;
    const int64_t n = n0 + row;  // this lane's B-operand column
    const int nb = (int)(n / d.L), nl = (int)(n % d.L);
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int kk = 0; kk < K; kk += 16) {
        bf16x4 a, b;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int kidx = kk + kq + i;
            const int o = m0 + row;
            float av = 0.f, bv = 0.f;
            if (kidx < K) {
                const int c = kidx / KT, t = kidx % KT;
                if (o < d.O) av = W[((int64_t)o * d.C + c) * KT + t];
                const int li = nl + t - (KT / 2);
                if (n < N && li >= 0 && li < d.L) bv = X[((int64_t)nb * d.C + c) * d.L + li];
            }
            a[i] = to_bf16(av);
            b[i] = to_bf16(bv);
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
    }
    const int64_t nc = n0 + (lane & 15);
    if (nc >= N) return;
    const int cb = (int)(nc / d.L), cl = (int)(nc % d.L);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int o = m0 + (lane >> 4) * 4 + i;
        if (o >= d.O) continue;
        float y = acc[i] + bias[o];
        if (relu) y = y > 0.f ? y : 0.f;
        Y[((int64_t)cb * d.O + o) * d.L + cl] = y;
    }
}

// The same product staged through LDS (the inference path).  A workgroup
// owns one sample b, 64 positions l0 .. l0+63 and 32 output channels: it
// converts the 32 weight rows and the im2col tile of x (k = (c, t) fastest
// in each column) to bfloat16 in LDS once, then each wavefront computes two
// 16 x 16 output tiles, reading its A and B fragments as 8-byte LDS words.
// Rows are padded to Kpad + 4 halves (Kpad = K rounded up to 16).
template <int KT>
__global__ __launch_bounds__(256) void conv_fwd_lds_kernel(ConvDims d, const float *__restrict__ X,
                                                           const float *__restrict__ W,
                                                           const float *__restrict__ bias, int relu,
                                                           float *__restrict__ Y, int Kpad) {
    extern __shared__ short lds[];
    const int S = Kpad + 4;
    short *wt = lds;           // [32][S]
    short *xt = lds + 32 * S;  // [64][S]
    const int tiles_l = (d.L + 63) / 64;
    const int b = blockIdx.x / tiles_l, l0 = (blockIdx.x % tiles_l) * 64;
    const int o0 = blockIdx.y * 32;
    const int K = d.C * KT;
    for (int e = threadIdx.x; e < 32 * Kpad; e += 256) {
        const int r = e / Kpad, k = e % Kpad;
        const int o = o0 + r;
        float v = 0.f;
        if (o < d.O && k < K) v = W[(int64_t)o * K + k];
        wt[r * S + k] = to_bf16(v);
    }
    for (int e = threadIdx.x; e < Kpad * 64; e += 256) {
        const int k = e / 64, col = e % 64;
        float v = 0.f;
        if (k < K) {
            const int c = k / KT, t = k % KT;
            const int l = l0 + col + t - KT / 2;
            if (l0 + col < d.L && l >= 0 && l < d.L) v = X[((int64_t)b * d.C + c) * d.L + l];
        }
        xt[col * S + k] = to_bf16(v);
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int r0 = (wv & 1) * 16, c0 = (wv >> 1) * 32;
    const int row = lane & 15, kq = (lane >> 4) * 4;
    f32x4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
    for (int kk = 0; kk < Kpad; kk += 16) {
        const bf16x4 a = *(const bf16x4 *)&wt[(r0 + row) * S + kk + kq];
        const bf16x4 b0 = *(const bf16x4 *)&xt[(c0 + row) * S + kk + kq];
        const bf16x4 b1 = *(const bf16x4 *)&xt[(c0 + 16 + row) * S + kk + kq];
        acc0 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b0, acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b1, acc1, 0, 0, 0);
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const f32x4 acc = h ? acc1 : acc0;
        const int l = l0 + c0 + h * 16 + (lane & 15);
        if (l >= d.L) continue;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int o = o0 + r0 + kq + i;
            if (o >= d.O) continue;
            float y = acc[i] + bias[o];
            if (relu) y = y > 0.f ? y : 0.f;
            Y[((int64_t)b * d.O + o) * d.L + l] = y;
        }
    }
}

// The product with K ordered (t, c) instead of (c, t), so that the B fragment
// (4 consecutive k) is 4 consecutive channels at one tap: the LDS holds the
// raw input window [position][channel] once (no im2col copies) and every
// fragment is one 8-byte read.  A workgroup owns one sample, 256 positions
// and 32 output channels; each wavefront computes 8 of the 16 x 16 tiles.
// Cp = channels rounded up to 4; K = KT Cp rounded up to 16 (zero fragments
// past KT Cp).
template <int KT>
__global__ __launch_bounds__(256) void conv_fwd_win_kernel(ConvDims d, const float *__restrict__ X,
                                                           const float *__restrict__ W,
                                                           const float *__restrict__ bias, int relu,
                                                           float *__restrict__ Y, int Cp, int Kpad) {
    extern __shared__ short lds[];
    constexpr int kPos = 256;
    const int SW = Kpad + 4, SX = Cp + 4;
    const int P = kPos + KT - 1;
    short *wt = lds;            // [32][SW]
    short *xw = lds + 32 * SW;  // [P][SX]
    const int tiles_l = (d.L + kPos - 1) / kPos;
    const int b = blockIdx.x / tiles_l, l0 = (blockIdx.x % tiles_l) * kPos;
    const int o0 = blockIdx.y * 32;
    for (int e = threadIdx.x; e < 32 * Kpad; e += 256) {
        const int r = e / Kpad, k = e % Kpad;
        const int t = k / Cp, c = k % Cp, o = o0 + r;
        float v = 0.f;
        if (o < d.O && t < KT && c < d.C) v = W[((int64_t)o * d.C + c) * KT + t];
        wt[r * SW + k] = to_bf16(v);
    }
    for (int e = threadIdx.x; e < Cp * P; e += 256) {
        const int c = e / P, pos = e % P;
        const int l = l0 + pos - KT / 2;
        float v = 0.f;
        if (c < d.C && l >= 0 && l < d.L) v = X[((int64_t)b * d.C + c) * d.L + l];
        xw[pos * SX + c] = to_bf16(v);
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int r0 = (wv & 1) * 16, c0 = (wv >> 1) * 128;
    const int row = lane & 15, kq = (lane >> 4) * 4;
    f32x4 acc[8];
#pragma unroll
    for (int h = 0; h < 8; ++h) acc[h] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int kk = 0; kk < Kpad; kk += 16) {
        const int k = kk + kq;
        const int t = k / Cp, c = k % Cp;
        const bf16x4 a = *(const bf16x4 *)&wt[(r0 + row) * SW + k];
#pragma unroll
        for (int h = 0; h < 8; ++h) {
            bf16x4 bv = {0, 0, 0, 0};
            if (t < KT) bv = *(const bf16x4 *)&xw[(c0 + h * 16 + row + t) * SX + c];
            acc[h] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bv, acc[h], 0, 0, 0);
        }
    }
#pragma unroll
    for (int h = 0; h < 8; ++h) {
        const int l = l0 + c0 + h * 16 + (lane & 15);
        if (l >= d.L) continue;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int o = o0 + r0 + kq + i;
            if (o >= d.O) continue;
            float y = acc[h][i] + bias[o];
            if (relu) y = y > 0.f ? y : 0.f;
            Y[((int64_t)b * d.O + o) * d.L + l] = y;
        }
    }
}

// dX = conv^T(dY; W), times the mask (H > 0) of the layer below when H is given.
// GEMM rows c, columns n = (b, l), K = (o, t): dX[b][c][l] = sum W[o][c][t] dY[b][o][l - t + p].
template <int KT>  // taps (1 or 5), zero padding KT / 2
__global__ __launch_bounds__(256) void conv_bwd_data_kernel(ConvDims d, const float *__restrict__ dY,
                                                            const float *__restrict__ W,
                                                            const float *__restrict__ H,
                                                            float *__restrict__ dX) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t N = (int64_t)d.B * d.L;
    const int64_t n0 = ((int64_t)blockIdx.x * 4 + wv) * 16;
    const int m0 = blockIdx.y * 16;
    const int K = d.O * KT;
    const int row = lane & 15, kq = (lane >> 4) * 4;
    const int64_t n = n0 + row;
    const int nb = (int)(n / d.L), nl = (int)(n % d.L);
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int kk = 0; kk < K; kk += 16) {
        bf16x4 a, b;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int kidx = kk + kq + i;
            const int c = m0 + row;
            float av = 0.f, bv = 0.f;
            if (kidx < K) {
                const int o = kidx / KT, t = kidx % KT;
                if (c < d.C) av = W[((int64_t)o * d.C + c) * KT + t];
                const int li = nl - t + (KT / 2);
                if (n < N && li >= 0 && li < d.L) bv = dY[((int64_t)nb * d.O + o) * d.L + li];
            }
            a[i] = to_bf16(av);
            b[i] = to_bf16(bv);
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
    }
    const int64_t nc = n0 + (lane & 15);
    if (nc >= N) return;
    const int cb = (int)(nc / d.L), cl = (int)(nc % d.L);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int c = m0 + (lane >> 4) * 4 + i;
        if (c >= d.C) continue;
        const int64_t off = ((int64_t)cb * d.C + c) * d.L + cl;
        float g = acc[i];
        if (H && !(H[off] > 0.f)) g = 0.f;
        dX[off] = g;
    }
}

// Partial weight gradients over a chunk of columns: GEMM rows o, columns
// (c, t), K = n = (b, l) in [chunk * kc, (chunk + 1) kc):
//   part[chunk][o][c][t] = sum_n dY[b][o][l] X[b][c][l + t - p].
template <int KT>  // taps (1 or 5), zero padding KT / 2
__global__ __launch_bounds__(256) void conv_bwd_weight_kernel(ConvDims d, const float *__restrict__ dY,
                                                              const float *__restrict__ X, int64_t kc,
                                                              float *__restrict__ part) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int CK = d.C * KT;
    const int j0 = (blockIdx.x * 4 + wv) * 16;  // column tile over (c, t)
    const int m0 = blockIdx.y * 16;
    const int64_t N = (int64_t)d.B * d.L;
    const int64_t k_begin = (int64_t)blockIdx.z * kc;
    const int64_t k_end = k_begin + kc < N ? k_begin + kc : N;
    const int row = lane & 15, kq = (lane >> 4) * 4;
    const int jcol = j0 + row;
    const int bc = jcol < CK ? jcol / KT : 0, bt = jcol < CK ? jcol % KT : 0;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int64_t kk = k_begin; kk < k_end; kk += 16) {
        bf16x4 a, b;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t n = kk + kq + i;
            float av = 0.f, bv = 0.f;
            if (n < k_end) {
                const int nb = (int)(n / d.L), nl = (int)(n % d.L);
                const int o = m0 + row;
                if (o < d.O) av = dY[((int64_t)nb * d.O + o) * d.L + nl];
                const int li = nl + bt - (KT / 2);
                if (jcol < CK && li >= 0 && li < d.L) bv = X[((int64_t)nb * d.C + bc) * d.L + li];
            }
            a[i] = to_bf16(av);
            b[i] = to_bf16(bv);
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
    }
    const int jc = j0 + (lane & 15);
    if (jc >= CK) return;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int o = m0 + (lane >> 4) * 4 + i;
        if (o < d.O) part[((int64_t)blockIdx.z * d.O + o) * CK + jc] = acc[i];
    }
}

// Sum of the chunk partials in chunk order (deterministic) into grad.
__global__ void sum_chunks_kernel(const float *part, int chunks, int64_t n, float *grad) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    float s = 0.f;
    for (int q = 0; q < chunks; ++q) s += part[(int64_t)q * n + i];
    grad[i] = s;
}

// Bias gradient: db[o] = sum_{b,l} dY[b][o][l], one block per o, fixed order.
__global__ __launch_bounds__(256) void bias_grad_kernel(const float *dY, int B, int O, int L, float *db) {
    __shared__ float sh[256];
    const int o = blockIdx.x;
    float s = 0.f;
    for (int64_t n = threadIdx.x; n < (int64_t)B * L; n += 256) {
        const int b = (int)(n / L), l = (int)(n % L);
        s += dY[((int64_t)b * O + o) * L + l];
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) db[o] = sh[0];
}

struct CnnLayout {
    int64_t off[8];  // W1 b1 W2 b2 W3 b3 W4 b4
    int64_t total;
};

__host__ __device__ inline CnnLayout cnn_layout(int c_in, int c_out) {
    CnnLayout L;
    const int64_t sz[8] = {(int64_t)kWidth * c_in * kTaps, kWidth, (int64_t)kWidth * kWidth * kTaps, kWidth,
                           (int64_t)kWidth * kWidth * kTaps, kWidth, (int64_t)c_out * kWidth, c_out};
    int64_t o = 0;
    for (int i = 0; i < 8; ++i) {
        L.off[i] = o;
        o += sz[i];
    }
    L.total = o;
    return L;
}

int64_t cnn_n_params(int c_in, int c_out) { return cnn_layout(c_in, c_out).total; }

// ---------------------------------------------------------------------------
// Inference: the whole network for one sample per workgroup (L <= 256, at
// most 32 input channels and 32 logits per position).  The weights are first
// packed as BF16 matrices [32 rows][Kw] with K ordered (t, c) and zero
// padding (cnn_pack_kernel); each wavefront keeps its A fragments of a layer
// in registers.  The input window and the two hidden activations live in LDS
// as BF16, so only the input and the logits cross HBM.  Each layer is the
// product of conv_fwd_win_kernel (the same fragments, zero padding and
// accumulation order), so the logits equal those of the layer-by-layer
// forward pass bit for bit.  Activation rows hold position row - 2 (two zero
// rows of halo on each side of the 256 positions; positions >= L are zero).
constexpr int kInferPos = 256, kInferRows = kInferPos + 4, kInferSH = kWidth + 4;

struct CnnPacked {
    int Cp1, Kw1;       // input channels rounded to 4; layer 1's K rounded to 16
    int64_t o[4];       // offsets (shorts) of the four packed [32][Kw] matrices
    int64_t total;
};

__host__ __device__ inline CnnPacked cnn_packed(int c_in) {
    CnnPacked P;
    P.Cp1 = (c_in + 3) / 4 * 4;
    P.Kw1 = (kTaps * P.Cp1 + 15) / 16 * 16;
    const int kw[4] = {P.Kw1, kTaps * kWidth, kTaps * kWidth, kWidth};
    int64_t o = 0;
    for (int i = 0; i < 4; ++i) {
        P.o[i] = o;
        o += 32 * (int64_t)kw[i];
    }
    P.total = o;
    return P;
}

// Packed[r][k] = bf16(W[r][c][t]) with k = t Cp + c, zero for r >= O,
// c >= C or t >= KT (one thread per entry of the four matrices).
__global__ void cnn_pack_kernel(const float *__restrict__ params, CnnOffsets off, int c_in, int c_out,
                                CnnPacked P, short *__restrict__ packed) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= P.total) return;
    int layer = 3;
    while (layer > 0 && e < P.o[layer]) --layer;
    const int Kw = layer == 0 ? P.Kw1 : layer == 3 ? kWidth : kTaps * kWidth;
    const int Cp = layer == 0 ? P.Cp1 : kWidth, C = layer == 0 ? c_in : kWidth;
    const int KT = layer == 3 ? 1 : kTaps, O = layer == 3 ? c_out : kWidth;
    const int64_t q = e - P.o[layer];
    const int r = (int)(q / Kw), k = (int)(q % Kw);
    const int t = k / Cp, c = k % Cp;
    float v = 0.f;
    if (r < O && t < KT && c < C) v = params[off.o[2 * layer] + ((int64_t)r * C + c) * KT + t];
    packed[e] = to_bf16(v);
}

// One layer: 32 output rows (o < O) over the 256 positions from input rows
// `in` (SXin shorts per row).  Hidden layers write bf16(relu(acc + bias)) to
// `out` (zero at positions >= L); the last writes acc + bias to gout (when
// given) and, with score given, the proposal-block scores of ltgw_propose:
// block k of fine group g covers positions [k pb, k pb + pb) of channels 2g
// and 2g + 1 (fine f0 index 2 l + ch % 2, blocks of 2 pb f0), and scores the
// largest of those logits (pb = 8, 16 or 32).
// Inlined with its shapes as constants: a call would pass them at run time
// (integer divisions for every operand address) and its registers would
// stay allocated across the whole kernel.
template <int KT, int KW, int Cp, int SXin>
__device__ __attribute__((always_inline)) inline void infer_layer(const short *__restrict__ wp,
                                                                  const float *__restrict__ bias, int O,
                                                                  const short *in, int L, bool relu, short *out,
                                                                  float *__restrict__ gout,
                                                                  float *__restrict__ score = nullptr, int pb = 0,
                                                                  int nbg = 0) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int r0 = (wv & 1) * 16, c0 = (wv >> 1) * 128;
    const int row = lane & 15, kq = (lane >> 4) * 4;
    constexpr int NK = KW / 16;
    bf16x4 a[NK];
#pragma unroll
    for (int s = 0; s < NK; ++s) a[s] = *(const bf16x4 *)&wp[(r0 + row) * KW + s * 16 + kq];
    f32x4 acc[8];
#pragma unroll
    for (int h = 0; h < 8; ++h) acc[h] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < NK; ++s) {
        const int k = s * 16 + kq;
        const int t = k / Cp, c = k % Cp;
#pragma unroll
        for (int h = 0; h < 8; ++h) {
            // taps past KT are the zero padding of K: read a valid row, use zero
            const bf16x4 raw = *(const bf16x4 *)&in[(c0 + h * 16 + row + (t < KT ? t : KT - 1) + 2 - KT / 2) * SXin + c];
            const bf16x4 zero = {0, 0, 0, 0};
            const bf16x4 bv = t < KT ? raw : zero;
            acc[h] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[s], bv, acc[h], 0, 0, 0);
        }
    }
    if (out) {  // hidden layers (O = 32): the lane's four channels as one 8-byte write
        float bo[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) bo[i] = bias[r0 + kq + i];
#pragma unroll
        for (int h = 0; h < 8; ++h) {
            const int l = c0 + h * 16 + (lane & 15);
            const bool in = l < L;
            bf16x4 v;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                float y = acc[h][i] + bo[i];
                if (relu) y = y > 0.f ? y : 0.f;
                v[i] = to_bf16(in ? y : 0.f);  // positions >= L hold zero (bf16 of 0)
            }
            *(bf16x4 *)&out[(l + 2) * kInferSH + r0 + kq] = v;
        }
    } else if (gout) {
#pragma unroll
        for (int h = 0; h < 8; ++h) {
            const int l = c0 + h * 16 + (lane & 15);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int o = r0 + kq + i;
                if (o < O && l < L) gout[(int64_t)o * L + l] = acc[h][i] + bias[o];
            }
        }
    }
    if (!score) return;
    // a lane holds channels r0 + kq .. + 3, i.e. groups (r0 + kq) / 2 and + 1,
    // at position c0 + 16 h + (lane % 16): reduce over pb positions
    const int span = pb < 16 ? pb : 16;
    float m[8][2];
#pragma unroll
    for (int h = 0; h < 8; ++h) {
        const int l = c0 + h * 16 + (lane & 15);
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int o = r0 + kq + 2 * j;
            float v = -__builtin_inff();
            if (l < L && o < O) {
                const float y0 = acc[h][2 * j] + bias[o], y1 = acc[h][2 * j + 1] + bias[o + 1];
                v = y1 > y0 ? y1 : y0;
            }
            for (int sh = 1; sh < span; sh <<= 1) {
                const float w = __shfl_xor(v, sh, 64);
                v = w > v ? w : v;
            }
            m[h][j] = v;
        }
    }
#pragma unroll
    for (int h = 0; h < 8; ++h) {
        const int l = c0 + h * 16 + (lane & 15);
        if ((lane & 15) % span != 0 || (pb == 32 && (h & 1)) || l >= L) continue;
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int o = r0 + kq + 2 * j;
            if (o >= O) continue;
            float v = m[h][j];
            if (pb == 32) v = m[h + 1][j] > v ? m[h + 1][j] : v;  // the block's second 16 positions
            score[(o / 2) * nbg + l / pb] = v;
        }
    }
}

template <int CP1>
__global__ __launch_bounds__(256) void cnn_infer_kernel(const float *__restrict__ params,
                                                        const short *__restrict__ packed,
                                                        const float *__restrict__ X, int c_in, int c_out, int L,
                                                        CnnOffsets off, CnnPacked P, float *__restrict__ logits,
                                                        float *__restrict__ score, int pb, int nbg) {
    constexpr int KW1 = (kTaps * CP1 + 15) / 16 * 16, SX0 = CP1 + 4;
    __shared__ short hA[kInferRows * kInferSH], hB[kInferRows * kInferSH];
    short *x0 = hB;  // the input window [260][CP1 + 4] until layer 2 writes hB
    const int b = blockIdx.x;
    for (int e = threadIdx.x; e < kInferRows * CP1; e += 256) {
        const int rr = e / CP1, c = e % CP1, l = rr - 2;
        float v = 0.f;
        if (c < c_in && l >= 0 && l < L) v = X[((int64_t)b * c_in + c) * L + l];
        x0[rr * SX0 + c] = to_bf16(v);
    }
    for (int e = threadIdx.x; e < 4 * kWidth; e += 256) {  // halo rows of hA
        const int rr = e / kWidth, c = e % kWidth;
        hA[(rr < 2 ? rr : kInferRows - 4 + rr) * kInferSH + c] = 0;
    }
    __syncthreads();
    infer_layer<kTaps, KW1, CP1, SX0>(packed + P.o[0], params + off.o[1], kWidth, x0, L, true, hA, nullptr);
    __syncthreads();
    for (int e = threadIdx.x; e < 4 * kWidth; e += 256) {  // halo rows of hB (the input window is spent)
        const int rr = e / kWidth, c = e % kWidth;
        hB[(rr < 2 ? rr : kInferRows - 4 + rr) * kInferSH + c] = 0;
    }
    infer_layer<kTaps, kTaps * kWidth, kWidth, kInferSH>(packed + P.o[1], params + off.o[3], kWidth, hA, L, true,
                                                         hB, nullptr);
    __syncthreads();
    infer_layer<kTaps, kTaps * kWidth, kWidth, kInferSH>(packed + P.o[2], params + off.o[5], kWidth, hB, L, true,
                                                         hA, nullptr);
    __syncthreads();
    infer_layer<1, kWidth, kWidth, kInferSH>(packed + P.o[3], params + off.o[7], c_out, hA, L, false, nullptr,
                           logits ? logits + (int64_t)b * c_out * L : nullptr,
                           score ? score + (int64_t)b * (c_out / 2) * nbg : nullptr, pb, nbg);
}

static hipError_t conv_fwd(const ConvDims &d, const float *X, const float *W, const float *b, int relu,
                           float *Y, hipStream_t st) {
    {
        const int Cp = (d.C + 3) / 4 * 4;
        const int Kw = (d.k * Cp + 15) / 16 * 16;
        const size_t lds = ((size_t)32 * (Kw + 4) + (size_t)(256 + d.k - 1) * (Cp + 4)) * sizeof(short);
        const int64_t ltiles = (int64_t)d.B * ((d.L + 255) / 256);
        if (lds <= 48 * 1024 && ltiles <= 0x7fffffff) {
            dim3 grid((unsigned)ltiles, (unsigned)((d.O + 31) / 32)), block(256);
            if (d.k == kTaps)
                hipLaunchKernelGGL(conv_fwd_win_kernel<kTaps>, grid, block, lds, st, d, X, W, b, relu, Y, Cp, Kw);
            else
                hipLaunchKernelGGL(conv_fwd_win_kernel<1>, grid, block, lds, st, d, X, W, b, relu, Y, Cp, Kw);
            return hipGetLastError();
        }
    }
    const int Kpad = (d.C * d.k + 15) / 16 * 16;
    const size_t lds = (size_t)(32 + 64) * (Kpad + 4) * sizeof(short);
    const int64_t ltiles = (int64_t)d.B * ((d.L + 63) / 64);
    if (lds <= 48 * 1024 && ltiles <= 0x7fffffff) {
        dim3 grid((unsigned)ltiles, (unsigned)((d.O + 31) / 32)), block(256);
        if (d.k == kTaps)
            hipLaunchKernelGGL(conv_fwd_lds_kernel<kTaps>, grid, block, lds, st, d, X, W, b, relu, Y, Kpad);
        else
            hipLaunchKernelGGL(conv_fwd_lds_kernel<1>, grid, block, lds, st, d, X, W, b, relu, Y, Kpad);
        return hipGetLastError();
    }
    const int64_t N = (int64_t)d.B * d.L;
    const int64_t tiles = (N + 15) / 16;
    dim3 grid((unsigned)((tiles + 3) / 4), (unsigned)((d.O + 15) / 16)), block(256);
    if (d.k == kTaps)
        hipLaunchKernelGGL(conv_fwd_kernel<kTaps>, grid, block, 0, st, d, X, W, b, relu, Y);
    else
        hipLaunchKernelGGL(conv_fwd_kernel<1>, grid, block, 0, st, d, X, W, b, relu, Y);
    return hipGetLastError();
}

hipError_t launch_cnn_forward(const float *params, const float *x, int B, int c_in, int c_out, int L,
                              float *act, float *logits, hipStream_t st) {
    const CnnLayout P = cnn_layout(c_in, c_out);
    const int64_t la = (int64_t)B * kWidth * L;
    float *h1 = act, *h2 = act + la, *h3 = act + 2 * la;
    hipError_t e;
    ConvDims d1{B, c_in, L, kWidth, kTaps, kTaps / 2};
    if ((e = conv_fwd(d1, x, params + P.off[0], params + P.off[1], 1, h1, st)) != hipSuccess) return e;
    ConvDims d2{B, kWidth, L, kWidth, kTaps, kTaps / 2};
    if ((e = conv_fwd(d2, h1, params + P.off[2], params + P.off[3], 1, h2, st)) != hipSuccess) return e;
    if ((e = conv_fwd(d2, h2, params + P.off[4], params + P.off[5], 1, h3, st)) != hipSuccess) return e;
    ConvDims d4{B, kWidth, L, c_out, 1, 0};
    return conv_fwd(d4, h3, params + P.off[6], params + P.off[7], 0, logits, st);
}

bool cnn_infer_supported(int c_in, int c_out, int L) {
    return c_in >= 1 && c_in <= kWidth && c_out >= 1 && c_out <= kWidth && L >= 1 && L <= kInferPos;
}

int64_t cnn_infer_scratch_shorts(int c_in) { return cnn_packed(c_in).total; }

hipError_t launch_cnn_infer(const float *params, const float *x, int B, int c_in, int c_out, int L, short *scratch,
                            float *logits, float *score, int W, hipStream_t st) {
    if (B < 1 || !cnn_infer_supported(c_in, c_out, L)) return hipErrorInvalidValue;
    if (score && ((W != 16 && W != 32 && W != 64) || (c_out & 1))) return hipErrorInvalidValue;
    const int pb = score ? W / 2 : 0, nbg = score ? (2 * L + W - 1) / W : 0;
    const CnnLayout PL = cnn_layout(c_in, c_out);
    CnnOffsets off;
    for (int i = 0; i < 8; ++i) off.o[i] = PL.off[i];
    const CnnPacked P = cnn_packed(c_in);
    hipLaunchKernelGGL(cnn_pack_kernel, dim3((unsigned)((P.total + 255) / 256)), dim3(256), 0, st, params, off, c_in,
                       c_out, P, scratch);
    const dim3 grid((unsigned)B), block(256);
    // input channels rounded to 4 (layer 1's K: 5 taps x those, rounded to 16)
#define LTGW_INFER(CP)                                                                                            \
    hipLaunchKernelGGL(cnn_infer_kernel<CP>, grid, block, 0, st, params, scratch, x, c_in, c_out, L, off, P, logits, \
                       score, pb, nbg)
    switch (P.Cp1) {
        case 4: LTGW_INFER(4); break;
        case 8: LTGW_INFER(8); break;
        case 12: LTGW_INFER(12); break;
        case 16: LTGW_INFER(16); break;
        case 20: LTGW_INFER(20); break;
        case 24: LTGW_INFER(24); break;
        case 28: LTGW_INFER(28); break;
        default: LTGW_INFER(32); break;
    }
#undef LTGW_INFER
    return hipGetLastError();
}

// Work area of the backward pass: two activation-sized gradients plus the
// weight-gradient chunk partials.
constexpr int64_t kWgradChunk = 4096;
static int64_t wgrad_chunks(int B, int L) { return ((int64_t)B * L + kWgradChunk - 1) / kWgradChunk; }

int64_t cnn_work_floats(int B, int c_in, int c_out, int L) {
    const int64_t la = (int64_t)B * kWidth * L;
    const int64_t wmax = (int64_t)kWidth * (c_in > kWidth ? c_in : kWidth) * kTaps;
    const int64_t w4 = (int64_t)c_out * kWidth;
    return 2 * la + wgrad_chunks(B, L) * (wmax > w4 ? wmax : w4);
}

static hipError_t weight_grad(const ConvDims &d, const float *dY, const float *X, float *part, float *dW,
                              float *db, hipStream_t st) {
    const int CK = d.C * d.k;
    const int64_t chunks = wgrad_chunks(d.B, d.L);
    dim3 grid((unsigned)(((CK + 15) / 16 + 3) / 4), (unsigned)((d.O + 15) / 16), (unsigned)chunks);
    if (d.k == kTaps)
        hipLaunchKernelGGL(conv_bwd_weight_kernel<kTaps>, grid, dim3(256), 0, st, d, dY, X, kWgradChunk, part);
    else
        hipLaunchKernelGGL(conv_bwd_weight_kernel<1>, grid, dim3(256), 0, st, d, dY, X, kWgradChunk, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t n = (int64_t)d.O * CK;
    hipLaunchKernelGGL(sum_chunks_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, part,
                       (int)chunks, n, dW);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(bias_grad_kernel, dim3(d.O), dim3(256), 0, st, dY, d.B, d.O, d.L, db);
    return hipGetLastError();
}

static hipError_t data_grad(const ConvDims &d, const float *dY, const float *W, const float *H, float *dX,
                            hipStream_t st) {
    const int64_t N = (int64_t)d.B * d.L;
    const int64_t tiles = (N + 15) / 16;
    dim3 grid((unsigned)((tiles + 3) / 4), (unsigned)((d.C + 15) / 16)), block(256);
    if (d.k == kTaps)
        hipLaunchKernelGGL(conv_bwd_data_kernel<kTaps>, grid, block, 0, st, d, dY, W, H, dX);
    else
        hipLaunchKernelGGL(conv_bwd_data_kernel<1>, grid, block, 0, st, d, dY, W, H, dX);
    return hipGetLastError();
}

hipError_t launch_cnn_backward(const float *params, const float *x, int B, int c_in, int c_out, int L,
                               const float *act, const float *dlogits, float *work, int64_t work_floats,
                               float *grads, hipStream_t st) {
    if (work_floats < cnn_work_floats(B, c_in, c_out, L)) return hipErrorInvalidValue;
    const CnnLayout P = cnn_layout(c_in, c_out);
    const int64_t la = (int64_t)B * kWidth * L;
    const float *h1 = act, *h2 = act + la, *h3 = act + 2 * la;
    float *ga = work, *gb = work + la, *part = work + 2 * la;
    hipError_t e;
    ConvDims d4{B, kWidth, L, c_out, 1, 0};
    ConvDims d3{B, kWidth, L, kWidth, kTaps, kTaps / 2};
    ConvDims d1{B, c_in, L, kWidth, kTaps, kTaps / 2};
    // layer 4: dW4, db4 and dh3 (masked by h3 > 0)
    if ((e = weight_grad(d4, dlogits, h3, part, grads + P.off[6], grads + P.off[7], st)) != hipSuccess) return e;
    if ((e = data_grad(d4, dlogits, params + P.off[6], h3, ga, st)) != hipSuccess) return e;
    // layer 3
    if ((e = weight_grad(d3, ga, h2, part, grads + P.off[4], grads + P.off[5], st)) != hipSuccess) return e;
    if ((e = data_grad(d3, ga, params + P.off[4], h2, gb, st)) != hipSuccess) return e;
    // layer 2
    if ((e = weight_grad(d3, gb, h1, part, grads + P.off[2], grads + P.off[3], st)) != hipSuccess) return e;
    if ((e = data_grad(d3, gb, params + P.off[2], h1, ga, st)) != hipSuccess) return e;
    // layer 1 (no gradient for the input)
    return weight_grad(d1, ga, x, part, grads + P.off[0], grads + P.off[1], st);
}

// Softmax cross-entropy per sample over n_cells logits against one target
// cell (target < 0: loss 0, gradient 0); gradients divided by n_valid.
__global__ __launch_bounds__(256) void softmax_xent_kernel(const float *logits, int n_cells,
                                                           const int32_t *target, int n_valid,
                                                           float *loss, float *dlogits) {
    __shared__ float sh[256];
    const int b = blockIdx.x;
    const float *z = logits + (int64_t)b * n_cells;
    float *dz = dlogits + (int64_t)b * n_cells;
    const int tg = target[b];
    if (tg < 0) {
        for (int i = threadIdx.x; i < n_cells; i += 256) dz[i] = 0.f;
        if (threadIdx.x == 0) loss[b] = 0.f;
        return;
    }
    float m = -3.4e38f;
    for (int i = threadIdx.x; i < n_cells; i += 256) m = fmaxf(m, z[i]);
    sh[threadIdx.x] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] = fmaxf(sh[threadIdx.x], sh[threadIdx.x + w]);
        __syncthreads();
    }
    m = sh[0];
    __syncthreads();
    float s = 0.f;
    for (int i = threadIdx.x; i < n_cells; i += 256) s += expf(z[i] - m);
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    s = sh[0];
    const float inv = 1.0f / ((float)n_valid * s);
    for (int i = threadIdx.x; i < n_cells; i += 256) {
        float g = expf(z[i] - m) * inv;
        if (i == tg) g -= 1.0f / (float)n_valid;
        dz[i] = g;
    }
    if (threadIdx.x == 0) loss[b] = logf(s) + m - z[tg];
}

hipError_t launch_softmax_xent(const float *logits, int B, int n_cells, const int32_t *target,
                               int n_valid, float *loss, float *dlogits, hipStream_t st) {
    if (B < 1 || n_cells < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(softmax_xent_kernel, dim3(B), dim3(256), 0, st, logits, n_cells, target,
                       n_valid < 1 ? 1 : n_valid, loss, dlogits);
    return hipGetLastError();
}

// Adam (Kingma and Ba) on FP32 master weights.
__global__ void adam_kernel(float *p, const float *g, float *m, float *v, int64_t n, float lr, float b1,
                            float b2, float eps, float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

hipError_t launch_adam(float *p, const float *g, float *m, float *v, int64_t n, float lr, float b1,
                       float b2, float eps, int step, hipStream_t st) {
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, g, m, v, n, lr,
                       b1, b2, eps, c1, c2);
    return hipGetLastError();
}

// Per row of n scores: the indices of the M largest (ties to the lower index;
// NaN ranks below everything), written in ascending index order.  One
// workgroup per row.  Scores become order-preserving 32-bit keys; the M-th
// largest key is found bit by bit from the top (32 rounds of a block-wide
// count), then every key above it and the first (in index order) keys equal
// to it are written through a block-wide prefix sum.  Thread k holds the
// contiguous indices [k q, k q + q), q = ceil(n / 256) <= 32.
constexpr int kSelMax = 8192;
constexpr int kSelPer = kSelMax / 256;

__device__ inline uint32_t order_key(float v) {
    if (!(v == v)) return 0u;  // NaN: below every number
    const uint32_t u = __float_as_uint(v);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// Block-wide sum of v (256 threads); every thread receives it.
__device__ inline int block_sum(int v, int *sh) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    return sh[0] + sh[1] + sh[2] + sh[3];
}

// Exclusive prefix over the block of v in thread order; also the total.
__device__ inline int block_exclusive(int v, int *sh, int &total) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int x = v;
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    __syncthreads();
    if (lane == 63) sh[wv] = x;
    __syncthreads();
    int off = 0;
    for (int k = 0; k < wv; ++k) off += sh[k];
    total = sh[0] + sh[1] + sh[2] + sh[3];
    return off + x - v;
}

__global__ __launch_bounds__(256) void select_top_kernel(const float *score, int n, int M, int32_t *out) {
    __shared__ int sh[4];
    const float *row = score + (int64_t)blockIdx.x * n;
    const int q = (n + 255) / 256;
    const int i0 = threadIdx.x * q;
    uint32_t key[kSelPer];
#pragma unroll
    for (int r = 0; r < kSelPer; ++r) key[r] = (r < q && i0 + r < n) ? order_key(row[i0 + r]) : 0u;
    // the largest T with #(key >= T) >= M (keys of padding are 0 and are never
    // written: T >= 1 whenever M <= n counts only real entries, see below)
    uint32_t T = 0u;
    for (int bit = 31; bit >= 0; --bit) {
        const uint32_t cand = T | (1u << bit);
        int cnt = 0;
#pragma unroll
        for (int r = 0; r < kSelPer; ++r) cnt += (r < q && i0 + r < n && key[r] >= cand) ? 1 : 0;
        if (block_sum(cnt, sh) >= M) T = cand;
    }
    int gt = 0, eq = 0;
#pragma unroll
    for (int r = 0; r < kSelPer; ++r) {
        const bool real = r < q && i0 + r < n;
        gt += (real && key[r] > T) ? 1 : 0;
        eq += (real && key[r] == T) ? 1 : 0;
    }
    int n_gt = 0, n_eq = 0;
    const int eq_before = block_exclusive(eq, sh, n_eq);
    const int gt_before = block_exclusive(gt, sh, n_gt);
    (void)n_eq;
    const int take_eq = M - n_gt;  // keys equal to T taken, lowest indices first
    // position of this thread's first output: selected entries of lower threads
    int sel = 0;
    {
        int e = 0;
#pragma unroll
        for (int r = 0; r < kSelPer; ++r) {
            const bool real = r < q && i0 + r < n;
            if (real && key[r] > T) ++sel;
            if (real && key[r] == T) {
                if (eq_before + e < take_eq) ++sel;
                ++e;
            }
        }
    }
    int total = 0;
    int pos = block_exclusive(sel, sh, total);
    (void)gt_before;
    int e = 0;
    int32_t *o = out + (int64_t)blockIdx.x * M;
#pragma unroll
    for (int r = 0; r < kSelPer; ++r) {
        const bool real = r < q && i0 + r < n;
        bool take = real && key[r] > T;
        if (real && key[r] == T) {
            take = eq_before + e < take_eq;
            ++e;
        }
        if (take && pos < M) o[pos++] = i0 + r;
    }
}

// The same selection with one wavefront per row, for n <= 64 Q: entry i sits
// in slot i / 64 of lane i % 64.  Counts are ballots, so the threshold search
// runs on wave-uniform values with no barrier; the output position of an
// entry is the number of entries taken in lower slots plus those of lower
// lanes in its own slot (mbcnt), which lists them in ascending index order.
__device__ inline int lanes_below(unsigned long long m) {
    return (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

template <int Q>
__global__ __launch_bounds__(256) void select_top_wave_kernel(const float *score, int R, int n, int M,
                                                              int32_t *out) {
    const int row = blockIdx.x * 4 + (int)(threadIdx.x >> 6);
    if (row >= R) return;  // whole wavefronts; the kernel has no barrier
    const int lane = threadIdx.x & 63;
    const float *s = score + (int64_t)row * n;
    uint32_t key[Q];
    bool real[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        real[q] = q * 64 + lane < n;
        key[q] = real[q] ? order_key(s[q * 64 + lane]) : 0u;
    }
    uint32_t T = 0u;  // the largest T with #(key >= T) >= M over the real entries
    for (int bit = 31; bit >= 0; --bit) {
        const uint32_t cand = T | (1u << bit);
        int cnt = 0;
#pragma unroll
        for (int q = 0; q < Q; ++q) cnt += __popcll(__ballot(real[q] && key[q] >= cand));
        if (cnt >= M) T = cand;
    }
    int n_gt = 0;
#pragma unroll
    for (int q = 0; q < Q; ++q) n_gt += __popcll(__ballot(real[q] && key[q] > T));
    const int take_eq = M - n_gt;  // keys equal to T taken, lowest indices first
    int32_t *o = out + (int64_t)row * M;
    int pos = 0, eq_seen = 0;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const bool eq = real[q] && key[q] == T;
        const unsigned long long eqm = __ballot(eq);
        const bool take = (real[q] && key[q] > T) || (eq && eq_seen + lanes_below(eqm) < take_eq);
        const unsigned long long tm = __ballot(take);
        const int at = pos + lanes_below(tm);
        if (take && at < M) o[at] = q * 64 + lane;
        pos += __popcll(tm);
        eq_seen += __popcll(eqm);
    }
}

hipError_t launch_select_top(const float *score, int R, int n, int M, int32_t *out, hipStream_t st) {
    if (n < 1 || n > kSelMax || M < 1 || M > n || R < 1) return hipErrorInvalidValue;
    const int q = (n + 63) / 64;
    const dim3 wg((unsigned)((R + 3) / 4)), b(256);
    if (q <= 1)
        hipLaunchKernelGGL(select_top_wave_kernel<1>, wg, b, 0, st, score, R, n, M, out);
    else if (q <= 2)
        hipLaunchKernelGGL(select_top_wave_kernel<2>, wg, b, 0, st, score, R, n, M, out);
    else if (q <= 4)
        hipLaunchKernelGGL(select_top_wave_kernel<4>, wg, b, 0, st, score, R, n, M, out);
    else if (q <= 8)
        hipLaunchKernelGGL(select_top_wave_kernel<8>, wg, b, 0, st, score, R, n, M, out);
    else if (q <= 16)
        hipLaunchKernelGGL(select_top_wave_kernel<16>, wg, b, 0, st, score, R, n, M, out);
    else
        hipLaunchKernelGGL(select_top_kernel, dim3(R), dim3(256), 0, st, score, n, M, out);
    return hipGetLastError();
}

}  // namespace ltgw
