// Data preparation (Sec. 2): strain -> Hann-windowed short Fourier transforms
// -> normalised power rho = P ln 2 / (running median of P over frequency).
//
// Segment j is samples [j N, (j + 1) N) of the strain.  Per chunk of segments:
//   one batched real-to-complex FFT (hipFFT, FP32) of the raw segments;
//   normalise_kernel: the Hann window applied in frequency: with the periodic
//   window w_n = 1/2 - 1/2 cos(2 pi n / N) = 1/2 - e^{2 pi i n/N}/4 - e^{-2 pi i n/N}/4
//   the windowed transform is X_k/2 - (X_{k-1} + X_{k+1})/4 (X_{-1} = conj X_1 and
//   X_{N/2+1} = conj X_{N/2-1} for real input); P_k = |.|^2 for a 256-bin tile of the band
//   and its median halo, a bitonic sort of (P, position) in LDS, then each bin's median is the
//   (h + 1)-th smallest value whose position lies in its window: position
//   masks of the sorted tile's blocks of 64 entries, counted against the
//   bin's window, give the block that holds it, and a scan of that block the
//   entry.  Under Gaussian noise P_k is exponential with
//   mean S_k and median S_k ln 2, hence rho_k = P_k ln 2 / median.
#include <hip/hip_runtime.h>
#include <hipfft/hipfft.h>

#include <cmath>
#include <cstdio>
#include <vector>

#include "ltgw_ctx.h"

#pragma clang fp contract(off)

namespace ltgw {

constexpr int kSftTile = 256;      // output bins per workgroup
constexpr int kSftSort = 512;      // sorted entries: tile + halo, padded to a power of two
constexpr int kSftMaxWindow = kSftSort - kSftTile + 1;  // 257

// One workgroup: segment blockIdx.y, output bins [t0, t0 + 256) of the band;
// lane t takes bin t0 + t.  (Wider tiles that fill all 512 sorted entries
// were measured slower: the per-bin scans, not the sort, dominate.)
__device__ __forceinline__ float2 spec_at(const float2 *row, int64_t k, int64_t half) {
    // X_{-1} = conj X_1, X_{half+1} = conj X_{half-1} (real input)
    if (k < 0) {
        const float2 z = row[-k];
        return make_float2(z.x, -z.y);
    }
    if (k > half) {
        const float2 z = row[2 * half - k];
        return make_float2(z.x, -z.y);
    }
    return row[k];
}

__global__ __launch_bounds__(256) void normalise_kernel(const float2 *__restrict__ spec, int64_t spec_pitch,
                                                        int64_t k_lo, int n_bins, int h, float *__restrict__ out) {
    __shared__ float val[kSftSort];
    __shared__ __attribute__((aligned(16))) short pos[kSftSort];
    __shared__ float pw[kSftSort];
    // bit p of bmask[b][p / 64]: position p holds one of sorted entries 64 b .. 64 b + 63
    constexpr int kBlk = kSftSort / 64;
    __shared__ unsigned long long bmask[kBlk][kSftSort / 64];
    const int t = threadIdx.x;
    const int T = kSftTile;
    const int t0 = blockIdx.x * T;
    const int seg = blockIdx.y;
    const float2 *row = spec + (int64_t)seg * spec_pitch;
    // tile positions p = 0 .. 255 + 2h hold bin k_lo + t0 - h + p; positions
    // past the last needed bin (band end + h) are padding that sorts last
    const int n_pos = T + 2 * h;
    const int last_needed = n_bins - 1 - t0 + 2 * h;  // last position any output reads
    for (int p = t; p < kSftSort; p += 256) {
        float v = __builtin_inff();
        if (p < n_pos && p <= last_needed) {
            const int64_t k = k_lo + t0 - h + p;
            const int64_t half = spec_pitch - 1;
            const float2 z = row[k], zm = spec_at(row, k - 1, half), zp = spec_at(row, k + 1, half);
            const float re = 0.5f * z.x - 0.25f * (zm.x + zp.x);
            const float im = 0.5f * z.y - 0.25f * (zm.y + zp.y);
            const float a = re * re;
            const float b = im * im;
            v = a + b;
        }
        val[p] = v;
        pw[p] = v;
        pos[p] = (short)p;
    }
    if (t < kBlk * (kSftSort / 64)) (&bmask[0][0])[t] = 0ull;
    __syncthreads();
    // bitonic sort of (val, pos) ascending in val (a workgroup barrier per
    // stage: ordering the 39 stages that stay inside a wavefront by wavefront
    // fences instead was measured slower)
    for (int size = 2; size <= kSftSort; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            const int a = 2 * t - (t & (stride - 1));
            const int b = a + stride;
            const bool up = (a & size) == 0;
            const float va = val[a], vb = val[b];
            if ((va > vb) == up) {
                val[a] = vb;
                val[b] = va;
                const short pa = pos[a];
                pos[a] = pos[b];
                pos[b] = pa;
            }
            __syncthreads();
        }
    }
    for (int k = t; k < kSftSort; k += 256) {
        const int p = pos[k];
        atomicOr(&bmask[k >> 6][p >> 6], 1ull << (p & 63));
    }
    __syncthreads();
    // output o: window positions [o, o + 2h]; its median is the (h + 1)-th
    // smallest value among them.  The in-window counts of the sorted blocks,
    // in order, locate the block of that entry; within the block, four sorted
    // positions per LDS read, and the group that holds it is resolved entry by
    // entry.  The entry is the one a scan of the whole sorted tile finds.
    const short4 *pos4 = reinterpret_cast<const short4 *>(pos);
    for (int o = t; o < T && t0 + o < n_bins; o += 256) {
        const int lo = o, hi = o + 2 * h;
        const int w0 = lo >> 6, w1 = hi >> 6;
        int cnt = 0, blk = 0;
        for (; blk < kBlk - 1; ++blk) {
            int c = 0;
            for (int w = w0; w <= w1; ++w) {
                unsigned long long m = bmask[blk][w];
                if (w == w0) m &= ~0ull << (lo & 63);
                if (w == w1) m &= ~0ull >> (63 - (hi & 63));
                c += __popcll(m);
            }
            if (cnt + c > h) break;
            cnt += c;
        }
        float med = 0.0f;
        for (int g = 16 * blk; g < 16 * blk + 16 && cnt <= h; ++g) {
            const short4 q = pos4[g];
            const int i0 = (q.x >= lo && q.x <= hi), i1 = (q.y >= lo && q.y <= hi);
            const int i2 = (q.z >= lo && q.z <= hi), i3 = (q.w >= lo && q.w <= hi);
            const int c = cnt + ((i0 + i1) + (i2 + i3));
            if (c > h) {
                int k = h + 1 - cnt, e = 0;
                if (i0 && --k == 0) e = 0;
                else if (i1 && --k == 0) e = 1;
                else if (i2 && --k == 0) e = 2;
                else e = 3;
                med = val[4 * g + e];
            }
            cnt = c;
        }
        const float P = pw[o + h];
        // rho = P ln2 / median; a window whose median is 0 carries no noise-floor estimate: 0
        const double r = med > 0.0f ? (double)P * 0.69314718055994530942 / (double)med : 0.0;
        out[(int64_t)seg * n_bins + t0 + o] = (float)r;
    }
}

void sft_release(ltgw_ctx *c) {
    for (auto &pl : c->sft_plans) (void)hipfftDestroy((hipfftHandle)pl.plan);
    c->sft_plans.clear();
    release(c->sft_spec);
    release(c->sft_spec2);
}

}  // namespace ltgw

namespace {

const char *fft_error(hipfftResult r) {
    switch (r) {
        case HIPFFT_ALLOC_FAILED: return "allocation failed";
        case HIPFFT_INVALID_VALUE: return "invalid value";
        case HIPFFT_INVALID_SIZE: return "invalid size";
        case HIPFFT_EXEC_FAILED: return "execution failed";
        case HIPFFT_SETUP_FAILED: return "setup failed";
        default: return "error";
    }
}

}  // namespace

using namespace ltgw;

// A chunk of strain rows (n_fft reals each) into the transform buffer's rows
// of n_fft + 2 reals: 8-byte moves (n_fft is even, so every row of both is
// 8-byte aligned), a grid-stride loop over each row.
__global__ __launch_bounds__(256) void pad_rows_kernel(const float2 *__restrict__ src, int64_t src_pitch,
                                                       float2 *__restrict__ dst, int64_t dst_pitch, int64_t pairs) {
    const float2 *s = src + (int64_t)blockIdx.y * src_pitch;
    float2 *d = dst + (int64_t)blockIdx.y * dst_pitch;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < pairs; i += (int64_t)gridDim.x * 256) d[i] = s[i];
}

extern "C" {

int32_t ltgw_sft_normalise(ltgw_ctx *c, const float *strain, int32_t n_seg, int32_t n_fft, int64_t k_lo,
                           int32_t n_bins, int32_t window, float *out) {
    if (!c) return LTGW_E_INVALID_ARG;
    Enter en(c);
    if (!strain || !out) return fail(c, LTGW_E_INVALID_ARG, "strain or out is NULL");
    if (!is_device_ptr(strain) || !is_device_ptr(out))
        return fail(c, LTGW_E_INVALID_ARG, "strain and out must be device memory");
    if (n_seg < 1 || n_seg > 65535) return fail(c, LTGW_E_INVALID_ARG, "n_seg must be in 1 .. 65535");
    if (n_fft < 2 || (n_fft & 1) || n_fft > (1 << 24))
        return fail(c, LTGW_E_INVALID_ARG, "n_fft must be even and in 2 .. 2^24");
    if (window < 1 || !(window & 1) || window > kSftMaxWindow)
        return fail(c, LTGW_E_INVALID_ARG, "window must be odd and in 1 .. %d", kSftMaxWindow);
    const int h = window / 2;
    if (n_bins < 1 || k_lo < h || k_lo + n_bins - 1 + h > n_fft / 2)
        return fail(c, LTGW_E_INVALID_ARG, "band [k_lo - window/2, k_lo + n_bins - 1 + window/2] must lie in 0 .. n_fft/2");
    int rc;
    // chunks of segments: spectra within about 512 MB
    const int64_t per_seg = (int64_t)(n_fft / 2 + 1) * 8;
    int batch = (int)std::max<int64_t>(1, std::min<int64_t>(n_seg, ((int64_t)512 << 20) / per_seg));
    if ((rc = ensure(c, c->sft_spec, (size_t)batch * (n_fft / 2 + 1) * 8, "spectra")) != LTGW_OK) return rc;
    // More than one chunk: alternate two spectra buffers, and normalise on the
    // side stream, so that a chunk's normalisation (LDS-bound) overlaps the
    // next chunk's copy and transform (HBM-bound).  The copy into a buffer
    // waits for the normalisation that last read it; the context's stream
    // waits for the last normalisations before the call's work ends.
    const bool two = n_seg > batch;
    if (two && (rc = ensure(c, c->sft_spec2, (size_t)batch * (n_fft / 2 + 1) * 8, "spectra")) != LTGW_OK)
        return rc;
    int k = 0;
    for (int j0 = 0; j0 < n_seg; j0 += batch, ++k) {
        const int nb = std::min(batch, n_seg - j0);
        const int b = k & 1;
        void *const spec = b ? c->sft_spec2.p : c->sft_spec.p;
        // a plan per (n_fft, batch size), kept for later calls
        hipfftHandle plan = nullptr;
        for (auto &pl : c->sft_plans)
            if (pl.n_fft == n_fft && pl.batch == nb) plan = (hipfftHandle)pl.plan;
        if (!plan) {
            // in place: rows of n_fft + 2 reals in, n_fft / 2 + 1 complex out
            int n = n_fft, in_len = n_fft + 2, out_len = n_fft / 2 + 1;
            const hipfftResult r = hipfftPlanMany(&plan, 1, &n, &in_len, 1, n_fft + 2, &out_len, 1, n_fft / 2 + 1,
                                                  HIPFFT_R2C, nb);
            if (r != HIPFFT_SUCCESS) return fail(c, LTGW_E_DEVICE, "FFT plan: %s", fft_error(r));
            c->sft_plans.push_back({n_fft, nb, (void *)plan});
        }
        // the chunk's segments are copied into the spectra buffer (rows padded
        // to n_fft + 2 reals) and transformed there in place: the library's
        // transform may use its input as scratch, and the caller's strain is
        // only read
        if (two && k >= 2) HIP_TRY(c, hipStreamWaitEvent(c->stream, c->ev_sft[2 + b], 0), "spectra reuse");
        {
            const int64_t pairs = n_fft / 2;
            const unsigned gx = (unsigned)std::min<int64_t>((pairs + 255) / 256, 16);
            hipLaunchKernelGGL(pad_rows_kernel, dim3(gx, (unsigned)nb), dim3(256), 0, c->stream,
                               (const float2 *)(strain + (int64_t)j0 * n_fft), pairs, (float2 *)spec,
                               (int64_t)(n_fft / 2 + 1), pairs);
            HIP_TRY(c, hipGetLastError(), "strain copy launch");
        }
        hipfftResult r = hipfftSetStream(plan, c->stream);
        if (r == HIPFFT_SUCCESS) r = hipfftExecR2C(plan, (hipfftReal *)spec, (hipfftComplex *)spec);
        if (r != HIPFFT_SUCCESS) return fail(c, LTGW_E_DEVICE, "FFT: %s", fft_error(r));
        hipStream_t ns = c->stream;
        if (two) {
            HIP_TRY(c, hipEventRecord(c->ev_sft[b], c->stream), "event record");
            HIP_TRY(c, hipStreamWaitEvent(c->side, c->ev_sft[b], 0), "normalise order");
            ns = c->side;
        }
        hipLaunchKernelGGL(normalise_kernel, dim3((unsigned)((n_bins + kSftTile - 1) / kSftTile), (unsigned)nb),
                           dim3(256), 0, ns, (const float2 *)spec, (int64_t)(n_fft / 2 + 1), k_lo, n_bins, h,
                           out + (int64_t)j0 * n_bins);
        HIP_TRY(c, hipGetLastError(), "normalise launch");
        if (two) HIP_TRY(c, hipEventRecord(c->ev_sft[2 + b], c->side), "event record");
    }
    if (two)
        for (int b = 0; b < 2 && b < k; ++b)
            HIP_TRY(c, hipStreamWaitEvent(c->stream, c->ev_sft[2 + b], 0), "normalise join");
    return LTGW_OK;
}

}  // extern "C"
