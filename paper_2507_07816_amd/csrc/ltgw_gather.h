// Device code shared by the statistic kernels (ltgw_kernels.hip) and the
// stack kernels of the learned proposer (ltgw_stack.hip): the gather from a
// stored spectrogram, the per-segment accumulation, the results, the XCD
// order of workgroups and the in-band segment windows.
#pragma once
#include "ltgw_internal.h"

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

template <>
struct Store<kStoreCoarse> {
    static constexpr int kBytes = 4;
    // the upper half is the bfloat16 power sum, the low byte the count
    __device__ static float get(__amdgpu_buffer_rsrc_t r, int i, int soff, int &cnt) {
        const unsigned u = __float_as_uint(ltgw_sbuf_f32(r, i, 0, soff, 0));
        cnt += (int)(u & 0xffu);
        return __uint_as_float(u & 0xffff0000u);
    }
};

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
    // the weights are read unconditionally (wave-uniform loads, selected per
    // lane): a load guarded by the lane's in-band test would become a branch
    float wv[U];
    if (MOMENTS) {
#pragma unroll
        for (int k = 0; k < U; ++k) wv[k] = D.w[j + k];
    }
#pragma unroll
    for (int k = 0; k < U; ++k) {
        const float wq = D.wq[j + k];
#pragma unroll
        for (int t = 0; t < TPL; ++t) {
            sc[t] = __builtin_fmaf(wq, p[t][k], sc[t]);
            if (MOMENTS) {
                const bool inb = (idx[t][k] - 1u) < nb;
                acc.nin[t] += inb ? 1 : 0;
                const float wj = inb ? wv[k] : 0.0f;
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

// An element every lane of the wavefront reads at the same address, through
// the constant address space: for arrays no kernel writes while it runs,
// this makes the read a scalar load.
template <typename T>
__device__ inline T uniform_load(const T *p, int64_t i) {
    return ((const __attribute__((address_space(4))) T *)p)[i];
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

}  // namespace ltgw
