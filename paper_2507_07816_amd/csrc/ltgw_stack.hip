// Kernels over stacks of realisations (the learned proposer's data): the
// statistic of every template or of listed templates on each realisation,
// the selection of proposal blocks, per-row best entries and the fallback
// rule.  They use the statistic's gather and accumulation (ltgw_gather.h).
#include "ltgw_gather.h"
#include "ltgw_proposer.h"

#pragma clang fp contract(off)

namespace ltgw {

// ---------------------------------------------------------------------------
// Stacks of realisations (the learned proposer's data): R spectrograms of one
// geometry, realisation r at byte offset r * stack_bytes of the store and
// r * stack_rows of the per-row weights.  The weights are the same for every
// realisation, so each template's moments W1, W2, N are formed once per
// lattice (stack_moments_kernel) in the order the in-loop sums would take:
// FP32 over chunks of 32 segments, carried in FP64.
template <int SHIFT>
__global__ __launch_bounds__(256) void stack_moments_kernel(const EvalArgs a, double *__restrict__ w1,
                                                            double *__restrict__ w2, int32_t *__restrict__ n) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= (int64_t)a.n_groups * a.n_f0) return;
    const int grp = (int)(t / a.n_f0), i = (int)(t % a.n_f0);
    const DetView &D = a.det[0];
    const double f0 = a.f0_min + (double)i * a.f0_step;
    const double *__restrict__ H = D.H + (int64_t)grp * D.n_seg;
    const unsigned nb = (unsigned)D.n_bins;
    double W1 = 0.0, W2 = 0.0;
    int N = 0;
    for (int j0 = 0; j0 < D.n_seg; j0 += kChunk) {
        const int je = min(j0 + kChunk, D.n_seg);
        float c1 = 0.0f, c2 = 0.0f;
        for (int j = j0; j < je; ++j) {
            const double x = f0 * H[j];
            const double vv = x + D.cshift;
            const unsigned idx = (unsigned)__double2int_rz(vv) >> SHIFT;
            const bool inb = (idx - 1u) < nb;
            N += inb ? 1 : 0;
            const float wv = D.w[j];
            const float wj = inb ? wv : 0.0f;
            c1 += wj;
            c2 = __builtin_fmaf(wj, wj, c2);
        }
        W1 += (double)c1;
        W2 += (double)c2;
    }
    w1[t] = W1;
    w2[t] = W2;
    n[t] = N;
}

hipError_t launch_stack_moments(int shift, const EvalArgs &a, double *w1, double *w2, int32_t *n, hipStream_t st) {
    const int64_t t = (int64_t)a.n_groups * a.n_f0;
    if (t < 1 || t > 0x7fffffffLL) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((t + 255) / 256)), block(256);
    if (shift == 0)
        hipLaunchKernelGGL(stack_moments_kernel<0>, grid, block, 0, st, a, w1, w2, n);
    else
        hipLaunchKernelGGL(stack_moments_kernel<1>, grid, block, 0, st, a, w1, w2, n);
    return hipGetLastError();
}

// The critical ratio of template tt from its power sum s and the moments:
//     Psi = (s - mu W1) / sqrt(var W2)
// with the per-pixel noise mean mu and variance var of the store (Exp(1):
// 1, 1; a sum of m Exp(1): m, m); N = 0 gives NaN (or 0 with nan_to_zero).
__device__ inline double stack_ratio(double s, const StackMoments &m, int64_t tt, double mu, double var,
                                     int nan_to_zero) {
    if (m.n[tt] == 0) return nan_to_zero ? 0.0 : __builtin_nan("");
    const double num = s - mu * m.w1[tt];
    return num / sqrt(var * m.w2[tt]);
}

// The ratio a stack kernel writes for a template with power sum s and count
// c: power (above), or with m.count the count ratio in the operation order of
// the single-search ratio (the same value bit for bit).
__device__ inline double stack_stat(double s, int c, const StackMoments &m, int64_t tt, double mu, double var,
                                    int nan_to_zero) {
    if (!m.count) return stack_ratio(s, m, tt, mu, var, nan_to_zero);
    const int nn = m.n[tt];
    if (nn == 0) return nan_to_zero ? 0.0 : __builtin_nan("");
    const double Nq = (double)nn * m.q;
    const double num = (double)c - Nq;
    return num / sqrt(Nq * (1.0 - m.q));
}

// Every template of a grid on every realisation: the power critical ratio.
// One workgroup per (256 f0, group, output row) and pass.  The hardware deals
// workgroups to the XCDs in turn; workgroup w goes to row x + 8 (k / per_row)
// of XCD x = w % 8 (k = w / 8), so the workgroups of one row run on one XCD
// and share its L2, and rows 0, 1, 2 ... go to different XCDs (the listed
// rows of a fallback are the first ones).  A grid of P rows (P a multiple of
// 8) visits rows rr, rr + P, rr + 2P ...  Output row rr holds realisation
// rmap[rr] (rr without a map); rows rr >= R, or >= *n_rows when that device
// count is given, are skipped.
template <int STORE, int SHIFT>
__global__ __launch_bounds__(256) void stack_eval_kernel(const EvalArgs a, int R, int64_t stack_bytes,
                                                         int64_t stack_rows, double mu, double var,
                                                         int nan_to_zero, const int32_t *__restrict__ rmap,
                                                         const int32_t *__restrict__ n_rows, const StackMoments m,
                                                         double *__restrict__ out_psi) {
    const int n_tiles = (a.n_f0 + 255) / 256;
    const int per_row = n_tiles * a.n_groups;
    const int P = (int)gridDim.x / per_row;
    const int x = (int)blockIdx.x % kXcds, k = (int)blockIdx.x / kXcds;
    const int q = k % per_row;
    const int tile = q / a.n_groups, grp = q % a.n_groups;
    // a wave whose 64 f0 all lie past the grid has nothing to do (no barrier follows)
    if (tile * 256 + (int)(threadIdx.x & ~63u) >= a.n_f0) return;
    const int rows = n_rows ? min(R, *n_rows) : R;
    const int i = tile * 256 + (int)threadIdx.x;
    const double f0[1] = {a.f0_min + (double)i * a.f0_step};
    const int64_t tt = (int64_t)grp * a.n_f0 + i;
    for (int rr = x + kXcds * (k / per_row); rr < rows; rr += P) {
        const int r = rmap ? rmap[rr] : rr;
        DetView D = a.det[0];
        D.store = (const char *)D.store + (int64_t)r * stack_bytes;
        D.wq += (int64_t)r * stack_rows;
        D.w += (int64_t)r * stack_rows;
        Acc<1> acc;
        acc.zero();
        accumulate_det<STORE, false, 1, 16, HTable, SHIFT>(D, HTable{D.H + (int64_t)grp * D.n_seg}, f0, acc);
        if (i < a.n_f0)
            out_psi[(int64_t)rr * ((int64_t)a.n_groups * a.n_f0) + tt] =
                stack_stat(acc.s[0], acc.cnt[0], m, tt, mu, var, nan_to_zero);
    }
}

hipError_t launch_stack_eval(int store, int shift, const EvalArgs &a, int R, int64_t stack_bytes,
                             int64_t stack_rows, double mu, double var, int nan_to_zero, const int32_t *rmap,
                             const int32_t *n_rows, StackMoments m, double *out_psi, hipStream_t st) {
    // rows per pass: all of them rounded up to a multiple of the XCD count (the
    // extra workgroups return), or at most 256 when a device count may leave
    // most rows idle
    const int P = (n_rows && R > 256 ? 256 : R + kXcds - 1) / kXcds * kXcds;
    const int64_t blocks = (int64_t)((a.n_f0 + 255) / 256) * a.n_groups * P;
    if (blocks > 0x7fffffff || R > 65535 || R < 1) return hipErrorInvalidValue;
    dim3 grid((unsigned)blocks), block(256);
#define LTGW_STACK_EVAL(S, SH)                                                                                     \
    hipLaunchKernelGGL((stack_eval_kernel<S, SH>), grid, block, 0, st, a, R, stack_bytes, stack_rows, mu, var, \
                       nan_to_zero, rmap, n_rows, m, out_psi)
    if (store == LTGW_STORE_F32 && shift == 0)
        LTGW_STACK_EVAL(LTGW_STORE_F32, 0);
    else if (store == LTGW_STORE_BF16 && shift == 0)
        LTGW_STACK_EVAL(LTGW_STORE_BF16, 0);
    else if (store == kStoreCoarse && shift == 1)
        LTGW_STACK_EVAL(kStoreCoarse, 1);
    else if (store == LTGW_STORE_FP8 && shift == 0)
        LTGW_STACK_EVAL(LTGW_STORE_FP8, 0);
    else
        return hipErrorInvalidValue;
#undef LTGW_STACK_EVAL
    return hipGetLastError();
}

// The network's input on the coarse store: for every template of the coarse
// grid and every realisation, the power critical ratio (mean and variance
// mu = 2 S per pixel) into channel g and, with counts, the number-count
// critical ratio into channel G + g (G coarse groups): (c - N m q) /
// sqrt(N m q (1 - q)) with m = 2 S pixels per coarse pixel, N the in-band
// coarse segments, q = exp(-rho_th).  x[r][channel][f0] in FP32, 0 where N = 0.
// psi (optional): the power ratio in FP64 as stack_eval_kernel writes it
// (NaN -> 0), for the per-row coarse maximum.  One workgroup per (256 f0,
// group, realisation), the XCD order of stack_eval_kernel.
__global__ __launch_bounds__(256) void stack_features_kernel(const EvalArgs a, int R, int64_t stack_bytes,
                                                             int64_t stack_rows, double mu, double q, int counts,
                                                             const StackMoments m, float *__restrict__ x,
                                                             double *__restrict__ psi) {
    const int n_tiles = (a.n_f0 + 255) / 256;
    const int per_row = n_tiles * a.n_groups;
    const int P = (int)gridDim.x / per_row;
    const int xc = (int)blockIdx.x % kXcds, k = (int)blockIdx.x / kXcds;
    const int qq = k % per_row;
    const int tile = qq / a.n_groups, grp = qq % a.n_groups;
    if (tile * 256 + (int)(threadIdx.x & ~63u) >= a.n_f0) return;
    const int i = tile * 256 + (int)threadIdx.x;
    const double f0[1] = {a.f0_min + (double)i * a.f0_step};
    const int64_t tt = (int64_t)grp * a.n_f0 + i;
    const int64_t n_tpl = (int64_t)a.n_groups * a.n_f0;
    const int channels = counts ? 2 * a.n_groups : a.n_groups;
    for (int r = xc + kXcds * (k / per_row); r < R; r += P) {
        DetView D = a.det[0];
        D.store = (const char *)D.store + (int64_t)r * stack_bytes;
        D.wq += (int64_t)r * stack_rows;
        D.w += (int64_t)r * stack_rows;
        Acc<1> acc;
        acc.zero();
        accumulate_det<kStoreCoarse, false, 1, 16, HTable, 1>(D, HTable{D.H + (int64_t)grp * D.n_seg}, f0, acc);
        if (i >= a.n_f0) continue;
        const double rp = stack_ratio(acc.s[0], m, tt, mu, mu, 1);
        float *xr = x + (int64_t)r * channels * a.n_f0;
        xr[tt] = (float)rp;
        if (psi) psi[(int64_t)r * n_tpl + tt] = rp;
        if (counts) {
            const int nn = m.n[tt];
            double rc = 0.0;
            if (nn > 0) {
                const double e = ((double)nn * mu) * q;  // N m q: the count's mean under noise
                rc = ((double)acc.cnt[0] - e) / sqrt(e * (1.0 - q));
            }
            xr[n_tpl + tt] = (float)rc;
        }
    }
}

hipError_t launch_stack_features(const EvalArgs &a, int R, int64_t stack_bytes, int64_t stack_rows, double mu,
                                 double q, int counts, StackMoments m, float *x, double *psi, hipStream_t st) {
    const int P = (R + kXcds - 1) / kXcds * kXcds;
    const int64_t blocks = (int64_t)((a.n_f0 + 255) / 256) * a.n_groups * P;
    if (blocks > 0x7fffffff || R > 65535 || R < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(stack_features_kernel, dim3((unsigned)blocks), dim3(256), 0, st, a, R, stack_bytes,
                       stack_rows, mu, q, counts, m, x, psi);
    return hipGetLastError();
}

// The ranking without a network (the method alone): block b of fine group
// G = b / nbg, fine f0 indices (b % nbg) W .. + W - 1 (below 2 L), scores the
// largest coarse power ratio x[r][ch][i / 2] over its f0 and over the coarse
// channels map[G][0], map[G][1] (-1: none) of the coarse groups nearest G.
__global__ void coarse_block_scores_kernel(const float *__restrict__ x, int R, int nb, int c_in, int L, int W,
                                           int nbg, const int32_t *__restrict__ map, float *__restrict__ score) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (int64_t)R * nb) return;
    const int r = (int)(e / nb), b = (int)(e % nb);
    const int G = b / nbg, i0 = (b % nbg) * W, i1 = min(i0 + W, 2 * L);
    const float *xr = x + (int64_t)r * c_in * L;
    float best = -__builtin_inff();
    for (int h = 0; h < 2; ++h) {
        const int ch = map[2 * G + h];
        if (ch < 0) continue;
        for (int l = i0 / 2; l <= (i1 - 1) / 2; ++l) best = fmaxf(best, xr[(int64_t)ch * L + l]);
    }
    score[e] = best;
}

hipError_t launch_coarse_block_scores(const float *x, int R, int nb, int c_in, int L, int W, int nbg,
                                      const int32_t *map, float *score, hipStream_t st) {
    const int64_t total = (int64_t)R * nb;
    if (total < 1 || (total + 255) / 256 > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(coarse_block_scores_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, x, R,
                       nb, c_in, L, W, nbg, map, score);
    return hipGetLastError();
}

// Explicit template lists: lane q of realisation r evaluates template
// idx[r][q] of the grid (any order; each lane reads its own group's track
// factors).  Writes the power critical ratio (mu = var = 1) or NaN.  Rows
// rr >= *n_rows are skipped when the device count n_rows is given.
template <int STORE>
__global__ __launch_bounds__(256) void list_eval_kernel(const EvalArgs a, int64_t stack_bytes,
                                                        int64_t stack_rows, const int32_t *__restrict__ idx,
                                                        int m, const int32_t *__restrict__ rmap,
                                                        const int32_t *__restrict__ n_rows, const StackMoments mom,
                                                        double *__restrict__ out_psi) {
    const int q = blockIdx.x * 256 + threadIdx.x;
    const int rr = blockIdx.y;                  // row of idx and out_psi
    if (n_rows && rr >= *n_rows) return;
    const int r = rmap ? rmap[rr] : rr;         // realisation of the stack
    DetView D = a.det[0];
    D.store = (const char *)D.store + (int64_t)r * stack_bytes;
    D.wq += (int64_t)r * stack_rows;
    const int64_t n_tpl = (int64_t)a.n_groups * a.n_f0;
    int t = q < m ? idx[(int64_t)rr * m + q] : 0;
    const bool bad = t < 0 || t >= n_tpl;  // not a template of the grid: NaN
    if (bad) t = 0;
    const int i_f0 = t % a.n_f0, grp = t / a.n_f0;
    const double f0 = a.f0_min + (double)i_f0 * a.f0_step;
    const double *__restrict__ H = D.H + (int64_t)grp * D.n_seg;
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        (void *)D.store, Store<STORE>::kBytes, D.n_bins + 2, kBufDword3);
    double s = 0.0;
    int cnt = 0;
    for (int j0 = 0; j0 < D.n_seg; j0 += kChunk) {
        const int je = min(j0 + kChunk, D.n_seg);
        float sc = 0.0f;
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
            for (int k = 0; k < 8; ++k) sc = __builtin_fmaf(D.wq[j + k], p[k], sc);
        }
        for (; j < je; ++j) {
            const double x = f0 * H[j];
            const double vv = x + D.cshift;
            const unsigned ix = (unsigned)__double2int_rz(vv);
            sc = __builtin_fmaf(D.wq[j], Store<STORE>::get(rs, (int)ix, j * D.pitch_bytes, cnt), sc);
        }
        s += (double)sc;
    }
    if (q >= m) return;
    out_psi[(int64_t)rr * m + q] = bad ? __builtin_nan("") : stack_stat(s, cnt, mom, t, 1.0, 1.0, 0);
}

hipError_t launch_list_eval(int store, const EvalArgs &a, int R, int64_t stack_bytes, int64_t stack_rows,
                            const int32_t *idx, int m, const int32_t *rmap, const int32_t *n_rows, StackMoments mom,
                            double *out_psi, hipStream_t st) {
    if (R > 65535 || R < 1 || m < 1) return hipErrorInvalidValue;
    dim3 grid((unsigned)((m + 255) / 256), (unsigned)R), block(256);
    if (store == LTGW_STORE_F32)
        hipLaunchKernelGGL(list_eval_kernel<LTGW_STORE_F32>, grid, block, 0, st, a, stack_bytes, stack_rows, idx, m, rmap, n_rows, mom, out_psi);
    else if (store == LTGW_STORE_BF16)
        hipLaunchKernelGGL(list_eval_kernel<LTGW_STORE_BF16>, grid, block, 0, st, a, stack_bytes, stack_rows, idx, m, rmap, n_rows, mom, out_psi);
    else
        hipLaunchKernelGGL(list_eval_kernel<LTGW_STORE_FP8>, grid, block, 0, st, a, stack_bytes, stack_rows, idx, m, rmap, n_rows, mom, out_psi);
    return hipGetLastError();
}

// Proposal blocks evaluated in place: workgroup (x, rr) of TPB threads takes
// NB = TPB / W blocks blk[r][x NB .. x NB + NB) of realisation r = rmap[rr]
// (or rr), W lanes per block, lane l on fine f0 index (b % nbg) W + l of
// group b / nbg.  Workgroups of one wavefront serve block counts that are not
// a multiple of 256 / W (a realisation's last workgroup is then at most one
// wavefront short of full).
// Each wavefront stages its own blocks' track factors in LDS per chunk of 32
// segments (no workgroup barrier: a wavefront's LDS accesses complete in
// order), so the only vector-memory access per template and segment is the
// gather; the sums are those of the listed evaluation, in the same order.
// Writes the expanded template (-1 past the grid) and its ratio (NaN there).
// SB: segments per batch of gathers in flight.
template <int STORE, int W, int SB, int TPB>
__global__ __launch_bounds__(TPB) void block_eval_kernel(const EvalArgs a, int R, int64_t stack_bytes,
                                                         int64_t stack_rows, const int32_t *__restrict__ blk, int K,
                                                         int nbg, const int32_t *__restrict__ rmap,
                                                         const int32_t *__restrict__ n_rows, const StackMoments mom,
                                                         int32_t *__restrict__ out_tpl,
                                                         double *__restrict__ out_psi) {
    constexpr int NB = TPB / W, SPW = 64 / W;  // blocks per workgroup, per wavefront
    __shared__ double sh[NB][kChunk];
    // XCD order as in stack_eval_kernel: the workgroups of one row share an
    // XCD (and its L2), consecutive rows go to different XCDs
    const int per_row = (K + NB - 1) / NB;
    const int xcd = (int)blockIdx.x % kXcds, kk = (int)blockIdx.x / kXcds;
    const int rr = xcd + kXcds * (kk / per_row), part = kk % per_row;
    if (rr >= R || (n_rows && rr >= *n_rows)) return;  // the whole workgroup
    const int r = rmap ? rmap[rr] : rr;
    const int slot = (int)threadIdx.x / W, lf = (int)threadIdx.x % W;
    const int lane = (int)threadIdx.x & 63, slot0 = ((int)threadIdx.x >> 6) * SPW;
    const int q = part * NB + slot;
    const int b = q < K ? blk[(int64_t)r * K + q] : -1;
    const int i = (b >= 0 ? (b % nbg) * W : 0) + lf;
    const bool valid = b >= 0 && i < a.n_f0;
    const int grp = b >= 0 ? b / nbg : 0;
    // the group of each of this wavefront's slots, for its staging lanes
    int sgrp[SPW];
#pragma unroll
    for (int u = 0; u < SPW; ++u) sgrp[u] = __shfl(grp, u * W, 64);
    DetView D = a.det[0];
    D.store = (const char *)D.store + (int64_t)r * stack_bytes;
    D.wq += (int64_t)r * stack_rows;
    const double f0 = a.f0_min + (double)(valid ? i : 0) * a.f0_step;
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        (void *)D.store, Store<STORE>::kBytes, D.n_bins + 2, kBufDword3);
    const double *hrow = sh[slot];
    double s = 0.0;
    int cnt = 0;
    for (int j0 = 0; j0 < D.n_seg; j0 += kChunk) {
        const int nj = min(kChunk, D.n_seg - j0);
        // the previous chunk's reads of this wavefront are ahead of these writes
#pragma unroll
        for (int u = 0; u < (SPW * kChunk + 63) / 64; ++u) {
            const int e = u * 64 + lane;
            if (e < SPW * kChunk) {
                const int sl = e / kChunk, k = e % kChunk;
                sh[slot0 + sl][k] = k < nj ? D.H[(int64_t)sgrp[sl] * D.n_seg + j0 + k] : 0.0;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        float sc = 0.0f;
        if (nj == kChunk) {
#pragma unroll 1
            for (int k0 = 0; k0 < kChunk; k0 += SB) {
                unsigned ix[SB];
#pragma unroll
                for (int k = 0; k < SB; ++k) {
                    const double x = f0 * hrow[k0 + k];
                    const double vv = x + D.cshift;
                    ix[k] = (unsigned)__double2int_rz(vv);
                }
                float p[SB];
#pragma unroll
                for (int k = 0; k < SB; ++k)
                    p[k] = Store<STORE>::get(rs, (int)ix[k], (j0 + k0 + k) * D.pitch_bytes, cnt);
#pragma unroll
                for (int k = 0; k < SB; ++k) sc = __builtin_fmaf(uniform_load(D.wq, j0 + k0 + k), p[k], sc);
            }
        } else {
            for (int k = 0; k < nj; ++k) {
                const double x = f0 * hrow[k];
                const double vv = x + D.cshift;
                const unsigned ix = (unsigned)__double2int_rz(vv);
                sc = __builtin_fmaf(uniform_load(D.wq, j0 + k),
                                    Store<STORE>::get(rs, (int)ix, (j0 + k) * D.pitch_bytes, cnt), sc);
            }
        }
        s += (double)sc;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    if (q >= K) return;
    const int64_t o = (int64_t)rr * K * W + (int64_t)q * W + lf;
    const int64_t tt = (int64_t)grp * a.n_f0 + i;
    out_tpl[o] = valid ? (int32_t)tt : -1;
    out_psi[o] = valid ? stack_ratio(s, mom, tt, 1.0, 1.0, 0) : __builtin_nan("");
}

bool block_eval_supported(int W) { return W == 16 || W == 32 || W == 64; }

hipError_t launch_block_eval(int store, int W, const EvalArgs &a, int R, int64_t stack_bytes, int64_t stack_rows,
                             const int32_t *blk, int K, int nbg, const int32_t *rmap, const int32_t *n_rows,
                             StackMoments mom, int32_t *out_tpl, double *out_psi, hipStream_t st) {
    if (R > 65535 || R < 1 || K < 1 || !block_eval_supported(W)) return hipErrorInvalidValue;
    const int tpb = K % (256 / W) == 0 ? 256 : 64;
    const int NB = tpb / W;
    // rows rounded up to a multiple of the XCD count (the extra workgroups return)
    const int64_t wgs = (int64_t)((K + NB - 1) / NB) * ((R + kXcds - 1) / kXcds * kXcds);
    if (wgs > 0x7fffffff) return hipErrorInvalidValue;
    const dim3 grid((unsigned)wgs), block(tpb);
#define LTGW_BLOCK_EVAL(S, WW)                                                                                         \
    if (tpb == 256)                                                                                                    \
        hipLaunchKernelGGL((block_eval_kernel<S, WW, 16, 256>), grid, block, 0, st, a, R, stack_bytes, stack_rows, blk, \
                           K, nbg, rmap, n_rows, mom, out_tpl, out_psi);                                               \
    else                                                                                                               \
        hipLaunchKernelGGL((block_eval_kernel<S, WW, 16, 64>), grid, block, 0, st, a, R, stack_bytes, stack_rows, blk,  \
                           K, nbg, rmap, n_rows, mom, out_tpl, out_psi)
#define LTGW_BLOCK_EVAL_W(S)          \
    if (W == 16)                      \
        LTGW_BLOCK_EVAL(S, 16);       \
    else if (W == 32)                 \
        LTGW_BLOCK_EVAL(S, 32);       \
    else                              \
        LTGW_BLOCK_EVAL(S, 64)
    if (store == LTGW_STORE_F32) {
        LTGW_BLOCK_EVAL_W(LTGW_STORE_F32);
    } else if (store == LTGW_STORE_BF16) {
        LTGW_BLOCK_EVAL_W(LTGW_STORE_BF16);
    } else {
        LTGW_BLOCK_EVAL_W(LTGW_STORE_FP8);
    }
#undef LTGW_BLOCK_EVAL_W
#undef LTGW_BLOCK_EVAL
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
// lists blk[r][0..K) expanded to W consecutive f0 each (-1 past the grid);
// rows q >= *n_rows are skipped when the device count is given.
__global__ void expand_blocks_kernel(const int32_t *blk, int K, int W, int two_L, int nbg, const int32_t *rmap,
                                     const int32_t *n_rows, int64_t total, int32_t *tpl) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= total) return;
    const int64_t row = e / ((int64_t)K * W);
    if (n_rows && row >= *n_rows) return;
    const int rem = (int)(e % ((int64_t)K * W));
    const int q = rem / W, j = rem % W;
    const int64_t r = rmap ? rmap[row] : row;
    const int b = blk[r * K + q];
    const int g = b / nbg, i = (b % nbg) * W + j;
    tpl[e] = (b >= 0 && i < two_L) ? g * two_L + i : -1;
}

hipError_t launch_expand_blocks(const int32_t *blk, int K, int W, int two_L, int nbg, const int32_t *rmap,
                                const int32_t *n_rows, int rows, int32_t *tpl, hipStream_t st) {
    const int64_t total = (int64_t)rows * K * W;
    hipLaunchKernelGGL(expand_blocks_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, blk, K, W,
                       two_L, nbg, rmap, n_rows, total, tpl);
    return hipGetLastError();
}

// Best entry of each row of psi[rows][n] (largest finite value, ties to the
// lowest index; index = position, or idx[row][position] when idx is given):
// one block per row, strided scan and an LDS tree.  No finite value: -1, -inf.
__device__ inline bool best_before(double a, int ia, double b, int ib) {
    return a > b || (a == b && (unsigned)ia < (unsigned)ib);
}

__global__ __launch_bounds__(256) void row_best_kernel(const double *psi, int64_t n, const int32_t *idx,
                                                       const int32_t *n_rows, int32_t *best_idx,
                                                       double *best_psi) {
    __shared__ double sv[256];
    __shared__ int si[256];
    const int64_t row = blockIdx.x;
    if (n_rows && row >= *n_rows) return;  // the whole block: no barrier is skipped by part of it
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

hipError_t launch_row_best(const double *psi, int rows, int64_t n, const int32_t *idx, const int32_t *n_rows,
                           int32_t *best_idx, double *best_psi, hipStream_t st) {
    if (rows < 1 || n < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(row_best_kernel, dim3(rows), dim3(256), 0, st, psi, n, idx, n_rows, best_idx, best_psi);
    return hipGetLastError();
}

// The realisations that take the next step of a proposal, in ascending order,
// and their count (one workgroup): those whose best ratio does not pass thr
// and, with cm given (the fallback rule), whose largest coarse ratio exceeds
// cthr.  flag[r] (when given) receives each decision.
__global__ __launch_bounds__(256) void take_rows_kernel(int R, const double *best_psi, double thr,
                                                        const double *cm, double cthr, int32_t *rows,
                                                        int32_t *count, int32_t *flag) {
    __shared__ int sh[4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int base = 0;
    for (int r0 = 0; r0 < R; r0 += 256) {  // uniform trip count: every thread meets every barrier
        const int r = r0 + (int)threadIdx.x;
        bool take = false;
        if (r < R) {
            take = !(best_psi[r] > thr) && (!cm || cm[r] > cthr);
            if (flag) flag[r] = take ? 1 : 0;
        }
        const unsigned long long m = __ballot(take);
        const int before = __popcll(m & ((1ull << lane) - 1ull));
        if (lane == 0) sh[wv] = __popcll(m);
        __syncthreads();
        int off = base;
        for (int k = 0; k < wv; ++k) off += sh[k];
        if (take) rows[off + before] = r;
        base += sh[0] + sh[1] + sh[2] + sh[3];
        __syncthreads();
    }
    if (threadIdx.x == 0) *count = base;
}

hipError_t launch_take_rows(int R, const double *best_psi, double thr, const double *cm, double cthr, int32_t *rows,
                            int32_t *count, int32_t *flag, hipStream_t st) {
    if (R < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(take_rows_kernel, dim3(1), dim3(256), 0, st, R, best_psi, thr, cm, cthr, rows, count, flag);
    return hipGetLastError();
}

// Later results (bi[q], bp[q]) for realisation rows[q], q < *count, merged
// into its best: the larger ratio, ties to the lower index.
__global__ void merge_rows_kernel(const int32_t *rows, const int32_t *count, const int32_t *bi, const double *bp,
                                  int32_t *best_idx, double *best_psi) {
    const int q = blockIdx.x * 256 + threadIdx.x;
    if (q >= *count) return;
    const int r = rows[q];
    const int32_t i = bi[q];
    const double v = bp[q];
    if (i < 0 || !(v == v)) return;
    const int32_t i0 = best_idx[r];
    const double v0 = best_psi[r];
    if (i0 < 0 || v > v0 || (v == v0 && i < i0)) {
        best_idx[r] = i;
        best_psi[r] = v;
    }
}

hipError_t launch_merge_rows(int R, const int32_t *rows, const int32_t *count, const int32_t *bi, const double *bp,
                             int32_t *best_idx, double *best_psi, hipStream_t st) {
    hipLaunchKernelGGL(merge_rows_kernel, dim3((unsigned)((R + 255) / 256)), dim3(256), 0, st, rows, count, bi, bp,
                       best_idx, best_psi);
    return hipGetLastError();
}

// The three per-realisation outputs of a proposal in one array of records,
// so that one copy brings them to the host.
__global__ void pack_results_kernel(int R, const int32_t *best_idx, const double *best_psi, const int32_t *fb,
                                    ProposeRecord *out) {
    const int r = blockIdx.x * 256 + threadIdx.x;
    if (r >= R) return;
    out[r] = ProposeRecord{best_psi[r], best_idx[r], fb[r]};
}

hipError_t launch_pack_results(int R, const int32_t *best_idx, const double *best_psi, const int32_t *fb,
                               ProposeRecord *out, hipStream_t st) {
    hipLaunchKernelGGL(pack_results_kernel, dim3((unsigned)((R + 255) / 256)), dim3(256), 0, st, R, best_idx,
                       best_psi, fb, out);
    return hipGetLastError();
}

// The evaluated blocks of each realisation: its K1 first-tier blocks, then
// its K2 second-tier blocks where flag2[r] says it took them, else -1.
__global__ void blocks_out_kernel(int64_t total, const int32_t *blk1, int K1, const int32_t *blk2, int K2,
                                  const int32_t *flag2, int32_t *out) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= total) return;
    const int KB = K1 + K2;
    const int64_t r = e / KB;
    const int k = (int)(e % KB);
    out[e] = k < K1 ? blk1[r * K1 + k] : (flag2[r] ? blk2[r * K2 + (k - K1)] : -1);
}

hipError_t launch_blocks_out(int R, const int32_t *blk1, int K1, const int32_t *blk2, int K2, const int32_t *flag2,
                             int32_t *out, hipStream_t st) {
    const int64_t total = (int64_t)R * (K1 + K2);
    hipLaunchKernelGGL(blocks_out_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, total, blk1, K1,
                       blk2, K2, flag2, out);
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

}  // namespace ltgw
