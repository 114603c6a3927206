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

}  // namespace ltgw
