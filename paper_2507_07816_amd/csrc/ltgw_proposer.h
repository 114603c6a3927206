// Internal interface of the learned proposer's kernels (ltgw_stack.hip,
// ltgw_proposer.hip) for its C-ABI layer (ltgw_proposer_api.hip).  Not part
// of the public boundary.
#pragma once
#include "ltgw_internal.h"

namespace ltgw {

// Per-template moments of a stack level (the weights are the same for every
// realisation): W1 = sum of in-band weights, W2 = sum of their squares, N =
// in-band segments, each in the statistic's own summation order.
// The ratio the stack kernels write: the power ratio, or with count set the
// number-count ratio (c - N q) / sqrt(N q (1 - q)) with q = exp(-rho_th).
struct StackMoments {
    const double *w1, *w2;
    const int32_t *n;
    int count = 0;
    double q = 0.0;
};

hipError_t launch_stack_moments(int shift, const EvalArgs &a, double *w1, double *w2, int32_t *n, hipStream_t st);

hipError_t launch_stack_eval(int store, int shift, const EvalArgs &a, int R, int64_t stack_bytes,
                             int64_t stack_rows, double mu, double var, int nan_to_zero, const int32_t *rmap,
                             const int32_t *n_rows, StackMoments m, double *out_psi, hipStream_t st);
// The network's input from the coarse store (power ratios, and count ratios
// with counts != 0) in FP32 x[R][channels][n_f0]; psi (optional) the FP64
// power ratios [R][n_templates], NaN -> 0.
hipError_t launch_stack_features(const EvalArgs &a, int R, int64_t stack_bytes, int64_t stack_rows, double mu,
                                 double q, int counts, StackMoments m, float *x, double *psi, hipStream_t st);
// Block scores from the coarse power ratios alone (no network): the largest
// ratio of the coarse channels map[G][0..1] over the block's f0.
hipError_t launch_coarse_block_scores(const float *x, int R, int nb, int c_in, int L, int W, int nbg,
                                      const int32_t *map, float *score, hipStream_t st);
hipError_t launch_list_eval(int store, const EvalArgs &a, int R, int64_t stack_bytes, int64_t stack_rows,
                            const int32_t *idx, int m, const int32_t *rmap, const int32_t *n_rows, StackMoments mom,
                            double *out_psi, hipStream_t st);
// Whether launch_block_eval takes blocks of W templates.
bool block_eval_supported(int W);
hipError_t launch_block_eval(int store, int W, const EvalArgs &a, int R, int64_t stack_bytes, int64_t stack_rows,
                             const int32_t *blk, int K, int nbg, const int32_t *rmap, const int32_t *n_rows,
                             StackMoments mom, int32_t *out_tpl, double *out_psi, hipStream_t st);
hipError_t launch_cells_to_templates(const int32_t *cells, int64_t n, int L, int32_t *tpl, hipStream_t st);
hipError_t launch_block_scores(const float *logits, int R, int c_out, int L, int W, int nbg, float *score,
                               hipStream_t st);
hipError_t launch_mask_blocks(float *score, const int32_t *blk, int R, int K, int nb, hipStream_t st);
hipError_t launch_expand_blocks(const int32_t *blk, int K, int W, int two_L, int nbg, const int32_t *rmap,
                                const int32_t *n_rows, int rows, int32_t *tpl, hipStream_t st);
hipError_t launch_take_rows(int R, const double *best_psi, double thr, const double *cm, double cthr, int32_t *rows,
                            int32_t *count, int32_t *flag, hipStream_t st);
hipError_t launch_merge_rows(int R, const int32_t *rows, const int32_t *count, const int32_t *bi, const double *bp,
                             int32_t *best_idx, double *best_psi, hipStream_t st);
struct ProposeRecord {
    double psi;
    int32_t idx, fallback;
};
hipError_t launch_pack_results(int R, const int32_t *best_idx, const double *best_psi, const int32_t *fb,
                               ProposeRecord *out, hipStream_t st);
hipError_t launch_blocks_out(int R, const int32_t *blk1, int K1, const int32_t *blk2, int K2, const int32_t *flag2,
                             int32_t *out, hipStream_t st);
hipError_t launch_row_best(const double *psi, int rows, int64_t n, const int32_t *idx, const int32_t *n_rows,
                           int32_t *best_idx, double *best_psi, hipStream_t st);
hipError_t launch_templates_to_cells(const int32_t *tpl, int n, int L, const int32_t *mask, const double *psi,
                                     double min_psi, int32_t *cells, hipStream_t st);
hipError_t launch_noise(uint64_t seed, uint32_t stream, int r0, int R, int64_t n_per, float *out,
                        hipStream_t st);
hipError_t launch_inject_stack(float *power, int R, int32_t n_seg, int32_t n_bins, int64_t k_lo,
                               double t_sft, const double *t_seg, const double *v, const float *w,
                               const double *params, double sx, double sy, double sz, double t0,
                               unsigned long long *undecided, hipStream_t st);
hipError_t launch_cnn_forward(const float *params, const float *x, int B, int c_in, int c_out, int L,
                              float *act /* [3][B][32][L] */, float *logits, hipStream_t st);
// The forward pass for inference only, fused in one kernel (no activations
// kept); the same logits bit for bit.  Supported for c_in, c_out <= 32, L <= 256.
// scratch: cnn_infer_scratch_shorts(c_in) shorts of device memory (the packed
// weights).  logits and score may each be NULL; score receives the scores of
// ltgw_propose's blocks of W fine f0 (W = 16, 32 or 64) as launch_block_scores.
bool cnn_infer_supported(int c_in, int c_out, int L);
int64_t cnn_infer_scratch_shorts(int c_in);
hipError_t launch_cnn_infer(const float *params, const float *x, int B, int c_in, int c_out, int L, short *scratch,
                            float *logits, float *score, int W, hipStream_t st);
hipError_t launch_cnn_backward(const float *params, const float *x, int B, int c_in, int c_out, int L,
                               const float *act, const float *dlogits, float *work, int64_t work_floats,
                               float *grads, hipStream_t st);
int64_t cnn_work_floats(int B, int c_in, int c_out, int L);
int64_t cnn_n_params(int c_in, int c_out);
hipError_t launch_softmax_xent(const float *logits, int B, int n_cells, const int32_t *target,
                               int n_valid, float *loss, float *dlogits, hipStream_t st);
hipError_t launch_adam(float *p, const float *g, float *m, float *v, int64_t n, float lr, float b1,
                       float b2, float eps, int step, hipStream_t st);
hipError_t launch_select_top(const float *score, int R, int n, int M, int32_t *out_idx, hipStream_t st);

}  // namespace ltgw
