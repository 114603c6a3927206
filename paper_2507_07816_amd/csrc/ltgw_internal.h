// Internal interface between the C-ABI layer (ltgw_api.hip) and the kernels
// (ltgw_kernels.hip).  Not part of the public boundary.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ltgw.h"

namespace ltgw {

constexpr double kC = 299792458.0;  // m/s, exact by SI definition
constexpr double kInvC = 1.0 / kC;  // RN(1/c), folded by the compiler

// Internal store format (beside LTGW_STORE_F32/BF16/FP8): the proposer's
// coarse store, 32-bit words holding a bfloat16 power sum in the upper half
// and the count of the block's pixels above rho_th in the low byte.
constexpr int kStoreCoarse = 3;

// One detector as the evaluation kernel sees it.
struct DetView {
    const void *store;      // [n_seg][pitch] elements, element 0 of a row = 0 guard
    int32_t pitch_bytes;    // bytes between rows (whole store < 2^31 bytes)
    const double *H;        // [n_groups][n_seg] bin-scaled track factor (0 = masked), or
                            // NULL: formed on the fly from g and D
    const double *g;        // [n_tn][n_seg] spin-down factors (Eq. 1)
    const double *D;        // [n_sky][n_seg] Doppler factors (Eq. 2)
    double t_sft;
    const float *wq;        // [n_seg] weight times per-segment store scale
    const float *w;         // [n_seg] weights (for W1, W2)
    const int64_t *wfix;    // [n_seg][3] exact fixed-point w, w^2 high, w^2 low (moments pass)
    double cshift;          // 1.5 - k_lo
    int32_t n_seg;
    int32_t n_bins;
    const int2 *win;        // [n_groups][win_blocks] first and last segment where a run of win_run
                            // f0 has a lane in band ({n_seg, -1}: none), or NULL: every segment
    int32_t win_blocks;     // runs per group
    int32_t win_run;        // f0 per run (64: batch tiles; 256: single-search tiles)
    int32_t w_sky_stride;   // 0: wq, w shared by every group; else they are [n_sky][n_seg]
                            // (antenna-pattern weights) with rows this far apart
};

struct EvalArgs {
    DetView det[LTGW_MAX_SEARCH_DET];  // detectors one search sums
    int32_t n_det;
    int32_t n_f0;
    int32_t n_groups;       // n_sky * n_brake * n_tau
    int32_t n_tn;           // n_brake * n_tau
    double f0_min, f0_step;
    float w_uniform;        // weight value when all weights are equal
    // context-owned results
    double *s;
    int32_t *c;
    int32_t *n;
    double *w1;
    double *w2;
    // optional caller outputs
    float *out_s;
    int32_t *out_c;
    int32_t *out_n;
    unsigned long long *in_band_total;
};

// Kernel launchers (all asynchronous on `st`; return the launch status).
hipError_t launch_ingest(int store, const float *power, int32_t n_seg, int32_t n_bins,
                         int64_t pitch, void *out, float *scale, const float *w, float *wq,
                         float rho_th, unsigned long long *bad, hipStream_t st);
// The learned proposer's stacks: realisations [R][n_seg][n_bins] into the fine
// store (as launch_ingest per row) and, in the same pass, the coarse store of
// S x 2 blocks: [R][n_seg / S][pitch2] words (bfloat16 sum << 16 | count);
// crs NULL: the fine store alone, S rows per workgroup (n_bins even).
hipError_t launch_stack_ingest(int store, const float *power, int R, int32_t n_seg, int32_t n_bins, int S,
                               int64_t pitch, void *out, float *scale, const float *w, float *wq, float rho_th,
                               int64_t pitch2, unsigned *crs, unsigned long long *bad, hipStream_t st);
hipError_t launch_check_velocity(const double *v, int32_t n_seg, unsigned long long *bad,
                                 hipStream_t st);
hipError_t launch_spin_factor(const double *t_seg, int32_t n_seg, double t0, const double *tau,
                              int32_t n_tau, const double *brake, int32_t n_brake, double *g,
                              unsigned long long *pow_counts, hipStream_t st);  // [2]: undecided, slow phase
hipError_t launch_track_factor(const double *g, int32_t n_tn, const double *v, int32_t n_seg,
                               const double *sky, int32_t n_sky, double t_sft, double *H,
                               hipStream_t st);
// Statistic kernel.  moments_in_loop: also accumulate N, W1, W2 per segment
// (used when the weights have no exact fixed-point form); otherwise only s
// and c, with N, W1, W2 from launch_moments.  variant & 3: tile shape
// (templates per lane, segments per gather batch) = (1,8), (1,16), (2,8),
// (2,16); variant & 4: the grid is launched in generations of the blocks the
// device holds at once (cu_count x resident blocks per CU), so that the
// blocks of a launch walk the segments together and share rows in L2;
// variant & 8 (one detector): the segments are walked in slabs of 1024, one
// launch per slab, so that the blocks of a launch stay within a slab.
constexpr int kNumShapes = 4;
constexpr int kNumVariants = 16;
int variant_templates_per_block(int variant);
// *launches receives the number of statistic-kernel dispatches queued.
hipError_t launch_eval(int store, bool moments_in_loop, int variant, const EvalArgs &a, int cu_count,
                       hipStream_t st, int *launches);

// Batched searches (device-resident descriptors).
struct BatchSearch {
    DetView det[LTGW_MAX_SEARCH_DET];
    int32_t n_det;
    int32_t n_f0;
    int32_t n_tn;           // n_brake * n_tau; group = sky * n_tn + tn
    int32_t n_tiles;        // tiles of this search
    double f0_min, f0_step;
    double *s;
    int32_t *c;
    int32_t *n;
    double *w1;
    double *w2;
    unsigned *tiles_done;
    unsigned long long *t_done;
};
struct BatchTile {
    int32_t search, grp, tile, pad;
};
struct BatchArgs {
    const BatchSearch *searches;
    const BatchTile *tiles;
    int32_t n_tiles;
    unsigned *counter;
    unsigned long long *t_start;
    unsigned long long *in_band_total;
};
hipError_t launch_batch(int store, bool moments_in_loop, int variant, const BatchArgs &a, int grid,
                        hipStream_t st);
int batch_blocks_per_cu(int store, bool moments_in_loop, int variant);
// In-band segment windows of every (group, run of win_run f0) of one detector.
hipError_t launch_windows(const DetView &D, int n_groups, int n_tn, double f0_min, double f0_step, int n_f0,
                          int2 *win, hipStream_t st);
hipError_t launch_doppler(const double *v, int32_t n_seg, const double *sky, int32_t n_sky,
                          double *D, hipStream_t st);
hipError_t launch_fill_u32(unsigned *p, int n, unsigned v, hipStream_t st);
hipError_t launch_f64_to_f32(const double *in, float *out, int64_t n, hipStream_t st);

hipError_t launch_fill_u64(unsigned long long *p, int n, unsigned long long v, hipStream_t st);

// In-band moments N, W1, W2 of every template from the in-band f0 range of
// each (group, segment): exact int64 range-adds into diff (4 arrays of
// [n_groups][n_f0 + 1], zeroed here) and a prefix scan per group.
// weights: 0 = uniform (W1 = N w, W2 = N w^2), 1 = fixed point
// (W1 = sum wfix * 2^e0, W2 = (sum hi * 2^32 + sum lo) * 2^(2 e0)).
hipError_t launch_moments(const EvalArgs &a, int weights, int e0, int64_t *diff,
                          hipStream_t st);
hipError_t launch_psi(uint32_t stat, int64_t n, const double *s, const int32_t *c,
                      const int32_t *N, const double *w1, const double *w2, double q,
                      double *out, hipStream_t st);

// How a top-k record gets its parameters: from the lattice's index split, or,
// for an explicit template list, from the device copy of that list (sky = -1).
struct TopkDecode {
    double f0_min, f0_step;
    int32_t n_f0, n_tau, n_brake;
    const double *tau;
    const double *brake;
    const ltgw_template *list = nullptr;
};
// Scratch for top-k: two candidate buffers of (psi, index) pairs.
hipError_t launch_topk(uint32_t stat, int64_t n, const double *s, const int32_t *c,
                       const int32_t *N, const double *w1, const double *w2, double q, int32_t k,
                       double *cand_psi_a, int64_t *cand_idx_a, double *cand_psi_b,
                       int64_t *cand_idx_b, int64_t cand_cap, const TopkDecode &dec,
                       ltgw_candidate *out_dev, int32_t *n_out_dev, hipStream_t st);
int64_t topk_scratch_entries(int64_t n, int32_t k);

hipError_t launch_inject(float *power, int32_t n_seg, int32_t n_bins, int64_t k_lo,
                         double t_sft, const double *t_seg, const double *v, const float *w,
                         double f0, double tau, double brake, double sx, double sy, double sz,
                         double t0, float amp, unsigned long long *undecided, hipStream_t st);

}  // namespace ltgw
