// Internal interface between the C-ABI layer (ltgw_api.hip) and the kernels
// (ltgw_kernels.hip).  Not part of the public boundary.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ltgw.h"

namespace ltgw {

constexpr double kC = 299792458.0;  // m/s, exact by SI definition

// One detector as the evaluation kernel sees it.
struct DetView {
    const void *store;      // [n_seg][pitch] elements, element 0 of a row = 0 guard
    int32_t pitch_bytes;    // bytes between rows (whole store < 2^31 bytes)
    int32_t store_elems;    // n_seg * pitch
    const double *H;        // [n_groups][n_seg] bin-scaled track factor (0 = masked)
    const float *wq;        // [n_seg] weight times per-segment store scale
    const float *w;         // [n_seg] weights (for W1, W2)
    double cshift;          // 1.5 - k_lo
    int32_t n_seg;
    int32_t n_bins;
};

struct EvalArgs {
    DetView det[LTGW_MAX_DET];
    int32_t n_det;
    int32_t n_f0;
    int32_t n_groups;       // n_sky * n_brake * n_tau
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
hipError_t launch_check_velocity(const double *v, int32_t n_seg, unsigned long long *bad,
                                 hipStream_t st);
hipError_t launch_spin_factor(const double *t_seg, int32_t n_seg, double t0, const double *tau,
                              int32_t n_tau, const double *brake, int32_t n_brake, double *g,
                              unsigned long long *undecided, hipStream_t st);
hipError_t launch_track_factor(const double *g, int32_t n_tn, const double *v, int32_t n_seg,
                               const double *sky, int32_t n_sky, double t_sft, double *H,
                               hipStream_t st);
hipError_t launch_eval(int store, bool weighted, const EvalArgs &a, hipStream_t st);
hipError_t launch_psi(uint32_t stat, int64_t n, const double *s, const int32_t *c,
                      const int32_t *N, const double *w1, const double *w2, double q,
                      double *out, hipStream_t st);

struct TopkDecode {
    double f0_min, f0_step;
    int32_t n_f0, n_tau, n_brake;
    const double *tau;
    const double *brake;
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
