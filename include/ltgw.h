/*
 * ltgw — template-bank evaluation of the long-transient gravitational-wave
 * detection statistic on AMD Instinct MI355X (gfx950).
 *
 * Method: Merou, Tenorio, Sintes, "GPU-Accelerated Searches for
 * Long-Transient Gravitational Waves from Newborn Neutron Stars".
 *   - track      f_gw(t) = f0 ((t - T0)/tau + 1)^(1/(1-n))           Sec. 1, Eq. 1
 *   - Doppler    f^(t)   = f_gw(t) (1 + v(t).n/c)                      Sec. 1, Eq. 2
 *   - statistic  normalised power (or number count) of the data bins the
 *                track selects, weighted, summed over segments         Sec. 2
 *   - ratio      Psi = (s - <s>) / sigma_s                             Sec. 2, Eq. 4
 *   - bank       cubic lattice in (f0, tau, n) per sky direction       Sec. 2
 *
 * Conventions shared by every entry point
 *   - Return value: LTGW_OK (0) or a negative LTGW_E_* code.  No C++
 *     exception crosses this boundary.  After an error the context stays
 *     usable and ltgw_last_error() describes the failure.
 *   - Pointers are plain host or device addresses.  Where an argument may be
 *     either, the library asks the HIP runtime which one it is.
 *   - All device work is enqueued on the context's stream.  Calls marked
 *     "synchronous" wait for that stream before returning.
 *   - A context is used by one host thread at a time.
 *
 * Arithmetic contract (the bin of every template and segment is exact)
 *   For detector d, segment j (reference time t_j) and template
 *   (f0, tau, n, sky unit vector nhat), with every operation a single
 *   correctly rounded FP64 operation in the order written:
 *     masked if t_j < T0
 *     u  = 1 + (t_j - T0)/tau      e = 1/(1 - n)      g = RN(u^e)
 *     vn = (vx nx + vy ny) + vz nz D = 1 + vn/c       (c = 299792458 m/s)
 *     h  = g*D   H = h*T_sft   f0 = f0_min + i*f0_step   x = f0*H
 *     b  = floor(x + 0.5) - k_lo   in band iff 0 <= b < n_bins
 *   g is the correctly rounded power; the library computes it in
 *   double-double arithmetic and counts any value whose rounding it cannot
 *   decide (ltgw_diagnostics).  In-band segments add
 *     s += w_j * P_d[j][b]   (FP32 products, FP32 partial sums of <= 32
 *                             segments, FP64 running total)
 *     c += (rho_d[j][b] > rho_th)  (decided on the FP32 input power)
 *     N += 1, W1 += w_j, W2 += w_j^2
 */
#ifndef LTGW_H
#define LTGW_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define LTGW_OK 0
#define LTGW_E_INVALID_ARG (-1) /* NaN/inf, n <= 1, tau <= 0, f0 <= 0, non-unit sky,
                                   |v| >= c, shape mismatch, k out of range, NULL */
#define LTGW_E_STATE (-2)       /* call order: eval before load/velocity, topk before eval,
                                   unknown detector */
#define LTGW_E_NOMEM (-3)       /* device allocation failed */
#define LTGW_E_DEVICE (-4)      /* HIP runtime error; text in ltgw_last_error */
#define LTGW_E_UNSUPPORTED (-5) /* valid request outside what this build supports */

/* ---- storage of the spectrogram on the device -------------------------- */
#define LTGW_STORE_F32 0  /* IEEE binary32                                     */
#define LTGW_STORE_BF16 1 /* bfloat16, round to nearest even                   */
#define LTGW_STORE_FP8 2  /* OCP E4M3 (E4M3FN), per-segment FP32 scale =
                             rowmax/448 (1 for an all-zero row), value/scale
                             rounded to nearest even, saturating at 448        */

/* ---- statistics -------------------------------------------------------- */
#define LTGW_STAT_POWER 1u /* weighted normalised-power sum s (Sec. 2)          */
#define LTGW_STAT_COUNT 2u /* number count c of pixels above rho_th (Sec. 2)    */

#define LTGW_MAX_DET 4    /* detectors per context                              */
#define LTGW_MAX_TOPK 256 /* largest k accepted by ltgw_topk_candidates         */

typedef struct ltgw_ctx ltgw_ctx;

/* ltgw_create: open a context on HIP device `device`.
 *   hip_stream: a hipStream_t to enqueue all work on, or NULL for the
 *               device's null stream.  The library never destroys it.
 *   out: receives the context (owned by the caller; free with ltgw_destroy).
 * Errors: INVALID_ARG (bad device, NULL out), DEVICE. */
int32_t ltgw_create(int32_t device, void *hip_stream, ltgw_ctx **out);

/* ltgw_destroy: wait for the context's stream, free every device buffer the
 * library allocated and the context itself.  NULL is ignored. */
void ltgw_destroy(ltgw_ctx *ctx);

/* ltgw_last_error: text of the last failure on ctx (empty string if none).
 * Valid until the next call on ctx.  With ctx == NULL: the last failure of
 * ltgw_create on this thread. */
const char *ltgw_last_error(const ltgw_ctx *ctx);

/* ---- load_spectrogram ------------------------------------------------------
 * Normalised power rho_j of 8-s Hann-windowed SFTs (Sec. 2) of one detector:
 * a time x frequency map whose row j is segment j and column b is absolute
 * frequency bin k_lo + b, i.e. frequency (k_lo + b)/t_sft. */
typedef struct {
    int32_t n_seg;        /* rows (segments), >= 1                                 */
    int32_t n_bins;       /* columns, >= 1                                         */
    int64_t k_lo;         /* absolute bin index of column 0, 2 <= k_lo < 2^30      */
    double t_sft;         /* segment length in seconds, > 0 (bin width 1/t_sft)    */
    const double *t_seg;  /* [n_seg] reference time of each segment (host or
                             device), same epoch as T0                             */
    const float *weights; /* [n_seg] per-segment weights w_j > 0 (host or device),
                             or NULL for all 1 (antenna-pattern and noise-floor
                             weighting, Sec. 2)                                    */
    float rho_th;         /* number-count threshold (compared in FP32, strict >)  */
    int32_t store;        /* LTGW_STORE_*                                          */
} ltgw_spec_desc;

/* ltgw_load_spectrogram: copy detector `det`'s spectrogram into a
 * library-owned device store.
 *   power: FP32 [n_seg][n_bins], row-major, contiguous, host or device.
 *          Values must be finite and >= 0 (normalised power).
 * The store keeps the power in the requested format with the number-count
 * bit (rho > rho_th, decided on the FP32 input) in the sign bit, which is
 * free because power is non-negative.  Reloading a detector replaces it and
 * drops its velocity table.  Synchronous: the caller may reuse `power` on
 * return.
 * Errors: INVALID_ARG (shape, NULL, negative or non-finite power, bad store,
 * det outside [0, LTGW_MAX_DET)), NOMEM, DEVICE. */
int32_t ltgw_load_spectrogram(ltgw_ctx *ctx, int32_t det, const ltgw_spec_desc *d,
                              const float *power);

/* ---- set_velocity_table ----------------------------------------------------
 * Detector velocity relative to the solar-system barycentre (Eq. 2), FP64
 * [n_seg][3] in m/s, equatorial Cartesian, at the segment reference times;
 * host or device.  n_seg must equal the loaded spectrogram's.  |v| < c for
 * every row.  Synchronous.
 * Errors: STATE (no spectrogram for det), INVALID_ARG, NOMEM, DEVICE. */
int32_t ltgw_set_velocity_table(ltgw_ctx *ctx, int32_t det, const double *v_xyz, int32_t n_seg);

/* ---- eval_templates --------------------------------------------------------
 * Cubic-lattice bank (Sec. 2).  Template index order (f0 fastest):
 *     index = ((sky * n_brake + i_n) * n_tau + i_tau) * n_f0 + i_f0 */
typedef struct {
    double f0_min;       /* > 0, Hz                                         */
    double f0_step;      /* >= 0, Hz; f0_i = f0_min + i*f0_step             */
    int32_t n_f0;        /* >= 1                                            */
    const double *tau;   /* [n_tau] host, each > 0 (s)                      */
    int32_t n_tau;       /* >= 1                                            */
    const double *brake; /* [n_brake] host, each > 1 (braking index n)      */
    int32_t n_brake;     /* >= 1                                            */
    const double *sky;   /* [n_sky][3] host, unit vectors (|1 - |n|| <= 1e-12) */
    int32_t n_sky;       /* >= 1                                            */
    double t0;           /* T0 of Eq. 1, same epoch as t_seg                */
    uint32_t det_mask;   /* bit d selects detector d; 0 = every loaded one  */
} ltgw_grid;

/* ltgw_eval_templates: statistic of every template of the grid, summed over
 * the selected detectors.
 *   stats: LTGW_STAT_POWER | LTGW_STAT_COUNT (both are always computed; the
 *          mask is validated and recorded for ltgw_topk_candidates).
 *   out_s: FP32 [n_templates] device buffer or NULL (power sum s).
 *   out_c: int32 [n_templates] device buffer or NULL (number count c).
 *   out_n: int32 [n_templates] device buffer or NULL (in-band segments N).
 * Results (s, c, N, W1, W2) are also kept in the context for
 * ltgw_topk_candidates and ltgw_psi until the next eval.  Asynchronous.
 * Errors: STATE (no detector loaded / velocity missing for a selected one),
 * INVALID_ARG (grid values, x = f0*H beyond 2^30, more than 2^31 templates),
 * NOMEM, DEVICE. */
int32_t ltgw_eval_templates(ltgw_ctx *ctx, const ltgw_grid *g, uint32_t stats, float *out_s,
                            int32_t *out_c, int32_t *out_n);

/* ---- critical ratios ---------------------------------------------------------
 * Eq. 4 with Exp(1) noise moments: power Psi = (s - W1)/sqrt(W2); count
 * Psi = (c - N q)/sqrt(N q (1 - q)) with q = exp(-(double)rho_th) taken from
 * the host C library.  Templates with N = 0 get NaN. */

/* ltgw_psi: FP64 critical ratio of every template of the last eval into
 * out_psi (device buffer, [n_templates]).  stat: one LTGW_STAT_* value.
 * Asynchronous.  Errors: STATE (no eval), INVALID_ARG. */
int32_t ltgw_psi(ltgw_ctx *ctx, uint32_t stat, double *out_psi);

/* One ranked template. */
typedef struct {
    int64_t index;   /* template index                                 */
    double f0;       /* f0_min + i_f0*f0_step (FP64, as evaluated)     */
    double tau;
    double brake;
    int32_t sky;     /* sky index                                      */
    int32_t n_valid; /* in-band segments N                             */
    double stat;     /* s (power) or c (count) as FP64                 */
    double psi;      /* critical ratio                                 */
} ltgw_candidate;

/* ltgw_topk_candidates: the k templates of the last eval with the largest
 * critical ratio for statistic `stat`, ordered by (psi descending, index
 * ascending); templates with N = 0 never rank.  Detection compares these
 * ratios with a noise-only threshold (Sec. 3).
 *   k: 1 .. LTGW_MAX_TOPK.  out_host: caller-owned host array of k records.
 *   n_out: receives the number written (<= k).
 * Synchronous.  Errors: STATE (no eval), INVALID_ARG, DEVICE. */
int32_t ltgw_topk_candidates(ltgw_ctx *ctx, uint32_t stat, int32_t k, ltgw_candidate *out_host,
                             int32_t *n_out);

/* ---- diagnostics --------------------------------------------------------- */
typedef struct {
    int64_t pow_undecided;  /* powers of Eq. 1 whose correct rounding the
                               double-double evaluation could not decide (the
                               nearer double was used); expected 0          */
    int64_t templates;      /* templates in the last eval                    */
    int64_t evals;          /* template x segment evaluations in the last eval */
    int64_t in_band;        /* sum of N over the last eval                  */
    double eval_kernel_ms;  /* duration of the last eval's statistic kernel,
                               from HIP events on the context's stream       */
    double tables_ms;       /* duration of the last eval's track-table kernels
                               (Eq. 1 powers, Eq. 2 factors)                 */
} ltgw_diag;

/* ltgw_diagnostics: synchronous; reads the device counters of the last eval. */
int32_t ltgw_diagnostics(ltgw_ctx *ctx, ltgw_diag *out);

/* ltgw_inject_track: add amp * w_j to the FP32 spectrogram `power`
 * ([n_seg][n_bins] device buffer of detector det's shape) at the bin of
 * template (f0, tau, brake, sky) in every in-band segment, using the
 * detector's loaded segment times, weights and velocity table and the same
 * bin arithmetic as the evaluation.  Builds synthetic signal-plus-noise
 * data (Sec. 3 injections) on the device; the store itself is untouched.
 * Asynchronous.  Errors: STATE, INVALID_ARG, DEVICE. */
int32_t ltgw_inject_track(ltgw_ctx *ctx, int32_t det, float *power, double f0, double tau,
                          double brake, const double *sky3, double t0, float amp);

/* ltgw_read_store: copy detector det's device store to host for inspection.
 *   out_host: n_seg rows of n_bins elements (guards dropped), each element 4
 *             (F32), 2 (BF16) or 1 (FP8) bytes as stored, sign bit = count
 *             bit (rho > rho_th).
 *   scale_host: [n_seg] FP32 per-segment scales (1 except FP8), or NULL.
 * Synchronous.  Errors: STATE (not loaded), INVALID_ARG, DEVICE. */
int32_t ltgw_read_store(ltgw_ctx *ctx, int32_t det, void *out_host, float *scale_host);

#ifdef __cplusplus
}
#endif
#endif /* LTGW_H */
