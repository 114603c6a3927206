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
#define LTGW_E_NOMEM (-3)       /* device (or pinned host) allocation failed */
#define LTGW_E_DEVICE (-4)      /* HIP runtime error; text in ltgw_last_error */
#define LTGW_E_UNSUPPORTED (-5) /* valid request outside what the library supports */
#define LTGW_E_IO (-6)          /* a file could not be opened, read or written, or is
                                   not a valid file of the kind asked for        */

/* ---- storage of the spectrogram on the device -------------------------- */
#define LTGW_STORE_F32 0  /* IEEE binary32                                     */
#define LTGW_STORE_BF16 1 /* bfloat16, round to nearest even                   */
#define LTGW_STORE_FP8 2  /* OCP E4M3 (E4M3FN), per-segment FP32 scale =
                             rowmax/448 (1 for an all-zero row), value/scale
                             rounded to nearest even, saturating at 448        */

/* ---- statistics -------------------------------------------------------- */
#define LTGW_STAT_POWER 1u /* weighted normalised-power sum s (Sec. 2)          */
#define LTGW_STAT_COUNT 2u /* number count c of pixels above rho_th (Sec. 2)    */

#define LTGW_MAX_DET 256        /* detector slots per context                      */
#define LTGW_MAX_SEARCH_DET 4   /* detectors summed by one search                  */
#define LTGW_MAX_TOPK 256       /* largest k accepted by the top-k calls           */

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
 * Valid until the next call on ctx.  With ctx == NULL: the last failure on
 * this thread of a call made without a context (ltgw_create, and
 * ltgw_proposer_save / ltgw_proposer_load with ctx NULL). */
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

/* ltgw_set_antenna: antenna-pattern weights for detector slot det.  Sec. 2
 * weights the statistics by the antenna patterns as well as the noise floor;
 * after this call the weight of segment j for a template with sky direction n
 * is w_j * A_j(n) in place of w_j, where w_j is the loaded weight and
 * A_j(n) = F+^2 + Fx^2 is the summed response of the detector to the two
 * polarisations of a wave from n (independent of the polarisation angle).
 *   arms: host [2][3] unit vectors (|1 - |a|| <= 1e-12) of the two arms in the
 *         Earth-fixed frame (z on the rotation axis), or NULL to clear.
 *   era:  [n_seg] host or device, the Earth rotation angle (rad) at each
 *         segment: the rotation about z that carries the Earth-fixed frame
 *         into the frame of the velocities and sky directions.
 * The power sum and W1, W2 use the product rounded once to FP32 (the count
 * and N do not use weights).  Honoured by ltgw_eval_templates (one weight row
 * per sky point of the grid; W1, W2 are then summed by the statistic kernel)
 * and ltgw_eval_list; ltgw_eval_batch rejects such a detector (UNSUPPORTED).
 * A new ltgw_load_spectrogram on the slot clears it.  Synchronous.
 * Errors: STATE (nothing loaded), INVALID_ARG (values, n_seg not the
 * spectrogram's, arms in device memory), NOMEM, DEVICE. */
int32_t ltgw_set_antenna(ltgw_ctx *ctx, int32_t det, const double *arms, const double *era, int32_t n_seg);

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
    uint32_t det_mask;   /* bit d selects detector slot d (< 32); 0 = every
                            loaded slot below 32; at most LTGW_MAX_SEARCH_DET */
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

/* ---- evaluation without device allocation ----------------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.
 *
 * ltgw_eval_templates_noalloc: ltgw_eval_templates (same arguments, same
 * kernels, the same results bit for bit) with every table, window, moment
 * array and per-template sum placed in the library's static device scratch
 * array of LTGW_NOALLOC_SCRATCH_BYTES instead of buffers of the context.  It
 * calls no hipMalloc or hipFree and no allocating library routine; the
 * caller passes the outputs (device buffers, as for ltgw_eval_templates) and
 * must have loaded the detectors (ltgw_load_spectrogram and
 * ltgw_set_velocity_table allocate).
 *   - Each device holds one scratch array for the life of the process,
 *     shared by every context and call on it, and keeping the last call's
 *     contents (the call clears what it accumulates).  Calls that overlap
 *     on one device (contexts on different streams, threads) race.
 *   - The results are not kept in the context: ltgw_psi and
 *     ltgw_topk_candidates answer STATE after this call, and ltgw_read_tables
 *     holds no tables of it.
 *   - Limits: the search's buffers must fit the array (the realistic day of
 *     10800 segments x 8000 bins with 2,304,000 templates takes about 198 MB);
 *     at most LTGW_NOALLOC_MAX_AXIS tau, brake and sky values each.
 * Asynchronous.  Errors: as ltgw_eval_templates, and UNSUPPORTED when the
 * search exceeds a limit (the message gives the bytes it needs). */
#define LTGW_NOALLOC_SCRATCH_BYTES (256ull << 20) /* 256 MiB per device */
#define LTGW_NOALLOC_MAX_AXIS 4096
int32_t ltgw_eval_templates_noalloc(ltgw_ctx *ctx, const ltgw_grid *g, uint32_t stats, float *out_s,
                                    int32_t *out_c, int32_t *out_n);

/* ---- eval_list ---------------------------------------------------------------
 * Uniform random template bank (Sec. 2): templates with their own parameters,
 * e.g. drawn uniformly over the parameter space. */
typedef struct {
    double f0;     /* > 0, Hz                                            */
    double tau;    /* > 0, s                                             */
    double brake;  /* > 1, braking index n                               */
    double sky[3]; /* unit vector (|1 - |n|| <= 1e-12)                    */
} ltgw_template;

/* ltgw_eval_list: statistic of each template of tpl[0..n) (host array), summed
 * over the detectors det_mask selects (as in ltgw_grid; 0 = every loaded slot
 * below 32), with T0 = t0.  Every template is evaluated exactly as a lattice
 * template with those parameters: Eq. 1's power correctly rounded per segment,
 * Eq. 2, the bin rule and FP32 sums over chunks of 32 segments carried in FP64,
 * so s, c and N of a lattice template are the lattice's bit for bit (W1, W2
 * are summed in that order too; the lattice forms them exactly, so they agree
 * to FP32 rounding of 32-term sums).  Each segment's column is decided from
 * an FP64 enclosure of the correctly rounded power (the column is monotone in
 * it); the power itself is computed only where the enclosure straddles a
 * column boundary (counted in ltgw_diag.pow_exact), so the results are those
 * of the correctly rounded power.  The evaluation runs in f0 order (2^16
 * buckets over the list's range; results stay in list order); no table is
 * shared between templates.  Outputs as ltgw_eval_templates, in list order;
 * the results are kept for ltgw_psi and ltgw_topk_candidates (whose records
 * then carry the listed parameters, index = list position and sky = -1).
 * Asynchronous (the list is copied before the call returns).  Errors:
 * INVALID_ARG (values, a device pointer for tpl, f0 * t_sft too large),
 * STATE (no detector selected, or one without velocities), NOMEM, DEVICE. */
int32_t ltgw_eval_list(ltgw_ctx *ctx, const ltgw_template *tpl, int64_t n, double t0, uint32_t det_mask,
                       float *out_s, int32_t *out_c, int32_t *out_n);

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

/* ---- data preparation ------------------------------------------------------
 * ltgw_sft_normalise: the normalised power rho of Sec. 2 from a strain series:
 * Hann-windowed short Fourier transforms of consecutive segments, P = |X|^2,
 * and rho = P ln 2 / median, the median taken over the `window` bins centred
 * on each bin (under Gaussian noise P is exponential with mean S and median
 * S ln 2, so the median / ln 2 estimates the noise floor S).
 *   strain: device FP32 [n_seg * n_fft]; segment j is samples
 *           [j n_fft, (j + 1) n_fft) (no overlap); n_fft = T_sft * sample rate.
 *   Window w_n = 1/2 - 1/2 cos(2 pi n / n_fft) (periodic Hann), applied in
 *   frequency: with Y the FP32 transform of the raw segment (hipFFT, real to
 *   complex, on a copy of the segment in the context's buffer: the strain
 *   is only read, never written), X_k = Y_k/2 -
 *   (Y_{k-1} + Y_{k+1})/4, which equals sum_n x_n w_n e^{-2 pi i k n / n_fft}.
 *   out: device FP32 [n_seg][n_bins], column b = bin k_lo + b (frequency
 *        k / T_sft), ready for ltgw_load_spectrogram.  A window whose median
 *        is 0 (e.g. zero strain) gives rho = 0.
 *   n_fft even, 2 .. 2^24; n_seg 1 .. 65535; window odd, 1 .. 257; the bins
 *   k_lo - window/2 .. k_lo + n_bins - 1 + window/2 must lie in 0 .. n_fft/2.
 * Non-finite strain propagates to rho (ltgw_load_spectrogram rejects it).
 * Works in chunks of segments with about 512 MB of spectra; FFT plans are
 * kept per (n_fft, chunk).  Asynchronous.  Errors: INVALID_ARG (sizes,
 * host pointers), NOMEM, DEVICE. */
int32_t ltgw_sft_normalise(ltgw_ctx *ctx, const float *strain, int32_t n_seg, int32_t n_fft, int64_t k_lo,
                           int32_t n_bins, int32_t window, float *out);

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
                               (Eq. 1 powers, Eq. 2 factors, in-band windows);
                               the in-band moments run beside the statistic
                               kernel on a second stream of the context    */
    int32_t tile_shape;     /* tile shape of the last eval's statistic kernel */
    int32_t eval_launches;  /* dispatches of the statistic kernel in the last
                               eval (segment slabs, generations of workgroups) */
    double ingest_ms;       /* duration of the store kernels of the last
                               ltgw_load_spectrogram or ltgw_load_stack (HIP
                               events on the context's stream; a stack's
                               coarse store is written in the same pass)     */
    int64_t pow_slow;       /* powers of Eq. 1 (since the context was created)
                               that the fast evaluation could not round with
                               certainty and the double-double one took     */
    int64_t pow_exact;      /* evaluations of explicit template lists (since
                               the context was created) whose column an
                               enclosure of the Eq. 1 power could not decide,
                               so the correctly rounded power was taken     */
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

/* ---- many searches in one launch --------------------------------------------
 * A batch of independent searches (own detectors, T_obs, band, sky patch and
 * lattice; Sec. 2 bank, wide sky coverage of the abstract, batched templates
 * of Sec. 3).  The work is split into tiles (search, (sky, n, tau) group,
 * run of 64 x templates-per-lane f0) processed by one persistent launch:
 * every resident wavefront takes the next tile from an atomic counter,
 * largest search first, until the list is exhausted.  The whole sequence of a batch (Eq. 1 and Eq. 2
 * tables, in-band moments, the statistic, critical ratios and per-search
 * top-k) is captured into a HIP graph on first use and replayed by later
 * calls with an identical batch.  The tile shape is chosen by the context's
 * autotuner (timed on the batch itself on first use, or taken from the
 * tuning cache). */
typedef struct {
    ltgw_grid grid;                     /* lattice; grid.det_mask is ignored */
    int32_t dets[LTGW_MAX_SEARCH_DET];  /* detector slots this search sums   */
    int32_t n_dets;                     /* 1 .. LTGW_MAX_SEARCH_DET          */
} ltgw_search;

typedef struct {
    int32_t graph_replayed;  /* 1 when this call replayed a captured graph       */
    int32_t variant;         /* tile shape used (index into the shapes below)    */
    int32_t templates_per_lane;
    int32_t segments_per_batch;
    int32_t workgroups;      /* persistent grid size (4 wavefronts each)        */
    int32_t tiles;           /* wavefront tiles                                 */
    int64_t templates;
    int64_t evals;           /* template x segment evaluations of the batch     */
    int64_t in_band;
    double kernel_ms;        /* persistent statistic launch, start to last tile */
    double total_ms;         /* whole batch sequence, HIP events                 */
} ltgw_batch_stats;

/* ltgw_eval_batch: evaluate n_searches searches and rank each.
 *   searches: host array; every referenced slot must hold a spectrogram and
 *             velocity table; all searches use the same store format.
 *   k: 1 .. LTGW_MAX_TOPK candidates per search and statistic.
 *   top_power, top_count: host arrays [n_searches][k] (caller-owned).
 *   n_power, n_count: host arrays [n_searches], records written per search.
 *   stats: optional host struct.
 * Per-search results stay in the context until the next batch
 * (ltgw_batch_results).  Synchronous.
 * Errors: INVALID_ARG, STATE (slot not loaded), UNSUPPORTED (mixed stores),
 * NOMEM, DEVICE. */
int32_t ltgw_eval_batch(ltgw_ctx *ctx, const ltgw_search *searches, int32_t n_searches, int32_t k,
                        ltgw_candidate *top_power, ltgw_candidate *top_count, int32_t *n_power,
                        int32_t *n_count, ltgw_batch_stats *stats);

/* ltgw_batch_results: copy search i's per-template results of the last batch
 * into device buffers (each optional): FP32 s, int32 c, int32 N, FP64
 * critical ratios of the power (psi_power) and of the count (psi_count).
 * Asynchronous.  Errors: STATE (no batch), INVALID_ARG. */
int32_t ltgw_batch_results(ltgw_ctx *ctx, int32_t search, float *out_s, int32_t *out_c,
                           int32_t *out_n, double *psi_power, double *psi_count);

/* ltgw_batch_latency: per-search completion time of the last batch launch,
 * milliseconds from the start of its persistent statistic launch to the end
 * of the search's last tile (device wall clock), into out_ms[n_searches]
 * (host).  Errors: STATE (no batch), INVALID_ARG. */
int32_t ltgw_batch_latency(ltgw_ctx *ctx, double *out_ms);

/* ---- autotuner -----------------------------------------------------------
 * Tile shapes (templates per lane, segments per gather batch):
 *   0 = (1, 8)   1 = (1, 16)   2 = (2, 8)   3 = (2, 16)
 and, for the single-search statistic kernel, bit 4 = the same shape
 * launched in generations of as many workgroups as the device holds at once
 * (the workgroups of a generation walk the segments together and share the
 * spectrogram rows in L2) and bit 8 = one search detector's segments walked
 * in slabs of 1024, one launch per slab (results bit-identical to one pass).
 * Variants 0..15.  A batch uses shape (value & 3): its persistent launch is
 * one generation already.
 * Keys describe the work (single search or batch, store, moment mode and
 * size classes); values are the fastest variant measured on this device.
 * ltgw_autotune times every variant on the given grid (single search) and
 * records the winner; ltgw_eval_batch tunes a new batch key by itself.
 * ltgw_tune_save / ltgw_tune_load write and read the cache as JSON text
 * ({"ltgw_tune": {"<key>": <variant>, ...}}). */
int32_t ltgw_autotune(ltgw_ctx *ctx, const ltgw_grid *g, int32_t *best_variant);
/* ltgw_set_tile_shape: use variant `variant` (0..15) for every later
 * evaluation, or -1 to return to the autotuner.  Drops a captured batch. */
int32_t ltgw_set_tile_shape(ltgw_ctx *ctx, int32_t variant);
int32_t ltgw_tune_save(ltgw_ctx *ctx, const char *path);
int32_t ltgw_tune_load(ltgw_ctx *ctx, const char *path);

/* ---- learned proposer -------------------------------------------------------
 * A system pattern on top of the method (not part of the paper): a small
 * network reads a coarse statistic map and picks the fine-grid cells that
 * are then evaluated exactly; the exhaustive grid stays the fallback and the
 * reference its recall is measured against (detection as in Sec. 3: Psi above
 * the largest noise-only value).  Training data are realisations generated on
 * the device. */

/* ltgw_generate_noise: Exp(1) noise for realisations r0 .. r0+R-1, n values
 * each, into the device array out[R][n].  Element e of realisation r is word
 * e % 4 of Philox4x32-10 (Salmon et al., SC11) with counter (e/4 low, e/4
 * high, r, stream) and key (seed low, seed high); u = (word + 1/2) 2^-32 and
 * the value is -log(u) in FP64 rounded to FP32.  Asynchronous. */
int32_t ltgw_generate_noise(ltgw_ctx *ctx, uint64_t seed, uint32_t stream, int32_t r0, int32_t R,
                            int64_t n, float *out);

/* ltgw_inject_stack: add injected tracks to a device stack of R spectrograms
 * ([R][n_seg][n_bins] FP32, the shape of detector slot det) using det's
 * segment times, weights and velocity table: realisation r gets amp * w_j at
 * the bin of template params[r] = (f0, tau, brake, amp) (FP64, host or
 * device; amp 0 = none) in every in-band segment. */
int32_t ltgw_inject_stack(ltgw_ctx *ctx, int32_t det, float *stack, int32_t R, const double *params,
                          const double *sky3, double t0);  /* synchronous */

/* ltgw_load_stack: R realisations of detector slot det's geometry (its
 * segment times, weights and velocity table are used for all): a fine store
 * of format `store` from the device FP32 stack [R][n_seg][n_bins], and with
 * coarse = S (2, 4 or 8; 1 means 2) a coarsened BF16 store: sums over groups of
 * S consecutive segments and pairs of bins (n_seg a multiple of S, n_bins
 * even); a group's weight is the mean of its S weights.  coarse = 0: none.
 * The stack data must be finite and >= 0.  Synchronous.  Errors: STATE (slot
 * not loaded), INVALID_ARG, NOMEM. */
int32_t ltgw_load_stack(ltgw_ctx *ctx, int32_t det, int32_t R, const float *stack, int32_t store,
                        int32_t coarse);

/* ltgw_stack_psi: power critical ratio of every template of grid g on every
 * realisation of the loaded stack into the device array out_psi[R][n_templates].
 * level 0: fine store (Exp(1) pixels: mean 1, variance 1); level 1: coarse
 * store, the track's column halved at the first segment of each group
 * (pixels are sums of 2 S Exp(1): mean 2 S, variance 2 S).  N = 0 gives NaN, or 0 with
 * nan_to_zero.  Asynchronous.  Errors: STATE (no stack / no coarse store). */
int32_t ltgw_stack_psi(ltgw_ctx *ctx, const ltgw_grid *g, int32_t level, int32_t nan_to_zero,
                       double *out_psi);

/* ltgw_stack_psi_list: critical ratios on the fine store for listed
 * templates: idx[R][m] (device int32 template indices of g; an index outside
 * the grid gives NaN) -> out_psi[R][m] (device), for stat LTGW_STAT_POWER or
 * LTGW_STAT_COUNT (Eq. 4 for the number count: (c - N q) / sqrt(N q (1 - q)),
 * q = exp(-rho_th), the value ltgw_psi gives the same template bit for bit).
 * Asynchronous. */
int32_t ltgw_stack_psi_list(ltgw_ctx *ctx, const ltgw_grid *g, uint32_t stat, const int32_t *idx, int32_t m,
                            double *out_psi);

/* ltgw_stack_features: the network's input from the coarse store, FP32
 * x[R][channels][n_f0] (device), 0 where a template has no in-band segment:
 * channel gr < G (G the groups of grid g) the coarse power critical ratio of
 * group gr, and with counts = 1 channel G + gr its coarse number-count
 * critical ratio (c - N m q) / sqrt(N m q (1 - q)): c the count of pixels
 * above rho_th in the track's coarse blocks, N the in-band coarse segments,
 * m = 2 S pixels per block, q = exp(-rho_th) (Eq. 4 for the count of Sec. 2
 * on the coarse blocks).  Asynchronous.  Errors: STATE (no coarse store). */
int32_t ltgw_stack_features(ltgw_ctx *ctx, const ltgw_grid *g, int32_t counts, float *x);

/* ltgw_stack_best: exhaustive search of grid g on every realisation of the
 * fine store for statistic stat (LTGW_STAT_POWER or LTGW_STAT_COUNT): best
 * template (largest Psi, ties to the lowest index; -1 and -inf when no
 * template has N > 0) into device best_index[R], best_psi[R].
 * Asynchronous. */
int32_t ltgw_stack_best(ltgw_ctx *ctx, const ltgw_grid *g, uint32_t stat, int32_t *best_index, double *best_psi);

/* ltgw_cells_from_templates: fine template t (group g, f0 index i, with fine
 * n_f0 = 2 L) -> network cell (2 g + i % 2) L + i / 2; -1 where t < 0,
 * mask[k] == 0 (mask may be NULL) or psi[k] is not above min_psi (psi may be
 * NULL).  Device arrays of n; asynchronous. */
int32_t ltgw_cells_from_templates(ltgw_ctx *ctx, const int32_t *tpl, int32_t n, int32_t L, const int32_t *mask,
                                  const double *psi, double min_psi, int32_t *cells);

/* The ranking network: x[B][c_in][L] -> logits[B][c_out][L] through three
 * width-32, kernel-5 convolutions with ReLU and a kernel-1 output
 * convolution; parameters are one FP32 vector W1 b1 W2 b2 W3 b3 W4 b4
 * (W[o][c][t] row-major, ltgw_cnn_param_count values).  Products on BF16
 * matrix cores with FP32 accumulation.  act: device [3][B][32][L] (the three
 * hidden activations, kept for the backward pass), or NULL for inference
 * only (one fused pass with the activations in on-chip memory, the same
 * logits bit for bit; c_in, c_out <= 32 and L <= 256).  All pointers device;
 * asynchronous. */
int64_t ltgw_cnn_param_count(int32_t c_in, int32_t c_out);
int64_t ltgw_cnn_work_floats(int32_t B, int32_t c_in, int32_t c_out, int32_t L);
int32_t ltgw_cnn_forward(ltgw_ctx *ctx, const float *params, const float *x, int32_t B, int32_t c_in,
                         int32_t c_out, int32_t L, float *act, float *logits);
/* grads[ltgw_cnn_param_count]: gradient of the loss whose logit gradient is
 * dlogits; work: ltgw_cnn_work_floats floats.  Deterministic. */
int32_t ltgw_cnn_backward(ltgw_ctx *ctx, const float *params, const float *x, int32_t B, int32_t c_in,
                          int32_t c_out, int32_t L, const float *act, const float *dlogits, float *work,
                          int64_t work_floats, float *grads);
/* Softmax cross-entropy of each sample's n_cells logits against target[b]
 * (-1: no target); loss[B] per sample, dlogits already divided by n_valid. */
int32_t ltgw_softmax_xent(ltgw_ctx *ctx, const float *logits, int32_t B, int32_t n_cells,
                          const int32_t *target, int32_t n_valid, float *loss, float *dlogits);
/* One Adam step (Kingma and Ba) on FP32 master weights; step counts from 1. */
int32_t ltgw_adam_step(ltgw_ctx *ctx, float *params, const float *grads, float *m, float *v, int64_t n,
                       float lr, float beta1, float beta2, float eps, int32_t step);
/* Per row of n scores (n <= 8192): the indices of the M best scores (ties go
 * to the lower index, NaN ranks last), written in ascending index order. */
int32_t ltgw_select_top(ltgw_ctx *ctx, const float *score, int32_t R, int32_t n, int32_t M,
                        int32_t *out_idx);

typedef struct {
    const float *params;      /* network parameters (device), or NULL: rank by the
                                 coarse power ratios alone (coarse_map)          */
    int32_t c_in, c_out, L;   /* network shape: c_in = G (the coarse power ratios
                                 of the G coarse groups) or 2 G (then the count
                                 ratios), c_out = 2 x fine groups               */
    int32_t n_select;         /* fine cells evaluated exactly per realisation     */
    int32_t block;            /* cells are taken in blocks of this many
                                 consecutive f0 of one fine group (1 .. 64)       */
    int32_t n_select2;        /* second tier: further cells for the realisations
                                 with no cell above psi_threshold (0: none)       */
    double psi_threshold;     /* detection threshold on Psi (largest noise value)  */
    double coarse_threshold;  /* fallback when the coarse map exceeds this but no
                                 selected cell passes psi_threshold               */
    double tier2_threshold;   /* the second tier is taken only where the largest
                                 coarse ratio exceeds this (finite; a very
                                 negative value: wherever no cell passes)    */
    int32_t *blocks;          /* optional host output (NULL: none), [R][K1 + K2]
                                 with K1 = ceil(n_select / block), K2 =
                                 ceil(n_select2 / block): the blocks evaluated
                                 exactly, tier 1 in ascending order, then tier 2
                                 (-1 where the realisation did not take it).
                                 Block b covers fine group b / nbg, f0 indices
                                 (b % nbg) block .. + block - 1 (below 2 L),
                                 nbg = ceil(2 L / block).  A fallback
                                 realisation evaluated every template.        */
    const int32_t *coarse_map; /* with params NULL: host [fine groups][2], the
                                 coarse groups (-1: none) whose power ratios
                                 score fine group g's cells, e.g. the nearest
                                 in tau and n; ignored with a network          */
} ltgw_proposer;

/* ltgw_propose: on the loaded stack, for every realisation: coarse critical
 * ratios on the coarse grid (channels = its (tau, n) groups, positions = its
 * f0) -> network logits over the fine cells -> blocks of `block` consecutive
 * fine f0 of one group, scored by their largest logit -> the
 * ceil(n_select / block) best blocks -> exact fine critical ratios of their
 * templates -> the best.  Realisations with no template above psi_threshold
 * whose largest coarse ratio exceeds tier2_threshold then get the next
 * ceil(n_select2 / block) blocks; those still below psi_threshold whose
 * largest coarse ratio exceeds coarse_threshold are evaluated
 * exhaustively on the fine grid (the fallback).  Cell (channel ch, position
 * l) is fine template ((ch / 2) group, f0 index 2 l + ch % 2): the fine grid
 * has twice the coarse positions in f0 and c_out / 2 (tau, n) groups.
 * Outputs (host, [R]): best template index and Psi (ties to the lower index),
 * fallback flag.  Synchronous. */
int32_t ltgw_propose(ltgw_ctx *ctx, const ltgw_grid *fine, const ltgw_grid *coarse,
                     const ltgw_proposer *p, int32_t *best_index, double *best_psi, int32_t *fallback);

/* ltgw_proposer_save: write a ranking network to the file `path` (replaced
 * whole: written beside it, then renamed over it).  params: the
 * ltgw_cnn_param_count(c_in, c_out) FP32 parameters, device or host memory;
 * with ctx NULL they must be host memory and no device call is made.  The
 * file is a 64-byte header (magic "LTGWCNN", format version 1, c_in, c_out,
 * width 32, taps 5, parameter count, FNV-1a 64-bit hash of the parameter
 * bytes) and the parameters, little-endian.  Synchronous.  Errors:
 * INVALID_ARG (NULL path or params, shape out of range), IO, DEVICE. */
int32_t ltgw_proposer_save(ltgw_ctx *ctx, const char *path, const float *params, int32_t c_in, int32_t c_out);

/* ltgw_proposer_load: read a network written by ltgw_proposer_save.
 *   c_in, c_out: receive the network's shape (each may be NULL);
 *   params: NULL to read the shape only, else n_params floats (device or
 *           host memory; host only when ctx is NULL), n_params equal to the
 *           file's parameter count, receiving the parameters bit for bit.
 * The header, the shape, the length and the hash are checked before params
 * is written.  Synchronous.  Errors: INVALID_ARG (NULL path, n_params
 * mismatch), IO (missing, short, corrupt or foreign file), UNSUPPORTED (other
 * format version), DEVICE. */
int32_t ltgw_proposer_load(ltgw_ctx *ctx, const char *path, int32_t *c_in, int32_t *c_out, float *params,
                           int64_t n_params);

/* ltgw_read_store: copy detector det's device store to host for inspection.
 *   out_host: n_seg rows of n_bins elements (guards dropped), each element 4
 *             (F32), 2 (BF16) or 1 (FP8) bytes as stored, sign bit = count
 *             bit (rho > rho_th).
 *   scale_host: [n_seg] FP32 per-segment scales (1 except FP8), or NULL.
 * Synchronous.  Errors: STATE (not loaded), INVALID_ARG, DEVICE. */
int32_t ltgw_read_store(ltgw_ctx *ctx, int32_t det, void *out_host, float *scale_host);

/* ltgw_read_tables: copy the per-segment track tables that the last
 * ltgw_eval_templates built for detector det to host memory, for inspection:
 *   g_host: FP64 [n_brake * n_tau][n_seg], row i_n * n_tau + i_tau, the spin-down
 *           factor g = RN(u^e) of Eq. 1 (u = 1 + (t_j - T0)/tau, e = 1/(1 - n);
 *           0 where t_j < T0), or NULL;
 *   h_host: FP64 [n_sky * n_brake * n_tau][n_seg], row (sky * n_brake + i_n) *
 *           n_tau + i_tau, the bin-scaled track factor RN(RN(g D) t_sft) with
 *           D = 1 + v.n/c of Eq. 2, or NULL;
 *   n_rows: host int32[2] receiving the two row counts, or NULL.
 * Buffers are caller-owned and must hold the row counts of the last eval's
 * grid.  Synchronous.  Errors: STATE (no eval used det since it was loaded),
 * INVALID_ARG, DEVICE. */
int32_t ltgw_read_tables(ltgw_ctx *ctx, int32_t det, double *g_host, double *h_host, int32_t *n_rows);

#ifdef __cplusplus
}
#endif
#endif /* LTGW_H */
