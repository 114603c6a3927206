/*
 * Plain FP64 CPU oracle for the template-bank detection statistic.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may call, link or
 * load this file: only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no code, header, table or constant with
 * the HIP library; the two are compared, never combined.
 *
 * Every floating-point operation below is a single correctly rounded FP64
 * operation (round to nearest, ties to even) in the order written.  The file
 * must be compiled with -ffp-contract=off so that no multiply-add is fused.
 *
 * Method (Merou, Tenorio, Sintes, "GPU-Accelerated Searches for Long-Transient
 * Gravitational Waves from Newborn Neutron Stars"):
 *   - frequency track f_gw(t) = f0 ((t - T0)/tau + 1)^(1/(1-n))   (Sec. 1, Eq. 1)
 *   - Doppler factor f^ = f_gw (1 + v.n/c)                          (Sec. 1, Eq. 2)
 *   - statistic: weighted power (or number count) summed over the data
 *     bins that the track selects                                   (Sec. 2)
 *   - critical ratio Psi = (s - <s>)/sigma_s                        (Sec. 2, Eq. 4)
 *
 * Readings where the paper is silent: one bin per segment at the segment
 * reference time; the nearest bin, ties up; out-of-band and t < T0 segments
 * contribute nothing; per-segment weights on the power; an unweighted
 * integer count.
 */
#include <math.h>
#include <quadmath.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_C_LIGHT 299792458.0 /* m/s, exact by SI definition */

/* ------------------------------------------------------------------------ */
/* Eq. 1 (Sec. 1): spin-down factor g = (1 + (t - T0)/tau)^(1/(1-n)).
 * Returned correctly rounded: u and e are formed in FP64, the power is taken
 * in binary128 (libquadmath powq, ~1 ulp of a 113-bit significand) and
 * rounded once to FP64.  Returns 0.0 for t < T0: Eq. 1 is not defined
 * before the remnant forms, so such segments are masked. */
double oracle_spin_factor(double t, double t0, double tau, double brake)
{
    if (t < t0) return 0.0;
    double d = t - t0;
    double q = d / tau;
    double u = 1.0 + q;
    double e = 1.0 / (1.0 - brake);
    return (double)powq((__float128)u, (__float128)e);
}

/* Eq. 2 (Sec. 1): Doppler factor D = 1 + (v . n)/c, first order, with the
 * dot product summed as (vx nx + vy ny) + vz nz. */
double oracle_doppler(const double *v, const double *n)
{
    double a = v[0] * n[0];
    double b = v[1] * n[1];
    double z = v[2] * n[2];
    double vn = (a + b) + z;
    double r = vn / ORACLE_C_LIGHT;
    return 1.0 + r;
}

/* Frequency-bin index of the Doppler-shifted track at one segment.
 * The detector-frame frequency is f0 * g * D (Eqs. 1-2); the bin of width
 * 1/T_sft nearest to it is floor(x + 1/2) with x = f * T_sft.  The factor
 * ratio f^/f0 = g*D is formed first, scaled to bins, then multiplied by f0:
 *     h = g*D ; H = h*T_sft ; x = f0*H ; k = floor(x + 0.5) ; b = k - k_lo.
 * Returns b, the column in a spectrogram whose column 0 is absolute bin k_lo. */
int64_t oracle_bin(double f0, double g, double D, double t_sft, int64_t k_lo)
{
    double h = g * D;
    double H = h * t_sft;
    double x = f0 * H;
    double y = x + 0.5;
    double k = floor(y);
    return (int64_t)k - k_lo;
}

/* f0 of lattice point i (Sec. 2, cubic lattice): f0_min + i*step. */
double oracle_lattice_f0(double f0_min, double f0_step, int64_t i)
{
    double a = (double)i * f0_step;
    return f0_min + a;
}

/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t n_seg;       /* segments (SFTs) of this detector                    */
    int32_t n_bins;      /* spectrogram columns                                 */
    int64_t k_lo;        /* absolute bin index of column 0                      */
    double t_sft;        /* SFT length in seconds (bin width 1/t_sft)           */
    const double *t_seg; /* [n_seg] segment reference times, same epoch as T0   */
    const float *w;      /* [n_seg] per-segment weights, NULL means all 1       */
    const double *v;     /* [n_seg][3] detector velocity in m/s                  */
    const double *P;     /* [n_seg][n_bins] power values that are summed         */
    const float *rho;    /* [n_seg][n_bins] FP32 normalised power (count source) */
    float rho_th;        /* number-count threshold, compared in FP32             */
    const double *arms;  /* [2][3] unit arm vectors in the Earth-fixed frame, or
                            NULL: no antenna factor on the weights             */
    const double *era;   /* [n_seg] Earth rotation angle (rad) at each segment  */
} oracle_det;

/* ------------------------------------------------------------------------ */
/* Antenna response of an interferometer (the weighting of Sec. 2): the sum
 * F+^2 + Fx^2 of the two polarisation responses to a wave from direction n.
 * The arms a, b (unit vectors, Earth-fixed frame, z on the rotation axis) are
 * carried into the equatorial frame of n by a rotation of era about z.  With
 * the detector tensor Dt = (a a^T - b b^T)/2 and a polarisation basis (p, q)
 * orthogonal to n, F+ = p^T Dt p - q^T Dt q and Fx = p^T Dt q + q^T Dt p;
 * their squares summed do not depend on the polarisation angle, so any such
 * basis serves: p along z x n (x when n is on the z axis), q = n x p. */
static void cross3(const double *u, const double *v, double *o)
{
    o[0] = u[1] * v[2] - u[2] * v[1];
    o[1] = u[2] * v[0] - u[0] * v[2];
    o[2] = u[0] * v[1] - u[1] * v[0];
}

static double quad_form(const double Dt[3][3], const double *u, const double *v)
{
    double acc = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int k = 0; k < 3; ++k) acc = acc + u[i] * Dt[i][k] * v[k];
    return acc;
}

double oracle_antenna(const double *arms, double era, const double *n)
{
    double c = cos(era), sn = sin(era);
    double a[3], b[3];
    a[0] = c * arms[0] - sn * arms[1];
    a[1] = sn * arms[0] + c * arms[1];
    a[2] = arms[2];
    b[0] = c * arms[3] - sn * arms[4];
    b[1] = sn * arms[3] + c * arms[4];
    b[2] = arms[5];
    double Dt[3][3];
    for (int i = 0; i < 3; ++i)
        for (int k = 0; k < 3; ++k) Dt[i][k] = 0.5 * (a[i] * a[k] - b[i] * b[k]);
    const double zax[3] = {0.0, 0.0, 1.0};
    double p[3], q[3];
    cross3(zax, n, p);
    double pn = sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
    if (pn < 1e-12) {
        p[0] = 1.0; p[1] = 0.0; p[2] = 0.0;
    } else {
        p[0] = p[0] / pn; p[1] = p[1] / pn; p[2] = p[2] / pn;
    }
    cross3(n, p, q);
    double fp = quad_form(Dt, p, p) - quad_form(Dt, q, q);
    double fx = quad_form(Dt, p, q) + quad_form(Dt, q, p);
    return fp * fp + fx * fx;
}

typedef struct {
    double f0_min, f0_step;
    int32_t n_f0;
    const double *tau;
    int32_t n_tau;
    const double *brake;
    int32_t n_brake;
    const double *sky; /* [n_sky][3] unit vectors */
    int32_t n_sky;
    double t0;
} oracle_grid;

/* Template index order: ((sky*n_brake + i_n)*n_tau + i_tau)*n_f0 + i_f0. */
static void decode_index(const oracle_grid *g, int64_t t, int64_t *i_f0,
                         int64_t *i_tau, int64_t *i_n, int64_t *i_sky)
{
    *i_f0 = t % g->n_f0;
    int64_t grp = t / g->n_f0;
    *i_tau = grp % g->n_tau;
    int64_t r = grp / g->n_tau;
    *i_n = r % g->n_brake;
    *i_sky = r / g->n_brake;
}

/* Per-segment tables that do not depend on f0: g[d][n][tau][j] and
 * D[d][sky][j].  Hoisting them changes no result (both are pure functions
 * of their arguments). */
static double **build_g(const oracle_det *dets, int32_t n_det, const oracle_grid *g,
                        const unsigned char *need /* [n_brake*n_tau] or NULL = all */)
{
    double **tab = (double **)calloc((size_t)n_det, sizeof(double *));
    for (int32_t d = 0; d < n_det; ++d) {
        int64_t ns = dets[d].n_seg;
        int64_t ng = (int64_t)g->n_brake * g->n_tau;
        tab[d] = (double *)malloc((size_t)(ng * ns) * sizeof(double));
        double *T = tab[d];
#pragma omp parallel for schedule(dynamic, 256)
        for (int64_t q = 0; q < ng * ns; ++q) {
            int64_t j = q % ns, grp = q / ns;
            if (need && !need[grp]) { T[q] = 0.0; continue; }
            int64_t it = grp % g->n_tau, in = grp / g->n_tau;
            T[q] = oracle_spin_factor(dets[d].t_seg[j], g->t0, g->tau[it], g->brake[in]);
        }
    }
    return tab;
}

static double **build_D(const oracle_det *dets, int32_t n_det, const oracle_grid *g)
{
    double **tab = (double **)calloc((size_t)n_det, sizeof(double *));
    for (int32_t d = 0; d < n_det; ++d) {
        int64_t ns = dets[d].n_seg;
        tab[d] = (double *)malloc((size_t)(g->n_sky * ns) * sizeof(double));
        for (int64_t s = 0; s < g->n_sky; ++s)
            for (int64_t j = 0; j < ns; ++j)
                tab[d][s * ns + j] = oracle_doppler(dets[d].v + 3 * j, g->sky + 3 * s);
    }
    return tab;
}

/* A[d][sky][j]: antenna response of detector d at segment j to sky point
 * sky, or NULL for a detector without one. */
static double **build_A(const oracle_det *dets, int32_t n_det, const oracle_grid *g)
{
    double **tab = (double **)calloc((size_t)n_det, sizeof(double *));
    for (int32_t d = 0; d < n_det; ++d) {
        if (!dets[d].arms) continue;
        int64_t ns = dets[d].n_seg;
        tab[d] = (double *)malloc((size_t)(g->n_sky * ns) * sizeof(double));
        for (int64_t s = 0; s < g->n_sky; ++s)
            for (int64_t j = 0; j < ns; ++j)
                tab[d][s * ns + j] = oracle_antenna(dets[d].arms, dets[d].era[j], g->sky + 3 * s);
    }
    return tab;
}

static void free_tabs(double **t, int32_t n)
{
    for (int32_t i = 0; i < n; ++i) free(t[i]);
    free(t);
}

/* Statistic over templates [t_begin, t_end) (Sec. 2):
 *   s  = sum over in-band (d, j) of w_j * P_d[j][b]        (FP64, segment order)
 *   with w_j the segment weight, times the antenna response A_d(sky, j) for a
 *   detector that has one (the product formed in FP64)
 *   c  = number of in-band (d, j) with rho_d[j][b] > rho_th (FP32 compare)
 *   N  = number of in-band (d, j); W1 = sum w_j ; W2 = sum w_j^2
 * Outputs are indexed by t - t_begin.  Masked (t_j < T0) and out-of-band
 * segments contribute nothing. */
static void eval_templates(const oracle_det *dets, int32_t n_det, const oracle_grid *g,
                           const int64_t *list, int64_t t_begin, int64_t n, double *s,
                           int32_t *c, int32_t *N, double *W1, double *W2)
{
    unsigned char *need = NULL;
    if (list) {
        need = (unsigned char *)calloc((size_t)g->n_brake * g->n_tau, 1);
        for (int64_t q = 0; q < n; ++q) need[(list[q] / g->n_f0) % ((int64_t)g->n_brake * g->n_tau)] = 1;
    }
    double **gt = build_g(dets, n_det, g, need);
    double **Dt = build_D(dets, n_det, g);
    double **At = build_A(dets, n_det, g);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t o = 0; o < n; ++o) {
        int64_t t = list ? list[o] : t_begin + o;
        int64_t i_f0, i_tau, i_n, i_sky;
        decode_index(g, t, &i_f0, &i_tau, &i_n, &i_sky);
        double f0 = oracle_lattice_f0(g->f0_min, g->f0_step, i_f0);
        double acc = 0.0, w1 = 0.0, w2 = 0.0;
        int32_t cnt = 0, nin = 0;
        for (int32_t d = 0; d < n_det; ++d) {
            const oracle_det *D = dets + d;
            const double *grow = gt[d] + (i_n * g->n_tau + i_tau) * (int64_t)D->n_seg;
            const double *drow = Dt[d] + i_sky * (int64_t)D->n_seg;
            const double *arow = At[d] ? At[d] + i_sky * (int64_t)D->n_seg : NULL;
            for (int32_t j = 0; j < D->n_seg; ++j) {
                if (D->t_seg[j] < g->t0) continue;
                int64_t b = oracle_bin(f0, grow[j], drow[j], D->t_sft, D->k_lo);
                if (b < 0 || b >= D->n_bins) continue;
                double wj = D->w ? (double)D->w[j] : 1.0;
                if (arow) wj = wj * arow[j];
                int64_t off = (int64_t)j * D->n_bins + b;
                acc = acc + wj * D->P[off];
                if (D->rho[off] > D->rho_th) cnt += 1;
                nin += 1;
                w1 = w1 + wj;
                w2 = w2 + wj * wj;
            }
        }
        if (s) s[o] = acc;
        if (c) c[o] = cnt;
        if (N) N[o] = nin;
        if (W1) W1[o] = w1;
        if (W2) W2[o] = w2;
    }
    free_tabs(gt, n_det);
    free_tabs(Dt, n_det);
    free_tabs(At, n_det);
    free(need);
}

void oracle_eval(const oracle_det *dets, int32_t n_det, const oracle_grid *g,
                 int64_t t_begin, int64_t t_end, double *s, int32_t *c,
                 int32_t *N, double *W1, double *W2)
{
    eval_templates(dets, n_det, g, NULL, t_begin, t_end - t_begin, s, c, N, W1, W2);
}

/* The same statistic for an explicit list of template indices. */
void oracle_eval_list(const oracle_det *dets, int32_t n_det, const oracle_grid *g,
                      const int64_t *list, int64_t n, double *s, int32_t *c, int32_t *N,
                      double *W1, double *W2)
{
    eval_templates(dets, n_det, g, list, 0, n, s, c, N, W1, W2);
}

/* The statistic of explicit templates (the uniform random template bank of
 * Sec. 2): params[q] = (f0, tau, n, sky x, y, z).  Each template is evaluated
 * exactly as a lattice template with those parameters would be. */
void oracle_eval_params(const oracle_det *dets, int32_t n_det, const double *params, int64_t n, double t0,
                        double *s, int32_t *c, int32_t *N, double *W1, double *W2)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t o = 0; o < n; ++o) {
        const double *p = params + 6 * o;
        double acc = 0.0, w1 = 0.0, w2 = 0.0;
        int32_t cnt = 0, nin = 0;
        for (int32_t d = 0; d < n_det; ++d) {
            const oracle_det *D = dets + d;
            for (int32_t j = 0; j < D->n_seg; ++j) {
                if (D->t_seg[j] < t0) continue;
                double gj = oracle_spin_factor(D->t_seg[j], t0, p[1], p[2]);
                double Dj = oracle_doppler(D->v + 3 * j, p + 3);
                int64_t b = oracle_bin(p[0], gj, Dj, D->t_sft, D->k_lo);
                if (b < 0 || b >= D->n_bins) continue;
                double wj = D->w ? (double)D->w[j] : 1.0;
                if (D->arms) wj = wj * oracle_antenna(D->arms, D->era[j], p + 3);
                int64_t off = (int64_t)j * D->n_bins + b;
                acc = acc + wj * D->P[off];
                if (D->rho[off] > D->rho_th) cnt += 1;
                nin += 1;
                w1 = w1 + wj;
                w2 = w2 + wj * wj;
            }
        }
        s[o] = acc;
        c[o] = cnt;
        N[o] = nin;
        W1[o] = w1;
        W2[o] = w2;
    }
}

/* Bins of one template on one detector: b_out[j] = column, or INT64_MIN for a
 * masked segment (t_j < T0).  Out-of-band columns are returned as computed. */
void oracle_track_bins(const oracle_det *D, double f0, double tau, double brake,
                       const double *sky, double t0, int64_t *b_out)
{
    for (int32_t j = 0; j < D->n_seg; ++j) {
        if (D->t_seg[j] < t0) { b_out[j] = INT64_MIN; continue; }
        double gj = oracle_spin_factor(D->t_seg[j], t0, tau, brake);
        double Dj = oracle_doppler(D->v + 3 * j, sky);
        b_out[j] = oracle_bin(f0, gj, Dj, D->t_sft, D->k_lo);
    }
}

/* Eq. 4 (Sec. 2): critical ratio.  Under the noise-only hypothesis each
 * normalised-power pixel is Exp(1) (mean 1, variance 1) and each count pixel
 * is Bernoulli(q), q = P(rho > rho_th) = exp(-rho_th).  Hence
 *   power: <s> = W1, var = W2          -> Psi = (s - W1)/sqrt(W2)
 *   count: <c> = N q, var = N q (1-q)  -> Psi = (c - N q)/sqrt(N q (1-q))
 * sigma_s is the square root of the variance.  N = 0 gives NaN. */
double oracle_count_q(float rho_th) { return exp(-(double)rho_th); }

void oracle_psi_power(int64_t n, const double *s, const int32_t *N,
                      const double *W1, const double *W2, double *psi)
{
    for (int64_t i = 0; i < n; ++i) {
        if (N[i] == 0) { psi[i] = NAN; continue; }
        double num = s[i] - W1[i];
        double den = sqrt(W2[i]);
        psi[i] = num / den;
    }
}

void oracle_psi_count(int64_t n, const int32_t *c, const int32_t *N, float rho_th,
                      double *psi)
{
    double q = oracle_count_q(rho_th);
    double omq = 1.0 - q;
    for (int64_t i = 0; i < n; ++i) {
        if (N[i] == 0) { psi[i] = NAN; continue; }
        double Nq = (double)N[i] * q;
        double num = (double)c[i] - Nq;
        double var = Nq * omq;
        psi[i] = num / sqrt(var);
    }
}

/* ------------------------------------------------------------------------ */
/* Storage formats, written from the bit-level format definitions.
 *
 * bfloat16: the upper 16 bits of an IEEE binary32, rounded to nearest with
 * ties to even on the 16 discarded bits; NaN stays a quiet NaN. */
static uint32_t f2u(float f) { uint32_t u; memcpy(&u, &f, 4); return u; }
static float u2f(uint32_t u) { float f; memcpy(&f, &u, 4); return f; }

uint16_t oracle_bf16_rne(float x)
{
    uint32_t u = f2u(x);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu))
        return (uint16_t)((u >> 16) | 0x0040u); /* quiet NaN */
    uint32_t keep = u >> 16, drop = u & 0xffffu;
    if (drop > 0x8000u || (drop == 0x8000u && (keep & 1u))) keep += 1u;
    return (uint16_t)keep;
}

float oracle_bf16_decode(uint16_t h) { return u2f((uint32_t)h << 16); }

/* OCP 8-bit E4M3 ("E4M3FN"): 1 sign, 4 exponent bits (bias 7), 3 mantissa
 * bits; no infinities; S.1111.111 is NaN; largest finite 448 = 1.75 * 2^8;
 * subnormals m * 2^-9.  Encoding rounds to nearest, ties to even, and
 * saturates finite values beyond 448 to +-448. */
float oracle_e4m3_decode(uint8_t b)
{
    int s = b >> 7, e = (b >> 3) & 15, m = b & 7;
    double v;
    if (e == 15 && m == 7) return NAN;
    if (e == 0) v = ldexp((double)m, -9);
    else v = ldexp(1.0 + m / 8.0, e - 7);
    return (float)(s ? -v : v);
}

uint8_t oracle_e4m3_rne_sat(float x)
{
    if (isnan(x)) return 0x7f;
    uint8_t sign = signbit(x) ? 0x80 : 0x00;
    double a = fabs((double)x);
    /* Walk the 127 non-negative finite codes in increasing order and pick the
     * nearest; ties go to the code with an even mantissa (even code). */
    if (a >= 448.0) return sign | 0x7e;
    uint8_t best = 0;
    for (uint8_t c = 0; c < 0x7e; ++c) {
        double lo = oracle_e4m3_decode(c), hi = oracle_e4m3_decode((uint8_t)(c + 1));
        if (a >= lo && a <= hi) {
            double dlo = a - lo, dhi = hi - a;
            if (dlo < dhi) best = c;
            else if (dhi < dlo) best = (uint8_t)(c + 1);
            else best = (c & 1) ? (uint8_t)(c + 1) : c;
            break;
        }
    }
    return sign | best;
}

/* Per-segment FP8 scale: rowmax/448 in FP32, or 1 for an all-zero row. */
float oracle_fp8_row_scale(const float *row, int32_t n)
{
    float m = 0.0f;
    for (int32_t i = 0; i < n; ++i)
        if (row[i] > m) m = row[i];
    if (m == 0.0f) return 1.0f;
    return m / 448.0f;
}

/* Values a quantised store reproduces, in FP64, for rows of n_bins FP32
 * powers: store 1 = bfloat16, store 2 = E4M3 with per-row scale (value =
 * scale * decode(code), exact in FP64).  scale_out may be NULL. */
void oracle_dequantised(const float *rho, int32_t n_seg, int32_t n_bins, int32_t store,
                        double *out, float *scale_out)
{
    for (int32_t j = 0; j < n_seg; ++j) {
        const float *row = rho + (int64_t)j * n_bins;
        double *o = out + (int64_t)j * n_bins;
        if (store == 1) {
            for (int32_t b = 0; b < n_bins; ++b)
                o[b] = (double)oracle_bf16_decode(oracle_bf16_rne(row[b]));
        } else if (store == 2) {
            float sc = oracle_fp8_row_scale(row, n_bins);
            if (scale_out) scale_out[j] = sc;
            for (int32_t b = 0; b < n_bins; ++b) {
                float r = row[b] / sc;
                o[b] = (double)sc * (double)oracle_e4m3_decode(oracle_e4m3_rne_sat(r));
            }
        } else {
            for (int32_t b = 0; b < n_bins; ++b) o[b] = (double)row[b];
        }
    }
}

void oracle_bf16_rne_array(const float *x, int64_t n, uint16_t *out)
{
    for (int64_t i = 0; i < n; ++i) out[i] = oracle_bf16_rne(x[i]);
}

void oracle_e4m3_rne_sat_array(const float *x, int64_t n, uint8_t *out)
{
    for (int64_t i = 0; i < n; ++i) out[i] = oracle_e4m3_rne_sat(x[i]);
}

void oracle_spin_factor_array(const double *t, int64_t n, double t0, double tau,
                              double brake, double *out)
{
    for (int64_t i = 0; i < n; ++i) out[i] = oracle_spin_factor(t[i], t0, tau, brake);
}

/* Threads the oracle's parallel loops use. */
int32_t oracle_threads(void)
{
#ifdef _OPENMP
    return (int32_t)omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Counter-based random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw,
 * "Parallel random numbers: as easy as 1, 2, 3", SC11).  Ten rounds of
 *   (c0, c1, c2, c3) -> (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0))
 * with the key advanced by the Weyl constants between rounds.  Used for the
 * synthetic noise of the learned proposer's training data; the library has
 * its own implementation and the tests compare the two. */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)PHILOX_M0 * c0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += PHILOX_W0;
        k1 += PHILOX_W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Exp(1) noise for realisation r of a [n_seg][n_bins] spectrogram: element e
 * takes word e % 4 of Philox(counter = (e/4 low, e/4 high, r, stream),
 * key = (seed low, seed high)); u = (word + 1/2) 2^-32 in (0, 1) is exact in
 * FP64, and the value is RN_32(-log(u)) with log taken in FP64. */
void oracle_exp_noise(uint64_t seed, uint32_t stream, int32_t r, int64_t n, float *out)
{
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t w[4];
    for (int64_t e = 0; e < n; ++e) {
        if ((e & 3) == 0 || e == 0) {
            const uint64_t b = (uint64_t)e >> 2;
            const uint32_t ctr[4] = {(uint32_t)b, (uint32_t)(b >> 32), (uint32_t)r, stream};
            oracle_philox4x32_10(ctr, key, w);
        }
        double u = ((double)w[e & 3] + 0.5) * 0x1p-32;
        out[e] = (float)(-log(u));
    }
}
