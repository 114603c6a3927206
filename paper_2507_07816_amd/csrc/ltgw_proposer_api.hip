// C-ABI of the learned proposer (declarations and contracts in
// include/ltgw.h): device-generated training stacks, coarse and listed
// critical ratios on them, the ranking network's passes, the loss, Adam,
// top-M selection, and the propose call with its exhaustive fallback.
#include <hip/hip_runtime.h>

#include <cmath>
#include <algorithm>
#include <cstring>
#include <vector>

#include "ltgw_ctx.h"
#include "ltgw_proposer.h"

using namespace ltgw;

namespace ltgw {

void free_stack(StackState &S) {
    DevBuf *all[] = {&S.fine,   &S.crs,      &S.w,        &S.wq,    &S.scale,  &S.w2,     &S.t,
                     &S.v,      &S.t2,       &S.v2,       &S.params, &S.psi_c, &S.x,      &S.act,
                     &S.logits, &S.cells,    &S.tpl,      &S.psi_sel, &S.best_idx, &S.best_psi, &S.fb,
                     &S.rmap,   &S.psi_all, &S.bscore, &S.blk, &S.blk2, &S.tpl2, &S.psi2,
                     &S.cm_idx, &S.cm,      &S.rows2,   &S.flag2, &S.bi2,  &S.bp2,   &S.counts, &S.blocks,
                     &S.records, &S.cmap};
    for (DevBuf *b : all) release(*b);
    for (StackLevel &L : S.lv) {
        release(L.tau);
        release(L.brake);
        release(L.sky);
        release(L.g);
        release(L.H);
        release(L.mw1);
        release(L.mw2);
        release(L.mn);
    }
    if (S.ev_h2d) (void)hipEventDestroy(S.ev_h2d);
    S = StackState();
}

}  // namespace ltgw

namespace {

int esize(int store) { return store == LTGW_STORE_F32 ? 4 : store == LTGW_STORE_BF16 ? 2 : 1; }

bool on_device(const void *p) { return p && is_device_ptr(p); }

int need_device(ltgw_ctx *c, const void *p, const char *what) {
    if (!on_device(p)) return fail(c, LTGW_E_INVALID_ARG, "%s must be a device pointer", what);
    return LTGW_OK;
}

int need_stack(ltgw_ctx *c, int level) {
    const StackState &S = c->stack;
    if (!S.valid) return fail(c, LTGW_E_STATE, "no stack loaded");
    if (level == 1 && !S.coarse) return fail(c, LTGW_E_STATE, "the stack has no coarse store");
    return LTGW_OK;
}

EvalArgs stack_args(const StackState &S, int level, const ltgw_grid *g, const SearchPlan &P,
                    int64_t &stack_bytes, int64_t &stack_rows);

// The per-template moments of a level on g's lattice, formed once per set of
// tables and lattice (the weights are those of every realisation).
int stack_moments(ltgw_ctx *c, const ltgw_grid *g, int level, const SearchPlan &P) {
    StackState &S = c->stack;
    StackLevel &L = S.lv[level];
    if (L.mom && L.m_f0_min == g->f0_min && L.m_f0_step == g->f0_step && L.m_n_f0 == g->n_f0) return LTGW_OK;
    L.mom = false;
    const int64_t n = P.n_tpl;
    int rc;
    if ((rc = ensure(c, L.mw1, (size_t)n * 8, "moments")) != LTGW_OK) return rc;
    if ((rc = ensure(c, L.mw2, (size_t)n * 8, "moments")) != LTGW_OK) return rc;
    if ((rc = ensure(c, L.mn, (size_t)n * 4, "moments")) != LTGW_OK) return rc;
    int64_t sb = 0, sr = 0;
    const EvalArgs a = stack_args(S, level, g, P, sb, sr);
    HIP_TRY(c, launch_stack_moments(level, a, (double *)L.mw1.p, (double *)L.mw2.p, (int32_t *)L.mn.p, c->stream),
            "moments launch");
    L.m_f0_min = g->f0_min;
    L.m_f0_step = g->f0_step;
    L.m_n_f0 = g->n_f0;
    L.mom = true;
    return LTGW_OK;
}

StackMoments level_moments(const StackState &S, int level) {
    const StackLevel &L = S.lv[level];
    return StackMoments{(const double *)L.mw1.p, (const double *)L.mw2.p, (const int32_t *)L.mn.p};
}

// Validate grid g against the stack's detector slot, upload its axes for
// stack level `level` and form the spin-down (Eq. 1) and track-factor
// (Eqs. 1-2) tables at the level's segment times and velocities: level 0
// every segment, level 1 the first segment of each pair.
int stack_tables(ltgw_ctx *c, const ltgw_grid *g, int level, SearchPlan &P) {
    StackState &S = c->stack;
    int slot = S.det;
    int rc = plan_search(c, g, &slot, 1, P);
    if (rc != LTGW_OK) return rc;
    const Det &D = c->det[slot];
    if (D.n_seg != S.n_seg || D.n_bins != S.n_bins || D.k_lo != S.k_lo || D.t_sft != S.t_sft)
        return fail(c, LTGW_E_STATE, "detector slot %d changed shape since the stack was loaded", slot);
    StackLevel &L = S.lv[level];
    // the same axes and T0 as the last call on this level: the tables stand
    if (L.tables && L.t0 == g->t0 && L.h_tau.size() == (size_t)g->n_tau &&
        L.h_brake.size() == (size_t)g->n_brake && L.h_sky.size() == 3 * (size_t)g->n_sky &&
        std::equal(L.h_tau.begin(), L.h_tau.end(), g->tau) &&
        std::equal(L.h_brake.begin(), L.h_brake.end(), g->brake) &&
        std::equal(L.h_sky.begin(), L.h_sky.end(), g->sky))
        return stack_moments(c, g, level, P);
    L.tables = false;
    L.mom = false;
    HIP_TRY(c, hipEventSynchronize(S.ev_h2d), "previous grid upload");
    L.h_tau.assign(g->tau, g->tau + g->n_tau);
    L.h_brake.assign(g->brake, g->brake + g->n_brake);
    L.h_sky.assign(g->sky, g->sky + 3 * (size_t)g->n_sky);
    const int ns = level ? S.n_seg / S.S : S.n_seg;
    if ((rc = ensure(c, L.tau, L.h_tau.size() * 8, "tau")) != LTGW_OK) return rc;
    if ((rc = ensure(c, L.brake, L.h_brake.size() * 8, "brake")) != LTGW_OK) return rc;
    if ((rc = ensure(c, L.sky, L.h_sky.size() * 8, "sky")) != LTGW_OK) return rc;
    if ((rc = ensure(c, L.g, (size_t)P.n_tn * ns * 8, "spin-factor table")) != LTGW_OK) return rc;
    if ((rc = ensure(c, L.H, (size_t)P.n_groups * ns * 8, "track-factor table")) != LTGW_OK) return rc;
    if ((rc = h2d(c, L.tau.p, L.h_tau.data(), L.h_tau.size() * 8, "tau upload")) != LTGW_OK) return rc;
    if ((rc = h2d(c, L.brake.p, L.h_brake.data(), L.h_brake.size() * 8, "brake upload")) != LTGW_OK) return rc;
    if ((rc = h2d(c, L.sky.p, L.h_sky.data(), L.h_sky.size() * 8, "sky upload")) != LTGW_OK) return rc;
    HIP_TRY(c, hipEventRecord(S.ev_h2d, c->stream), "event record");
    HIP_TRY(c, launch_spin_factor((const double *)(level ? S.t2.p : S.t.p), ns, g->t0, (const double *)L.tau.p,
                                  g->n_tau, (const double *)L.brake.p, g->n_brake, (double *)L.g.p,
                                  (unsigned long long *)c->counters.p + kCntUndecided, c->stream),
            "spin-factor launch");
    HIP_TRY(c, launch_track_factor((const double *)L.g.p, P.n_tn, (const double *)(level ? S.v2.p : S.v.p), ns,
                                   (const double *)L.sky.p, g->n_sky, S.t_sft, (double *)L.H.p, c->stream),
            "track-factor launch");
    L.t0 = g->t0;
    L.tables = true;
    return stack_moments(c, g, level, P);
}

// The evaluation arguments of a stack level (realisation 0; the kernels
// offset store and weights per realisation).
EvalArgs stack_args(const StackState &S, int level, const ltgw_grid *g, const SearchPlan &P,
                    int64_t &stack_bytes, int64_t &stack_rows) {
    EvalArgs a;
    std::memset(&a, 0, sizeof a);
    DetView &V = a.det[0];
    const StackLevel &L = S.lv[level];
    if (level == 0) {
        V.store = S.fine.p;
        V.pitch_bytes = (int32_t)(S.pitch * esize(S.store));
        V.wq = (const float *)S.wq.p;
        V.w = (const float *)S.w.p;
        V.cshift = 1.5 - (double)S.k_lo;
        V.n_seg = S.n_seg;
        V.n_bins = S.n_bins;
        stack_bytes = (int64_t)S.n_seg * S.pitch * esize(S.store);
        stack_rows = S.n_seg;
    } else {
        // coarse column of fine column b is b >> 1: index trunc(x + 2.5 - k_lo) >> 1;
        // 32-bit words (bfloat16 power sum, count)
        V.store = S.crs.p;
        V.pitch_bytes = (int32_t)(S.pitch2 * 4);
        V.wq = (const float *)S.w2.p;
        V.w = (const float *)S.w2.p;
        V.cshift = 2.5 - (double)S.k_lo;
        V.n_seg = S.n_seg / S.S;
        V.n_bins = S.n_bins / 2;
        stack_bytes = (int64_t)(S.n_seg / S.S) * S.pitch2 * 4;
        stack_rows = S.n_seg / S.S;
    }
    V.H = (const double *)L.H.p;
    V.g = (const double *)L.g.p;
    V.D = nullptr;
    V.t_sft = S.t_sft;
    V.wfix = nullptr;
    a.n_det = 1;
    a.n_f0 = g->n_f0;
    a.n_groups = (int32_t)P.n_groups;
    a.n_tn = P.n_tn;
    a.f0_min = g->f0_min;
    a.f0_step = g->f0_step;
    a.w_uniform = 1.0f;
    return a;
}

// The moments of a level with the statistic to write: POWER, or COUNT (the
// fine level) with q = exp(-rho_th) of the stack's detector.
StackMoments stat_moments(ltgw_ctx *c, int level, uint32_t stat) {
    StackMoments m = level_moments(c->stack, level);
    if (stat == LTGW_STAT_COUNT) {
        m.count = 1;
        m.q = std::exp(-(double)c->det[c->stack.det].rho_th);
    }
    return m;
}

int stack_psi_impl(ltgw_ctx *c, const ltgw_grid *g, int level, int nan_to_zero, double *out_psi,
                   uint32_t stat = LTGW_STAT_POWER) {
    int rc = need_stack(c, level);
    if (rc != LTGW_OK) return rc;
    if (level != 0 && level != 1) return fail(c, LTGW_E_INVALID_ARG, "level must be 0 or 1");
    if ((rc = need_device(c, out_psi, "out_psi")) != LTGW_OK) return rc;
    SearchPlan P;
    if ((rc = stack_tables(c, g, level, P)) != LTGW_OK) return rc;
    int64_t sb = 0, sr = 0;
    const EvalArgs a = stack_args(c->stack, level, g, P, sb, sr);
    const int shift = level;
    const int store = level ? kStoreCoarse : c->stack.store;
    const double mu = level ? 2.0 * c->stack.S : 1.0;  // a coarse pixel sums 2 S Exp(1) values
    HIP_TRY(c, launch_stack_eval(store, shift, a, c->stack.R, sb, sr, mu, mu, nan_to_zero, nullptr, nullptr,
                                 stat_moments(c, level, stat), out_psi, c->stream),
            "stack evaluation launch");
    return LTGW_OK;
}

// The network's input on the coarse store: FP32 power ratios per coarse
// group, then (counts) the count ratios; psi (optional) the FP64 power ratios.
int features_impl(ltgw_ctx *c, const ltgw_grid *coarse, int counts, float *x, double *psi) {
    int rc = need_stack(c, 1);
    if (rc != LTGW_OK) return rc;
    SearchPlan P;
    if ((rc = stack_tables(c, coarse, 1, P)) != LTGW_OK) return rc;
    StackState &S = c->stack;
    int64_t sb = 0, sr = 0;
    const EvalArgs a = stack_args(S, 1, coarse, P, sb, sr);
    const double q = std::exp(-(double)c->det[S.det].rho_th);  // count probability of a noise pixel
    HIP_TRY(c, launch_stack_features(a, S.R, sb, sr, 2.0 * S.S, q, counts, level_moments(S, 1), x, psi, c->stream),
            "features launch");
    return LTGW_OK;
}

int list_psi_impl(ltgw_ctx *c, const ltgw_grid *g, const int32_t *idx, int rows, int32_t m,
                  const int32_t *rmap, const int32_t *n_rows, double *out_psi, SearchPlan *plan_out,
                  uint32_t stat = LTGW_STAT_POWER) {
    SearchPlan P;
    int rc = stack_tables(c, g, 0, P);
    if (rc != LTGW_OK) return rc;
    int64_t sb = 0, sr = 0;
    const EvalArgs a = stack_args(c->stack, 0, g, P, sb, sr);
    HIP_TRY(c, launch_list_eval(c->stack.store, a, rows, sb, sr, idx, m, rmap, n_rows, stat_moments(c, 0, stat),
                                out_psi, c->stream),
            "listed evaluation launch");
    if (plan_out) *plan_out = P;
    return LTGW_OK;
}

}  // namespace

extern "C" {

int32_t ltgw_generate_noise(ltgw_ctx *c, uint64_t seed, uint32_t stream, int32_t r0, int32_t R, int64_t n,
                            float *out) {
    if (!c) return LTGW_E_INVALID_ARG;
    Enter en(c);
    if (R < 1 || R > 65535) return fail(c, LTGW_E_INVALID_ARG, "R must be in 1 .. 65535");
    if (r0 < 0 || (int64_t)r0 + R > ((int64_t)1 << 31)) return fail(c, LTGW_E_INVALID_ARG, "r0 out of range");
    if (n < 1 || n > ((int64_t)1 << 40)) return fail(c, LTGW_E_INVALID_ARG, "n must be in 1 .. 2^40");
    int rc = need_device(c, out, "out");
    if (rc != LTGW_OK) return rc;
    HIP_TRY(c, launch_noise(seed, stream, r0, R, n, out, c->stream), "noise launch");
    return LTGW_OK;
}

int32_t ltgw_inject_stack(ltgw_ctx *c, int32_t det, float *stack, int32_t R, const double *params,
                          const double *sky3, double t0) {
    if (!c) return LTGW_E_INVALID_ARG;
    Enter en(c);
    if (det < 0 || det >= LTGW_MAX_DET) return fail(c, LTGW_E_INVALID_ARG, "detector %d out of range", det);
    const Det &D = c->det[det];
    if (!D.loaded || !D.has_v) return fail(c, LTGW_E_STATE, "detector %d needs a spectrogram and a velocity table", det);
    if (R < 1 || R > 65535) return fail(c, LTGW_E_INVALID_ARG, "R must be in 1 .. 65535");
    if (!params || !sky3) return fail(c, LTGW_E_INVALID_ARG, "params or sky is NULL");
    int rc = need_device(c, stack, "stack");
    if (rc != LTGW_OK) return rc;
    if (!fin(t0)) return fail(c, LTGW_E_INVALID_ARG, "t0 must be finite");
    double sky[3];
    if ((rc = to_host(c, sky, sky3, sizeof sky, "sky")) != LTGW_OK) return rc;
    if (!fin(sky[0]) || !fin(sky[1]) || !fin(sky[2]) ||
        std::fabs(std::sqrt(sky[0] * sky[0] + sky[1] * sky[1] + sky[2] * sky[2]) - 1.0) > 1e-12)
        return fail(c, LTGW_E_INVALID_ARG, "sky must be a finite unit vector");
    std::vector<double> hp(4 * (size_t)R);
    if ((rc = to_host(c, hp.data(), params, hp.size() * 8, "params")) != LTGW_OK) return rc;
    for (int32_t r = 0; r < R; ++r) {
        const double *q = &hp[4 * (size_t)r];
        if (!fin(q[3]) || q[3] < 0.0) return fail(c, LTGW_E_INVALID_ARG, "amplitude %d must be finite and >= 0", r);
        if (q[3] == 0.0) continue;
        if (!fin(q[0]) || !(q[0] > 0.0) || !fin(q[1]) || !(q[1] > 0.0) || !fin(q[2]) || !(q[2] > 1.0))
            return fail(c, LTGW_E_INVALID_ARG, "injection %d needs f0 > 0, tau > 0, n > 1", r);
        if (!(q[0] * D.t_sft * (1.0 + D.v_max) < (double)(1 << 30) - 4.0))
            return fail(c, LTGW_E_INVALID_ARG, "injection %d: f0 * t_sft too large", r);
    }
    StackState &S = c->stack;
    if ((rc = ensure(c, S.params, hp.size() * 8, "injection parameters")) != LTGW_OK) return rc;
    if ((rc = h2d(c, S.params.p, hp.data(), hp.size() * 8, "injection upload")) != LTGW_OK) return rc;
    HIP_TRY(c, launch_inject_stack(stack, R, D.n_seg, D.n_bins, D.k_lo, D.t_sft, (const double *)D.t_seg.p,
                                   (const double *)D.v.p, (const float *)D.w.p, (const double *)S.params.p,
                                   sky[0], sky[1], sky[2], t0,
                                   (unsigned long long *)c->counters.p + kCntUndecided, c->stream),
            "injection launch");
    HIP_TRY(c, hipStreamSynchronize(c->stream), "injection");
    return LTGW_OK;
}

int32_t ltgw_load_stack(ltgw_ctx *c, int32_t det, int32_t R, const float *stack, int32_t store,
                        int32_t coarse) {
    if (!c) return LTGW_E_INVALID_ARG;
    Enter en(c);
    StackState &S = c->stack;
    S.valid = false;
    S.lv[0].tables = S.lv[1].tables = false;
    if (det < 0 || det >= LTGW_MAX_DET) return fail(c, LTGW_E_INVALID_ARG, "detector %d out of range", det);
    const Det &D = c->det[det];
    if (!D.loaded || !D.has_v) return fail(c, LTGW_E_STATE, "detector %d needs a spectrogram and a velocity table", det);
    if (R < 1 || R > 65535) return fail(c, LTGW_E_INVALID_ARG, "R must be in 1 .. 65535");
    if (store != LTGW_STORE_F32 && store != LTGW_STORE_BF16 && store != LTGW_STORE_FP8)
        return fail(c, LTGW_E_INVALID_ARG, "unknown store %d", store);
    int rc = need_device(c, stack, "stack");
    if (rc != LTGW_OK) return rc;
    const int64_t ns = D.n_seg, nb = D.n_bins;
    const int Sg = coarse == 1 ? 2 : coarse;  // segments per coarse row
    if (coarse < 0 || (coarse > 0 && Sg != 2 && Sg != 4 && Sg != 8))
        return fail(c, LTGW_E_INVALID_ARG, "coarse must be 0 (none), 1 or 2 (pairs of segments), 4 or 8");
    if (coarse && ((ns % Sg) || (nb & 1)))
        return fail(c, LTGW_E_INVALID_ARG, "a coarse store needs n_seg a multiple of %d and even n_bins (have %lld, %lld)",
                    Sg, (long long)ns, (long long)nb);
    if ((int64_t)R * ns >= ((int64_t)1 << 31)) return fail(c, LTGW_E_UNSUPPORTED, "R * n_seg exceeds 2^31 rows");
    const int64_t pitch = ((nb + 2 + 63) / 64) * 64;
    if (ns * pitch * esize(store) >= ((int64_t)1 << 31))
        return fail(c, LTGW_E_UNSUPPORTED, "one realisation's store exceeds 2^31 bytes");
    if (!S.ev_h2d) HIP_TRY(c, hipEventCreateWithFlags(&S.ev_h2d, hipEventDisableTiming), "event create");
    HIP_TRY(c, hipEventSynchronize(S.ev_h2d), "previous upload");
    const int64_t rows = (int64_t)R * ns;
    if ((rc = ensure(c, S.fine, (size_t)(rows * pitch * esize(store)), "stack store")) != LTGW_OK) return rc;
    if ((rc = ensure(c, S.w, (size_t)rows * 4, "stack weights")) != LTGW_OK) return rc;
    if ((rc = ensure(c, S.wq, (size_t)rows * 4, "stack scaled weights")) != LTGW_OK) return rc;
    if ((rc = ensure(c, S.scale, (size_t)rows * 4, "stack scales")) != LTGW_OK) return rc;
    if ((rc = ensure(c, S.t, (size_t)ns * 8, "stack segment times")) != LTGW_OK) return rc;
    if ((rc = ensure(c, S.v, (size_t)ns * 24, "stack velocities")) != LTGW_OK) return rc;
    std::vector<float> hw((size_t)rows);
    for (int64_t r = 0; r < R; ++r) std::memcpy(&hw[(size_t)(r * ns)], D.h_w.data(), (size_t)ns * 4);
    if ((rc = h2d(c, S.w.p, hw.data(), hw.size() * 4, "stack weights upload")) != LTGW_OK) return rc;
    if ((rc = h2d(c, S.t.p, D.h_t.data(), (size_t)ns * 8, "segment times upload")) != LTGW_OK) return rc;
    if ((rc = h2d(c, S.v.p, D.h_v.data(), (size_t)ns * 24, "velocity upload")) != LTGW_OK) return rc;
    std::vector<float> hw2;
    std::vector<double> ht2, hv2;
    int64_t pitch2 = 0;
    if (coarse) {
        const int64_t ns2 = ns / Sg, nb2 = nb / 2;
        pitch2 = ((nb2 + 2 + 31) / 32) * 32;  // rows of whole 128-byte lines
        if (ns2 * pitch2 * 4 >= ((int64_t)1 << 31))
            return fail(c, LTGW_E_UNSUPPORTED, "one realisation's coarse store exceeds 2^31 bytes");
        if ((rc = ensure(c, S.crs, (size_t)(R * ns2 * pitch2 * 4), "coarse store")) != LTGW_OK) return rc;
        if ((rc = ensure(c, S.w2, (size_t)(R * ns2) * 4, "coarse weights")) != LTGW_OK) return rc;
        if ((rc = ensure(c, S.t2, (size_t)ns2 * 8, "coarse segment times")) != LTGW_OK) return rc;
        if ((rc = ensure(c, S.v2, (size_t)ns2 * 24, "coarse velocities")) != LTGW_OK) return rc;
        // a group's weight: its S weights summed in order, times 1/S (FP32)
        hw2.resize((size_t)(R * ns2));
        for (int64_t j = 0; j < ns2; ++j) {
            float acc = D.h_w[(size_t)(Sg * j)];
            for (int k = 1; k < Sg; ++k) acc = acc + D.h_w[(size_t)(Sg * j + k)];
            hw2[(size_t)j] = acc * (1.0f / (float)Sg);
        }
        for (int64_t r = 1; r < R; ++r) std::memcpy(&hw2[(size_t)(r * ns2)], hw2.data(), (size_t)ns2 * 4);
        ht2.resize((size_t)ns2);
        hv2.resize((size_t)ns2 * 3);
        for (int64_t j = 0; j < ns2; ++j) {
            ht2[(size_t)j] = D.h_t[(size_t)(Sg * j)];
            for (int k = 0; k < 3; ++k) hv2[3 * (size_t)j + k] = D.h_v[3 * (size_t)(Sg * j) + k];
        }
        if ((rc = h2d(c, S.w2.p, hw2.data(), hw2.size() * 4, "coarse weights upload")) != LTGW_OK) return rc;
        if ((rc = h2d(c, S.t2.p, ht2.data(), ht2.size() * 8, "coarse times upload")) != LTGW_OK) return rc;
        if ((rc = h2d(c, S.v2.p, hv2.data(), hv2.size() * 8, "coarse velocity upload")) != LTGW_OK) return rc;
    }
    if ((rc = zero_counter(c, kCntBad, 1)) != LTGW_OK) return rc;
    // the stores: fine alone, or fine and coarse from one read of the stack
    c->have_ingest = false;
    HIP_TRY(c, hipEventRecord(c->ev_ing[0], c->stream), "event record");
    if (coarse)
        HIP_TRY(c, launch_stack_ingest(store, stack, R, (int32_t)ns, (int32_t)nb, Sg, pitch, S.fine.p,
                                       (float *)S.scale.p, (const float *)S.w.p, (float *)S.wq.p, D.rho_th, pitch2,
                                       (unsigned *)S.crs.p, (unsigned long long *)c->counters.p + kCntBad,
                                       c->stream),
                "stack ingest launch");
    else if ((nb & 1) == 0)  // the same kernel without the coarse store: 4, 2 or 1 rows per workgroup
        HIP_TRY(c, launch_stack_ingest(store, stack, R, (int32_t)ns, (int32_t)nb, ns % 4 == 0 ? 4 : ns % 2 == 0 ? 2 : 1,
                                       pitch, S.fine.p, (float *)S.scale.p, (const float *)S.w.p, (float *)S.wq.p,
                                       D.rho_th, 0, nullptr, (unsigned long long *)c->counters.p + kCntBad,
                                       c->stream),
                "stack ingest launch");
    else
        HIP_TRY(c, launch_ingest(store, stack, (int32_t)rows, (int32_t)nb, pitch, S.fine.p, (float *)S.scale.p,
                                 (const float *)S.w.p, (float *)S.wq.p, D.rho_th,
                                 (unsigned long long *)c->counters.p + kCntBad, c->stream),
                "stack ingest launch");
    HIP_TRY(c, hipEventRecord(c->ev_ing[1], c->stream), "event record");
    c->have_ingest = true;
    unsigned long long bad = 0;
    if ((rc = read_counter(c, kCntBad, &bad)) != LTGW_OK) return rc;  // synchronises: host vectors may go
    if (bad) return fail(c, LTGW_E_INVALID_ARG, "%llu stack values are negative or not finite", bad);
    S.lv[0].tables = S.lv[1].tables = false;  // new geometry (segment times, velocities)
    S.det = det;
    S.R = R;
    S.store = store;
    S.n_seg = (int)ns;
    S.n_bins = (int)nb;
    S.k_lo = D.k_lo;
    S.t_sft = D.t_sft;
    S.pitch = pitch;
    S.pitch2 = pitch2;
    S.coarse = coarse != 0;
    S.S = coarse ? Sg : 2;
    S.valid = true;
    return LTGW_OK;
}

int32_t ltgw_stack_psi(ltgw_ctx *c, const ltgw_grid *g, int32_t level, int32_t nan_to_zero, double *out_psi) {
    if (!c) return LTGW_E_INVALID_ARG;
    Enter en(c);
    return stack_psi_impl(c, g, level, nan_to_zero, out_psi);
}

int32_t ltgw_stack_psi_list(ltgw_ctx *c, const ltgw_grid *g, uint32_t stat, const int32_t *idx, int32_t m,
                            double *out_psi) {
    if (!c) return LTGW_E_INVALID_ARG;
    Enter en(c);
    int rc = need_stack(c, 0);
    if (rc != LTGW_OK) return rc;
    if (stat != LTGW_STAT_POWER && stat != LTGW_STAT_COUNT)
        return fail(c, LTGW_E_INVALID_ARG, "stat must be POWER or COUNT");
    if (m < 1) return fail(c, LTGW_E_INVALID_ARG, "m must be >= 1");
    if ((rc = need_device(c, idx, "idx")) != LTGW_OK) return rc;
    if ((rc = need_device(c, out_psi, "out_psi")) != LTGW_OK) return rc;
    return list_psi_impl(c, g, idx, c->stack.R, m, nullptr, nullptr, out_psi, nullptr, stat);
}

int64_t ltgw_cnn_param_count(int32_t c_in, int32_t c_out) {
    if (c_in < 1 || c_out < 1 || c_in > 4096 || c_out > 4096) return LTGW_E_INVALID_ARG;
    return cnn_n_params(c_in, c_out);
}

int64_t ltgw_cnn_work_floats(int32_t B, int32_t c_in, int32_t c_out, int32_t L) {
    if (B < 1 || L < 1 || c_in < 1 || c_out < 1 || c_in > 4096 || c_out > 4096) return LTGW_E_INVALID_ARG;
    return cnn_work_floats(B, c_in, c_out, L);
}

static int cnn_shape_ok(ltgw_ctx *c, int32_t B, int32_t c_in, int32_t c_out, int32_t L) {
    if (B < 1 || L < 1 || c_in < 1 || c_out < 1 || c_in > 4096 || c_out > 4096)
        return fail(c, LTGW_E_INVALID_ARG, "network shape must have B, L, c_in, c_out >= 1 (c <= 4096)");
    if ((int64_t)B * L >= ((int64_t)1 << 31) / 64)
        return fail(c, LTGW_E_UNSUPPORTED, "B * L too large");
    return LTGW_OK;
}

int32_t ltgw_cnn_forward(ltgw_ctx *c, const float *params, const float *x, int32_t B, int32_t c_in,
                         int32_t c_out, int32_t L, float *act, float *logits) {
    if (!c) return LTGW_E_INVALID_ARG;
    Enter en(c);
    int rc = cnn_shape_ok(c, B, c_in, c_out, L);
    if (rc != LTGW_OK) return rc;
    const void *ptrs[] = {params, x, logits};
    for (const void *p : ptrs)
        if ((rc = need_device(c, p, "network arrays")) != LTGW_OK) return rc;
    if (!act) {  // inference only: the fused pass where the shape allows it
        if (cnn_infer_supported(c_in, c_out, L)) {
            if ((rc = ensure(c, c->cnn_packed, (size_t)cnn_infer_scratch_shorts(c_in) * 2, "packed weights")) !=
                LTGW_OK)
                return rc;
            HIP_TRY(c, launch_cnn_infer(params, x, B, c_in, c_out, L, (short *)c->cnn_packed.p, logits, nullptr, 0,
                                        c->stream),
                    "network forward");
            return LTGW_OK;
        }
        return fail(c, LTGW_E_INVALID_ARG, "act may be NULL only for c_in, c_out <= 32 and L <= 256");
    }
    if ((rc = need_device(c, act, "network activations")) != LTGW_OK) return rc;
    HIP_TRY(c, launch_cnn_forward(params, x, B, c_in, c_out, L, act, logits, c->stream), "network forward");
    return LTGW_OK;
}

int32_t ltgw_cnn_backward(ltgw_ctx *c, const float *params, const float *x, int32_t B, int32_t c_in,
                          int32_t c_out, int32_t L, const float *act, const float *dlogits, float *work,
                          int64_t work_floats, float *grads) {
    if (!c) return LTGW_E_INVALID_ARG;
    Enter en(c);
    int rc = cnn_shape_ok(c, B, c_in, c_out, L);
    if (rc != LTGW_OK) return rc;
    const void *ptrs[] = {params, x, act, dlogits, work, grads};
    for (const void *p : ptrs)
        if ((rc = need_device(c, p, "network arrays")) != LTGW_OK) return rc;
    if (work_floats < cnn_work_floats(B, c_in, c_out, L))
        return fail(c, LTGW_E_INVALID_ARG, "work area of %lld floats, need %lld", (long long)work_floats,
                    (long long)cnn_work_floats(B, c_in, c_out, L));
    HIP_TRY(c, launch_cnn_backward(params, x, B, c_in, c_out, L, act, dlogits, work, work_floats, grads, c->stream),
            "network backward");
    return LTGW_OK;
}

int32_t ltgw_softmax_xent(ltgw_ctx *c, const float *logits, int32_t B, int32_t n_cells, const int32_t *target,
                          int32_t n_valid, float *loss, float *dlogits) {
    if (!c) return LTGW_E_INVALID_ARG;
    Enter en(c);
    if (B < 1 || n_cells < 1 || n_valid < 0) return fail(c, LTGW_E_INVALID_ARG, "B, n_cells >= 1, n_valid >= 0");
    int rc;
    const void *ptrs[] = {logits, target, loss, dlogits};
    for (const void *p : ptrs)
        if ((rc = need_device(c, p, "loss arrays")) != LTGW_OK) return rc;
    HIP_TRY(c, launch_softmax_xent(logits, B, n_cells, target, n_valid, loss, dlogits, c->stream), "loss launch");
    return LTGW_OK;
}

int32_t ltgw_adam_step(ltgw_ctx *c, float *params, const float *grads, float *m, float *v, int64_t n, float lr,
                       float beta1, float beta2, float eps, int32_t step) {
    if (!c) return LTGW_E_INVALID_ARG;
    Enter en(c);
    if (n < 1 || step < 1 || !(lr > 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) ||
        !(eps > 0.0f))
        return fail(c, LTGW_E_INVALID_ARG, "Adam needs n, step >= 1, lr > 0, betas in [0, 1), eps > 0");
    int rc;
    const void *ptrs[] = {params, grads, m, v};
    for (const void *p : ptrs)
        if ((rc = need_device(c, p, "Adam arrays")) != LTGW_OK) return rc;
    HIP_TRY(c, launch_adam(params, grads, m, v, n, lr, beta1, beta2, eps, step, c->stream), "Adam launch");
    return LTGW_OK;
}

int32_t ltgw_select_top(ltgw_ctx *c, const float *score, int32_t R, int32_t n, int32_t M, int32_t *out_idx) {
    if (!c) return LTGW_E_INVALID_ARG;
    Enter en(c);
    if (R < 1 || n < 1 || n > 8192 || M < 1 || M > n)
        return fail(c, LTGW_E_INVALID_ARG, "select_top needs R >= 1, 1 <= M <= n <= 8192");
    int rc;
    if ((rc = need_device(c, score, "score")) != LTGW_OK) return rc;
    if ((rc = need_device(c, out_idx, "out_idx")) != LTGW_OK) return rc;
    HIP_TRY(c, launch_select_top(score, R, n, M, out_idx, c->stream), "selection launch");
    return LTGW_OK;
}

int32_t ltgw_stack_features(ltgw_ctx *c, const ltgw_grid *coarse, int32_t counts, float *x) {
    if (!c) return LTGW_E_INVALID_ARG;
    Enter en(c);
    int rc = need_stack(c, 1);
    if (rc != LTGW_OK) return rc;
    if ((rc = need_device(c, x, "x")) != LTGW_OK) return rc;
    if (!coarse) return fail(c, LTGW_E_INVALID_ARG, "grid is NULL");
    if (counts != 0 && counts != 1) return fail(c, LTGW_E_INVALID_ARG, "counts must be 0 or 1");
    return features_impl(c, coarse, counts, x, nullptr);
}

int32_t ltgw_stack_best(ltgw_ctx *c, const ltgw_grid *g, uint32_t stat, int32_t *best_index, double *best_psi) {
    if (!c) return LTGW_E_INVALID_ARG;
    Enter en(c);
    int rc = need_stack(c, 0);
    if (rc != LTGW_OK) return rc;
    if (stat != LTGW_STAT_POWER && stat != LTGW_STAT_COUNT)
        return fail(c, LTGW_E_INVALID_ARG, "stat must be POWER or COUNT");
    if ((rc = need_device(c, best_index, "best_index")) != LTGW_OK) return rc;
    if ((rc = need_device(c, best_psi, "best_psi")) != LTGW_OK) return rc;
    if (!g) return fail(c, LTGW_E_INVALID_ARG, "grid is NULL");
    StackState &S = c->stack;
    const int64_t n = (int64_t)g->n_f0 * g->n_tau * g->n_brake * g->n_sky;
    if (n < 1) return fail(c, LTGW_E_INVALID_ARG, "empty grid");
    if ((rc = ensure(c, S.psi_all, (size_t)(S.R * n) * 8, "fine ratios")) != LTGW_OK) return rc;
    if ((rc = stack_psi_impl(c, g, 0, 0, (double *)S.psi_all.p, stat)) != LTGW_OK) return rc;
    HIP_TRY(c, launch_row_best((const double *)S.psi_all.p, S.R, n, nullptr, nullptr, best_index, best_psi,
                               c->stream),
            "reduction launch");
    return LTGW_OK;
}

int32_t ltgw_cells_from_templates(ltgw_ctx *c, const int32_t *tpl, int32_t n, int32_t L, const int32_t *mask,
                                  const double *psi, double min_psi, int32_t *cells) {
    if (!c) return LTGW_E_INVALID_ARG;
    Enter en(c);
    if (n < 1 || L < 1) return fail(c, LTGW_E_INVALID_ARG, "n and L must be >= 1");
    int rc;
    if ((rc = need_device(c, tpl, "tpl")) != LTGW_OK) return rc;
    if ((rc = need_device(c, cells, "cells")) != LTGW_OK) return rc;
    if (mask && (rc = need_device(c, mask, "mask")) != LTGW_OK) return rc;
    if (psi && (rc = need_device(c, psi, "psi")) != LTGW_OK) return rc;
    HIP_TRY(c, launch_templates_to_cells(tpl, n, L, mask, psi, min_psi, cells, c->stream), "cell mapping launch");
    return LTGW_OK;
}

int32_t ltgw_propose(ltgw_ctx *c, const ltgw_grid *fine, const ltgw_grid *coarse, const ltgw_proposer *p,
                     int32_t *best_index, double *best_psi, int32_t *fallback) {
    if (!c) return LTGW_E_INVALID_ARG;
    Enter en(c);
    int rc = need_stack(c, 1);
    if (rc != LTGW_OK) return rc;
    if (!fine || !coarse || !p || !best_index || !best_psi || !fallback)
        return fail(c, LTGW_E_INVALID_ARG, "NULL argument");
    StackState &S = c->stack;
    const int R = S.R;
    const int L = p->L;
    const bool net = p->params != nullptr;  // else: the coarse power ratios alone rank the blocks
    if (net && (rc = need_device(c, p->params, "proposer parameters")) != LTGW_OK) return rc;
    if (!net && !p->coarse_map) return fail(c, LTGW_E_INVALID_ARG, "without a network the coarse_map is required");
    if (L < 1 || coarse->n_f0 != L || fine->n_f0 != 2 * L)
        return fail(c, LTGW_E_INVALID_ARG, "coarse grid needs L f0 points and the fine grid 2 L");
    const int64_t g_c = (int64_t)coarse->n_tau * coarse->n_brake * coarse->n_sky;
    const int64_t g_f = (int64_t)fine->n_tau * fine->n_brake * fine->n_sky;
    if ((p->c_in != g_c && p->c_in != 2 * g_c) || p->c_out != 2 * g_f)
        return fail(c, LTGW_E_INVALID_ARG,
                    "network channels must be (coarse groups %lld, or twice that with the count ratios; "
                    "2 x fine groups = %lld)",
                    (long long)g_c, (long long)(2 * g_f));
    const int with_counts = p->c_in == 2 * g_c ? 1 : 0;
    if (!net)
        for (int64_t q = 0; q < 2 * g_f; ++q)
            if (p->coarse_map[q] < -1 || p->coarse_map[q] >= g_c || (q % 2 == 0 && p->coarse_map[q] < 0))
                return fail(c, LTGW_E_INVALID_ARG,
                            "coarse_map[%lld] = %d: each fine group needs a first coarse group in 0 .. %lld "
                            "and a second one or -1",
                            (long long)(q / 2), (int)p->coarse_map[q], (long long)(g_c - 1));
    if ((rc = cnn_shape_ok(c, R, p->c_in, p->c_out, L)) != LTGW_OK) return rc;
    const int W = p->block;
    if (W < 1 || W > 64) return fail(c, LTGW_E_INVALID_ARG, "block must be in 1 .. 64");
    const int nbg = (2 * L + W - 1) / W;          // blocks per fine group
    const int64_t nb = g_f * nbg;                  // blocks per realisation
    const int K1 = (p->n_select + W - 1) / W, K2 = p->n_select2 > 0 ? (p->n_select2 + W - 1) / W : 0;
    if (nb > 8192 || p->n_select < 1 || p->n_select2 < 0 || K1 + K2 > nb)
        return fail(c, LTGW_E_INVALID_ARG, "need 1 <= n_select, 0 <= n_select2, blocks of both <= %lld <= 8192",
                    (long long)nb);
    if (!fin(p->psi_threshold) || !fin(p->coarse_threshold) || !fin(p->tier2_threshold))
        return fail(c, LTGW_E_INVALID_ARG, "thresholds must be finite");
    const int64_t nc = g_c * L, n_cells = (int64_t)p->c_out * L, nx = (int64_t)p->c_in * L;
    const int M1 = K1 * W, M2 = K2 * W;
    // the fused network pass keeps activations and logits on chip
    const bool fused = !net || (cnn_infer_supported(p->c_in, p->c_out, L) && (W == 16 || W == 32 || W == 64));
    struct {
        DevBuf *b;
        size_t bytes;
    } need[] = {{&S.psi_c, (size_t)(R * nc) * 8},       {&S.x, (size_t)(R * nx) * 4},
                {&S.cmap, net ? 0 : (size_t)g_f * 2 * 4},
                {&S.act, fused ? 0 : (size_t)R * 3 * 32 * L * 4},
                {&S.logits, fused ? 0 : (size_t)(R * n_cells) * 4},
                {&S.bscore, (size_t)(R * nb) * 4},       {&S.blk, (size_t)R * K1 * 4},
                {&S.tpl, (size_t)R * M1 * 4},            {&S.psi_sel, (size_t)R * M1 * 8},
                {&S.best_idx, (size_t)R * 4},            {&S.best_psi, (size_t)R * 8},
                {&S.cm_idx, (size_t)R * 4},              {&S.cm, (size_t)R * 8}};
    for (auto &n : need)
        if ((rc = ensure(c, *n.b, n.bytes, "proposer buffers")) != LTGW_OK) return rc;
    // Every step is queued on the stream; the host waits once, for the outputs.
    // 1. coarse map -> network -> block scores -> the K1 best blocks -> their exact fine ratios
    if ((rc = features_impl(c, coarse, with_counts, (float *)S.x.p, (double *)S.psi_c.p)) != LTGW_OK) return rc;
    // the network and the block scores: one fused pass where the shape allows it
    if (!net) {
        // the method alone: each block scored by its nearest coarse groups' power ratios
        if ((rc = h2d(c, S.cmap.p, p->coarse_map, (size_t)g_f * 2 * 4, "coarse map upload")) != LTGW_OK) return rc;
        HIP_TRY(c, launch_coarse_block_scores((const float *)S.x.p, R, (int)nb, p->c_in, L, W, nbg,
                                              (const int32_t *)S.cmap.p, (float *)S.bscore.p, c->stream),
                "coarse block score launch");
    } else if (fused) {
        if ((rc = ensure(c, c->cnn_packed, (size_t)cnn_infer_scratch_shorts(p->c_in) * 2, "packed weights")) !=
            LTGW_OK)
            return rc;
        HIP_TRY(c, launch_cnn_infer(p->params, (const float *)S.x.p, R, p->c_in, p->c_out, L,
                                    (short *)c->cnn_packed.p, nullptr, (float *)S.bscore.p, W, c->stream),
                "network forward");
    } else {
        HIP_TRY(c, launch_cnn_forward(p->params, (const float *)S.x.p, R, p->c_in, p->c_out, L, (float *)S.act.p,
                                      (float *)S.logits.p, c->stream),
                "network forward");
        HIP_TRY(c, launch_block_scores((const float *)S.logits.p, R, p->c_out, L, W, nbg, (float *)S.bscore.p,
                                       c->stream),
                "block score launch");
    }
    HIP_TRY(c, launch_select_top((const float *)S.bscore.p, R, (int)nb, K1, (int32_t *)S.blk.p, c->stream),
            "selection launch");
    SearchPlan P;
    if ((rc = stack_tables(c, fine, 0, P)) != LTGW_OK) return rc;
    int64_t sb = 0, sr = 0;
    const EvalArgs fa = stack_args(S, 0, fine, P, sb, sr);
    const StackMoments fm = level_moments(S, 0);
    // the templates of the chosen blocks and their exact ratios: in place for
    // blocks of 16, 32 or 64, else through an expanded list
    auto eval_blocks = [&](const int32_t *blk, int K, const int32_t *rmap, const int32_t *n_rows, int32_t *tpl,
                           double *psi) -> int {
        if (block_eval_supported(W)) {
            HIP_TRY(c, launch_block_eval(S.store, W, fa, R, sb, sr, blk, K, nbg, rmap, n_rows, fm, tpl, psi, c->stream),
                    "block evaluation launch");
            return LTGW_OK;
        }
        HIP_TRY(c, launch_expand_blocks(blk, K, W, 2 * L, nbg, rmap, n_rows, R, tpl, c->stream),
                "block expansion launch");
        HIP_TRY(c, launch_list_eval(S.store, fa, R, sb, sr, tpl, K * W, rmap, n_rows, fm, psi, c->stream),
                "listed evaluation launch");
        return LTGW_OK;
    };
    if ((rc = eval_blocks((const int32_t *)S.blk.p, K1, nullptr, nullptr, (int32_t *)S.tpl.p,
                          (double *)S.psi_sel.p)) != LTGW_OK)
        return rc;
    int32_t *best_i = (int32_t *)S.best_idx.p;
    double *best_p = (double *)S.best_psi.p;
    HIP_TRY(c, launch_row_best((const double *)S.psi_sel.p, R, M1, (const int32_t *)S.tpl.p, nullptr, best_i, best_p,
                               c->stream),
            "reduction launch");
    HIP_TRY(c, launch_row_best((const double *)S.psi_c.p, R, nc, nullptr, nullptr, (int32_t *)S.cm_idx.p,
                               (double *)S.cm.p, c->stream),
            "coarse maximum launch");
    const double thr = p->psi_threshold;
    const int64_t n_tpl = P.n_tpl;
    if ((int64_t)R * n_tpl > ((int64_t)1 << 31))
        return fail(c, LTGW_E_UNSUPPORTED, "fallback ratios of %d realisations x %lld templates too large", R,
                    (long long)n_tpl);
    struct {
        DevBuf *b;
        size_t bytes;
    } need2[] = {{&S.rmap, (size_t)R * 4}, {&S.fb, (size_t)R * 4},        {&S.bi2, (size_t)R * 4},
                 {&S.bp2, (size_t)R * 8},  {&S.counts, 2 * sizeof(int32_t)}, {&S.psi_all, (size_t)(R * n_tpl) * 8}};
    for (auto &n : need2)
        if ((rc = ensure(c, *n.b, n.bytes, "proposer buffers")) != LTGW_OK) return rc;
    int32_t *counts = (int32_t *)S.counts.p;
    // 2. realisations with no template above the threshold (listed on the device): the next K2 blocks
    if (K2 > 0) {
        struct {
            DevBuf *b;
            size_t bytes;
        } need3[] = {{&S.blk2, (size_t)R * K2 * 4}, {&S.tpl2, (size_t)R * M2 * 4}, {&S.psi2, (size_t)R * M2 * 8},
                     {&S.rows2, (size_t)R * 4},     {&S.flag2, (size_t)R * 4}};
        for (auto &n : need3)
            if ((rc = ensure(c, *n.b, n.bytes, "proposer buffers")) != LTGW_OK) return rc;
        const int32_t *rows2 = (const int32_t *)S.rows2.p;
        HIP_TRY(c, launch_take_rows(R, best_p, thr, (const double *)S.cm.p, p->tier2_threshold, (int32_t *)S.rows2.p,
                                    counts, (int32_t *)S.flag2.p, c->stream),
                "second-tier rows launch");
        HIP_TRY(c, launch_mask_blocks((float *)S.bscore.p, (const int32_t *)S.blk.p, R, K1, (int)nb, c->stream),
                "block mask launch");
        HIP_TRY(c, launch_select_top((const float *)S.bscore.p, R, (int)nb, K2, (int32_t *)S.blk2.p, c->stream),
                "selection launch");
        if ((rc = eval_blocks((const int32_t *)S.blk2.p, K2, rows2, counts, (int32_t *)S.tpl2.p,
                              (double *)S.psi2.p)) != LTGW_OK)
            return rc;
        HIP_TRY(c, launch_row_best((const double *)S.psi2.p, R, M2, (const int32_t *)S.tpl2.p, counts,
                                   (int32_t *)S.bi2.p, (double *)S.bp2.p, c->stream),
                "reduction launch");
        HIP_TRY(c, launch_merge_rows(R, rows2, counts, (const int32_t *)S.bi2.p, (const double *)S.bp2.p, best_i,
                                     best_p, c->stream),
                "merge launch");
    }
    // 3. the fallback rule: a loud coarse map and still no template above the
    // threshold -> the exhaustive fine search of those realisations (the same
    // sums as a list of every template)
    HIP_TRY(c, launch_take_rows(R, best_p, thr, (const double *)S.cm.p, p->coarse_threshold, (int32_t *)S.rmap.p,
                                counts + 1, (int32_t *)S.fb.p, c->stream),
            "fallback rows launch");
    HIP_TRY(c, launch_stack_eval(S.store, 0, fa, R, sb, sr, 1.0, 1.0, 0, (const int32_t *)S.rmap.p, counts + 1, fm,
                                 (double *)S.psi_all.p, c->stream),
            "fallback evaluation launch");
    HIP_TRY(c, launch_row_best((const double *)S.psi_all.p, R, n_tpl, nullptr, counts + 1, (int32_t *)S.bi2.p,
                               (double *)S.bp2.p, c->stream),
            "reduction launch");
    HIP_TRY(c, launch_merge_rows(R, (const int32_t *)S.rmap.p, counts + 1, (const int32_t *)S.bi2.p,
                                 (const double *)S.bp2.p, best_i, best_p, c->stream),
            "merge launch");
    const int KB = K1 + K2;
    if (p->blocks) {
        if ((rc = ensure(c, S.blocks, (size_t)R * KB * 4, "proposer buffers")) != LTGW_OK) return rc;
        HIP_TRY(c, launch_blocks_out(R, (const int32_t *)S.blk.p, K1, (const int32_t *)S.blk2.p, K2,
                                     (const int32_t *)S.flag2.p, (int32_t *)S.blocks.p, c->stream),
                "block output launch");
        HIP_TRY(c, hipMemcpyAsync(p->blocks, S.blocks.p, (size_t)R * KB * 4, hipMemcpyDeviceToHost, c->stream),
                "copy");
    }
    if ((rc = ensure(c, S.records, (size_t)R * sizeof(ProposeRecord), "proposer results")) != LTGW_OK) return rc;
    HIP_TRY(c, launch_pack_results(R, best_i, best_p, (const int32_t *)S.fb.p, (ProposeRecord *)S.records.p,
                                   c->stream),
            "result packing launch");
    std::vector<ProposeRecord> rec((size_t)R);
    HIP_TRY(c, hipMemcpyAsync(rec.data(), S.records.p, (size_t)R * sizeof(ProposeRecord), hipMemcpyDeviceToHost,
                              c->stream),
            "copy");
    HIP_TRY(c, hipStreamSynchronize(c->stream), "propose");
    for (int r = 0; r < R; ++r) {
        best_index[r] = rec[(size_t)r].idx;
        best_psi[r] = rec[(size_t)r].psi;
        fallback[r] = rec[(size_t)r].fallback;
    }
    return LTGW_OK;
}

}  // extern "C"
