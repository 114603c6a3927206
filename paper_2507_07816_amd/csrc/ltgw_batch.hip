// Many searches in one persistent, graph-captured launch (ltgw_eval_batch),
// per-search results, and the batch autotuner.  Contracts in include/ltgw.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "ltgw_ctx.h"

using namespace ltgw;

namespace ltgw {

void free_batch(BatchState &B) {
    if (B.exec) (void)hipGraphExecDestroy(B.exec);
    if (B.graph) (void)hipGraphDestroy(B.graph);
    if (B.cap_stream) (void)hipStreamDestroy(B.cap_stream);
    if (B.ev0) (void)hipEventDestroy(B.ev0);
    if (B.ev1) (void)hipEventDestroy(B.ev1);
    DevBuf *all[] = {&B.searches, &B.tiles, &B.ctr, &B.tiles_done, &B.t_done, &B.t_start,
                     &B.in_band, &B.s, &B.c, &B.n_res, &B.w1, &B.w2, &B.gtab, &B.dtab, &B.win,
                     &B.tau, &B.brake, &B.sky, &B.cand, &B.n_out, &B.diff, &B.pa, &B.ia,
                     &B.pb, &B.ib};
    for (DevBuf *b : all) release(*b);
    B = BatchState();
}

}  // namespace ltgw

namespace {


template <class T>
void put(std::vector<unsigned char> &v, const T &x) {
    const unsigned char *p = (const unsigned char *)&x;
    v.insert(v.end(), p, p + sizeof(T));
}
template <class T>
void put_array(std::vector<unsigned char> &v, const T *p, size_t n) {
    v.insert(v.end(), (const unsigned char *)p, (const unsigned char *)(p + n));
}

// Everything a captured batch graph depends on: the descriptors, the device
// buffers of the detectors it reads, and their weights (the moment mode and
// fixed-point weights are baked in at build time).
std::vector<unsigned char> signature(ltgw_ctx *c, const ltgw_search *S, int n, int k) {
    std::vector<unsigned char> v;
    put(v, n);
    put(v, k);
    for (int i = 0; i < n; ++i) {
        const ltgw_grid &g = S[i].grid;
        put(v, g.f0_min);
        put(v, g.f0_step);
        put(v, g.n_f0);
        put(v, g.n_tau);
        put(v, g.n_brake);
        put(v, g.n_sky);
        put(v, g.t0);
        if (g.tau) put_array(v, g.tau, (size_t)std::max(g.n_tau, 0));
        if (g.brake) put_array(v, g.brake, (size_t)std::max(g.n_brake, 0));
        if (g.sky) put_array(v, g.sky, 3 * (size_t)std::max(g.n_sky, 0));
        put(v, S[i].n_dets);
        for (int q = 0; q < S[i].n_dets && q < LTGW_MAX_SEARCH_DET; ++q) {
            const int d = S[i].dets[q];
            put(v, d);
            if (d < 0 || d >= LTGW_MAX_DET) continue;
            const Det &D = c->det[d];
            put(v, D.store_buf.p);
            put(v, D.wq.p);
            put(v, D.w.p);
            put(v, D.v.p);
            put(v, D.t_seg.p);
            put(v, D.n_seg);
            put(v, D.n_bins);
            put(v, D.k_lo);
            put(v, D.t_sft);
            put(v, D.rho_th);
            put(v, D.store);
            put(v, D.pitch);
            put(v, D.loaded);
            put(v, D.has_v);
            put(v, D.has_antenna);
            put_array(v, D.h_w.data(), D.h_w.size());
        }
    }
    return v;
}

int tpl_of(int variant) { return variant_templates_per_block(variant) / 256; }

// Tile list for a tile shape: searches largest first (segments per template);
// within a search, f0 tile by f0 tile, and for each the (tau, n) groups with
// their sky points innermost; a tile is one wavefront's 64 x TPL f0 of one
// (tau, n, sky) group.  The tracks of one f0 tile and (tau, n) differ across
// the sky points only by their Doppler shifts (a bin or two), and start at
// the same bins for every (tau, n): in this order the tiles in flight at any
// time read nearly the same lines, which the caches then serve.
int upload_tiles(ltgw_ctx *c, BatchState &B, int variant) {
    const int W = 64 * tpl_of(variant);
    std::vector<BatchTile> tiles;
    int64_t total = 0;
    for (int i = 0; i < B.n; ++i) total += ((B.plans[i].n_f0 + W - 1) / W) * B.plans[i].n_groups;
    if (total >= INT_MAX) return fail(c, LTGW_E_UNSUPPORTED, "batch of %lld tiles is too large", (long long)total);
    tiles.reserve((size_t)total);
    for (int oi = 0; oi < B.n; ++oi) {
        const int i = B.order[oi];
        const SearchPlan &P = B.plans[i];
        const int nt = (P.n_f0 + W - 1) / W;
        B.hsearch[i].n_tiles = (int32_t)(nt * P.n_groups);
        const int64_t n_sky = P.n_groups / P.n_tn;  // group = tn + n_tn * sky
        for (int t = 0; t < nt; ++t)
            for (int tn = 0; tn < P.n_tn; ++tn)
                for (int64_t sky = 0; sky < n_sky; ++sky)
                    tiles.push_back(BatchTile{i, (int32_t)(tn + P.n_tn * sky), t, 0});
    }
    B.n_tiles = (int)total;
    int rc;
    if ((rc = ensure(c, B.tiles, tiles.size() * sizeof(BatchTile), "batch tiles")) != LTGW_OK) return rc;
    if ((rc = ensure(c, B.searches, B.hsearch.size() * sizeof(BatchSearch), "batch searches")) != LTGW_OK) return rc;
    HIP_TRY(c, hipMemcpy(B.tiles.p, tiles.data(), tiles.size() * sizeof(BatchTile), hipMemcpyHostToDevice),
            "tile upload");
    HIP_TRY(c, hipMemcpy(B.searches.p, B.hsearch.data(), B.hsearch.size() * sizeof(BatchSearch),
                         hipMemcpyHostToDevice),
            "search upload");
    B.grid = (int)std::min<int64_t>((total + 3) / 4, (int64_t)c->cu_count *
                                               batch_blocks_per_cu(B.store, B.moments_in_loop, variant));
    if (B.grid < 1) B.grid = 1;
    return LTGW_OK;
}

// The whole batch sequence on stream st (eager or being captured).
int enqueue(ltgw_ctx *c, BatchState &B, hipStream_t st, int variant, bool with_topk, int tile_limit) {
    HIP_TRY(c, launch_fill_u32((unsigned *)B.ctr.p, 1, 0u, st), "batch reset");
    HIP_TRY(c, launch_fill_u32((unsigned *)B.tiles_done.p, B.n, 0u, st), "batch reset");
    HIP_TRY(c, launch_fill_u64((unsigned long long *)B.t_start.p, 1, ~0ull, st), "batch reset");
    HIP_TRY(c, launch_fill_u64((unsigned long long *)B.in_band.p, 1, 0ull, st), "batch reset");
    HIP_TRY(c, launch_fill_u64((unsigned long long *)B.t_done.p, B.n, 0ull, st), "batch reset");
    for (int i = 0; i < B.n; ++i) {
        const SearchPlan &P = B.plans[i];
        for (int q = 0; q < P.n_sel; ++q) {
            const Det &D = c->det[P.sel[q]];
            const DetView &V = B.hsearch[i].det[q];
            HIP_TRY(c, launch_spin_factor((const double *)D.t_seg.p, D.n_seg, B.t0[i],
                                          (const double *)B.tau.p + B.tau_off[i], P.n_tau,
                                          (const double *)B.brake.p + B.brake_off[i], P.n_brake,
                                          (double *)V.g, (unsigned long long *)c->counters.p + kCntUndecided, st),
                    "batch spin-factor launch");
            HIP_TRY(c, launch_doppler((const double *)D.v.p, D.n_seg, (const double *)B.sky.p + B.sky_off[i],
                                      P.n_sky, (double *)V.D, st),
                    "batch Doppler launch");
            HIP_TRY(c, launch_windows(V, (int)P.n_groups, P.n_tn, B.hsearch[i].f0_min, B.hsearch[i].f0_step, P.n_f0,
                                      (int2 *)V.win, st),
                    "batch window launch");
        }
    }
    if (!B.moments_in_loop)
        for (int i = 0; i < B.n; ++i)
            HIP_TRY(c, launch_moments(B.args[i], B.mom[i].mode, B.e0, (int64_t *)B.diff.p, st),
                    "batch moments launch");
    BatchArgs ba;
    ba.searches = (const BatchSearch *)B.searches.p;
    ba.tiles = (const BatchTile *)B.tiles.p;
    ba.n_tiles = std::min(B.n_tiles, tile_limit);
    ba.counter = (unsigned *)B.ctr.p;
    ba.t_start = (unsigned long long *)B.t_start.p;
    ba.in_band_total = (unsigned long long *)B.in_band.p;
    const int grid = std::min(B.grid, std::max((ba.n_tiles + 3) / 4, 1));  // 4 waves per workgroup
    if (!with_topk) HIP_TRY(c, hipEventRecord(B.ev0, st), "event record");
    HIP_TRY(c, launch_batch(B.store, B.moments_in_loop, variant, ba, grid, st), "batch launch");
    if (!with_topk) HIP_TRY(c, hipEventRecord(B.ev1, st), "event record");
    if (with_topk) {
        for (int i = 0; i < B.n; ++i) {
            const int64_t o = B.tpl_off[i];
            const double q = std::exp(-(double)B.plans[i].rho_th);
            for (int st_i = 0; st_i < 2; ++st_i) {
                const uint32_t stat = st_i == 0 ? LTGW_STAT_POWER : LTGW_STAT_COUNT;
                HIP_TRY(c, launch_topk(stat, B.plans[i].n_tpl, (const double *)B.s.p + o,
                                       (const int32_t *)B.c.p + o, (const int32_t *)B.n_res.p + o,
                                       (const double *)B.w1.p + o, (const double *)B.w2.p + o, q, B.k,
                                       (double *)B.pa.p, (int64_t *)B.ia.p, (double *)B.pb.p,
                                       (int64_t *)B.ib.p, B.topk_cap, B.dec[i],
                                       (ltgw_candidate *)B.cand.p + ((int64_t)i * 2 + st_i) * B.k,
                                       (int32_t *)B.n_out.p + i * 2 + st_i, st),
                        "batch top-k launch");
            }
        }
    }
    return LTGW_OK;
}

int build(ltgw_ctx *c, const ltgw_search *S, int n, int k) {
    free_batch(c->batch);
    BatchState &B = c->batch;
    B.n = n;
    B.k = k;
    B.plans.resize(n);
    int rc;
    std::vector<int> all_slots;
    for (int i = 0; i < n; ++i) {
        if (S[i].n_dets < 1 || S[i].n_dets > LTGW_MAX_SEARCH_DET)
            return fail(c, LTGW_E_INVALID_ARG, "search %d: n_dets must be 1..%d", i, LTGW_MAX_SEARCH_DET);
        if ((rc = plan_search(c, &S[i].grid, S[i].dets, S[i].n_dets, B.plans[i])) != LTGW_OK) {
            const std::string e = c->err;
            return fail(c, rc, "search %d: %s", i, e.c_str());
        }
        if (B.plans[i].store != B.plans[0].store)
            return fail(c, LTGW_E_UNSUPPORTED, "searches of one batch must use one store format");
        for (int q = 0; q < S[i].n_dets; ++q)
            if (c->det[S[i].dets[q]].has_antenna)
                return fail(c, LTGW_E_UNSUPPORTED, "search %d: detector %d has antenna-pattern weights, which "
                            "a batch does not take", i, S[i].dets[q]);
        for (int q = 0; q < S[i].n_dets; ++q)
            if (std::find(all_slots.begin(), all_slots.end(), S[i].dets[q]) == all_slots.end())
                all_slots.push_back(S[i].dets[q]);
    }
    B.store = B.plans[0].store;
    // moments: one fixed-point exponent over every slot of the batch
    const Moments Mg = plan_moments(c, all_slots.data(), (int)all_slots.size());
    B.moments_in_loop = Mg.mode == 2;
    B.e0 = Mg.e0;
    B.mom.resize(n);
    for (int i = 0; i < n; ++i) {
        const SearchPlan &P = B.plans[i];
        Moments M;
        M.w_uniform = c->det[P.sel[0]].w_uniform;
        bool uniform = true;
        for (int q = 0; q < P.n_sel; ++q) {
            const Det &D = c->det[P.sel[q]];
            uniform &= !D.weighted && D.w_uniform == M.w_uniform;
        }
        M.mode = B.moments_in_loop ? 2 : (uniform ? 0 : 1);
        M.e0 = B.e0;
        B.mom[i] = M;
    }
    // sizes and offsets
    B.tpl_off.resize(n);
    B.t0.resize(n);
    B.tau_off.resize(n);
    B.brake_off.resize(n);
    B.sky_off.resize(n);
    B.g_off.assign((size_t)n * LTGW_MAX_SEARCH_DET, 0);
    B.d_off.assign((size_t)n * LTGW_MAX_SEARCH_DET, 0);
    B.win_off.assign((size_t)n * LTGW_MAX_SEARCH_DET, 0);
    int64_t tpl = 0, gtot = 0, dtot = 0, wtot = 0, ntau = 0, nbrake = 0, nsky = 0, diff_max = 0, topk_max = 0;
    std::vector<double> htau, hbrake, hsky;
    for (int i = 0; i < n; ++i) {
        const SearchPlan &P = B.plans[i];
        const ltgw_grid &g = S[i].grid;
        B.tpl_off[i] = tpl;
        tpl += P.n_tpl;
        B.evals += P.n_evals;
        B.t0[i] = g.t0;
        B.tau_off[i] = ntau;
        B.brake_off[i] = nbrake;
        B.sky_off[i] = nsky;
        htau.insert(htau.end(), g.tau, g.tau + g.n_tau);
        hbrake.insert(hbrake.end(), g.brake, g.brake + g.n_brake);
        hsky.insert(hsky.end(), g.sky, g.sky + 3 * (size_t)g.n_sky);
        ntau += g.n_tau;
        nbrake += g.n_brake;
        nsky += 3 * (int64_t)g.n_sky;
        for (int q = 0; q < P.n_sel; ++q) {
            const Det &D = c->det[P.sel[q]];
            B.g_off[(size_t)i * LTGW_MAX_SEARCH_DET + q] = gtot;
            B.d_off[(size_t)i * LTGW_MAX_SEARCH_DET + q] = dtot;
            B.win_off[(size_t)i * LTGW_MAX_SEARCH_DET + q] = wtot;
            gtot += (int64_t)P.n_tn * D.n_seg;
            dtot += (int64_t)P.n_sky * D.n_seg;
            wtot += P.n_groups * (int64_t)((P.n_f0 + 63) / 64);
        }
        diff_max = std::max(diff_max, (int64_t)(B.mom[i].mode ? 4 : 1) * P.n_groups * (P.n_f0 + 1));
        topk_max = std::max(topk_max, topk_scratch_entries(P.n_tpl, k));
    }
    B.templates = tpl;
    B.topk_cap = topk_max;
    B.diff_entries = B.moments_in_loop ? 0 : diff_max;
    struct {
        DevBuf *b;
        size_t bytes;
        const char *what;
    } allocs[] = {
        {&B.s, (size_t)tpl * 8, "batch s"},          {&B.c, (size_t)tpl * 4, "batch c"},
        {&B.n_res, (size_t)tpl * 4, "batch N"},      {&B.w1, (size_t)tpl * 8, "batch W1"},
        {&B.w2, (size_t)tpl * 8, "batch W2"},        {&B.gtab, (size_t)gtot * 8, "batch spin-factor tables"},
        {&B.dtab, (size_t)dtot * 8, "batch Doppler tables"},
        {&B.win, (size_t)wtot * sizeof(int2), "batch segment windows"},
        {&B.tau, (size_t)ntau * 8, "batch tau"},     {&B.brake, (size_t)nbrake * 8, "batch brake"},
        {&B.sky, (size_t)nsky * 8, "batch sky"},
        {&B.cand, (size_t)n * 2 * k * sizeof(ltgw_candidate), "batch candidates"},
        {&B.n_out, (size_t)n * 2 * 4, "batch candidate counts"},
        {&B.ctr, 8, "batch counter"},                {&B.tiles_done, (size_t)n * 4, "batch tile counts"},
        {&B.t_done, (size_t)n * 8, "batch times"},   {&B.t_start, 8, "batch time"},
        {&B.in_band, 8, "batch in-band count"},      {&B.diff, (size_t)B.diff_entries * 8, "batch moments"},
        {&B.pa, (size_t)topk_max * 8, "batch top-k"}, {&B.ia, (size_t)topk_max * 8, "batch top-k"},
        {&B.pb, (size_t)topk_max * 8, "batch top-k"}, {&B.ib, (size_t)topk_max * 8, "batch top-k"},
    };
    for (auto &a : allocs)
        if ((rc = ensure(c, *a.b, a.bytes, a.what)) != LTGW_OK) return rc;
    HIP_TRY(c, hipMemcpy(B.tau.p, htau.data(), htau.size() * 8, hipMemcpyHostToDevice), "batch upload");
    HIP_TRY(c, hipMemcpy(B.brake.p, hbrake.data(), hbrake.size() * 8, hipMemcpyHostToDevice), "batch upload");
    HIP_TRY(c, hipMemcpy(B.sky.p, hsky.data(), hsky.size() * 8, hipMemcpyHostToDevice), "batch upload");
    if (Mg.mode == 1)
        for (int d : all_slots) {
            Det &D = c->det[d];
            if ((rc = ensure(c, D.wfix, D.h_wfix.size() * 8, "fixed-point weights")) != LTGW_OK) return rc;
            HIP_TRY(c, hipMemcpy(D.wfix.p, D.h_wfix.data(), D.h_wfix.size() * 8, hipMemcpyHostToDevice),
                    "weights upload");
        }
    // descriptors
    B.hsearch.assign(n, BatchSearch());
    B.args.assign(n, EvalArgs());
    B.dec.resize(n);
    for (int i = 0; i < n; ++i) {
        const SearchPlan &P = B.plans[i];
        const ltgw_grid &g = S[i].grid;
        BatchSearch &H = B.hsearch[i];
        std::memset(&H, 0, sizeof H);
        EvalArgs &a = B.args[i];
        std::memset(&a, 0, sizeof a);
        for (int q = 0; q < P.n_sel; ++q) {
            const Det &D = c->det[P.sel[q]];
            DetView V;
            std::memset(&V, 0, sizeof V);
            V.store = D.store_buf.p;
            V.pitch_bytes = (int32_t)(D.pitch * (D.store == LTGW_STORE_F32 ? 4 : D.store == LTGW_STORE_BF16 ? 2 : 1));
            V.H = nullptr;
            V.g = (const double *)B.gtab.p + B.g_off[(size_t)i * LTGW_MAX_SEARCH_DET + q];
            V.D = (const double *)B.dtab.p + B.d_off[(size_t)i * LTGW_MAX_SEARCH_DET + q];
            V.t_sft = D.t_sft;
            V.wq = (const float *)D.wq.p;
            V.w = (const float *)D.w.p;
            V.wfix = Mg.mode == 1 ? (const int64_t *)D.wfix.p : nullptr;
            V.cshift = 1.5 - (double)D.k_lo;
            V.n_seg = D.n_seg;
            V.n_bins = D.n_bins;
            V.win = (const int2 *)B.win.p + B.win_off[(size_t)i * LTGW_MAX_SEARCH_DET + q];
            V.win_run = 64;
            V.win_blocks = (P.n_f0 + 63) / 64;
            H.det[q] = V;
            a.det[q] = V;
        }
        const int64_t o = B.tpl_off[i];
        H.n_det = P.n_sel;
        H.n_f0 = P.n_f0;
        H.n_tn = P.n_tn;
        H.f0_min = g.f0_min;
        H.f0_step = g.f0_step;
        H.s = (double *)B.s.p + o;
        H.c = (int32_t *)B.c.p + o;
        H.n = (int32_t *)B.n_res.p + o;
        H.w1 = (double *)B.w1.p + o;
        H.w2 = (double *)B.w2.p + o;
        H.tiles_done = (unsigned *)B.tiles_done.p + i;
        H.t_done = (unsigned long long *)B.t_done.p + i;
        a.n_det = P.n_sel;
        a.n_f0 = P.n_f0;
        a.n_groups = (int32_t)P.n_groups;
        a.n_tn = P.n_tn;
        a.f0_min = g.f0_min;
        a.f0_step = g.f0_step;
        a.w_uniform = B.mom[i].w_uniform;
        a.s = H.s;
        a.c = H.c;
        a.n = H.n;
        a.w1 = H.w1;
        a.w2 = H.w2;
        a.in_band_total = (unsigned long long *)B.in_band.p;
        TopkDecode &dc = B.dec[i];
        dc.f0_min = g.f0_min;
        dc.f0_step = g.f0_step;
        dc.n_f0 = P.n_f0;
        dc.n_tau = P.n_tau;
        dc.n_brake = P.n_brake;
        dc.tau = (const double *)B.tau.p + B.tau_off[i];
        dc.brake = (const double *)B.brake.p + B.brake_off[i];
    }
    // largest search first (segments per template, then templates)
    B.order.resize(n);
    std::iota(B.order.begin(), B.order.end(), 0);
    std::stable_sort(B.order.begin(), B.order.end(), [&](int x, int y) {
        if (B.plans[x].n_seg_total != B.plans[y].n_seg_total) return B.plans[x].n_seg_total > B.plans[y].n_seg_total;
        return B.plans[x].n_tpl > B.plans[y].n_tpl;
    });
    HIP_TRY(c, hipEventCreate(&B.ev0), "event create");
    HIP_TRY(c, hipEventCreate(&B.ev1), "event create");
    HIP_TRY(c, hipStreamCreateWithFlags(&B.cap_stream, hipStreamNonBlocking), "capture stream");
    // tile shape: from the tuning cache, else time each shape on a leading
    // part of the batch (the same templates for every shape) and keep the fastest
    const std::string key = tune_key_batch(B.store, B.moments_in_loop, n, B.evals);
    const auto it = c->tune.find(key);
    int variant = 1;
    if (c->forced_variant >= 0) {
        variant = c->forced_variant & 3;  // the persistent launch is one generation already
    } else if (it != c->tune.end()) {
        variant = it->second & 3;
    } else {
        float best = 0.0f;
        int best_v = -1;
        int64_t tiles1 = 0;  // tiles of the one-template-per-lane shapes
        for (int i = 0; i < n; ++i) tiles1 += ((B.plans[i].n_f0 + 63) / 64) * B.plans[i].n_groups;
        const int64_t lead = std::min<int64_t>(tiles1, std::max<int64_t>((int64_t)c->cu_count * 64, tiles1 / 10));
        for (int v = 0; v < kNumShapes; ++v) {
            if ((rc = upload_tiles(c, B, v)) != LTGW_OK) return rc;
            // the first lead/TPL tiles cover (nearly) the same templates for every shape
            const int lim = (int)std::max<int64_t>(1, lead / tpl_of(v));
            if ((rc = enqueue(c, B, c->stream, v, false, lim)) != LTGW_OK) return rc;
            HIP_TRY(c, hipEventSynchronize(B.ev1), "batch tuning");
            float ms = 0.0f;
            HIP_TRY(c, hipEventElapsedTime(&ms, B.ev0, B.ev1), "batch tuning");
            if (best_v < 0 || ms < best) {
                best = ms;
                best_v = v;
            }
        }
        variant = best_v;
        c->tune[key] = variant;
    }
    B.variant = variant;
    if ((rc = upload_tiles(c, B, variant)) != LTGW_OK) return rc;
    HIP_TRY(c, hipDeviceSynchronize(), "batch build");
    // capture the whole sequence
    HIP_TRY(c, hipStreamBeginCapture(B.cap_stream, hipStreamCaptureModeThreadLocal), "begin capture");
    rc = enqueue(c, B, B.cap_stream, variant, true, INT_MAX);
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(B.cap_stream, &graph);
    if (rc != LTGW_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (ec != hipSuccess) return hip_fail(c, ec, "end capture");
    B.graph = graph;
    HIP_TRY(c, hipGraphInstantiate(&B.exec, B.graph, nullptr, nullptr, 0), "graph instantiate");
    B.sig = signature(c, S, n, k);
    B.latency_ms.assign(n, 0.0);
    B.valid = true;
    return LTGW_OK;
}

}  // namespace

extern "C" {

int32_t ltgw_eval_batch(ltgw_ctx *c, const ltgw_search *S, int32_t n, int32_t k,
                        ltgw_candidate *top_power, ltgw_candidate *top_count, int32_t *n_power,
                        int32_t *n_count, ltgw_batch_stats *stats) {
    if (!c) return LTGW_E_INVALID_ARG;
    Enter en(c);
    if (!S || n < 1) return fail(c, LTGW_E_INVALID_ARG, "need at least one search");
    if (k < 1 || k > LTGW_MAX_TOPK) return fail(c, LTGW_E_INVALID_ARG, "k must be in 1..%d", LTGW_MAX_TOPK);
    if (!top_power || !top_count || !n_power || !n_count)
        return fail(c, LTGW_E_INVALID_ARG, "output pointers are NULL");
    for (int i = 0; i < n; ++i)
        if (S[i].n_dets < 1 || S[i].n_dets > LTGW_MAX_SEARCH_DET)
            return fail(c, LTGW_E_INVALID_ARG, "search %d: n_dets must be 1..%d", i, LTGW_MAX_SEARCH_DET);
    BatchState &B = c->batch;
    bool replay = B.valid && B.sig == signature(c, S, n, k);
    if (!replay) {
        const int rc = build(c, S, n, k);
        if (rc != LTGW_OK) {
            const std::string e = c->err;
            free_batch(c->batch);
            return fail(c, rc, "%s", e.c_str());
        }
    }
    HIP_TRY(c, hipEventRecord(B.ev0, c->stream), "event record");
    HIP_TRY(c, hipGraphLaunch(B.exec, c->stream), "graph launch");
    HIP_TRY(c, hipEventRecord(B.ev1, c->stream), "event record");
    std::vector<ltgw_candidate> cand((size_t)n * 2 * k);
    std::vector<int32_t> cnt((size_t)n * 2);
    std::vector<unsigned long long> tdone(n);
    unsigned long long tstart = 0, inb = 0;
    HIP_TRY(c, hipMemcpyAsync(cand.data(), B.cand.p, cand.size() * sizeof(ltgw_candidate), hipMemcpyDeviceToHost, c->stream), "batch download");
    HIP_TRY(c, hipMemcpyAsync(cnt.data(), B.n_out.p, cnt.size() * 4, hipMemcpyDeviceToHost, c->stream), "batch download");
    HIP_TRY(c, hipMemcpyAsync(tdone.data(), B.t_done.p, (size_t)n * 8, hipMemcpyDeviceToHost, c->stream), "batch download");
    HIP_TRY(c, hipMemcpyAsync(&tstart, B.t_start.p, 8, hipMemcpyDeviceToHost, c->stream), "batch download");
    HIP_TRY(c, hipMemcpyAsync(&inb, B.in_band.p, 8, hipMemcpyDeviceToHost, c->stream), "batch download");
    HIP_TRY(c, hipStreamSynchronize(c->stream), "batch");
    unsigned long long tend = 0;
    for (int i = 0; i < n; ++i) {
        std::memcpy(top_power + (size_t)i * k, &cand[((size_t)i * 2 + 0) * k], (size_t)k * sizeof(ltgw_candidate));
        std::memcpy(top_count + (size_t)i * k, &cand[((size_t)i * 2 + 1) * k], (size_t)k * sizeof(ltgw_candidate));
        n_power[i] = cnt[(size_t)i * 2 + 0];
        n_count[i] = cnt[(size_t)i * 2 + 1];
        B.latency_ms[i] = tdone[i] >= tstart ? (double)(tdone[i] - tstart) / (double)c->wall_khz : 0.0;
        tend = std::max(tend, tdone[i]);
    }
    if (stats) {
        float total = 0.0f;
        (void)hipEventElapsedTime(&total, B.ev0, B.ev1);
        stats->graph_replayed = replay ? 1 : 0;
        stats->variant = B.variant;
        stats->templates_per_lane = tpl_of(B.variant);
        stats->segments_per_batch = B.variant % 2 ? 16 : 8;
        stats->workgroups = B.grid;
        stats->tiles = B.n_tiles;
        stats->templates = B.templates;
        stats->evals = B.evals;
        stats->in_band = (int64_t)inb;
        stats->kernel_ms = tend >= tstart ? (double)(tend - tstart) / (double)c->wall_khz : 0.0;
        stats->total_ms = total;
    }
    return LTGW_OK;
}

int32_t ltgw_batch_results(ltgw_ctx *c, int32_t i, float *out_s, int32_t *out_c, int32_t *out_n,
                           double *psi_power, double *psi_count) {
    if (!c) return LTGW_E_INVALID_ARG;
    Enter en(c);
    BatchState &B = c->batch;
    if (!B.valid) return fail(c, LTGW_E_STATE, "no batch evaluated");
    if (i < 0 || i >= B.n) return fail(c, LTGW_E_INVALID_ARG, "search %d out of range", i);
    const int64_t o = B.tpl_off[i], m = B.plans[i].n_tpl;
    if (out_s) HIP_TRY(c, launch_f64_to_f32((const double *)B.s.p + o, out_s, m, c->stream), "convert");
    if (out_c) HIP_TRY(c, hipMemcpyAsync(out_c, (const int32_t *)B.c.p + o, m * 4, hipMemcpyDeviceToDevice, c->stream), "copy");
    if (out_n) HIP_TRY(c, hipMemcpyAsync(out_n, (const int32_t *)B.n_res.p + o, m * 4, hipMemcpyDeviceToDevice, c->stream), "copy");
    const double q = std::exp(-(double)B.plans[i].rho_th);
    if (psi_power)
        HIP_TRY(c, launch_psi(LTGW_STAT_POWER, m, (const double *)B.s.p + o, (const int32_t *)B.c.p + o,
                              (const int32_t *)B.n_res.p + o, (const double *)B.w1.p + o,
                              (const double *)B.w2.p + o, q, psi_power, c->stream),
                "psi");
    if (psi_count)
        HIP_TRY(c, launch_psi(LTGW_STAT_COUNT, m, (const double *)B.s.p + o, (const int32_t *)B.c.p + o,
                              (const int32_t *)B.n_res.p + o, (const double *)B.w1.p + o,
                              (const double *)B.w2.p + o, q, psi_count, c->stream),
                "psi");
    return LTGW_OK;
}

int32_t ltgw_batch_latency(ltgw_ctx *c, double *out_ms) {
    if (!c) return LTGW_E_INVALID_ARG;
    Enter en(c);
    BatchState &B = c->batch;
    if (!B.valid) return fail(c, LTGW_E_STATE, "no batch evaluated");
    if (!out_ms) return fail(c, LTGW_E_INVALID_ARG, "out_ms is NULL");
    std::memcpy(out_ms, B.latency_ms.data(), (size_t)B.n * sizeof(double));
    return LTGW_OK;
}

}  // extern "C"
