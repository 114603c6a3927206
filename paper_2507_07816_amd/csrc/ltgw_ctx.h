// Context state and host helpers shared by the C-ABI translation units
// (ltgw_api.hip, ltgw_batch.hip).  Not part of the public boundary.
#pragma once
#include <hip/hip_runtime.h>

#include <functional>
#include <map>
#include <string>
#include <vector>

#include "ltgw_internal.h"

namespace ltgw {

struct DevBuf {
    void *p = nullptr;
    size_t cap = 0;
};

struct Det {
    bool loaded = false, has_v = false;
    int32_t n_seg = 0, n_bins = 0, store = 0;
    int64_t k_lo = 0, pitch = 0;
    double t_sft = 0.0;
    float rho_th = 1.6f;
    bool weighted = false;        // weights not all equal
    float w_uniform = 1.0f;       // the weight when they are
    double v_max = 0.0;           // max |v| / c
    std::vector<float> h_w;       // weights as loaded
    std::vector<double> h_t;      // segment times as loaded
    std::vector<double> h_v;      // velocity table as set
    std::vector<int64_t> h_wfix;  // [n_seg][3] fixed-point w, w^2 high, w^2 low
    bool has_antenna = false;     // weights times the antenna response (ltgw_set_antenna)
    double arms[6] = {0, 0, 0, 0, 0, 0};
    DevBuf store_buf, t_seg, w, wq, scale, v, g, H, wfix, win, era, w_sky, wq_sky;
    // shape of the Eq. 1 and Eq. 2 tables in g and H as the last single-search
    // eval left them ([tab_n_tn][n_seg] and [tab_n_groups][n_seg]; 0: none)
    int32_t tab_n_tn = 0, tab_n_groups = 0;
};

// How the in-band moments W1, W2 are formed for a set of detectors.
struct Moments {
    int mode = 0;            // 0 uniform weights, 1 exact fixed point, 2 in the statistic kernel
    int e0 = 0;              // fixed point: w = wfix * 2^e0
    float w_uniform = 1.0f;  // mode 0
};

// A validated search: grid plus detector slots.
struct SearchPlan {
    int sel[LTGW_MAX_SEARCH_DET] = {0, 0, 0, 0};
    int n_sel = 0;
    int store = 0;
    float rho_th = 1.6f;
    int32_t n_f0 = 0, n_tau = 0, n_brake = 0, n_sky = 0, n_tn = 0;
    int64_t n_groups = 0, n_tpl = 0, n_evals = 0, n_seg_total = 0;
    int32_t max_bins = 0;
};

struct BatchState {
    bool valid = false;
    std::vector<unsigned char> sig;  // everything a captured graph depends on
    int n = 0, k = 0, store = 0, variant = 0, grid = 0, n_tiles = 0;
    bool moments_in_loop = false;
    int64_t templates = 0, evals = 0;
    std::vector<SearchPlan> plans;
    std::vector<Moments> mom;
    int e0 = 0;                           // shared fixed-point exponent of the weights
    std::vector<double> t0;               // T0 of each search
    std::vector<int64_t> tau_off, brake_off, sky_off;
    std::vector<double> latency_ms;       // per search, last launch
    std::vector<int32_t> order;           // searches, largest first
    std::vector<int64_t> tpl_off;         // first template of each search in the result arrays
    std::vector<EvalArgs> args;           // per search, for moments and ranking
    std::vector<TopkDecode> dec;
    std::vector<BatchSearch> hsearch;     // host copy of the device descriptors
    std::vector<int64_t> g_off, d_off;    // per (search, det) offsets into the g and D tables
    DevBuf searches, tiles, ctr, tiles_done, t_done, t_start, in_band;
    DevBuf s, c, n_res, w1, w2, gtab, dtab, tau, brake, sky, cand, n_out, diff, win;
    std::vector<int64_t> win_off;         // per (search, det) offsets into the window table
    DevBuf pa, ia, pb, ib;
    int64_t topk_cap = 0, diff_entries = 0;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
};

// Grid axes and track-factor tables of one level of a stack.
struct StackLevel {
    std::vector<double> h_tau, h_brake, h_sky;  // host copies of the last upload
    double t0 = 0.0;
    bool tables = false;                        // g and H hold the last upload's tables
    DevBuf tau, brake, sky, g, H;
    // per-template moments (W1, W2, N) of the level's weights on the lattice
    // (m_f0_min, m_f0_step, m_n_f0) of the current tables
    bool mom = false;
    double m_f0_min = 0.0, m_f0_step = 0.0;
    int m_n_f0 = 0;
    DevBuf mw1, mw2, mn;
};

// A stack of realisations sharing one detector slot's geometry (the learned
// proposer's data): fine store [R][n_seg][pitch], coarse BF16 store
// [R][n_seg / 2][pitch2], weights replicated per realisation.
struct StackState {
    bool valid = false, coarse = false;
    int det = 0, R = 0, store = 0, n_seg = 0, n_bins = 0;
    int S = 2;                    // segments per coarse row
    int64_t k_lo = 0, pitch = 0, pitch2 = 0;
    double t_sft = 0.0;
    DevBuf fine, crs, w, wq, scale, w2, t, v, t2, v2, params;
    StackLevel lv[2];
    hipEvent_t ev_h2d = nullptr;  // after the last grid upload
    DevBuf psi_c, x, act, logits, cells, tpl, psi_sel, best_idx, best_psi, fb, rmap, psi_all;
    DevBuf bscore, blk, blk2, tpl2, psi2, cm_idx, cm, cmap;
    // per-realisation step lists of a proposal: rows and flags of the second
    // tier and of the fallback, their counts, the later bests, the block output
    DevBuf rows2, flag2, bi2, bp2, counts, blocks, records;
};

}  // namespace ltgw

struct ltgw_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    ltgw::Det det[LTGW_MAX_DET];
    ltgw::DevBuf staging, counters;
    ltgw::DevBuf cnn_packed;  // BF16 weights of the fused inference pass
    ltgw::DevBuf tau_d, brake_d, sky_d;
    ltgw::DevBuf res_s, res_c, res_n, res_w1, res_w2, diff;
    ltgw::DevBuf cand_pa, cand_ia, cand_pb, cand_ib, cand_out, n_out;
    std::vector<double> h_tau, h_brake, h_sky;
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};  // tables start, eval start, eval end
    hipEvent_t ev_h2d = nullptr;  // after the grid uploads from h_tau/h_brake/h_sky
    hipEvent_t ev_ing[2] = {nullptr, nullptr};  // around the last load's store kernels
    bool have_ingest = false;
    // second stream (default priority): the in-band moments run there beside the
    // statistic kernel; ev_fork orders them after the tables, ev_join before
    // anything on `stream` that reads them
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    int cu_count = 256;
    int wall_khz = 100000;        // device wall-clock rate
    // autotuner cache: key -> tile shape (transparent comparison: looked up
    // by a character buffer without building a string)
    std::map<std::string, int, std::less<>> tune;
    // last single-search eval; results_kept: its per-template results are in
    // res_* for ltgw_psi and ltgw_topk_candidates
    bool have_eval = false, results_kept = false;
    int64_t n_templates = 0, n_evals = 0;
    double f0_min = 0.0, f0_step = 0.0;
    int32_t n_f0 = 0, n_tau = 0, n_brake = 0, n_sky = 0;
    float rho_th = 1.6f;
    int last_variant = 1;
    int last_launches = 0;  // statistic-kernel dispatches of the last eval
    bool list_mode = false;      // the last eval was an explicit template list
    ltgw::DevBuf h_list, h_perm;  // pinned host staging of its templates and of their evaluation order
    ltgw::DevBuf list_d, perm_d;
    ltgw::DevBuf list_dop, list_sky;    // Doppler tables of a one-sky list, and that sky
    // data preparation (ltgw_sft_normalise): spectra of a chunk, FFT plans
    struct SftPlan {
        int n_fft, batch;
        void *plan;  // hipfftHandle
    };
    ltgw::DevBuf sft_spec, sft_spec2;  // spectra of alternate chunks
    // data preparation across chunks: [0..1] transform of the chunk in buffer
    // b done, [2..3] its normalisation done (the normalisation runs on `side`)
    hipEvent_t ev_sft[4] = {nullptr, nullptr, nullptr, nullptr};
    std::vector<SftPlan> sft_plans;
    int forced_variant = -1;      // ltgw_set_tile_shape; -1 = autotuner
    // device address of this device's static scratch array (the no-allocation
    // entry point), resolved by ltgw_create; NULL when the device has none
    void *scratch = nullptr;
    ltgw::BatchState batch;
    ltgw::StackState stack;
};

namespace ltgw {

int fail(ltgw_ctx *c, int code, const char *fmt, ...);
int hip_fail(ltgw_ctx *c, hipError_t e, const char *what);
int ensure(ltgw_ctx *c, DevBuf &b, size_t bytes, const char *what);
void release(DevBuf &b);
// pinned host staging, grown like ensure()
int ensure_pinned(ltgw_ctx *c, DevBuf &b, size_t bytes, const char *what);
void release_pinned(DevBuf &b);
bool is_device_ptr(const void *p);
void sft_release(ltgw_ctx *c);  // FFT plans and buffers of the data preparation
int to_host(ltgw_ctx *c, void *dst, const void *src, size_t n, const char *what);
int h2d(ltgw_ctx *c, void *dst, const void *src, size_t n, const char *what);
bool fin(double x);

// Context counters: [0] powers the double-double phase could not decide,
// [1] powers that took the double-double phase (the kernels of Eq. 1 get
// &counters[0] and count both), [2] bad power values, [3] in-band total.
constexpr int kCntUndecided = 0, kCntSlow = 1, kCntBad = 2, kCntInBand = 3, kCntExact = 4, kNumCnt = 5;
int zero_counter(ltgw_ctx *c, int first, int n);
int read_counter(ltgw_ctx *c, int i, unsigned long long *out);

// Sets the context's device and clears its error for the duration of a call.
struct Enter {
    explicit Enter(ltgw_ctx *c) {
        if (c) {
            c->err.clear();
            (void)hipSetDevice(c->device);
        }
    }
};

// Validate a grid and its detector slots (grid->det_mask is not used here).
int plan_search(ltgw_ctx *c, const ltgw_grid *g, const int *slots, int n_slots, SearchPlan &P);
// Choose the moment mode for a set of slots; fixed point fills Det::h_wfix.
Moments plan_moments(ltgw_ctx *c, const int *slots, int n_slots);
// Autotuner keys.
std::string tune_key_eval(const SearchPlan &P, bool moments_in_loop);
void tune_key_eval(const SearchPlan &P, bool moments_in_loop, char (&buf)[160]);
std::string tune_key_batch(int store, bool moments_in_loop, int n_searches, int64_t evals);
void free_batch(BatchState &B);
void free_stack(StackState &S);

}  // namespace ltgw

#define HIP_TRY(ctx, expr, what)                                         \
    do {                                                                 \
        hipError_t e_ = (expr);                                          \
        if (e_ != hipSuccess) return ::ltgw::hip_fail(ctx, e_, what);    \
    } while (0)
