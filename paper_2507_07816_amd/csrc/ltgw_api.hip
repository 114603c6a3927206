// C-ABI of the ltgw library: context, validation, device buffers, launches.
// The declarations and their contracts are in include/ltgw.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "ltgw_ctx.h"
#include "ltgw_antenna.h"
#include "ltgw_list.h"

using namespace ltgw;

namespace {
thread_local std::string g_create_error;
}  // namespace

// Device memory of ltgw_eval_templates_noalloc: one static array, of which
// every device the library runs on holds its own copy until the process
// ends.  In host code `scratch` is only a stand-in for the symbol, not a
// device address: ltgw_create resolves the address on each device once
// (hipGetSymbolAddress with that device current) and the contexts on that
// device use only the resolved address.
__device__ __align__(256) unsigned char scratch[LTGW_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kScratchDevices = 64;     // devices whose scratch address is kept
std::mutex g_scratch_mu;
void *g_scratch_addr[kScratchDevices];  // resolved address per device, NULL until then

// The address of `scratch` on the current device `device` (resolved once).
hipError_t scratch_address(int device, void **out) {
    *out = nullptr;
    if (device < 0 || device >= kScratchDevices) return hipSuccess;  // no scratch there
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_addr[device] = p;
    }
    *out = g_scratch_addr[device];
    return hipSuccess;
}
}  // namespace

namespace ltgw {

int fail(ltgw_ctx *c, int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c)
        c->err = buf;
    else
        g_create_error = buf;  // a call made without a context: ltgw_last_error(NULL)
    return code;
}

int hip_fail(ltgw_ctx *c, hipError_t e, const char *what) {
    return fail(c, e == hipErrorOutOfMemory ? LTGW_E_NOMEM : LTGW_E_DEVICE, "%s: %s (%s)", what,
                hipGetErrorName(e), hipGetErrorString(e));
}

int ensure(ltgw_ctx *c, DevBuf &b, size_t bytes, const char *what) {
    if (bytes == 0) bytes = 16;
    if (b.cap >= bytes) return LTGW_OK;
    if (b.p) {
        hipError_t e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "synchronize before realloc");
        (void)hipFree(b.p);
        b.p = nullptr;
        b.cap = 0;
    }
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(c, LTGW_E_NOMEM, "device allocation of %zu bytes for %s failed: %s", bytes, what,
                    hipGetErrorString(e));
    }
    b.p = p;
    b.cap = bytes;
    return LTGW_OK;
}

void release(DevBuf &b) {
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.cap = 0;
}

// Pinned host staging (hipHostMalloc), grown like ensure(); the caller has
// waited for every copy that reads the old buffer.
int ensure_pinned(ltgw_ctx *c, DevBuf &b, size_t bytes, const char *what) {
    if (bytes == 0) bytes = 16;
    if (b.cap >= bytes) return LTGW_OK;
    if (b.p) (void)hipHostFree(b.p);
    b.p = nullptr;
    b.cap = 0;
    void *p = nullptr;
    hipError_t e = hipHostMalloc(&p, bytes, hipHostMallocDefault);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(c, LTGW_E_NOMEM, "pinned host allocation of %zu bytes for %s failed: %s", bytes, what,
                    hipGetErrorString(e));
    }
    b.p = p;
    b.cap = bytes;
    return LTGW_OK;
}

void release_pinned(DevBuf &b) {
    if (b.p) (void)hipHostFree(b.p);
    b.p = nullptr;
    b.cap = 0;
}

bool is_device_ptr(const void *p) {
    hipPointerAttribute_t attr;
    hipError_t e = hipPointerGetAttributes(&attr, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
}

// Copy n bytes from a host-or-device pointer to host memory.
int to_host(ltgw_ctx *c, void *dst, const void *src, size_t n, const char *what) {
    if (n == 0) return LTGW_OK;
    if (is_device_ptr(src)) {
        HIP_TRY(c, hipMemcpyAsync(dst, src, n, hipMemcpyDeviceToHost, c->stream), what);
        HIP_TRY(c, hipStreamSynchronize(c->stream), what);
    } else {
        std::memcpy(dst, src, n);
    }
    return LTGW_OK;
}

int h2d(ltgw_ctx *c, void *dst, const void *src, size_t n, const char *what) {
    if (n == 0) return LTGW_OK;
    HIP_TRY(c, hipMemcpyAsync(dst, src, n, hipMemcpyHostToDevice, c->stream), what);
    return LTGW_OK;
}

bool fin(double x) { return std::isfinite(x); }

}  // namespace ltgw

namespace ltgw {

__global__ void zero_u64_kernel(unsigned long long *p, int n) {
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0ull;
}

int zero_counter(ltgw_ctx *c, int first, int n) {
    hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(64), 0, c->stream,
                       (unsigned long long *)c->counters.p + first, n);
    HIP_TRY(c, hipGetLastError(), "zero counters");
    return LTGW_OK;
}

int read_counter(ltgw_ctx *c, int i, unsigned long long *out) {
    HIP_TRY(c, hipMemcpyAsync(out, (unsigned long long *)c->counters.p + i, sizeof *out,
                              hipMemcpyDeviceToHost, c->stream),
            "read counter");
    HIP_TRY(c, hipStreamSynchronize(c->stream), "read counter");
    return LTGW_OK;
}

}  // namespace ltgw


// What is wrong with a listed template, or NULL.
static const char *template_error(const ltgw_template &T) {
    if (!fin(T.f0) || !(T.f0 > 0.0)) return "f0 must be > 0";
    if (!fin(T.tau) || !(T.tau > 0.0)) return "tau must be > 0";
    if (!fin(T.brake) || !(T.brake > 1.0)) return "the braking index must be > 1";
    const double *k = T.sky;
    if (!fin(k[0]) || !fin(k[1]) || !fin(k[2]) ||
        std::fabs(std::sqrt(k[0] * k[0] + k[1] * k[1] + k[2] * k[2]) - 1.0) > 1e-12)
        return "sky is not a unit vector";
    return nullptr;
}

// The host's work on a long list (checks, f0 range, ordering, the copy into
// the staging) runs on several threads, each over one contiguous chunk.
static int list_threads(int64_t n) {
    if (n < ((int64_t)1 << 17)) return 1;
    const unsigned hc = std::thread::hardware_concurrency();
    return (int)std::min<unsigned>(16u, hc ? hc : 1u);
}
static int64_t chunk_lo(int64_t n, int nt, int t) { return n * t / nt; }
// f(t) for t in [0, nt): t = 0 on the calling thread; where a thread cannot be
// started, its chunk runs on the calling thread instead
template <class F>
static void run_chunks(int nt, const F &f) {
    std::vector<std::thread> th;
    std::vector<int> inline_t;
    for (int t = 1; t < nt; ++t) {
        try {
            th.emplace_back(f, t);
        } catch (...) {
            inline_t.push_back(t);
        }
    }
    f(0);
    for (int t : inline_t) f(t);
    for (auto &x : th) x.join();
}

extern "C" {

int32_t ltgw_create(int32_t device, void *hip_stream, ltgw_ctx **out) {
    g_create_error.clear();
    if (!out) {
        g_create_error = "ltgw_create: out is NULL";
        return LTGW_E_INVALID_ARG;
    }
    *out = nullptr;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n == 0) {
        (void)hipGetLastError();
        g_create_error = std::string("ltgw_create: no HIP device: ") + hipGetErrorString(e);
        return LTGW_E_DEVICE;
    }
    if (device < 0 || device >= n) {
        g_create_error = "ltgw_create: device index out of range";
        return LTGW_E_INVALID_ARG;
    }
    if ((e = hipSetDevice(device)) != hipSuccess) {
        g_create_error = std::string("ltgw_create: hipSetDevice: ") + hipGetErrorString(e);
        return LTGW_E_DEVICE;
    }
    ltgw_ctx *c = new (std::nothrow) ltgw_ctx();
    if (!c) {
        g_create_error = "ltgw_create: host allocation failed";
        return LTGW_E_NOMEM;
    }
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    int rc = ensure(c, c->counters, kNumCnt * sizeof(unsigned long long), "counters");
    if (rc == LTGW_OK) rc = zero_counter(c, 0, kNumCnt);
    for (int i = 0; i < 3 && rc == LTGW_OK; ++i) {
        hipError_t ee = hipEventCreate(&c->ev[i]);
        if (ee != hipSuccess) rc = hip_fail(c, ee, "event create");
    }
    if (rc == LTGW_OK) {
        hipError_t ee = hipEventCreateWithFlags(&c->ev_h2d, hipEventDisableTiming);
        if (ee == hipSuccess) ee = hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming);
        if (ee == hipSuccess) ee = hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming);
        if (ee == hipSuccess) ee = hipEventCreate(&c->ev_ing[0]);
        if (ee == hipSuccess) ee = hipEventCreate(&c->ev_ing[1]);
        if (ee == hipSuccess) ee = hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking);
        for (auto &e : c->ev_sft)
            if (ee == hipSuccess) ee = hipEventCreateWithFlags(&e, hipEventDisableTiming);
        if (ee != hipSuccess) rc = hip_fail(c, ee, "event/stream create");
    }
    if (rc == LTGW_OK) {
        const hipError_t ee = scratch_address(device, &c->scratch);
        if (ee != hipSuccess) rc = hip_fail(c, ee, "address of the static scratch array");
    }
    if (rc == LTGW_OK) {
        // host staging of the grid lists, sized once so that the
        // no-allocation entry point never grows them
        c->h_tau.reserve(LTGW_NOALLOC_MAX_AXIS);
        c->h_brake.reserve(LTGW_NOALLOC_MAX_AXIS);
        c->h_sky.reserve(3 * (size_t)LTGW_NOALLOC_MAX_AXIS);
    }
    if (rc == LTGW_OK) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && v > 0)
            c->cu_count = v;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeWallClockRate, device) == hipSuccess && v > 0)
            c->wall_khz = v;
        (void)hipGetLastError();
    }
    if (rc != LTGW_OK) {
        g_create_error = c->err;
        ltgw_destroy(c);
        return rc;
    }
    *out = c;
    return LTGW_OK;
}

void ltgw_destroy(ltgw_ctx *c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    if (c->side) (void)hipStreamSynchronize(c->side);
    for (hipEvent_t e : c->ev)
        if (e) (void)hipEventDestroy(e);
    if (c->ev_h2d) (void)hipEventDestroy(c->ev_h2d);
    if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
    if (c->ev_join) (void)hipEventDestroy(c->ev_join);
    for (hipEvent_t e : c->ev_ing)
        if (e) (void)hipEventDestroy(e);
    for (auto &e : c->ev_sft)
        if (e) (void)hipEventDestroy(e);
    if (c->side) (void)hipStreamDestroy(c->side);
    free_batch(c->batch);
    free_stack(c->stack);
    sft_release(c);
    for (auto &d : c->det) {
        release(d.store_buf); release(d.t_seg); release(d.w); release(d.wq);
        release(d.scale); release(d.v); release(d.g); release(d.H); release(d.wfix); release(d.win);
        release(d.era); release(d.w_sky); release(d.wq_sky);
    }
    DevBuf *all[] = {&c->staging, &c->counters, &c->cnn_packed, &c->list_d, &c->perm_d, &c->list_dop, &c->list_sky,
                     &c->tau_d,   &c->brake_d,  &c->sky_d,      &c->res_s, &c->res_c, &c->res_n, &c->res_w1, &c->res_w2, &c->diff,
                     &c->cand_pa, &c->cand_ia, &c->cand_pb, &c->cand_ib, &c->cand_out, &c->n_out};
    for (DevBuf *b : all) release(*b);
    release_pinned(c->h_list);
    release_pinned(c->h_perm);
    delete c;
}

const char *ltgw_last_error(const ltgw_ctx *c) {
    return c ? c->err.c_str() : g_create_error.c_str();
}

int32_t ltgw_load_spectrogram(ltgw_ctx *c, int32_t det, const ltgw_spec_desc *d,
                              const float *power) {
    if (!c) return LTGW_E_INVALID_ARG;
    Enter en(c);
    if (det < 0 || det >= LTGW_MAX_DET) return fail(c, LTGW_E_INVALID_ARG, "detector %d out of range", det);
    if (!d || !power) return fail(c, LTGW_E_INVALID_ARG, "descriptor or power is NULL");
    if (d->n_seg < 1 || d->n_bins < 1) return fail(c, LTGW_E_INVALID_ARG, "n_seg and n_bins must be >= 1");
    if (d->k_lo < 2 || d->k_lo + d->n_bins >= (int64_t)1 << 30)
        return fail(c, LTGW_E_INVALID_ARG, "k_lo must satisfy 2 <= k_lo and k_lo + n_bins < 2^30");
    if (!(d->t_sft > 0.0) || !fin(d->t_sft)) return fail(c, LTGW_E_INVALID_ARG, "t_sft must be finite and > 0");
    if (!d->t_seg) return fail(c, LTGW_E_INVALID_ARG, "t_seg is NULL");
    if (!std::isfinite(d->rho_th)) return fail(c, LTGW_E_INVALID_ARG, "rho_th must be finite");
    if (d->store != LTGW_STORE_F32 && d->store != LTGW_STORE_BF16 && d->store != LTGW_STORE_FP8)
        return fail(c, LTGW_E_INVALID_ARG, "unknown store %d", d->store);
    Det &D = c->det[det];
    D.loaded = false;
    D.has_v = false;
    D.has_antenna = false;
    D.tab_n_tn = D.tab_n_groups = 0;
    const int64_t ns = d->n_seg, nb = d->n_bins;
    std::vector<double> ht(ns);
    std::vector<float> hw(ns, 1.0f);
    int rc;
    if ((rc = to_host(c, ht.data(), d->t_seg, ns * sizeof(double), "t_seg")) != LTGW_OK) return rc;
    if (d->weights && (rc = to_host(c, hw.data(), d->weights, ns * sizeof(float), "weights")) != LTGW_OK)
        return rc;
    for (int64_t j = 0; j < ns; ++j) {
        if (!fin(ht[j])) return fail(c, LTGW_E_INVALID_ARG, "t_seg[%lld] is not finite", (long long)j);
        if (!(hw[j] > 0.0f) || !std::isfinite(hw[j]))
            return fail(c, LTGW_E_INVALID_ARG, "weights[%lld] must be finite and > 0", (long long)j);
    }
    bool weighted = false;
    for (int64_t j = 1; j < ns; ++j) weighted |= (hw[j] != hw[0]);
    const int esize = d->store == LTGW_STORE_F32 ? 4 : d->store == LTGW_STORE_BF16 ? 2 : 1;
    const int64_t pitch = ((nb + 2 + 63) / 64) * 64;
    if (ns * pitch * esize >= ((int64_t)1 << 31))
        return fail(c, LTGW_E_UNSUPPORTED, "spectrogram store of %lld bytes exceeds 2^31 per detector",
                    (long long)(ns * pitch * esize));
    if ((rc = ensure(c, D.store_buf, (size_t)(ns * pitch * esize), "spectrogram store")) != LTGW_OK) return rc;
    if ((rc = ensure(c, D.t_seg, ns * sizeof(double), "t_seg")) != LTGW_OK) return rc;
    if ((rc = ensure(c, D.w, ns * sizeof(float), "weights")) != LTGW_OK) return rc;
    if ((rc = ensure(c, D.wq, ns * sizeof(float), "scaled weights")) != LTGW_OK) return rc;
    if ((rc = ensure(c, D.scale, ns * sizeof(float), "scales")) != LTGW_OK) return rc;
    if ((rc = h2d(c, D.t_seg.p, ht.data(), ns * sizeof(double), "t_seg upload")) != LTGW_OK) return rc;
    if ((rc = h2d(c, D.w.p, hw.data(), ns * sizeof(float), "weights upload")) != LTGW_OK) return rc;
    const float *src = power;
    if (!is_device_ptr(power)) {
        if ((rc = ensure(c, c->staging, (size_t)(ns * nb) * sizeof(float), "power staging")) != LTGW_OK)
            return rc;
        if ((rc = h2d(c, c->staging.p, power, (size_t)(ns * nb) * sizeof(float), "power upload")) != LTGW_OK)
            return rc;
        src = (const float *)c->staging.p;
    }
    if ((rc = zero_counter(c, kCntBad, 1)) != LTGW_OK) return rc;
    c->have_ingest = false;
    HIP_TRY(c, hipEventRecord(c->ev_ing[0], c->stream), "event record");
    HIP_TRY(c, launch_ingest(d->store, src, d->n_seg, d->n_bins, pitch, D.store_buf.p,
                             (float *)D.scale.p, (const float *)D.w.p, (float *)D.wq.p, d->rho_th,
                             (unsigned long long *)c->counters.p + kCntBad, c->stream),
            "ingest launch");
    HIP_TRY(c, hipEventRecord(c->ev_ing[1], c->stream), "event record");
    c->have_ingest = true;
    unsigned long long bad = 0;
    if ((rc = read_counter(c, kCntBad, &bad)) != LTGW_OK) return rc;
    if (bad) return fail(c, LTGW_E_INVALID_ARG, "%llu power values are negative or not finite", bad);
    D.n_seg = d->n_seg;
    D.n_bins = d->n_bins;
    D.store = d->store;
    D.k_lo = d->k_lo;
    D.pitch = pitch;
    D.t_sft = d->t_sft;
    D.rho_th = d->rho_th;
    D.weighted = weighted;
    D.w_uniform = hw[0];
    D.h_w = hw;
    D.h_t = ht;
    D.h_wfix.reserve(3 * (size_t)D.n_seg);  // the fixed-point weights' staging never grows at eval
    D.loaded = true;
    c->have_eval = false;
    return LTGW_OK;
}

int32_t ltgw_set_velocity_table(ltgw_ctx *c, int32_t det, const double *v, int32_t n_seg) {
    if (!c) return LTGW_E_INVALID_ARG;
    Enter en(c);
    if (det < 0 || det >= LTGW_MAX_DET) return fail(c, LTGW_E_INVALID_ARG, "detector %d out of range", det);
    Det &D = c->det[det];
    if (!D.loaded) return fail(c, LTGW_E_STATE, "no spectrogram loaded for detector %d", det);
    if (!v) return fail(c, LTGW_E_INVALID_ARG, "velocity table is NULL");
    if (n_seg != D.n_seg)
        return fail(c, LTGW_E_INVALID_ARG, "velocity table has %d rows, spectrogram %d", n_seg, D.n_seg);
    std::vector<double> hv((size_t)n_seg * 3);
    int rc;
    if ((rc = to_host(c, hv.data(), v, hv.size() * sizeof(double), "velocity")) != LTGW_OK) return rc;
    double vmax = 0.0;
    for (int32_t j = 0; j < n_seg; ++j) {
        const double *r = &hv[3 * (size_t)j];
        if (!fin(r[0]) || !fin(r[1]) || !fin(r[2]))
            return fail(c, LTGW_E_INVALID_ARG, "velocity row %d is not finite", j);
        const double m = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]) / kC;
        if (!(m < 1.0)) return fail(c, LTGW_E_INVALID_ARG, "|v| >= c at row %d", j);
        vmax = m > vmax ? m : vmax;
    }
    if ((rc = ensure(c, D.v, hv.size() * sizeof(double), "velocity")) != LTGW_OK) return rc;
    if ((rc = h2d(c, D.v.p, hv.data(), hv.size() * sizeof(double), "velocity upload")) != LTGW_OK) return rc;
    HIP_TRY(c, hipStreamSynchronize(c->stream), "velocity upload");
    D.v_max = vmax;
    D.h_v = hv;
    D.has_v = true;
    c->have_eval = false;
    return LTGW_OK;
}

int32_t ltgw_set_antenna(ltgw_ctx *c, int32_t det, const double *arms, const double *era, int32_t n_seg) {
    if (!c) return LTGW_E_INVALID_ARG;
    Enter en(c);
    if (det < 0 || det >= LTGW_MAX_DET) return fail(c, LTGW_E_INVALID_ARG, "detector %d out of range", det);
    Det &D = c->det[det];
    if (!D.loaded) return fail(c, LTGW_E_STATE, "no spectrogram loaded for detector %d", det);
    c->have_eval = false;
    if (!arms) {
        D.has_antenna = false;
        return LTGW_OK;
    }
    if (is_device_ptr(arms)) return fail(c, LTGW_E_INVALID_ARG, "arms must be host memory");
    if (!era) return fail(c, LTGW_E_INVALID_ARG, "era is NULL");
    if (n_seg != D.n_seg)
        return fail(c, LTGW_E_INVALID_ARG, "era has %d entries, spectrogram %d segments", n_seg, D.n_seg);
    for (int k = 0; k < 2; ++k) {
        const double *a = arms + 3 * k;
        if (!fin(a[0]) || !fin(a[1]) || !fin(a[2]) ||
            std::fabs(std::sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]) - 1.0) > 1e-12)
            return fail(c, LTGW_E_INVALID_ARG, "arm %d is not a unit vector", k);
    }
    std::vector<double> he((size_t)n_seg);
    int rc;
    if ((rc = to_host(c, he.data(), era, he.size() * sizeof(double), "era")) != LTGW_OK) return rc;
    for (int32_t j = 0; j < n_seg; ++j)
        if (!fin(he[j])) return fail(c, LTGW_E_INVALID_ARG, "era[%d] is not finite", j);
    if ((rc = ensure(c, D.era, he.size() * sizeof(double), "rotation angles")) != LTGW_OK) return rc;
    if ((rc = h2d(c, D.era.p, he.data(), he.size() * sizeof(double), "rotation angle upload")) != LTGW_OK) return rc;
    HIP_TRY(c, hipStreamSynchronize(c->stream), "rotation angle upload");
    std::memcpy(D.arms, arms, sizeof D.arms);
    D.has_antenna = true;
    return LTGW_OK;
}

}  // extern "C"

namespace ltgw {

int plan_search(ltgw_ctx *c, const ltgw_grid *g, const int *slots, int n_slots, SearchPlan &P) {
    if (!g) return fail(c, LTGW_E_INVALID_ARG, "grid is NULL");
    if (g->n_f0 < 1 || g->n_tau < 1 || g->n_brake < 1 || g->n_sky < 1)
        return fail(c, LTGW_E_INVALID_ARG, "grid axes must have at least one point");
    if (!g->tau || !g->brake || !g->sky) return fail(c, LTGW_E_INVALID_ARG, "grid arrays are NULL");
    if (!fin(g->f0_min) || !(g->f0_min > 0.0)) return fail(c, LTGW_E_INVALID_ARG, "f0_min must be finite and > 0");
    if (!fin(g->f0_step) || g->f0_step < 0.0) return fail(c, LTGW_E_INVALID_ARG, "f0_step must be finite and >= 0");
    if (!fin(g->t0)) return fail(c, LTGW_E_INVALID_ARG, "t0 must be finite");
    for (int i = 0; i < g->n_tau; ++i)
        if (!fin(g->tau[i]) || !(g->tau[i] > 0.0))
            return fail(c, LTGW_E_INVALID_ARG, "tau[%d] must be finite and > 0", i);
    for (int i = 0; i < g->n_brake; ++i)
        if (!fin(g->brake[i]) || !(g->brake[i] > 1.0))
            return fail(c, LTGW_E_INVALID_ARG, "braking index [%d] must be finite and > 1", i);
    for (int i = 0; i < g->n_sky; ++i) {
        const double *s = g->sky + 3 * i;
        if (!fin(s[0]) || !fin(s[1]) || !fin(s[2]))
            return fail(c, LTGW_E_INVALID_ARG, "sky[%d] is not finite", i);
        if (std::fabs(std::sqrt(s[0] * s[0] + s[1] * s[1] + s[2] * s[2]) - 1.0) > 1e-12)
            return fail(c, LTGW_E_INVALID_ARG, "sky[%d] is not a unit vector", i);
    }
    const double f0_max = g->f0_min + (double)(g->n_f0 - 1) * g->f0_step;
    if (!fin(f0_max)) return fail(c, LTGW_E_INVALID_ARG, "f0 range overflows");
    P = SearchPlan();
    P.n_f0 = g->n_f0;
    P.n_tau = g->n_tau;
    P.n_brake = g->n_brake;
    P.n_sky = g->n_sky;
    P.n_tn = g->n_tau * g->n_brake;
    P.n_groups = (int64_t)P.n_tn * g->n_sky;
    P.n_tpl = P.n_groups * g->n_f0;
    if (P.n_tpl >= ((int64_t)1 << 31) || P.n_groups >= ((int64_t)1 << 24))
        return fail(c, LTGW_E_UNSUPPORTED, "grid of %lld templates (%lld groups) exceeds 2^31 templates or 2^24 groups",
                    (long long)P.n_tpl, (long long)P.n_groups);
    if (n_slots < 1) return fail(c, LTGW_E_STATE, "no detector selected");
    if (n_slots > LTGW_MAX_SEARCH_DET)
        return fail(c, LTGW_E_UNSUPPORTED, "a search sums at most %d detectors", LTGW_MAX_SEARCH_DET);
    for (int q = 0; q < n_slots; ++q) {
        const int d = slots[q];
        if (d < 0 || d >= LTGW_MAX_DET) return fail(c, LTGW_E_INVALID_ARG, "detector slot %d out of range", d);
        for (int r = 0; r < q; ++r)
            if (slots[r] == d) return fail(c, LTGW_E_INVALID_ARG, "detector slot %d listed twice", d);
        const Det &D = c->det[d];
        if (!D.loaded) return fail(c, LTGW_E_STATE, "detector %d selected but not loaded", d);
        if (!D.has_v) return fail(c, LTGW_E_STATE, "detector %d has no velocity table", d);
        if (q > 0 && D.rho_th != c->det[slots[0]].rho_th)
            return fail(c, LTGW_E_UNSUPPORTED, "selected detectors have different rho_th");
        if (q > 0 && D.store != c->det[slots[0]].store)
            return fail(c, LTGW_E_UNSUPPORTED, "selected detectors have different stores");
        // g <= 1 (u >= 1, e < 0) and D < 1 + v_max: x < 2^30 keeps the bin arithmetic exact
        if (!(f0_max * D.t_sft * (1.0 + D.v_max) < (double)(1 << 30) - 4.0))
            return fail(c, LTGW_E_INVALID_ARG, "f0_max * t_sft too large for detector %d", d);
        P.sel[q] = d;
        P.n_evals += (int64_t)D.n_seg * P.n_tpl;
        P.n_seg_total += D.n_seg;
        P.max_bins = D.n_bins > P.max_bins ? D.n_bins : P.max_bins;
    }
    P.n_sel = n_slots;
    P.store = c->det[slots[0]].store;
    P.rho_th = c->det[slots[0]].rho_th;
    return LTGW_OK;
}

// In-band moments: uniform weights need only N; otherwise the weights get an
// exact fixed-point form w = wfix * 2^e0 (w^2 = (hi * 2^32 + lo) * 2^(2 e0))
// when their exponents span at most 7 binades, so W1 and W2 come from exact
// integer range sums; failing that, the statistic kernel accumulates them.
Moments plan_moments(ltgw_ctx *c, const int *slots, int n_slots) {
    Moments M;
    M.w_uniform = c->det[slots[0]].w_uniform;
    for (int q = 0; q < n_slots; ++q)
        if (c->det[slots[q]].has_antenna) {  // weights per (sky, segment): summed by the statistic kernel
            M.mode = 2;
            return M;
        }
    bool uniform = true;
    for (int q = 0; q < n_slots; ++q) {
        const Det &D = c->det[slots[q]];
        uniform &= !D.weighted && D.w_uniform == M.w_uniform;
    }
    if (uniform) return M;
    int emin = 1 << 30, emax = -(1 << 30);
    for (int q = 0; q < n_slots; ++q)
        for (float wv : c->det[slots[q]].h_w) {
            int ex;
            (void)std::frexp(wv, &ex);  // w = f 2^ex, f in [0.5, 1)
            emin = ex < emin ? ex : emin;
            emax = ex > emax ? ex : emax;
        }
    if (emax - emin > 7) {
        M.mode = 2;
        return M;
    }
    M.mode = 1;
    M.e0 = emin - 24;
    for (int q = 0; q < n_slots; ++q) {
        Det &D = c->det[slots[q]];
        D.h_wfix.resize(3 * (size_t)D.n_seg);
        for (int32_t j = 0; j < D.n_seg; ++j) {
            const uint64_t m = (uint64_t)std::ldexp((double)D.h_w[j], -M.e0);  // exact integer
            const unsigned __int128 m2 = (unsigned __int128)m * m;
            D.h_wfix[3 * (size_t)j + 0] = (int64_t)m;
            D.h_wfix[3 * (size_t)j + 1] = (int64_t)(uint64_t)(m2 >> 32);
            D.h_wfix[3 * (size_t)j + 2] = (int64_t)(uint64_t)(m2 & 0xffffffffu);
        }
    }
    return M;
}

static int ilog2(int64_t v) {
    int r = 0;
    while (v > 1) {
        v >>= 1;
        ++r;
    }
    return r;
}

void tune_key_eval(const SearchPlan &P, bool moments_in_loop, char (&buf)[160]) {
    snprintf(buf, sizeof buf, "eval/store%d/mom%d/seg%d/bins%d/tpl%d", P.store, moments_in_loop ? 1 : 0,
             ilog2(P.n_seg_total), ilog2(P.max_bins), ilog2(P.n_tpl));
}

std::string tune_key_eval(const SearchPlan &P, bool moments_in_loop) {
    char buf[160];
    tune_key_eval(P, moments_in_loop, buf);
    return buf;
}

std::string tune_key_batch(int store, bool moments_in_loop, int n_searches, int64_t evals) {
    char buf[160];
    snprintf(buf, sizeof buf, "batch/store%d/mom%d/n%d/evals%d", store, moments_in_loop ? 1 : 0,
             ilog2(n_searches), ilog2(evals));
    return buf;
}

}  // namespace ltgw

namespace {

// Device memory of one single-search evaluation: the context's own buffers,
// grown on demand, or consecutive 256-byte aligned slices of the device's
// static scratch array (the no-allocation entry point).  In scratch mode the
// caller has checked the total (eval_bytes) before anything is enqueued.
struct EvalMem {
    ltgw_ctx *c;
    char *base = nullptr;  // scratch base (device address), or NULL: context buffers
    size_t cap = 0;        // scratch bytes
    size_t used = 0;
    int get(DevBuf &b, size_t bytes, const char *what, void **p) {
        if (!base) {
            const int rc = ensure(c, b, bytes, what);
            *p = b.p;
            return rc;
        }
        used = (used + 255) & ~(size_t)255;
        const size_t n = bytes ? bytes : 16;
        if (used > cap || n > cap - used)  // eval_bytes was checked first: never taken
            return fail(c, LTGW_E_UNSUPPORTED, "device scratch exhausted at %s", what);
        *p = base + used;
        used += n;
        return LTGW_OK;
    }
};

// Bytes of scratch the evaluation of plan P takes (every table, window,
// moment array and per-template result), each slice rounded up to 256.
size_t eval_bytes(const ltgw_ctx *c, const SearchPlan &P, const Moments &M, const ltgw_grid *g) {
    auto r = [](size_t b) { return ((b ? b : 16) + 255) & ~(size_t)255; };
    size_t t = r((size_t)g->n_tau * 8) + r((size_t)g->n_brake * 8) + r((size_t)g->n_sky * 24);
    const size_t win_blocks = (size_t)(g->n_f0 + 255) / 256;
    for (int q = 0; q < P.n_sel; ++q) {
        const Det &D = c->det[P.sel[q]];
        t += r((size_t)P.n_tn * D.n_seg * 8) + r((size_t)P.n_groups * D.n_seg * 8);
        if (D.has_antenna) t += 2 * r((size_t)g->n_sky * D.n_seg * 4);
        if (M.mode == 1) t += r((size_t)D.n_seg * 3 * 8);
        t += r((size_t)P.n_groups * win_blocks * sizeof(int2));
    }
    const size_t n = (size_t)P.n_tpl;
    t += r(n * 8) + r(n * 4) + r(n * 4) + r(n * 8) + r(n * 8);
    if (M.mode != 2) t += r((size_t)(M.mode ? 4 : 1) * (size_t)P.n_groups * (size_t)(g->n_f0 + 1) * 8);
    return t;
}

// The single-search evaluation; variant < 0 takes the tuned (or default)
// shape.  scratch != NULL: every buffer is a slice of it (no allocation) and
// the results are not kept for ltgw_psi / ltgw_topk_candidates.
int eval_single(ltgw_ctx *c, const ltgw_grid *g, uint32_t stats, float *out_s, int32_t *out_c,
                int32_t *out_n, int variant, void *scratch = nullptr, size_t scratch_cap = 0) {
    c->have_eval = false;
    c->results_kept = false;
    if (!g) return fail(c, LTGW_E_INVALID_ARG, "grid is NULL");
    if (stats == 0 || (stats & ~(LTGW_STAT_POWER | LTGW_STAT_COUNT)))
        return fail(c, LTGW_E_INVALID_ARG, "stats must be a non-empty mask of POWER and COUNT");
    int slots[32], n_slots = 0;
    for (int d = 0; d < 32; ++d) {
        const bool want = g->det_mask ? ((g->det_mask >> d) & 1u) : c->det[d].loaded;
        if (!want) continue;
        if (n_slots == LTGW_MAX_SEARCH_DET)
            return fail(c, LTGW_E_UNSUPPORTED, "a search sums at most %d detectors", LTGW_MAX_SEARCH_DET);
        slots[n_slots++] = d;
    }
    SearchPlan P;
    int rc = plan_search(c, g, slots, n_slots, P);
    if (rc != LTGW_OK) return rc;
    // grid arrays to the device; the host copies must outlive the previous upload
    HIP_TRY(c, hipEventSynchronize(c->ev_h2d), "previous grid upload");
    const Moments M = plan_moments(c, P.sel, P.n_sel);
    const bool moments_in_loop = M.mode == 2;
    EvalMem mem{c};
    if (scratch) {
        if (g->n_tau > LTGW_NOALLOC_MAX_AXIS || g->n_brake > LTGW_NOALLOC_MAX_AXIS ||
            g->n_sky > LTGW_NOALLOC_MAX_AXIS)
            return fail(c, LTGW_E_UNSUPPORTED,
                        "the no-allocation entry point takes at most %d tau, brake and sky values each "
                        "(use ltgw_eval_templates)",
                        LTGW_NOALLOC_MAX_AXIS);
        const size_t need = eval_bytes(c, P, M, g);
        if (need > scratch_cap)
            return fail(c, LTGW_E_UNSUPPORTED,
                        "this search needs %zu bytes of device scratch; the no-allocation entry point "
                        "has %zu (use ltgw_eval_templates)",
                        need, scratch_cap);
        mem.base = (char *)scratch;
        mem.cap = scratch_cap;
    }
    c->h_tau.assign(g->tau, g->tau + g->n_tau);
    c->h_brake.assign(g->brake, g->brake + g->n_brake);
    c->h_sky.assign(g->sky, g->sky + 3 * (size_t)g->n_sky);
    void *tau_p, *brake_p, *sky_p;
    if ((rc = mem.get(c->tau_d, c->h_tau.size() * 8, "tau", &tau_p)) != LTGW_OK) return rc;
    if ((rc = mem.get(c->brake_d, c->h_brake.size() * 8, "brake", &brake_p)) != LTGW_OK) return rc;
    if ((rc = mem.get(c->sky_d, c->h_sky.size() * 8, "sky", &sky_p)) != LTGW_OK) return rc;
    if ((rc = h2d(c, tau_p, c->h_tau.data(), c->h_tau.size() * 8, "tau upload")) != LTGW_OK) return rc;
    if ((rc = h2d(c, brake_p, c->h_brake.data(), c->h_brake.size() * 8, "brake upload")) != LTGW_OK) return rc;
    if ((rc = h2d(c, sky_p, c->h_sky.data(), c->h_sky.size() * 8, "sky upload")) != LTGW_OK) return rc;
    HIP_TRY(c, hipEventRecord(c->ev[0], c->stream), "event record");
    EvalArgs a;
    std::memset(&a, 0, sizeof a);
    for (int q = 0; q < P.n_sel; ++q) {
        Det &D = c->det[P.sel[q]];
        D.tab_n_tn = D.tab_n_groups = 0;  // the tables below are the last eval's once filled
        void *g_p, *H_p;
        if ((rc = mem.get(D.g, (size_t)P.n_tn * D.n_seg * 8, "spin-factor table", &g_p)) != LTGW_OK) return rc;
        if ((rc = mem.get(D.H, (size_t)P.n_groups * D.n_seg * 8, "track-factor table", &H_p)) != LTGW_OK) return rc;
        HIP_TRY(c, launch_spin_factor((const double *)D.t_seg.p, D.n_seg, g->t0, (const double *)tau_p,
                                      g->n_tau, (const double *)brake_p, g->n_brake, (double *)g_p,
                                      (unsigned long long *)c->counters.p + kCntUndecided, c->stream),
                "spin-factor launch");
        HIP_TRY(c, launch_track_factor((const double *)g_p, P.n_tn, (const double *)D.v.p, D.n_seg,
                                       (const double *)sky_p, g->n_sky, D.t_sft, (double *)H_p, c->stream),
                "track-factor launch");
        if (!scratch) {
            D.tab_n_tn = P.n_tn;
            D.tab_n_groups = (int32_t)P.n_groups;
        }
        DetView &V = a.det[q];
        V.store = D.store_buf.p;
        V.pitch_bytes = (int32_t)(D.pitch * (D.store == LTGW_STORE_F32 ? 4 : D.store == LTGW_STORE_BF16 ? 2 : 1));
        V.H = (const double *)H_p;
        V.g = (const double *)g_p;
        V.D = nullptr;
        V.t_sft = D.t_sft;
        V.wq = (const float *)D.wq.p;
        V.w = (const float *)D.w.p;
        V.cshift = 1.5 - (double)D.k_lo;
        V.wfix = nullptr;
        V.n_seg = D.n_seg;
        V.n_bins = D.n_bins;
        V.w_sky_stride = 0;
        if (D.has_antenna) {  // one row of weights per sky point of the grid
            const size_t nw = (size_t)g->n_sky * (size_t)D.n_seg;
            void *ws_p, *wqs_p;
            if ((rc = mem.get(D.w_sky, nw * 4, "antenna weights", &ws_p)) != LTGW_OK) return rc;
            if ((rc = mem.get(D.wq_sky, nw * 4, "antenna weights", &wqs_p)) != LTGW_OK) return rc;
            Arms A;
            std::memcpy(A.a, D.arms, sizeof A.a);
            std::memcpy(A.b, D.arms + 3, sizeof A.b);
            HIP_TRY(c, launch_antenna_weights(A, (const double *)D.era.p, D.n_seg, (const double *)sky_p,
                                              g->n_sky, (const float *)D.w.p, (const float *)D.scale.p,
                                              (float *)ws_p, (float *)wqs_p, c->stream),
                    "antenna weight launch");
            V.w = (const float *)ws_p;
            V.wq = (const float *)wqs_p;
            V.w_sky_stride = D.n_seg;
        }
        if (M.mode == 1) {
            void *wf_p;
            if ((rc = mem.get(D.wfix, D.h_wfix.size() * 8, "fixed-point weights", &wf_p)) != LTGW_OK) return rc;
            if ((rc = h2d(c, wf_p, D.h_wfix.data(), D.h_wfix.size() * 8, "weights upload")) != LTGW_OK)
                return rc;
            V.wfix = (const int64_t *)wf_p;
        }
        // in-band segment windows of every (group, run of 256 f0)
        V.win_run = 256;  // the statistic kernel's tiles are whole multiples of 256 f0
        V.win_blocks = (g->n_f0 + 255) / 256;
        void *win_p;
        if ((rc = mem.get(D.win, (size_t)P.n_groups * V.win_blocks * sizeof(int2), "segment windows", &win_p)) !=
            LTGW_OK)
            return rc;
        V.win = (const int2 *)win_p;
        HIP_TRY(c, launch_windows(V, (int)P.n_groups, P.n_tn, g->f0_min, g->f0_step, g->n_f0, (int2 *)win_p,
                                  c->stream),
                "window launch");
    }
    const int64_t n_tpl = P.n_tpl;
    void *s_p, *c_p, *n_p, *w1_p, *w2_p;
    if ((rc = mem.get(c->res_s, n_tpl * 8, "results s", &s_p)) != LTGW_OK) return rc;
    if ((rc = mem.get(c->res_c, n_tpl * 4, "results c", &c_p)) != LTGW_OK) return rc;
    if ((rc = mem.get(c->res_n, n_tpl * 4, "results N", &n_p)) != LTGW_OK) return rc;
    if ((rc = mem.get(c->res_w1, n_tpl * 8, "results W1", &w1_p)) != LTGW_OK) return rc;
    if ((rc = mem.get(c->res_w2, n_tpl * 8, "results W2", &w2_p)) != LTGW_OK) return rc;
    if ((rc = zero_counter(c, kCntInBand, 1)) != LTGW_OK) return rc;
    a.n_det = P.n_sel;
    a.n_f0 = g->n_f0;
    a.n_groups = (int32_t)P.n_groups;
    a.n_tn = P.n_tn;
    a.f0_min = g->f0_min;
    a.f0_step = g->f0_step;
    a.w_uniform = M.w_uniform;
    a.s = (double *)s_p;
    a.c = (int32_t *)c_p;
    a.n = (int32_t *)n_p;
    a.w1 = (double *)w1_p;
    a.w2 = (double *)w2_p;
    a.out_s = out_s;
    a.out_c = out_c;
    a.out_n = out_n;
    a.in_band_total = (unsigned long long *)c->counters.p + kCntInBand;
    // The in-band moments (N, W1, W2, out_n, the in-band total) read only the
    // tables and the weights, and the statistic kernel without moments reads
    // none of them: they run beside it on the second stream.  `join` makes the
    // context's stream wait for them on every way out of this call.
    struct Join {
        ltgw_ctx *c;
        bool on = false;
        ~Join() {
            if (on) (void)hipStreamWaitEvent(c->stream, c->ev_join, 0);
        }
    } join{c};
    if (!moments_in_loop) {
        const size_t n_diff = (size_t)(M.mode ? 4 : 1) * (size_t)P.n_groups * (size_t)(g->n_f0 + 1);
        void *diff_p;
        if ((rc = mem.get(c->diff, n_diff * 8, "moment difference arrays", &diff_p)) != LTGW_OK) return rc;
        HIP_TRY(c, hipEventRecord(c->ev_fork, c->stream), "event record");
        HIP_TRY(c, hipStreamWaitEvent(c->side, c->ev_fork, 0), "stream wait");
        const hipError_t me = launch_moments(a, M.mode, M.e0, (int64_t *)diff_p, c->side);
        const hipError_t je = hipEventRecord(c->ev_join, c->side);
        join.on = je == hipSuccess;
        HIP_TRY(c, me, "moments launch");
        HIP_TRY(c, je, "event record");
    }
    if (variant < 0) variant = c->forced_variant;
    if (variant < 0) {
        char key[160];
        tune_key_eval(P, moments_in_loop, key);
        const auto it = c->tune.find(key);
        variant = it == c->tune.end() ? 1 : it->second;
    }
    HIP_TRY(c, hipEventRecord(c->ev_h2d, c->stream), "event record");
    HIP_TRY(c, hipEventRecord(c->ev[1], c->stream), "event record");
    int launches = 0;
    HIP_TRY(c, launch_eval(P.store, moments_in_loop, variant, a, c->cu_count, c->stream, &launches), "eval launch");
    c->last_launches = launches;
    HIP_TRY(c, hipEventRecord(c->ev[2], c->stream), "event record");
    c->have_eval = true;
    c->results_kept = scratch == nullptr;
    c->list_mode = false;
    c->last_variant = variant;
    c->n_templates = n_tpl;
    c->n_evals = P.n_evals;
    c->f0_min = g->f0_min;
    c->f0_step = g->f0_step;
    c->n_f0 = g->n_f0;
    c->n_tau = g->n_tau;
    c->n_brake = g->n_brake;
    c->n_sky = g->n_sky;
    c->rho_th = P.rho_th;
    return LTGW_OK;
}

}  // namespace

extern "C" {

int32_t ltgw_eval_templates(ltgw_ctx *c, const ltgw_grid *g, uint32_t stats, float *out_s,
                            int32_t *out_c, int32_t *out_n) {
    if (!c) return LTGW_E_INVALID_ARG;
    Enter en(c);
    return eval_single(c, g, stats, out_s, out_c, out_n, -1);
}

int32_t ltgw_eval_templates_noalloc(ltgw_ctx *c, const ltgw_grid *g, uint32_t stats, float *out_s,
                                    int32_t *out_c, int32_t *out_n) {
    if (!c) return LTGW_E_INVALID_ARG;
    Enter en(c);
    c->have_eval = false;
    if (!c->scratch)
        return fail(c, LTGW_E_UNSUPPORTED, "device %d has no static scratch array (devices 0 .. %d do)", c->device,
                    kScratchDevices - 1);
    return eval_single(c, g, stats, out_s, out_c, out_n, -1, c->scratch, LTGW_NOALLOC_SCRATCH_BYTES);
}

int32_t ltgw_eval_list(ltgw_ctx *c, const ltgw_template *tpl, int64_t n, double t0, uint32_t det_mask,
                       float *out_s, int32_t *out_c, int32_t *out_n) {
    if (!c) return LTGW_E_INVALID_ARG;
    Enter en(c);
    c->have_eval = false;
    if (!tpl) return fail(c, LTGW_E_INVALID_ARG, "template list is NULL");
    if (n < 1 || n >= ((int64_t)1 << 31)) return fail(c, LTGW_E_INVALID_ARG, "n must be in 1 .. 2^31 - 1");
    if (is_device_ptr(tpl)) return fail(c, LTGW_E_INVALID_ARG, "the template list must be host memory");
    if (!fin(t0)) return fail(c, LTGW_E_INVALID_ARG, "t0 must be finite");
    // checks, f0 range and whether every template has the first one's sky
    // direction, per chunk; the first invalid template is reported
    const int nt = list_threads(n);
    struct ChunkScan {
        int64_t bad = -1;
        double f0_lo = 0.0, f0_hi = 0.0;
        bool one_sky = true;
    };
    std::vector<ChunkScan> scan(nt);
    run_chunks(nt, [&](int t) {
        ChunkScan &r = scan[t];
        const int64_t lo = chunk_lo(n, nt, t), hi = chunk_lo(n, nt, t + 1);
        r.f0_lo = tpl[lo].f0;
        r.f0_hi = tpl[lo].f0;
        for (int64_t q = lo; q < hi; ++q) {
            const ltgw_template &T = tpl[q];
            if (template_error(T)) {
                r.bad = q;
                return;
            }
            r.f0_lo = T.f0 < r.f0_lo ? T.f0 : r.f0_lo;
            r.f0_hi = T.f0 > r.f0_hi ? T.f0 : r.f0_hi;
            r.one_sky = r.one_sky && std::memcmp(T.sky, tpl[0].sky, sizeof T.sky) == 0;
        }
    });
    double f0_max = 0.0, f0_lo = 0.0;
    bool one_sky = true;
    for (int t = 0; t < nt; ++t) {
        if (scan[t].bad >= 0)
            return fail(c, LTGW_E_INVALID_ARG, "template %lld: %s", (long long)scan[t].bad,
                        template_error(tpl[scan[t].bad]));
        f0_max = t == 0 || scan[t].f0_hi > f0_max ? scan[t].f0_hi : f0_max;
        f0_lo = t == 0 || scan[t].f0_lo < f0_lo ? scan[t].f0_lo : f0_lo;
        one_sky = one_sky && scan[t].one_sky;
    }
    int slots[LTGW_MAX_SEARCH_DET], n_slots = 0;
    for (int d = 0; d < 32; ++d) {
        const bool want = det_mask ? ((det_mask >> d) & 1u) : c->det[d].loaded;
        if (!want) continue;
        if (n_slots == LTGW_MAX_SEARCH_DET)
            return fail(c, LTGW_E_UNSUPPORTED, "a search sums at most %d detectors", LTGW_MAX_SEARCH_DET);
        slots[n_slots++] = d;
    }
    if (n_slots < 1) return fail(c, LTGW_E_STATE, "no detector selected");
    ListArgs a;
    std::memset(&a, 0, sizeof a);
    int64_t n_seg_total = 0;
    for (int q = 0; q < n_slots; ++q) {
        const Det &D = c->det[slots[q]];
        if (!D.loaded) return fail(c, LTGW_E_STATE, "detector %d selected but not loaded", slots[q]);
        if (!D.has_v) return fail(c, LTGW_E_STATE, "detector %d has no velocity table", slots[q]);
        if (q > 0 && (D.rho_th != c->det[slots[0]].rho_th || D.store != c->det[slots[0]].store))
            return fail(c, LTGW_E_UNSUPPORTED, "selected detectors differ in rho_th or store");
        if (!(f0_max * D.t_sft * (1.0 + D.v_max) < (double)(1 << 30) - 4.0))
            return fail(c, LTGW_E_INVALID_ARG, "f0_max * t_sft too large for detector %d", slots[q]);
        ListDet &V = a.det[q];
        V.store = D.store_buf.p;
        V.pitch_bytes = (int32_t)(D.pitch * (D.store == LTGW_STORE_F32 ? 4 : D.store == LTGW_STORE_BF16 ? 2 : 1));
        V.n_seg = D.n_seg;
        V.n_bins = D.n_bins;
        V.t = (const double *)D.t_seg.p;
        V.v = (const double *)D.v.p;
        V.wq = (const float *)D.wq.p;
        V.w = (const float *)D.w.p;
        V.t_sft = D.t_sft;
        V.cshift = 1.5 - (double)D.k_lo;
        V.scale = (const float *)D.scale.p;
        V.era = D.has_antenna ? (const double *)D.era.p : nullptr;
        std::memcpy(V.arms.a, D.arms, sizeof V.arms.a);
        std::memcpy(V.arms.b, D.arms + 3, sizeof V.arms.b);
        n_seg_total += D.n_seg;
    }
    // evaluation order: f0 in 2^16 buckets over the list's range (a stable
    // counting sort), so that neighbouring lanes gather neighbouring columns;
    // every result goes to its list position, so the order changes none
    // the staging is pinned (the uploads run at DMA rate) and reused: wait for
    // the previous call's uploads from it first
    HIP_TRY(c, hipEventSynchronize(c->ev_h2d), "previous upload");
    int rc;
    if ((rc = ensure_pinned(c, c->h_list, (size_t)n * sizeof(ltgw_template), "template staging")) != LTGW_OK)
        return rc;
    if ((rc = ensure_pinned(c, c->h_perm, (size_t)n * 4, "template order staging")) != LTGW_OK) return rc;
    // Each chunk counts its keys per bucket and copies itself into the
    // staging; a bucket's positions then go to the chunks in list order, so
    // the scatter below gives the serial stable order.
    constexpr int kBuckets = 1 << 16;
    const double bscale = f0_max > f0_lo ? (kBuckets - 1) / (f0_max - f0_lo) : 0.0;
    std::vector<uint16_t> key((size_t)n);
    std::vector<int32_t> pos((size_t)nt * kBuckets, 0);  // [chunk][bucket]
    run_chunks(nt, [&](int t) {
        const int64_t lo = chunk_lo(n, nt, t), hi = chunk_lo(n, nt, t + 1);
        int32_t *cnt = pos.data() + (size_t)t * kBuckets;
        for (int64_t q = lo; q < hi; ++q) {
            const int b = (int)((tpl[q].f0 - f0_lo) * bscale);
            key[(size_t)q] = (uint16_t)(b < 0 ? 0 : b > kBuckets - 1 ? kBuckets - 1 : b);
            ++cnt[key[(size_t)q]];
        }
        std::memcpy((ltgw_template *)c->h_list.p + lo, tpl + lo, (size_t)(hi - lo) * sizeof(ltgw_template));
    });
    // the staging holds the whole list now: its upload runs while the host
    // finishes the order
    if ((rc = ensure(c, c->list_d, (size_t)n * sizeof(ltgw_template), "template list")) != LTGW_OK) return rc;
    if ((rc = ensure(c, c->perm_d, (size_t)n * 4, "template order")) != LTGW_OK) return rc;
    if ((rc = h2d(c, c->list_d.p, c->h_list.p, (size_t)n * sizeof(ltgw_template), "template upload")) != LTGW_OK)
        return rc;
    int32_t next = 0;
    for (int b = 0; b < kBuckets; ++b)
        for (int t = 0; t < nt; ++t) {
            int32_t &p = pos[(size_t)t * kBuckets + b];
            const int32_t m = p;
            p = next;
            next += m;
        }
    int32_t *perm = (int32_t *)c->h_perm.p;
    run_chunks(nt, [&](int t) {
        int32_t *at = pos.data() + (size_t)t * kBuckets;
        for (int64_t q = chunk_lo(n, nt, t), hi = chunk_lo(n, nt, t + 1); q < hi; ++q)
            perm[at[key[(size_t)q]]++] = (int32_t)q;
    });
    if ((rc = h2d(c, c->perm_d.p, c->h_perm.p, (size_t)n * 4, "template order upload")) != LTGW_OK) return rc;
    if ((rc = ensure(c, c->res_s, n * 8, "results s")) != LTGW_OK) return rc;
    if ((rc = ensure(c, c->res_c, n * 4, "results c")) != LTGW_OK) return rc;
    if ((rc = ensure(c, c->res_n, n * 4, "results N")) != LTGW_OK) return rc;
    if ((rc = ensure(c, c->res_w1, n * 8, "results W1")) != LTGW_OK) return rc;
    if ((rc = ensure(c, c->res_w2, n * 8, "results W2")) != LTGW_OK) return rc;
    if ((rc = zero_counter(c, kCntInBand, 1)) != LTGW_OK) return rc;
    a.n_det = n_slots;
    a.t0 = t0;
    a.tpl = (const ltgw_template *)c->list_d.p;
    a.perm = (const int32_t *)c->perm_d.p;
    a.n = n;
    a.s = (double *)c->res_s.p;
    a.c = (int32_t *)c->res_c.p;
    a.n_in = (int32_t *)c->res_n.p;
    a.w1 = (double *)c->res_w1.p;
    a.w2 = (double *)c->res_w2.p;
    a.out_s = out_s;
    a.out_c = out_c;
    a.out_n = out_n;
    a.in_band_total = (unsigned long long *)c->counters.p + kCntInBand;
    a.pow_counts = (unsigned long long *)c->counters.p + kCntUndecided;
    a.exact_count = (unsigned long long *)c->counters.p + kCntExact;
    // one sky direction for the whole list (and no antenna weights): each
    // detector's Doppler factors 1 + v.n/c as the lattice forms them (the
    // same operations in the same order), read per segment by the kernel
    bool any_ant = false;
    for (int q = 0; q < n_slots; ++q) any_ant = any_ant || a.det[q].era != nullptr;
    if (one_sky && !any_ant) {
        int64_t off = 0, tot = 0;
        for (int q = 0; q < n_slots; ++q) tot += c->det[slots[q]].n_seg;
        if ((rc = ensure(c, c->list_dop, (size_t)tot * 8, "list Doppler tables")) != LTGW_OK) return rc;
        if ((rc = ensure(c, c->list_sky, 3 * sizeof(double), "list sky")) != LTGW_OK) return rc;
        // from the context's host copy of the list (kept until the next upload has run)
        if ((rc = h2d(c, c->list_sky.p, ((const ltgw_template *)c->h_list.p)[0].sky, 3 * sizeof(double),
                      "list sky upload")) != LTGW_OK)
            return rc;
        for (int q = 0; q < n_slots; ++q) {
            const Det &D = c->det[slots[q]];
            double *dq = (double *)c->list_dop.p + off;
            HIP_TRY(c, launch_doppler((const double *)D.v.p, D.n_seg, (const double *)c->list_sky.p, 1, dq, c->stream),
                    "list Doppler launch");
            a.det[q].dop = dq;
            off += D.n_seg;
        }
    }
    HIP_TRY(c, hipEventRecord(c->ev_h2d, c->stream), "event record");
    HIP_TRY(c, hipEventRecord(c->ev[0], c->stream), "event record");
    HIP_TRY(c, hipEventRecord(c->ev[1], c->stream), "event record");
    HIP_TRY(c, launch_template_list(c->det[slots[0]].store, a, c->stream), "template list launch");
    HIP_TRY(c, hipEventRecord(c->ev[2], c->stream), "event record");
    c->have_eval = true;
    c->results_kept = true;
    c->list_mode = true;
    c->last_variant = -1;
    c->last_launches = 1;
    c->n_templates = n;
    c->n_evals = n * n_seg_total;
    c->rho_th = c->det[slots[0]].rho_th;
    return LTGW_OK;
}

int32_t ltgw_autotune(ltgw_ctx *c, const ltgw_grid *g, int32_t *best_variant) {
    if (!c) return LTGW_E_INVALID_ARG;
    Enter en(c);
    float best_ms = 0.0f;
    int best = -1;
    std::string key;
    for (int v = 0; v < kNumVariants; ++v) {
        int rc = eval_single(c, g, LTGW_STAT_POWER | LTGW_STAT_COUNT, nullptr, nullptr, nullptr, v);
        if (rc != LTGW_OK) return rc;
        HIP_TRY(c, hipEventSynchronize(c->ev[2]), "autotune");
        float ms = 0.0f;
        HIP_TRY(c, hipEventElapsedTime(&ms, c->ev[1], c->ev[2]), "autotune timing");
        if (best < 0 || ms < best_ms) {
            best = v;
            best_ms = ms;
        }
    }
    {
        int slots[32], n_slots = 0;
        for (int d = 0; d < 32 && n_slots < LTGW_MAX_SEARCH_DET; ++d)
            if (g->det_mask ? ((g->det_mask >> d) & 1u) : c->det[d].loaded) slots[n_slots++] = d;
        SearchPlan P;
        int rc = plan_search(c, g, slots, n_slots, P);
        if (rc != LTGW_OK) return rc;
        const Moments M = plan_moments(c, P.sel, P.n_sel);
        c->tune[tune_key_eval(P, M.mode == 2)] = best;
    }
    if (best_variant) *best_variant = best;
    c->have_eval = false;  // the last tuning run left results of a forced shape; evaluate again
    return LTGW_OK;
}

int32_t ltgw_set_tile_shape(ltgw_ctx *c, int32_t variant) {
    if (!c) return LTGW_E_INVALID_ARG;
    Enter en(c);
    if (variant < -1 || variant >= kNumVariants)
        return fail(c, LTGW_E_INVALID_ARG, "tile shape must be -1 or 0..%d", kNumVariants - 1);
    c->forced_variant = variant;
    free_batch(c->batch);  // a captured batch used the previous shape
    return LTGW_OK;
}

int32_t ltgw_tune_save(ltgw_ctx *c, const char *path) {
    if (!c) return LTGW_E_INVALID_ARG;
    Enter en(c);
    if (!path) return fail(c, LTGW_E_INVALID_ARG, "path is NULL");
    FILE *f = fopen(path, "w");
    if (!f) return fail(c, LTGW_E_INVALID_ARG, "cannot write %s", path);
    fprintf(f, "{\"ltgw_tune\": {");
    bool first = true;
    for (const auto &kv : c->tune) {
        fprintf(f, "%s\n  \"%s\": %d", first ? "" : ",", kv.first.c_str(), kv.second);
        first = false;
    }
    fprintf(f, "\n}}\n");
    fclose(f);
    return LTGW_OK;
}

int32_t ltgw_tune_load(ltgw_ctx *c, const char *path) {
    if (!c) return LTGW_E_INVALID_ARG;
    Enter en(c);
    if (!path) return fail(c, LTGW_E_INVALID_ARG, "path is NULL");
    FILE *f = fopen(path, "r");
    if (!f) return fail(c, LTGW_E_INVALID_ARG, "cannot read %s", path);
    std::string txt;
    char buf[4096];
    size_t n;
    while ((n = fread(buf, 1, sizeof buf, f)) > 0) txt.append(buf, n);
    fclose(f);
    // entries are "key": integer pairs after the top-level "ltgw_tune" key
    size_t pos = txt.find("\"ltgw_tune\"");
    if (pos == std::string::npos) return fail(c, LTGW_E_INVALID_ARG, "%s has no ltgw_tune object", path);
    pos = txt.find('{', pos);
    std::map<std::string, int> got;
    while (pos != std::string::npos) {
        const size_t k0 = txt.find('"', pos + 1);
        if (k0 == std::string::npos) break;
        const size_t k1 = txt.find('"', k0 + 1);
        if (k1 == std::string::npos) break;
        const size_t colon = txt.find(':', k1);
        if (colon == std::string::npos) break;
        char *end = nullptr;
        const long v = strtol(txt.c_str() + colon + 1, &end, 10);
        if (end == txt.c_str() + colon + 1 || v < 0 || v >= kNumVariants)
            return fail(c, LTGW_E_INVALID_ARG, "%s: bad tile shape for %s", path, txt.substr(k0 + 1, k1 - k0 - 1).c_str());
        got[txt.substr(k0 + 1, k1 - k0 - 1)] = (int)v;
        pos = txt.find_first_of(",}", (size_t)(end - txt.c_str()));
        if (pos == std::string::npos || txt[pos] == '}') break;
    }
    for (const auto &kv : got) c->tune[kv.first] = kv.second;
    return LTGW_OK;
}

int32_t ltgw_psi(ltgw_ctx *c, uint32_t stat, double *out) {
    if (!c) return LTGW_E_INVALID_ARG;
    Enter en(c);
    if (!c->have_eval || !c->results_kept) return fail(c, LTGW_E_STATE, "no evaluation to rank");
    if (stat != LTGW_STAT_POWER && stat != LTGW_STAT_COUNT) return fail(c, LTGW_E_INVALID_ARG, "stat must be POWER or COUNT");
    if (!out) return fail(c, LTGW_E_INVALID_ARG, "out_psi is NULL");
    const double q = std::exp(-(double)c->rho_th);
    HIP_TRY(c, launch_psi(stat, c->n_templates, (const double *)c->res_s.p, (const int32_t *)c->res_c.p,
                          (const int32_t *)c->res_n.p, (const double *)c->res_w1.p,
                          (const double *)c->res_w2.p, q, out, c->stream),
            "psi launch");
    return LTGW_OK;
}

int32_t ltgw_topk_candidates(ltgw_ctx *c, uint32_t stat, int32_t k, ltgw_candidate *out_host,
                             int32_t *n_out) {
    if (!c) return LTGW_E_INVALID_ARG;
    Enter en(c);
    if (!c->have_eval || !c->results_kept) return fail(c, LTGW_E_STATE, "no evaluation to rank");
    if (stat != LTGW_STAT_POWER && stat != LTGW_STAT_COUNT) return fail(c, LTGW_E_INVALID_ARG, "stat must be POWER or COUNT");
    if (k < 1 || k > LTGW_MAX_TOPK) return fail(c, LTGW_E_INVALID_ARG, "k must be in 1..%d", LTGW_MAX_TOPK);
    if (!out_host || !n_out) return fail(c, LTGW_E_INVALID_ARG, "output pointers are NULL");
    const int64_t cap = topk_scratch_entries(c->n_templates, k);
    int rc;
    if ((rc = ensure(c, c->cand_pa, cap * 8, "top-k scratch")) != LTGW_OK) return rc;
    if ((rc = ensure(c, c->cand_ia, cap * 8, "top-k scratch")) != LTGW_OK) return rc;
    if ((rc = ensure(c, c->cand_pb, cap * 8, "top-k scratch")) != LTGW_OK) return rc;
    if ((rc = ensure(c, c->cand_ib, cap * 8, "top-k scratch")) != LTGW_OK) return rc;
    if ((rc = ensure(c, c->cand_out, (size_t)k * sizeof(ltgw_candidate), "top-k records")) != LTGW_OK) return rc;
    if ((rc = ensure(c, c->n_out, 8, "top-k count")) != LTGW_OK) return rc;
    TopkDecode dec;
    dec.f0_min = c->f0_min;
    dec.f0_step = c->f0_step;
    dec.n_f0 = c->n_f0;
    dec.n_tau = c->n_tau;
    dec.n_brake = c->n_brake;
    dec.tau = (const double *)c->tau_d.p;
    dec.brake = (const double *)c->brake_d.p;
    dec.list = c->list_mode ? (const ltgw_template *)c->list_d.p : nullptr;
    const double q = std::exp(-(double)c->rho_th);
    HIP_TRY(c, launch_topk(stat, c->n_templates, (const double *)c->res_s.p, (const int32_t *)c->res_c.p,
                           (const int32_t *)c->res_n.p, (const double *)c->res_w1.p,
                           (const double *)c->res_w2.p, q, k, (double *)c->cand_pa.p,
                           (int64_t *)c->cand_ia.p, (double *)c->cand_pb.p, (int64_t *)c->cand_ib.p,
                           cap, dec, (ltgw_candidate *)c->cand_out.p, (int32_t *)c->n_out.p, c->stream),
            "top-k launch");
    HIP_TRY(c, hipMemcpyAsync(out_host, c->cand_out.p, (size_t)k * sizeof(ltgw_candidate),
                              hipMemcpyDeviceToHost, c->stream),
            "top-k download");
    HIP_TRY(c, hipMemcpyAsync(n_out, c->n_out.p, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream),
            "top-k download");
    HIP_TRY(c, hipStreamSynchronize(c->stream), "top-k");
    return LTGW_OK;
}

int32_t ltgw_diagnostics(ltgw_ctx *c, ltgw_diag *out) {
    if (!c) return LTGW_E_INVALID_ARG;
    Enter en(c);
    if (!out) return fail(c, LTGW_E_INVALID_ARG, "out is NULL");
    unsigned long long v[kNumCnt];
    HIP_TRY(c, hipMemcpyAsync(v, c->counters.p, sizeof v, hipMemcpyDeviceToHost, c->stream), "diagnostics");
    HIP_TRY(c, hipStreamSynchronize(c->stream), "diagnostics");
    out->pow_undecided = (int64_t)v[kCntUndecided];
    out->pow_slow = (int64_t)v[kCntSlow];
    out->pow_exact = (int64_t)v[kCntExact];
    out->templates = c->have_eval ? c->n_templates : 0;
    out->evals = c->have_eval ? c->n_evals : 0;
    out->in_band = c->have_eval ? (int64_t)v[kCntInBand] : 0;
    out->eval_kernel_ms = 0.0;
    out->tables_ms = 0.0;
    out->tile_shape = c->have_eval ? c->last_variant : -1;
    out->eval_launches = c->have_eval ? c->last_launches : 0;
    out->ingest_ms = 0.0;
    if (c->have_ingest) {
        float a = 0.f;
        if (hipEventElapsedTime(&a, c->ev_ing[0], c->ev_ing[1]) == hipSuccess) out->ingest_ms = a;
        (void)hipGetLastError();
    }
    if (c->have_eval) {
        float a = 0.f, b = 0.f;
        if (hipEventElapsedTime(&a, c->ev[1], c->ev[2]) == hipSuccess) out->eval_kernel_ms = a;
        if (hipEventElapsedTime(&b, c->ev[0], c->ev[1]) == hipSuccess) out->tables_ms = b;
        (void)hipGetLastError();
    }
    return LTGW_OK;
}

int32_t ltgw_inject_track(ltgw_ctx *c, int32_t det, float *power, double f0, double tau,
                          double brake, const double *sky3, double t0, float amp) {
    if (!c) return LTGW_E_INVALID_ARG;
    Enter en(c);
    if (det < 0 || det >= LTGW_MAX_DET) return fail(c, LTGW_E_INVALID_ARG, "detector %d out of range", det);
    Det &D = c->det[det];
    if (!D.loaded || !D.has_v) return fail(c, LTGW_E_STATE, "detector %d needs a spectrogram and a velocity table", det);
    if (!power || !sky3) return fail(c, LTGW_E_INVALID_ARG, "power or sky is NULL");
    if (!is_device_ptr(power)) return fail(c, LTGW_E_INVALID_ARG, "power must be a device buffer");
    if (!fin(f0) || !(f0 > 0.0) || !fin(tau) || !(tau > 0.0) || !fin(brake) || !(brake > 1.0) ||
        !fin(t0) || !std::isfinite(amp))
        return fail(c, LTGW_E_INVALID_ARG, "invalid template parameters");
    const double n2 = sky3[0] * sky3[0] + sky3[1] * sky3[1] + sky3[2] * sky3[2];
    if (!fin(n2) || std::fabs(std::sqrt(n2) - 1.0) > 1e-12) return fail(c, LTGW_E_INVALID_ARG, "sky is not a unit vector");
    if (!(f0 * D.t_sft * (1.0 + D.v_max) < (double)(1 << 30))) return fail(c, LTGW_E_INVALID_ARG, "f0 too large");
    HIP_TRY(c, launch_inject(power, D.n_seg, D.n_bins, D.k_lo, D.t_sft, (const double *)D.t_seg.p,
                             (const double *)D.v.p, (const float *)D.w.p, f0, tau, brake, sky3[0],
                             sky3[1], sky3[2], t0, amp,
                             (unsigned long long *)c->counters.p + kCntUndecided, c->stream),
            "inject launch");
    return LTGW_OK;
}

int32_t ltgw_read_tables(ltgw_ctx *c, int32_t det, double *g_host, double *h_host, int32_t *n_rows) {
    if (!c) return LTGW_E_INVALID_ARG;
    Enter en(c);
    if (det < 0 || det >= LTGW_MAX_DET) return fail(c, LTGW_E_INVALID_ARG, "detector %d out of range", det);
    const Det &D = c->det[det];
    if (!D.loaded || D.tab_n_tn == 0) return fail(c, LTGW_E_STATE, "detector %d has no tables of an evaluation", det);
    if (n_rows) {
        n_rows[0] = D.tab_n_tn;
        n_rows[1] = D.tab_n_groups;
    }
    if (g_host)
        HIP_TRY(c, hipMemcpyAsync(g_host, D.g.p, (size_t)D.tab_n_tn * D.n_seg * 8, hipMemcpyDeviceToHost, c->stream),
                "spin-factor table download");
    if (h_host)
        HIP_TRY(c, hipMemcpyAsync(h_host, D.H.p, (size_t)D.tab_n_groups * D.n_seg * 8, hipMemcpyDeviceToHost,
                                  c->stream),
                "track-factor table download");
    HIP_TRY(c, hipStreamSynchronize(c->stream), "table download");
    return LTGW_OK;
}

int32_t ltgw_read_store(ltgw_ctx *c, int32_t det, void *out_host, float *scale_host) {
    if (!c) return LTGW_E_INVALID_ARG;
    Enter en(c);
    if (det < 0 || det >= LTGW_MAX_DET) return fail(c, LTGW_E_INVALID_ARG, "detector %d out of range", det);
    Det &D = c->det[det];
    if (!D.loaded) return fail(c, LTGW_E_STATE, "no spectrogram loaded for detector %d", det);
    if (!out_host) return fail(c, LTGW_E_INVALID_ARG, "out_host is NULL");
    const size_t es = D.store == LTGW_STORE_F32 ? 4 : D.store == LTGW_STORE_BF16 ? 2 : 1;
    HIP_TRY(c, hipMemcpy2DAsync(out_host, (size_t)D.n_bins * es, (const char *)D.store_buf.p + es,
                                (size_t)D.pitch * es, (size_t)D.n_bins * es, (size_t)D.n_seg,
                                hipMemcpyDeviceToHost, c->stream),
            "store download");
    if (scale_host)
        HIP_TRY(c, hipMemcpyAsync(scale_host, D.scale.p, (size_t)D.n_seg * 4, hipMemcpyDeviceToHost, c->stream),
                "scale download");
    HIP_TRY(c, hipStreamSynchronize(c->stream), "store download");
    return LTGW_OK;
}

}  // extern "C"
