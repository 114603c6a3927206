// File form of the ranking network (ltgw_proposer_save / ltgw_proposer_load):
// host code only.  Layout, little-endian:
//   bytes  0..7   magic "LTGWCNN" and a zero byte
//   bytes  8..11  uint32 format version (1)
//   bytes 12..27  int32 c_in, c_out, width, taps (width 32, taps 5)
//   bytes 28..31  zero
//   bytes 32..39  int64 parameter count (ltgw_cnn_param_count(c_in, c_out))
//   bytes 40..47  uint64 FNV-1a (64-bit) hash of the parameter bytes
//   bytes 48..63  zero
//   bytes 64..    FP32 parameters W1 b1 W2 b2 W3 b3 W4 b4, as ltgw_cnn_forward takes them
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "ltgw_ctx.h"
#include "ltgw_proposer.h"

using namespace ltgw;

namespace {

constexpr char kMagic[8] = {'L', 'T', 'G', 'W', 'C', 'N', 'N', 0};
constexpr uint32_t kVersion = 1;
constexpr int32_t kWidth = 32, kTaps = 5;
constexpr size_t kHeader = 64;

uint64_t fnv1a64(const unsigned char *p, size_t n) {
    uint64_t h = 14695981039346656037ull;  // FNV-1a offset basis and prime (Fowler, Noll, Vo)
    for (size_t i = 0; i < n; ++i) {
        h ^= p[i];
        h *= 1099511628211ull;
    }
    return h;
}

struct Header {
    char magic[8];
    uint32_t version;
    int32_t c_in, c_out, width, taps, zero0;
    int64_t n_params;
    uint64_t hash;
    unsigned char zero1[16];
};
static_assert(sizeof(Header) == kHeader, "header layout");

struct File {
    FILE *f = nullptr;
    ~File() {
        if (f) std::fclose(f);
    }
};

bool shape_ok(int32_t c_in, int32_t c_out) { return c_in >= 1 && c_out >= 1 && c_in <= 4096 && c_out <= 4096; }

// params (n floats) into host memory: device memory through the context's
// stream, host memory (always, when c is NULL) by a plain copy
int params_to_host(ltgw_ctx *c, float *dst, const float *src, int64_t n) {
    if (c) return to_host(c, dst, src, (size_t)n * 4, "network parameters to host");
    std::memcpy(dst, src, (size_t)n * 4);
    return LTGW_OK;
}

int params_from_host(ltgw_ctx *c, float *dst, const float *src, int64_t n) {
    if (c && is_device_ptr(dst)) {
        HIP_TRY(c, hipMemcpyAsync(dst, src, (size_t)n * 4, hipMemcpyHostToDevice, c->stream), "network upload");
        HIP_TRY(c, hipStreamSynchronize(c->stream), "network upload");
        return LTGW_OK;
    }
    std::memcpy(dst, src, (size_t)n * 4);
    return LTGW_OK;
}

}  // namespace

extern "C" {

int32_t ltgw_proposer_save(ltgw_ctx *c, const char *path, const float *params, int32_t c_in, int32_t c_out) {
    Enter en(c);
    if (!path || !params) return fail(c, LTGW_E_INVALID_ARG, "ltgw_proposer_save: path and params are required");
    if (!shape_ok(c_in, c_out)) return fail(c, LTGW_E_INVALID_ARG, "ltgw_proposer_save: c_in, c_out must be 1 .. 4096");
    const int64_t n = cnn_n_params(c_in, c_out);
    std::vector<float> h((size_t)n);
    int rc = params_to_host(c, h.data(), params, n);
    if (rc != LTGW_OK) return rc;
    Header hd;
    std::memset(&hd, 0, sizeof hd);
    std::memcpy(hd.magic, kMagic, sizeof kMagic);
    hd.version = kVersion;
    hd.c_in = c_in;
    hd.c_out = c_out;
    hd.width = kWidth;
    hd.taps = kTaps;
    hd.n_params = n;
    hd.hash = fnv1a64((const unsigned char *)h.data(), (size_t)n * 4);
    // written beside the target and renamed over it, so a reader never sees half a file
    const std::string tmp = std::string(path) + ".tmp";
    {
        File f;
        f.f = std::fopen(tmp.c_str(), "wb");
        if (!f.f) return fail(c, LTGW_E_IO, "ltgw_proposer_save: cannot open %s for writing", tmp.c_str());
        if (std::fwrite(&hd, sizeof hd, 1, f.f) != 1 || std::fwrite(h.data(), 4, (size_t)n, f.f) != (size_t)n ||
            std::fflush(f.f) != 0) {
            std::fclose(f.f);
            f.f = nullptr;
            std::remove(tmp.c_str());
            return fail(c, LTGW_E_IO, "ltgw_proposer_save: write to %s failed", tmp.c_str());
        }
        if (std::fclose(f.f) != 0) {
            f.f = nullptr;
            std::remove(tmp.c_str());
            return fail(c, LTGW_E_IO, "ltgw_proposer_save: write to %s failed", tmp.c_str());
        }
        f.f = nullptr;
    }
    if (std::rename(tmp.c_str(), path) != 0) {
        std::remove(tmp.c_str());
        return fail(c, LTGW_E_IO, "ltgw_proposer_save: cannot rename %s to %s", tmp.c_str(), path);
    }
    return LTGW_OK;
}

int32_t ltgw_proposer_load(ltgw_ctx *c, const char *path, int32_t *c_in, int32_t *c_out, float *params,
                           int64_t n_params) {
    Enter en(c);
    if (!path) return fail(c, LTGW_E_INVALID_ARG, "ltgw_proposer_load: path is required");
    File f;
    f.f = std::fopen(path, "rb");
    if (!f.f) return fail(c, LTGW_E_IO, "ltgw_proposer_load: cannot open %s", path);
    Header hd;
    if (std::fread(&hd, sizeof hd, 1, f.f) != 1)
        return fail(c, LTGW_E_IO, "ltgw_proposer_load: %s is shorter than the %zu-byte header", path, kHeader);
    if (std::memcmp(hd.magic, kMagic, sizeof kMagic) != 0)
        return fail(c, LTGW_E_IO, "ltgw_proposer_load: %s is not a network file (magic)", path);
    if (hd.version != kVersion)
        return fail(c, LTGW_E_UNSUPPORTED, "ltgw_proposer_load: %s has format version %u (this library reads %u)", path,
                    hd.version, kVersion);
    if (!shape_ok(hd.c_in, hd.c_out) || hd.width != kWidth || hd.taps != kTaps ||
        hd.n_params != cnn_n_params(hd.c_in, hd.c_out))
        return fail(c, LTGW_E_IO, "ltgw_proposer_load: %s has an inconsistent shape (c_in %d, c_out %d, width %d, "
                    "taps %d, %lld parameters)", path, hd.c_in, hd.c_out, hd.width, hd.taps, (long long)hd.n_params);
    if (c_in) *c_in = hd.c_in;
    if (c_out) *c_out = hd.c_out;
    if (!params) return LTGW_OK;  // shape query
    if (n_params != hd.n_params)
        return fail(c, LTGW_E_INVALID_ARG, "ltgw_proposer_load: the buffer holds %lld parameters, the file %lld",
                    (long long)n_params, (long long)hd.n_params);
    std::vector<float> h((size_t)hd.n_params);
    if (std::fread(h.data(), 4, h.size(), f.f) != h.size())
        return fail(c, LTGW_E_IO, "ltgw_proposer_load: %s is truncated", path);
    if (std::fgetc(f.f) != EOF) return fail(c, LTGW_E_IO, "ltgw_proposer_load: %s has bytes past the parameters", path);
    if (fnv1a64((const unsigned char *)h.data(), h.size() * 4) != hd.hash)
        return fail(c, LTGW_E_IO, "ltgw_proposer_load: %s fails its checksum", path);
    return params_from_host(c, params, h.data(), hd.n_params);
}

}  // extern "C"
