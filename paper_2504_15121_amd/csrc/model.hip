// Model files of the learned denoiser: the FP32 parameters, the Adam moments and
// the optimiser step in one versioned binary file with a CRC-32, read and
// written by the library itself so that C callers need no other format code.
// The layout is stated in snx.h.  Saving writes a temporary file next to the
// target and renames it over the target, so a file on disk is always complete.
#include <stdio.h>
#include <string.h>

#include <new>
#include <string>
#include <vector>

#include "snx_internal.hpp"

namespace snx {
snx_status api_failf(snx_status st, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
snx_status api_hip_fail(hipError_t e, const char *where);
void api_clear();
}  // namespace snx

namespace {

constexpr char kMagic[4] = {'S', 'N', 'X', 'M'};
constexpr uint32_t kVersion = 1;
constexpr size_t kHeader = 40;
constexpr uint32_t kFlagMoments = 1u;

// CRC-32 with the reflected IEEE 802.3 polynomial 0xEDB88320, initial value and
// final xor 0xFFFFFFFF (the checksum of zlib's crc32 and of PNG), table-driven.
struct CrcTable {
    uint32_t t[256];
    CrcTable()
    {
        for (uint32_t i = 0; i < 256; ++i) {
            uint32_t c = i;
            for (int k = 0; k < 8; ++k) c = (c & 1u) ? 0xEDB88320u ^ (c >> 1) : c >> 1;
            t[i] = c;
        }
    }
};

uint32_t crc32(const unsigned char *p, size_t n)
{
    static const CrcTable table;
    uint32_t c = 0xFFFFFFFFu;
    for (size_t i = 0; i < n; ++i) c = table.t[(c ^ p[i]) & 0xFFu] ^ (c >> 8);
    return c ^ 0xFFFFFFFFu;
}

template <class T>
void put(std::vector<unsigned char> &b, size_t at, T v)
{
    memcpy(b.data() + at, &v, sizeof v);
}

template <class T>
T get(const std::vector<unsigned char> &b, size_t at)
{
    T v;
    memcpy(&v, b.data() + at, sizeof v);
    return v;
}

}  // namespace

struct snx_model {
    std::vector<float> params, m, v;   // m, v empty when the model has no Adam state
    snx_model_info info;
    // device copies made by snx_model_bind (owned, freed by snx_model_destroy)
    float *d_params = nullptr;
    void *d_packed = nullptr;
    void *d_ws = nullptr;
    size_t ws_bytes = 0;
};

extern "C" {

snx_status snx_model_create(const float *params, const float *adam_m, const float *adam_v,
                            const snx_model_info *info, snx_model **model)
{
    snx::api_clear();
    if (!model) return snx::api_failf(SNX_ERR_ARG, "model is NULL");
    *model = nullptr;
    if (!params) return snx::api_failf(SNX_ERR_ARG, "params is NULL");
    if (!adam_m != !adam_v) return snx::api_failf(SNX_ERR_ARG, "give both Adam moments or neither");
    const size_t n = (size_t)snx_cnn_param_count();
    snx_model *md = new (std::nothrow) snx_model();
    if (!md) return snx::api_failf(SNX_ERR_ARG, "out of host memory");
    md->params.assign(params, params + n);
    if (adam_m) {
        md->m.assign(adam_m, adam_m + n);
        md->v.assign(adam_v, adam_v + n);
    }
    md->info = info ? *info : snx_model_info{};
    md->info.has_moments = adam_m ? 1 : 0;
    *model = md;
    return SNX_OK;
}

snx_status snx_model_load(const char *path, snx_model **model)
{
    snx::api_clear();
    if (!model) return snx::api_failf(SNX_ERR_ARG, "model is NULL");
    *model = nullptr;
    if (!path) return snx::api_failf(SNX_ERR_ARG, "path is NULL");
    FILE *f = fopen(path, "rb");
    if (!f) return snx::api_failf(SNX_ERR_IO, "cannot open %s", path);
    std::vector<unsigned char> b;
    unsigned char chunk[1 << 16];
    size_t got;
    while ((got = fread(chunk, 1, sizeof chunk, f)) > 0) b.insert(b.end(), chunk, chunk + got);
    const bool rd_err = ferror(f) != 0;
    fclose(f);
    if (rd_err) return snx::api_failf(SNX_ERR_IO, "read error on %s", path);
    if (b.size() < kHeader + 4) return snx::api_failf(SNX_ERR_MODEL, "%s: truncated header", path);
    if (memcmp(b.data(), kMagic, 4) != 0) return snx::api_failf(SNX_ERR_MODEL, "%s: not a model file", path);
    const uint32_t version = get<uint32_t>(b, 4);
    if (version != kVersion)
        return snx::api_failf(SNX_ERR_MODEL, "%s: version %u (this library reads %u)", path, version,
                        kVersion);
    const uint32_t n = get<uint32_t>(b, 8), flags = get<uint32_t>(b, 12);
    if (n != (uint32_t)snx_cnn_param_count())
        return snx::api_failf(SNX_ERR_MODEL, "%s: %u parameters (the network has %d)", path, n,
                        snx_cnn_param_count());
    if (flags & ~kFlagMoments) return snx::api_failf(SNX_ERR_MODEL, "%s: unknown flags %#x", path, flags);
    const size_t arrays = (flags & kFlagMoments) ? 3 : 1;
    const size_t want = kHeader + arrays * (size_t)n * sizeof(float) + 4;
    if (b.size() != want)
        return snx::api_failf(SNX_ERR_MODEL, "%s: %zu bytes, expected %zu (truncated or padded)", path,
                        b.size(), want);
    if (crc32(b.data(), want - 4) != get<uint32_t>(b, want - 4))
        return snx::api_failf(SNX_ERR_MODEL, "%s: CRC mismatch", path);
    snx_model *md = new (std::nothrow) snx_model();
    if (!md) return snx::api_failf(SNX_ERR_ARG, "out of host memory");
    md->info.step = get<int64_t>(b, 16);
    md->info.normal_window = get<int32_t>(b, 24);
    md->info.seed = get<int32_t>(b, 28);
    md->info.fidelity = get<float>(b, 32);
    md->info.has_moments = (flags & kFlagMoments) ? 1 : 0;
    const float *p = reinterpret_cast<const float *>(b.data() + kHeader);
    md->params.assign(p, p + n);
    if (arrays == 3) {
        md->m.assign(p + n, p + 2 * (size_t)n);
        md->v.assign(p + 2 * (size_t)n, p + 3 * (size_t)n);
    }
    *model = md;
    return SNX_OK;
}

snx_status snx_model_save(const snx_model *model, const char *path)
{
    snx::api_clear();
    if (!model || !path) return snx::api_failf(SNX_ERR_ARG, "model or path is NULL");
    const size_t n = model->params.size();
    const bool mom = !model->m.empty();
    const size_t arrays = mom ? 3 : 1;
    std::vector<unsigned char> b(kHeader + arrays * n * sizeof(float) + 4, 0);
    memcpy(b.data(), kMagic, 4);
    put<uint32_t>(b, 4, kVersion);
    put<uint32_t>(b, 8, (uint32_t)n);
    put<uint32_t>(b, 12, mom ? kFlagMoments : 0u);
    put<int64_t>(b, 16, model->info.step);
    put<int32_t>(b, 24, model->info.normal_window);
    put<int32_t>(b, 28, model->info.seed);
    put<float>(b, 32, model->info.fidelity);
    memcpy(b.data() + kHeader, model->params.data(), n * sizeof(float));
    if (mom) {
        memcpy(b.data() + kHeader + n * sizeof(float), model->m.data(), n * sizeof(float));
        memcpy(b.data() + kHeader + 2 * n * sizeof(float), model->v.data(), n * sizeof(float));
    }
    put<uint32_t>(b, b.size() - 4, crc32(b.data(), b.size() - 4));
    const std::string tmp = std::string(path) + ".tmp";
    FILE *f = fopen(tmp.c_str(), "wb");
    if (!f) return snx::api_failf(SNX_ERR_IO, "cannot create %s", tmp.c_str());
    const bool ok = fwrite(b.data(), 1, b.size(), f) == b.size() && fflush(f) == 0;
    if (fclose(f) != 0 || !ok) {
        remove(tmp.c_str());
        return snx::api_failf(SNX_ERR_IO, "write error on %s", tmp.c_str());
    }
    if (rename(tmp.c_str(), path) != 0) {
        remove(tmp.c_str());
        return snx::api_failf(SNX_ERR_IO, "cannot rename %s to %s", tmp.c_str(), path);
    }
    return SNX_OK;
}

snx_status snx_model_read(const snx_model *model, float *params, float *adam_m, float *adam_v,
                          snx_model_info *info)
{
    snx::api_clear();
    if (!model) return snx::api_failf(SNX_ERR_ARG, "model is NULL");
    if ((adam_m || adam_v) && model->m.empty())
        return snx::api_failf(SNX_ERR_MODEL, "the model holds no Adam moments");
    const size_t n = model->params.size();
    if (params) memcpy(params, model->params.data(), n * sizeof(float));
    if (adam_m) memcpy(adam_m, model->m.data(), n * sizeof(float));
    if (adam_v) memcpy(adam_v, model->v.data(), n * sizeof(float));
    if (info) *info = model->info;
    return SNX_OK;
}

snx_status snx_model_bind(snx_model *model, int32_t width, int32_t height, void *stream,
                          snx_cnn_model *view)
{
    snx::api_clear();
    if (!model || !view) return snx::api_failf(SNX_ERR_ARG, "model or view is NULL");
    const size_t need = snx_cnn_workspace_size(width, height, 1, 0);
    if (width <= 0 || height <= 0 || need == 0)
        return snx::api_failf(SNX_ERR_ARG, "bad frame size %d x %d", width, height);
    hipError_t e = hipSuccess;
    const size_t pbytes = model->params.size() * sizeof(float);
    if (!model->d_params) {
        if ((e = hipMalloc((void **)&model->d_params, pbytes)) != hipSuccess ||
            (e = hipMalloc(&model->d_packed, snx_cnn_packed_bytes())) != hipSuccess)
            return snx::api_hip_fail(e, "snx_model_bind");
    }
    if (model->ws_bytes < need) {
        if (model->d_ws && (e = hipFree(model->d_ws)) != hipSuccess)
            return snx::api_hip_fail(e, "snx_model_bind");
        model->d_ws = nullptr;
        model->ws_bytes = 0;
        if ((e = hipMalloc(&model->d_ws, need)) != hipSuccess) return snx::api_hip_fail(e, "snx_model_bind");
        model->ws_bytes = need;
    }
    hipStream_t s = (hipStream_t)stream;
    if ((e = hipMemcpyAsync(model->d_params, model->params.data(), pbytes, hipMemcpyHostToDevice,
                            s)) != hipSuccess)
        return snx::api_hip_fail(e, "snx_model_bind");
    const snx_status st = snx_cnn_pack(model->d_params, model->d_packed, stream);
    if (st != SNX_OK) return st;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return snx::api_hip_fail(e, "snx_model_bind");
    view->params = model->d_params;
    view->packed = model->d_packed;
    view->workspace = model->d_ws;
    view->workspace_bytes = model->ws_bytes;
    return SNX_OK;
}

snx_status snx_model_destroy(snx_model *model)
{
    snx::api_clear();
    if (!model) return SNX_OK;
    hipError_t e = hipSuccess, e2;
    if (model->d_params && (e2 = hipFree(model->d_params)) != hipSuccess) e = e2;
    if (model->d_packed && (e2 = hipFree(model->d_packed)) != hipSuccess) e = e2;
    if (model->d_ws && (e2 = hipFree(model->d_ws)) != hipSuccess) e = e2;
    delete model;
    return e == hipSuccess ? SNX_OK : snx::api_hip_fail(e, "snx_model_destroy");
}

}  // extern "C"
