// C ABI of the learned denoiser: validation, workspace carving and launches.
#include <math.h>
#include <stdint.h>
#include <string.h>

#include "snx_cnn.hpp"

namespace snx {
snx_status api_fail(snx_status st, const char *msg);
snx_status api_hip_fail(hipError_t e, const char *where);
}  // namespace snx

namespace {

using snx::api_fail;
using snx::api_hip_fail;

size_t al(size_t x) { return (x + 255) / 256 * 256; }

struct CnnWs {
    float *mu, *dt, *coefA, *coefB, *coefOwn, *grad_y, *partial, *inv_n;
    uint16_t *acts[5], *gbuf[2];
    double *part_loss;
    int *part_used;
    size_t bytes;
};

// Carve the workspace; with base == nullptr only the size is computed.
CnnWs carve(char *base, int W, int H, int B, bool training)
{
    CnnWs w;
    memset(&w, 0, sizeof w);
    const size_t px = (size_t)W * H * B;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char *p = base ? base + off : nullptr;
        off += al(bytes);
        return p;
    };
    w.mu = (float *)take(px * 4);
    // inference keeps every activation in LDS (fused kernel): only mu is needed
    if (training) {
        for (int i = 0; i < 5; ++i) w.acts[i] = (uint16_t *)take(px * 64);
        for (int i = 0; i < 2; ++i) w.gbuf[i] = (uint16_t *)take(px * 64);
        w.dt = (float *)take(px * 4);
        w.coefA = (float *)take(px * 4);
        w.coefB = (float *)take(px * 4);
        w.coefOwn = (float *)take(px * 4);
        w.grad_y = (float *)take(px * 4);
        w.partial = (float *)take((size_t)snx::cnn_partial_blocks(W, H, B) * snx::kLayerParams[1] * 4);
        const size_t hb = (size_t)snx::cnn_head_blocks(W, H, B);
        w.part_loss = (double *)take(hb * 16);
        w.part_used = (int *)take(hb * 8);
        w.inv_n = (float *)take(8);
    }
    w.bytes = off;
    return w;
}

bool aligned16(const void *p) { return ((uintptr_t)p & 15) == 0; }

bool dims_ok(int32_t w, int32_t h, int32_t b)
{
    return w > 0 && h > 0 && b > 0 && (int64_t)w * h * b < (1LL << 31);
}

snx_status run_mu(const float *disp, int64_t stride, int W, int H, int B, int64_t crop_stride,
                  float *mu, hipStream_t s)
{
    for (int b = 0; b < B; ++b) {
        snx::StencilArgs a;
        memset(&a, 0, sizeof a);
        a.src = disp + (int64_t)b * crop_stride;
        a.ld_src = stride;
        a.W = W;
        a.H = H;
        a.rf = 1;
        a.rg = 0;
        a.need_f = 3;
        a.dn = mu + (int64_t)b * W * H;
        a.ld_dn = W;
        a.th = snx::stencil_pick_tile_height(1, 0);
        hipError_t e = snx::launch_stencil(a, s);
        if (e != hipSuccess) return api_hip_fail(e, "cnn filter");
    }
    return SNX_OK;
}

}  // namespace

extern "C" {

int32_t snx_cnn_param_count(void) { return snx::kCnnParams; }
size_t snx_cnn_packed_bytes(void) { return (size_t)snx::kPackedElems * 2; }

size_t snx_cnn_workspace_size(int32_t width, int32_t height, int32_t batch, int32_t training)
{
    if (!dims_ok(width, height, batch)) return 0;
    return carve(nullptr, width, height, batch, training != 0).bytes;
}

snx_status snx_cnn_pack(const float *params, void *packed, void *stream)
{
    if (!params || !packed) return api_fail(SNX_ERR_ARG, "params or packed is NULL");
    if (!aligned16(params) || !aligned16(packed))
        return api_fail(SNX_ERR_ARG, "params and packed must be 16-byte aligned");
    hipError_t e = snx::cnn_pack(params, (uint16_t *)packed, (hipStream_t)stream);
    return e == hipSuccess ? SNX_OK : api_hip_fail(e, "snx_cnn_pack");
}

snx_status snx_cnn_denoise(const float *disp, int64_t stride, int32_t width, int32_t height,
                           const snx_cnn_model *model, float *out, int64_t out_stride,
                           void *stream)
{
    if (width == 0 || height == 0) return SNX_OK;
    if (!dims_ok(width, height, 1)) return api_fail(SNX_ERR_ARG, "bad size");
    if (!disp || !out || stride < width || out_stride < width)
        return api_fail(SNX_ERR_ARG, "disp/out NULL or stride < width");
    if (!model || !model->params || !model->packed || !model->workspace)
        return api_fail(SNX_ERR_MODEL, "model, params, packed or workspace is NULL");
    if (!aligned16(model->params) || !aligned16(model->packed) || !aligned16(model->workspace))
        return api_fail(SNX_ERR_ARG, "model buffers must be 16-byte aligned");
    const CnnWs w0 = carve(nullptr, width, height, 1, false);
    if (model->workspace_bytes < w0.bytes) return api_fail(SNX_ERR_WORKSPACE, "cnn workspace too small");
    const CnnWs w = carve((char *)model->workspace, width, height, 1, false);
    hipStream_t s = (hipStream_t)stream;
    snx_status st = run_mu(disp, stride, width, height, 1, 0, w.mu, s);
    if (st) return st;
    snx::CnnFusedArgs f;
    memset(&f, 0, sizeof f);
    f.W = width;
    f.H = height;
    f.D = disp;
    f.ldD = stride;
    f.mu = w.mu;
    f.params = model->params;
    f.packed = (const uint16_t *)model->packed;
    f.out = out;
    f.ld_out = out_stride;
    f.s = snx::kCnnScale;
    hipError_t e = snx::cnn_forward_fused(f, s);
    return e == hipSuccess ? SNX_OK : api_hip_fail(e, "snx_cnn_denoise");
}

snx_status snx_cnn_train_step(const float *disp, const float *normals, const float *clean,
                              float fidelity, const snx_camera *cams,
                              int32_t width, int32_t height, int32_t batch,
                              int32_t normal_window, float *params, void *packed, float *grad,
                              float *adam_m, float *adam_v, int32_t step, float lr,
                              float beta1, float beta2, float eps, double *loss_out,
                              void *workspace, size_t workspace_bytes, void *stream)
{
    if (!dims_ok(width, height, batch)) return api_fail(SNX_ERR_ARG, "bad size");
    if (batch > snx::kCnnMaxBatch) return api_fail(SNX_ERR_UNSUPPORTED, "batch > 64");
    if (!disp || !normals || !cams || !params || !packed || !grad || !loss_out)
        return api_fail(SNX_ERR_ARG, "NULL argument");
    if (!aligned16(params) || !aligned16(packed) || !aligned16(workspace))
        return api_fail(SNX_ERR_ARG, "params, packed and workspace must be 16-byte aligned");
    if (step < 0 || (step > 0 && (!adam_m || !adam_v)))
        return api_fail(SNX_ERR_ARG, "step < 0 or Adam moments missing");
    if (!(isfinite(fidelity) && fidelity >= 0))
        return api_fail(SNX_ERR_ARG, "fidelity weight must be finite and >= 0");
    if (normal_window < 3 || normal_window % 2 == 0 || normal_window > 63)
        return api_fail(SNX_ERR_ARG, "normal_window must be odd, 3..63");
    for (int b = 0; b < batch; ++b)
        if (!(cams[b].fx > 0) || !(cams[b].fy > 0) || !isfinite(cams[b].u0) || !isfinite(cams[b].v0))
            return api_fail(SNX_ERR_ARG, "bad camera");
    if (step > 0 && !(lr >= 0 && beta1 >= 0 && beta1 < 1 && beta2 >= 0 && beta2 < 1 && eps > 0))
        return api_fail(SNX_ERR_ARG, "bad Adam hyper-parameters");
    const CnnWs w0 = carve(nullptr, width, height, batch, true);
    if (!workspace || workspace_bytes < w0.bytes) return api_fail(SNX_ERR_WORKSPACE, "cnn workspace too small");
    const CnnWs w = carve((char *)workspace, width, height, batch, true);
    hipStream_t s = (hipStream_t)stream;
    const int64_t plane = (int64_t)width * height;

    snx_status st = run_mu(disp, width, width, height, batch, plane, w.mu, s);
    if (st) return st;
    snx::CnnForwardArgs f;
    memset(&f, 0, sizeof f);
    f.W = width;
    f.H = height;
    f.B = batch;
    f.D = disp;
    f.ldD = width;
    f.crop_stride_D = plane;
    f.mu = w.mu;
    f.params = params;
    f.packed = (const uint16_t *)packed;
    for (int i = 0; i < 5; ++i) f.acts[i] = w.acts[i];
    f.gbuf[0] = w.gbuf[0];
    f.gbuf[1] = w.gbuf[1];
    f.out = w.dt;
    f.ld_out = width;
    f.crop_stride_out = plane;
    hipError_t e = snx::cnn_forward(f, s);
    if (e != hipSuccess) return api_hip_fail(e, "cnn forward");
    snx::HeadArgs h;
    memset(&h, 0, sizeof h);
    h.W = width;
    h.H = height;
    h.B = batch;
    h.rg = normal_window / 2;
    h.need_g = (normal_window * normal_window + 1) / 2;
    h.Dt = w.dt;
    h.n_gt = normals;
    h.clean = clean;
    h.fid_w = clean ? fidelity : 0.0f;
    for (int b = 0; b < batch; ++b) h.cams[b] = {cams[b].fx, cams[b].fy, cams[b].u0, cams[b].v0};
    h.coefA = w.coefA;
    h.coefB = w.coefB;
    h.coefOwn = w.coefOwn;
    h.part_loss = w.part_loss;
    h.part_used = w.part_used;
    h.inv_n = w.inv_n;
    h.grad_y = w.grad_y;
    h.s = snx::kCnnScale;
    if ((e = snx::cnn_head(h, loss_out, s)) != hipSuccess) return api_hip_fail(e, "cnn head");
    if ((e = snx::cnn_backward(f, w.grad_y, w.partial, grad, s)) != hipSuccess)
        return api_hip_fail(e, "cnn backward");
    if (step > 0 &&
        (e = snx::cnn_adam(params, grad, adam_m, adam_v, step, lr, beta1, beta2, eps,
                           (uint16_t *)packed, s)) != hipSuccess)
        return api_hip_fail(e, "cnn adam");
    return SNX_OK;
}

}  // extern "C"
