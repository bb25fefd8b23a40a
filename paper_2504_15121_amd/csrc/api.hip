// C ABI of libsnx: argument validation, workspace carving and kernel launches.
// Every entry point validates all arguments before the first HIP call, so an
// invalid call enqueues nothing and writes nothing.
#include <cmath>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include "snx_internal.hpp"

namespace {

thread_local char g_err[256] = "";

snx_status fail(snx_status st, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
snx_status fail(snx_status st, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return st;
}

snx_status hip_fail(hipError_t e, const char *where)
{
    (void)hipGetLastError();  // clear the sticky launch error
    return fail(SNX_ERR_HIP, "%s: %s", where, hipGetErrorString(e));
}

bool size_ok(int32_t w, int32_t h) { return w >= 0 && h >= 0 && (int64_t)w * h < (1LL << 31); }

bool cam_ok(const snx_camera *c)
{
    return c && isfinite(c->fx) && c->fx > 0 && isfinite(c->fy) && c->fy > 0 &&
           isfinite(c->baseline) && c->baseline > 0 && isfinite(c->u0) && isfinite(c->v0);
}

snx_status check_image(const void *p, int64_t stride, int32_t w, const char *name)
{
    if (!p) return fail(SNX_ERR_ARG, "%s is NULL", name);
    if (stride < w) return fail(SNX_ERR_ARG, "%s stride %lld < width %d", name, (long long)stride, w);
    return SNX_OK;
}

snx_status check_denoise(const snx_denoise_params *p)
{
    if (!p) return fail(SNX_ERR_ARG, "denoise params are NULL");
    if (p->window < 1 || p->window % 2 == 0)
        return fail(SNX_ERR_ARG, "filter window %d must be odd and >= 1", p->window);
    if (p->window > snx::kMaxWindow)
        return fail(SNX_ERR_UNSUPPORTED, "filter window %d > %d", p->window, snx::kMaxWindow);
    if (p->mode == SNX_FILTER_CNN) {
        const snx_cnn_model *m = static_cast<const snx_cnn_model *>(p->model);
        if (!m || !m->params || !m->packed || !m->workspace)
            return fail(SNX_ERR_MODEL, "CNN filter needs a model with params, packed weights "
                                       "and workspace");
        return SNX_OK;
    }
    if (p->mode != SNX_FILTER_LSQ) return fail(SNX_ERR_UNSUPPORTED, "filter mode %d", p->mode);
    if (p->model) return fail(SNX_ERR_ARG, "LSQ filter takes no model");
    return SNX_OK;
}

snx_status check_normal(const snx_normal_params *p)
{
    if (!p) return fail(SNX_ERR_ARG, "normal params are NULL");
    if (p->window < 3 || p->window % 2 == 0)
        return fail(SNX_ERR_ARG, "gradient window %d must be odd and >= 3", p->window);
    if (p->window > snx::kMaxWindow)
        return fail(SNX_ERR_UNSUPPORTED, "gradient window %d > %d", p->window, snx::kMaxWindow);
    return SNX_OK;
}

snx_status check_comp(const snx_component_params *p)
{
    if (!p) return fail(SNX_ERR_ARG, "component params are NULL");
    if (!(isfinite(p->k_rel) && p->k_rel >= 0) || !(isfinite(p->t_abs) && p->t_abs >= 0))
        return fail(SNX_ERR_ARG, "component thresholds must be finite and >= 0");
    return SNX_OK;
}

int need_g(const snx_normal_params *p)
{
    return p->min_support > 0 ? p->min_support : (p->window * p->window + 1) / 2;
}

int need_f(const snx_denoise_params *p) { return p->min_support > 3 ? p->min_support : 3; }

size_t ws_components(int32_t w, int32_t h)
{
    if (!size_ok(w, h)) return 0;
    return 256 + (size_t)w * (size_t)h * sizeof(int32_t);
}

snx_status fill_stencil(snx::StencilArgs &a, const float *src, int64_t ld, int32_t w, int32_t h,
                        int rf, int rg, int nf, int ng, const snx_camera *cam)
{
    memset(&a, 0, sizeof a);
    a.src = src;
    a.ld_src = ld;
    a.W = w;
    a.H = h;
    a.rf = rf;
    a.rg = rg;
    a.need_f = nf;
    a.need_g = ng;
    if (cam) {
        a.fx = cam->fx; a.fy = cam->fy; a.b = cam->baseline; a.u0 = cam->u0; a.v0 = cam->v0;
    }
    a.th = snx::tuned_tile_height(rf, rg, w, h);
    if (a.th == 0) a.th = snx::stencil_pick_tile_height(rf, rg);
    if (a.th == 0) return fail(SNX_ERR_UNSUPPORTED, "windows too large for one tile in LDS");
    return SNX_OK;
}

}  // namespace

namespace snx {
snx_status api_fail(snx_status st, const char *msg)
{
    g_err[0] = 0;
    return fail(st, "%s", msg);
}
snx_status api_hip_fail(hipError_t e, const char *where) { return hip_fail(e, where); }
void api_clear() { g_err[0] = 0; }
snx_status api_failf(snx_status st, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return st;
}
}  // namespace snx

extern "C" {

const char *snx_status_string(snx_status s)
{
    switch (s) {
    case SNX_OK: return "SNX_OK";
    case SNX_ERR_ARG: return "SNX_ERR_ARG";
    case SNX_ERR_UNSUPPORTED: return "SNX_ERR_UNSUPPORTED";
    case SNX_ERR_WORKSPACE: return "SNX_ERR_WORKSPACE";
    case SNX_ERR_HIP: return "SNX_ERR_HIP";
    case SNX_ERR_MODEL: return "SNX_ERR_MODEL";
    case SNX_ERR_IO: return "SNX_ERR_IO";
    }
    return "SNX_ERR_UNKNOWN";
}

const char *snx_last_error(void) { return g_err; }

int32_t snx_version(void) { return 100; }

snx_status snx_denoise(const float *disp, int64_t disp_stride, float *out, int64_t out_stride,
                       int32_t width, int32_t height, const snx_denoise_params *params,
                       void *stream)
{
    g_err[0] = 0;
    if (!size_ok(width, height)) return fail(SNX_ERR_ARG, "bad size %d x %d", width, height);
    snx_status st = check_denoise(params);
    if (st) return st;
    if (width == 0 || height == 0) return SNX_OK;
    if ((st = check_image(disp, disp_stride, width, "disp"))) return st;
    if ((st = check_image(out, out_stride, width, "out"))) return st;
    if (params->mode == SNX_FILTER_CNN)
        return snx_cnn_denoise(disp, disp_stride, width, height,
                               static_cast<const snx_cnn_model *>(params->model), out, out_stride,
                               stream);
    snx::StencilArgs a;
    if ((st = fill_stencil(a, disp, disp_stride, width, height, params->window / 2, 0,
                           need_f(params), 0, nullptr)))
        return st;
    a.dn = out;
    a.ld_dn = out_stride;
    hipError_t e = snx::launch_stencil(a, (hipStream_t)stream);
    return e == hipSuccess ? SNX_OK : hip_fail(e, "snx_denoise");
}

snx_status snx_affine_normals(const float *disp_dn, int64_t stride, int32_t width, int32_t height,
                              const snx_camera *cam, const snx_normal_params *params,
                              float *affine, float *normals, int64_t out_stride, void *stream)
{
    g_err[0] = 0;
    if (!size_ok(width, height)) return fail(SNX_ERR_ARG, "bad size %d x %d", width, height);
    snx_status st = check_normal(params);
    if (st) return st;
    if (!cam_ok(cam)) return fail(SNX_ERR_ARG, "camera is NULL or not finite/positive");
    if (width == 0 || height == 0) return SNX_OK;
    if ((st = check_image(disp_dn, stride, width, "disp_dn"))) return st;
    if (!affine && !normals) return fail(SNX_ERR_ARG, "affine and normals are both NULL");
    if (out_stride < width) return fail(SNX_ERR_ARG, "out_stride < width");
    snx::StencilArgs a;
    if ((st = fill_stencil(a, disp_dn, stride, width, height, 0, params->window / 2, 0,
                           need_g(params), cam)))
        return st;
    a.aff = affine;
    a.nrm = normals;
    a.ld_out = out_stride;
    a.plane_out = out_stride * (int64_t)height;
    hipError_t e = snx::launch_stencil(a, (hipStream_t)stream);
    return e == hipSuccess ? SNX_OK : hip_fail(e, "snx_affine_normals");
}

static size_t ws_compact(int32_t w, int32_t h)
{
    if (!size_ok(w, h)) return 0;
    return 256 + sizeof(int32_t) * (size_t)snx::compact_chunks((int64_t)w * h);
}

size_t snx_compact_points_workspace_size(int32_t width, int32_t height)
{
    return ws_compact(width, height);
}

snx_status snx_compact_points(const snx_point *points, int32_t width, int32_t height,
                              snx_point *out, int32_t *count, void *workspace,
                              size_t workspace_bytes, void *stream)
{
    g_err[0] = 0;
    if (!size_ok(width, height)) return fail(SNX_ERR_ARG, "bad size %d x %d", width, height);
    if (!count) return fail(SNX_ERR_ARG, "count is NULL");
    hipStream_t s = (hipStream_t)stream;
    if (width == 0 || height == 0) {
        hipError_t e = snx::launch_fill_i32(count, 0, 1, s);
        return e == hipSuccess ? SNX_OK : hip_fail(e, "snx_compact_points");
    }
    if (!points || !out) return fail(SNX_ERR_ARG, "points or out is NULL");
    const int64_t n = (int64_t)width * height;
    const char *pb = reinterpret_cast<const char *>(points), *ob = reinterpret_cast<const char *>(out);
    const int64_t bytes = n * (int64_t)sizeof(snx_point);
    if (pb < ob + bytes && ob < pb + bytes) return fail(SNX_ERR_ARG, "out overlaps points");
    if (!workspace || workspace_bytes < ws_compact(width, height))
        return fail(SNX_ERR_WORKSPACE, "workspace needs %zu bytes", ws_compact(width, height));
    // the chunk counts on a 256-byte boundary inside the workspace's slack
    int32_t *cc = reinterpret_cast<int32_t *>(((uintptr_t)workspace + 255) & ~(uintptr_t)255);
    hipError_t e = snx::launch_compact(points, n, out, count, cc, s);
    return e == hipSuccess ? SNX_OK : hip_fail(e, "snx_compact_points");
}

snx_status snx_compact_points_noalloc(const snx_point *points, int32_t width, int32_t height,
                                      snx_point *out, int32_t *count, void *stream)
{
    g_err[0] = 0;
    if (!size_ok(width, height)) return fail(SNX_ERR_ARG, "bad size %d x %d", width, height);
    if (!count) return fail(SNX_ERR_ARG, "count is NULL");
    const int64_t n = (int64_t)width * height;
    if (n > snx::compact_noalloc_max_records())
        return fail(SNX_ERR_UNSUPPORTED, "%lld records exceed the allocation-free limit of %lld",
                    (long long)n, (long long)snx::compact_noalloc_max_records());
    hipStream_t s = (hipStream_t)stream;
    if (n == 0) {
        hipError_t e = snx::launch_fill_i32(count, 0, 1, s);
        return e == hipSuccess ? SNX_OK : hip_fail(e, "snx_compact_points_noalloc");
    }
    if (!points || !out) return fail(SNX_ERR_ARG, "points or out is NULL");
    const char *pb = reinterpret_cast<const char *>(points), *ob = reinterpret_cast<const char *>(out);
    const int64_t bytes = n * (int64_t)sizeof(snx_point);
    if (pb < ob + bytes && ob < pb + bytes) return fail(SNX_ERR_ARG, "out overlaps points");
    int32_t *cc = nullptr;
    hipError_t e = snx::compact_noalloc_scratch(&cc);
    if (e != hipSuccess) return hip_fail(e, "snx_compact_points_noalloc (scratch address)");
    e = snx::launch_compact(points, n, out, count, cc, s);
    return e == hipSuccess ? SNX_OK : hip_fail(e, "snx_compact_points_noalloc");
}

snx_status snx_affine_normals_labels(const float *disp_dn, int64_t stride, const int32_t *labels,
                                     int64_t label_stride, int32_t width, int32_t height,
                                     const snx_camera *cam, const snx_normal_params *params,
                                     float *affine, float *normals, int64_t out_stride,
                                     void *stream)
{
    g_err[0] = 0;
    if (!size_ok(width, height)) return fail(SNX_ERR_ARG, "bad size %d x %d", width, height);
    snx_status st = check_normal(params);
    if (st) return st;
    if (!cam_ok(cam)) return fail(SNX_ERR_ARG, "camera is NULL or not finite/positive");
    if (width == 0 || height == 0) return SNX_OK;
    if ((st = check_image(disp_dn, stride, width, "disp_dn"))) return st;
    if ((st = check_image(labels, label_stride, width, "labels"))) return st;
    if (!affine && !normals) return fail(SNX_ERR_ARG, "affine and normals are both NULL");
    if (out_stride < width) return fail(SNX_ERR_ARG, "out_stride < width");
    snx::RestrictArgs a;
    a.src = disp_dn;
    a.ld_src = stride;
    a.labels = labels;
    a.ld_lab = label_stride;
    a.W = width;
    a.H = height;
    a.r = params->window / 2;
    a.need_g = need_g(params);
    a.fx = cam->fx;
    a.fy = cam->fy;
    a.u0 = cam->u0;
    a.v0 = cam->v0;
    a.aff = affine;
    a.nrm = normals;
    a.ld_out = out_stride;
    a.plane_out = out_stride * (int64_t)height;
    hipError_t e = snx::launch_affine_labels(a, (hipStream_t)stream);
    return e == hipSuccess ? SNX_OK : hip_fail(e, "snx_affine_normals_labels");
}

snx_status snx_affine_normals_star(const float *disp_dn, int64_t stride, int32_t width,
                                   int32_t height, const snx_camera *cam,
                                   const snx_star_params *params, float *affine, float *normals,
                                   int64_t out_stride, void *stream)
{
    g_err[0] = 0;
    if (!size_ok(width, height)) return fail(SNX_ERR_ARG, "bad size %d x %d", width, height);
    if (!params) return fail(SNX_ERR_ARG, "params is NULL");
    if (params->directions <= 0) return fail(SNX_ERR_ARG, "directions %d", params->directions);
    if (params->directions != 4 && params->directions != 8 && params->directions != 16)
        return fail(SNX_ERR_UNSUPPORTED, "directions %d (4, 8 or 16 supported)",
                    params->directions);
    if (params->steps < 1 || params->steps > 32)
        return fail(SNX_ERR_ARG, "steps %d outside 1..32", params->steps);
    if (params->stop != SNX_STOP_CD && params->stop != SNX_STOP_ST)
        return fail(SNX_ERR_ARG, "unknown stopping rule %d", params->stop);
    if (!std::isfinite(params->threshold) || params->threshold < 0.0)
        return fail(SNX_ERR_ARG, "threshold must be finite and >= 0");
    if (!cam_ok(cam)) return fail(SNX_ERR_ARG, "camera is NULL or not finite/positive");
    if (width == 0 || height == 0) return SNX_OK;
    snx_status st;
    if ((st = check_image(disp_dn, stride, width, "disp_dn"))) return st;
    if (!affine && !normals) return fail(SNX_ERR_ARG, "affine and normals are both NULL");
    if (out_stride < width) return fail(SNX_ERR_ARG, "out_stride < width");
    snx::StarArgs a;
    a.src = disp_dn;
    a.ld_src = stride;
    a.W = width;
    a.H = height;
    a.dirs = params->directions;
    a.steps = params->steps;
    a.stop = params->stop == SNX_STOP_CD ? snx::kStopCD : snx::kStopST;
    a.need_g = params->min_support > 0 ? params->min_support : params->directions;
    a.thr = params->threshold;
    a.fxb = (double)cam->fx * (double)cam->baseline;
    a.fx = cam->fx;
    a.fy = cam->fy;
    a.u0 = cam->u0;
    a.v0 = cam->v0;
    a.aff = affine;
    a.nrm = normals;
    a.ld_out = out_stride;
    a.plane_out = out_stride * (int64_t)height;
    hipError_t e = snx::launch_star(a, (hipStream_t)stream);
    return e == hipSuccess ? SNX_OK : hip_fail(e, "snx_affine_normals_star");
}

size_t snx_components_workspace_size(int32_t width, int32_t height) { return ws_components(width, height); }

static snx_status components_impl(const float *disp, int64_t stride, int32_t width, int32_t height,
                                  const snx_component_params *p, int32_t *labels,
                                  int64_t label_stride, int32_t *num_components, void *workspace,
                                  size_t workspace_bytes, hipStream_t s, const char *who,
                                  const float *nrm = nullptr, int64_t nrm_stride = 0,
                                  double crease_cos = 0.0)
{
    snx::CclArgs c;
    c.D = disp;
    c.ld = stride;
    c.W = width;
    c.H = height;
    c.k_rel = (double)p->k_rel;
    c.t_abs = (double)p->t_abs;
    c.labels = labels;
    c.ld_lab = label_stride;
    c.parent = label_stride == width ? labels : reinterpret_cast<int32_t *>(
                                                    static_cast<char *>(workspace) + 256);
    c.count = num_components;
    c.nrm = nrm;
    c.ld_nrm = nrm_stride;
    c.plane_nrm = nrm_stride * (int64_t)height;
    c.crease_cos = crease_cos;
    (void)workspace_bytes;
    hipError_t e = snx::launch_components(c, s);
    return e == hipSuccess ? SNX_OK : hip_fail(e, who);
}

snx_status snx_components(const float *disp_raw, int64_t stride, int32_t width, int32_t height,
                          const snx_component_params *params, int32_t *labels,
                          int64_t label_stride, int32_t *num_components, void *workspace,
                          size_t workspace_bytes, void *stream)
{
    g_err[0] = 0;
    if (!size_ok(width, height)) return fail(SNX_ERR_ARG, "bad size %d x %d", width, height);
    snx_status st = check_comp(params);
    if (st) return st;
    if (width == 0 || height == 0) {
        if (!num_components) return SNX_OK;
        hipError_t e = snx::launch_fill_i32(num_components, 0, 1, (hipStream_t)stream);
        return e == hipSuccess ? SNX_OK : hip_fail(e, "snx_components");
    }
    if ((st = check_image(disp_raw, stride, width, "disp_raw"))) return st;
    if ((st = check_image(labels, label_stride, width, "labels"))) return st;
    if (!workspace || workspace_bytes < ws_components(width, height))
        return fail(SNX_ERR_WORKSPACE, "workspace needs %zu bytes", ws_components(width, height));
    return components_impl(disp_raw, stride, width, height, params, labels, label_stride,
                           num_components, workspace, workspace_bytes, (hipStream_t)stream,
                           "snx_components");
}

snx_status snx_components_from_edges(const uint8_t *edges, int64_t stride, int32_t width,
                                     int32_t height, int32_t *labels, int64_t label_stride,
                                     int32_t *num_components, void *workspace,
                                     size_t workspace_bytes, void *stream)
{
    g_err[0] = 0;
    if (!size_ok(width, height)) return fail(SNX_ERR_ARG, "bad size %d x %d", width, height);
    hipStream_t s = (hipStream_t)stream;
    if (width == 0 || height == 0) {
        if (!num_components) return SNX_OK;
        hipError_t e = snx::launch_fill_i32(num_components, 0, 1, s);
        return e == hipSuccess ? SNX_OK : hip_fail(e, "snx_components_from_edges");
    }
    snx_status st;
    if ((st = check_image(edges, stride, width, "edges"))) return st;
    if ((st = check_image(labels, label_stride, width, "labels"))) return st;
    if (!workspace || workspace_bytes < ws_components(width, height))
        return fail(SNX_ERR_WORKSPACE, "workspace needs %zu bytes", ws_components(width, height));
    snx::CclArgs c = {};
    c.ld = stride;
    c.W = width;
    c.H = height;
    c.labels = labels;
    c.ld_lab = label_stride;
    c.parent = label_stride == width ? labels : reinterpret_cast<int32_t *>(
                                                    static_cast<char *>(workspace) + 256);
    c.count = num_components;
    c.edges = edges;
    hipError_t e = snx::launch_components(c, s);
    return e == hipSuccess ? SNX_OK : hip_fail(e, "snx_components_from_edges");
}

snx_status snx_components_creases(const float *disp_raw, int64_t stride, const float *normals,
                                  int64_t normals_stride, int32_t width, int32_t height,
                                  const snx_component_params *params, double crease_cos,
                                  int32_t *labels, int64_t label_stride, int32_t *num_components,
                                  void *workspace, size_t workspace_bytes, void *stream)
{
    g_err[0] = 0;
    if (!size_ok(width, height)) return fail(SNX_ERR_ARG, "bad size %d x %d", width, height);
    snx_status st = check_comp(params);
    if (st) return st;
    if (!std::isfinite(crease_cos) || crease_cos < -1.0 || crease_cos > 1.0)
        return fail(SNX_ERR_ARG, "crease_cos must be in [-1, 1]");
    if (width == 0 || height == 0) {
        if (!num_components) return SNX_OK;
        hipError_t e = snx::launch_fill_i32(num_components, 0, 1, (hipStream_t)stream);
        return e == hipSuccess ? SNX_OK : hip_fail(e, "snx_components_creases");
    }
    if ((st = check_image(disp_raw, stride, width, "disp_raw"))) return st;
    if ((st = check_image(normals, normals_stride, width, "normals"))) return st;
    if ((st = check_image(labels, label_stride, width, "labels"))) return st;
    if (!workspace || workspace_bytes < ws_components(width, height))
        return fail(SNX_ERR_WORKSPACE, "workspace needs %zu bytes", ws_components(width, height));
    return components_impl(disp_raw, stride, width, height, params, labels, label_stride,
                           num_components, workspace, workspace_bytes, (hipStream_t)stream,
                           "snx_components_creases", normals, normals_stride, crease_cos);
}

snx_status snx_point_cloud(const float *disp_dn, int64_t disp_stride, const float *normals,
                           int64_t normals_stride, const int32_t *labels, int64_t label_stride,
                           int32_t width, int32_t height, const snx_camera *cam, snx_point *out,
                           void *stream)
{
    g_err[0] = 0;
    if (!size_ok(width, height)) return fail(SNX_ERR_ARG, "bad size %d x %d", width, height);
    if (!cam_ok(cam)) return fail(SNX_ERR_ARG, "camera is NULL or not finite/positive");
    if (width == 0 || height == 0) return SNX_OK;
    snx_status st;
    if ((st = check_image(disp_dn, disp_stride, width, "disp_dn"))) return st;
    if ((st = check_image(normals, normals_stride, width, "normals"))) return st;
    if (labels && label_stride < width) return fail(SNX_ERR_ARG, "label_stride < width");
    if (!out) return fail(SNX_ERR_ARG, "out is NULL");
    snx::CloudArgs a;
    a.dn = disp_dn;
    a.ld_dn = disp_stride;
    a.nrm = normals;
    a.ld_nrm = normals_stride;
    a.plane_nrm = normals_stride * (int64_t)height;
    a.labels = labels;
    a.ld_lab = label_stride;
    a.W = width;
    a.H = height;
    a.fx = cam->fx; a.fy = cam->fy; a.b = cam->baseline; a.u0 = cam->u0; a.v0 = cam->v0;
    a.out = out;
    hipError_t e = snx::launch_point_cloud(a, (hipStream_t)stream);
    return e == hipSuccess ? SNX_OK : hip_fail(e, "snx_point_cloud");
}

static snx_status fused_impl(const float *disp, int64_t stride, int32_t width, int32_t height,
                             const snx_camera *cam, const snx_denoise_params *denoise,
                             const snx_normal_params *normal, const int32_t *labels,
                             int64_t label_stride, float *disp_dn, float *affine, float *normals,
                             int64_t out_stride, snx_point *points, hipStream_t s, const char *who)
{
    snx::StencilArgs a;
    snx_status st = fill_stencil(a, disp, stride, width, height, denoise->window / 2,
                                 normal->window / 2, need_f(denoise), need_g(normal), cam);
    if (st) return st;
    a.dn = disp_dn;
    a.ld_dn = out_stride;
    a.aff = affine;
    a.nrm = normals;
    a.ld_out = out_stride;
    a.plane_out = out_stride * (int64_t)height;
    a.labels = const_cast<int32_t *>(labels);   // read only: no forest to resolve
    a.ld_lab = label_stride;
    a.rec = points;
    hipError_t e = snx::launch_stencil(a, s);
    return e == hipSuccess ? SNX_OK : hip_fail(e, who);
}

// Arguments of the fused and pipeline calls; with `one_kernel` also that the
// filter and the gradient fit one tile (the fused call), else that each fits
// its own pass (the pipeline filters in a pass of its own when rf > 1).
static snx_status check_fused(const float *disp, int64_t stride, int32_t width, int32_t height,
                              const snx_camera *cam, const snx_denoise_params *denoise,
                              const snx_normal_params *normal, float *disp_dn, float *affine,
                              float *normals, int64_t out_stride, snx_point *points,
                              bool one_kernel = true)
{
    snx_status st;
    if ((st = check_denoise(denoise)) || (st = check_normal(normal))) return st;
    if (!cam_ok(cam)) return fail(SNX_ERR_ARG, "camera is NULL or not finite/positive");
    if (width == 0 || height == 0) return SNX_OK;
    if ((st = check_image(disp, stride, width, "disp"))) return st;
    if (!points) return fail(SNX_ERR_ARG, "points is NULL");
    if ((disp_dn || affine || normals) && out_stride < width)
        return fail(SNX_ERR_ARG, "out_stride < width");
    snx::StencilArgs a;
    const bool cnn = denoise->mode == SNX_FILTER_CNN;
    const int rf = cnn ? 0 : denoise->window / 2;
    if (one_kernel)
        return fill_stencil(a, disp, stride, width, height, rf, normal->window / 2,
                            need_f(denoise), need_g(normal), cam);
    if (rf > 1 && (st = fill_stencil(a, disp, stride, width, height, rf, 0, need_f(denoise), 0,
                                     nullptr)))
        return st;
    return fill_stencil(a, disp, stride, width, height, 0, normal->window / 2, 0,
                        need_g(normal), cam);
}

snx_status snx_oriented_point_cloud(const float *disp, int64_t stride, int32_t width,
                                    int32_t height, const snx_camera *cam,
                                    const snx_denoise_params *denoise,
                                    const snx_normal_params *normal, const int32_t *labels,
                                    int64_t label_stride, float *disp_dn, float *affine,
                                    float *normals, int64_t out_stride, snx_point *points,
                                    void *stream)
{
    g_err[0] = 0;
    if (!size_ok(width, height)) return fail(SNX_ERR_ARG, "bad size %d x %d", width, height);
    snx_status st = check_fused(disp, stride, width, height, cam, denoise, normal, disp_dn,
                                affine, normals, out_stride, points);
    if (st || width == 0 || height == 0) return st;
    if (denoise->mode == SNX_FILTER_CNN)
        return fail(SNX_ERR_UNSUPPORTED, "the fused call runs the LSQ filter only; use "
                                         "snx_pipeline for the learned filter");
    if (labels && label_stride < width) return fail(SNX_ERR_ARG, "label_stride < width");
    return fused_impl(disp, stride, width, height, cam, denoise, normal, labels, label_stride,
                      disp_dn, affine, normals, out_stride, points, (hipStream_t)stream,
                      "snx_oriented_point_cloud");
}

static size_t plane_bytes(int32_t w, int32_t h)
{
    return ((size_t)w * (size_t)h * sizeof(float) + 255) / 256 * 256;
}

// Seam records of the 3x3-filter front: two int32 per tile-seam pair.
static size_t seam_bytes(int32_t w, int32_t h)
{
    if (w <= 0 || h <= 0) return 0;
    return ((size_t)snx::merge_pairs(w, h) * sizeof(int32_t) + 255) / 256 * 256;
}

size_t snx_pipeline_workspace_size(int32_t width, int32_t height)
{
    if (!size_ok(width, height)) return 0;
    return 256 + 2 * plane_bytes(width, height) + 2 * seam_bytes(width, height);
}

snx_status snx_pipeline_part(const float *disp, int64_t stride, int32_t width, int32_t height,
                             const snx_camera *cam, const snx_denoise_params *denoise,
                             const snx_normal_params *normal, const snx_component_params *comp,
                             float *disp_dn, float *affine, float *normals, int64_t out_stride,
                             int32_t *labels, int64_t label_stride, int32_t *num_components,
                             snx_point *points, void *workspace, size_t workspace_bytes,
                             int32_t parts, void *stream)
{
    g_err[0] = 0;
    if (!size_ok(width, height)) return fail(SNX_ERR_ARG, "bad size %d x %d", width, height);
    if (parts < 1 || parts > 3) return fail(SNX_ERR_ARG, "parts must be 1, 2 or 3");
    snx_status st;
    if ((st = check_comp(comp))) return st;
    if ((st = check_fused(disp, stride, width, height, cam, denoise, normal, disp_dn, affine,
                          normals, out_stride, points, false)))
        return st;
    hipStream_t s = (hipStream_t)stream;
    if (width == 0 || height == 0) {
        if (!num_components || !(parts & 1)) return SNX_OK;
        hipError_t e = snx::launch_fill_i32(num_components, 0, 1, s);
        return e == hipSuccess ? SNX_OK : hip_fail(e, "snx_pipeline");
    }
    if ((st = check_image(labels, label_stride, width, "labels"))) return st;
    const size_t need = snx_pipeline_workspace_size(width, height);
    if (!workspace || workspace_bytes < need)
        return fail(SNX_ERR_WORKSPACE, "workspace needs %zu bytes", need);

    char *ws = static_cast<char *>(workspace);
    int32_t *forest = label_stride == width ? labels : reinterpret_cast<int32_t *>(ws + 256);
    float *dn = disp_dn ? disp_dn : reinterpret_cast<float *>(ws + 256 + plane_bytes(width, height));
    const int64_t ld_dn = disp_dn ? out_stride : width;
    const bool cnn = denoise->mode == SNX_FILTER_CNN;
    const int rf = cnn ? 0 : denoise->window / 2, rg = normal->window / 2;
    const double k_rel = (double)comp->k_rel, t_abs = (double)comp->t_abs;
    hipError_t e = hipSuccess;

    if ((parts & 1) && cnn) {
        // part 1 with the learned filter: the network, then the forest
        st = snx_cnn_denoise(disp, stride, width, height,
                             static_cast<const snx_cnn_model *>(denoise->model), dn, ld_dn, stream);
        if (st) return st;
    }
    if (parts & 1) {
        // part 1: label forest and filtered disparity
        snx::FrontArgs f;
        f.D = disp;
        f.ld = stride;
        f.W = width;
        f.H = height;
        f.k_rel = k_rel;
        f.t_abs = t_abs;
        f.rf = rf <= 1 ? rf : 0;
        f.need_f = need_f(denoise);
        f.dn = !cnn && rf <= 1 ? dn : nullptr;
        f.ld_dn = ld_dn;
        f.forest = forest;
        f.count = num_components;
        if (f.rf == 1 && f.dn) {
            // the 3x3 filter's halo lets the front decide the seam pairs: the
            // merge then reads two records per pair
            char *sb = ws + 256 + 2 * plane_bytes(width, height);
            f.seam_a = reinterpret_cast<int32_t *>(sb);
            f.seam_b = reinterpret_cast<int32_t *>(sb + seam_bytes(width, height));
        }
        if ((e = snx::launch_front(f, s)) != hipSuccess) return hip_fail(e, "snx_pipeline");
        if (f.seam_a)
            e = snx::launch_merge_seams(f.seam_a, f.seam_b, snx::merge_pairs(width, height),
                                        forest, s);
        else
            e = snx::launch_merge(disp, stride, width, height, k_rel, t_abs, forest, s);
        if (e != hipSuccess) return hip_fail(e, "snx_pipeline");
        if (rf > 1) {
            snx::StencilArgs a;
            if ((st = fill_stencil(a, disp, stride, width, height, rf, 0, need_f(denoise), 0,
                                   nullptr)))
                return st;
            a.dn = dn;
            a.ld_dn = ld_dn;
            if ((e = snx::launch_stencil(a, s)) != hipSuccess) return hip_fail(e, "snx_pipeline");
        }
    }
    if (parts & 2) {
        // part 2: gradients, A, normals, label resolution, point records
        snx::StencilArgs a;
        if ((st = fill_stencil(a, dn, ld_dn, width, height, 0, rg, 0, need_g(normal), cam)))
            return st;
        a.aff = affine;
        a.nrm = normals;
        a.ld_out = out_stride;
        a.plane_out = out_stride * (int64_t)height;
        a.forest = forest;
        a.labels = labels;
        a.ld_lab = label_stride;
        a.count = num_components;
        a.rec = points;
        if ((e = snx::launch_stencil(a, s)) != hipSuccess) return hip_fail(e, "snx_pipeline");
    }
    return SNX_OK;
}

snx_status snx_autotune(int32_t width, int32_t height, const snx_denoise_params *denoise,
                        const snx_normal_params *normal, int32_t *chosen, void *stream)
{
    g_err[0] = 0;
    if (!size_ok(width, height) || width == 0 || height == 0)
        return fail(SNX_ERR_ARG, "bad size %d x %d", width, height);
    snx_status st;
    if ((st = check_denoise(denoise)) || (st = check_normal(normal))) return st;
    const int rf = denoise->mode == SNX_FILTER_CNN ? 0 : denoise->window / 2;
    const int rg = normal->window / 2;
    int th_fused = 0, th_grad = 0;
    hipError_t e = snx::autotune_stencil(rf, rg, need_f(denoise), need_g(normal), width, height,
                                         (hipStream_t)stream, &th_fused);
    if (e == hipSuccess && rf > 0)
        e = snx::autotune_stencil(0, rg, 3, need_g(normal), width, height, (hipStream_t)stream,
                                  &th_grad);
    if (e != hipSuccess) return hip_fail(e, "snx_autotune");
    if (chosen) {
        chosen[0] = th_fused;
        chosen[1] = rf > 0 ? th_grad : th_fused;
    }
    return SNX_OK;
}

snx_status snx_tune_set(int32_t width, int32_t height, int32_t filter_window,
                        int32_t normal_window, int32_t tile_height)
{
    g_err[0] = 0;
    if (!size_ok(width, height) || width == 0 || height == 0)
        return fail(SNX_ERR_ARG, "bad size %d x %d", width, height);
    if (filter_window < 1 || filter_window % 2 == 0 || normal_window < 0 ||
        (normal_window > 0 && normal_window % 2 == 0) || filter_window > snx::kMaxWindow ||
        normal_window > snx::kMaxWindow)
        return fail(SNX_ERR_ARG, "bad windows %d, %d", filter_window, normal_window);
    if (!snx::set_tile_height(filter_window / 2, normal_window / 2, width, height, tile_height))
        return fail(SNX_ERR_UNSUPPORTED, "no compiled tile height %d for windows %d, %d",
                    tile_height, filter_window, normal_window);
    return SNX_OK;
}

snx_status snx_pipeline(const float *disp, int64_t stride, int32_t width, int32_t height,
                        const snx_camera *cam, const snx_denoise_params *denoise,
                        const snx_normal_params *normal, const snx_component_params *comp,
                        float *disp_dn, float *affine, float *normals, int64_t out_stride,
                        int32_t *labels, int64_t label_stride, int32_t *num_components,
                        snx_point *points, void *workspace, size_t workspace_bytes, void *stream)
{
    return snx_pipeline_part(disp, stride, width, height, cam, denoise, normal, comp, disp_dn,
                             affine, normals, out_stride, labels, label_stride, num_components,
                             points, workspace, workspace_bytes, 3, stream);
}

}  // extern "C"
