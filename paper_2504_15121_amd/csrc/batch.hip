// Batch plans: many frames of uneven size through the whole path with one
// persistent launch per stage over a device-side (frame, tile) work list, the
// launches captured once in a hipGraph and replayed on every run.
//
//   reset   zero the two work counters and every frame's component count
//   front   persistent workgroups fetch (frame, tile) items: 3x3 filter + local
//           forest (with the learned filter: the 3x3 filter is the network's mu)
//   merge   one thread per tile-seam pair of every frame
//   [cnn    learned filter: the fused network over the tiles of every frame]
//   back    persistent workgroups fetch (frame, tile) items: gradients, A,
//           normals, label resolution, point records
//
// A plan of one frame with the LSQ filter runs the single-frame kernels
// instead (front, seam merge from the front's seam records, fused back
// stencil): with no other frame to fill the chip, the work-list claims and the
// reset launch would only lengthen the frame's latency chain.
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <vector>

#include "snx_cnn.hpp"

namespace snx {
snx_status api_fail(snx_status st, const char *msg);
snx_status api_hip_fail(hipError_t e, const char *where);
}  // namespace snx

struct snx_plan {
    int n = 0;
    bool cnn = false;
    snx_cnn_model model{};
    int rf = 0, rg = 0, th = 16;
    std::vector<snx::BatchFrame> host;
    snx::BatchFrame *d_frames = nullptr;
    int *d_front_off = nullptr, *d_back_off = nullptr, *d_counters = nullptr;
    int *d_front_frame = nullptr, *d_back_frame = nullptr, *d_merge_frame = nullptr;
    snx::CnnFusedArgs cnn_common{};                 // params and packed weights
    snx::CnnFusedArgs *d_cnn = nullptr;             // per-frame network arguments
    int *d_cnn_off = nullptr, *d_cnn_frame = nullptr;
    int cnn_total = 0;
    int64_t *d_seam_off = nullptr;
    int64_t seam_total = 0;
    int grid_front = 1, grid_back = 1;
    bool direct = false;                            // one frame: single-frame kernels
    int32_t *seam_a = nullptr, *seam_b = nullptr;   // seam records (fronts with the 3x3 halo)
    std::vector<void *> owned;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t captured_on = nullptr;
};

namespace {

using snx::api_fail;
using snx::api_hip_fail;

void release(snx_plan *p)
{
    if (!p) return;
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    for (void *q : p->owned) (void)hipFree(q);
    (void)hipFree(p->d_frames);
    (void)hipFree(p->d_front_off);
    (void)hipFree(p->d_back_off);
    (void)hipFree(p->d_seam_off);
    (void)hipFree(p->d_counters);
    (void)hipFree(p->d_cnn);
    (void)hipFree(p->d_cnn_off);
    (void)hipFree(p->d_cnn_frame);
    (void)hipFree(p->d_front_frame);
    (void)hipFree(p->d_back_frame);
    (void)hipFree(p->d_merge_frame);
    delete p;
}

hipError_t enqueue(snx_plan *p, hipStream_t s)
{
    hipError_t e;
    if (p->direct) {
        const snx::BatchFrame &b = p->host[0];
        snx::FrontArgs f = b.front;          // the front zeroes the component count
        f.seam_a = p->seam_a;
        f.seam_b = p->seam_b;
        if ((e = snx::launch_front(f, s)) != hipSuccess) return e;
        e = f.seam_a ? snx::launch_merge_seams(f.seam_a, f.seam_b, snx::merge_pairs(f.W, f.H),
                                               f.forest, s)
                     : snx::launch_merge(f.D, f.ld, f.W, f.H, f.k_rel, f.t_abs, f.forest, s);
        if (e != hipSuccess) return e;
        return snx::launch_stencil(b.back, s);
    }
    e = snx::launch_batch_reset(p->d_counters, 2, p->d_frames, p->n, s);
    if (e != hipSuccess) return e;
    // the front filters with window 3 also for the learned filter (its mu)
    if ((e = snx::launch_batch_front(p->d_frames, p->d_front_off, p->d_front_frame, p->n,
                                     p->cnn ? 1 : p->rf, p->d_counters, p->grid_front, s)) !=
        hipSuccess)
        return e;
    if ((e = snx::launch_batch_merge(p->d_frames, p->d_seam_off, p->d_merge_frame, p->n,
                                     p->seam_total, s, p->seam_a, p->seam_b)) != hipSuccess)
        return e;
    if (p->cnn &&
        (e = snx::cnn_forward_fused_batch(p->cnn_common, p->d_cnn, p->d_cnn_off, p->d_cnn_frame,
                                          p->n, p->cnn_total, s)) != hipSuccess)
        return e;
    return snx::launch_batch_back(p->d_frames, p->d_back_off, p->d_back_frame, p->n, p->rg, p->th,
                                  p->d_counters + 1, p->grid_back, s);
}

}  // namespace

extern "C" {

snx_status snx_plan_create(const snx_frame *frames, int32_t n, const snx_denoise_params *dp,
                           const snx_normal_params *np, const snx_component_params *cp,
                           snx_plan **out)
{
    if (!out) return api_fail(SNX_ERR_ARG, "plan output pointer is NULL");
    *out = nullptr;
    if (!frames || n < 1 || !dp || !np || !cp) return api_fail(SNX_ERR_ARG, "NULL argument or n < 1");
    const bool cnn = dp->mode == SNX_FILTER_CNN;
    if (!cnn && dp->mode != SNX_FILTER_LSQ) return api_fail(SNX_ERR_UNSUPPORTED, "filter mode");
    if (!cnn && (dp->window != 1 && dp->window != 3))
        return api_fail(SNX_ERR_UNSUPPORTED, "batch plans filter with window 1 or 3");
    if (cnn) {
        const snx_cnn_model *m = static_cast<const snx_cnn_model *>(dp->model);
        if (!m || !m->params || !m->packed)
            return api_fail(SNX_ERR_MODEL, "CNN filter needs the model's params and packed weights");
        if (((uintptr_t)m->params & 15) || ((uintptr_t)m->packed & 15))
            return api_fail(SNX_ERR_ARG, "model buffers must be 16-byte aligned");
    }
    if (np->window < 3 || np->window % 2 == 0 || np->window > snx::kMaxWindow)
        return api_fail(SNX_ERR_ARG, "gradient window must be odd, 3..63");
    if (!(isfinite(cp->k_rel) && cp->k_rel >= 0 && isfinite(cp->t_abs) && cp->t_abs >= 0))
        return api_fail(SNX_ERR_ARG, "component thresholds");
    const int rg = np->window / 2;
    int maxW = 0, maxH = 0;
    for (int i = 0; i < n; ++i) {
        const snx_frame &f = frames[i];
        if (f.width < 1 || f.height < 1 || (int64_t)f.width * f.height >= (1LL << 31))
            return api_fail(SNX_ERR_ARG, "frame size");
        if (!f.disp || f.stride < f.width || !f.labels || f.label_stride < f.width || !f.points)
            return api_fail(SNX_ERR_ARG, "frame buffers or strides");
        if (f.disp_dn && f.dn_stride < f.width) return api_fail(SNX_ERR_ARG, "dn_stride");
        const snx_camera &c = f.cam;
        if (!(isfinite(c.fx) && c.fx > 0 && isfinite(c.fy) && c.fy > 0 && isfinite(c.baseline) &&
              c.baseline > 0 && isfinite(c.u0) && isfinite(c.v0)))
            return api_fail(SNX_ERR_ARG, "frame camera");
        if ((int64_t)f.width * f.height > (int64_t)maxW * maxH) { maxW = f.width; maxH = f.height; }
    }
    const int need_g = np->min_support > 0 ? np->min_support : (np->window * np->window + 1) / 2;
    int th = snx::tuned_tile_height(0, rg, maxW, maxH);
    if (th == 0) {
        // not tuned for this size class yet: tune the gradient pass on the
        // largest frame's size (a set-up cost of a few milliseconds)
        hipError_t te = snx::autotune_stencil(0, rg, 3, need_g, maxW, maxH, nullptr, &th);
        if (te != hipSuccess) return api_hip_fail(te, "snx_plan_create autotune");
    }
    if (!snx::batch_has_instance(rg, th)) th = 16;
    if (!snx::batch_has_instance(rg, th)) th = 8;
    if (!snx::batch_has_instance(rg, th)) th = 4;
    if (!snx::batch_has_instance(rg, th))
        return api_fail(SNX_ERR_UNSUPPORTED, "no batched kernel for this gradient window");

    snx_plan *p = new snx_plan;
    p->n = n;
    p->cnn = cnn;
    if (cnn) p->model = *static_cast<const snx_cnn_model *>(dp->model);
    p->rf = cnn ? 0 : dp->window / 2;
    p->rg = rg;
    p->th = th;
    p->host.resize(n);
    std::vector<int> foff(n + 1, 0), boff(n + 1, 0), coff(n + 1, 0);
    std::vector<snx::CnnFusedArgs> cnn_args(cnn ? n : 0);
    std::vector<int64_t> soff(n + 1, 0);
    hipError_t e = hipSuccess;
    for (int i = 0; i < n && e == hipSuccess; ++i) {
        const snx_frame &f = frames[i];
        int32_t *forest = f.labels;
        if (f.label_stride != f.width) {
            void *q = nullptr;
            e = hipMalloc(&q, (size_t)f.width * f.height * 4);
            if (e == hipSuccess) p->owned.push_back(q);
            forest = static_cast<int32_t *>(q);
        }
        float *dn = f.disp_dn;
        int64_t ld_dn = f.dn_stride;
        if (!dn && e == hipSuccess) {
            void *q = nullptr;
            e = hipMalloc(&q, (size_t)f.width * f.height * 4);
            if (e == hipSuccess) p->owned.push_back(q);
            dn = static_cast<float *>(q);
            ld_dn = f.width;
        }
        // the learned filter's mu (3x3 LSQ filter, support 3) written by the front
        float *mu = nullptr;
        if (cnn && e == hipSuccess) {
            void *q = nullptr;
            e = hipMalloc(&q, (size_t)f.width * f.height * 4);
            if (e == hipSuccess) p->owned.push_back(q);
            mu = static_cast<float *>(q);
        }
        snx::BatchFrame &b = p->host[i];
        memset(&b, 0, sizeof b);
        b.front.D = f.disp;
        b.front.ld = f.stride;
        b.front.W = f.width;
        b.front.H = f.height;
        b.front.k_rel = cp->k_rel;
        b.front.t_abs = cp->t_abs;
        b.front.rf = cnn ? 1 : p->rf;
        b.front.need_f = cnn ? 3 : (dp->min_support > 3 ? dp->min_support : 3);
        b.front.dn = cnn ? mu : dn;
        b.front.ld_dn = cnn ? f.width : ld_dn;
        if (cnn) {
            snx::CnnFusedArgs &c = cnn_args[i];
            memset(&c, 0, sizeof c);
            c.W = f.width;
            c.H = f.height;
            c.D = f.disp;
            c.ldD = f.stride;
            c.mu = mu;
            c.params = p->model.params;
            c.packed = static_cast<const uint16_t *>(p->model.packed);
            c.out = dn;
            c.ld_out = ld_dn;
            c.s = snx::kCnnScale;
        }
        b.front.forest = forest;
        b.front.count = f.num_components;
        b.back.src = dn;
        b.back.ld_src = ld_dn;
        b.back.W = f.width;
        b.back.H = f.height;
        b.back.rf = 0;
        b.back.rg = rg;
        b.back.need_g = need_g;
        b.back.fx = f.cam.fx;
        b.back.fy = f.cam.fy;
        b.back.b = f.cam.baseline;
        b.back.u0 = f.cam.u0;
        b.back.v0 = f.cam.v0;
        b.back.forest = forest;
        b.back.labels = f.labels;
        b.back.ld_lab = f.label_stride;
        b.back.count = f.num_components;
        b.back.rec = f.points;
        b.back.th = th;
        foff[i + 1] = foff[i] + snx::front_tiles(f.width, f.height);
        coff[i + 1] = coff[i] + (cnn ? snx::cnn_fused_tiles(f.width, f.height) : 0);
        boff[i + 1] = boff[i] + snx::back_tiles(f.width, f.height, th);
        soff[i + 1] = soff[i] + snx::merge_pairs(f.width, f.height);
    }
    // item -> frame tables (front tiles, back tiles) and the frame of each
    // merge block's first seam pair
    std::vector<int> front_frame(foff[n]), back_frame(boff[n]), cnn_frame(coff[n]);
    for (int i = 0; i < n; ++i) {
        for (int t = foff[i]; t < foff[i + 1]; ++t) front_frame[t] = i;
        for (int t = boff[i]; t < boff[i + 1]; ++t) back_frame[t] = i;
        for (int t = coff[i]; t < coff[i + 1]; ++t) cnn_frame[t] = i;
    }
    const int64_t merge_blocks = (soff[n] + 255) / 256;
    std::vector<int> merge_frame((size_t)(merge_blocks > 0 ? merge_blocks : 1), 0);
    for (int i = 0, f = 0; i < merge_blocks; ++i) {
        while (soff[f + 1] <= (int64_t)i * 256) ++f;
        merge_frame[i] = f;
    }
    auto upload = [&](int **dst, const std::vector<int> &v) {
        if (e != hipSuccess) return;
        e = hipMalloc(dst, sizeof(int) * (v.empty() ? 1 : v.size()));
        if (e == hipSuccess && !v.empty())
            e = hipMemcpy(*dst, v.data(), sizeof(int) * v.size(), hipMemcpyHostToDevice);
    };
    upload(&p->d_front_frame, front_frame);
    upload(&p->d_back_frame, back_frame);
    upload(&p->d_merge_frame, merge_frame);
    if (cnn) {
        upload(&p->d_cnn_off, coff);
        upload(&p->d_cnn_frame, cnn_frame);
        if (e == hipSuccess) e = hipMalloc(&p->d_cnn, sizeof(snx::CnnFusedArgs) * n);
        if (e == hipSuccess)
            e = hipMemcpy(p->d_cnn, cnn_args.data(), sizeof(snx::CnnFusedArgs) * n,
                          hipMemcpyHostToDevice);
        p->cnn_total = coff[n];
        p->cnn_common = cnn_args[0];
    }
    // seam records: every front with the 3x3 halo (LSQ window 3, and the learned
    // filter's mu) decides its seam pairs; one-frame plans allocate theirs below
    if (e == hipSuccess && !(!cnn && n == 1) && (cnn || p->rf == 1) && soff[n] > 0) {
        void *q = nullptr;
        e = hipMalloc(&q, sizeof(int32_t) * 2 * (size_t)soff[n]);
        if (e == hipSuccess) {
            p->owned.push_back(q);
            p->seam_a = static_cast<int32_t *>(q);
            p->seam_b = p->seam_a + soff[n];
            for (int i = 0; i < n; ++i) {
                p->host[i].front.seam_a = p->seam_a + soff[i];
                p->host[i].front.seam_b = p->seam_b + soff[i];
            }
        }
    }
    if (e == hipSuccess) e = hipMalloc(&p->d_frames, sizeof(snx::BatchFrame) * n);
    if (e == hipSuccess) e = hipMalloc(&p->d_front_off, sizeof(int) * (n + 1));
    if (e == hipSuccess) e = hipMalloc(&p->d_back_off, sizeof(int) * (n + 1));
    if (e == hipSuccess) e = hipMalloc(&p->d_seam_off, sizeof(int64_t) * (n + 1));
    if (e == hipSuccess) e = hipMalloc(&p->d_counters, sizeof(int) * 2);
    if (e == hipSuccess)
        e = hipMemcpy(p->d_frames, p->host.data(), sizeof(snx::BatchFrame) * n, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(p->d_front_off, foff.data(), sizeof(int) * (n + 1), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(p->d_back_off, boff.data(), sizeof(int) * (n + 1), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(p->d_seam_off, soff.data(), sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        release(p);
        return api_hip_fail(e, "snx_plan_create");
    }
    p->seam_total = soff[n];
    p->direct = !cnn && n == 1;
    if (p->direct && p->rf == 1 && soff[1] > 0) {
        void *q = nullptr;
        e = hipMalloc(&q, sizeof(int32_t) * 2 * (size_t)soff[1]);
        if (e != hipSuccess) {
            release(p);
            return api_hip_fail(e, "snx_plan_create");
        }
        p->owned.push_back(q);
        p->seam_a = static_cast<int32_t *>(q);
        p->seam_b = p->seam_a + soff[1];
    }
    int dev = 0, cus = 256;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
        cus = prop.multiProcessorCount;
    // persistent grids: enough workgroups to fill every CU at full LDS occupancy
    const int per_cu_back = (int)(160 * 1024 / snx::stencil_lds_bytes(0, rg, th));
    p->grid_front = foff[n] < cus * 8 ? foff[n] : cus * 8;
    p->grid_back = boff[n] < cus * per_cu_back ? boff[n] : cus * per_cu_back;
    if (p->grid_back < 1) p->grid_back = 1;
    *out = p;
    return SNX_OK;
}

snx_status snx_plan_run(snx_plan *plan, void *stream)
{
    if (!plan) return api_fail(SNX_ERR_ARG, "plan is NULL");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e;
    if (!s) {
        // the legacy default stream cannot be captured: launch directly
        e = enqueue(plan, s);
        return e == hipSuccess ? SNX_OK : api_hip_fail(e, "snx_plan_run");
    }
    if (!plan->exec || plan->captured_on != s) {
        if (plan->exec) { (void)hipGraphExecDestroy(plan->exec); plan->exec = nullptr; }
        if (plan->graph) { (void)hipGraphDestroy(plan->graph); plan->graph = nullptr; }
        if ((e = hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed)) != hipSuccess)
            return api_hip_fail(e, "snx_plan_run capture");
        const hipError_t le = enqueue(plan, s);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(s, &g);
        if (le != hipSuccess || e != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return api_hip_fail(le != hipSuccess ? le : e, "snx_plan_run capture");
        }
        plan->graph = g;
        if ((e = hipGraphInstantiate(&plan->exec, g, nullptr, nullptr, 0)) != hipSuccess)
            return api_hip_fail(e, "snx_plan_run instantiate");
        plan->captured_on = s;
    }
    e = hipGraphLaunch(plan->exec, s);
    return e == hipSuccess ? SNX_OK : api_hip_fail(e, "snx_plan_run");
}

snx_status snx_plan_destroy(snx_plan *plan)
{
    release(plan);
    return SNX_OK;
}

}  // extern "C"
