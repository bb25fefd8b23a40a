// Tile-height autotuner for the stencil kernel.
//
// The best tile height of k_stencil depends on the two window radii (they set
// the halo and the LDS footprint, hence the occupancy) and on the frame size
// (how many workgroups fill the 256 CUs).  snx_autotune times every compiled
// candidate on the calling stream with HIP events on a synthetic frame of the
// requested size and records the fastest per (architecture, rf, rg, size
// class).  The table is process-wide, guarded by a mutex, and optionally
// persisted as text lines "arch rf rg class th" in the file named by the
// SNX_AUTOTUNE_CACHE environment variable (entries of another architecture are
// ignored).  Without an entry the heuristic default of stencil_pick_tile_height
// is used.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "snx_internal.hpp"

namespace snx {
namespace {

std::mutex g_mu;
std::map<std::tuple<int, int, int>, int> g_table;
bool g_loaded = false;
std::string g_arch;

int size_class(int W, int H)
{
    const double px = (double)W * (double)H;
    return px <= 1.0 ? 0 : (int)floor(log2(px));
}

const std::string &arch_name()
{
    if (g_arch.empty()) {
        int dev = 0;
        hipDeviceProp_t p;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&p, dev) == hipSuccess)
            g_arch = p.gcnArchName;
        else
            g_arch = "unknown";
        const size_t colon = g_arch.find(':');
        if (colon != std::string::npos) g_arch = g_arch.substr(0, colon);
    }
    return g_arch;
}

void load_cache_locked()
{
    if (g_loaded) return;
    g_loaded = true;
    const char *path = getenv("SNX_AUTOTUNE_CACHE");
    if (!path) return;
    FILE *f = fopen(path, "r");
    if (!f) return;
    char arch[64];
    int rf, rg, cls, th;
    const std::string &me = arch_name();
    while (fscanf(f, "%63s %d %d %d %d", arch, &rf, &rg, &cls, &th) == 5) {
        if (me == arch && stencil_has_instance(rf, rg, th)) g_table[{rf, rg, cls}] = th;
    }
    fclose(f);
}

void store_locked(int rf, int rg, int cls, int th)
{
    g_table[{rf, rg, cls}] = th;
    const char *path = getenv("SNX_AUTOTUNE_CACHE");
    if (!path) return;
    FILE *f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "%s %d %d %d %d\n", arch_name().c_str(), rf, rg, cls, th);
    fclose(f);
}

// Synthetic frame: a slanted plane with a regular pattern of holes.
__global__ void k_synth(float *d, int W, int H)
{
    const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y;
    if (x >= W) return;
    const unsigned h = (unsigned)(x * 73856093) ^ (unsigned)(y * 19349663);
    d[(int64_t)y * W + x] = (h % 17u == 0u) ? __builtin_nanf("") : 20.0f + 0.01f * x - 0.02f * y;
}

// Synthetic label forest for the synthetic frame, shaped like the one part 1
// leaves: every valid pixel points to the corner of its 64 x 32 block (a tile
// root), and every corner to pixel 0 (the merged root): chains of two.
__global__ void k_synth_forest(int32_t *f, const float *d, int W, int H)
{
    const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y;
    if (x >= W) return;
    const int64_t i = (int64_t)y * W + x;
    const bool corner = (x & 63) == 0 && (y & 31) == 0;
    int32_t v = d[i] == d[i] ? (int32_t)((int64_t)(y & ~31) * W + (x & ~63)) : -1;
    if (corner) v = 0;
    f[i] = v;
}

}  // namespace

int tuned_tile_height(int rf, int rg, int W, int H)
{
    std::lock_guard<std::mutex> lk(g_mu);
    load_cache_locked();
    const auto it = g_table.find({rf, rg, size_class(W, H)});
    return it == g_table.end() ? 0 : it->second;
}

bool set_tile_height(int rf, int rg, int W, int H, int th)
{
    std::lock_guard<std::mutex> lk(g_mu);
    load_cache_locked();
    const auto key = std::make_tuple(rf, rg, size_class(W, H));
    if (th == 0) {
        g_table.erase(key);
        return true;
    }
    if (!stencil_has_instance(rf, rg, th)) return false;
    g_table[key] = th;
    return true;
}

hipError_t autotune_stencil(int rf, int rg, int need_f, int need_g, int W, int H, hipStream_t s,
                            int *chosen)
{
    *chosen = 0;
    std::vector<int> cands;
    for (int th : {4, 8, 16, 24, 32})
        if (stencil_has_instance(rf, rg, th) && stencil_lds_bytes(rf, rg, th) <= 160 * 1024)
            cands.push_back(th);
    if (cands.empty()) return hipSuccess;
    float *d = nullptr, *dn = nullptr;
    int32_t *lab = nullptr;
    snx_point *rec = nullptr;
    const size_t px = (size_t)W * H;
    hipError_t e;
    if ((e = hipMalloc(&d, px * 4)) != hipSuccess) return e;
    if ((e = hipMalloc(&dn, px * 4)) != hipSuccess) { hipFree(d); return e; }
    // labels (px), the forest (px) and the root count (1)
    if ((e = hipMalloc(&lab, (2 * px + 1) * 4)) != hipSuccess) { hipFree(d); hipFree(dn); return e; }
    if ((e = hipMalloc(&rec, px * sizeof(snx_point))) != hipSuccess) {
        hipFree(d); hipFree(dn); hipFree(lab);
        return e;
    }
    int32_t *forest = lab + px, *count = lab + 2 * px;
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    hipLaunchKernelGGL(k_synth, dim3((W + 255) / 256, H), dim3(256), 0, s, d, W, H);
    hipLaunchKernelGGL(k_synth_forest, dim3((W + 255) / 256, H), dim3(256), 0, s, forest, d, W, H);
    e = hipGetLastError();
    if (e == hipSuccess) e = launch_fill_i32(lab, -1, (int64_t)px, s);
    if (e == hipSuccess) e = launch_fill_i32(count, 0, 1, s);
    // three interleaved rounds over the candidates, each candidate's fastest
    // round kept: a single sample per candidate is at the mercy of clock
    // ramps and of whatever ran just before
    std::vector<float> best(cands.size(), 1e30f);
    for (int round = 0; round < 3 && e == hipSuccess; ++round) {
        for (size_t ci = 0; ci < cands.size(); ++ci) {
            StencilArgs a;
            memset(&a, 0, sizeof a);
            a.src = d;
            a.ld_src = W;
            a.W = W;
            a.H = H;
            a.rf = rf;
            a.rg = rg;
            a.need_f = need_f;
            a.need_g = need_g;
            a.fx = a.fy = 1000.0f;
            a.b = 0.1f;
            a.u0 = 0.5f * (W - 1);
            a.v0 = 0.5f * (H - 1);
            a.ld_dn = W;
            a.labels = lab;
            a.ld_lab = W;
            a.ld_out = W;
            if (rg > 0) {
                // the pipeline's second part: resolve the forest into labels,
                // count the roots, write the records
                a.forest = forest;
                a.count = count;
                a.rec = rec;
            } else {
                a.dn = dn;
            }
            a.th = cands[ci];
            if ((e = launch_stencil(a, s)) != hipSuccess) break;
            (void)hipEventRecord(e0, s);
            for (int i = 0; i < 8 && e == hipSuccess; ++i) e = launch_stencil(a, s);
            (void)hipEventRecord(e1, s);
            if (e != hipSuccess || (e = hipEventSynchronize(e1)) != hipSuccess) break;
            float ms = 0.0f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (ms < best[ci]) best[ci] = ms;
        }
    }
    if (e == hipSuccess) {
        size_t bi = 0;
        for (size_t ci = 1; ci < cands.size(); ++ci)
            if (best[ci] < best[bi]) bi = ci;
        *chosen = cands[bi];
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    hipFree(d);
    hipFree(dn);
    hipFree(lab);
    hipFree(rec);
    if (e == hipSuccess && *chosen) {
        std::lock_guard<std::mutex> lk(g_mu);
        load_cache_locked();
        store_locked(rf, rg, size_class(W, H), *chosen);
    }
    return e;
}

}  // namespace snx
