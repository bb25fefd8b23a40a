// Connected surface components: union-find labelling on the GPU.
//
// Edges join 4-neighbours whose raw disparities pass the pairwise covered-depth
// predicate |D_p - D_q| <= max(t_abs, k_rel * min(D_p, D_q)) in binary64 (the
// stopping rule of Sec. 3.4 applied between neighbours).  Labels are the
// smallest linear index of each component, which the union-find produces by
// always hooking the larger root under the smaller one (parent[x] <= x holds at
// all times, so every root is the minimum of its tree).
//
//   k_ccl_local   one 64 x 16 tile per workgroup: union-find over the tile's
//                 edges in LDS (atomicMin hooking), then each pixel's global
//                 parent = the global index of its local root
//   k_ccl_merge   one thread per tile-seam pixel pair: global union with
//                 atomicMin hooking on the parent array
//   k_ccl_flatten each pixel follows its parent chain to the root, writes the
//                 label, and roots are counted with a wave ballot
#include "snx_internal.hpp"

namespace snx {
namespace {

constexpr int kCW = 64;    // tile width (one wave per row)
constexpr int kCH = 16;    // tile height

__device__ inline bool joined(float p, float q, double k_rel, double t_abs)
{
#pragma clang fp contract(off)
    const double a = (double)p, b = (double)q;
    const double d = fabs(a - b);
    const double t = fmax(t_abs, k_rel * fmin(a, b));
    return d <= t;
}

__device__ inline int lds_find(const int *par, int x)
{
    int p = par[x];
    while (p != x) {
        x = p;
        p = par[x];
    }
    return x;
}

__device__ inline void lds_union(int *par, int a, int b)
{
    while (true) {
        a = lds_find(par, a);
        b = lds_find(par, b);
        if (a == b) return;
        if (a < b) { const int t = a; a = b; b = t; }
        const int old = atomicMin(&par[a], b);
        if (old == a) return;
        a = old;
    }
}

__device__ inline int gload(const int32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline int g_find(const int32_t *par, int x)
{
    int p = gload(par + x);
    while (p != x) {
        x = p;
        p = gload(par + x);
    }
    return x;
}

__device__ inline void g_union(int32_t *par, int a, int b)
{
    while (true) {
        a = g_find(par, a);
        b = g_find(par, b);
        if (a == b) return;
        if (a < b) { const int t = a; a = b; b = t; }
        const int old = atomicMin(par + a, b);
        if (old == a) return;
        a = old;
    }
}

__global__ void __launch_bounds__(256)
k_ccl_local(CclArgs a)
{
    __shared__ float sd[kCH * kCW];
    __shared__ int par[kCH * kCW];
    const int x0 = blockIdx.x * kCW, y0 = blockIdx.y * kCH;
    const int tid = threadIdx.x;
    if (a.count && blockIdx.x == 0 && blockIdx.y == 0 && tid == 0) *a.count = 0;
    for (int l = tid; l < kCH * kCW; l += 256) {
        const int lx = l & 63, ly = l >> 6;
        const int gx = x0 + lx, gy = y0 + ly;
        float v = 0.0f;
        if (gx < a.W && gy < a.H) {
            const float d = a.D[(int64_t)gy * a.ld + gx];
            v = valid_disp(d) ? d : 0.0f;
        }
        sd[l] = v;
        par[l] = v > 0.0f ? l : -1;
    }
    __syncthreads();
    for (int l = tid; l < kCH * kCW; l += 256) {
        const float v = sd[l];
        if (!(v > 0.0f)) continue;
        const int lx = l & 63, ly = l >> 6;
        if (lx > 0 && sd[l - 1] > 0.0f && joined(v, sd[l - 1], a.k_rel, a.t_abs))
            lds_union(par, l, l - 1);
        if (ly > 0 && sd[l - kCW] > 0.0f && joined(v, sd[l - kCW], a.k_rel, a.t_abs))
            lds_union(par, l, l - kCW);
    }
    __syncthreads();
    for (int l = tid; l < kCH * kCW; l += 256) {
        const int lx = l & 63, ly = l >> 6;
        const int gx = x0 + lx, gy = y0 + ly;
        if (gx >= a.W || gy >= a.H) continue;
        int g = -1;
        if (sd[l] > 0.0f) {
            const int r = lds_find(par, l);
            g = (y0 + (r >> 6)) * a.W + x0 + (r & 63);
        }
        a.parent[(int64_t)gy * a.W + gx] = g;
    }
}

// Seam pairs: for every vertical tile seam (between columns x0-1 and x0) one
// thread per row, and for every horizontal seam one thread per column.
__global__ void __launch_bounds__(256)
k_ccl_merge(CclArgs a, int n_vseams, int n_hseams)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t nv = (int64_t)n_vseams * a.H;
    int p, q;
    if (i < nv) {
        const int s = (int)(i / a.H), y = (int)(i - (int64_t)s * a.H);
        const int x = (s + 1) * kCW;          // first column of the right tile
        p = y * a.W + x - 1;
        q = p + 1;
        const float dp = a.D[(int64_t)y * a.ld + x - 1];
        const float dq = a.D[(int64_t)y * a.ld + x];
        if (!valid_disp(dp) || !valid_disp(dq) || !joined(dp, dq, a.k_rel, a.t_abs)) return;
    } else {
        const int64_t j = i - nv;
        if (j >= (int64_t)n_hseams * a.W) return;
        const int s = (int)(j / a.W), x = (int)(j - (int64_t)s * a.W);
        const int y = (s + 1) * kCH;          // first row of the lower tile
        p = (y - 1) * a.W + x;
        q = p + a.W;
        const float dp = a.D[(int64_t)(y - 1) * a.ld + x];
        const float dq = a.D[(int64_t)y * a.ld + x];
        if (!valid_disp(dp) || !valid_disp(dq) || !joined(dp, dq, a.k_rel, a.t_abs)) return;
    }
    g_union(a.parent, p, q);
}

__global__ void __launch_bounds__(256)
k_ccl_flatten(CclArgs a)
{
    const int gx = blockIdx.x * 64 + (threadIdx.x & 63);
    const int gy = blockIdx.y * 4 + (threadIdx.x >> 6);
    const bool in = gx < a.W && gy < a.H;
    bool root = false;
    if (in) {
        const int x = gy * a.W + gx;
        const int p = gload(a.parent + x);
        int lab = -1;
        if (p >= 0) {
            lab = g_find(a.parent, x);
            root = lab == x;
            if (a.labels == a.parent) {
                if (lab != p) a.parent[x] = lab;
            }
        }
        if (a.labels != a.parent) a.labels[(int64_t)gy * a.ld_lab + gx] = lab;
    }
    if (a.count) {
        const unsigned long long b = __ballot(root);
        if ((threadIdx.x & 63) == 0 && b) atomicAdd(a.count, (int)__popcll(b));
    }
}

__global__ void k_fill_i32(int32_t *p, int32_t value, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = value;
}

}  // namespace

hipError_t launch_fill_i32(int32_t *p, int32_t value, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, value, n);
    return hipGetLastError();
}

hipError_t launch_components(const CclArgs &a, hipStream_t s)
{
    const int tx = (a.W + kCW - 1) / kCW, ty = (a.H + kCH - 1) / kCH;
    hipLaunchKernelGGL(k_ccl_local, dim3(tx, ty), dim3(256), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int nv = tx - 1, nh = ty - 1;
    const int64_t pairs = (int64_t)nv * a.H + (int64_t)nh * a.W;
    if (pairs > 0) {
        hipLaunchKernelGGL(k_ccl_merge, dim3((unsigned)((pairs + 255) / 256)), dim3(256), 0, s,
                           a, nv, nh);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_ccl_flatten, dim3(tx, (a.H + 3) / 4), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace snx
