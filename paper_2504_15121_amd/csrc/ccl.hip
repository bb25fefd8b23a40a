// Connected surface components: union-find labelling on the GPU.
//
// Edges join 4-neighbours whose raw disparities pass the pairwise covered-depth
// predicate |D_p - D_q| <= max(t_abs, k_rel * min(D_p, D_q)) in binary64 (the
// stopping rule of Sec. 3.4 applied between neighbours).  Labels are the
// smallest linear index of each component, which the union-find produces by
// always hooking the larger root under the smaller one (parent[x] <= x holds at
// all times, so every root is the minimum of its tree).
//
//   k_ccl_local   one 64 x 32 tile per workgroup, one wave per row at a time
//                 (lane = column): horizontal edges as a 64-bit ballot give the
//                 row runs, whose first pixel is the initial root; vertical
//                 edges are united in LDS (atomicMin hooking) except where the
//                 edge to the left already connects the same two runs; each
//                 pixel's global parent is the global index of its local root.
//   k_ccl_merge   one thread per tile-seam pixel pair; a pair is skipped when
//                 the previous pair along the seam is joined and both sides are
//                 joined to it inside their tiles (so the union is implied);
//                 the rest are united in the global parent array.
//   k_ccl_flatten every pixel follows its parent chain to the root, writes its
//                 own label and counts roots with a wave ballot.
//
// During the merge, parent loads bypass L1 and a hook that lost a race is
// retried from the value the atomic returned.  The flatten runs after every hook
// is done; there, a pixel's entry only changes to its root, so ordinary loads
// that see an older value still lead to the right root.
#include "snx_internal.hpp"

namespace snx {
namespace {

constexpr int kCW = 64;    // tile width (one wave = one row of the tile)
constexpr int kCH = 32;    // tile height
constexpr int kCWaves = 4;

__device__ inline bool joined(float p, float q, double k_rel, double t_abs)
{
#pragma clang fp contract(off)
    const double a = (double)p, b = (double)q;
    const double d = fabs(a - b);
    const double t = fmax(t_abs, k_rel * fmin(a, b));
    return d <= t;
}

__device__ inline bool edge(float p, float q, double k_rel, double t_abs)
{
    return valid_disp(p) && valid_disp(q) && joined(p, q, k_rel, t_abs);
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

// Loads that bypass the per-CU L1 (the merge runs concurrently with hooks done
// by other CUs).
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

// Root of x after every hook is done: parents only move to ancestors during the
// flatten, so plain loads that see an older value still reach the root.
__device__ inline int flat_find(const int32_t *par, int x)
{
    int p = par[x];
    while (p != x) {
        x = p;
        p = par[x];
    }
    return x;
}

// Highest set bit position at or below `lane` of the run-start mask: the start
// of the run that contains `lane`.
__device__ inline int run_start(unsigned long long starts, int lane)
{
    const unsigned long long upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
    return 63 - __clzll(starts & upto);
}

__global__ void __launch_bounds__(kCWaves * 64)
k_ccl_local(CclArgs a)
{
    __shared__ float sd[kCH * kCW];
    __shared__ int par[kCH * kCW];
    __shared__ unsigned long long hmask[kCH];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int x0 = blockIdx.x * kCW, y0 = blockIdx.y * kCH;
    const int gx = x0 + lane;
    if (a.count && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) *a.count = 0;

    // rows: values, horizontal-edge ballots, run-start parents
    for (int ly = wave; ly < kCH; ly += kCWaves) {
        const int gy = y0 + ly;
        float v = 0.0f;
        if (gx < a.W && gy < a.H) {
            const float d = a.D[(int64_t)gy * a.ld + gx];
            v = valid_disp(d) ? d : 0.0f;
        }
        const float left = __shfl_up(v, 1);
        const bool ok = v > 0.0f;
        const bool h = ok && lane > 0 && left > 0.0f && joined(v, left, a.k_rel, a.t_abs);
        const unsigned long long hb = __ballot(h);
        const unsigned long long vb = __ballot(ok);
        sd[ly * kCW + lane] = v;
        par[ly * kCW + lane] = ok ? ly * kCW + run_start(vb & ~hb, lane) : -1;
        if (lane == 0) hmask[ly] = hb;
    }
    __syncthreads();
    // vertical edges between row ly-1 and ly
    for (int ly = 1 + wave; ly < kCH; ly += kCWaves) {
        const float v = sd[ly * kCW + lane];
        const float up = sd[(ly - 1) * kCW + lane];
        const bool e = v > 0.0f && up > 0.0f && joined(v, up, a.k_rel, a.t_abs);
        const unsigned long long eb = __ballot(e);
        // the edge at lane-1 already joins the same two runs when both rows
        // continue their run from lane-1 to lane
        const unsigned long long implied = (eb << 1) & hmask[ly] & hmask[ly - 1];
        if (e && !((implied >> lane) & 1ull)) lds_union(par, ly * kCW + lane, (ly - 1) * kCW + lane);
    }
    __syncthreads();
    for (int ly = wave; ly < kCH; ly += kCWaves) {
        const int gy = y0 + ly;
        if (gx >= a.W || gy >= a.H) continue;
        const int l = ly * kCW + lane;
        int g = -1;
        if (par[l] >= 0) {
            const int r = lds_find(par, l);
            g = (y0 + (r >> 6)) * a.W + x0 + (r & 63);
        }
        a.parent[(int64_t)gy * a.W + gx] = g;
    }
}

// Seam pairs.  Vertical seam s (between columns x-1 and x = (s+1)*kCW): thread
// per row y.  Horizontal seam s (between rows y-1 and y = (s+1)*kCH): thread per
// column x.  Pair i is implied by pair i-1 along the same seam when pair i-1 is
// joined and each side of pair i is joined to its side of pair i-1 (those edges
// lie inside one tile and were united by k_ccl_local).
__global__ void __launch_bounds__(256)
k_ccl_merge(CclArgs a, int n_vseams, int n_hseams)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t nv = (int64_t)n_vseams * a.H;
    int p, q;
    if (i < nv) {
        const int s = (int)(i / a.H), y = (int)(i - (int64_t)s * a.H);
        const int x = (s + 1) * kCW;
        const float *r = a.D + (int64_t)y * a.ld;
        const float dp = r[x - 1], dq = r[x];
        if (!edge(dp, dq, a.k_rel, a.t_abs)) return;
        if (y % kCH != 0) {
            const float *u = r - a.ld;
            const float up = u[x - 1], uq = u[x];
            if (edge(up, uq, a.k_rel, a.t_abs) && edge(up, dp, a.k_rel, a.t_abs) &&
                edge(uq, dq, a.k_rel, a.t_abs))
                return;
        }
        p = y * a.W + x - 1;
        q = p + 1;
    } else {
        const int64_t j = i - nv;
        if (j >= (int64_t)n_hseams * a.W) return;
        const int s = (int)(j / a.W), x = (int)(j - (int64_t)s * a.W);
        const int y = (s + 1) * kCH;
        const float *ra = a.D + (int64_t)(y - 1) * a.ld;
        const float *rb = ra + a.ld;
        const float dp = ra[x], dq = rb[x];
        if (!edge(dp, dq, a.k_rel, a.t_abs)) return;
        if (x % kCW != 0) {
            const float lp = ra[x - 1], lq = rb[x - 1];
            if (edge(lp, lq, a.k_rel, a.t_abs) && edge(lp, dp, a.k_rel, a.t_abs) &&
                edge(lq, dq, a.k_rel, a.t_abs))
                return;
        }
        p = (y - 1) * a.W + x;
        q = p + a.W;
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
        const int p = a.parent[x];
        int lab = -1;
        if (p >= 0) {
            // each thread writes only its own entry: with in-place labels every
            // entry is some pixel's final label
            lab = flat_find(a.parent, p);
            root = lab == x;
            if (a.labels == a.parent && p != lab) a.parent[x] = lab;
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
    hipLaunchKernelGGL(k_ccl_local, dim3(tx, ty), dim3(kCWaves * 64), 0, s, a);
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
