// Union-find helpers for connected surface components, shared by the
// components kernels and the fused front kernel.
//
// Edges join 4-neighbours whose raw disparities pass the pairwise covered-depth
// predicate |D_p - D_q| <= max(t_abs, k_rel * min(D_p, D_q)) in binary64 (the
// stopping rule of Sec. 3.4 applied between neighbours).  Labels are the
// smallest linear index of each component: the union-find always hooks the
// larger root under the smaller one, so parent[x] <= x holds at all times and
// every root is the minimum of its tree.
#pragma once

#include "snx_internal.hpp"

namespace snx {

constexpr int kCW = 64;    // components tile width (one wave = one tile row)
constexpr int kCH = 32;    // components tile height

__device__ __forceinline__ bool joined(float p, float q, double k_rel, double t_abs)
{
#pragma clang fp contract(off)
    const double a = (double)p, b = (double)q;
    const double d = fabs(a - b);
    const double t = fmax(t_abs, k_rel * fmin(a, b));
    return d <= t;
}

__device__ __forceinline__ bool edge(float p, float q, double k_rel, double t_abs)
{
    return valid_disp(p) && valid_disp(q) && joined(p, q, k_rel, t_abs);
}

// Normal-crease test of crease-aware components: the two unit normals agree,
// ((ax bx + ay by) + az bz) >= cos_min in binary64 (each product of two float32
// values is exact); an undefined (NaN) normal imposes no test.
__device__ __forceinline__ bool crease_ok(float ax, float ay, float az, float bx, float by,
                                          float bz, double cos_min)
{
#pragma clang fp contract(off)
    if (ax != ax || bx != bx) return true;
    const double d = ((double)ax * (double)bx + (double)ay * (double)by) + (double)az * (double)bz;
    return d >= cos_min;
}

__device__ __forceinline__ int lds_find(const int *par, int x)
{
    int p = par[x];
    while (p != x) {
        x = p;
        p = par[x];
    }
    return x;
}

__device__ __forceinline__ void lds_union(int *par, int a, int b)
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

// Root of x once every hook is done: entries only change to their root, so
// plain loads that see an older value still reach the root.
__device__ __forceinline__ int flat_find(const int32_t *par, int x)
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
__device__ __forceinline__ int run_start(unsigned long long starts, int lane)
{
    const unsigned long long upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
    return 63 - __clzll(starts & upto);
}

// Edges of a tile for local_forest, from validity-coded values in LDS at
// val(ly, lane) (0 = invalid) and the covered-depth predicate;
// extra(ly_a, x_a, ly_b, x_b) is a further condition on an edge (always true for
// the covered-depth components).  Every lane of the wave calls left() together.
template <class Val, class Extra>
struct DispTileEdges {
    Val val;
    Extra extra;
    double k_rel, t_abs;
    __device__ __forceinline__ bool ok(int ly, int lane) const { return val(ly, lane) > 0.0f; }
    // edge between (ly, lane - 1) and (ly, lane)
    __device__ __forceinline__ bool left(int ly, int lane) const
    {
        const float v = val(ly, lane);
        const float l = __shfl_up(v, 1);
        return v > 0.0f && lane > 0 && l > 0.0f && joined(v, l, k_rel, t_abs) &&
               extra(ly, lane > 0 ? lane - 1 : lane, ly, lane);
    }
    // edge between (ly - 1, lane) and (ly, lane)
    __device__ __forceinline__ bool up(int ly, int lane) const
    {
        const float v = val(ly, lane), u = val(ly - 1, lane);
        return v > 0.0f && u > 0.0f && joined(v, u, k_rel, t_abs) && extra(ly - 1, lane, ly, lane);
    }
};

template <class Val, class Extra>
__device__ __forceinline__ DispTileEdges<Val, Extra> disp_edges(Val val, Extra extra,
                                                                double k_rel, double t_abs)
{
    return DispTileEdges<Val, Extra>{val, extra, k_rel, t_abs};
}

// Edges of a tile given explicitly (the labelling's test hook): per-pixel bits
// in LDS at f[ly * kCW + lane]: bit 0 present, bit 1 edge to the left
// neighbour, bit 2 edge to the upper neighbour; an edge needs both pixels.
struct BitTileEdges {
    const uint8_t *f;
    __device__ __forceinline__ bool ok(int ly, int lane) const { return f[ly * kCW + lane] & 1; }
    __device__ __forceinline__ bool left(int ly, int lane) const
    {
        const int c = f[ly * kCW + lane];
        const int l = __shfl_up(c, 1);
        return (c & 1) && lane > 0 && (l & 1) && (c & 2);
    }
    __device__ __forceinline__ bool up(int ly, int lane) const
    {
        const int c = f[ly * kCW + lane], u = f[(ly - 1) * kCW + lane];
        return (c & 1) && (u & 1) && (c & 4);
    }
};

// Local labelling of one kCW x kCH tile with the edges of E, in two phases that
// each take every nwaves-th row starting at `wave`: forest_runs gives the row
// runs from a 64-bit ballot of the horizontal edges (the first pixel of a run is
// its initial root); after a barrier, forest_unions unites the vertical edges
// with atomicMin hooking, except where the edge at lane-1 already joins the same
// two runs.  After a second barrier par[] holds a local forest over
// ly*kCW + lane.
template <class Edges>
__device__ __forceinline__ void forest_runs(const Edges &E, int *par, unsigned long long *hmask,
                                            int lane, int wave, int nwaves)
{
    for (int ly = wave; ly < kCH; ly += nwaves) {
        const bool ok = E.ok(ly, lane);
        const bool h = E.left(ly, lane);
        const unsigned long long hb = __ballot(h);
        const unsigned long long vb = __ballot(ok);
        par[ly * kCW + lane] = ok ? ly * kCW + run_start(vb & ~hb, lane) : -1;
        if (lane == 0) hmask[ly] = hb;
    }
}

// The vertical unions between rows ly - 1 and ly (1 <= ly < kCH).
template <class Edges>
__device__ __forceinline__ void forest_union_row(const Edges &E, int *par,
                                                 const unsigned long long *hmask, int lane, int ly)
{
    const bool e = E.up(ly, lane);
    const unsigned long long eb = __ballot(e);
    const unsigned long long implied = (eb << 1) & hmask[ly] & hmask[ly - 1];
    if (e && !((implied >> lane) & 1ull)) lds_union(par, ly * kCW + lane, (ly - 1) * kCW + lane);
}

template <class Edges>
__device__ __forceinline__ void forest_unions(const Edges &E, int *par,
                                              const unsigned long long *hmask, int lane, int wave,
                                              int nwaves)
{
    for (int ly = 1 + wave; ly < kCH; ly += nwaves) forest_union_row(E, par, hmask, lane, ly);
}

template <class Edges>
__device__ __forceinline__ void local_forest(const Edges &E, int *par, unsigned long long *hmask,
                                             int lane, int wave, int nwaves)
{
    forest_runs(E, par, hmask, lane, wave, nwaves);
    __syncthreads();
    forest_unions(E, par, hmask, lane, wave, nwaves);
    __syncthreads();
}

}  // namespace snx
