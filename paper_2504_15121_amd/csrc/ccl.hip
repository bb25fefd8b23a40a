// Connected surface components on the GPU (union-find; helpers in ccl.hpp).
//
//   k_front       one 64 x 32 tile per workgroup: the local forest of the tile
//                 (ballot row runs + LDS union-find), written as the global
//                 index of each pixel's local root; optionally the filter of the
//                 same tile (window 1 or 3) from the same read of the disparity,
//                 and with the 3x3 filter's halo the tile's seam records (which
//                 of its seam pairs need a union, and the tile roots involved).
//   k_ccl_merge   one thread per tile-seam pixel pair; a pair is skipped when
//                 the previous pair along the seam is joined and both sides are
//                 joined to it inside their tiles (so the union is implied); the
//                 rest are united in the global forest with atomicMin hooking.
//   k_ccl_merge_seams  the same from the seam records (two coalesced loads a
//                 pair, one union per distinct root pair of a wave).
//   k_ccl_flatten every pixel follows its parent chain to the root, writes its
//                 own label and counts roots with a wave ballot.
//
// During the merge, parent loads bypass L1 and a hook that lost a race is
// retried from the value the atomic returned.  After the merge a pixel's entry
// only ever changes to its root, so ordinary loads that see an older value still
// lead to the right root.
#include "ccl.hpp"
#include "device.hpp"
#include "lsq.hpp"

namespace snx {
namespace {

constexpr int kFrontWaves = 8;   // 512 threads per 64 x 32 tile: four rows per wave

typedef float f32x4 __attribute__((ext_vector_type(4)));

// Loads that bypass the per-CU L1 (the merge runs concurrently with hooks done
// by other CUs).
__device__ __forceinline__ int gload(const int32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Find with path halving: a non-root entry is pointed at its grandparent.  Only
// roots are ever hooked and a non-root never becomes a root again, so the
// halving cannot undo a concurrent hook; atomicMin keeps every entry
// monotonically decreasing along its chain of ancestors.
// Roots of a and b with both chains advancing together (one round trip per
// step for the pair instead of one per chain).
__device__ __forceinline__ void g_find2(int32_t *par, int &a, int &b)
{
    bool ra = false, rb = false;
    while (!(ra && rb)) {
        const int pa = ra ? a : gload(par + a);
        const int pb = rb ? b : gload(par + b);
        ra = ra || pa == a;
        rb = rb || pb == b;
        if (ra && rb) break;
        const int ga = ra ? a : gload(par + pa);
        const int gb = rb ? b : gload(par + pb);
        if (!ra) {
            if (ga == pa) { a = pa; ra = true; }
            else { atomicMin(par + a, ga); a = ga; }
        }
        if (!rb) {
            if (gb == pb) { b = pb; rb = true; }
            else { atomicMin(par + b, gb); b = gb; }
        }
    }
}

__device__ __forceinline__ void g_union(int32_t *par, int a, int b)
{
    while (true) {
        g_find2(par, a, b);
        if (a == b) return;
        if (a < b) { const int t = a; a = b; b = t; }
        const int old = atomicMin(par + a, b);
        if (old == a) return;
        a = old;
    }
}

// The tile's local forest as global indices of each pixel's local root (-1 for
// an invalid pixel).
__device__ __forceinline__ void write_forest(const FrontArgs &a, const int *par, int x0, int y0,
                                             int lane, int wave, int nwaves = kFrontWaves)
{
    const int gx = x0 + lane;
    for (int ly = wave; ly < kCH; ly += nwaves) {
        const int gy = y0 + ly;
        if (gx >= a.W || gy >= a.H) continue;
        const int l = ly * kCW + lane;
        int g = -1;
        if (par[l] >= 0) {
            const int r = lds_find(par, l);
            g = (y0 + (r >> 6)) * a.W + x0 + (r & 63);
        }
        a.forest[(int64_t)gy * a.W + gx] = g;
    }
}

// Seam records of one tile from its halo (needs the 1-pixel halo of the 3x3
// filter, RF = 1): wave 0 the right seam, wave 1 the left, wave 2 the bottom,
// wave 3 the top.  A pair of the right or bottom seam needs a union when it is
// an edge and is not implied by the previous pair along the seam (the previous
// pair is an edge and each side of this pair is joined to its side of that one
// inside its tile), the rule the seam merge applies; its record is then the
// tile root of this tile's pixel.  The left and top seams record this tile's
// roots for the neighbours' pairs.
template <int RF>
__device__ __forceinline__ void write_seams(const FrontArgs &a, const int *par, const float *sIn,
                                            int x0, int y0, int bx, int by, int lane, int wave)
{
    constexpr int inW = kCW + 2 * RF;
    const int tx = (a.W + kCW - 1) / kCW, ty = (a.H + kCH - 1) / kCH;
    const int64_t nv = (int64_t)(tx - 1) * a.H;
    auto groot = [&](int l) {
        if (par[l] < 0) return -1;
        const int r = lds_find(par, l);
        return (y0 + (r >> 6)) * a.W + x0 + (r & 63);
    };
    auto v = [&](int ly, int lx) { return sIn[(ly + RF) * inW + lx + RF]; };
    auto e = [&](float p, float q) { return p > 0.0f && q > 0.0f && joined(p, q, a.k_rel, a.t_abs); };
    if (wave == 0 && bx < tx - 1 && lane < kCH && y0 + lane < a.H) {
        const int ly = lane;
        const bool need = e(v(ly, kCW - 1), v(ly, kCW)) &&
                          !(ly > 0 && e(v(ly - 1, kCW - 1), v(ly - 1, kCW)) &&
                            e(v(ly - 1, kCW - 1), v(ly, kCW - 1)) && e(v(ly - 1, kCW), v(ly, kCW)));
        a.seam_a[(int64_t)bx * a.H + y0 + ly] = need ? groot(ly * kCW + kCW - 1) : -1;
    } else if (wave == 1 && bx > 0 && lane < kCH && y0 + lane < a.H) {
        a.seam_b[(int64_t)(bx - 1) * a.H + y0 + lane] = groot(lane * kCW);
    } else if (wave == 2 && by < ty - 1 && x0 + lane < a.W) {
        const int lx = lane;
        const bool need = e(v(kCH - 1, lx), v(kCH, lx)) &&
                          !(lx > 0 && e(v(kCH - 1, lx - 1), v(kCH, lx - 1)) &&
                            e(v(kCH - 1, lx - 1), v(kCH - 1, lx)) && e(v(kCH, lx - 1), v(kCH, lx)));
        a.seam_a[nv + (int64_t)by * a.W + x0 + lx] = need ? groot((kCH - 1) * kCW + lx) : -1;
    } else if (wave == 3 && by > 0 && x0 + lane < a.W) {
        a.seam_b[nv + (int64_t)(by - 1) * a.W + x0 + lane] = groot(lane);
    }
}

template <int RF, bool CREASE = false>
struct FrontSmem {
    static constexpr int inW = kCW + 2 * RF, inH = kCH + 2 * RF;
    float sIn[inH * inW];
    int par[kCH * kCW];
    unsigned long long hmask[kCH];
    float nrm[CREASE ? 3 * kCH * kCW : 1];    // crease-aware: the tile's normals
};

// One 64 x 32 tile by NW waves: filter (window 1 or 3) and local component
// forest (crease-aware with CREASE: every edge also passes crease_ok).
template <int RF, bool CREASE = false, int NW = kFrontWaves>
__device__ __forceinline__ void front_tile(const FrontArgs &a, int bx, int by,
                                           FrontSmem<RF, CREASE> &sm)
{
    constexpr int inW = FrontSmem<RF, CREASE>::inW, inH = FrontSmem<RF, CREASE>::inH;
    float *sIn = sm.sIn;
    int *par = sm.par;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int x0 = bx * kCW, y0 = by * kCH;

    // issue every load of the tile before the first wait.  A tile inside the
    // frame horizontally with 16-byte aligned rows reads the 64 columns of each
    // row as 16 aligned 16-byte loads and the two halo columns as single floats
    // (no sector is fetched for a one-float overhang); other tiles read element
    // by element.
    constexpr int NTH = NW * 64;
    const int tid = threadIdx.x;
    if (x0 + kCW <= a.W && (a.ld & 3) == 0 && ((uintptr_t)a.D & 15) == 0) {
        constexpr int NB4 = inH * (kCW / 4), NL4 = (NB4 + NTH - 1) / NTH;
        f32x4 b4[NL4];
#pragma unroll
        for (int k = 0; k < NL4; ++k) {
            const int e = tid + k * NTH;
            const int ly = e / (kCW / 4), c = e - ly * (kCW / 4);
            const int gy = y0 - RF + ly;
            b4[k] = (f32x4){0.0f, 0.0f, 0.0f, 0.0f};
            if (e < NB4 && gy >= 0 && gy < a.H)
                b4[k] = __builtin_nontemporal_load(
                    reinterpret_cast<const f32x4 *>(a.D + (int64_t)gy * a.ld + x0) + c);
        }
        float hv = 0.0f;
        const int hly = tid >> 1, hside = tid & 1;
        if (RF > 0 && tid < 2 * inH) {
            const int gy = y0 - RF + hly, gx = hside ? x0 + kCW : x0 - 1;
            if (gy >= 0 && gy < a.H && gx >= 0 && gx < a.W)
                hv = __builtin_nontemporal_load(a.D + (int64_t)gy * a.ld + gx);
        }
#pragma unroll
        for (int k = 0; k < NL4; ++k) {
            const int e = tid + k * NTH;
            if (e < NB4) {
                const int ly = e / (kCW / 4), c = e - ly * (kCW / 4);
                float *d = sIn + ly * inW + RF + 4 * c;
#pragma unroll
                for (int i = 0; i < 4; ++i) d[i] = valid_disp(b4[k][i]) ? b4[k][i] : 0.0f;
            }
        }
        if (RF > 0 && tid < 2 * inH)
            sIn[hly * inW + (hside ? inW - 1 : 0)] = valid_disp(hv) ? hv : 0.0f;
    } else {
        constexpr int NT = inH * inW, NL = (NT + NTH - 1) / NTH;
        float v[NL];
#pragma unroll
        for (int k = 0; k < NL; ++k) {
            const int e = tid + k * NTH;
            const int ly = e / inW, lx = e - ly * inW;
            const int gy = y0 - RF + ly, gx = x0 - RF + lx;
            v[k] = 0.0f;
            if (e < NT && gy >= 0 && gy < a.H && gx >= 0 && gx < a.W)
                v[k] = __builtin_nontemporal_load(a.D + (int64_t)gy * a.ld + gx);
        }
#pragma unroll
        for (int k = 0; k < NL; ++k) {
            const int e = tid + k * NTH;
            if (e < NT) sIn[e] = valid_disp(v[k]) ? v[k] : 0.0f;
        }
    }
    if (CREASE) {
        for (int e = threadIdx.x; e < 3 * kCH * kCW; e += NW * 64) {
            const int c = e / (kCH * kCW), l = e - c * (kCH * kCW);
            const int gy = y0 + (l >> 6), gxx = x0 + (l & 63);
            float n = __builtin_nanf("");
            if (gy < a.H && gxx < a.W) n = a.nrm[c * a.plane_nrm + (int64_t)gy * a.ld_nrm + gxx];
            sm.nrm[e] = n;
        }
    }
    __syncthreads();

    const int gx = x0 + lane;
    auto filter_row = [&](int ly) {
        const int gy = y0 + ly;
        if (gx >= a.W || gy >= a.H) return;
        const float *p = sIn + (ly + RF) * inW + lane + RF;
        float out = __builtin_nanf("");
        if (p[0] > 0.0f) out = RF == 1 ? filter3x3(p, inW, a.need_f) : p[0];
        a.dn[(int64_t)gy * a.ld_dn + gx] = out;
    };
    auto val = [&](int ly, int ln) { return sIn[(ly + RF) * inW + ln + RF]; };
    if (!CREASE) {
        // the filter rows interleaved with the vertical unions: the waves of a
        // CU then mix the filter's arithmetic with the unions' LDS round trips
        // instead of running the two phases one after the other
        const auto E = disp_edges(val, [](int, int, int, int) { return true; }, a.k_rel, a.t_abs);
        forest_runs(E, par, sm.hmask, lane, wave, NW);
        __syncthreads();
        for (int ly = wave; ly < kCH; ly += NW) {
            if (a.dn) filter_row(ly);
            if (ly + 1 < kCH) forest_union_row(E, par, sm.hmask, lane, ly + 1);
        }
        __syncthreads();
    } else {
        if (a.dn)
            for (int ly = wave; ly < kCH; ly += NW) filter_row(ly);

        const float *n = sm.nrm;
        constexpr int P = kCH * kCW;
        local_forest(disp_edges(val,
                                [&](int la, int xa, int lb, int xb) {
                                    const int i = la * kCW + xa, j = lb * kCW + xb;
                                    return crease_ok(n[i], n[P + i], n[2 * P + i], n[j], n[P + j],
                                                     n[2 * P + j], a.crease_cos);
                                },
                                a.k_rel, a.t_abs),
                     par, sm.hmask, lane, wave, NW);
    }
    write_forest(a, par, x0, y0, lane, wave, NW);
    if (RF == 1 && !CREASE && a.seam_a) write_seams<RF>(a, par, sIn, x0, y0, bx, by, lane, wave);
}


// Local forests of an explicitly given edge graph (the labelling's test hook):
// per-pixel bits as in BitTileEdges, row stride a.ld_edges.
__global__ void __launch_bounds__(kFrontWaves * 64)
k_front_edges(FrontArgs a)
{
    __shared__ uint8_t f[kCH * kCW];
    __shared__ int par[kCH * kCW];
    __shared__ unsigned long long hmask[kCH];
    if (a.count && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) *a.count = 0;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int x0 = blockIdx.x * kCW, y0 = blockIdx.y * kCH;
    for (int e = threadIdx.x; e < kCH * kCW; e += kFrontWaves * 64) {
        const int gy = y0 + (e >> 6), gx = x0 + (e & 63);
        f[e] = gy < a.H && gx < a.W ? a.edges[(int64_t)gy * a.ld_edges + gx] : (uint8_t)0;
    }
    __syncthreads();
    local_forest(BitTileEdges{f}, par, hmask, lane, wave, kFrontWaves);
    write_forest(a, par, x0, y0, lane, wave);
}

// NW = 16 (two rows a wave) for frames of no more tiles than the chip has CUs,
// where each tile's own critical path is the kernel's time.
template <int RF, bool CREASE, int NW = kFrontWaves>
__global__ void __launch_bounds__(NW * 64)
k_front(FrontArgs a)
{
    __shared__ FrontSmem<RF, CREASE> sm;
    if (a.count && blockIdx.x == 0 && threadIdx.x == 0) *a.count = 0;
    const int tx = (a.W + kCW - 1) / kCW, ty = (a.H + kCH - 1) / kCH;
    const int t = xcd_tile(blockIdx.x, tx * ty);
    front_tile<RF, CREASE, NW>(a, t % tx, t / tx, sm);
}

// Persistent front over the (frame, tile) work list of a batch: workgroups
// fetch items with an atomic counter until the list is exhausted.
template <int RF>
__global__ void __launch_bounds__(kFrontWaves * 64)
k_front_batch(const BatchFrame *frames, const int *tile_off, const int *tile_frame, int n,
              int *counter)
{
    __shared__ FrontSmem<RF> sm;
    __shared__ int item;
    const int total = tile_off[n];
    if (threadIdx.x == 0) item = atomicAdd(counter, 1);
    __syncthreads();
    int it = item;
    while (it < total) {
        // the next item is claimed now, so the atomic's latency overlaps this tile
        int nxt = 0;
        if (threadIdx.x == 0) nxt = atomicAdd(counter, 1);
        // uniform across the workgroup: keep the index and the arguments in
        // scalar registers
        const int f = __builtin_amdgcn_readfirstlane(tile_frame[__builtin_amdgcn_readfirstlane(it)]);
        const FrontArgs a = frames[f].front;
        const int local = it - tile_off[f];
        const int tx = (a.W + kCW - 1) / kCW;
        front_tile<RF>(a, local % tx, local / tx, sm);
        __syncthreads();
        if (threadIdx.x == 0) item = nxt;
        __syncthreads();
        it = item;
    }
}

// Seam pairs.  Vertical seam s (between columns x-1 and x = (s+1)*kCW): thread
// per row y.  Horizontal seam s (between rows y-1 and y = (s+1)*kCH): thread per
// column x.  Pair i is implied by pair i-1 along the same seam when pair i-1 is
// joined and each side of pair i is joined to its side of pair i-1 (those edges
// lie inside one tile and were united by the front kernel).
// nrm (crease-aware components; else NULL): the normal planes, and every
// seam pair also passes crease_ok (the implied-pair shortcut is not taken).
__device__ __forceinline__ bool seam_crease(const float *nrm, int64_t ld_nrm, int64_t plane,
                                            double ccos, int yp, int xp, int yq, int xq)
{
    const int64_t i = (int64_t)yp * ld_nrm + xp, j = (int64_t)yq * ld_nrm + xq;
    return crease_ok(nrm[i], nrm[plane + i], nrm[2 * plane + i], nrm[j], nrm[plane + j],
                     nrm[2 * plane + j], ccos);
}

// Seam edges from the raw disparity (covered depth; crease-aware when nrm is
// set).
struct DispSeamEdges {
    const float *D;
    int64_t ld;
    double k_rel, t_abs;
    const float *nrm;
    int64_t ld_nrm, plane_nrm;
    double ccos;
    __device__ __forceinline__ bool operator()(int yp, int xp, int yq, int xq) const
    {
        if (!edge(D[(int64_t)yp * ld + xp], D[(int64_t)yq * ld + xq], k_rel, t_abs)) return false;
        return !nrm || seam_crease(nrm, ld_nrm, plane_nrm, ccos, yp, xp, yq, xq);
    }
};

// Seam edges of an explicitly given graph (bits as in BitTileEdges); q is the
// right or lower pixel of the pair.
struct BitSeamEdges {
    const uint8_t *f;
    int64_t ld;
    __device__ __forceinline__ bool operator()(int yp, int xp, int yq, int xq) const
    {
        const int a = f[(int64_t)yp * ld + xp], b = f[(int64_t)yq * ld + xq];
        return (a & 1) && (b & 1) && (b & (yq == yp ? 2 : 4));
    }
};

// One seam pair under the edges E; `shortcut` skips a pair implied by the
// previous pair along the seam.
template <class E>
__device__ __forceinline__ void merge_pair(const E &edge_at, bool shortcut, int W, int H,
                                           int32_t *par, int n_vseams, int n_hseams, int64_t i)
{
    const int64_t nv = (int64_t)n_vseams * H;
    int p, q, yp, xp, yq, xq;
    bool vert;
    if (i < nv) {
        const int s = (int)(i / H), y = (int)(i - (int64_t)s * H);
        const int x = (s + 1) * kCW;
        yp = yq = y;
        xp = x - 1;
        xq = x;
        p = y * W + x - 1;
        q = p + 1;
        vert = true;
    } else {
        const int64_t j = i - nv;
        if (j >= (int64_t)n_hseams * W) return;
        const int s = (int)(j / W), x = (int)(j - (int64_t)s * W);
        const int y = (s + 1) * kCH;
        yp = y - 1;
        yq = y;
        xp = xq = x;
        p = (y - 1) * W + x;
        q = p + W;
        vert = false;
    }
    if (!edge_at(yp, xp, yq, xq)) return;
    if (shortcut) {
        if (vert ? yp % kCH != 0 && edge_at(yp - 1, xp, yp - 1, xq) &&
                       edge_at(yp - 1, xp, yp, xp) && edge_at(yq - 1, xq, yq, xq)
                 : xp % kCW != 0 && edge_at(yp, xp - 1, yq, xq - 1) &&
                       edge_at(yp, xp - 1, yp, xp) && edge_at(yq, xq - 1, yq, xq))
            return;
    }
    // Hook first: the entries of p and q are ancestors of them (their tile
    // roots, or nearer the root after halving), so the larger is hooked under
    // the smaller at once.  If it was still a root the union is done in two
    // round trips; otherwise its old parent, like it an ancestor of one side,
    // is united with the other side by the general path.
    int a = gload(par + p), b = gload(par + q);
    if (a == b) return;
    if (a < b) { const int t = a; a = b; b = t; }
    const int old = atomicMin(par + a, b);
    if (old == a) return;
    g_union(par, old, b);
}

__device__ __forceinline__ void merge_pair(const float *D, int64_t ld, int W, int H, double k_rel,
                                           double t_abs, int32_t *par, int n_vseams,
                                           int n_hseams, int64_t i, const float *nrm = nullptr,
                                           int64_t ld_nrm = 0, int64_t plane_nrm = 0,
                                           double ccos = 0.0)
{
    merge_pair(DispSeamEdges{D, ld, k_rel, t_abs, nrm, ld_nrm, plane_nrm, ccos}, !nrm, W, H, par,
               n_vseams, n_hseams, i);
}

// Unites the root pairs (a, b) of the active lanes (a, b tile roots of the
// forest par of frame f, a != b).  Pairs of one seam are consecutive threads,
// and a seam often joins the same two tile roots at several pairs that the
// implied-pair rule does not catch: within a wave only the first lane of each
// distinct (frame, root pair) is united (the others would only find the roots
// already joined, after contending for them).
__device__ __forceinline__ void unite_root_pairs(int32_t *par, int a, int b, int f, bool act)
{
    if (a < b) { const int t = a; a = b; b = t; }
    const int lane = threadIdx.x & 63;
    bool lead = false;
    unsigned long long m = __ballot(act);
    while (m) {
        const int l = __ffsll((long long)m) - 1;
        const int la = __builtin_amdgcn_readlane(a, l), lb = __builtin_amdgcn_readlane(b, l);
        const int lf = __builtin_amdgcn_readlane(f, l);
        const bool same = act && a == la && b == lb && f == lf;
        lead = lead || lane == l;
        m &= ~__ballot(same);
    }
    if (!lead) return;
    const int old = atomicMin(par + a, b);
    if (old == a) return;
    g_union(par, old, b);
}

// Seam pairs from the front's seam records: only pairs that need a union do
// any further work (one round trip for the records, then the hook).
__global__ void __launch_bounds__(256)
k_ccl_merge_seams(const int32_t *seam_a, const int32_t *seam_b, int64_t pairs, int32_t *par)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    int a = -1, b = -1;
    if (i < pairs) {
        a = seam_a[i];
        b = seam_b[i];
    }
    unite_root_pairs(par, a, b, 0, a >= 0 && a != b);
}

// The same over the seam records of every frame of a batch (frame f's records
// at seam_off[f]).
__global__ void __launch_bounds__(256)
k_merge_batch_seams(const BatchFrame *frames, const int64_t *seam_off, const int *block_frame,
                    int n, const int32_t *seam_a, const int32_t *seam_b)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    int a = -1, b = -1, f = 0;
    int32_t *par = nullptr;
    if (i < seam_off[n]) {
        f = block_frame[blockIdx.x];
        while (seam_off[f + 1] <= i) ++f;
        a = seam_a[i];
        b = seam_b[i];
        par = frames[f].front.forest;
    }
    unite_root_pairs(par, a, b, f, a >= 0 && a != b);
}

__global__ void __launch_bounds__(256)
k_ccl_merge_edges(const uint8_t *f, int64_t ld, int W, int H, int32_t *par, int n_vseams,
                  int n_hseams)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    merge_pair(BitSeamEdges{f, ld}, true, W, H, par, n_vseams, n_hseams, i);
}

__global__ void __launch_bounds__(256)
k_ccl_merge(const float *D, int64_t ld, int W, int H, double k_rel, double t_abs, int32_t *par,
            int n_vseams, int n_hseams, const float *nrm, int64_t ld_nrm, int64_t plane_nrm,
            double ccos)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    merge_pair(D, ld, W, H, k_rel, t_abs, par, n_vseams, n_hseams, i, nrm, ld_nrm, plane_nrm,
               ccos);
}

// Seam pairs of every frame of a batch, one thread each.
// Pair i of the batch; the frame of a block's first pair comes from a table and
// the frames of later pairs in the block by stepping forward.
__global__ void __launch_bounds__(256)
k_merge_batch(const BatchFrame *frames, const int64_t *seam_off, const int *block_frame, int n)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= seam_off[n]) return;
    int f = block_frame[blockIdx.x];
    while (seam_off[f + 1] <= i) ++f;
    const FrontArgs &a = frames[f].front;
    const int tx = (a.W + kCW - 1) / kCW, ty = (a.H + kCH - 1) / kCH;
    merge_pair(a.D, a.ld, a.W, a.H, a.k_rel, a.t_abs, a.forest, tx - 1, ty - 1, i - seam_off[f]);
}

// Work counters and per-frame component counts start at zero on every run.
__global__ void k_batch_reset(int *counters, int n_counters, const BatchFrame *frames, int n)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n_counters) counters[i] = 0;
    if (i < n && frames[i].front.count) *frames[i].front.count = 0;
}

__global__ void __launch_bounds__(256)
k_ccl_flatten(CclArgs a)
{
    __shared__ int s_roots;   // roots of this block, one global atomic per block
    if (threadIdx.x == 0) s_roots = 0;
    __syncthreads();
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
        if ((threadIdx.x & 63) == 0 && b) atomicAdd(&s_roots, (int)__popcll(b));
        __syncthreads();
        if (threadIdx.x == 0 && s_roots) atomicAdd(a.count, s_roots);
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

hipError_t launch_front(const FrontArgs &a, hipStream_t s)
{
    const int tiles = ((a.W + kCW - 1) / kCW) * ((a.H + kCH - 1) / kCH);
    const dim3 grid(tiles);
    int cus = 0;
    hipError_t e = device_cus(&cus);
    if (e != hipSuccess) return e;
    // a frame whose tiles all get a CU of their own: 16 waves a tile
    const bool wide = tiles <= cus;
    if (a.nrm) {
        if (a.rf != 0 || a.dn) return hipErrorInvalidValue;   // crease-aware: forest only
        hipLaunchKernelGGL((k_front<0, true>), grid, dim3(kFrontWaves * 64), 0, s, a);
    } else if (a.rf == 0) {
        if (wide) hipLaunchKernelGGL((k_front<0, false, 16>), grid, dim3(16 * 64), 0, s, a);
        else hipLaunchKernelGGL((k_front<0, false>), grid, dim3(kFrontWaves * 64), 0, s, a);
    } else if (a.rf == 1) {
        if (wide) hipLaunchKernelGGL((k_front<1, false, 16>), grid, dim3(16 * 64), 0, s, a);
        else hipLaunchKernelGGL((k_front<1, false>), grid, dim3(kFrontWaves * 64), 0, s, a);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int front_tiles(int W, int H) { return ((W + kCW - 1) / kCW) * ((H + kCH - 1) / kCH); }

int64_t merge_pairs(int W, int H)
{
    const int tx = (W + kCW - 1) / kCW, ty = (H + kCH - 1) / kCH;
    return (int64_t)(tx - 1) * H + (int64_t)(ty - 1) * W;
}

hipError_t launch_batch_front(const BatchFrame *frames, const int *tile_off, const int *tile_frame,
                              int n, int rf, int *counter, int grid, hipStream_t s)
{
    if (rf == 0)
        hipLaunchKernelGGL(k_front_batch<0>, dim3(grid), dim3(kFrontWaves * 64), 0, s, frames,
                           tile_off, tile_frame, n, counter);
    else if (rf == 1)
        hipLaunchKernelGGL(k_front_batch<1>, dim3(grid), dim3(kFrontWaves * 64), 0, s, frames,
                           tile_off, tile_frame, n, counter);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_batch_merge(const BatchFrame *frames, const int64_t *seam_off,
                              const int *block_frame, int n, int64_t total, hipStream_t s,
                              const int32_t *seam_a, const int32_t *seam_b)
{
    if (total <= 0) return hipSuccess;
    if (seam_a)
        hipLaunchKernelGGL(k_merge_batch_seams, dim3((unsigned)((total + 255) / 256)), dim3(256),
                           0, s, frames, seam_off, block_frame, n, seam_a, seam_b);
    else
        hipLaunchKernelGGL(k_merge_batch, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s,
                           frames, seam_off, block_frame, n);
    return hipGetLastError();
}

hipError_t launch_batch_reset(int *counters, int n_counters, const BatchFrame *frames, int n,
                              hipStream_t s)
{
    const int m = n > n_counters ? n : n_counters;
    hipLaunchKernelGGL(k_batch_reset, dim3((m + 255) / 256), dim3(256), 0, s, counters,
                       n_counters, frames, n);
    return hipGetLastError();
}

hipError_t launch_merge(const float *D, int64_t ld, int W, int H, double k_rel, double t_abs,
                        int32_t *forest, hipStream_t s, const float *nrm, int64_t ld_nrm,
                        int64_t plane_nrm, double crease_cos)
{
    const int tx = (W + kCW - 1) / kCW, ty = (H + kCH - 1) / kCH;
    const int nv = tx - 1, nh = ty - 1;
    const int64_t pairs = (int64_t)nv * H + (int64_t)nh * W;
    if (pairs <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_ccl_merge, dim3((unsigned)((pairs + 255) / 256)), dim3(256), 0, s, D, ld,
                       W, H, k_rel, t_abs, forest, nv, nh, nrm, ld_nrm, plane_nrm, crease_cos);
    return hipGetLastError();
}

hipError_t launch_merge_seams(const int32_t *seam_a, const int32_t *seam_b, int64_t pairs,
                              int32_t *forest, hipStream_t s)
{
    if (pairs <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_ccl_merge_seams, dim3((unsigned)((pairs + 255) / 256)), dim3(256), 0, s,
                       seam_a, seam_b, pairs, forest);
    return hipGetLastError();
}

hipError_t launch_components(const CclArgs &a, hipStream_t s)
{
    if (a.edges) {
        // explicitly given edge graph: its own forest and seam kernels, the
        // same union-find and flattening
        FrontArgs f = {};
        f.W = a.W;
        f.H = a.H;
        f.forest = a.parent;
        f.count = a.count;
        f.edges = a.edges;
        f.ld_edges = a.ld;
        const dim3 grid((a.W + kCW - 1) / kCW, (a.H + kCH - 1) / kCH);
        hipLaunchKernelGGL(k_front_edges, grid, dim3(kFrontWaves * 64), 0, s, f);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        const int nv = (int)grid.x - 1, nh = (int)grid.y - 1;
        const int64_t pairs = (int64_t)nv * a.H + (int64_t)nh * a.W;
        if (pairs > 0) {
            hipLaunchKernelGGL(k_ccl_merge_edges, dim3((unsigned)((pairs + 255) / 256)), dim3(256),
                               0, s, a.edges, a.ld, a.W, a.H, a.parent, nv, nh);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
        hipLaunchKernelGGL(k_ccl_flatten, dim3((a.W + 63) / 64, (a.H + 3) / 4), dim3(256), 0, s, a);
        return hipGetLastError();
    }
    FrontArgs f;
    f.D = a.D;
    f.ld = a.ld;
    f.W = a.W;
    f.H = a.H;
    f.k_rel = a.k_rel;
    f.t_abs = a.t_abs;
    f.rf = 0;
    f.need_f = 3;
    f.dn = nullptr;
    f.ld_dn = 0;
    f.forest = a.parent;
    f.count = a.count;
    f.nrm = a.nrm;
    f.ld_nrm = a.ld_nrm;
    f.plane_nrm = a.plane_nrm;
    f.crease_cos = a.crease_cos;
    hipError_t e = launch_front(f, s);
    if (e != hipSuccess) return e;
    e = launch_merge(a.D, a.ld, a.W, a.H, a.k_rel, a.t_abs, a.parent, s, a.nrm, a.ld_nrm,
                     a.plane_nrm, a.crease_cos);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_ccl_flatten, dim3((a.W + 63) / 64, (a.H + 3) / 4), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace snx
