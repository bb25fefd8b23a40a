// Fused LDS-tiled stencil: masked LSQ filter -> masked anchored LSQ slope ->
// affine A -> normal -> point record, for one 64 x TH output tile per workgroup.
//
// Filter (Sec. 3.2 over-determined LSQ with a constant column, solved by
// Cramer's rule on the exact integer normal matrix): a 3x3 window is evaluated
// directly with all six mask moments packed in one int32; larger windows use the
// separable row/column moments of lsq.hpp.  Slope (Sec. 3.2-3.3 eqs. convprep /
// convprep2 with per-pixel alpha, beta, gamma as in the two-pass scheme of
// Sec. 3.4) always uses the separable moments.  Then a1 = 1 - g_u, a2 = -g_v
// (Sec. 2 eq. affine_mtx, positive-disparity convention) and the normal of
// Sec. 3.1.
//
// The kernel is a template on the two radii and the tile height so that the
// common windows are fully unrolled with constant tap offsets and constant
// divisors; a runtime instance serves every other window.
#include "ccl.hpp"
#include "lsq.hpp"

namespace snx {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

struct Layout {
    int R, inW, inH, dtW, dtH;
    size_t off_dt, off_ab, off_s, bytes;
};

__host__ __device__ constexpr size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

__host__ __device__ inline Layout make_layout(int rf, int rg, int th)
{
    Layout L;
    L.R = rf + rg;
    L.inW = kTileW + 2 * L.R;
    L.inH = th + 2 * L.R;
    L.dtW = kTileW + 2 * rg;
    L.dtH = th + 2 * rg;
    size_t off = align_up(sizeof(float) * (size_t)L.inH * L.inW, 16);
    L.off_dt = off;
    if (rf > 0) off = align_up(off + sizeof(float) * (size_t)L.dtH * L.dtW, 16);
    size_t nrow = 0;
    if (rf >= 2) nrow = (size_t)L.inH * L.dtW;
    if (rg > 0 && (size_t)L.dtH * kTileW > nrow) nrow = (size_t)L.dtH * kTileW;
    L.off_ab = off;
    off = align_up(off + sizeof(int2) * nrow, 16);
    L.off_s = off;
    off = align_up(off + sizeof(double2) * nrow, 16);
    L.bytes = off;
    return L;
}

// Threads per workgroup of an instance: 512 (8 waves, 4 resident per SIMD with
// two workgroups' LDS on a CU) for tiles of 16 rows or more, else 256.
__host__ __device__ constexpr int stencil_block(int th) { return th >= 16 ? 512 : kBlock; }

// Waves per SIMD an unrolled instance is built for: as many workgroups as its
// LDS lets share a CU, at most four waves a SIMD (then at most 128 VGPRs); the
// large windows, one workgroup a CU, get the registers they need unspilled.
__host__ __device__ constexpr size_t layout_bytes(int rf, int rg, int th)
{
    // make_layout's total, for compile-time use
    const int R = rf + rg, inW = kTileW + 2 * R, inH = th + 2 * R;
    const int dtW = kTileW + 2 * rg, dtH = th + 2 * rg;
    size_t off = align_up(sizeof(float) * (size_t)inH * inW, 16);
    if (rf > 0) off = align_up(off + sizeof(float) * (size_t)dtH * dtW, 16);
    size_t nrow = 0;
    if (rf >= 2) nrow = (size_t)inH * dtW;
    if (rg > 0 && (size_t)dtH * kTileW > nrow) nrow = (size_t)dtH * kTileW;
    off = align_up(off + 8 * nrow, 16);
    return align_up(off + 16 * nrow, 16);
}

__host__ __device__ constexpr int stencil_waves(int rf, int rg, int th)
{
    const size_t wgs = (size_t)160 * 1024 / layout_bytes(rf, rg, th);
    const int w = (stencil_block(th) / 256) * (int)(wgs < 1 ? 1 : wgs);
    return w > 4 ? 4 : w;
}

// One 64 x th output tile of the stencil.
template <int RF, int RG, int TH>
__device__ __forceinline__ void stencil_tile(const StencilArgs &a, int bx, int by,
                                             unsigned char *smem)
{
    constexpr int NB = stencil_block(TH);        // threads
    // Outputs: thread (wave w, lane x) owns runs of RPT consecutive rows of
    // column x, rows RPT w + kRowStep j .. + RPT - 1, j = 0, 1, ...: the column
    // sums of a run's first row are direct, the others slide down one row
    constexpr int RPT = TH > 0 && TH * 64 / NB > 2 ? TH * 64 / NB : 2;
    constexpr int kRowStep = RPT * (NB / 64);   // rows covered by one round of runs
    const int rf = RF >= 0 ? RF : a.rf;
    const int rg = RG >= 0 ? RG : a.rg;
    const int th = TH > 0 ? TH : a.th;
    const Layout L = make_layout(rf, rg, th);
    float *sIn = reinterpret_cast<float *>(smem);
    float *sDt = rf > 0 ? reinterpret_cast<float *>(smem + L.off_dt) : sIn;
    int2 *sAB = reinterpret_cast<int2 *>(smem + L.off_ab);
    double2 *sS = reinterpret_cast<double2 *>(smem + L.off_s);

    const int tid = threadIdx.x;
    const int x0 = bx * kTileW;
    const int y0 = by * th;
    const int R = L.R;

    // ---- A: validity-coded input tile with halo R --------------------------
    // Labels (or the label forest) of this thread's outputs are fetched first so
    // their latency overlaps the LDS phases.
    const int px_col = tid & 63, px_row = RPT * (tid >> 6);
    constexpr int kPairs = TH > 0 ? (TH + kRowStep - 1) / kRowStep : 1;
    int32_t lab0[RPT * kPairs], labr[RPT * kPairs];   // forest entries, their roots
    if (TH > 0) {
#pragma unroll
        for (int j = 0; j < kPairs; ++j)
#pragma unroll
            for (int h = 0; h < RPT; ++h) {
                const int ty = px_row + kRowStep * j + h;
                const int gx = x0 + px_col, gy = y0 + ty;
                int32_t v = -1;
                if (rg > 0 && ty < th && gx < a.W && gy < a.H) {
                    if (a.forest) v = a.forest[gy * a.W + gx];
                    else if (a.labels) v = a.labels[(int64_t)gy * a.ld_lab + gx];
                }
                lab0[RPT * j + h] = v;
                labr[RPT * j + h] = v;
            }
    }
    if (RF >= 0 && RG >= 0 && TH > 0) {
        // static tile: issue every load before the first wait
        constexpr int sR = (RF > 0 ? RF : 0) + (RG > 0 ? RG : 0);
        constexpr int sW = kTileW + 2 * sR, sH = (TH > 0 ? TH : 1) + 2 * sR;
        constexpr int NT = sW * sH, NL = (NT + NB - 1) / NB;
        // a tile whose rows (with halo) lie inside the frame and start on a
        // 16-byte boundary reads them as aligned 16-byte loads
        constexpr int Q = sW / 4, NQ = Q * sH, NLQ = (NQ + NB - 1) / NB;
        const bool vec = sR % 4 == 0 && x0 - sR >= 0 && x0 + kTileW + sR <= a.W &&
                         (a.ld_src & 3) == 0 && ((uintptr_t)a.src & 15) == 0;
        float v[NL];
        f32x4 q[NLQ];
        if (vec) {
#pragma unroll
            for (int k = 0; k < NLQ; ++k) {
                const int e = tid + k * NB;
                const int ly = e / Q, c = e - ly * Q;
                const int gy = y0 - sR + ly;
                q[k] = (f32x4){0.0f, 0.0f, 0.0f, 0.0f};
                if (e < NQ && gy >= 0 && gy < a.H)
                    q[k] = __builtin_nontemporal_load(
                        reinterpret_cast<const f32x4 *>(a.src + (int64_t)gy * a.ld_src + x0 - sR) + c);
            }
        } else {
#pragma unroll
            for (int k = 0; k < NL; ++k) {
                const int e = tid + k * NB;
                const int ly = e / sW, lx = e - ly * sW;
                const int gy = y0 - sR + ly, gx = x0 - sR + lx;
                v[k] = 0.0f;
                if (e < NT && gy >= 0 && gy < a.H && gx >= 0 && gx < a.W)
                    v[k] = __builtin_nontemporal_load(a.src + (int64_t)gy * a.ld_src + gx);
            }
        }
        if (vec) {
#pragma unroll
            for (int k = 0; k < NLQ; ++k) {
                const int e = tid + k * NB;
                if (e < NQ) {
                    float *d = sIn + 4 * e;     // row-major with sW = 4 Q floats a row
#pragma unroll
                    for (int i = 0; i < 4; ++i) d[i] = valid_disp(q[k][i]) ? q[k][i] : 0.0f;
                }
            }
        } else {
#pragma unroll
            for (int k = 0; k < NL; ++k) {
                const int e = tid + k * NB;
                if (e < NT) sIn[e] = valid_disp(v[k]) ? v[k] : 0.0f;
            }
        }
    } else {
        for (int e = tid; e < L.inH * L.inW; e += NB) {
            const int ly = e / L.inW, lx = e - ly * L.inW;
            const int gy = y0 - R + ly, gx = x0 - R + lx;
            float v = 0.0f;
            if (gy >= 0 && gy < a.H && gx >= 0 && gx < a.W) {
                const float d = __builtin_nontemporal_load(a.src + (int64_t)gy * a.ld_src + gx);
                v = valid_disp(d) ? d : 0.0f;
            }
            sIn[e] = v;
        }
    }
    __syncthreads();

    // ---- B: filter into sDt (validity-coded) and the optional plane ---------
    if (rf > 0) {
        if (rf >= 2) {
            for (int e = tid; e < L.inH * L.dtW; e += NB) {
                const int ly = e / L.dtW, j = e - ly * L.dtW;
                const RowMom m = row_moments<RF>(sIn + ly * L.inW + j, rf);
                sAB[e] = make_int2(m.a, m.b);
                sS[e] = make_double2(m.s0, m.s1);
            }
            __syncthreads();
        }
        for (int e = tid; e < L.dtH * L.dtW; e += NB) {
            const int ty = e / L.dtW, j = e - ty * L.dtW;
            const float Dc = sIn[(ty + rf) * L.inW + j + rf];
            float outv = __builtin_nanf("");
            if (Dc > 0.0f) {
                if (rf == 1) {
                    outv = filter3x3(sIn + (ty + 1) * L.inW + j + 1, L.inW, a.need_f);
                } else {
                    const ColMom m = col_moments<RF, true>(sAB + e, sS + e, L.dtW, rf);
                    outv = filter_solve(m, Dc, a.need_f);
                }
            }
            const int gx = x0 - rg + j, gy = y0 - rg + ty;
            const bool inimg = gx >= 0 && gx < a.W && gy >= 0 && gy < a.H;
            sDt[e] = inimg && valid_disp(outv) ? outv : 0.0f;
            if (a.dn && inimg && ty >= rg && ty < rg + th && j >= rg && j < rg + kTileW)
                a.dn[(int64_t)gy * a.ld_dn + gx] = outv;
        }
        __syncthreads();
    } else if (a.dn) {
        for (int e = tid; e < th * kTileW; e += NB) {
            const int ty = e >> 6, tx = e & 63;
            const int gx = x0 + tx, gy = y0 + ty;
            if (gx < a.W && gy < a.H) {
                const float v = sIn[(ty + R) * L.inW + tx + R];
                a.dn[(int64_t)gy * a.ld_dn + gx] = v > 0.0f ? v : __builtin_nanf("");
            }
        }
    }
    if (rg == 0) return;

    // ---- C: anchored masked LSQ slope, A, normal, labels, records ------------
    // Roots found in this tile are counted in LDS and added to the global count
    // once per tile: one contended atomic per workgroup instead of one per wave
    // and row.
    __shared__ int s_roots;
    if (tid == 0) s_roots = 0;
    // row moments: runs of 4 consecutive centres per thread (sliding window).
    // Within a row, the moments of column x sit at slot (x % 4) * 16 + x / 4, so
    // at every step of the runs the lanes of a wave write consecutive slots (no
    // LDS bank conflicts), and a row's 64 columns still fill its 64 slots.
    constexpr int kRun = 4, kRuns = kTileW / kRun;
    // The owned pixels' forest entries are resolved to their roots around the
    // row pass: the first step's loads are issued before it and consumed after
    // it (global loads and LDS work wait on separate counters), the rest of the
    // chains advance together afterwards.
    constexpr bool kChase = RF >= 0 && RG >= 0 && TH > 0;
    int32_t hop[kChase ? RPT * kPairs : 1];
    if (kChase && a.forest) {
#pragma unroll
        for (int k = 0; k < RPT * kPairs; ++k) hop[k] = labr[k] >= 0 ? a.forest[labr[k]] : labr[k];
    }
    for (int e = tid; e < L.dtH * kRuns; e += NB) {
        const int ly = e / kRuns, run = e - ly * kRuns;
        row_moments_run<RG, kRun, kRuns>(sDt + ly * L.dtW + run * kRun, rg,
                                         sAB + ly * kTileW + run, sS + ly * kTileW + run);
    }
    __syncthreads();
    if (kChase && a.forest) {
        bool again = false;
#pragma unroll
        for (int k = 0; k < RPT * kPairs; ++k)
            if (hop[k] != labr[k]) {
                labr[k] = hop[k];
                again = true;
            }
        while (again) {
            again = false;
#pragma unroll
            for (int k = 0; k < RPT * kPairs; ++k) hop[k] = labr[k] >= 0 ? a.forest[labr[k]] : labr[k];
#pragma unroll
            for (int k = 0; k < RPT * kPairs; ++k)
                if (hop[k] != labr[k]) {
                    labr[k] = hop[k];
                    again = true;
                }
        }
    }
    // column moments: the first row of a run by direct sums, the others by
    // sliding the window down one row.  The runs are unrolled for the static
    // tile heights so that the per-run label registers are indexed statically.
    auto pair = [&](int j) {
        const int ty0 = px_row + kRowStep * j, tx = px_col;
        const int eo = ty0 * kTileW + (tx % kRun) * kRuns + tx / kRun;
        ColMom m = col_moments<RG, true>(sAB + eo, sS + eo, kTileW, rg);
#pragma unroll
        for (int h = 0; h < RPT; ++h) {
            const int ty = ty0 + h;
            if (h >= 1) {
                if (ty >= th) break;
                m = col_slide(m, sAB + eo + (h - 1) * kTileW, sS + eo + (h - 1) * kTileW, kTileW,
                              rg);
            }
            const int gx = x0 + tx, gy = y0 + ty;
            const bool in = gx < a.W && gy < a.H;
            const float Dc = sDt[(ty + rg) * L.dtW + tx + rg];
            float nx = __builtin_nanf(""), ny = nx, nz = nx, a1 = nx, a2 = nx;
            if (in && Dc > 0.0f) {
                double gu, gv;
                if (slope_solve(m, Dc, a.need_g, gu, gv)) {
                    a1 = (float)(1.0 - gu);
                    a2 = (float)(-gv);
                    normal_from_slope(gu, gv, Dc, gx, gy, a.fx, a.fy, a.u0, a.v0, nx, ny, nz);
                }
            }
            int32_t lab = -1;
            bool root = false;
            int32_t first = -1;
            if (in) {
                if (TH > 0) first = lab0[RPT * j + h];
                else if (a.forest) first = a.forest[gy * a.W + gx];
                else if (a.labels) first = a.labels[(int64_t)gy * a.ld_lab + gx];
            }
            if (in && a.forest) {
                const int x = gy * a.W + gx;
                const int p = first;
                if (p >= 0) {
                    lab = (RF >= 0 && RG >= 0 && TH > 0) ? labr[RPT * j + h] : flat_find(a.forest, p);
                    root = lab == x;
                    if (a.labels == a.forest) {
                        if (lab != p) a.forest[x] = lab;
                    }
                }
                if (a.labels != a.forest) a.labels[(int64_t)gy * a.ld_lab + gx] = lab;
            } else if (in && a.labels) {
                lab = first;
            }
            if (a.count) {
                const unsigned long long b = __ballot(root);
                if ((tid & 63) == 0 && b) atomicAdd(&s_roots, (int)__popcll(b));
            }
            if (!in) continue;
            const int64_t o = (int64_t)gy * a.ld_out + gx;
            if (a.aff) {
                a.aff[o] = a1;
                a.aff[o + a.plane_out] = a2;
            }
            if (a.nrm) {
                a.nrm[o] = nx;
                a.nrm[o + a.plane_out] = ny;
                a.nrm[o + 2 * a.plane_out] = nz;
            }
            if (a.rec) {
                const snx_point p = make_point(gx, gy, Dc > 0.0f ? Dc : 0.0f, nx, ny, nz, lab,
                                               a.fx, a.fy, a.b, a.u0, a.v0);
                store_point(a.rec + (int64_t)gy * a.W + gx, p);
            }
        }
    };
    if (TH > 0) {
#pragma unroll
        for (int j = 0; j < kPairs; ++j)
            if (px_row + kRowStep * j < th) pair(j);
    } else {
        for (int j = 0; px_row + kRowStep * j < th; ++j) pair(j);
    }
    if (a.count) {
        __syncthreads();
        if (tid == 0 && s_roots) atomicAdd(a.count, s_roots);
    }
}

// two 512-thread workgroups per CU need at most 128 VGPRs (4 waves a SIMD)
template <int RF, int RG, int TH>
__global__ void __launch_bounds__(stencil_block(TH))
__attribute__((amdgpu_waves_per_eu(TH > 0 && RF >= 0 && RG >= 0 ? stencil_waves(RF, RG, TH) : 4)))
k_stencil(StencilArgs a)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const int th = TH > 0 ? TH : a.th;
    const int tx = (a.W + kTileW - 1) / kTileW, ty = (a.H + th - 1) / th;
    const int t = xcd_tile(blockIdx.x, tx * ty);
    stencil_tile<RF, RG, TH>(a, t % tx, t / tx, smem);
}

// Persistent back stage over the (frame, tile) work list of a batch.
template <int RG, int TH>
__global__ void __launch_bounds__(stencil_block(TH))
__attribute__((amdgpu_waves_per_eu(stencil_waves(0, RG, TH))))
k_back_batch(const BatchFrame *frames, const int *tile_off, const int *tile_frame, int n,
             int *counter)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
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
        const StencilArgs a = frames[f].back;
        const int local = it - tile_off[f];
        const int tx = (a.W + kTileW - 1) / kTileW;
        stencil_tile<0, RG, TH>(a, local % tx, local / tx, smem);
        __syncthreads();
        if (threadIdx.x == 0) item = nxt;
        __syncthreads();
        it = item;
    }
}

using KernelFn = void (*)(StencilArgs);

template <int RF, int RG, int TH>
constexpr KernelFn kfn() { return &k_stencil<RF, RG, TH>; }

// (rf, rg, th) with a fully unrolled instance; the autotuner chooses among the
// tile heights compiled for a window pair.
struct Inst { int rf, rg, th; KernelFn fn; };
constexpr Inst kInst[] = {
    // gradient only (snx_affine_normals, second part of snx_pipeline)
    {0, 1, 16, kfn<0, 1, 16>()}, {0, 1, 32, kfn<0, 1, 32>()},
    {0, 2, 16, kfn<0, 2, 16>()}, {0, 2, 32, kfn<0, 2, 32>()},
    {0, 3, 16, kfn<0, 3, 16>()}, {0, 3, 32, kfn<0, 3, 32>()},
    {0, 4, 8, kfn<0, 4, 8>()},   {0, 4, 16, kfn<0, 4, 16>()}, {0, 4, 24, kfn<0, 4, 24>()},
    {0, 4, 32, kfn<0, 4, 32>()},
    {0, 7, 8, kfn<0, 7, 8>()},   {0, 7, 16, kfn<0, 7, 16>()}, {0, 7, 32, kfn<0, 7, 32>()},
    {0, 10, 8, kfn<0, 10, 8>()}, {0, 10, 16, kfn<0, 10, 16>()}, {0, 10, 32, kfn<0, 10, 32>()},
    {0, 15, 8, kfn<0, 15, 8>()}, {0, 15, 16, kfn<0, 15, 16>()}, {0, 15, 32, kfn<0, 15, 32>()},
    {0, 22, 4, kfn<0, 22, 4>()}, {0, 22, 8, kfn<0, 22, 8>()},   {0, 22, 16, kfn<0, 22, 16>()},
    {0, 22, 32, kfn<0, 22, 32>()},
    {0, 30, 4, kfn<0, 30, 4>()}, {0, 30, 8, kfn<0, 30, 8>()},   {0, 30, 16, kfn<0, 30, 16>()},
    // fused 3x3 filter + gradient (snx_oriented_point_cloud)
    {1, 1, 16, kfn<1, 1, 16>()}, {1, 2, 16, kfn<1, 2, 16>()}, {1, 3, 16, kfn<1, 3, 16>()},
    {1, 4, 8, kfn<1, 4, 8>()},   {1, 4, 16, kfn<1, 4, 16>()}, {1, 4, 32, kfn<1, 4, 32>()},
    {1, 7, 16, kfn<1, 7, 16>()},
    {2, 2, 16, kfn<2, 2, 16>()}, {2, 4, 16, kfn<2, 4, 16>()}, {4, 4, 16, kfn<4, 4, 16>()},
    // filter only (snx_denoise)
    {1, 0, 16, kfn<1, 0, 16>()}, {1, 0, 32, kfn<1, 0, 32>()},
    {2, 0, 16, kfn<2, 0, 16>()}, {4, 0, 16, kfn<4, 0, 16>()},
};

}  // namespace

size_t stencil_lds_bytes(int rf, int rg, int th) { return make_layout(rf, rg, th).bytes; }

// the compile-time LDS size used for the instances' occupancy agrees with the layout
static_assert(layout_bytes(0, 4, 32) == 72960 && layout_bytes(1, 4, 16) > 0, "layout size");

int back_tiles(int W, int H, int th) { return ((W + kTileW - 1) / kTileW) * ((H + th - 1) / th); }

using BatchFn = void (*)(const BatchFrame *, const int *, const int *, int, int *);
struct BatchInst { int rg, th; BatchFn fn; };
constexpr BatchInst kBatchInst[] = {
    {1, 16, &k_back_batch<1, 16>}, {2, 16, &k_back_batch<2, 16>}, {3, 16, &k_back_batch<3, 16>},
    {4, 8, &k_back_batch<4, 8>},   {4, 16, &k_back_batch<4, 16>}, {4, 24, &k_back_batch<4, 24>},
    {4, 32, &k_back_batch<4, 32>},
    {7, 8, &k_back_batch<7, 8>},   {7, 16, &k_back_batch<7, 16>}, {10, 8, &k_back_batch<10, 8>},
    {10, 16, &k_back_batch<10, 16>}, {10, 32, &k_back_batch<10, 32>},
    {15, 8, &k_back_batch<15, 8>}, {15, 16, &k_back_batch<15, 16>}, {15, 32, &k_back_batch<15, 32>},
    {22, 4, &k_back_batch<22, 4>}, {22, 8, &k_back_batch<22, 8>}, {22, 16, &k_back_batch<22, 16>},
    {22, 32, &k_back_batch<22, 32>},
    {30, 4, &k_back_batch<30, 4>}, {30, 8, &k_back_batch<30, 8>}, {30, 16, &k_back_batch<30, 16>},
};

bool batch_has_instance(int rg, int th)
{
    for (const BatchInst &i : kBatchInst)
        if (i.rg == rg && i.th == th) return true;
    return false;
}

hipError_t launch_batch_back(const BatchFrame *frames, const int *tile_off, const int *tile_frame,
                             int n, int rg, int th, int *counter, int grid, hipStream_t s)
{
    for (const BatchInst &i : kBatchInst)
        if (i.rg == rg && i.th == th) {
            hipLaunchKernelGGL(i.fn, dim3(grid), dim3(stencil_block(th)),
                               stencil_lds_bytes(0, rg, th), s,
                               frames, tile_off, tile_frame, n, counter);
            return hipGetLastError();
        }
    return hipErrorInvalidValue;
}

bool stencil_has_instance(int rf, int rg, int th)
{
    for (const Inst &i : kInst)
        if (i.rf == rf && i.rg == rg && i.th == th) return true;
    return false;
}

// Default tile height: the first of 16, 8, 4, 32 that has an unrolled instance
// and fits 64 KB of LDS (several workgroups per CU), else one with an instance
// that fits the 160 KB of one gfx950 CU, else the tallest that fits for the
// generic (runtime-window) kernel.
int stencil_pick_tile_height(int rf, int rg)
{
    for (size_t cap : {(size_t)64 * 1024, (size_t)160 * 1024})
        for (int th : {16, 8, 4, 32})
            if (stencil_has_instance(rf, rg, th) && stencil_lds_bytes(rf, rg, th) <= cap)
                return th;
    for (size_t cap : {(size_t)64 * 1024, (size_t)160 * 1024})
        for (int th : {16, 8, 4, 2, 1})
            if (stencil_lds_bytes(rf, rg, th) <= cap) return th;
    return 0;
}

hipError_t launch_stencil(const StencilArgs &a, hipStream_t s)
{
    const size_t lds = stencil_lds_bytes(a.rf, a.rg, a.th);
    if (lds > 160 * 1024) return hipErrorInvalidConfiguration;
    const dim3 grid(((a.W + kTileW - 1) / kTileW) * ((a.H + a.th - 1) / a.th));
    KernelFn fn = &k_stencil<-1, -1, 0>;
    int nb = kBlock;
    for (const Inst &i : kInst)
        if (i.rf == a.rf && i.rg == a.rg && i.th == a.th) {
            fn = i.fn;
            nb = stencil_block(i.th);
        }
    hipLaunchKernelGGL(fn, grid, dim3(nb), lds, s, a);
    return hipGetLastError();
}

}  // namespace snx
