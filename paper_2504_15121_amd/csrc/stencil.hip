// Fused LDS-tiled stencil: masked LSQ filter -> masked anchored LSQ slope ->
// affine A -> normal -> point record, for one 64 x TH output tile per workgroup.
//
// Both LSQ stages need, per pixel, the same separable window moments of a
// validity-coded image v (v_i = D_i if valid else 0, m_i = [v_i > 0]):
//     mask moments   sum m, sum m dx, sum m dy, sum m dx^2, sum m dx dy, sum m dy^2
//     data moments   sum v, sum dx v, sum dy v
// They are computed as a row pass (per row, over dx) stored in LDS, followed by a
// column pass (over dy).  The three row mask moments are small integers packed
// into one int32; the data moments are accumulated in FP64 (full-rate on CDNA4
// vector ALUs once packed FP32 is off), so the uncentred sums lose nothing to
// cancellation before the centring D_i - D_c is applied algebraically.  Every
// determinant is an integer below 2^53 and is formed exactly in FP64.
//
// Filter (Sec. 3.2 LSQ with a constant column, solved by Cramer's rule on the
// exact integer normal matrix) and slope (Sec. 3.2-3.3 eqs. convprep /
// convprep2 with per-pixel alpha, beta, gamma as in the two-pass scheme of
// Sec. 3.4) follow; then a1 = 1 - g_u, a2 = -g_v (Sec. 2 eq. affine_mtx with the
// positive-disparity convention) and the normal of Sec. 3.1.
//
// The kernel is a template on the two radii so that the common windows are fully
// unrolled with constant tap offsets and constant-divisor index arithmetic; a
// runtime-radius instance serves every other window.
#include "snx_internal.hpp"

namespace snx {
namespace {

// Packed row mask moments: c0 in bits 0..5, (c1 + 512) in bits 6..15, c2 in
// bits 16..30.  Exact for windows up to 63 (c0 <= 63, |c1| <= 496, c2 <= 20832).
constexpr int kC1Off = 512;
__device__ inline int pack_tap(int dx) { return 1 + dx * 64 + dx * dx * 65536; }
__device__ inline void unpack(int p, int &c0, int &c1, int &c2)
{
    c0 = p & 63;
    c1 = ((p >> 6) & 1023) - kC1Off;
    c2 = p >> 16;
}

struct Layout {
    int R, inW, inH, dtW, dtH;
    size_t off_dt, off_c, off_s0, off_s1, bytes;
};

__host__ __device__ inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

__host__ __device__ inline Layout make_layout(int rf, int rg, int th)
{
    Layout L;
    L.R = rf + rg;
    L.inW = kTileW + 2 * L.R;
    L.inH = th + 2 * L.R;
    L.dtW = kTileW + 2 * rg;
    L.dtH = th + 2 * rg;
    // the filter row pass covers inH rows x dtW columns, the slope row pass
    // dtH rows x kTileW columns; one set of buffers serves both
    size_t off = align_up(sizeof(float) * (size_t)L.inH * L.inW, 16);
    L.off_dt = off;
    if (rf > 0) off = align_up(off + sizeof(float) * (size_t)L.dtH * L.dtW, 16);
    L.off_c = off;
    const size_t nrow = (size_t)L.inH * L.dtW;
    off = align_up(off + sizeof(int) * nrow, 16);
    L.off_s0 = off;
    off = align_up(off + sizeof(double) * nrow, 16);
    L.off_s1 = off;
    off = align_up(off + sizeof(double) * nrow, 16);
    L.bytes = off;
    return L;
}

// Row pass: packed mask moments and FP64 data moments of the window
// p[0 .. 2r] (centre p[r]).
template <int RC>
__device__ inline void row_moments(const float *p, int r_rt, int &c, double &s0, double &s1)
{
    const int r = RC >= 0 ? RC : r_rt;
    c = kC1Off * 64;
    s0 = 0.0;
    s1 = 0.0;
#pragma unroll
    for (int k = 0; k <= 2 * r; ++k) {
        const float v = p[k];
        const int dx = k - r;
        c += v > 0.0f ? pack_tap(dx) : 0;
        const double dv = (double)v;
        s0 += dv;
        s1 += (double)dx * dv;
    }
}

template <int RF, int RG, int TH>
__global__ void __launch_bounds__(kBlock)
k_stencil(StencilArgs a)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const int rf = RF >= 0 ? RF : a.rf;
    const int rg = RG >= 0 ? RG : a.rg;
    const int th = TH > 0 ? TH : a.th;
    const Layout L = make_layout(rf, rg, th);
    float *sIn = reinterpret_cast<float *>(smem);
    float *sDt = rf > 0 ? reinterpret_cast<float *>(smem + L.off_dt) : sIn;
    int *sC = reinterpret_cast<int *>(smem + L.off_c);
    double *sS0 = reinterpret_cast<double *>(smem + L.off_s0);
    double *sS1 = reinterpret_cast<double *>(smem + L.off_s1);

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    constexpr int kWaves = kBlock / 64;
    const int x0 = blockIdx.x * kTileW;
    const int y0 = blockIdx.y * th;
    const int R = L.R;

    // ---- A: validity-coded input tile with halo R --------------------------
    for (int ly = wave; ly < L.inH; ly += kWaves) {
        const int gy = y0 - R + ly;
        const bool rowin = gy >= 0 && gy < a.H;
        const float *row = a.src + (int64_t)(rowin ? gy : 0) * a.ld_src;
        for (int lx = lane; lx < L.inW; lx += 64) {
            const int gx = x0 - R + lx;
            float v = 0.0f;
            if (rowin && gx >= 0 && gx < a.W) {
                const float d = __builtin_nontemporal_load(row + gx);
                v = valid_disp(d) ? d : 0.0f;
            }
            sIn[ly * L.inW + lx] = v;
        }
    }
    __syncthreads();

    // ---- B: filter (masked LSQ plane intercept) into sDt --------------------
    if (rf > 0) {
        // B1: row moments over dx for inH rows x dtW columns
        for (int e = tid; e < L.inH * L.dtW; e += kBlock) {
            const int ly = e / L.dtW, j = e - ly * L.dtW;
            int c;
            double s0, s1;
            row_moments<RF>(sIn + ly * L.inW + j, rf, c, s0, s1);
            sC[e] = c;
            sS0[e] = s0;
            sS1[e] = s1;
        }
        __syncthreads();
        // B2: column moments over dy, solve, store the validity-coded result
        for (int e = tid; e < L.dtH * L.dtW; e += kBlock) {
            const int ty = e / L.dtW, j = e - ty * L.dtW;
            const float Dc = sIn[(ty + rf) * L.inW + j + rf];
            float out = 0.0f;      // coded (0 = invalid)
            float outv = __builtin_nanf("");
            if (Dc > 0.0f) {
                int N = 0, Sx = 0, Sy = 0, Sxx = 0, Sxy = 0, Syy = 0;
                double R0 = 0.0, Rx = 0.0, Ry = 0.0;
#pragma unroll
                for (int k = 0; k <= 2 * rf; ++k) {
                    const int dy = k - rf;
                    const int idx = e + k * L.dtW;
                    int c0, c1, c2;
                    unpack(sC[idx], c0, c1, c2);
                    N += c0; Sx += c1; Sy += dy * c0;
                    Sxx += c2; Sxy += dy * c1; Syy += dy * dy * c0;
                    const double s0 = sS0[idx];
                    R0 += s0;
                    Rx += sS1[idx];
                    Ry += (double)dy * s0;
                }
                double h = (double)Dc;
                if (N >= a.need_f) {
                    // exact integers below 2^53 for windows up to 63
                    const double n = N, sx = Sx, sy = Sy, sxx = Sxx, sxy = Sxy, syy = Syy;
                    const double m11 = sxx * syy - sxy * sxy;
                    const double m12 = sx * syy - sxy * sy;
                    const double m13 = sx * sxy - sxx * sy;
                    const double det = n * m11 - sx * m12 + sy * m13;
                    if (det != 0.0) {
                        const double dc = (double)Dc;
                        const double r0 = R0 - n * dc;
                        const double r1 = Rx - sx * dc;
                        const double r2 = Ry - sy * dc;
                        const double num = r0 * m11 - sx * (r1 * syy - sxy * r2)
                                         + sy * (r1 * sxy - sxx * r2);
                        h = dc + num / det;
                    }
                }
                outv = (float)h;
                out = valid_disp(outv) ? outv : 0.0f;
            }
            const int gx = x0 - rg + j, gy = y0 - rg + ty;
            const bool inimg = gx >= 0 && gx < a.W && gy >= 0 && gy < a.H;
            sDt[e] = inimg ? out : 0.0f;
            if (a.dn && inimg && ty >= rg && ty < rg + th && j >= rg && j < rg + kTileW)
                a.dn[(int64_t)gy * a.ld_dn + gx] = outv;
        }
        __syncthreads();
    } else if (a.dn) {
        // identity filter: copy the (coded) centre values out
        for (int e = tid; e < th * kTileW; e += kBlock) {
            const int ty = e >> 6, tx = e & 63;
            const int gx = x0 + tx, gy = y0 + ty;
            if (gx < a.W && gy < a.H) {
                const float v = sIn[(ty + R) * L.inW + tx + R];
                a.dn[(int64_t)gy * a.ld_dn + gx] = v > 0.0f ? v : __builtin_nanf("");
            }
        }
    }
    if (rg == 0) return;

    // ---- C: anchored masked LSQ slope, A, normal, records --------------------
    // C1: row moments over dx for dtH rows x 64 columns (centre column rg + tx)
    for (int e = tid; e < L.dtH * kTileW; e += kBlock) {
        const int ly = e >> 6, tx = e & 63;
        int c;
        double s0, s1;
        row_moments<RG>(sDt + ly * L.dtW + tx, rg, c, s0, s1);
        sC[e] = c;
        sS0[e] = s0;
        sS1[e] = s1;
    }
    __syncthreads();
    // C2: column moments, slope, outputs
    for (int e = tid; e < th * kTileW; e += kBlock) {
        const int ty = e >> 6, tx = e & 63;
        const int gx = x0 + tx, gy = y0 + ty;
        if (gx >= a.W || gy >= a.H) continue;
        const float Dc = sDt[(ty + rg) * L.dtW + tx + rg];
        float nx = __builtin_nanf(""), ny = nx, nz = nx, a1 = nx, a2 = nx;
        if (Dc > 0.0f) {
            int N = 0, Sx = 0, Sy = 0, Sxx = 0, Sxy = 0, Syy = 0;
            double Px = 0.0, Py = 0.0;
#pragma unroll
            for (int k = 0; k <= 2 * rg; ++k) {
                const int dy = k - rg;
                const int idx = e + k * kTileW;
                int c0, c1, c2;
                unpack(sC[idx], c0, c1, c2);
                N += c0; Sx += c1; Sy += dy * c0;
                Sxx += c2; Sxy += dy * c1; Syy += dy * dy * c0;
                Px += sS1[idx];
                Py += (double)dy * sS0[idx];
            }
            const int Ng = N - 1;   // the centre itself is not a neighbour
            const double al = Sxx, be = Sxy, ga = Syy;
            const double det = al * ga - be * be;   // exact
            if (Ng >= a.need_g && det > 0.0) {
                const double dc = (double)Dc;
                const double S1 = Px - (double)Sx * dc;
                const double S2 = Py - (double)Sy * dc;
                const double inv = 1.0 / det;
                const double gu = (ga * S1 - be * S2) * inv;
                const double gv = (al * S2 - be * S1) * inv;
                a1 = (float)(1.0 - gu);
                a2 = (float)(-gv);
                const double mxd = (double)a.fx * gu;
                const double myd = (double)a.fy * gv;
                const double mzd = dc - ((double)gx - (double)a.u0) * gu
                                      - ((double)gy - (double)a.v0) * gv;
                const float mx = (float)mxd, my = (float)myd, mz = (float)mzd;
                const float s = -__frsqrt_rn(mx * mx + my * my + mz * mz);
                nx = mx * s;
                ny = my * s;
                nz = mz * s;
            }
        }
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
            const int32_t lab = a.labels ? a.labels[(int64_t)gy * a.ld_lab + gx] : -1;
            const snx_point p = make_point(gx, gy, Dc > 0.0f ? Dc : 0.0f, nx, ny, nz, lab,
                                           a.fx, a.fy, a.b, a.u0, a.v0);
            store_point(a.rec + (int64_t)gy * a.W + gx, p);
        }
    }
}

using KernelFn = void (*)(StencilArgs);

template <int RF, int RG, int TH>
constexpr KernelFn kfn() { return &k_stencil<RF, RG, TH>; }

// (rf, rg) pairs with a fully unrolled instance at tile height 16.
struct Inst { int rf, rg; KernelFn fn; };
constexpr Inst kInst[] = {
    {1, 4, kfn<1, 4, 16>()}, {0, 4, kfn<0, 4, 16>()}, {1, 0, kfn<1, 0, 16>()},
    {0, 1, kfn<0, 1, 16>()}, {0, 2, kfn<0, 2, 16>()}, {0, 3, kfn<0, 3, 16>()},
    {0, 7, kfn<0, 7, 16>()}, {1, 1, kfn<1, 1, 16>()}, {1, 2, kfn<1, 2, 16>()},
    {1, 3, kfn<1, 3, 16>()}, {1, 7, kfn<1, 7, 16>()}, {2, 4, kfn<2, 4, 16>()},
    {2, 2, kfn<2, 2, 16>()}, {2, 7, kfn<2, 7, 16>()}, {2, 0, kfn<2, 0, 16>()},
    {4, 0, kfn<4, 0, 16>()}, {4, 4, kfn<4, 4, 16>()},
};

}  // namespace

size_t stencil_lds_bytes(int rf, int rg, int th) { return make_layout(rf, rg, th).bytes; }

// Tallest tile whose LDS fits 64 KB (several workgroups per CU), else the
// tallest that fits the 160 KB of one gfx950 CU.
int stencil_pick_tile_height(int rf, int rg)
{
    for (int th : {16, 8, 4}) {
        if (stencil_lds_bytes(rf, rg, th) <= 64 * 1024) return th;
    }
    for (int th : {16, 8, 4, 2, 1}) {
        if (stencil_lds_bytes(rf, rg, th) <= 160 * 1024) return th;
    }
    return 0;
}

hipError_t launch_stencil(const StencilArgs &a, hipStream_t s)
{
    const size_t lds = stencil_lds_bytes(a.rf, a.rg, a.th);
    dim3 grid((a.W + kTileW - 1) / kTileW, (a.H + a.th - 1) / a.th);
    KernelFn fn = &k_stencil<-1, -1, 0>;
    if (a.th == 16) {
        for (const Inst &i : kInst)
            if (i.rf == a.rf && i.rg == a.rg) fn = i.fn;
    }
    hipLaunchKernelGGL(fn, grid, dim3(kBlock), lds, s, a);
    return hipGetLastError();
}

}  // namespace snx
