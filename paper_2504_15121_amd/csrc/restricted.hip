// Component-restricted gradient window: the anchored LSQ slope, A and normal
// over the pixels of the n_g x n_g window that are valid and carry the centre's
// surface-component label (the concern of Sec. 3.4 that points of a
// neighbouring surface smooth the normals, met with the components of the
// covered-depth predicate).  One 64 x 16 output tile per 256-thread workgroup.
//
// The mask depends on the centre's label, so the window sums are not
// separable in general: each centre walks its window in LDS (validity-coded D~
// and the labels, halo r), one row at a time; a row's integer moments and its
// two data sums (exact FP64 sums of float32 values times small integers) are
// combined into the column moments with the row offset.  Each wave owns four
// consecutive output rows; where every valid pixel that its windows reach
// carries one label, the mask of every centre there is the plain validity
// mask, and the wave takes the separable route instead: per column, the row
// moments of its 2r + 1 rows summed once, then the window slid down a row at a
// time.  Every sum is exact either way, so both routes give the same numbers.
// The solve, A and normal are the square-window ones.
#include "lsq.hpp"

namespace snx {
namespace {

constexpr int kRsW = 64, kRsH = 16, kRsBlock = 256;

template <int RC>
__global__ void __launch_bounds__(kRsBlock)
k_affine_labels(RestrictArgs a)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const int r = RC > 0 ? RC : a.r;
    const int LW = kRsW + 2 * r, LH = kRsH + 2 * r;
    float *sD = reinterpret_cast<float *>(smem);
    int32_t *sL = reinterpret_cast<int32_t *>(smem + sizeof(float) * (size_t)LW * LH);
    const int tid = threadIdx.x;
    const int x0 = blockIdx.x * kRsW, y0 = blockIdx.y * kRsH;

    for (int e = tid; e < LW * LH; e += kRsBlock) {
        const int ly = e / LW, lx = e - ly * LW;
        const int gy = y0 - r + ly, gx = x0 - r + lx;
        float v = 0.0f;
        int32_t l = -1;
        if (gy >= 0 && gy < a.H && gx >= 0 && gx < a.W) {
            const float d = a.src[(int64_t)gy * a.ld_src + gx];
            v = valid_disp(d) ? d : 0.0f;
            l = a.labels[(int64_t)gy * a.ld_lab + gx];
        }
        sD[e] = v;
        sL[e] = l;
    }
    __syncthreads();

    const int tx = tid & 63, wave = tid >> 6;
    constexpr int kRows = kRsH / (kRsBlock / 64);   // output rows per wave
    const int ty0 = kRows * wave;
    auto output = [&](int ty, float a1, float a2, float nx, float ny, float nz) {
        const int64_t o = (int64_t)(y0 + ty) * a.ld_out + x0 + tx;
        if (a.aff) {
            a.aff[o] = a1;
            a.aff[o + a.plane_out] = a2;
        }
        if (a.nrm) {
            a.nrm[o] = nx;
            a.nrm[o + a.plane_out] = ny;
            a.nrm[o + 2 * a.plane_out] = nz;
        }
    };
    // one label among the valid pixels of LDS rows ty0 .. ty0 + kRows - 1 + 2r
    // (every window of this wave's outputs)?
    int lmin = 0x7fffffff, lmax = -0x7fffffff - 1;
    for (int ly = ty0; ly < ty0 + kRows + 2 * r && ly < LH; ++ly)
        for (int lx = tx; lx < LW; lx += 64) {
            const int e = ly * LW + lx;
            if (sD[e] > 0.0f) {
                lmin = min(lmin, sL[e]);
                lmax = max(lmax, sL[e]);
            }
        }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        lmin = min(lmin, __shfl_xor(lmin, o));
        lmax = max(lmax, __shfl_xor(lmax, o));
    }
    __shared__ int s_mixed[kRsBlock / 64], s_next;
    if (tx == 0) s_mixed[wave] = lmin < lmax;
    if (tid == 0) s_next = 0;
    __syncthreads();
    const bool gx_in = x0 + tx < a.W;
    if (lmin >= lmax) {
        // separable route: row moments of LDS row ly for this column's window
        auto rowm = [&](int ly) { return row_moments<(RC > 0 ? RC : -1)>(sD + ly * LW + tx, r); };
        ColMom m;
        m.N = m.Sx = m.Sy = m.Sxx = m.Sxy = m.Syy = 0;
        m.R0 = m.Rx = m.Ry = 0.0;
        for (int dy = -r; dy <= r; ++dy) {
            const RowMom q = rowm(ty0 + r + dy);
            const int c0 = q.a & 0xffff, c1 = (q.a >> 16) - kColOff;
            m.N += c0;
            m.Sx += c1;
            m.Sy += dy * c0;
            m.Sxx += q.b;
            m.Sxy += dy * c1;
            m.Syy += dy * dy * c0;
            m.R0 += q.s0;
            m.Rx += q.s1;
            m.Ry += (double)dy * q.s0;
        }
#pragma unroll
        for (int h = 0; h < kRows; ++h) {
            const int ty = ty0 + h;
            if (h > 0) {
                // drop the window's top row, add the next one below, re-centre
                const RowMom qo = rowm(ty - 1), qn = rowm(ty + 2 * r);
                const int c0o = qo.a & 0xffff, c1o = (qo.a >> 16) - kColOff;
                const int c0n = qn.a & 0xffff, c1n = (qn.a >> 16) - kColOff;
                ColMom u;
                u.N = m.N - c0o + c0n;
                u.Sx = m.Sx - c1o + c1n;
                u.Sxx = m.Sxx - qo.b + qn.b;
                const int t0 = m.Sy + r * c0o + (r + 1) * c0n;
                u.Sy = t0 - u.N;
                u.Syy = (m.Syy - r * r * c0o + (r + 1) * (r + 1) * c0n) - 2 * t0 + u.N;
                u.Sxy = (m.Sxy + r * c1o + (r + 1) * c1n) - u.Sx;
                u.R0 = (m.R0 - qo.s0) + qn.s0;
                u.Rx = (m.Rx - qo.s1) + qn.s1;
                u.Ry = ((m.Ry + (double)r * qo.s0) + (double)(r + 1) * qn.s0) - u.R0;
                m = u;
            }
            if (!gx_in || y0 + ty >= a.H) continue;
            const int pc = (ty + r) * LW + tx + r;
            const float Dc = sD[pc];
            float nx = __builtin_nanf(""), ny = nx, nz = nx, a1 = nx, a2 = nx;
            if (Dc > 0.0f && sL[pc] >= 0) {
                double gu, gv;
                if (slope_solve(m, Dc, a.need_g, gu, gv)) {
                    a1 = (float)(1.0 - gu);
                    a2 = (float)(-gv);
                    normal_from_slope(gu, gv, Dc, x0 + tx, y0 + ty, a.fx, a.fy, a.u0, a.v0, nx,
                                      ny, nz);
                }
            }
            output(ty, a1, a2, nx, ny, nz);
        }
    }
    // The rows of the mixed bands are shared out row by row from an LDS
    // counter, so a wave that has finished its own band takes on the rows of
    // the others' instead of idling beside them.
    int mixed_rows = 0;
#pragma unroll
    for (int w = 0; w < kRsBlock / 64; ++w) mixed_rows += s_mixed[w] ? kRows : 0;
    while (true) {
        int i = 0;
        if (tx == 0) i = atomicAdd(&s_next, 1);
        i = __shfl(i, 0);
        if (i >= mixed_rows) break;
        // row i % kRows of the (i / kRows)-th mixed band
        int band = -1;
        for (int k = i / kRows; k >= 0; --k)
            do ++band; while (!s_mixed[band]);
        const int ty = kRows * band + i % kRows;
        const int gx = x0 + tx, gy = y0 + ty;
        if (gx >= a.W || gy >= a.H) continue;
        const int pc = (ty + r) * LW + tx + r;
        const float Dc = sD[pc];
        const int32_t lc = sL[pc];
        float nx = __builtin_nanf(""), ny = nx, nz = nx, a1 = nx, a2 = nx;
        if (Dc > 0.0f && lc >= 0) {
            int N = 0, Sx = 0, Sy = 0, Sxx = 0, Sxy = 0, Syy = 0;
            double Rx = 0.0, Ry = 0.0;
            for (int dy = -r; dy <= r; ++dy) {
                const float *pD = sD + (ty + r + dy) * LW + tx;
                const int32_t *pL = sL + (ty + r + dy) * LW + tx;
                int nr = 0, sxr = 0, sxxr = 0;
                double s0 = 0.0, s1 = 0.0;
                auto tap = [&](int k) {
                    const int dx = k - r;
                    const float v = pD[k];
                    const bool m = pL[k] == lc && v > 0.0f;
                    const double vm = m ? (double)v : 0.0;
                    nr += m ? 1 : 0;
                    sxr += m ? dx : 0;
                    sxxr += m ? dx * dx : 0;
                    s0 += vm;
                    s1 += (double)dx * vm;
                };
                if (RC > 0) {
#pragma unroll
                    for (int k = 0; k <= 2 * (RC > 0 ? RC : 0); ++k) tap(k);
                } else {
                    for (int k = 0; k <= 2 * r; ++k) tap(k);
                }
                N += nr;
                Sx += sxr;
                Sy += dy * nr;
                Sxx += sxxr;
                Sxy += dy * sxr;
                Syy += dy * dy * nr;
                Rx += s1;
                Ry += (double)dy * s0;
            }
            ColMom mo;
            mo.N = N; mo.Sx = Sx; mo.Sy = Sy; mo.Sxx = Sxx; mo.Sxy = Sxy; mo.Syy = Syy;
            mo.R0 = 0.0; mo.Rx = Rx; mo.Ry = Ry;
            double gu, gv;
            if (slope_solve(mo, Dc, a.need_g, gu, gv)) {
                a1 = (float)(1.0 - gu);
                a2 = (float)(-gv);
                normal_from_slope(gu, gv, Dc, gx, gy, a.fx, a.fy, a.u0, a.v0, nx, ny, nz);
            }
        }
        output(ty, a1, a2, nx, ny, nz);
    }
}

using RsFn = void (*)(RestrictArgs);
struct RsInst { int r; RsFn fn; };
constexpr RsInst kRsInst[] = {
    {1, &k_affine_labels<1>}, {2, &k_affine_labels<2>}, {3, &k_affine_labels<3>},
    {4, &k_affine_labels<4>}, {7, &k_affine_labels<7>}, {10, &k_affine_labels<10>},
    {15, &k_affine_labels<15>},
};

}  // namespace

size_t restrict_lds_bytes(int r)
{
    return (sizeof(float) + sizeof(int32_t)) * (size_t)(kRsW + 2 * r) * (kRsH + 2 * r);
}

hipError_t launch_affine_labels(const RestrictArgs &a, hipStream_t s)
{
    const dim3 grid((a.W + kRsW - 1) / kRsW, (a.H + kRsH - 1) / kRsH);
    RsFn fn = &k_affine_labels<-1>;
    for (const RsInst &i : kRsInst)
        if (i.r == a.r) fn = i.fn;
    hipLaunchKernelGGL(fn, grid, dim3(kRsBlock), restrict_lds_bytes(a.r), s, a);
    return hipGetLastError();
}

}  // namespace snx
