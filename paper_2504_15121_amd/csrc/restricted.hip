// Component-restricted gradient window: the anchored LSQ slope, A and normal
// over the pixels of the n_g x n_g window that are valid and carry the centre's
// surface-component label (the concern of Sec. 3.4 that points of a
// neighbouring surface smooth the normals, met with the components of the
// covered-depth predicate).  One 64 x 16 output tile per 256-thread workgroup.
//
// The mask depends on the centre's label, so the window sums are not
// separable: each centre walks its window in LDS (validity-coded D~ and the
// labels, halo r), one row at a time; a row's integer moments and its two data
// sums (exact FP64 sums of float32 values times small integers) are combined
// into the column moments with the row offset.  The solve, A and normal are the
// square-window ones.
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

    const int tx = tid & 63;
    for (int ty = tid >> 6; ty < kRsH; ty += kRsBlock / 64) {
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
