// Adaptive star-fill support (Sec. 3.4, Adaptive Region Estimation) -> slope,
// A and normal, for one 64 x 16 output tile per 256-thread workgroup.
//
// From a valid centre c, rays leave in M = 4 (axes), 8 (axes and diagonals) or
// 16 directions -- the directions 2 pi m / M scaled to a unit larger component
// -- and take c + round(k e_m), k = 1 .. steps, stopping before the first pixel
// that is invalid or outside the image or meets the stopping rule:
//   CD  D_c (b - a) > k_cd (a b), with a, b the smallest and largest disparity
//       of c and the ray's pixels so far including the new one (the depth
//       range f B (1/a - 1/b) exceeds k_cd times the depth of c), binary64;
//   ST  the 4-neighbour depth Laplacian ((z_r + z_l) + (z_d + z_u)) - 4 z with
//       z = f_x B / D (binary64) at the new pixel is undefined or exceeds t in
//       magnitude.
// The slope is the anchored LSQ over the pixels the rays take (the two-pass
// scheme of Sec. 3.4 with the star as the support), then A and the normal as
// for the square windows.
//
// The rays of the compass directions never share a pixel, so a ray's moments
// follow from its length n alone (sum k = n(n+1)/2, sum k^2 = n(n+1)(2n+1)/6
// times the direction's components) plus one exact FP64 sum of k D per ray;
// the rays of a pixel advance in lock step.  With M = 16 the eight rays in
// between (angles (2j+1) pi / 8) take c + k A_j + r_k B_j, A_j and B_j unit
// compass vectors along and across the ray and r_k = round(k tan(pi/8)); their
// first pixel (r_1 = 0) is the first pixel of the axis ray beside them, taken
// or refused by that ray under the same test, so the support (the union of the
// rays' pixels) counts it once: these rays add their pixels from k = 2 on, with
// integer moment sums and two exact FP64 sums (of k D and of r_k D) each.
// The tile (validity-coded, halo = steps, + 1 for ST) and, for ST, a byte
// plane of edge flags sit in LDS.
#include "lsq.hpp"

namespace snx {
namespace {

constexpr int kStW = 64, kStH = 16, kStBlock = 256;

// compass directions in the order of the angle 2 pi m / 8 (v downwards)
__device__ __forceinline__ constexpr int dir_x(int m) { return m == 0 || m == 1 || m == 7 ? 1 : (m == 2 || m == 6 ? 0 : -1); }
__device__ __forceinline__ constexpr int dir_y(int m) { return m == 1 || m == 2 || m == 3 ? 1 : (m == 0 || m == 4 ? 0 : -1); }

// the rays between the compass directions (M = 16), j = 0 .. 7 at the angle
// (2j + 1) pi / 8: the compass vector along the ray (A) and across it (B)
__device__ __forceinline__ constexpr int odd_ax(int j) { return j == 0 || j == 7 ? 1 : (j == 3 || j == 4 ? -1 : 0); }
__device__ __forceinline__ constexpr int odd_ay(int j) { return j == 1 || j == 2 ? 1 : (j == 5 || j == 6 ? -1 : 0); }
__device__ __forceinline__ constexpr int odd_bx(int j) { return j == 1 || j == 6 ? 1 : (j == 2 || j == 5 ? -1 : 0); }
__device__ __forceinline__ constexpr int odd_by(int j) { return j == 0 || j == 3 ? 1 : (j == 4 || j == 7 ? -1 : 0); }

// round(k tan(pi / 8)) for k = 1 .. 32: k tan(pi/8) is never within 0.015 of a
// half-integer there, so the binary64 product rounds the same as the exact one
__device__ __forceinline__ int cross_step(int k)
{
    return (int)((double)k * 0.41421356237309503 + 0.5);
}

template <int M, int STOP>
__global__ void __launch_bounds__(kStBlock)
k_star(StarArgs a)
{
#pragma clang fp contract(off)
    constexpr int MC = M < 8 ? M : 8;            // compass rays
    constexpr int MO = M == 16 ? 8 : 0;          // rays in between
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const int s = a.steps;
    const int R = s + (STOP == kStopST ? 1 : 0);     // halo of the value tile
    const int LW = kStW + 2 * R, LH = kStH + 2 * R;
    float *sD = reinterpret_cast<float *>(smem);
    const int EW = kStW + 2 * s, EH = kStH + 2 * s;   // edge flags: halo s
    unsigned char *sE = smem + sizeof(float) * (size_t)LW * LH;
    const int tid = threadIdx.x;
    const int x0 = blockIdx.x * kStW, y0 = blockIdx.y * kStH;

    for (int e = tid; e < LW * LH; e += kStBlock) {
        const int ly = e / LW, lx = e - ly * LW;
        const int gy = y0 - R + ly, gx = x0 - R + lx;
        float v = 0.0f;
        if (gy >= 0 && gy < a.H && gx >= 0 && gx < a.W) {
            const float d = a.src[(int64_t)gy * a.ld_src + gx];
            v = valid_disp(d) ? d : 0.0f;
        }
        sD[e] = v;
    }
    __syncthreads();
    if (STOP == kStopST) {
        for (int e = tid; e < EW * EH; e += kStBlock) {
            const int ey = e / EW, ex = e - ey * EW;
            const float *p = sD + (ey + 1) * LW + ex + 1;       // same pixel in the value tile
            const float c = p[0], r = p[1], l = p[-1], d = p[LW], u = p[-LW];
            unsigned char edge = 1;
            if (c > 0.0f && r > 0.0f && l > 0.0f && d > 0.0f && u > 0.0f) {
                const double zc = a.fxb / (double)c, zr = a.fxb / (double)r;
                const double zl = a.fxb / (double)l, zd = a.fxb / (double)d;
                const double zu = a.fxb / (double)u;
                const double L = ((zr + zl) + (zd + zu)) - 4.0 * zc;
                edge = fabs(L) > a.thr ? 1 : 0;
            }
            sE[e] = edge;
        }
        __syncthreads();
    }

    const int tx = tid & 63;
    for (int ty = tid >> 6; ty < kStH; ty += kStBlock / 64) {
        const int gx = x0 + tx, gy = y0 + ty;
        if (gx >= a.W || gy >= a.H) continue;
        const int pc = (ty + R) * LW + tx + R;
        const int ec = (ty + s) * EW + tx + s;
        const float Dc = sD[pc];
        float nx = __builtin_nanf(""), ny = nx, nz = nx, a1 = nx, a2 = nx;
        if (Dc > 0.0f) {
            // The rays advance together, one step per pass: their LDS reads are
            // in flight at once, and a stopped ray is carried as a predicate
            // (a stopped ray reads pixels still inside the tile and adds 0).
            const double dc64 = (double)Dc;
            // range of the ray so far, as binary64 (exact images of the float
            // values); once a ray has stopped its range is never read again,
            // so it is updated without a select
            double lo[MC], hi[MC];
            double wk[MC];
            int nk[MC], pp[MC], pe[MC];
            bool alive[MC];
#pragma unroll
            for (int mi = 0; mi < MC; ++mi) {
                lo[mi] = hi[mi] = dc64;
                wk[mi] = 0.0;
                nk[mi] = 0;
                pp[mi] = pc;
                pe[mi] = ec;
                alive[mi] = true;
            }
            // rays in between: range, position, and sums over k >= 2 of 1, k,
            // k^2, r, r^2, k r (integers) and of k D, r D (binary64, exact)
            double olo[MO > 0 ? MO : 1], ohi[MO > 0 ? MO : 1];
            double owk[MO > 0 ? MO : 1], owr[MO > 0 ? MO : 1];
            int on[MO > 0 ? MO : 1], osk[MO > 0 ? MO : 1], oskk[MO > 0 ? MO : 1];
            int osr[MO > 0 ? MO : 1], osrr[MO > 0 ? MO : 1], oskr[MO > 0 ? MO : 1];
            int opp[MO > 0 ? MO : 1], ope[MO > 0 ? MO : 1];
            bool oalive[MO > 0 ? MO : 1];
#pragma unroll
            for (int j = 0; j < MO; ++j) {
                olo[j] = ohi[j] = dc64;
                owk[j] = owr[j] = 0.0;
                on[j] = osk[j] = oskk[j] = osr[j] = osrr[j] = oskr[j] = 0;
                opp[j] = pc;
                ope[j] = ec;
                oalive[j] = true;
            }
            int r_prev = 0;
            for (int k = 1; k <= s; ++k) {
                const double kd = (double)k;
                float vv[MC];
#pragma unroll
                for (int mi = 0; mi < MC; ++mi) {
                    const int m = mi * (8 / MC);
                    pp[mi] += dir_y(m) * LW + dir_x(m);
                    vv[mi] = sD[pp[mi]];
                }
                const int r = MO ? cross_step(k) : 0;
                const int dr = r - r_prev;
                r_prev = r;
                float ov[MO > 0 ? MO : 1];
#pragma unroll
                for (int j = 0; j < MO; ++j) {
                    opp[j] += odd_ay(j) * LW + odd_ax(j) + dr * (odd_by(j) * LW + odd_bx(j));
                    ov[j] = sD[opp[j]];
                }
                bool any = false;
#pragma unroll
                for (int j = 0; j < MO; ++j) {
                    const double v = (double)ov[j];
                    bool ok = oalive[j] && v > 0.0;
                    if (STOP == kStopCD) {
                        const double da = fmin(v, olo[j]), db = fmax(v, ohi[j]);
                        ok = ok && !(dc64 * (db - da) > a.thr * (da * db));
                        olo[j] = da;
                        ohi[j] = db;
                    } else {
                        ope[j] += odd_ay(j) * EW + odd_ax(j) + dr * (odd_by(j) * EW + odd_bx(j));
                        ok = ok && !sE[ope[j]];
                    }
                    // the first pixel is the neighbouring axis ray's
                    const bool add = ok && k >= 2;
                    owk[j] = __builtin_fma(kd, add ? v : 0.0, owk[j]);
                    owr[j] = __builtin_fma((double)r, add ? v : 0.0, owr[j]);
                    on[j] += add ? 1 : 0;
                    osk[j] += add ? k : 0;
                    oskk[j] += add ? k * k : 0;
                    osr[j] += add ? r : 0;
                    osrr[j] += add ? r * r : 0;
                    oskr[j] += add ? k * r : 0;
                    oalive[j] = ok;
                    any = any || ok;
                }
#pragma unroll
                for (int mi = 0; mi < MC; ++mi) {
                    const int m = mi * (8 / MC);
                    const double v = (double)vv[mi];
                    bool ok = alive[mi] && v > 0.0;
                    if (STOP == kStopCD) {
                        const double da = fmin(v, lo[mi]), db = fmax(v, hi[mi]);
                        ok = ok && !(dc64 * (db - da) > a.thr * (da * db));
                        lo[mi] = da;
                        hi[mi] = db;
                    } else {
                        pe[mi] += dir_y(m) * EW + dir_x(m);
                        ok = ok && !sE[pe[mi]];
                    }
                    // k v is exact in binary64, so the fused form rounds as the
                    // separate product and sum do
                    wk[mi] = __builtin_fma(kd, ok ? v : 0.0, wk[mi]);
                    nk[mi] = ok ? k : nk[mi];
                    alive[mi] = ok;
                    any = any || ok;
                }
                if (!__any(any)) break;
            }
            int N = 1, Sx = 0, Sy = 0, Sxx = 0, Sxy = 0, Syy = 0;
            double Rx = 0.0, Ry = 0.0;
#pragma unroll
            for (int j = 0; j < MO; ++j) {
                const int ax = odd_ax(j), ay = odd_ay(j), bx = odd_bx(j), by = odd_by(j);
                N += on[j];
                Sx += ax * osk[j] + bx * osr[j];
                Sy += ay * osk[j] + by * osr[j];
                Sxx += ax * ax * oskk[j] + bx * bx * osrr[j];
                Syy += ay * ay * oskk[j] + by * by * osrr[j];
                Sxy += (ax * by + ay * bx) * oskr[j];
                Rx += (double)ax * owk[j] + (double)bx * owr[j];
                Ry += (double)ay * owk[j] + (double)by * owr[j];
            }
#pragma unroll
            for (int mi = 0; mi < MC; ++mi) {
                const int m = mi * (8 / MC);
                const int ex = dir_x(m), ey = dir_y(m), n = nk[mi];
                const int t1 = n * (n + 1) / 2, t2 = n * (n + 1) * (2 * n + 1) / 6;
                N += n;
                Sx += ex * t1;
                Sy += ey * t1;
                Sxx += ex * ex * t2;
                Sxy += ex * ey * t2;
                Syy += ey * ey * t2;
                Rx += (double)ex * wk[mi];
                Ry += (double)ey * wk[mi];
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

}  // namespace

size_t star_lds_bytes(int steps, int stop)
{
    const int R = steps + (stop == kStopST ? 1 : 0);
    size_t b = sizeof(float) * (size_t)(kStW + 2 * R) * (kStH + 2 * R);
    if (stop == kStopST) b += (size_t)(kStW + 2 * steps) * (kStH + 2 * steps);
    return b;
}

hipError_t launch_star(const StarArgs &a, hipStream_t s)
{
    const dim3 grid((a.W + kStW - 1) / kStW, (a.H + kStH - 1) / kStH);
    const size_t lds = star_lds_bytes(a.steps, a.stop);
    if (a.dirs == 16 && a.stop == kStopCD)
        hipLaunchKernelGGL((k_star<16, kStopCD>), grid, dim3(kStBlock), lds, s, a);
    else if (a.dirs == 16 && a.stop == kStopST)
        hipLaunchKernelGGL((k_star<16, kStopST>), grid, dim3(kStBlock), lds, s, a);
    else if (a.dirs == 8 && a.stop == kStopCD)
        hipLaunchKernelGGL((k_star<8, kStopCD>), grid, dim3(kStBlock), lds, s, a);
    else if (a.dirs == 8 && a.stop == kStopST)
        hipLaunchKernelGGL((k_star<8, kStopST>), grid, dim3(kStBlock), lds, s, a);
    else if (a.dirs == 4 && a.stop == kStopCD)
        hipLaunchKernelGGL((k_star<4, kStopCD>), grid, dim3(kStBlock), lds, s, a);
    else if (a.dirs == 4 && a.stop == kStopST)
        hipLaunchKernelGGL((k_star<4, kStopST>), grid, dim3(kStBlock), lds, s, a);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace snx
