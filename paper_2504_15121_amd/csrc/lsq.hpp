// Separable masked window moments and the two LSQ solves, shared by every kernel
// that filters or differentiates so that all of them produce bit-identical
// results for the same input.
//
// For a validity-coded image v (v_i = D_i if valid else 0; m_i = [v_i > 0]) and a
// window of offsets (dx, dy) around a centre, the LSQ steps need
//     mask moments   N = sum m, Sx = sum m dx, Sy = sum m dy,
//                    Sxx = sum m dx^2, Sxy = sum m dx dy, Syy = sum m dy^2
//     data moments   R0 = sum v, Rx = sum dx v, Ry = sum dy v
// A row pass sums over dx for every row; a column pass sums the row results
// over dy.  Row mask moments are accumulated as one packed int32 per tap and
// re-packed for the column pass; data moments are FP64 (uncentred sums in FP64
// lose nothing that matters before D_c is subtracted algebraically).
#pragma once

#include "snx_internal.hpp"

namespace snx {

// Row-pass packing: c0 in bits 0..5, (c1 + 512) in bits 6..15, c2 in bits
// 16..30 -- exact for windows up to 63.
constexpr int kRowOff = 512;
__device__ __forceinline__ int row_tap(int dx) { return 1 + dx * 64 + dx * dx * 65536; }

// Column-pass packing of one row result: A = c0 + (c1 + kColOff) * 2^16, B = c2.
// Summing A, dy*A and dy^2*A over the window then yields
//   sum A       = N  + (Sx + kColOff * rows) * 2^16
//   sum dy A    = Sy + Sxy * 2^16               (sum of dy over the window is 0)
//   sum dy^2 A  = Syy (low 16 bits)
// which is exact while N, Sx + kColOff*rows, Syy < 2^16 and |Sy|, |Sxy| < 2^15:
// true for windows up to 21 (kPackedMaxR = 10).
constexpr int kColOff = 512;
constexpr int kPackedMaxR = 10;

struct RowMom {
    int a;        // packed c0 / c1 (column format) or raw row packing
    int b;        // c2
    double s0;    // sum v
    double s1;    // sum dx v
};

// Row moments of the window p[0 .. 2r] (centre p[r]).
template <int RC>
__device__ __forceinline__ RowMom row_moments(const float *p, int r_rt)
{
    const int r = RC >= 0 ? RC : r_rt;
    int c = kRowOff * 64;
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int k = 0; k <= 2 * r; ++k) {
        const float v = p[k];
        const int dx = k - r;
        c += v > 0.0f ? row_tap(dx) : 0;
        const double dv = (double)v;
        s0 += dv;
        s1 += (double)dx * dv;
    }
    const int c0 = c & 63;
    const int c1 = ((c >> 6) & 1023) - kRowOff;
    const int c2 = c >> 16;
    RowMom m;
    m.a = c0 + (c1 + kColOff) * 65536;
    m.b = c2;
    m.s0 = s0;
    m.s1 = s1;
    return m;
}

// Row moments of KRUN consecutive centres p[r], p[r+1], ... (windows
// p[i .. i+2r]) written to ab[i STEP], s[i STEP] in the column-pass format: the first by
// direct sums, the others by sliding the window one pixel (remove the left
// tap, add the right one, re-centre).  Every sum is of integers or of float32
// values in FP64, exact for windows up to 63 and disparities spanning fewer
// than 2^29 between smallest and largest, so the results equal the direct sums.
template <int RC, int KRUN, int STEP = 1>
__device__ __forceinline__ void row_moments_run(const float *p, int r_rt, int2 *ab, double2 *s)
{
    const int r = RC >= 0 ? RC : r_rt;
    int n = 0, sx = 0, sxx = 0;
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int k = 0; k <= 2 * r; ++k) {
        const float v = p[k];
        const int dx = k - r;
        const int m = v > 0.0f ? 1 : 0;
        n += m;
        sx += m * dx;
        sxx += m * dx * dx;
        const double dv = (double)v;
        s0 += dv;
        s1 += (double)dx * dv;
    }
    ab[0] = make_int2(n + (sx + kColOff) * 65536, sxx);
    s[0] = make_double2(s0, s1);
#pragma unroll
    for (int i = 1; i < KRUN; ++i) {
        const float vo = p[i - 1], vn = p[i + 2 * r];
        const int mo = vo > 0.0f ? 1 : 0, mn = vn > 0.0f ? 1 : 0;
        const int t = sx + r * mo + (r + 1) * mn;              // sum of j m_j, j = -r+1 .. r+1
        const int u = sxx - r * r * mo + (r + 1) * (r + 1) * mn;
        n += mn - mo;
        sx = t - n;
        sxx = u - 2 * t + n;
        const double dvo = (double)vo, dvn = (double)vn;
        s0 = (s0 - dvo) + dvn;
        s1 = ((s1 + (double)r * dvo) + (double)(r + 1) * dvn) - s0;
        ab[i * STEP] = make_int2(n + (sx + kColOff) * 65536, sxx);
        s[i * STEP] = make_double2(s0, s1);
    }
}

struct ColMom {
    int N, Sx, Sy, Sxx, Sxy, Syy;
    double R0, Rx, Ry;
};

// Moves the column window of `m` (rows top .. top+2r of the row-moment arrays,
// stride apart) down by one row: removes row `top`, adds row top + 2r + 1 and
// re-centres.  Exact like row_moments_run.
__device__ __forceinline__ ColMom col_slide(const ColMom &m, const int2 *ab_top, const double2 *s_top,
                                            int stride, int r)
{
    const int2 wo = ab_top[0], wn = ab_top[(2 * r + 1) * stride];
    const double2 dO = s_top[0], dN = s_top[(2 * r + 1) * stride];
    const int c0o = wo.x & 0xffff, c1o = (wo.x >> 16) - kColOff, c2o = wo.y;
    const int c0n = wn.x & 0xffff, c1n = (wn.x >> 16) - kColOff, c2n = wn.y;
    ColMom o;
    o.N = m.N - c0o + c0n;
    o.Sx = m.Sx - c1o + c1n;
    o.Sxx = m.Sxx - c2o + c2n;
    const int t0 = m.Sy + r * c0o + (r + 1) * c0n;           // sum of j c0_j over the new rows
    o.Sy = t0 - o.N;
    o.Syy = (m.Syy - r * r * c0o + (r + 1) * (r + 1) * c0n) - 2 * t0 + o.N;
    o.Sxy = (m.Sxy + r * c1o + (r + 1) * c1n) - o.Sx;
    o.R0 = (m.R0 - dO.x) + dN.x;
    o.Rx = (m.Rx - dO.y) + dN.y;
    o.Ry = ((m.Ry + (double)r * dO.x) + (double)(r + 1) * dN.x) - o.R0;
    return o;
}

// Column pass over rows base[0], base[stride], ..., base[2r * stride] of the
// row-moment arrays (a/b as int2, s0/s1 as double2).
template <int RC, bool WANT_R0>
__device__ __forceinline__ ColMom col_moments(const int2 *ab, const double2 *s, int stride,
                                              int r_rt)
{
    const int r = RC >= 0 ? RC : r_rt;
    ColMom o;
    double R0 = 0.0, Rx = 0.0, Ry = 0.0;
    if (RC >= 0 && RC <= kPackedMaxR) {
        // unsigned: the packed sums wrap modulo 2^32 by design
        unsigned SA = 0, YA = 0, YYA = 0, SB = 0;
#pragma unroll
        for (int k = 0; k <= 2 * r; ++k) {
            const int dy = k - r;
            const int2 w = ab[k * stride];
            const double2 d = s[k * stride];
            const unsigned wa = (unsigned)w.x;
            SA += wa;
            YA += (unsigned)dy * wa;
            YYA += (unsigned)(dy * dy) * wa;
            SB += (unsigned)w.y;
            if (WANT_R0) R0 += d.x;
            Rx += d.y;
            Ry += (double)dy * d.x;
        }
        const int rows = 2 * r + 1;
        o.N = (int)(SA & 0xffffu);
        o.Sx = (int)(SA >> 16) - kColOff * rows;
        o.Sy = (int)(short)(YA & 0xffffu);
        o.Sxy = ((int)YA - o.Sy) >> 16;
        o.Syy = (int)(YYA & 0xffffu);
        o.Sxx = (int)SB;
    } else {
        int N = 0, Sx = 0, Sy = 0, Sxx = 0, Sxy = 0, Syy = 0;
        for (int k = 0; k <= 2 * r; ++k) {
            const int dy = k - r;
            const int2 w = ab[k * stride];
            const double2 d = s[k * stride];
            const int c0 = w.x & 0xffff;
            const int c1 = (w.x >> 16) - kColOff;
            N += c0; Sx += c1; Sy += dy * c0;
            Sxx += w.y; Sxy += dy * c1; Syy += dy * dy * c0;
            if (WANT_R0) R0 += d.x;
            Rx += d.y;
            Ry += (double)dy * d.x;
        }
        o.N = N; o.Sx = Sx; o.Sy = Sy; o.Sxx = Sxx; o.Sxy = Sxy; o.Syy = Syy;
    }
    o.R0 = R0;
    o.Rx = Rx;
    o.Ry = Ry;
    return o;
}

// 1/d for d >= 1 (an exact integer here): hardware reciprocal refined by two
// Newton steps, accurate to a few ulp of FP64.
__device__ __forceinline__ double recip(double d)
{
    double r = __builtin_amdgcn_rcp(d);
    r = __builtin_fma(__builtin_fma(-d, r, 1.0), r, r);
    r = __builtin_fma(__builtin_fma(-d, r, 1.0), r, r);
    return r;
}

// Filter (LSQ plane intercept at the centre): pass-through when fewer than
// need_f pixels are valid or the 3x3 normal matrix is singular.  Every
// determinant term is an exact integer below 2^53 for windows up to 63.
__device__ __forceinline__ float filter_solve(const ColMom &m, float Dc, int need_f)
{
    double h = (double)Dc;
    if (m.N >= need_f) {
        const double n = m.N, sx = m.Sx, sy = m.Sy, sxx = m.Sxx, sxy = m.Sxy, syy = m.Syy;
        const double m11 = sxx * syy - sxy * sxy;
        const double m12 = sx * syy - sxy * sy;
        const double m13 = sx * sxy - sxx * sy;
        const double det = n * m11 - sx * m12 + sy * m13;
        if (det != 0.0) {
            const double dc = (double)Dc;
            const double r0 = m.R0 - n * dc;
            const double r1 = m.Rx - sx * dc;
            const double r2 = m.Ry - sy * dc;
            const double num = r0 * m11 - sx * (r1 * syy - sxy * r2) + sy * (r1 * sxy - sxx * r2);
            h = dc + num * recip(det);
        }
    }
    return (float)h;
}

// Anchored slope (g_u, g_v) of Sec. 3.2-3.3 with the masked support of the
// window excluding the centre; returns false where it is undefined.
__device__ __forceinline__ bool slope_solve(const ColMom &m, float Dc, int need_g, double &gu,
                                            double &gv)
{
    const double al = m.Sxx, be = m.Sxy, ga = m.Syy;
    const double det = al * ga - be * be;   // exact
    if (m.N - 1 < need_g || !(det > 0.0)) return false;
    const double dc = (double)Dc;
    const double S1 = m.Rx - (double)m.Sx * dc;
    const double S2 = m.Ry - (double)m.Sy * dc;
    const double inv = recip(det);
    gu = (ga * S1 - be * S2) * inv;
    gv = (al * S2 - be * S1) * inv;
    return true;
}

// 3x3 filter by mask.  For the valid taps of a 3x3 window (9-bit mask, bit
// 3 (dy + 1) + dx + 1), the intercept of the LSQ plane is a fixed linear
// combination of the data moments: with the integer normal matrix
// M = sum (1, dx, dy)^T (1, dx, dy) and r = (R0, Rx, Ry),
//   h = (M^-1 r)_0 = (m11 R0 - m12 Rx + m13 Ry) / det M
// (m11 = Sxx Syy - Sxy^2, m12 = Sx Syy - Sxy Sy, m13 = Sx Sxy - Sxx Sy; the
// centred form D_c + (M^-1 (r - D_c M e_0))_0 is the same number).  The three
// weights of every mask are tabulated once; a singular M is marked by a NaN
// weight (pass-through).
struct Filter3Table {
    double w[512][4];
    constexpr Filter3Table() : w()
    {
        for (int m = 0; m < 512; ++m) {
            long long n = 0, sx = 0, sy = 0, sxx = 0, sxy = 0, syy = 0;
            for (int k = 0; k < 9; ++k) {
                if (!((m >> k) & 1)) continue;
                const long long dx = k % 3 - 1, dy = k / 3 - 1;
                n += 1;
                sx += dx;
                sy += dy;
                sxx += dx * dx;
                sxy += dx * dy;
                syy += dy * dy;
            }
            const long long m11 = sxx * syy - sxy * sxy;
            const long long m12 = sx * syy - sxy * sy;
            const long long m13 = sx * sxy - sxx * sy;
            const long long det = n * m11 - sx * m12 + sy * m13;
            if (det == 0) {
                w[m][0] = __builtin_nan("");
                w[m][1] = w[m][2] = w[m][3] = 0.0;
            } else {
                w[m][0] = (double)m11 / (double)det;
                w[m][1] = -(double)m12 / (double)det;
                w[m][2] = (double)m13 / (double)det;
                w[m][3] = 0.0;
            }
        }
    }
};
static __constant__ const Filter3Table kFilter3 = Filter3Table();

// Direct 3x3 filter around the validity-coded value p[0] (row stride ld), for
// a valid centre: pass-through when fewer than need_f taps are valid or the
// normal matrix is singular.  Every kernel that filters with n_f = 3 calls this.
__device__ __forceinline__ float filter3x3(const float *p, int ld, int need_f)
{
    int msk = 0;
    double R0 = 0.0, Rx = 0.0, Ry = 0.0;
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy) {
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
            const float v = p[dy * ld + dx];
            msk |= (v > 0.0f ? 1 : 0) << (3 * (dy + 1) + dx + 1);
            const double dv = (double)v;
            R0 += dv;
            if (dx != 0) Rx += (double)dx * dv;
            if (dy != 0) Ry += (double)dy * dv;
        }
    }
    const double *w = kFilter3.w[msk];
    const double w0 = w[0];
    if (__popc(msk) < need_f || w0 != w0) return p[0];
    return (float)(w0 * R0 + w[1] * Rx + w[2] * Ry);
}

// Unit normal n = -m/|m| with m = (f_x g_u, f_y g_v, D - (u-u0) g_u - (v-v0) g_v).
__device__ __forceinline__ void normal_from_slope(double gu, double gv, float Dc, int u, int v,
                                                  float fx, float fy, float u0, float v0,
                                                  float &nx, float &ny, float &nz)
{
    const double mxd = (double)fx * gu;
    const double myd = (double)fy * gv;
    const double mzd = (double)Dc - ((double)u - (double)u0) * gu - ((double)v - (double)v0) * gv;
    const float mx = (float)mxd, my = (float)myd, mz = (float)mzd;
    const float s = -__frsqrt_rn(mx * mx + my * my + mz * mz);
    nx = mx * s;
    ny = my * s;
    nz = mz * s;
}

}  // namespace snx
