/*
 * FP64 CPU oracle for the disparity -> oriented point cloud path of
 * "Robust and Real-time Surface Normal Estimation from Stereo Disparities using
 * Affine Transformations" (Kariko, Faisal, Hajder).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or helper with the GPU path and is deliberately plain and slow:
 * every window sum is taken pixel by pixel in the order the definitions state,
 * with OpenMP only splitting independent output rows.
 *
 * Conventions (readings of the paper, see the design notes):
 *   - u = column, v = row (downwards), pixel centres at integers; images are
 *     row-major W*H arrays.
 *   - D is the positive disparity u_L - u_R = f_x b / z.  The paper's d is
 *     u_R - u_L = -D (Sec. 3.2 notes d may be negative).
 *   - A pixel is valid iff its value is finite and > 0; pixels outside the image
 *     are invalid (no padding, clamping or mirroring).
 *
 * Functions (each cites the passage it implements):
 *   snxo_denoise        masked least-squares plane fit, intercept at the centre
 *                       (Sec. 3.2 over-determined LSQ with a constant column)
 *   snxo_affine         a1, a2 from the anchored LSQ of Sec. 3.2 / Sec. 3.3
 *                       (eqs. convprep, convprep2), masked support as in the
 *                       two-pass scheme of Sec. 3.4
 *   snxo_normals        n from the two constraint vectors of Sec. 3.1
 *                       (cross product of a1 v1 - v2 and a2 v3 - v4)
 *   snxo_components     4-connected components under the pairwise covered-depth
 *                       predicate (Sec. 3.4, CD), labels = minimum linear index,
 *                       breadth-first flood fill in raster order
 *   snxo_point_cloud    X from the rectified projections of Sec. 2 plus n
 *   snxo_components_crease  components whose 4-neighbour edges must also pass a
 *                       normal-crease test (depth-continuous creases, which the
 *                       covered-depth rule misses by Sec. 3.4's own account)
 *   snxo_affine_labels  a1, a2 with the n_g window restricted to the centre's
 *                       surface component (Sec. 3.4's concern about neighbouring
 *                       surfaces, with the components of snxo_components)
 *   snxo_star_mask,     the adaptive star-fill support of Sec. 3.4 (Adaptive
 *   snxo_star_affine    Region Estimation: rays in M directions with the ST or
 *                       CD stopping rule) and a1, a2 over it by the two-pass
 *                       anchored LSQ
 */
#include <math.h>
#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static int is_valid(double d) { return isfinite(d) && d > 0.0; }

/* ------------------------------------------------------------------------ */
/* Filter: masked LSQ plane fit D_i - D_c ~ (h - D_c) + g_u v_ix + g_v v_iy   */
/* over the valid pixels of the n_f x n_f window (centre included).          */
/* Output h.  Pass-through (h = D_c) when fewer than max(3, min_support)     */
/* pixels are valid or the 3x3 normal matrix is singular (exact integers).   */
/* ------------------------------------------------------------------------ */
static int64_t det3_int(const int64_t M[3][3])
{
    return M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1])
         - M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0])
         + M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0]);
}

int snxo_denoise(const double *D, int W, int H, int nf, int min_support,
                 double *out)
{
    if (nf < 1 || (nf % 2) == 0 || W < 1 || H < 1) return 1;
    const int r = (nf - 1) / 2;
    const int need = min_support > 3 ? min_support : 3;
#pragma omp parallel for schedule(dynamic, 1)
    for (int v = 0; v < H; ++v) {
        for (int u = 0; u < W; ++u) {
            const double Dc = D[(int64_t)v * W + u];
            double *o = &out[(int64_t)v * W + u];
            if (!is_valid(Dc)) { *o = NAN; continue; }
            int64_t M[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
            double rhs[3] = {0.0, 0.0, 0.0};
            int count = 0;
            for (int dy = -r; dy <= r; ++dy) {
                for (int dx = -r; dx <= r; ++dx) {
                    const int uu = u + dx, vv = v + dy;
                    if (uu < 0 || uu >= W || vv < 0 || vv >= H) continue;
                    const double Di = D[(int64_t)vv * W + uu];
                    if (!is_valid(Di)) continue;
                    const int64_t phi[3] = {1, dx, dy};
                    for (int a = 0; a < 3; ++a) {
                        for (int b = 0; b < 3; ++b) M[a][b] += phi[a] * phi[b];
                        rhs[a] += (double)phi[a] * (Di - Dc);
                    }
                    ++count;
                }
            }
            if (count < need) { *o = Dc; continue; }
            const int64_t det = det3_int(M);
            if (det == 0) { *o = Dc; continue; }
            /* Cramer's rule for the first unknown (h - D_c). */
            const double num =
                rhs[0] * (double)(M[1][1] * M[2][2] - M[1][2] * M[2][1])
              - (double)M[0][1] * (rhs[1] * (double)M[2][2] - (double)M[1][2] * rhs[2])
              + (double)M[0][2] * (rhs[1] * (double)M[2][1] - (double)M[1][1] * rhs[2]);
            *o = Dc + num / (double)det;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Affine parameters (Sec. 3.2-3.3).  With the paper's disparity d = -D and  */
/* v_i = p_i - c, the LSQ of V a = d over the valid neighbours i != c gives   */
/*   a1 - 1 = sum_i s_1i (d_i - d_c),  a2 = sum_i s_2i (d_i - d_c),           */
/*   s_1i = (gamma v_ix - beta v_iy)/(alpha gamma - beta^2),                  */
/*   s_2i = (-beta v_ix + alpha v_iy)/(alpha gamma - beta^2),                 */
/* with alpha, beta, gamma summed over the same (masked) support, i.e. the    */
/* first pass of the two-pass scheme of Sec. 3.4.  a3 = 0, a4 = 1 (Sec. 2).   */
/* defined[c] = 1 iff the centre is valid, the support holds >= min_support  */
/* pixels and alpha*gamma - beta^2 > 0 (exact integers).                     */
/* ------------------------------------------------------------------------ */
int snxo_affine(const double *Dt, int W, int H, int ng, int min_support,
                double *a1, double *a2, uint8_t *defined)
{
    if (ng < 3 || (ng % 2) == 0 || W < 1 || H < 1) return 1;
    const int r = (ng - 1) / 2;
#pragma omp parallel for schedule(dynamic, 1)
    for (int v = 0; v < H; ++v) {
        for (int u = 0; u < W; ++u) {
            const int64_t c = (int64_t)v * W + u;
            a1[c] = NAN; a2[c] = NAN; defined[c] = 0;
            const double dc = -Dt[c];
            if (!is_valid(Dt[c])) continue;
            /* pass 1: alpha, beta, gamma over the selected pixels */
            int64_t alpha = 0, beta = 0, gamma = 0;
            int count = 0;
            for (int dy = -r; dy <= r; ++dy)
                for (int dx = -r; dx <= r; ++dx) {
                    if (dx == 0 && dy == 0) continue;
                    const int uu = u + dx, vv = v + dy;
                    if (uu < 0 || uu >= W || vv < 0 || vv >= H) continue;
                    if (!is_valid(Dt[(int64_t)vv * W + uu])) continue;
                    alpha += (int64_t)dx * dx;
                    beta += (int64_t)dx * dy;
                    gamma += (int64_t)dy * dy;
                    ++count;
                }
            const int64_t det = alpha * gamma - beta * beta;
            if (count < min_support || det <= 0) continue;
            /* pass 2: the two weighted sums of eqs. convprep / convprep2 */
            double sum1 = 0.0, sum2 = 0.0;
            for (int dy = -r; dy <= r; ++dy)
                for (int dx = -r; dx <= r; ++dx) {
                    if (dx == 0 && dy == 0) continue;
                    const int uu = u + dx, vv = v + dy;
                    if (uu < 0 || uu >= W || vv < 0 || vv >= H) continue;
                    const double Di = Dt[(int64_t)vv * W + uu];
                    if (!is_valid(Di)) continue;
                    const double di = -Di;
                    const double s1 = ((double)gamma * dx - (double)beta * dy) / (double)det;
                    const double s2 = (-(double)beta * dx + (double)alpha * dy) / (double)det;
                    sum1 += s1 * (di - dc);
                    sum2 += s2 * (di - dc);
                }
            a1[c] = 1.0 + sum1;
            a2[c] = sum2;
            defined[c] = 1;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Component-restricted window: as snxo_affine, with neighbour i of the      */
/* n_g x n_g window taken only if it is valid and lab[i] == lab[c] (labels   */
/* of the surface components, e.g. from snxo_components; the paper's concern */
/* that points of a neighbouring surface smooth the normals, Sec. 3.4).      */
/* A centre with lab < 0 is undefined.                                        */
/* ------------------------------------------------------------------------ */
int snxo_affine_labels(const double *Dt, const int32_t *lab, int W, int H, int ng,
                       int min_support, double *a1, double *a2, uint8_t *defined)
{
    if (ng < 3 || (ng % 2) == 0 || W < 1 || H < 1) return 1;
    const int r = (ng - 1) / 2;
#pragma omp parallel for schedule(dynamic, 1)
    for (int v = 0; v < H; ++v) {
        for (int u = 0; u < W; ++u) {
            const int64_t c = (int64_t)v * W + u;
            a1[c] = NAN; a2[c] = NAN; defined[c] = 0;
            if (!is_valid(Dt[c]) || lab[c] < 0) continue;
            const double dc = -Dt[c];
            int64_t alpha = 0, beta = 0, gamma = 0;
            int count = 0;
            for (int dy = -r; dy <= r; ++dy)
                for (int dx = -r; dx <= r; ++dx) {
                    if (dx == 0 && dy == 0) continue;
                    const int uu = u + dx, vv = v + dy;
                    if (uu < 0 || uu >= W || vv < 0 || vv >= H) continue;
                    const int64_t i = (int64_t)vv * W + uu;
                    if (!is_valid(Dt[i]) || lab[i] != lab[c]) continue;
                    alpha += (int64_t)dx * dx;
                    beta += (int64_t)dx * dy;
                    gamma += (int64_t)dy * dy;
                    ++count;
                }
            const int64_t det = alpha * gamma - beta * beta;
            if (count < min_support || det <= 0) continue;
            double sum1 = 0.0, sum2 = 0.0;
            for (int dy = -r; dy <= r; ++dy)
                for (int dx = -r; dx <= r; ++dx) {
                    if (dx == 0 && dy == 0) continue;
                    const int uu = u + dx, vv = v + dy;
                    if (uu < 0 || uu >= W || vv < 0 || vv >= H) continue;
                    const int64_t i = (int64_t)vv * W + uu;
                    if (!is_valid(Dt[i]) || lab[i] != lab[c]) continue;
                    const double di = -Dt[i];
                    const double s1 = ((double)gamma * dx - (double)beta * dy) / (double)det;
                    const double s2 = (-(double)beta * dx + (double)alpha * dy) / (double)det;
                    sum1 += s1 * (di - dc);
                    sum2 += s2 * (di - dc);
                }
            a1[c] = 1.0 + sum1;
            a2[c] = sum2;
            defined[c] = 1;
        }
    }
    return 0;
}

/* Back-projection of pixel (u, v) with disparity D through the rectified pair
 * of Sec. 2: Pi_1u - Pi_2u = f_x b / z, so z = f_x b / D,
 * x = (u - u0) z / f_x, y = (v - v0) z / f_y. */
static void backproject(double u, double v, double D, double fx, double fy,
                        double b, double u0, double v0, double X[3])
{
    const double z = fx * b / D;
    X[0] = (u - u0) * z / fx;
    X[1] = (v - v0) * z / fy;
    X[2] = z;
}

/* ------------------------------------------------------------------------ */
/* Normal (Sec. 3.1): n is orthogonal to a1 v1 - v2 and a2 v3 - v4 with       */
/*   v1 = X, v2 = [x - b, y, z], v3 = f_y X, v4 = [0, -b f_x, 0],             */
/* so n is parallel to their cross product.  It is normalised and oriented   */
/* towards the camera (n . X < 0).                                           */
/* ------------------------------------------------------------------------ */
int snxo_normals(const double *Dt, const double *a1, const double *a2,
                 const uint8_t *defined, int W, int H, double fx, double fy,
                 double b, double u0, double v0, double *nrm /* H*W*3 */)
{
#pragma omp parallel for schedule(static)
    for (int v = 0; v < H; ++v) {
        for (int u = 0; u < W; ++u) {
            const int64_t c = (int64_t)v * W + u;
            double *n = &nrm[3 * c];
            if (!defined[c]) { n[0] = n[1] = n[2] = NAN; continue; }
            double X[3];
            backproject(u, v, Dt[c], fx, fy, b, u0, v0, X);
            const double p[3] = {a1[c] * X[0] - (X[0] - b),
                                 a1[c] * X[1] - X[1],
                                 a1[c] * X[2] - X[2]};
            const double q[3] = {a2[c] * fy * X[0] - 0.0,
                                 a2[c] * fy * X[1] + b * fx,
                                 a2[c] * fy * X[2] - 0.0};
            double m[3] = {p[1] * q[2] - p[2] * q[1],
                           p[2] * q[0] - p[0] * q[2],
                           p[0] * q[1] - p[1] * q[0]};
            const double len = sqrt(m[0] * m[0] + m[1] * m[1] + m[2] * m[2]);
            if (!(len > 0.0) || !isfinite(len)) { n[0] = n[1] = n[2] = NAN; continue; }
            const double s = (m[0] * X[0] + m[1] * X[1] + m[2] * X[2]) > 0.0 ? -1.0 : 1.0;
            n[0] = s * m[0] / len;
            n[1] = s * m[1] / len;
            n[2] = s * m[2] / len;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Components: 4-neighbours p, q are joined iff both are valid and           */
/*   |D_p - D_q| <= max(t_abs, k_rel * min(D_p, D_q))                         */
/* evaluated in binary64 on the float32 disparities with no contraction (built */
/* with -ffp-contract=off; the products are exact anyway) -- the            */
/* pairwise form of the covered-depth stopping rule, Sec. 3.4).  Label of a  */
/* pixel = smallest linear index v*W + u of its component; -1 if invalid.    */
/* Breadth-first flood fill started from each unlabelled valid pixel in      */
/* raster order, so the seed is the component's smallest index.              */
/* ------------------------------------------------------------------------ */
static int joined(float fp, float fq, float k_rel, float t_abs)
{
    const double a = (double)fp, b = (double)fq;
    if (!is_valid(a) || !is_valid(b)) return 0;
    volatile double d = fabs(a - b);
    volatile double prod = (double)k_rel * fmin(a, b);
    volatile double t = fmax((double)t_abs, prod);
    return d <= t;
}

int snxo_components(const float *D, int W, int H, float k_rel, float t_abs,
                    int32_t *labels, int64_t *num_components)
{
    const int64_t N = (int64_t)W * H;
    int64_t *queue = (int64_t *)malloc(sizeof(int64_t) * (size_t)(N > 0 ? N : 1));
    if (!queue) return 2;
    for (int64_t i = 0; i < N; ++i) labels[i] = -1;
    int64_t count = 0;
    for (int64_t s = 0; s < N; ++s) {
        if (labels[s] != -1 || !is_valid((double)D[s])) continue;
        ++count;
        int64_t head = 0, tail = 0;
        queue[tail++] = s;
        labels[s] = (int32_t)s;
        while (head < tail) {
            const int64_t p = queue[head++];
            const int u = (int)(p % W), v = (int)(p / W);
            const int64_t nb[4] = {u > 0 ? p - 1 : -1, u + 1 < W ? p + 1 : -1,
                                   v > 0 ? p - W : -1, v + 1 < H ? p + W : -1};
            for (int k = 0; k < 4; ++k) {
                const int64_t q = nb[k];
                if (q < 0 || labels[q] != -1) continue;
                if (!joined(D[p], D[q], k_rel, t_abs)) continue;
                labels[q] = (int32_t)s;
                queue[tail++] = q;
            }
        }
    }
    free(queue);
    *num_components = count;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Components of an explicitly given 4-neighbour graph (the test hook of the  */
/* labelling: every edge pattern can be posed, independently of validity).   */
/* flags[v * W + u]: bit 0 = pixel present, bit 1 = edge to (u - 1, v),      */
/* bit 2 = edge to (u, v - 1); an edge counts only between two present       */
/* pixels.  Labels and count as snxo_components (BFS in raster order).       */
/* ------------------------------------------------------------------------ */
/* Edge between p and its neighbour q in direction k (0 left, 1 right, 2 up,
 * 3 down): the bit sits on the right or lower pixel of the pair. */
static int edge_bits(const uint8_t *f, int64_t p, int64_t q, int k)
{
    if (!(f[p] & 1) || !(f[q] & 1)) return 0;
    switch (k) {
    case 0: return (f[p] >> 1) & 1;
    case 1: return (f[q] >> 1) & 1;
    case 2: return (f[p] >> 2) & 1;
    default: return (f[q] >> 2) & 1;
    }
}

int snxo_components_edges(const uint8_t *flags, int W, int H, int32_t *labels,
                          int64_t *num_components)
{
    const int64_t N = (int64_t)W * H;
    int64_t *queue = (int64_t *)malloc(sizeof(int64_t) * (size_t)(N > 0 ? N : 1));
    if (!queue) return 2;
    for (int64_t i = 0; i < N; ++i) labels[i] = -1;
    int64_t count = 0;
    for (int64_t s = 0; s < N; ++s) {
        if (labels[s] != -1 || !(flags[s] & 1)) continue;
        ++count;
        int64_t head = 0, tail = 0;
        queue[tail++] = s;
        labels[s] = (int32_t)s;
        while (head < tail) {
            const int64_t p = queue[head++];
            const int u = (int)(p % W), v = (int)(p / W);
            const int64_t nb[4] = {u > 0 ? p - 1 : -1, u + 1 < W ? p + 1 : -1,
                                   v > 0 ? p - W : -1, v + 1 < H ? p + W : -1};
            for (int k = 0; k < 4; ++k) {
                const int64_t q = nb[k];
                if (q < 0 || labels[q] != -1 || !edge_bits(flags, p, q, k)) continue;
                labels[q] = (int32_t)s;
                queue[tail++] = q;
            }
        }
    }
    free(queue);
    *num_components = count;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Crease-aware components: as snxo_components, and an edge also needs the   */
/* two pixels' unit normals (float32 planes nrm[0..2][v * W + u]) to agree:   */
/*   n_p . n_q = ((nx_p nx_q + ny_p ny_q) + nz_p nz_q) >= cos_min             */
/* in binary64 (each product of two float32 values is exact); a pixel whose  */
/* normal is undefined (NaN) imposes no crease test.  Sec. 3.4 notes that    */
/* covered depth misses depth-continuous (C0) edges; this is the test that   */
/* separates surfaces meeting at such a crease.                              */
/* ------------------------------------------------------------------------ */
static int crease_ok(const float *nrm, int64_t plane, int64_t p, int64_t q, double cmin)
{
    const double ax = nrm[p], ay = nrm[plane + p], az = nrm[2 * plane + p];
    const double bx = nrm[q], by = nrm[plane + q], bz = nrm[2 * plane + q];
    if (isnan(ax) || isnan(bx)) return 1;
    return ((ax * bx + ay * by) + az * bz) >= cmin;
}

int snxo_components_crease(const float *D, const float *nrm, int W, int H, float k_rel,
                           float t_abs, double cos_min, int32_t *labels,
                           int64_t *num_components)
{
    const int64_t N = (int64_t)W * H;
    int64_t *queue = (int64_t *)malloc(sizeof(int64_t) * (size_t)(N > 0 ? N : 1));
    if (!queue) return 2;
    for (int64_t i = 0; i < N; ++i) labels[i] = -1;
    int64_t count = 0;
    for (int64_t s = 0; s < N; ++s) {
        if (labels[s] != -1 || !is_valid((double)D[s])) continue;
        ++count;
        int64_t head = 0, tail = 0;
        queue[tail++] = s;
        labels[s] = (int32_t)s;
        while (head < tail) {
            const int64_t p = queue[head++];
            const int u = (int)(p % W), v = (int)(p / W);
            const int64_t nb[4] = {u > 0 ? p - 1 : -1, u + 1 < W ? p + 1 : -1,
                                   v > 0 ? p - W : -1, v + 1 < H ? p + W : -1};
            for (int k = 0; k < 4; ++k) {
                const int64_t q = nb[k];
                if (q < 0 || labels[q] != -1) continue;
                if (!joined(D[p], D[q], k_rel, t_abs)) continue;
                if (!crease_ok(nrm, N, p, q, cos_min)) continue;
                labels[q] = (int32_t)s;
                queue[tail++] = q;
            }
        }
    }
    free(queue);
    *num_components = count;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Dense oriented point cloud: where the normal is defined, X from the       */
/* rectified projections (Sec. 2) at the filtered disparity, plus n and the  */
/* component label; elsewhere NaN coordinates and normal, label kept.        */
/* out: H*W*6 doubles (x, y, z, nx, ny, nz).                                  */
/* ------------------------------------------------------------------------ */
int snxo_point_cloud(const double *Dt, const double *nrm, int W, int H,
                     double fx, double fy, double b, double u0, double v0,
                     double *out)
{
#pragma omp parallel for schedule(static)
    for (int v = 0; v < H; ++v) {
        for (int u = 0; u < W; ++u) {
            const int64_t c = (int64_t)v * W + u;
            double *o = &out[6 * c];
            const double *n = &nrm[3 * c];
            if (!isfinite(n[0]) || !is_valid(Dt[c])) {
                for (int k = 0; k < 6; ++k) o[k] = NAN;
                continue;
            }
            double X[3];
            backproject(u, v, Dt[c], fx, fy, b, u0, v0, X);
            o[0] = X[0]; o[1] = X[1]; o[2] = X[2];
            o[3] = n[0]; o[4] = n[1]; o[5] = n[2];
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Adaptive star-fill support (Sec. 3.4, Adaptive Region Estimation).        */
/* From a valid centre c, rays leave in M = 4, 8 or 16 directions e_m: the  */
/* directions at angles 2 pi m / M scaled so that their larger component is  */
/* 1 (for M = 8 the axes and the diagonals, for M = 4 the axes).  Ray m      */
/* takes the pixels c + round(k e_m), k = 1 .. steps, in order, and stops    */
/* before the first one that is invalid or outside the image or meets the    */
/* stopping rule:                                                            */
/*   CD  covered depth: with a, b the smallest and the largest disparity of  */
/*       c and of the ray's pixels up to and including the new one, stop     */
/*       when D_c (b - a) > k (a b): the depth range f_x B (1/a - 1/b)        */
/*       exceeds k times the depth f_x B / D_c of c (binary64, no            */
/*       contraction; b - a, a b and D_c (b - a) are exact);                 */
/*   ST  simple threshold on the depth Laplacian: stop when                  */
/*       L = ((z_r + z_l) + (z_d + z_u)) - 4 z  at the new pixel, with        */
/*       z = fxb / D (binary64), is undefined (a 4-neighbour invalid or       */
/*       outside the image) or |L| > t.                                       */
/* The support is the set of pixels taken by the rays (their union: for     */
/* M = 16 neighbouring rays share their first pixel); c anchors the fit.     */
/* ------------------------------------------------------------------------ */
#define SNXO_STOP_CD 0
#define SNXO_STOP_ST 1

/* Offset of step k along ray m of M (Sec. 3.4 star fill; the rasterisation is a
 * reading): the direction at angle 2 pi m / M, scaled so that its larger
 * component is 1, times k, each component rounded to the nearest pixel.  For
 * M = 4 and 8 this gives the axes and the diagonals exactly. */
static void star_offset(int m, int M, int k, int *dx, int *dy)
{
    const double th = 2.0 * M_PI * (double)m / (double)M;
    const double c = cos(th), s = sin(th);
    const double big = fabs(c) > fabs(s) ? fabs(c) : fabs(s);
    *dx = (int)lround((double)k * c / big);
    *dy = (int)lround((double)k * s / big);
}

static int star_valid_at(const double *Dt, int W, int H, int u, int v)
{
    return u >= 0 && u < W && v >= 0 && v < H && is_valid(Dt[(int64_t)v * W + u]);
}

/* 1 iff the depth Laplacian at (u, v) is undefined or exceeds t in magnitude */
static int star_st_edge(const double *Dt, int W, int H, int u, int v, double fxb, double t)
{
    static const int nb[4][2] = {{1, 0}, {-1, 0}, {0, 1}, {0, -1}};
    for (int i = 0; i < 4; ++i)
        if (!star_valid_at(Dt, W, H, u + nb[i][0], v + nb[i][1])) return 1;
    const double zc = fxb / Dt[(int64_t)v * W + u];
    const double zr = fxb / Dt[(int64_t)v * W + u + 1];
    const double zl = fxb / Dt[(int64_t)v * W + u - 1];
    const double zd = fxb / Dt[(int64_t)(v + 1) * W + u];
    const double zu = fxb / Dt[(int64_t)(v - 1) * W + u];
    const double L = ((zr + zl) + (zd + zu)) - 4.0 * zc;
    return fabs(L) > t;
}

/* Marks the support of centre (u, v) in mask[(dy + s) * (2s + 1) + dx + s]
 * (the centre itself is not marked) and returns the number of marked pixels,
 * or -1 for bad arguments or an invalid centre. */
int snxo_star_mask(const double *Dt, int W, int H, int u, int v, int dirs, int steps,
                   int stop, double thr, double fxb, uint8_t *mask)
{
    if ((dirs != 4 && dirs != 8 && dirs != 16) || steps < 1 ||
        (stop != SNXO_STOP_CD && stop != SNXO_STOP_ST))
        return -1;
    const int side = 2 * steps + 1;
    memset(mask, 0, (size_t)side * side);
    if (!star_valid_at(Dt, W, H, u, v)) return -1;
    const double Dc = Dt[(int64_t)v * W + u];
    int count = 0;
    for (int m = 0; m < dirs; ++m) {
        double a = Dc, b = Dc;
        for (int k = 1; k <= steps; ++k) {
            int ox, oy;
            star_offset(m, dirs, k, &ox, &oy);
            const int uu = u + ox, vv = v + oy;
            if (!star_valid_at(Dt, W, H, uu, vv)) break;
            const double Di = Dt[(int64_t)vv * W + uu];
            if (stop == SNXO_STOP_CD) {
                const double na = Di < a ? Di : a, nbv = Di > b ? Di : b;
                if (Dc * (nbv - na) > thr * (na * nbv)) break;
                a = na;
                b = nbv;
            } else if (star_st_edge(Dt, W, H, uu, vv, fxb, thr)) {
                break;
            }
            /* the support is the union of the pixels the rays visit */
            uint8_t *mk = &mask[(oy + steps) * side + ox + steps];
            if (!*mk) { *mk = 1; ++count; }
        }
    }
    return count;
}

/* a1, a2 and definedness over the star-fill support: the anchored LSQ of
 * snxo_affine with the window replaced by the support (pass 1: alpha, beta,
 * gamma; pass 2: the weighted sums).  defined iff the centre is valid, the
 * support holds >= min_support pixels and alpha gamma - beta^2 > 0. */
int snxo_star_affine(const double *Dt, int W, int H, int dirs, int steps, int stop,
                     double thr, double fxb, int min_support, double *a1, double *a2,
                     uint8_t *defined)
{
    if ((dirs != 4 && dirs != 8 && dirs != 16) || steps < 1 || steps > 64 || W < 1 || H < 1 ||
        (stop != SNXO_STOP_CD && stop != SNXO_STOP_ST))
        return 1;
    const int side = 2 * steps + 1;
    int fail = 0;
#pragma omp parallel
    {
        uint8_t *mask = (uint8_t *)malloc((size_t)side * side);
        if (!mask) {
#pragma omp atomic write
            fail = 1;
        }
#pragma omp for schedule(dynamic, 1)
        for (int v = 0; v < H; ++v) {
            for (int u = 0; u < W; ++u) {
                const int64_t c = (int64_t)v * W + u;
                a1[c] = NAN; a2[c] = NAN; defined[c] = 0;
                if (!mask) continue;
                const int count = snxo_star_mask(Dt, W, H, u, v, dirs, steps, stop, thr, fxb, mask);
                if (count < 0) continue;
                const double dc = -Dt[c];
                int64_t alpha = 0, beta = 0, gamma = 0;
                for (int dy = -steps; dy <= steps; ++dy)
                    for (int dx = -steps; dx <= steps; ++dx) {
                        if (!mask[(dy + steps) * side + dx + steps]) continue;
                        alpha += (int64_t)dx * dx;
                        beta += (int64_t)dx * dy;
                        gamma += (int64_t)dy * dy;
                    }
                const int64_t det = alpha * gamma - beta * beta;
                if (count < min_support || det <= 0) continue;
                double sum1 = 0.0, sum2 = 0.0;
                for (int dy = -steps; dy <= steps; ++dy)
                    for (int dx = -steps; dx <= steps; ++dx) {
                        if (!mask[(dy + steps) * side + dx + steps]) continue;
                        const double di = -Dt[(int64_t)(v + dy) * W + u + dx];
                        const double s1 = ((double)gamma * dx - (double)beta * dy) / (double)det;
                        const double s2 = (-(double)beta * dx + (double)alpha * dy) / (double)det;
                        sum1 += s1 * (di - dc);
                        sum2 += s2 * (di - dc);
                    }
                a1[c] = 1.0 + sum1;
                a2[c] = sum2;
                defined[c] = 1;
            }
        }
        free(mask);
    }
    return fail;
}

int snxo_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of later calls (the CPU baseline is timed on all cores and on one). */
int snxo_set_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}
