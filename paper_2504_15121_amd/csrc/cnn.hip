// Learned residual denoiser: 3x3 convolutions as BF16 MFMA with FP32 accumulation
// (v_mfma_f32_16x16x32_bf16 on gfx950), its training kernels and the normal-loss
// head.
//
// Model:  mu = LSQ filter (window 3) of the disparity; x = [(D - mu)/s, valid];
//         a_k = relu(conv(W_k, a_{k-1}) + b_k) for 2->32, 4 x 32->32;
//         y = conv(W_6, a_5) + b_6 (32->1); D~ = mu + s*y at valid pixels.
// conv is a 3x3 cross-correlation with zero padding.  Activations are stored
// NHWC bfloat16 (32 channels, 64 bytes per pixel); rounding to bfloat16 is round
// to nearest even.
//
// Implicit GEMM per 16 x 16 output tile (256 threads, 4 waves x 4 rows):
// M = 16 pixels of one row, N = 16 output channels, K = 32 = one tap x 32 input
// channels (middle layers) or all 9 taps x C input channels packed into one K
// slice (first layer C = 2, transposed last layer C = 1).  MFMA operand layout
// (16x16x32): lane l holds A[l%16][8(l/16) .. 8(l/16)+7] and
// B[8(l/16) .. +7][l%16]; the result C[4(l/16)+j][l%16], j = 0..3.
//
// Backward-data of a layer is the same convolution over the output gradient
// with flipped taps and transposed channels, followed by the mask of the
// previous ReLU.  Weight gradients are per-workgroup partial sums reduced in a
// fixed order (deterministic).
#include <stdint.h>

#include "lsq.hpp"
#include "snx_cnn.hpp"

namespace snx {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int kT = 16;          // output tile edge
constexpr int kIn = kT + 2;     // input tile edge (halo 1)

__device__ __forceinline__ uint16_t to_bf16(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ bf16x8 as_bf16x8(u32x4 v) { return __builtin_bit_cast(bf16x8, v); }

__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// ----------------------------------------------------------------------------
// Middle-layer convolution (32 -> 32 channels, or 32 -> 1 when LAST).
//   MODE 0: forward, bias (the accumulators' initial value) + ReLU, bf16 NHWC out
//   MODE 1: backward-data, multiply by [mask_src > 0], bf16 NHWC out
//   MODE 2: last layer forward: D~ = mu + s * y at valid pixels, y starting from
//           the bias (f32 out)
// wts: [9 taps][N][32] bf16 (N = 32, or 16 with only row 0 used for MODE 2).
// ----------------------------------------------------------------------------
template <int MODE>
__global__ void __launch_bounds__(256)
k_conv32(ConvArgs a)
{
    __shared__ __attribute__((aligned(16))) uint16_t tile[kIn * kIn * 32];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int x0 = blockIdx.x * kT, y0 = blockIdx.y * kT, b = blockIdx.z;
    const int W = a.W, H = a.H;
    const int64_t plane = (int64_t)W * H;
    const uint16_t *in = a.act_in + (int64_t)b * plane * 32;
    constexpr int NB = MODE == 2 ? 1 : 2;

    // weights -> registers (B operands), issued before the tile load
    u32x4 wb[9][NB];
    {
        const int n = lane & 15, g = lane >> 4;
#pragma unroll
        for (int t = 0; t < 9; ++t)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                const int N = MODE == 2 ? 16 : 32;
                wb[t][nb] = *reinterpret_cast<const u32x4 *>(a.wts + ((t * N + nb * 16 + n) * 32 + g * 8));
            }
    }
    // input tile with halo: 18 x 18 pixels x 64 bytes, 16 bytes per load
    for (int c = tid; c < kIn * kIn * 4; c += 256) {
        const int p = c >> 2, q = c & 3;
        const int ly = p / kIn, lx = p - ly * kIn;
        const int gy = y0 - 1 + ly, gx = x0 - 1 + lx;
        u32x4 v = {0u, 0u, 0u, 0u};
        if (gy >= 0 && gy < H && gx >= 0 && gx < W)
            v = *reinterpret_cast<const u32x4 *>(in + ((int64_t)gy * W + gx) * 32 + q * 8);
        *reinterpret_cast<u32x4 *>(tile + p * 32 + q * 8) = v;
    }
    __syncthreads();

    // the bias is the accumulators' initial value (lane: output channel nb*16 + l%16)
    f32x4 acc[4][NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
        const float b0 = MODE == 0 ? a.bias[nb * 16 + (lane & 15)] : MODE == 2 ? a.bias[0] : 0.0f;
#pragma unroll
        for (int mb = 0; mb < 4; ++mb) acc[mb][nb] = (f32x4){b0, b0, b0, b0};
    }
    {
        const int col = lane & 15, g = lane >> 4;
#pragma unroll
        for (int mb = 0; mb < 4; ++mb) {
            const int row = wave * 4 + mb;
#pragma unroll
            for (int t = 0; t < 9; ++t) {
                const int dy = t / 3 - 1, dx = t % 3 - 1;
                const int p = (row + 1 + dy) * kIn + col + 1 + dx;
                const bf16x8 av = as_bf16x8(*reinterpret_cast<const u32x4 *>(tile + p * 32 + g * 8));
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = mfma(av, as_bf16x8(wb[t][nb]), acc[mb][nb]);
            }
        }
    }

    if (MODE == 2) {
        // only output channel 0 is real: lanes with l%16 == 0
        if ((lane & 15) == 0) {
            const int g = lane >> 4;
#pragma unroll
            for (int mb = 0; mb < 4; ++mb) {
                const int gy = y0 + wave * 4 + mb;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int gx = x0 + 4 * g + j;
                    if (gx < W && gy < H) {
                        const int64_t o = (int64_t)b * plane + (int64_t)gy * W + gx;
                        const float mu = a.mu[o];
                        const float y = acc[mb][0][j];
                        a.out[(int64_t)b * a.crop_stride_out + (int64_t)gy * a.ld_out + gx] =
                            (mu == mu) ? mu + a.s * y : __builtin_nanf("");
                    }
                }
            }
        }
        return;
    }

    // transpose through LDS into [pixel][channel] bf16, then coalesced stores
    __syncthreads();
    {
        const int n = lane & 15, g = lane >> 4;
#pragma unroll
        for (int mb = 0; mb < 4; ++mb) {
            const int row = wave * 4 + mb;
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                const int ch = nb * 16 + n;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int p = row * kT + 4 * g + j;
                    float v = acc[mb][nb][j];
                    if (MODE == 0) v = v > 0.0f ? v : 0.0f;
                    tile[p * 32 + ch] = to_bf16(v);
                }
            }
        }
    }
    __syncthreads();
    uint16_t *out = a.act_out + (int64_t)b * plane * 32;
    const uint16_t *msk = MODE == 1 ? a.mask_src + (int64_t)b * plane * 32 : nullptr;
    for (int c = tid; c < kT * kT * 4; c += 256) {
        const int p = c >> 2, q = c & 3;
        const int gy = y0 + p / kT, gx = x0 + (p % kT);
        if (gy >= H || gx >= W) continue;
        const int64_t o = ((int64_t)gy * W + gx) * 32 + q * 8;
        u32x4 v = *reinterpret_cast<const u32x4 *>(tile + p * 32 + q * 8);
        if (MODE == 1) {
            const u32x4 m = *reinterpret_cast<const u32x4 *>(msk + o);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const uint32_t mw = m[i];
                uint32_t keep = 0;
                if ((mw & 0xffffu) != 0 && !(mw & 0x8000u)) keep |= 0xffffu;
                if ((mw >> 16) != 0 && !(mw & 0x80000000u)) keep |= 0xffff0000u;
                v[i] &= keep;
            }
        }
        *reinterpret_cast<u32x4 *>(out + o) = v;
    }
}

// ----------------------------------------------------------------------------
// Small-input convolution: C_IN = 2 (first layer; input built from D and mu) or
// C_IN = 1 (backward-data of the last layer; input = dL/dy in f32), 9 taps x C_IN
// packed into one K slice of 32.  Output: 32 channels bf16 NHWC, with bias+ReLU
// (first layer) or the mask [mask_src > 0] (backward).
// wts: [32 out][32 k-slots] bf16, slot = tap * C_IN + c (zero beyond 9 * C_IN).
// ----------------------------------------------------------------------------
template <int C_IN>
__global__ void __launch_bounds__(256)
k_conv_small(ConvArgs a)
{
    __shared__ float sx[C_IN][kIn * kIn];
    __shared__ __attribute__((aligned(16))) uint16_t tile[kT * kT * 32];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int x0 = blockIdx.x * kT, y0 = blockIdx.y * kT, b = blockIdx.z;
    const int W = a.W, H = a.H;
    const int64_t plane = (int64_t)W * H;

    u32x4 wb[2];
    {
        const int n = lane & 15, g = lane >> 4;
#pragma unroll
        for (int nb = 0; nb < 2; ++nb)
            wb[nb] = *reinterpret_cast<const u32x4 *>(a.wts + (nb * 16 + n) * 32 + g * 8);
    }
    for (int p = tid; p < kIn * kIn; p += 256) {
        const int ly = p / kIn, lx = p - ly * kIn;
        const int gy = y0 - 1 + ly, gx = x0 - 1 + lx;
        float v0 = 0.0f, v1 = 0.0f;
        if (gy >= 0 && gy < H && gx >= 0 && gx < W) {
            if (C_IN == 2) {
                const float d = a.D[(int64_t)b * a.crop_stride_D + (int64_t)gy * a.ldD + gx];
                const float mu = a.mu[(int64_t)b * plane + (int64_t)gy * W + gx];
                if (valid_disp(d)) {
                    v0 = from_bf16(to_bf16((d - mu) / a.s));
                    v1 = 1.0f;
                }
            } else {
                v0 = from_bf16(to_bf16(a.grad_in[(int64_t)b * plane + (int64_t)gy * W + gx]));
            }
        }
        sx[0][p] = v0;
        if (C_IN == 2) sx[C_IN - 1][p] = v1;
    }
    __syncthreads();

    f32x4 acc[4][2];
    const int col = lane & 15, g = lane >> 4;
    // first layer: the bias is the accumulators' initial value
    f32x4 bias0[2];
#pragma unroll
    for (int nb = 0; nb < 2; ++nb) {
        const float b0 = C_IN == 2 ? a.bias[nb * 16 + col] : 0.0f;
        bias0[nb] = (f32x4){b0, b0, b0, b0};
    }
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) {
        const int row = wave * 4 + mb;
        // A operand: K slots 8g .. 8g+7 -> (tap, channel)
        uint16_t av[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int slot = g * 8 + i;
            const int t = slot / C_IN, c = slot - t * C_IN;
            float v = 0.0f;
            if (t < 9) {
                const int dy = t / 3 - 1, dx = t % 3 - 1;
                v = sx[c][(row + 1 + dy) * kIn + col + 1 + dx];
            }
            av[i] = to_bf16(v);
        }
        u32x4 ap;
#pragma unroll
        for (int i = 0; i < 4; ++i) ap[i] = (uint32_t)av[2 * i] | ((uint32_t)av[2 * i + 1] << 16);
#pragma unroll
        for (int nb = 0; nb < 2; ++nb)
            acc[mb][nb] = mfma(as_bf16x8(ap), as_bf16x8(wb[nb]), bias0[nb]);
    }
    const int n = lane & 15;
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) {
        const int row = wave * 4 + mb;
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) {
            const int ch = nb * 16 + n;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                float v = acc[mb][nb][j];
                if (C_IN == 2) v = v > 0.0f ? v : 0.0f;
                tile[(row * kT + 4 * g + j) * 32 + ch] = to_bf16(v);
            }
        }
    }
    __syncthreads();
    uint16_t *out = a.act_out + (int64_t)b * plane * 32;
    const uint16_t *msk = C_IN == 1 ? a.mask_src + (int64_t)b * plane * 32 : nullptr;
    for (int c = tid; c < kT * kT * 4; c += 256) {
        const int p = c >> 2, q = c & 3;
        const int gy = y0 + p / kT, gx = x0 + (p % kT);
        if (gy >= H || gx >= W) continue;
        const int64_t o = ((int64_t)gy * W + gx) * 32 + q * 8;
        u32x4 v = *reinterpret_cast<const u32x4 *>(tile + p * 32 + q * 8);
        if (C_IN == 1) {
            const u32x4 m = *reinterpret_cast<const u32x4 *>(msk + o);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const uint32_t mw = m[i];
                uint32_t keep = 0;
                if ((mw & 0xffffu) != 0 && !(mw & 0x8000u)) keep |= 0xffffu;
                if ((mw >> 16) != 0 && !(mw & 0x80000000u)) keep |= 0xffff0000u;
                v[i] &= keep;
            }
        }
        *reinterpret_cast<u32x4 *>(out + o) = v;
    }
}

// ----------------------------------------------------------------------------
// Weight gradients, FP32 partial sums per workgroup over a 16 x 16 pixel tile
// (and one batch item):  dW[co][ci][t] = sum_p X[p + off(t)][ci] * G[p][co],
// db[co] = sum_p G[p][co].  X: NHWC32 bf16 (CI = 32) or the first-layer input
// rebuilt from D and mu (CI = 2); G: NHWC32 bf16 (CO = 32) or f32 (CO = 1).
// Each thread owns CO*CI*9/256 weights (or fewer); the partial of block k goes
// to partial[k * n_w ...].  k_wgrad_reduce sums the partials in block order.
// ----------------------------------------------------------------------------
template <int CI, int CO>
__global__ void __launch_bounds__(256)
k_wgrad(ConvArgs a, float *partial)
{
    __shared__ uint16_t sxv[CI][kIn * kIn];
    __shared__ float sg[CO][kT * kT];
    const int tid = threadIdx.x;
    const int x0 = blockIdx.x * kT, y0 = blockIdx.y * kT, b = blockIdx.z;
    const int W = a.W, H = a.H;
    const int64_t plane = (int64_t)W * H;
    for (int p = tid; p < kIn * kIn; p += 256) {
        const int ly = p / kIn, lx = p - ly * kIn;
        const int gy = y0 - 1 + ly, gx = x0 - 1 + lx;
        const bool in = gy >= 0 && gy < H && gx >= 0 && gx < W;
        if (CI == 2) {
            uint16_t v0 = 0, v1 = 0;
            if (in) {
                const float d = a.D[(int64_t)b * a.crop_stride_D + (int64_t)gy * a.ldD + gx];
                const float mu = a.mu[(int64_t)b * plane + (int64_t)gy * W + gx];
                if (valid_disp(d)) {
                    v0 = to_bf16((d - mu) / a.s);
                    v1 = to_bf16(1.0f);
                }
            }
            sxv[0][p] = v0;
            sxv[CI - 1][p] = v1;
        } else {
            const uint16_t *src = a.act_in + ((int64_t)b * plane + (int64_t)gy * W + gx) * 32;
            for (int c = 0; c < CI; ++c) sxv[c][p] = in ? src[c] : (uint16_t)0;
        }
    }
    for (int p = tid; p < kT * kT; p += 256) {
        const int gy = y0 + p / kT, gx = x0 + (p % kT);
        const bool in = gy < H && gx < W;
        if (CO == 1) {
            sg[0][p] = in ? a.grad_in[(int64_t)b * plane + (int64_t)gy * W + gx] : 0.0f;
        } else {
            const uint16_t *src = a.act_out + ((int64_t)b * plane + (int64_t)gy * W + gx) * 32;
            for (int c = 0; c < CO; ++c) sg[c][p] = in ? from_bf16(src[c]) : 0.0f;
        }
    }
    __syncthreads();
    constexpr int NW = CO * CI * 9;
    constexpr int NT = NW + CO;        // weights then biases, as in the flat layout
    const int64_t blk = ((int64_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    float *dst = partial + blk * NT;
    // one (co, ci) pair per thread and pass: all 9 taps share the gradient load
    for (int pr = tid; pr < CO * CI; pr += 256) {
        const int co = pr / CI, ci = pr - co * CI;
        float s[9];
#pragma unroll
        for (int t = 0; t < 9; ++t) s[t] = 0.0f;
        for (int py = 0; py < kT; ++py) {
            for (int px = 0; px < kT; ++px) {
                const float g = sg[co][py * kT + px];
#pragma unroll
                for (int t = 0; t < 9; ++t) {
                    const int dy = t / 3 - 1, dx = t % 3 - 1;
                    s[t] += from_bf16(sxv[ci][(py + 1 + dy) * kIn + px + 1 + dx]) * g;
                }
            }
        }
#pragma unroll
        for (int t = 0; t < 9; ++t) dst[(co * CI + ci) * 9 + t] = s[t];
    }
    for (int co = tid; co < CO; co += 256) {
        float s = 0.0f;
        for (int p = 0; p < kT * kT; ++p) s += sg[co][p];
        dst[NW + co] = s;
    }
}

__global__ void k_wgrad_reduce(const float *partial, int64_t nblk, int nt, float *grad)
{
    const int w = blockIdx.x * 256 + threadIdx.x;
    if (w >= nt) return;
    double s = 0.0;
    for (int64_t k = 0; k < nblk; ++k) s += (double)partial[k * nt + w];
    grad[w] = (float)s;
}

// ----------------------------------------------------------------------------
// Normal-loss head, per pixel: anchored masked LSQ slope of D~ over the n_g
// window (direct sums), normal n = -m/|m|; where a ground-truth normal exists,
// loss term 1 - n.g, and with G = (g - n (n.g)) / |m| (dL/dm before the 1/N),
//   Gu = G . (f_x, 0, -(u-u0)),  Gv = G . (0, f_y, -(v-v0)),
//   A = (gamma Gu - beta Gv)/det,  B = (-beta Gu + alpha Gv)/det,
//   own = G_z - (A Sx + B Sy);
// partial sums of the loss and of the number of used pixels per workgroup, and
// of the fidelity term (D~ - clean)^2 and its pixel count.
// ----------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
k_head(HeadArgs a)
{
    const int gx = blockIdx.x * 64 + (threadIdx.x & 63);
    const int gy = blockIdx.y * 4 + (threadIdx.x >> 6);
    const int b = blockIdx.z;
    const int W = a.W, H = a.H, r = a.rg;
    const int64_t plane = (int64_t)W * H;
    const float *D = a.Dt + (int64_t)b * plane;
    double loss = 0.0, fid = 0.0;
    int used = 0, fused_px = 0;
    if (gx < W && gy < H) {
        const int64_t o = (int64_t)b * plane + (int64_t)gy * W + gx;
        float A = 0.0f, B = 0.0f, own = 0.0f;
        const float Dc = D[(int64_t)gy * W + gx];
        if (a.clean && valid_disp(Dc)) {
            const float c = a.clean[o];
            if (c - c == 0.0f) {
                const double r = (double)Dc - (double)c;
                fid = r * r;
                fused_px = 1;
            }
        }
        if (valid_disp(Dc)) {
            int N = 0, Sx = 0, Sy = 0, al = 0, be = 0, ga = 0;
            double P1 = 0.0, P2 = 0.0;
            for (int dy = -r; dy <= r; ++dy) {
                const int yy = gy + dy;
                if (yy < 0 || yy >= H) continue;
                for (int dx = -r; dx <= r; ++dx) {
                    const int xx = gx + dx;
                    if (xx < 0 || xx >= W || (dx == 0 && dy == 0)) continue;
                    const float v = D[(int64_t)yy * W + xx];
                    if (!valid_disp(v)) continue;
                    ++N; Sx += dx; Sy += dy;
                    al += dx * dx; be += dx * dy; ga += dy * dy;
                    P1 += (double)dx * v;
                    P2 += (double)dy * v;
                }
            }
            const double det = (double)al * ga - (double)be * be;
            const float *ng = a.n_gt + (int64_t)b * 3 * plane + (int64_t)gy * W + gx;
            const double g0 = ng[0], g1 = ng[plane], g2 = ng[2 * plane];
            if (N >= a.need_g && det > 0.0 && g0 == g0) {
                const double dc = Dc;
                const double S1 = P1 - Sx * dc, S2 = P2 - Sy * dc;
                const double gu = (ga * S1 - be * S2) / det, gv = (al * S2 - be * S1) / det;
                const CnnCam cm = a.cams[b];
                const double mx = cm.fx * gu, my = cm.fy * gv;
                const double mz = dc - (gx - cm.u0) * gu - (gy - cm.v0) * gv;
                const double mn = sqrt(mx * mx + my * my + mz * mz);
                const double nx = -mx / mn, ny = -my / mn, nz = -mz / mn;
                const double dot = nx * g0 + ny * g1 + nz * g2;
                loss = 1.0 - dot;
                used = 1;
                const double Gx = (g0 - nx * dot) / mn, Gy = (g1 - ny * dot) / mn,
                             Gz = (g2 - nz * dot) / mn;
                const double Gu = Gx * cm.fx - Gz * (gx - cm.u0);
                const double Gv = Gy * cm.fy - Gz * (gy - cm.v0);
                const double Ad = (ga * Gu - be * Gv) / det, Bd = (-be * Gu + al * Gv) / det;
                A = (float)Ad;
                B = (float)Bd;
                own = (float)(Gz - (Ad * Sx + Bd * Sy));
            }
        }
        a.coefA[o] = A;
        a.coefB[o] = B;
        a.coefOwn[o] = own;
    }
    // workgroup partials (fixed order: wave ballots then lane 0 of wave 0)
    __shared__ double sl[256], sf[256];
    __shared__ int su[256], sc[256];
    sl[threadIdx.x] = loss;
    su[threadIdx.x] = used;
    sf[threadIdx.x] = fid;
    sc[threadIdx.x] = fused_px;
    __syncthreads();
    if (threadIdx.x == 0) {
        double L = 0.0, F = 0.0;
        int U = 0, C = 0;
        for (int i = 0; i < 256; ++i) { L += sl[i]; U += su[i]; F += sf[i]; C += sc[i]; }
        const int64_t blk = ((int64_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
        a.part_loss[2 * blk] = L;
        a.part_loss[2 * blk + 1] = F;
        a.part_used[2 * blk] = U;
        a.part_used[2 * blk + 1] = C;
    }
}

__global__ void k_head_total(const double *pl, const int *pu, int64_t n, float fid_w,
                             double *loss_out, float *inv_n)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double L = 0.0, F = 0.0;
    long long U = 0, C = 0;
    for (int64_t k = 0; k < n; ++k) {
        L += pl[2 * k];
        F += pl[2 * k + 1];
        U += pu[2 * k];
        C += pu[2 * k + 1];
    }
    const double N = U > 0 ? (double)U : 1.0;
    const double NF = C > 0 ? (double)C : 1.0;
    const double Ln = L / N, Lf = F / NF;
    loss_out[0] = Ln + (double)fid_w * Lf;
    loss_out[1] = (double)U;
    loss_out[2] = Ln;
    loss_out[3] = Lf;
    inv_n[0] = (float)(1.0 / N);
    inv_n[1] = (float)(2.0 * (double)fid_w / NF);
}

// dL/dy at pixel j = s * valid_j * [(own_j - sum_d (A_{j+d} d_x + B_{j+d} d_y)) / N
//                                  + 2 w (D~_j - clean_j) / N_f]
__global__ void __launch_bounds__(256)
k_head_bwd(HeadArgs a)
{
    const int gx = blockIdx.x * 64 + (threadIdx.x & 63);
    const int gy = blockIdx.y * 4 + (threadIdx.x >> 6);
    const int b = blockIdx.z;
    const int W = a.W, H = a.H, r = a.rg;
    if (gx >= W || gy >= H) return;
    const int64_t plane = (int64_t)W * H;
    const int64_t base = (int64_t)b * plane;
    float g = 0.0f;
    const float Dc = a.Dt[base + (int64_t)gy * W + gx];
    if (valid_disp(Dc)) {
        float s = a.coefOwn[base + (int64_t)gy * W + gx];
        for (int dy = -r; dy <= r; ++dy) {
            const int yy = gy + dy;
            if (yy < 0 || yy >= H) continue;
            for (int dx = -r; dx <= r; ++dx) {
                const int xx = gx + dx;
                if (xx < 0 || xx >= W || (dx == 0 && dy == 0)) continue;
                const int64_t o = base + (int64_t)yy * W + xx;
                s -= a.coefA[o] * dx + a.coefB[o] * dy;
            }
        }
        float f = 0.0f;
        if (a.clean) {
            const float c = a.clean[base + (int64_t)gy * W + gx];
            if (c - c == 0.0f) f = (Dc - c) * a.inv_n[1];
        }
        g = (s * a.inv_n[0] + f) * a.s;
    }
    a.grad_y[base + (int64_t)gy * W + gx] = g;
}

// ----------------------------------------------------------------------------
// Adam on the flat FP32 parameters, then repacking of the bf16 layouts.
// ----------------------------------------------------------------------------
__global__ void k_adam(float *p, const float *g, float *m, float *v, int n, float lr, float b1,
                       float b2, float eps, float c1, float c2)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// One thread per packed bf16 element; see snx_cnn.hpp for the layouts.
__global__ void k_pack(const float *params, uint16_t *packed)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= kPackedElems) return;
    float w = 0.0f;
    if (i < kPackFwd1 + 32 * 32) {
        // first layer forward: [n 32][slot 32], slot = tap*2 + c
        const int j = i - kPackFwd1, n = j / 32, slot = j % 32;
        if (slot < 18) w = params[kOffW[0] + (n * 2 + slot % 2) * 9 + slot / 2];
    } else if (i < kPackFwdMid + 4 * 9 * 32 * 32) {
        // middle layers forward: [layer][tap][n][k], W[n][k][tap]
        const int j = i - kPackFwdMid, L = j / (9 * 1024), r = j % (9 * 1024);
        const int t = r / 1024, n = (r / 32) % 32, k = r % 32;
        w = params[kOffW[1 + L] + (n * 32 + k) * 9 + t];
    } else if (i < kPackFwd6 + 9 * 16 * 32) {
        // last layer forward: [tap][n 16][k 32], only n = 0
        const int j = i - kPackFwd6, t = j / 512, n = (j / 32) % 16, k = j % 32;
        if (n == 0) w = params[kOffW[5] + k * 9 + t];
    } else if (i < kPackBwdMid + 4 * 9 * 32 * 32) {
        // middle layers backward-data: [layer][tap'][n=ci][k=co] = W[co][ci][8-tap']
        const int j = i - kPackBwdMid, L = j / (9 * 1024), r = j % (9 * 1024);
        const int t = r / 1024, n = (r / 32) % 32, k = r % 32;
        w = params[kOffW[1 + L] + (k * 32 + n) * 9 + (8 - t)];
    } else {
        // last layer backward-data: [n=ci 32][slot 32], slot = tap' -> W6[0][ci][8-tap']
        const int j = i - kPackBwd6, n = j / 32, slot = j % 32;
        if (slot < 9) w = params[kOffW[5] + n * 9 + (8 - slot)];
    }
    packed[i] = to_bf16(w);
}

}  // namespace

int64_t cnn_partial_blocks(int W, int H, int B)
{
    return (int64_t)((W + kT - 1) / kT) * ((H + kT - 1) / kT) * B;
}

int64_t cnn_head_blocks(int W, int H, int B) { return (int64_t)((W + 63) / 64) * ((H + 3) / 4) * B; }

hipError_t cnn_pack(const float *params, uint16_t *packed, hipStream_t s)
{
    hipLaunchKernelGGL(k_pack, dim3((kPackedElems + 255) / 256), dim3(256), 0, s, params, packed);
    return hipGetLastError();
}

hipError_t cnn_forward(const CnnForwardArgs &f, hipStream_t s)
{
    const dim3 grid((f.W + kT - 1) / kT, (f.H + kT - 1) / kT, f.B);
    ConvArgs a = {};
    a.W = f.W;
    a.H = f.H;
    a.D = f.D;
    a.ldD = f.ldD;
    a.crop_stride_D = f.crop_stride_D;
    a.mu = f.mu;
    a.s = kCnnScale;
    // layer 1
    a.wts = f.packed + kPackFwd1;
    a.bias = f.params + kOffB[0];
    a.act_out = f.acts[0];
    hipLaunchKernelGGL(k_conv_small<2>, grid, dim3(256), 0, s, a);
    hipError_t e = hipGetLastError();
    for (int L = 0; L < 4 && e == hipSuccess; ++L) {
        a.act_in = f.acts[L];
        a.act_out = f.acts[L + 1];
        a.wts = f.packed + kPackFwdMid + L * 9 * 1024;
        a.bias = f.params + kOffB[1 + L];
        hipLaunchKernelGGL(k_conv32<0>, grid, dim3(256), 0, s, a);
        e = hipGetLastError();
    }
    if (e != hipSuccess) return e;
    a.act_in = f.acts[4];
    a.wts = f.packed + kPackFwd6;
    a.bias = f.params + kOffB[5];
    a.out = f.out;
    a.ld_out = f.ld_out;
    a.crop_stride_out = f.crop_stride_out;
    hipLaunchKernelGGL(k_conv32<2>, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t cnn_head(const HeadArgs &h, double *loss_out, hipStream_t s)
{
    const dim3 grid((h.W + 63) / 64, (h.H + 3) / 4, h.B);
    hipLaunchKernelGGL(k_head, grid, dim3(256), 0, s, h);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t nblk = (int64_t)grid.x * grid.y * grid.z;
    hipLaunchKernelGGL(k_head_total, dim3(1), dim3(64), 0, s, h.part_loss, h.part_used, nblk,
                       h.fid_w, loss_out, h.inv_n);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_head_bwd, grid, dim3(256), 0, s, h);
    return hipGetLastError();
}

hipError_t cnn_backward(const CnnForwardArgs &f, const float *grad_y, float *partial,
                        float *grad, hipStream_t s)
{
    const dim3 grid((f.W + kT - 1) / kT, (f.H + kT - 1) / kT, f.B);
    const int64_t nblk = (int64_t)grid.x * grid.y * grid.z;
    ConvArgs a = {};
    a.W = f.W;
    a.H = f.H;
    a.D = f.D;
    a.ldD = f.ldD;
    a.crop_stride_D = f.crop_stride_D;
    a.mu = f.mu;
    a.s = kCnnScale;
    hipError_t e;
    // layer 6: dW6 from a5 and dL/dy; dL/da5 via the transposed last layer
    a.act_in = f.acts[4];
    a.grad_in = grad_y;
    hipLaunchKernelGGL((k_wgrad<32, 1>), grid, dim3(256), 0, s, a, partial);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_wgrad_reduce, dim3((kLayerParams[5] + 255) / 256), dim3(256), 0, s,
                       partial, nblk, kLayerParams[5], grad + kOffW[5]);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    a.wts = f.packed + kPackBwd6;
    a.mask_src = f.acts[4];
    a.act_out = f.gbuf[0];
    hipLaunchKernelGGL(k_conv_small<1>, grid, dim3(256), 0, s, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // middle layers 5..2: G_k in gbuf, dW_k from a_{k-1}, then G_{k-1}
    int cur = 0;
    for (int L = 3; L >= 0; --L) {
        a.act_in = f.acts[L];          // input of layer L+2
        a.act_out = f.gbuf[cur];       // its output gradient (read by k_wgrad)
        hipLaunchKernelGGL((k_wgrad<32, 32>), grid, dim3(256), 0, s, a, partial);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL(k_wgrad_reduce, dim3((kLayerParams[1 + L] + 255) / 256), dim3(256), 0,
                           s, partial, nblk, kLayerParams[1 + L], grad + kOffW[1 + L]);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        ConvArgs c = a;
        c.act_in = f.gbuf[cur];
        c.wts = f.packed + kPackBwdMid + L * 9 * 1024;
        c.mask_src = f.acts[L];
        c.act_out = f.gbuf[cur ^ 1];
        hipLaunchKernelGGL(k_conv32<1>, grid, dim3(256), 0, s, c);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        cur ^= 1;
    }
    // layer 1: dW1 from the rebuilt input and G_1
    a.act_out = f.gbuf[cur];
    hipLaunchKernelGGL((k_wgrad<2, 32>), grid, dim3(256), 0, s, a, partial);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_wgrad_reduce, dim3((kLayerParams[0] + 255) / 256), dim3(256), 0, s,
                       partial, nblk, kLayerParams[0], grad + kOffW[0]);
    return hipGetLastError();
}

hipError_t cnn_adam(float *params, const float *grad, float *m, float *v, int step, float lr,
                    float b1, float b2, float eps, uint16_t *packed, hipStream_t s)
{
    const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3((kCnnParams + 255) / 256), dim3(256), 0, s, params, grad, m,
                       v, kCnnParams, lr, b1, b2, eps, c1, c2);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return cnn_pack(params, packed, s);
}

}  // namespace snx
