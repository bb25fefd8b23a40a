// Learned denoiser inference with all six convolutions fused in one kernel.
//
// A workgroup owns a 24 x 24 output tile at a time and keeps every
// intermediate activation in LDS: layer k's output is computed on the region
// the remaining layers need (34, 32, 30, 28, 26 pixels square for layers 1..5,
// 24 for layer 6), so nothing but the disparity, the LSQ filter mu and D~
// touches HBM.  Region pixels outside the image are set to zero after every
// layer, which is the zero padding of each convolution.
//
// The kernel is persistent (one 512-thread workgroup per CU walks the tiles)
// and pipelined: each layer's weights are copied once per workgroup from
// global memory into LDS (fetched into registers during the previous layer,
// stored once every wave has taken the previous layer's weights into its
// registers), and the next tile's disparity and mu are fetched into registers
// during the current tile's last layers.  LDS bandwidth is the limit of this
// kernel, which is why the tile is as large as the 160 KB allow.
//
// MFMA orientation (v_mfma_f32_16x16x32_bf16): A = weights (16 output channels
// x 32 inputs), B = activations (32 inputs x 16 pixels), so that a lane's four
// results are four consecutive output channels of one pixel.  The 16 pixels of
// a B operand are 16 consecutive pixels of the row-major output region.
// Activations are NHWC bf16, 32 channels in 64 bytes a pixel, with the four
// 16-byte channel chunks of pixel p stored at chunk c ^ ((p >> 1) & 3), so the
// 8 lanes served together by a 16-byte LDS read (8 consecutive pixels, one
// chunk) hit 8 distinct bank groups; weight rows are swizzled the same way.
//
// Per output: the same MFMA over the taps in the same order as the
// layer-by-layer kernels, with the bias as the accumulator's initial value
// (they add it to the finished FP32 sum), then ReLU and bf16 RNE.
#include <stdint.h>

#include "device.hpp"
#include "snx_cnn.hpp"

namespace snx {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef short s16x2 __attribute__((ext_vector_type(2)));

constexpr int kFT = 24;                 // output tile edge
constexpr int kRA = kFT + 10;           // largest region held in buffer A (layer 1 output)
constexpr int kRB = kFT + 8;            // largest region held in buffer B (layer 2 output)
constexpr int kRF = kFT + 12;           // feature region (layer 1 input)
constexpr int kWaves = 8;               // waves per workgroup
constexpr int kThreads = kWaves * 64;

// One layer's weights in LDS: up to 9 x 32 rows of 32 bf16 (64 bytes), then
// 32 float biases.
constexpr int kWRows = 9 * 32;
constexpr int kWBias = kWRows * 64;                     // 18432
constexpr int kWBuf = kWBias + 32 * 4;                  // 18560
constexpr int kLdsA = 0;
constexpr int kLdsB = kLdsA + kRA * kRA * 64;           // 73984
constexpr int kLdsW = kLdsB + kRB * kRB * 64;           // 139520
constexpr int kLdsMu = kLdsW + kWBuf;                   // mu of the output tile (float)
constexpr size_t kFusedLds = kLdsMu + kFT * kFT * 4;    // 160384 bytes

// feature pixels per thread (36 x 36 region over 512 threads)
constexpr int kFeatPer = (kRF * kRF + kThreads - 1) / kThreads;   // 3

__device__ __forceinline__ uint16_t bf16_rne(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// two floats -> packed bf16 pair (round to nearest even), low = first
__device__ __forceinline__ uint32_t pack_bf16(float lo, float hi)
{
    const f32x2 v = {lo, hi};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2));
}

__device__ __forceinline__ f32x4 mfma(u32x4 a, u32x4 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                   __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

// Byte offset of 16-byte chunk c of weight row p.
__device__ __forceinline__ int chunk_off(int p, int c) { return p * 64 + ((c ^ ((p >> 1) & 3)) << 4); }

__device__ __forceinline__ u32x4 lds16(const unsigned char *base, int p, int c)
{
    return *reinterpret_cast<const u32x4 *>(base + chunk_off(p, c));
}

// Activations swizzle by the pixel's column x instead: chunk c of a pixel in
// column x sits at slot c ^ ((x >> 1) & 3).  Any 8 horizontally consecutive
// pixels then cover the 8 bank groups whatever the row pitch, and a lane that
// walks down a column keeps one swizzle, so its addresses differ by whole rows
// (immediate offsets).
__device__ __forceinline__ int act_slot(int x, int c) { return (c ^ ((x >> 1) & 3)) << 4; }

// ---------------------------------------------------------------------------
// Weight staging.  Stage s = 1..6 is layer s.  Its packed weights are
// contiguous rows of 32 bf16 (64 bytes): 32 rows (layer 1), 9 x 32 (layers
// 2..5), 9 x 16 (layer 6).  Thread t holds 16-byte chunks t, t + 512, t + 1024
// of the rows in registers until they are written to LDS; threads 0..7 also
// carry the bias (one float for layer 6).
// ---------------------------------------------------------------------------
struct StageRegs {
    u32x4 c[3];
    u32x4 bias;
};

__device__ __forceinline__ int stage_rows(int s) { return s == 1 ? 32 : (s == 6 ? 144 : 288); }

__device__ __forceinline__ void stage_fetch(const CnnFusedArgs &a, int s, int tid, StageRegs &r)
{
    const uint16_t *src = s == 1 ? a.packed + kPackFwd1
                        : s == 6 ? a.packed + kPackFwd6
                                 : a.packed + kPackFwdMid + (s - 2) * 9 * 1024;
    const int nchunks = stage_rows(s) * 4;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int c = tid + k * kThreads;
        if (c < nchunks) r.c[k] = *reinterpret_cast<const u32x4 *>(src + c * 8);
    }
    if (s < 6) {
        if (tid < 8) r.bias = *reinterpret_cast<const u32x4 *>(a.params + kOffB[s - 1] + tid * 4);
    } else if (tid == 0) {
        r.bias = (u32x4){__float_as_uint(a.params[kOffB[5]]), 0u, 0u, 0u};
    }
}

__device__ __forceinline__ void stage_store(unsigned char *wbuf, int s, int tid, const StageRegs &r)
{
    const int nchunks = stage_rows(s) * 4;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int c = tid + k * kThreads;
        if (c < nchunks) *reinterpret_cast<u32x4 *>(wbuf + chunk_off(c >> 2, c & 3)) = r.c[k];
    }
    if ((s < 6 && tid < 8) || (s == 6 && tid == 0))
        *reinterpret_cast<u32x4 *>(wbuf + kWBias + tid * 16) = r.bias;
}

// bl[mb][j] = bias of output channel mb * 16 + 4q + j: the accumulator's initial
// value in the MFMA layout.
__device__ __forceinline__ void load_bias(const unsigned char *wbuf, int q, f32x4 (&bl)[2])
{
    const float *b = reinterpret_cast<const float *>(wbuf + kWBias);
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int j = 0; j < 4; ++j) bl[mb][j] = b[mb * 16 + 4 * q + j];
}

// ---------------------------------------------------------------------------
// bf16, ReLU, zero outside the image, and store of one lane's results (bias
// already in the sums): output channels 4q..4q+3 (block 0) and 16+4q..16+4q+3
// (block 1) of a pixel.  px: the pixel's 64 bytes; o0 / o1: byte offsets of the
// two 8-byte halves (act_offsets).  ReLU is a signed 16-bit max with 0 on the
// packed bf16 pair: rounding to bf16 keeps the sign, so this equals rounding
// the ReLU of the FP32 value.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void act_offsets(int x, int q, int &o0, int &o1)
{
    // channels 4q.. sit in chunk q/2 (half q&1); channels 16+4q.. in chunk 2 + q/2
    o0 = act_slot(x, q >> 1) + ((q & 1) << 3);
    o1 = act_slot(x, 2 + (q >> 1)) + ((q & 1) << 3);
}

__device__ __forceinline__ uint32_t relu_bf16x2(uint32_t w)
{
    const s16x2 v = __builtin_bit_cast(s16x2, w);
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(v, (s16x2){0, 0}));
}

__device__ __forceinline__ void store_act(unsigned char *px, int o0, int o1, bool inside,
                                          const f32x4 &a0, const f32x4 &a1)
{
    uint32_t w[4];
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
        const f32x4 &a = mb ? a1 : a0;
        w[2 * mb] = inside ? relu_bf16x2(pack_bf16(a[0], a[1])) : 0u;
        w[2 * mb + 1] = inside ? relu_bf16x2(pack_bf16(a[2], a[3])) : 0u;
    }
    *reinterpret_cast<uint2 *>(px + o0) = make_uint2(w[0], w[1]);
    *reinterpret_cast<uint2 *>(px + o1) = make_uint2(w[2], w[3]);
}

// Strip decomposition of an output region of even edge RO in [16, 32] for the
// 8 waves: two 16-column segments (at 0 and at RO - 16, overlapping when
// RO < 32; the overlap is computed twice and written twice with the same
// values), each split into four runs of consecutive row pairs.  A wave walks
// its run downwards, keeping the input rows it still needs in registers, so
// each output row costs three 16-byte LDS reads per lane (the new input row at
// dx = -1, 0, +1) instead of nine.  Waves w and w + 4 share a SIMD; the second
// segment takes its runs in reverse order so that a long run and a short run
// share a SIMD whenever the pairs do not divide evenly.
template <int RO>
__device__ __forceinline__ void strip_of(int wave, int &xs, int &r0, int &r1)
{
    static_assert(RO % 2 == 0 && RO >= 16 && RO <= 32, "strip layout");
    constexpr int kPairs = RO / 2, kBase = kPairs / 4, kExtra = kPairs % 4;
    const int seg = wave >> 2;
    const int part = seg == 0 ? (wave & 3) : 3 - (wave & 3);
    const int p0 = part * kBase + (part < kExtra ? part : kExtra);
    const int np = kBase + (part < kExtra ? 1 : 0);
    xs = seg == 0 ? 0 : RO - 16;
    r0 = 2 * p0;
    r1 = 2 * (p0 + np);
}

// One 32 -> 32 layer from region RIN (`in`) to region RIN - 2 (`out`) with the
// weights already in registers.  (ox, oy): image coordinates of the output
// region's first pixel.  A step computes two output rows (four accumulator
// chains) from input rows 2s .. 2s + 3 of the wave's run (F[row][dx]); the
// steps are unrolled and software-pipelined: step s's MFMAs are issued in the
// same block as step s - 1's bias, ReLU, packing and stores, so the matrix
// core and the vector ALU of a wave work at the same time.
template <int RIN>
__device__ __forceinline__ void mid_layer(const unsigned char *in, unsigned char *out,
                                          const u32x4 (&wa)[9][2], const f32x4 (&bs)[2],
                                          int ox, int oy, int W, int H, int lane, int wave)
{
    constexpr int RO = RIN - 2, kSteps = (RO / 2 + 3) / 4;
    const int q = lane >> 4, col = lane & 15;
    int xs, r0, r1;
    strip_of<RO>(wave, xs, r0, r1);
    const bool full = r1 - r0 == 2 * kSteps;      // else the run has kSteps - 1 steps
    const int x = xs + col;                        // output column; input columns x .. x + 2
    const unsigned char *src[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) src[d] = in + (r0 * RIN + x + d) * 64 + act_slot(x + d, q);
    unsigned char *dst = out + (r0 * RO + x) * 64;
    int o0, o1;
    act_offsets(x, q, o0, o1);
    const int gx = ox + x, gy0 = oy + r0;
    const bool col_in = gx >= 0 && gx < W;

    u32x4 F[2 * kSteps + 2][3];
    f32x4 acc[kSteps][2][2];
    auto load_row = [&](int j) {
#pragma unroll
        for (int d = 0; d < 3; ++d) F[j][d] = *reinterpret_cast<const u32x4 *>(src[d] + j * RIN * 64);
    };
    auto compute = [&](int st) {
        load_row(2 * st + 2);
        load_row(2 * st + 3);
#pragma unroll
        for (int k = 0; k < 2; ++k)
#pragma unroll
            for (int mb = 0; mb < 2; ++mb) acc[st][k][mb] = bs[mb];
#pragma unroll
        for (int t = 0; t < 9; ++t)
#pragma unroll
            for (int mb = 0; mb < 2; ++mb)
#pragma unroll
                for (int k = 0; k < 2; ++k)
                    acc[st][k][mb] = mfma(wa[t][mb], F[2 * st + k + t / 3][t % 3], acc[st][k][mb]);
    };
    auto finish = [&](int st) {
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const bool inside = col_in && (unsigned)(gy0 + 2 * st + k) < (unsigned)H;
            store_act(dst + (2 * st + k) * RO * 64, o0, o1, inside, acc[st][k][0], acc[st][k][1]);
        }
    };
    load_row(0);
    load_row(1);
    compute(0);
#pragma unroll
    for (int st = 1; st < kSteps - 1; ++st) {
        compute(st);
        finish(st - 1);
    }
    if (full) {
        compute(kSteps - 1);
        finish(kSteps - 2);
        finish(kSteps - 1);
    } else {
        finish(kSteps - 2);
    }
}

__device__ __forceinline__ void load_mid_weights(const unsigned char *wbuf, int q, int col,
                                                 u32x4 (&wa)[9][2], f32x4 (&bs)[2])
{
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int mb = 0; mb < 2; ++mb) wa[t][mb] = lds16(wbuf, t * 32 + mb * 16 + col, q);
    load_bias(wbuf, q, bs);
}

// Disparity and mu of the feature pixels this thread builds, for tile (tx, ty).
struct FeatRegs {
    float d[kFeatPer], mu[kFeatPer];
};

__device__ __forceinline__ void feat_fetch(const CnnFusedArgs &a, int tx, int ty, int tid, FeatRegs &f)
{
#pragma unroll
    for (int k = 0; k < kFeatPer; ++k) {
        const int p = tid + k * kThreads;
        const int ly = p / kRF, lx = p - ly * kRF;
        const int gy = ty * kFT - 6 + ly, gx = tx * kFT - 6 + lx;
        f.d[k] = 0.0f;
        f.mu[k] = 0.0f;
        if (p < kRF * kRF && gy >= 0 && gy < a.H && gx >= 0 && gx < a.W) {
            f.d[k] = a.D[(int64_t)gy * a.ldD + gx];
            f.mu[k] = a.mu[(int64_t)gy * a.W + gx];
        }
    }
}

// Item `item` of the work: a tile of the single frame `a0`, or (BATCH) a tile of
// frame tile_frame[item] of `frames`.  The item and frame index are uniform
// across the workgroup, so the arguments come from scalar loads.
template <bool BATCH>
__device__ __forceinline__ void decode_item(const CnnFusedArgs &a0, const CnnFusedArgs *frames,
                                            const int *tile_off, const int *tile_frame, int item,
                                            CnnFusedArgs &A, int &tx, int &ty)
{
    int local = item;
    if (BATCH) {
        const int f = __builtin_amdgcn_readfirstlane(tile_frame[__builtin_amdgcn_readfirstlane(item)]);
        A = frames[f];
        local = item - tile_off[f];
    } else {
        A = a0;
    }
    const int ntx = (A.W + kFT - 1) / kFT;
    ty = local / ntx;
    tx = local - ty * ntx;
}

template <bool BATCH>
__global__ void __launch_bounds__(kThreads)
k_cnn_fused(CnnFusedArgs a, const CnnFusedArgs *frames, const int *tile_off, const int *tile_frame,
            int n)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    unsigned char *bufA = smem + kLdsA;
    unsigned char *bufB = smem + kLdsB;
    unsigned char *wbuf = smem + kLdsW;
    const int tid = threadIdx.x, lane0 = tid & 63, wave0 = tid >> 6;
    const int ntiles = BATCH ? tile_off[n]
                             : ((a.W + kFT - 1) / kFT) * ((a.H + kFT - 1) / kFT);

    int tile = blockIdx.x;
    if (tile >= ntiles) return;
    CnnFusedArgs A;
    int tx, ty;
    decode_item<BATCH>(a, frames, tile_off, tile_frame, tile, A, tx, ty);
    FeatRegs f;
    feat_fetch(A, tx, ty, tid, f);
    // Weight stages: the stage stored at a layer's start is fetched into
    // registers one layer earlier, at the previous layer's start.
    StageRegs r;
    stage_fetch(a, 1, tid, r);
    stage_store(wbuf, 1, tid, r);
    stage_fetch(a, 2, tid, r);

    u32x4 wa[9][2];
    f32x4 bs[2];
    while (true) {
        // Lane and wave indices redefined per tile: this keeps the compiler from
        // hoisting every layer's strip addresses out of the tile loop, which
        // would hold them in (spilled) registers for the whole kernel.
        int lane = lane0, wave = wave0;
        asm volatile("" : "+v"(lane), "+v"(wave));
        const int q = lane >> 4, col = lane & 15;
        const int W = A.W, H = A.H;
        const int x0 = tx * kFT, y0 = ty * kFT;
        // ---- features over the 36 x 36 region at (x0-6, y0-6): (x0 bf16, valid bf16);
        // mu of the 24 x 24 output pixels goes to its own LDS array for layer 6
        uint32_t *feat = reinterpret_cast<uint32_t *>(bufB);
        float *s_mu = reinterpret_cast<float *>(smem + kLdsMu);
#pragma unroll
        for (int k = 0; k < kFeatPer; ++k) {
            const int p = tid + k * kThreads;
            if (p < kRF * kRF) {
                uint32_t v = 0;
                if (valid_disp(f.d[k])) v = (uint32_t)bf16_rne((f.d[k] - f.mu[k]) / A.s) | (0x3f80u << 16);
                feat[p] = v;
                const int ly = p / kRF - 6, lx = p % kRF - 6;
                if ((unsigned)ly < (unsigned)kFT && (unsigned)lx < (unsigned)kFT) s_mu[ly * kFT + lx] = f.mu[k];
            }
        }
        __syncthreads();                                  // features and layer-1 weights ready

        // ---- layer 1: 2 -> 32, K slots = tap * 2 + channel (18 used)
        {
            u32x4 w1[2];
#pragma unroll
            for (int mb = 0; mb < 2; ++mb) w1[mb] = lds16(wbuf, mb * 16 + col, q);
            load_bias(wbuf, q, bs);
            __syncthreads();                              // every wave holds layer 1's weights
            stage_store(wbuf, 2, tid, r);
            stage_fetch(a, 3, tid, r);
            __syncthreads();                              // layer-2 weights in LDS
            // groups of 16 consecutive region pixels, group g to wave g % 8, taken
            // kL1Batch at a time so that their feature reads are in flight together
            constexpr int RO = kRA, NP = RO * RO, NG = (NP + 15) / 16;
            constexpr int kL1Batch = 5, kL1Iter = (NG + kWaves - 1) / kWaves;
            static_assert(kL1Iter % kL1Batch == 0, "layer-1 batching");
            // this lane's K slots 8q .. 8q+7 are taps 4q .. 4q+3 (x0, valid pairs);
            // slots past tap 8 read the pixel's own tap 0 and are zeroed
            int toff[4];
            bool tuse[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int t = 4 * q + i;
                tuse[i] = t < 9;
                toff[i] = tuse[i] ? (t / 3) * kRF + t % 3 : 0;
            }
#pragma unroll 1
            for (int j0 = 0; j0 < kL1Iter; j0 += kL1Batch) {
                u32x4 bv[kL1Batch];
#pragma unroll
                for (int b = 0; b < kL1Batch; ++b) {
                    const int p = (wave + kWaves * (j0 + b)) * 16 + col;
                    const int pc = p < NP ? p : NP - 1;
                    const int y = pc / RO;
                    const int base = pc + (kRF - RO) * y;          // feature index of tap 0
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const uint32_t v = feat[base + toff[i]];
                        bv[b][i] = tuse[i] ? v : 0u;
                    }
                }
#pragma unroll
                for (int b = 0; b < kL1Batch; ++b) {
                    const f32x4 a0 = mfma(w1[0], bv[b], bs[0]), a1 = mfma(w1[1], bv[b], bs[1]);
                    const int p = (wave + kWaves * (j0 + b)) * 16 + col;
                    if (p < NP) {
                        const int y = p / RO, x = p - y * RO;
                        const int gx = x0 - 5 + x, gy = y0 - 5 + y;
                        int o0, o1;
                        act_offsets(x, q, o0, o1);
                        store_act(bufA + p * 64, o0, o1, gx >= 0 && gx < W && gy >= 0 && gy < H, a0, a1);
                    }
                }
            }
        }
        // Each wave takes the next layer's weights from LDS as soon as its own
        // part of a layer is done; the barrier after that marks both the layer's
        // output and every wave's weights ready, the stage store that follows
        // refills the weight buffer, and one more barrier publishes it.
        load_mid_weights(wbuf, q, col, wa, bs);
        __syncthreads();                                  // layer 1 out, layer-2 weights taken
        stage_store(wbuf, 3, tid, r);
        stage_fetch(a, 4, tid, r);
        __syncthreads();
        mid_layer<kRA>(bufA, bufB, wa, bs, x0 - 4, y0 - 4, W, H, lane, wave);
        load_mid_weights(wbuf, q, col, wa, bs);
        __syncthreads();
        stage_store(wbuf, 4, tid, r);
        stage_fetch(a, 5, tid, r);
        __syncthreads();
        mid_layer<kRB>(bufB, bufA, wa, bs, x0 - 3, y0 - 3, W, H, lane, wave);
        load_mid_weights(wbuf, q, col, wa, bs);
        __syncthreads();
        stage_store(wbuf, 5, tid, r);
        stage_fetch(a, 6, tid, r);
        __syncthreads();
        mid_layer<kRB - 2>(bufA, bufB, wa, bs, x0 - 2, y0 - 2, W, H, lane, wave);
        load_mid_weights(wbuf, q, col, wa, bs);
        __syncthreads();
        stage_store(wbuf, 6, tid, r);
        stage_fetch(a, 1, tid, r);
        const int next = tile + gridDim.x;
        CnnFusedArgs An;
        int ntx_, nty_;
        if (next < ntiles) {
            decode_item<BATCH>(a, frames, tile_off, tile_frame, next, An, ntx_, nty_);
            feat_fetch(An, ntx_, nty_, tid, f);
        }
        __syncthreads();
        mid_layer<kRB - 4>(bufB, bufA, wa, bs, x0 - 1, y0 - 1, W, H, lane, wave);

        // ---- layer 6: 32 -> 1 on the 24 x 24 tile, strips as in the middle layers
        {
            constexpr int RIN = kFT + 2, RO = kFT;
            u32x4 w6[9];
#pragma unroll
            for (int t = 0; t < 9; ++t) w6[t] = lds16(wbuf, t * 16 + col, q);
            const float b6 = reinterpret_cast<const float *>(wbuf + kWBias)[0];
            __syncthreads();                              // layer 5 out, layer-6 weights taken
            stage_store(wbuf, 1, tid, r);                 // read after the next two barriers
            stage_fetch(a, 2, tid, r);
            // three steps of two rows for every wave, pipelined as in mid_layer
            static_assert(RO / 2 == 4 * 3, "layer-6 strip runs");
            int xs, r0, r1;
            strip_of<RO>(wave, xs, r0, r1);
            const int x = xs + col;
            const unsigned char *src[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) src[d] = bufA + (r0 * RIN + x + d) * 64 + act_slot(x + d, q);
            const int gx = x0 + x;
            const bool col_in = q == 0 && gx < W;       // output channel 0: lanes q == 0, element 0
            u32x4 F[8][3];
            f32x4 acc[3][2];
            auto load_row = [&](int j) {
#pragma unroll
                for (int d = 0; d < 3; ++d) F[j][d] = *reinterpret_cast<const u32x4 *>(src[d] + j * RIN * 64);
            };
            auto compute = [&](int st) {
                load_row(2 * st + 2);
                load_row(2 * st + 3);
                acc[st][0] = (f32x4){b6, b6, b6, b6};
                acc[st][1] = (f32x4){b6, b6, b6, b6};
#pragma unroll
                for (int t = 0; t < 9; ++t)
#pragma unroll
                    for (int k = 0; k < 2; ++k) acc[st][k] = mfma(w6[t], F[2 * st + k + t / 3][t % 3], acc[st][k]);
            };
            auto finish = [&](int st) {
#pragma unroll
                for (int k = 0; k < 2; ++k) {
                    const int ly = r0 + 2 * st + k, gy = y0 + ly;
                    if (col_in && gy < H) {
                        const float mu = s_mu[ly * kFT + x];
                        const float yv = acc[st][k][0];
                        A.out[(int64_t)gy * A.ld_out + gx] = (mu == mu) ? mu + A.s * yv : __builtin_nanf("");
                    }
                }
            };
            load_row(0);
            load_row(1);
            compute(0);
            compute(1);
            finish(0);
            compute(2);
            finish(1);
            finish(2);
        }
        __syncthreads();
        if (next >= ntiles) break;
        tile = next;
        A = An;
        tx = ntx_;
        ty = nty_;
    }
}

}  // namespace

hipError_t cnn_forward_fused(const CnnFusedArgs &f, hipStream_t s)
{
    const int ntiles = cnn_fused_tiles(f.W, f.H);
    int cus = 0;
    hipError_t e = device_cus(&cus);
    if (e != hipSuccess) return e;
    const int grid = ntiles < cus ? ntiles : cus;
    hipLaunchKernelGGL(k_cnn_fused<false>, dim3(grid), dim3(kThreads), kFusedLds, s, f,
                       (const CnnFusedArgs *)nullptr, (const int *)nullptr, (const int *)nullptr, 0);
    return hipGetLastError();
}

int cnn_fused_tiles(int W, int H) { return ((W + kFT - 1) / kFT) * ((H + kFT - 1) / kFT); }

hipError_t cnn_forward_fused_batch(const CnnFusedArgs &common, const CnnFusedArgs *frames,
                                   const int *tile_off, const int *tile_frame, int n, int total,
                                   hipStream_t s)
{
    int cus = 0;
    hipError_t e = device_cus(&cus);
    if (e != hipSuccess) return e;
    const int grid = total < cus ? total : cus;
    if (grid < 1) return hipSuccess;
    hipLaunchKernelGGL(k_cnn_fused<true>, dim3(grid), dim3(kThreads), kFusedLds, s, common, frames,
                       tile_off, tile_frame, n);
    return hipGetLastError();
}

}  // namespace snx
