// Layouts and arguments of the learned-denoiser kernels (cnn.hip).
#pragma once

#include <stdint.h>

#include "snx_internal.hpp"

namespace snx {

// Flat FP32 parameters, in layer order: W_k as [Cout][Cin][3][3], then b_k.
//   layer 1: 2 -> 32, layers 2..5: 32 -> 32, layer 6: 32 -> 1
constexpr int kLayerParams[6] = {32 * 2 * 9 + 32, 32 * 32 * 9 + 32, 32 * 32 * 9 + 32,
                                 32 * 32 * 9 + 32, 32 * 32 * 9 + 32, 1 * 32 * 9 + 1};
constexpr int kOffW[6] = {0, 608, 608 + 9248, 608 + 2 * 9248, 608 + 3 * 9248, 608 + 4 * 9248};
constexpr int kOffB[6] = {576, 608 + 9216, 608 + 9248 + 9216, 608 + 2 * 9248 + 9216,
                          608 + 3 * 9248 + 9216, 608 + 4 * 9248 + 288};
constexpr int kCnnParams = 608 + 4 * 9248 + 289;   // 37889

// Packed bf16 weights (one buffer), segments:
//   kPackFwd1   first layer forward  [n 32][slot 32], slot = tap*2 + c (18 used)
//   kPackFwdMid layers 2..5 forward  [layer][tap][n 32][k 32]
//   kPackFwd6   last layer forward   [tap][n 16][k 32], only n = 0 non-zero
//   kPackBwdMid layers 2..5 backward-data [layer][tap'][n = ci][k = co],
//               = W[co][ci][8 - tap'] (flipped taps, transposed channels)
//   kPackBwd6   last layer backward-data [n = ci 32][slot 32] = W6[0][ci][8 - slot]
constexpr int kPackFwd1 = 0;
constexpr int kPackFwdMid = 1024;
constexpr int kPackFwd6 = kPackFwdMid + 4 * 9 * 1024;
constexpr int kPackBwdMid = kPackFwd6 + 9 * 16 * 32;
constexpr int kPackBwd6 = kPackBwdMid + 4 * 9 * 1024;
constexpr int kPackedElems = kPackBwd6 + 1024;

constexpr float kCnnScale = 1.0f;   // disparity scale of the network input/output (px)

struct CnnCam {
    float fx, fy, u0, v0;
};

struct ConvArgs {
    int W, H;
    const float *D;            // raw disparity (first layer / weight gradient of layer 1)
    int64_t ldD, crop_stride_D;
    const float *mu;           // LSQ filter, B x H x W contiguous
    const uint16_t *act_in;    // NHWC32 bf16, B x H x W x 32
    const float *grad_in;      // dL/dy, B x H x W (last layer backward)
    const uint16_t *wts;
    const float *bias;
    const uint16_t *mask_src;  // backward-data: ReLU mask source
    uint16_t *act_out;         // NHWC32 bf16 (also: output gradient read by k_wgrad)
    float *out;                // last layer: denoised disparity
    int64_t ld_out, crop_stride_out;
    float s;
};

constexpr int kCnnMaxBatch = 64;

struct HeadArgs {
    int W, H, B, rg, need_g;
    const float *Dt;           // B x H x W denoised disparity
    const float *n_gt;         // B x 3 x H x W ground-truth normals (NaN = none)
    CnnCam cams[kCnnMaxBatch]; // passed by value with the launch
    const float *clean;        // B x H x W noise-free disparity (NaN = none), or null
    float fid_w;               // weight of the fidelity term
    float *coefA, *coefB, *coefOwn;   // B x H x W
    double *part_loss;         // per workgroup: sum of 1 - n.g, sum of (D~ - clean)^2
    int *part_used;            // per workgroup: normal pixels, fidelity pixels
    float *inv_n;              // device: 1/N (normal term), 2 w / N_f (fidelity term)
    float *grad_y;             // B x H x W dL/dy
    float s;
};

struct CnnForwardArgs {
    int W, H, B;
    const float *D;
    int64_t ldD, crop_stride_D;
    const float *mu;
    const float *params;
    const uint16_t *packed;
    uint16_t *acts[5];         // a_1 .. a_5, each B x H x W x 32 bf16
    uint16_t *gbuf[2];         // gradient ping-pong, same shape
    float *out;
    int64_t ld_out, crop_stride_out;
};

// Inference with all six layers fused per 16 x 16 tile (one frame).
struct CnnFusedArgs {
    int W, H;
    const float *D;            // raw disparity, row stride ldD
    int64_t ldD;
    const float *mu;           // LSQ filter, H x W contiguous
    const float *params;
    const uint16_t *packed;
    float *out;                // D~, row stride ld_out
    int64_t ld_out;
    float s;
};

hipError_t cnn_pack(const float *params, uint16_t *packed, hipStream_t s);
hipError_t cnn_forward_fused(const CnnFusedArgs &f, hipStream_t s);
// Number of tiles of the fused kernel for a W x H frame.
int cnn_fused_tiles(int W, int H);
// The fused network over the tiles of many frames in one persistent launch:
// frames = device array of per-frame arguments; item i is tile
// i - tile_off[f] of frame f = tile_frame[i]; `common` carries the params and
// packed weights (the same for every frame).
hipError_t cnn_forward_fused_batch(const CnnFusedArgs &common, const CnnFusedArgs *frames,
                                   const int *tile_off, const int *tile_frame, int n, int total,
                                   hipStream_t s);
hipError_t cnn_forward(const CnnForwardArgs &f, hipStream_t s);
hipError_t cnn_head(const HeadArgs &h, double *loss_out, hipStream_t s);
hipError_t cnn_backward(const CnnForwardArgs &f, const float *grad_y, float *partial,
                        float *grad, hipStream_t s);
hipError_t cnn_adam(float *params, const float *grad, float *m, float *v, int step, float lr,
                    float b1, float b2, float eps, uint16_t *packed, hipStream_t s);
// number of weight-gradient partial blocks for a batch (partial buffer holds
// cnn_partial_blocks * max layer parameter count floats)
int64_t cnn_partial_blocks(int W, int H, int B);
int64_t cnn_head_blocks(int W, int H, int B);

}  // namespace snx
