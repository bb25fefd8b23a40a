// Internal declarations shared by the HIP translation units of libsnx.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "snx.h"

namespace snx {

// A disparity sample is valid iff finite and > 0.  Inside the kernels invalid
// samples are stored as 0.0f, so "valid" reduces to "> 0".
__host__ __device__ inline bool valid_disp(float d) { return d > 0.0f && d < INFINITY; }

// XCD-aware tile order.  The dispatcher hands workgroup b of a launch to XCD
// b % 8 (eight XCDs, each with its own L2); tile indices are assigned so that
// the workgroups of one XCD cover one contiguous band of the n tiles (row-major
// over the frame), and a tile's halo is mostly in the L2 its neighbours filled.
constexpr int kXcds = 8;
__device__ inline int xcd_tile(int b, int n)
{
    const int x = b % kXcds, j = b / kXcds;
    const int per = n / kXcds, rem = n % kXcds;
    return x * per + (x < rem ? x : rem) + j;
}

// Output tile of the stencil kernel: TW columns (one wave's lanes) x th rows.
constexpr int kTileW = 64;
constexpr int kBlock = 256;
constexpr int kMaxWindow = 63;

struct StencilArgs {
    const float *src;      // raw disparity (rf > 0) or denoised disparity (rf == 0)
    int64_t ld_src;
    int W, H;
    int rf, rg;            // filter and gradient radii (0 = stage off)
    int need_f, need_g;    // support thresholds
    float fx, fy, b, u0, v0;
    float *dn;             // denoised plane out (nullable)
    int64_t ld_dn;
    float *aff;            // a1, a2 planes (nullable)
    float *nrm;            // nx, ny, nz planes (nullable)
    int64_t ld_out, plane_out;
    int32_t *forest;       // nullable: label forest (W*H, linear indices) to resolve
    int32_t *labels;       // nullable: final labels (input, or output when forest)
    int64_t ld_lab;
    int32_t *count;        // nullable: roots are counted while resolving a forest
    snx_point *rec;        // nullable
    int th;                // tile height
};

size_t stencil_lds_bytes(int rf, int rg, int th);
int stencil_pick_tile_height(int rf, int rg);
bool stencil_has_instance(int rf, int rg, int th);
hipError_t launch_stencil(const StencilArgs &a, hipStream_t s);
// autotuned tile height for (rf, rg) at this frame size, 0 if not tuned
int tuned_tile_height(int rf, int rg, int W, int H);
// pin (th > 0, a compiled candidate) or clear (th == 0) the entry for this size class
bool set_tile_height(int rf, int rg, int W, int H, int th);
hipError_t autotune_stencil(int rf, int rg, int need_f, int need_g, int W, int H, hipStream_t s,
                            int *chosen);

// Compacted point cloud (compact.hip): the defined records in raster order.
int64_t compact_chunks(int64_t n);
// chunk_count: compact_chunks(n) entries of device scratch
hipError_t launch_compact(const snx_point *in, int64_t n, snx_point *out, int32_t *count,
                          int32_t *chunk_count, hipStream_t s);
// Allocation-free variant: the largest record count it takes, and this device's
// chunk counts in the library's static device array.
int64_t compact_noalloc_max_records();
hipError_t compact_noalloc_scratch(int32_t **chunk_count);

// Component-restricted gradient window (restricted.hip): the n_g window keeps
// only the valid pixels whose label equals the centre's.
struct RestrictArgs {
    const float *src;      // denoised disparity
    int64_t ld_src;
    const int32_t *labels; // component labels (-1 = none)
    int64_t ld_lab;
    int W, H, r, need_g;
    float fx, fy, u0, v0;
    float *aff, *nrm;      // nullable planes
    int64_t ld_out, plane_out;
};
size_t restrict_lds_bytes(int r);
hipError_t launch_affine_labels(const RestrictArgs &a, hipStream_t s);

// Adaptive star-fill support (Sec. 3.4): rays in 4 or 8 compass directions,
// covered-depth or depth-Laplacian stopping, slope, A and normal (star.hip).
constexpr int kStopCD = 0, kStopST = 1;
struct StarArgs {
    const float *src;      // denoised disparity
    int64_t ld_src;
    int W, H;
    int dirs, steps, stop, need_g;
    double thr;            // k of the CD rule, or t of the ST rule
    double fxb;            // f_x * baseline (ST)
    float fx, fy, u0, v0;
    float *aff, *nrm;      // nullable planes
    int64_t ld_out, plane_out;
};
size_t star_lds_bytes(int steps, int stop);
hipError_t launch_star(const StarArgs &a, hipStream_t s);

// Front of the pipeline: local components forest of each 64 x 32 tile plus the
// filter (window 1 or 3) of the same tile, from one read of the raw disparity.
struct FrontArgs {
    const float *D;
    int64_t ld;
    int W, H;
    double k_rel, t_abs;
    int rf, need_f;
    float *dn;             // nullable: filtered plane out
    int64_t ld_dn;
    int32_t *forest;       // W*H contiguous
    int32_t *count;        // nullable: zeroed here
    const float *nrm = nullptr;   // crease-aware components: normal planes (else NULL)
    int64_t ld_nrm = 0, plane_nrm = 0;
    double crease_cos = 0.0;
    const uint8_t *edges = nullptr;   // explicitly given edge graph (test hook), else NULL
    int64_t ld_edges = 0;
    // Seam records (3x3-filter front only; else NULL), merge_pairs(W, H) entries
    // each in the merge's pair order: seam_a[i] = the tile root of the pair's
    // left/upper pixel where the pair needs a union (an edge not implied by the
    // previous pair), else -1; seam_b[i] = the tile root of its right/lower pixel.
    int32_t *seam_a = nullptr, *seam_b = nullptr;
};
hipError_t launch_front(const FrontArgs &a, hipStream_t s);
hipError_t launch_merge_seams(const int32_t *seam_a, const int32_t *seam_b, int64_t pairs,
                              int32_t *forest, hipStream_t s);
hipError_t launch_merge(const float *D, int64_t ld, int W, int H, double k_rel, double t_abs,
                        int32_t *forest, hipStream_t s, const float *nrm = nullptr,
                        int64_t ld_nrm = 0, int64_t plane_nrm = 0, double crease_cos = 0.0);

// One frame of a batch plan: the arguments of its front (filter + forest, and
// the seam merge) and back (gradients, normals, labels, records) stages.
struct BatchFrame {
    FrontArgs front;
    StencilArgs back;
};
int front_tiles(int W, int H);
int64_t merge_pairs(int W, int H);
hipError_t launch_batch_front(const BatchFrame *frames, const int *tile_off, const int *tile_frame,
                              int n, int rf, int *counter, int grid, hipStream_t s);
// seam_a/seam_b: the batch's seam records (every frame's front writes them at
// seam_off[f]), or NULL for the merge that decides the pairs itself.
hipError_t launch_batch_merge(const BatchFrame *frames, const int64_t *seam_off,
                              const int *block_frame, int n, int64_t total, hipStream_t s,
                              const int32_t *seam_a = nullptr, const int32_t *seam_b = nullptr);
hipError_t launch_batch_back(const BatchFrame *frames, const int *tile_off, const int *tile_frame,
                             int n, int rg, int th, int *counter, int grid, hipStream_t s);
hipError_t launch_batch_reset(int *counters, int n_counters, const BatchFrame *frames, int n,
                              hipStream_t s);
int back_tiles(int W, int H, int th);
bool batch_has_instance(int rg, int th);

struct CclArgs {
    const float *D;
    int64_t ld;
    int W, H;
    double k_rel, t_abs;
    int32_t *parent;       // W*H contiguous union-find array
    int32_t *labels;       // output (may equal parent when ld_lab == W)
    int64_t ld_lab;
    int32_t *count;        // nullable
    const float *nrm = nullptr;   // crease-aware components: normal planes (else NULL)
    int64_t ld_nrm = 0, plane_nrm = 0;
    double crease_cos = 0.0;
    const uint8_t *edges = nullptr;   // explicitly given edge graph (test hook; D unused,
                                      // ld = its row stride), else NULL
};
hipError_t launch_components(const CclArgs &a, hipStream_t s);

struct CloudArgs {
    const float *dn;
    int64_t ld_dn;
    const float *nrm;
    int64_t ld_nrm, plane_nrm;
    const int32_t *labels;
    int64_t ld_lab;
    int W, H;
    float fx, fy, b, u0, v0;
    snx_point *out;
};
hipError_t launch_point_cloud(const CloudArgs &a, hipStream_t s);

hipError_t launch_fill_i32(int32_t *p, int32_t value, int64_t n, hipStream_t s);

// Point record from the denoised disparity and the normal (shared by the fused
// stencil epilogue and the separate point-cloud kernel so both agree bitwise).
__device__ inline snx_point make_point(int u, int v, float D, float nx, float ny,
                                       float nz, int32_t label, float fx, float fy,
                                       float b, float u0, float v0)
{
    snx_point p;
    const bool def = valid_disp(D) && (nx == nx);
    if (def) {
        // reciprocals (about 1 ulp each) instead of IEEE divisions: the record
        // is a few ulp from the correctly rounded quotients
        const float z = (fx * b) * __builtin_amdgcn_rcpf(D);
        p.x = ((float)u - u0) * z * __builtin_amdgcn_rcpf(fx);
        p.y = ((float)v - v0) * z * __builtin_amdgcn_rcpf(fy);
        p.z = z;
        p.nx = nx; p.ny = ny; p.nz = nz;
    } else {
        p.x = p.y = p.z = p.nx = p.ny = p.nz = __builtin_nanf("");
    }
    p.label = label;
    p.flags = (def ? SNX_POINT_DEFINED : 0u) | (label >= 0 ? SNX_POINT_LABELLED : 0u);
    return p;
}

typedef float v4f __attribute__((ext_vector_type(4)));

// Streaming 2 x 16-byte store of one record (records are written once, never
// re-read by the path).
__device__ inline void store_point(snx_point *dst, const snx_point &p)
{
    const v4f lo = {p.x, p.y, p.z, p.nx};
    const v4f hi = {p.ny, p.nz, __int_as_float(p.label), __uint_as_float(p.flags)};
    v4f *d4 = reinterpret_cast<v4f *>(dst);
    __builtin_nontemporal_store(lo, d4);
    __builtin_nontemporal_store(hi, d4 + 1);
}

}  // namespace snx
