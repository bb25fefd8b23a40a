// Dense oriented point cloud from a denoised disparity, normal planes and labels:
// back-projection through the rectified pair of Sec. 2 (z = f_x b / D,
// x = (u - u0) z / f_x, y = (v - v0) z / f_y), one 32-byte record per pixel.
#include "snx_internal.hpp"

namespace snx {
namespace {

__global__ void __launch_bounds__(256)
k_point_cloud(CloudArgs a)
{
    const int gx = blockIdx.x * 64 + (threadIdx.x & 63);
    const int gy = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (gx >= a.W || gy >= a.H) return;
    const float d = a.dn[(int64_t)gy * a.ld_dn + gx];
    const int64_t o = (int64_t)gy * a.ld_nrm + gx;
    const float nx = a.nrm[o], ny = a.nrm[o + a.plane_nrm], nz = a.nrm[o + 2 * a.plane_nrm];
    const int32_t lab = a.labels ? a.labels[(int64_t)gy * a.ld_lab + gx] : -1;
    const snx_point p = make_point(gx, gy, valid_disp(d) ? d : 0.0f, nx, ny, nz, lab,
                                   a.fx, a.fy, a.b, a.u0, a.v0);
    store_point(a.out + (int64_t)gy * a.W + gx, p);
}

}  // namespace

hipError_t launch_point_cloud(const CloudArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_point_cloud, dim3((a.W + 63) / 64, (a.H + 3) / 4), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace snx
