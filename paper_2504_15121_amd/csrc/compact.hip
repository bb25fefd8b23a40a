// Compacted oriented point cloud: the records whose normal is defined
// (SNX_POINT_DEFINED), packed contiguously in raster order, and their count.
//
// Three kernels, no inter-workgroup waiting: (1) each workgroup counts the
// defined records of its 4096-record chunk; (2) one workgroup turns the chunk
// counts into exclusive offsets (and the total); (3) each workgroup writes its
// chunk's defined records from its offset, ranks within a wave from a ballot,
// wave offsets through LDS, so the output order is the input order.
#include <atomic>
#include <mutex>

#include "snx_internal.hpp"

// Scratch of the allocation-free compaction (snx_compact_points_noalloc): the
// chunk counts in the first half, the chunk offsets in the second.  Every kernel
// writes each entry it later reads, so nothing needs clearing between calls.
// Host code must not pass this name to a kernel (on the host it is only a
// stand-in): the per-device address comes from hipGetSymbolAddress below.
constexpr int64_t kNoAllocChunks = 8192;
static __device__ __align__(256) int32_t scratch[2 * kNoAllocChunks];

namespace snx {
namespace {

constexpr int kCpThreads = 256;
constexpr int kCpRounds = 16;
constexpr int kCpChunk = kCpThreads * kCpRounds;   // records per workgroup
constexpr int kScanThreads = 1024;

__device__ __forceinline__ bool defined_at(const snx_point *p, int64_t i, int64_t n)
{
    return i < n && (p[i].flags & SNX_POINT_DEFINED) != 0u;
}

__global__ void __launch_bounds__(kCpThreads)
k_compact_count(const snx_point *in, int64_t n, int32_t *chunk_count)
{
    __shared__ int s_sum;
    if (threadIdx.x == 0) s_sum = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kCpChunk;
    int c = 0;
#pragma unroll
    for (int j = 0; j < kCpRounds; ++j) c += defined_at(in, base + j * kCpThreads + threadIdx.x, n) ? 1 : 0;
    // wave sum, then one LDS atomic per wave
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
    if ((threadIdx.x & 63) == 0) atomicAdd(&s_sum, c);
    __syncthreads();
    if (threadIdx.x == 0) chunk_count[blockIdx.x] = s_sum;
}

// Exclusive prefix sums of nchunks counts (one workgroup, 1024 at a time).
__global__ void __launch_bounds__(kScanThreads)
k_compact_scan(const int32_t *chunk_count, int nchunks, int32_t *chunk_off, int32_t *total)
{
    __shared__ int s_wave[kScanThreads / 64];
    __shared__ int s_carry;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid == 0) s_carry = 0;
    __syncthreads();
    for (int b = 0; b < nchunks; b += kScanThreads) {
        const int i = b + tid;
        const int v = i < nchunks ? chunk_count[i] : 0;
        int x = v;                                    // inclusive scan within the wave
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(x, o);
            if (lane >= o) x += y;
        }
        if (lane == 63) s_wave[wave] = x;
        __syncthreads();
        int wbase = 0;
        for (int w = 0; w < wave; ++w) wbase += s_wave[w];
        const int carry = s_carry;
        if (i < nchunks) chunk_off[i] = carry + wbase + x - v;
        __syncthreads();
        if (tid == kScanThreads - 1) s_carry = carry + wbase + x;
        __syncthreads();
    }
    if (tid == 0) *total = s_carry;
}

__global__ void __launch_bounds__(kCpThreads)
k_compact_scatter(const snx_point *in, int64_t n, const int32_t *chunk_off, snx_point *out)
{
    __shared__ int s_wave[kCpThreads / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t base = (int64_t)blockIdx.x * kCpChunk;
    int off = chunk_off[blockIdx.x];
    for (int j = 0; j < kCpRounds; ++j) {
        const int64_t i = base + j * kCpThreads + tid;
        const bool d = defined_at(in, i, n);
        const unsigned long long bal = __ballot(d);
        const int rank = __popcll(bal & ((1ull << lane) - 1ull));
        if (lane == 0) s_wave[wave] = __popcll(bal);
        __syncthreads();
        int wbase = 0, all = 0;
#pragma unroll
        for (int w = 0; w < kCpThreads / 64; ++w) {
            const int c = s_wave[w];
            wbase += w < wave ? c : 0;
            all += c;
        }
        if (d) store_point(out + off + wbase + rank, in[i]);
        off += all;
        __syncthreads();
    }
}

}  // namespace

int64_t compact_chunks(int64_t n) { return (n + kCpChunk - 1) / kCpChunk; }

int64_t compact_noalloc_max_records() { return kNoAllocChunks * kCpChunk; }

namespace {
constexpr int kMaxDevices = 64;
std::atomic<int32_t *> g_scratch[kMaxDevices];
std::mutex g_scratch_mu;
}  // namespace

hipError_t compact_noalloc_scratch(int32_t **chunk_count, int32_t **chunk_off)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    int32_t *p = g_scratch[dev].load(std::memory_order_acquire);
    if (!p) {
        // first call on this device (which is current): look up this device's
        // copy of the array once and keep its address
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        p = g_scratch[dev].load(std::memory_order_relaxed);
        if (!p) {
            void *addr = nullptr;
            if ((e = hipGetSymbolAddress(&addr, HIP_SYMBOL(scratch))) != hipSuccess) return e;
            if (!addr) return hipErrorInvalidSymbol;
            p = static_cast<int32_t *>(addr);
            g_scratch[dev].store(p, std::memory_order_release);
        }
    }
    *chunk_count = p;
    *chunk_off = p + kNoAllocChunks;
    return hipSuccess;
}

hipError_t launch_compact(const snx_point *in, int64_t n, snx_point *out, int32_t *count,
                          int32_t *chunk_count, int32_t *chunk_off, hipStream_t s)
{
    const int64_t nc = compact_chunks(n);
    hipLaunchKernelGGL(k_compact_count, dim3((unsigned)nc), dim3(kCpThreads), 0, s, in, n,
                       chunk_count);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_compact_scan, dim3(1), dim3(kScanThreads), 0, s, chunk_count, (int)nc,
                       chunk_off, count);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_compact_scatter, dim3((unsigned)nc), dim3(kCpThreads), 0, s, in, n,
                       chunk_off, out);
    return hipGetLastError();
}

}  // namespace snx
