// Compacted oriented point cloud: the records whose normal is defined
// (SNX_POINT_DEFINED), packed contiguously in raster order, and their count.
//
// Two kernels, no inter-workgroup waiting: (1) each workgroup counts the
// defined records of its chunk of 4096; (2) each workgroup sums the counts of
// the chunks before its own (a few KB, read from L2 by every workgroup, with
// its first record loads already in flight) and then writes its chunk's
// defined records from that offset in 16 rounds, each round's records placed
// while the next round's loads are in flight: ranks within a wave from a
// ballot, wave offsets through LDS, so the output order is the input order.
// The last chunk writes the total.
#include <atomic>
#include <mutex>

#include "snx_internal.hpp"

// Scratch of the allocation-free compaction (snx_compact_points_noalloc): the
// chunk counts.  The count kernel writes every entry the scatter kernel reads,
// so nothing needs clearing between calls.  Host code must not pass this name
// to a kernel (on the host it is only a stand-in): the per-device address comes
// from hipGetSymbolAddress below.
constexpr int64_t kNoAllocChunks = 8192;
static __device__ __align__(256) int32_t scratch[kNoAllocChunks];

namespace snx {
namespace {

constexpr int kCpChunk = 4096;                       // records per chunk
constexpr int kCountThreads = 512;                   // count kernel: 8 records a thread
constexpr int kScatterThreads = 256;                 // scatter kernel: 16 rounds of 256
constexpr int kMaxWaves = kCountThreads / 64;

typedef unsigned v4u __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned wave_sum(unsigned v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Sum over a workgroup of NW waves of one value per thread (every thread gets
// it).
template <int NW>
__device__ __forceinline__ unsigned block_sum(unsigned v, unsigned *s_part)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    v = wave_sum(v);
    if (lane == 0) s_part[wave] = v;
    __syncthreads();
    unsigned t = lane < NW ? s_part[lane] : 0u;
#pragma unroll
    for (int o = 1; o < NW; o <<= 1) t += __shfl_xor(t, o);
    return __builtin_amdgcn_readfirstlane(t);
}

__global__ void __launch_bounds__(kCountThreads)
k_compact_count(const snx_point *in, int64_t n, int32_t *chunk_count)
{
    constexpr int kPer = kCpChunk / kCountThreads;
    __shared__ unsigned s_part[kMaxWaves];
    const int tid = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * kCpChunk;
    const v4u *in4 = reinterpret_cast<const v4u *>(in);
    // the upper half of each record (its flags), every load issued before the
    // first wait; indices past the end read the last record again and are not
    // counted.  Cached loads: the records then stay in the memory-side cache
    // for the scatter kernel's second read
    v4u hi[kPer];
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const int64_t i = base + j * kCountThreads + tid, ic = i < n ? i : n - 1;
        hi[j] = in4[2 * ic + 1];
    }
    unsigned c = 0;
#pragma unroll
    for (int j = 0; j < kPer; ++j)
        c += base + j * kCountThreads + tid < n && (hi[j].w & SNX_POINT_DEFINED) != 0u ? 1u : 0u;
    c = block_sum<kCountThreads / 64>(c, s_part);
    if (tid == 0) chunk_count[blockIdx.x] = (int32_t)c;
}

__global__ void __launch_bounds__(kScatterThreads)
k_compact_scatter(const snx_point *in, int64_t n, const int32_t *chunk_count, int nc,
                  snx_point *out, int32_t *count)
{
    constexpr int kWaves = kScatterThreads / 64, kRounds = kCpChunk / kScatterThreads;
    __shared__ unsigned s_part[kWaves];
    __shared__ int s_wave[2][kWaves];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int c = blockIdx.x;
    const int64_t base = (int64_t)c * kCpChunk;
    const v4u *in4 = reinterpret_cast<const v4u *>(in);
    // record of round j for this thread; indices past the end read the last
    // record again and count as not defined
    auto load = [&](int j, v4u &lo, v4u &hi) {
        const int64_t i = base + j * kScatterThreads + tid, ic = i < n ? i : n - 1;
        lo = in4[2 * ic];
        hi = in4[2 * ic + 1];
    };
    // this chunk's offset: the counts of every earlier chunk, the first four
    // per thread loaded ahead of round 0's records (which stay in flight
    // meanwhile), any further ones after them
    constexpr int kAhead = 4;
    unsigned q[kAhead];
#pragma unroll
    for (int t = 0; t < kAhead; ++t) {
        const int k = tid + t * kScatterThreads;
        q[t] = k < c ? (unsigned)chunk_count[k] : 0u;
    }
    v4u lo, hi;
    load(0, lo, hi);
    unsigned p = 0;
#pragma unroll
    for (int t = 0; t < kAhead; ++t) p += q[t];
    for (int k = tid + kAhead * kScatterThreads; k < c; k += kScatterThreads)
        p += (unsigned)chunk_count[k];
    unsigned off = block_sum<kWaves>(p, s_part);
    const unsigned long long below = (1ull << lane) - 1ull;
#pragma unroll
    for (int j = 0; j < kRounds; ++j) {
        // the next round's record in flight while this one is placed
        v4u nlo = lo, nhi = hi;
        if (j + 1 < kRounds) load(j + 1, nlo, nhi);
        const bool d = base + j * kScatterThreads + tid < n && (hi.w & SNX_POINT_DEFINED) != 0u;
        const unsigned long long bal = __ballot(d);
        // wave counts double-buffered in LDS: one barrier a round
        if (lane == 0) s_wave[j & 1][wave] = __popcll(bal);
        __syncthreads();
        unsigned before = 0, all = 0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) {
            const unsigned cw = (unsigned)s_wave[j & 1][w];
            before += w < wave ? cw : 0u;
            all += cw;
        }
        if (d) {
            v4u *dst = reinterpret_cast<v4u *>(out + off + before + __popcll(bal & below));
            __builtin_nontemporal_store(lo, dst);
            __builtin_nontemporal_store(hi, dst + 1);
        }
        off += all;
        lo = nlo;
        hi = nhi;
    }
    if (c == nc - 1 && tid == 0) *count = (int32_t)off;
}

}  // namespace

int64_t compact_chunks(int64_t n) { return (n + kCpChunk - 1) / kCpChunk; }

int64_t compact_noalloc_max_records() { return kNoAllocChunks * kCpChunk; }

namespace {
constexpr int kMaxDevices = 64;
std::atomic<int32_t *> g_scratch[kMaxDevices];
std::mutex g_scratch_mu;
}  // namespace

hipError_t compact_noalloc_scratch(int32_t **chunk_count)
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
    return hipSuccess;
}

hipError_t launch_compact(const snx_point *in, int64_t n, snx_point *out, int32_t *count,
                          int32_t *chunk_count, hipStream_t s)
{
    const int64_t nc = compact_chunks(n);
    if (nc <= 0 || nc >= (1LL << 31)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_compact_count, dim3((unsigned)nc), dim3(kCountThreads), 0, s, in, n,
                       chunk_count);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_compact_scatter, dim3((unsigned)nc), dim3(kScatterThreads), 0, s, in,
                       n, chunk_count, (int)nc, out, count);
    return hipGetLastError();
}

}  // namespace snx
