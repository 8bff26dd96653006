// jatam_tally.hip - histogram of deterministic shapes on the device.
//
// The paper histograms the shape hashes of each slice on the host, sorting
// them while the GPU classifies the next slice (§3.4).  Here the histogram
// stays on the device: an open-addressing table keyed by (hash, size) with
// 64-bit counts.  Each block first counts into a table of its own in LDS
// (a few shapes account for most DET records, so the LDS table absorbs the
// repeats), then adds its non-empty entries to the global table: one global
// atomic per block and distinct shape, never one per record.
#include "jatam_internal.hpp"

namespace jatam {

constexpr int kHistThreads = 256;
constexpr int kHistLocal = 1024;   // LDS entries per block (power of two)

__device__ __forceinline__ uint64_t shape_key(uint32_t hash, int32_t size)
{
    return ((uint64_t)(uint32_t)size << 32) | hash;   // size >= 1: never 0
}

__device__ __forceinline__ uint32_t slot_of(uint64_t key, int log2cap)
{
    return (uint32_t)((key * 0x9E3779B97F4A7C15ull) >> (64 - log2cap));
}

// Adds `count` to the entry of `key` in the global table; false if the table
// has no free entry left.
__device__ __forceinline__ bool global_add(jatam_shape_count_t* table, int log2cap, uint64_t key,
                                           uint64_t count)
{
    const uint32_t mask = (1u << log2cap) - 1u;
    uint32_t s = slot_of(key, log2cap);
    for (uint32_t probe = 0; probe <= mask; ++probe, s = (s + 1) & mask) {
        unsigned long long* kp = reinterpret_cast<unsigned long long*>(&table[s]);
        const unsigned long long seen = atomicCAS(kp, 0ull, (unsigned long long)key);
        if (seen == 0ull || seen == key) {
            atomicAdd(reinterpret_cast<unsigned long long*>(&table[s].count),
                      (unsigned long long)count);
            return true;
        }
    }
    return false;
}

__global__ __launch_bounds__(kHistThreads) void shape_hist_kernel(const jatam_result_t* __restrict__ recs,
                                                                  uint64_t n,
                                                                  jatam_shape_count_t* table,
                                                                  int log2cap, uint64_t* overflow,
                                                                  const uint32_t* slice)
{
    if (slice != nullptr)
        recs += (uint64_t)*slice * n;
    __shared__ unsigned long long keys[kHistLocal];
    __shared__ uint32_t counts[kHistLocal];
    for (int i = threadIdx.x; i < kHistLocal; i += kHistThreads) {
        keys[i] = 0ull;
        counts[i] = 0u;
    }
    __syncthreads();
    constexpr int kLog2Local = 10;
    static_assert((1 << kLog2Local) == kHistLocal, "LDS table size");
    uint64_t lost = 0;
    const uint64_t stride = (uint64_t)gridDim.x * kHistThreads;
    for (uint64_t i = (uint64_t)blockIdx.x * kHistThreads + threadIdx.x; i < n; i += stride) {
        const jatam_result_t r = recs[i];
        if (r.cls != JATAM_DET)
            continue;
        const uint64_t key = shape_key(r.hash, r.size);
        uint32_t s = slot_of(key, kLog2Local);
        bool placed = false;
        for (int probe = 0; probe < kHistLocal; ++probe, s = (s + 1) & (kHistLocal - 1)) {
            const unsigned long long seen = atomicCAS(&keys[s], 0ull, (unsigned long long)key);
            if (seen == 0ull || seen == key) {
                atomicAdd(&counts[s], 1u);
                placed = true;
                break;
            }
        }
        // a full LDS table (more than kHistLocal shapes in one block) goes
        // straight to the global table
        if (!placed && !global_add(table, log2cap, key, 1))
            ++lost;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kHistLocal; i += kHistThreads) {
        if (counts[i] != 0u && !global_add(table, log2cap, keys[i], counts[i]))
            lost += counts[i];
    }
    if (overflow != nullptr && lost != 0)
        atomicAdd(reinterpret_cast<unsigned long long*>(overflow), (unsigned long long)lost);
}

int launch_shape_hist(const jatam_result_t* recs, uint64_t n, jatam_shape_count_t* table,
                      int log2cap, uint64_t* overflow, int cus, const uint32_t* slice,
                      hipStream_t stream)
{
    if (n == 0)
        return JATAM_OK;
    // enough blocks to stream the records at full bandwidth, few enough that
    // the flush stays a small number of global atomics per shape
    const uint64_t want = (n + kHistThreads * 64 - 1) / (kHistThreads * 64);
    const uint64_t cap = (uint64_t)(cus > 0 ? cus : 256) * 4;
    const uint32_t blocks = (uint32_t)(want < cap ? want : cap);
    hipLaunchKernelGGL(shape_hist_kernel, dim3(blocks), dim3(kHistThreads), 0, stream, recs, n,
                       table, log2cap, overflow, slice);
    return hipGetLastError() == hipSuccess ? JATAM_OK : JATAM_E_HIP;
}

}  // namespace jatam
