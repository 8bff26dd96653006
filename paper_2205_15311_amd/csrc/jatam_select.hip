// jatam_select.hip - deterministic top-k selection on the device.
//
// Keeps the k of n candidates with the highest score, ties going to the
// lower index, and lists the kept indices in ascending order.  Scores become
// 32-bit keys whose ascending order is descending score (NaN last); a radix
// select over 4 digits of 8 bits finds the k-th key D; keys below D are kept,
// and of the keys equal to D the first (k - #below) by index.  Index order
// comes from exclusive scans, so nothing depends on thread timing.  No host
// synchronisation: every pass reads the previous pass's state from device
// memory.
#include "jatam_internal.hpp"

namespace jatam {

// Ascending key order == descending score order; NaN sorts after everything.
__device__ __forceinline__ uint32_t score_key(float f)
{
    const uint32_t u = __float_as_uint(f);
    if ((u & 0x7FFFFFFFu) > 0x7F800000u)
        return 0xFFFFFFFFu;
    const uint32_t ascending = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
    return ~ascending;
}

// state: [0] prefix of D found so far, [1] how many keys still to take below
// the prefix (k minus keys already known to be smaller), [2..257] histogram
__global__ __launch_bounds__(256) void select_init_kernel(uint32_t* state, uint32_t k)
{
    for (int i = threadIdx.x; i < kSelectState; i += 256)
        state[i] = 0;
    __syncthreads();
    if (threadIdx.x == 0)
        state[1] = k;
}

__global__ __launch_bounds__(256) void select_hist_kernel(const float* __restrict__ score,
                                                          uint32_t n, uint32_t* state, int pass)
{
    __shared__ uint32_t hist[256];
    hist[threadIdx.x] = 0;
    __syncthreads();
    const int shift = 24 - 8 * pass;
    const uint32_t prefix = state[0];
    const uint32_t pmask = pass == 0 ? 0u : 0xFFFFFFFFu << (32 - 8 * pass);
    for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
        const uint32_t key = score_key(score[i]);
        if ((key & pmask) == prefix)
            atomicAdd(&hist[(key >> shift) & 0xFFu], 1u);
    }
    __syncthreads();
    if (hist[threadIdx.x] != 0)
        atomicAdd(&state[2 + threadIdx.x], hist[threadIdx.x]);
}

// Picks the digit whose bin holds the need-th key; clears the histogram.
__global__ void select_pick_kernel(uint32_t* state, int pass)
{
    if (threadIdx.x != 0)
        return;
    uint32_t need = state[1], digit = 255;
    for (uint32_t d = 0; d < 256; ++d) {
        const uint32_t c = state[2 + d];
        if (need <= c) {
            digit = d;
            break;
        }
        need -= c;
    }
    state[0] |= digit << (24 - 8 * pass);
    state[1] = need;
    for (int d = 0; d < 256; ++d)
        state[2 + d] = 0;
}

// flag[i]: 1 if key < D, 2 if key == D, else 0.
__global__ __launch_bounds__(256) void select_flag_kernel(const float* __restrict__ score,
                                                          uint32_t n, const uint32_t* state,
                                                          uint32_t* flag)
{
    const uint32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n)
        return;
    const uint32_t key = score_key(score[i]), D = state[0];
    flag[i] = key < D ? 1u : key == D ? 2u : 0u;
}

// Block-level exclusive scan of pred(flag) in place into out; block totals
// into sums.  pred: mode 0 -> flag == 2, mode 1 -> flag != 0 (kept).
__device__ __forceinline__ uint32_t select_pred(uint32_t f, int mode, uint32_t rank_eq,
                                                uint32_t need)
{
    if (mode == 0)
        return f == 2u;
    return f == 1u || (f == 2u && rank_eq < need);
}

__global__ __launch_bounds__(1024) void select_scan_block_kernel(const uint32_t* flag,
                                                                 const uint32_t* rank_eq,
                                                                 const uint32_t* state,
                                                                 uint32_t n, int mode,
                                                                 uint32_t* out, uint32_t* sums)
{
    __shared__ uint32_t part[1024];
    const uint32_t i = blockIdx.x * 1024 + threadIdx.x;
    const uint32_t need = state[1];
    const uint32_t v = i < n ? select_pred(flag[i], mode, mode ? rank_eq[i] : 0u, need) : 0u;
    part[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const uint32_t add = (int)threadIdx.x >= off ? part[threadIdx.x - off] : 0u;
        __syncthreads();
        part[threadIdx.x] += add;
        __syncthreads();
    }
    if (i < n)
        out[i] = part[threadIdx.x] - v;
    if (threadIdx.x == 1023)
        sums[blockIdx.x] = part[1023];
}

// Exclusive scan of the block totals (one block, loops over them).
__global__ __launch_bounds__(1024) void select_scan_sums_kernel(uint32_t* sums, uint32_t nblocks)
{
    __shared__ uint32_t part[1024];
    const uint32_t per = (nblocks + 1023) / 1024;
    const uint32_t lo = threadIdx.x * per, hi = min(nblocks, lo + per);
    uint32_t s = 0;
    for (uint32_t b = lo; b < hi; ++b)
        s += sums[b];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const uint32_t add = (int)threadIdx.x >= off ? part[threadIdx.x - off] : 0u;
        __syncthreads();
        part[threadIdx.x] += add;
        __syncthreads();
    }
    uint32_t run = part[threadIdx.x] - s;
    for (uint32_t b = lo; b < hi; ++b) {
        const uint32_t v = sums[b];
        sums[b] = run;
        run += v;
    }
}

__global__ __launch_bounds__(1024) void select_scan_add_kernel(uint32_t* out, const uint32_t* sums,
                                                               uint32_t n)
{
    const uint32_t i = blockIdx.x * 1024 + threadIdx.x;
    if (i < n)
        out[i] += sums[blockIdx.x];
}

// Writes kept indices at their ranks (ascending index order).
__global__ __launch_bounds__(256) void select_compact_kernel(const uint32_t* flag,
                                                             const uint32_t* rank_eq,
                                                             const uint32_t* pos,
                                                             const uint32_t* state, uint32_t n,
                                                             uint32_t* out_idx)
{
    const uint32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n)
        return;
    if (select_pred(flag[i], 1, rank_eq[i], state[1]))
        out_idx[pos[i]] = i;
}

static void exclusive_scan(const SelectWork& w, uint32_t n, int mode, uint32_t* out,
                           hipStream_t s)
{
    const uint32_t nb = (n + 1023) / 1024;
    hipLaunchKernelGGL(select_scan_block_kernel, dim3(nb), dim3(1024), 0, s, w.flag, w.rank_eq,
                       w.state, n, mode, out, w.sums);
    hipLaunchKernelGGL(select_scan_sums_kernel, dim3(1), dim3(1024), 0, s, w.sums, nb);
    hipLaunchKernelGGL(select_scan_add_kernel, dim3(nb), dim3(1024), 0, s, out, w.sums, n);
}

int launch_select_top(const float* scores, uint32_t n, uint32_t k, uint32_t* out_idx,
                      const SelectWork& w, hipStream_t s)
{
    if (k == 0 || n == 0)
        return JATAM_OK;
    const uint32_t grid = min((n + 255) / 256, 1024u);
    hipLaunchKernelGGL(select_init_kernel, dim3(1), dim3(256), 0, s, w.state, k);
    for (int pass = 0; pass < 4; ++pass) {
        hipLaunchKernelGGL(select_hist_kernel, dim3(grid), dim3(256), 0, s, scores, n, w.state,
                           pass);
        hipLaunchKernelGGL(select_pick_kernel, dim3(1), dim3(64), 0, s, w.state, pass);
    }
    hipLaunchKernelGGL(select_flag_kernel, dim3((n + 255) / 256), dim3(256), 0, s, scores, n,
                       w.state, w.flag);
    exclusive_scan(w, n, 0, w.rank_eq, s);   // rank of each key == D among equals
    exclusive_scan(w, n, 1, w.pos, s);       // output position of each kept index
    hipLaunchKernelGGL(select_compact_kernel, dim3((n + 255) / 256), dim3(256), 0, s, w.flag,
                       w.rank_eq, w.pos, w.state, n, out_idx);
    return hipGetLastError() == hipSuccess ? JATAM_OK : JATAM_E_HIP;
}

// ---------------------------------------------------------------------------
// Queue order by predicted cost: a counting sort of n scores into 256
// buckets, highest cost first.  Blocks of kOrderBlock items histogram their
// buckets (bucket-major: entry b * nblocks + block), one exclusive scan of
// the histogram gives every (bucket, block) its first queue position, and
// each block scatters its items from there with LDS cursors.  Items of one
// bucket keep no particular order among themselves (the classification's
// records never depend on the queue order).
// ---------------------------------------------------------------------------
constexpr uint32_t kOrderBlock = 4096;

// Bucket of a score (expected DET size P(DET) e^pred - 1, at least -1):
// 16 log2(score + 2) clamped to 0..255, reversed so that high costs come
// first; NaN last.
__device__ __forceinline__ uint32_t cost_bucket(float score)
{
    if (!(score == score))
        return 255u;
    const float v = 16.f * __log2f(fmaxf(score, -1.f) + 2.f);
    const uint32_t q = v < 0.f ? 0u : v > 255.f ? 255u : (uint32_t)v;
    return 255u - q;
}

__global__ __launch_bounds__(256) void order_hist_kernel(const float* __restrict__ scores,
                                                         uint32_t n, uint32_t* hist)
{
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t lo = blockIdx.x * kOrderBlock, hi = min(n, lo + kOrderBlock);
    for (uint32_t i = lo + threadIdx.x; i < hi; i += 256)
        atomicAdd(&h[cost_bucket(scores[i])], 1u);
    __syncthreads();
    hist[threadIdx.x * gridDim.x + blockIdx.x] = h[threadIdx.x];
}

// In-place exclusive scan of m words, in three passes (per-1024 blocks,
// their totals, the block offsets added back).
__global__ __launch_bounds__(1024) void order_scan_block_kernel(uint32_t* x, uint32_t m,
                                                                uint32_t* sums)
{
    __shared__ uint32_t part[1024];
    const uint32_t i = blockIdx.x * 1024 + threadIdx.x;
    const uint32_t v = i < m ? x[i] : 0u;
    part[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const uint32_t add = (int)threadIdx.x >= off ? part[threadIdx.x - off] : 0u;
        __syncthreads();
        part[threadIdx.x] += add;
        __syncthreads();
    }
    if (i < m)
        x[i] = part[threadIdx.x] - v;
    if (threadIdx.x == 1023)
        sums[blockIdx.x] = part[1023];
}

__global__ __launch_bounds__(1024) void order_scan_add_kernel(uint32_t* x, const uint32_t* sums,
                                                              uint32_t m)
{
    const uint32_t i = blockIdx.x * 1024 + threadIdx.x;
    if (i < m)
        x[i] += sums[blockIdx.x];
}

__global__ __launch_bounds__(256) void order_scatter_kernel(const float* __restrict__ scores,
                                                            uint32_t n, const uint32_t* hist,
                                                            uint32_t* order)
{
    __shared__ uint32_t cursor[256];
    cursor[threadIdx.x] = hist[threadIdx.x * gridDim.x + blockIdx.x];
    __syncthreads();
    const uint32_t lo = blockIdx.x * kOrderBlock, hi = min(n, lo + kOrderBlock);
    for (uint32_t i = lo + threadIdx.x; i < hi; i += 256)
        order[atomicAdd(&cursor[cost_bucket(scores[i])], 1u)] = i;
}

uint64_t order_work_words(uint64_t n)
{
    const uint64_t m = 256 * ((n + kOrderBlock - 1) / kOrderBlock);
    return m + (m + 1023) / 1024 + 1;
}

int launch_order_by_cost(const float* scores, uint32_t n, uint32_t* order, uint32_t* work,
                         hipStream_t s)
{
    if (n == 0)
        return JATAM_OK;
    const uint32_t nb = (n + kOrderBlock - 1) / kOrderBlock;
    const uint32_t m = 256 * nb;
    uint32_t* hist = work;
    uint32_t* sums = work + m;
    const uint32_t sb = (m + 1023) / 1024;
    hipLaunchKernelGGL(order_hist_kernel, dim3(nb), dim3(256), 0, s, scores, n, hist);
    hipLaunchKernelGGL(order_scan_block_kernel, dim3(sb), dim3(1024), 0, s, hist, m, sums);
    // the block totals: at most 1024 of them for n up to 2^24 items, more in
    // a second level
    if (sb > 1) {
        hipLaunchKernelGGL(select_scan_sums_kernel, dim3(1), dim3(1024), 0, s, sums, sb);
        hipLaunchKernelGGL(order_scan_add_kernel, dim3(sb), dim3(1024), 0, s, hist, sums, m);
    }
    hipLaunchKernelGGL(order_scatter_kernel, dim3(nb), dim3(256), 0, s, scores, n, hist, order);
    return hipGetLastError() == hipSuccess ? JATAM_OK : JATAM_E_HIP;
}

}  // namespace jatam
