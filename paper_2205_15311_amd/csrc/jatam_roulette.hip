// jatam_roulette.hip - the paper's own genetic algorithm: global roulette
// wheel selection (§2.2, §3.1, App. C.1), single-point crossover (App. D.2)
// and Poisson-distributed bit-flip mutation (App. D.1); and the Fujiyama test
// bed (§4.2) with every simulation evolving inside one workgroup.
//
// Roulette: the wheel's areas are the running sums of the fitness (the
// paper's separate summation kernel gives its total); a dart
// d = floor(u S / 2^32) picks the first genome whose running sum exceeds d,
// found by binary search over the sums; with S = 0 a genome is drawn
// uniformly.  Crossover point p = floor(u L / 2^32): bit-string positions
// 0..p-1 (the high bits of the L-bit genome) come from the second parent.
// Mutation: k flips with k Poisson(lambda) (the first j with u < T_j, T_j =
// floor(2^32 P(k <= j)) from the host's double-precision recurrence), at
// most L, at k distinct positions drawn floor(u L / 2^32), a repeat drawn
// again, at most 1024 position draws.  Offspring i of generation g reads the
// Philox4x32-10 stream keyed by the GA seed at counter (i, g, block, 4 << 28),
// word q being word q % 4 of block q / 4: 0 parent a, 1 parent b, 2 the
// point, 3 the flip count, 4.. the positions.
//
// Fujiyama: fitness = Hamming weight; each simulation starts from the
// all-zero population, one workgroup per simulation with one lane per
// genome, the population, its running fitness sums and the next population
// in LDS, the generation loop inside the kernel (the paper synchronises all
// threads after every generation; here that is a workgroup barrier).
#include <math.h>

#include "jatam_device.hpp"
#include "jatam_internal.hpp"

namespace jatam {

// Threshold T_j is below u exactly when T_j >= 1 and u <= T_j - 1 (T_j takes
// 33 bits: 0 .. 2^32).
__device__ __forceinline__ bool below_threshold(const PoissonTable& t, int j, uint32_t u)
{
    return ((t.zero >> j) & 1ull) == 0ull && u <= t.tm1[j];
}

// Sequential reader of one offspring's words.
struct RouletteStream {
    uint32_t k0, k1, i, gen;
    uint32_t block;
    Words4 words;

    __device__ __forceinline__ uint32_t word(uint32_t q)
    {
        const uint32_t b = q >> 2;
        if (b != block) {
            words = philox4x32_10(i, gen, b, 4u << 28, k0, k1);
            block = b;
        }
        const uint32_t k = q & 3u;
        uint32_t u = words.w[0];
        u = k == 1u ? words.w[1] : u;
        u = k == 2u ? words.w[2] : u;
        u = k == 3u ? words.w[3] : u;
        return u;
    }
};

__device__ __forceinline__ uint32_t scale32(uint32_t u, uint32_t n)
{
    return (uint32_t)(((uint64_t)u * (uint64_t)n) >> 32);
}

// First index whose running sum (sums[i] = f_0 + .. + f_i) exceeds the dart,
// by binary search; uniform when the total is 0.
template <class Sums>
__device__ __forceinline__ uint32_t roulette_pick(const Sums& sums, uint32_t n, uint32_t total,
                                                  uint32_t u)
{
    if (total == 0u)
        return scale32(u, n);
    const uint32_t dart = (uint32_t)(((uint64_t)u * (uint64_t)total) >> 32);
    uint32_t lo = 0, hi = n - 1u;   // sums[hi] = total > dart
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (sums[mid] > dart)
            hi = mid;
        else
            lo = mid + 1u;
    }
    return lo;
}

// One offspring from the parents' genomes (pop) and running sums.
template <class Pop, class Sums>
__device__ __forceinline__ uint64_t make_offspring(const Pop& pop, const Sums& sums, uint32_t n,
                                                   uint32_t total, const RouletteArgs& r,
                                                   const PoissonTable& thr, uint32_t i,
                                                   uint32_t gen)
{
    RouletteStream rs{r.key0, r.key1, i, gen, 0xFFFFFFFFu, {{0, 0, 0, 0}}};
    const int L = r.length;
    const uint64_t mask = L == 64 ? ~0ull : ((1ull << L) - 1ull);
    uint64_t child = pop[roulette_pick(sums, n, total, rs.word(0))] & mask;
    if (r.crossover) {
        const uint64_t b = pop[roulette_pick(sums, n, total, rs.word(1))];
        const uint32_t point = scale32(rs.word(2), (uint32_t)L);
        // positions 0..point-1 are the top `point` bits of the L-bit genome
        const uint64_t top = point == 0u ? 0ull : (mask & ~(mask >> point));
        child = (child & ~top) | (b & top);
    }
    const uint32_t uk = rs.word(3);
    int flips = L;
    for (int j = 0; j < L; ++j)
        if (below_threshold(thr, j, uk)) {
            flips = j;
            break;
        }
    uint64_t chosen = 0;
    int done = 0;
    for (uint32_t q = 4; done < flips && q < 4u + 1024u; ++q) {
        const uint32_t pos = scale32(rs.word(q), (uint32_t)L);
        const uint64_t bit = 1ull << (L - 1 - (int)pos);
        if ((chosen & bit) == 0ull) {
            chosen |= bit;
            ++done;
        }
    }
    return child ^ chosen;
}

// ---------------------------------------------------------------------------
// One generation over a population in device memory.
// ---------------------------------------------------------------------------
// Running sums of fit into sums[0..n), one workgroup of 1024 lanes (n <= 2^16).
__global__ __launch_bounds__(1024) void roulette_sums_kernel(const uint32_t* __restrict__ fit,
                                                             uint32_t n, uint32_t* sums)
{
    __shared__ uint32_t wave_tot[16];
    __shared__ uint32_t carry;
    const int tid = (int)threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid == 0)
        carry = 0;
    __syncthreads();
    for (uint32_t base = 0; base < n; base += 1024u) {
        const uint32_t i = base + (uint32_t)tid;
        uint32_t v = i < n ? fit[i] : 0u;
        // inclusive scan in the wave
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t o = (uint32_t)__shfl_up((int)v, off);
            if (lane >= off)
                v += o;
        }
        if (lane == 63)
            wave_tot[wave] = v;
        __syncthreads();
        uint32_t before = carry;
        for (int w = 0; w < wave; ++w)
            before += wave_tot[w];
        if (i < n)
            sums[i] = before + v;
        __syncthreads();
        if (tid == 1023)
            carry = before + v;
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void roulette_offspring_kernel(
    const uint64_t* __restrict__ pop, const uint32_t* __restrict__ sums, uint32_t n,
    RouletteArgs r, int32_t generation, uint32_t n_out, uint64_t* __restrict__ out)
{
    const uint32_t i = blockIdx.x * 256u + threadIdx.x;
    if (i >= n_out)
        return;
    const uint32_t total = sums[n - 1u];
    out[i] = make_offspring(pop, sums, n, total, r, r.poisson, i, (uint32_t)generation);
}

int launch_roulette_offspring(const uint64_t* pop, const uint32_t* fit, uint32_t n,
                              const RouletteArgs& r, int32_t generation, uint32_t n_out,
                              uint32_t* sums, uint64_t* out, hipStream_t s)
{
    hipLaunchKernelGGL(roulette_sums_kernel, dim3(1), dim3(1024), 0, s, fit, n, sums);
    if (n_out > 0)
        hipLaunchKernelGGL(roulette_offspring_kernel, dim3((n_out + 255u) / 256u), dim3(256), 0,
                           s, pop, (const uint32_t*)sums, n, r, generation, n_out, out);
    return hipGetLastError() == hipSuccess ? JATAM_OK : JATAM_E_HIP;
}

// ---------------------------------------------------------------------------
// Fujiyama simulations: workgroup s*rates + k is simulation s at rate k.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kFujiMaxPop) void fujiyama_kernel(FujiyamaArgs f)
{
    __shared__ uint64_t popa[kFujiMaxPop], popb[kFujiMaxPop];
    __shared__ uint32_t sums[kFujiMaxPop];
    __shared__ uint32_t wave_tot[kFujiMaxPop / 64], wave_hit[kFujiMaxPop / 64];
    __shared__ PoissonTable thr;
    const int tid = (int)threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int waves = (int)(blockDim.x + 63) / 64;
    const uint32_t n = (uint32_t)f.pop;
    const uint32_t rate = blockIdx.x % (uint32_t)f.rates, sim = blockIdx.x / (uint32_t)f.rates;
    RouletteArgs r = f.r;
    const uint64_t seed = f.seed + sim;
    r.key0 = (uint32_t)seed;
    r.key1 = (uint32_t)(seed >> 32);
    if (tid <= f.r.length)
        thr.tm1[tid] = f.poisson[rate].tm1[tid];
    if (tid == 0)
        thr.zero = f.poisson[rate].zero;
    uint64_t* cur = popa;
    uint64_t* nxt = popb;
    if ((uint32_t)tid < n)
        cur[tid] = 0ull;
    __syncthreads();
    int32_t discovery = -1, adaptation = -1;
    for (int32_t g = 0;; ++g) {
        // fitness, its running sums over the population, and the count of
        // genomes at the target weight
        const bool live = (uint32_t)tid < n;
        uint32_t v = live ? (uint32_t)__popcll(cur[tid]) : 0u;
        const uint64_t hit = __ballot(live && v >= (uint32_t)f.target);
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t o = (uint32_t)__shfl_up((int)v, off);
            if (lane >= off)
                v += o;
        }
        if (lane == 63)
            wave_tot[wave] = v;
        if (lane == 0)
            wave_hit[wave] = (uint32_t)__popcll(hit);
        __syncthreads();
        uint32_t before = 0, reached = 0;
        for (int w = 0; w < waves; ++w) {
            before += w < wave ? wave_tot[w] : 0u;
            reached += wave_hit[w];
        }
        if (live)
            sums[tid] = before + v;
        if (discovery < 0 && reached > 0u)
            discovery = g;
        if (adaptation < 0 && 2u * reached >= n)
            adaptation = g;
        __syncthreads();   // sums complete; every lane has the same times
        if ((discovery >= 0 && adaptation >= 0) || g == f.cutoff)
            break;
        const uint32_t total = sums[n - 1u];
        if (live)
            nxt[tid] = make_offspring(cur, sums, n, total, r, thr, (uint32_t)tid, (uint32_t)g);
        __syncthreads();   // the next population complete, the old one read
        uint64_t* t = cur;
        cur = nxt;
        nxt = t;
    }
    const uint32_t run = blockIdx.x;
    if (tid == 0) {
        f.discovery[run] = discovery;
        f.adaptation[run] = adaptation;
    }
    if (f.final_pop != nullptr && (uint32_t)tid < n)
        f.final_pop[(size_t)run * n + (uint32_t)tid] = cur[tid];
}

int launch_fujiyama(const FujiyamaArgs& f, hipStream_t s)
{
    const int threads = (f.pop + 63) / 64 * 64;
    hipLaunchKernelGGL(fujiyama_kernel, dim3((unsigned)(f.rates * f.sims)), dim3(threads), 0, s,
                       f);
    return hipGetLastError() == hipSuccess ? JATAM_OK : JATAM_E_HIP;
}

}  // namespace jatam

// ---------------------------------------------------------------------------
// C ABI.
// ---------------------------------------------------------------------------
extern "C" {

// T_j = floor(2^32 P(k <= j)), j = 0..length, for k Poisson(lambda), by the
// recurrence p_0 = exp(-lambda), p_j = p_(j-1) * lambda / j in double
// precision (2^32 once the sum reaches 1); kept as T_j - 1 and a zero mask.
static void poisson_table(double lambda, int length, jatam::PoissonTable* t)
{
    double p = exp(-lambda);
    double cdf = p;
    t->zero = 0;
    for (int j = 0; j <= jatam::kPoissonMax; ++j) {
        if (j > 0 && j <= length) {
            p = p * lambda / (double)j;
            cdf = cdf + p;
        }
        const double scaled = cdf * 4294967296.0;
        const uint64_t thr = scaled >= 4294967296.0 ? (1ull << 32) : (uint64_t)floor(scaled);
        if (thr == 0)
            t->zero |= 1ull << j;
        t->tm1[j] = thr == 0 ? 0u : (uint32_t)(thr - 1);
    }
}

static bool roulette_params_ok(const jatam_roulette_params_t* p)
{
    return p != nullptr && p->length >= 1 && p->length <= 64 && p->crossover >= 0 &&
           p->crossover <= 1 && p->lambda >= 0.0 && p->lambda <= 64.0;
}

int64_t jatam_roulette_work_words(int64_t n) { return n < 0 ? 0 : n + 64; }

int jatam_roulette_offspring(const uint64_t* pop, const uint32_t* fit, int64_t n,
                             const jatam_roulette_params_t* p, int32_t generation, int64_t n_out,
                             uint32_t* work, uint64_t* out, void* stream)
{
    if (!roulette_params_ok(p) || n < 1 || n > 65536 || n_out < 0 || n_out > 0xFFFFFFFFll ||
        pop == nullptr || fit == nullptr || work == nullptr || (n_out > 0 && out == nullptr))
        return JATAM_E_INVALID_ARG;
    jatam::RouletteArgs r{};
    r.key0 = (uint32_t)p->seed;
    r.key1 = (uint32_t)(p->seed >> 32);
    r.length = p->length;
    r.crossover = p->crossover;
    poisson_table(p->lambda, p->length, &r.poisson);
    return jatam::launch_roulette_offspring(pop, fit, (uint32_t)n, r, generation,
                                            (uint32_t)n_out, work, out, (hipStream_t)stream);
}

int jatam_fujiyama(const jatam_roulette_params_t* p, const double* lambdas, int32_t rates,
                   int32_t sims, int32_t pop, int32_t target, int32_t cutoff, int32_t* discovery,
                   int32_t* adaptation, uint64_t* final_pop, void* stream)
{
    if (!roulette_params_ok(p) || lambdas == nullptr || rates < 1 ||
        rates > jatam::kFujiMaxRates || sims < 1 || sims > (1 << 20) || pop < 1 ||
        pop > jatam::kFujiMaxPop || target < 0 || target > p->length || cutoff < 0 ||
        discovery == nullptr || adaptation == nullptr)
        return JATAM_E_INVALID_ARG;
    jatam::FujiyamaArgs f{};
    for (int k = 0; k < rates; ++k) {
        if (!(lambdas[k] >= 0.0 && lambdas[k] <= 64.0))
            return JATAM_E_INVALID_ARG;
        poisson_table(lambdas[k], p->length, &f.poisson[k]);
    }
    f.r.length = p->length;
    f.r.crossover = p->crossover;
    f.seed = p->seed;
    f.rates = rates;
    f.sims = sims;
    f.pop = pop;
    f.target = target;
    f.cutoff = cutoff;
    f.discovery = discovery;
    f.adaptation = adaptation;
    f.final_pop = final_pop;
    return jatam::launch_fujiyama(f, (hipStream_t)stream);
}

}  // extern "C"
