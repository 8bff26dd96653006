// jatam_ga.hip - one generation of the genetic algorithm whose fitness is
// JaTAM assembly (§2.2, §3.1): one lane per offspring (the paper's "one
// thread per genome"), the population read from HBM/L2, every generation a
// separate launch so all offspring see the same parents (the paper's global
// synchronisation by kernel boundary).
//
// Operators (the configuration's, in place of the paper's roulette wheel and
// Poisson bit flips):
//   selection  tournament of T genomes drawn uniformly with replacement; the
//              fittest wins, ties go to the earliest draw;
//   crossover  uniform per edge: edge e comes from parent B when bit e of a
//              random word is set, else from parent A;
//   mutation   each edge mutates with probability num/den to a colour drawn
//              uniformly from the other c-1 colours; no elitism.
// Offspring i of generation g draws the Philox4x32-10 stream keyed by the GA
// seed at counter (i, g, block, 1 << 28): word q is word q % 4 of block q / 4;
// words 0..T-1 draw parent A, T..2T-1 parent B, 2T is the crossover mask,
// 2T+1+e the mutation test of edge e and 2T+1+E+e its new colour (E = 4t).
#include "jatam_device.hpp"
#include "jatam_internal.hpp"

namespace jatam {

// Sequential reader of an offspring's word stream (one Philox block cached).
struct GaStream {
    uint32_t k0, k1, i, gen;
    uint32_t block;
    Words4 words;

    __device__ __forceinline__ uint32_t word(int q)
    {
        const uint32_t b = (uint32_t)q >> 2;
        if (b != block) {
            words = philox4x32_10(i, gen, b, 1u << 28, k0, k1);
            block = b;
        }
        const int k = q & 3;
        uint32_t u = words.w[0];
        u = k == 1 ? words.w[1] : u;
        u = k == 2 ? words.w[2] : u;
        u = k == 3 ? words.w[3] : u;
        return u;
    }
};

__global__ __launch_bounds__(256) void ga_offspring_kernel(const uint64_t* __restrict__ pop,
                                                           const int32_t* __restrict__ fit,
                                                           uint32_t n, GaArgs g,
                                                           uint32_t n_out,
                                                           uint64_t* __restrict__ out)
{
    const uint32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n_out)
        return;
    GaStream rs{g.key0, g.key1, i, (uint32_t)g.generation, 0xFFFFFFFFu, {{0, 0, 0, 0}}};
    const int T = g.tournament, E = 4 * g.t;
    uint64_t parent[2];
#pragma unroll
    for (int side = 0; side < 2; ++side) {
        uint32_t best = 0;
        int32_t best_fit = 0;
        for (int k = 0; k < T; ++k) {
            const uint32_t d = __umulhi(rs.word(side * T + k), n);
            const int32_t f = fit[d];
            if (k == 0 || f > best_fit) {
                best = d;
                best_fit = f;
            }
        }
        parent[side] = pop[best];
    }
    const uint32_t mask = rs.word(2 * T);
    const uint64_t cmask = (uint64_t)(g.c - 1);
    uint64_t child = 0;
    for (int e = 0; e < E; ++e) {
        const int shift = g.bits * (E - 1 - e);
        const uint64_t src = (mask >> e) & 1u ? parent[1] : parent[0];
        uint32_t colour = (uint32_t)((src >> shift) & cmask);
        if (__umulhi(rs.word(2 * T + 1 + e), (uint32_t)g.mut_den) < (uint32_t)g.mut_num) {
            const uint32_t r = __umulhi(rs.word(2 * T + 1 + E + e), (uint32_t)(g.c - 1));
            colour = r < colour ? r : r + 1;
        }
        child |= (uint64_t)colour << shift;
    }
    out[i] = child;
}

// Fitness of a genotype: the size of its structure if DET, else 0.
__global__ __launch_bounds__(256) void ga_fitness_kernel(const jatam_result_t* __restrict__ rec,
                                                         uint32_t n, int32_t* __restrict__ fit)
{
    const uint32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) {
        const jatam_result_t r = rec[i];
        fit[i] = r.cls == JATAM_DET ? r.size : 0;
    }
}

__global__ __launch_bounds__(256) void gather_kernel(const uint64_t* __restrict__ src,
                                                     const uint32_t* __restrict__ idx, uint32_t n,
                                                     uint64_t* __restrict__ dst)
{
    const uint32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i < n)
        dst[i] = src[idx[i]];
}

int launch_gather(const uint64_t* src, const uint32_t* idx, uint32_t n, uint64_t* dst,
                  hipStream_t stream)
{
    if (n == 0)
        return JATAM_OK;
    hipLaunchKernelGGL(gather_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, src, idx, n,
                       dst);
    return hipGetLastError() == hipSuccess ? JATAM_OK : JATAM_E_HIP;
}

int launch_ga_offspring(const uint64_t* pop, const int32_t* fit, uint32_t n, const GaArgs& g,
                        uint32_t n_out, uint64_t* out, hipStream_t stream)
{
    if (n_out == 0)
        return JATAM_OK;
    hipLaunchKernelGGL(ga_offspring_kernel, dim3((n_out + 255) / 256), dim3(256), 0, stream, pop,
                       fit, n, g, n_out, out);
    return hipGetLastError() == hipSuccess ? JATAM_OK : JATAM_E_HIP;
}

int launch_ga_fitness(const jatam_result_t* rec, uint32_t n, int32_t* fit, hipStream_t stream)
{
    if (n == 0)
        return JATAM_OK;
    hipLaunchKernelGGL(ga_fitness_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, rec, n,
                       fit);
    return hipGetLastError() == hipSuccess ? JATAM_OK : JATAM_E_HIP;
}

}  // namespace jatam
