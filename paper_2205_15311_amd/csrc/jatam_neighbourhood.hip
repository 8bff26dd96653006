// jatam_neighbourhood.hip - robustness and evolvability of genotypes (§1.1).
//
// Robustness is the share of a genotype's single mutations that keep its
// phenotype, evolvability the number of different phenotypes its single
// mutations reach.  A single mutation flips one bit of the genome (the
// mutation operator flips bits, App. B.3), so a t-tile genotype has
// 4 t log2(c) single mutants.  A phenotype is UNBOUND, non-deterministic
// (either ND class) or a deterministic shape (size and D4 hash).
//
// Three kernels: the single mutants of a list or range of genotypes (for
// classification by any classify call); the counts from the genotypes' and
// their mutants' records; and the counts from the records of a whole space
// (S_{1,8}, S_{2,8}: every mutant is a member, so its record is gathered at
// genome ^ (1 << k), nothing is classified twice).  All integer work: one
// lane per genotype, its mutants' phenotype keys held in LDS for the
// distinct count.
#include "jatam_internal.hpp"

namespace jatam {

// 1: UNBOUND, 2: non-deterministic, else 4 + size * 2^32 + hash (DET).
__device__ __forceinline__ uint64_t phenotype_key(const jatam_result_t& r)
{
    if (r.cls == JATAM_DET)
        return 4ull + ((uint64_t)(uint32_t)r.size << 32) + (uint64_t)r.hash;
    return r.cls == JATAM_UNBOUND ? 1ull : 2ull;
}

__global__ __launch_bounds__(256) void mutants_kernel(const uint64_t* __restrict__ genomes,
                                                      uint64_t first, uint64_t n, int nbits,
                                                      uint64_t* __restrict__ out)
{
    const uint64_t e = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= n * (uint64_t)nbits)
        return;
    const uint64_t i = e / (uint64_t)nbits;
    const int k = (int)(e - i * (uint64_t)nbits);
    const uint64_t g = genomes != nullptr ? genomes[i] : first + i;
    out[e] = g ^ (1ull << k);
}

constexpr int kNbLanes = 64;   // one-wave blocks: 64 lanes x up to 64 keys in LDS

// Counts for genotype i, its mutants' keys already in keys[k * 64 + lane].
__device__ __forceinline__ jatam_neighbourhood_t count_neighbourhood(const uint64_t* keys,
                                                                     uint64_t own, int nbits)
{
    int robust = 0, evolv = 0;
    for (int k = 0; k < nbits; ++k) {
        const uint64_t kk = keys[k * kNbLanes];
        robust += kk == own;
        bool fresh = kk != own;
        for (int j = 0; j < k && fresh; ++j)
            fresh = keys[j * kNbLanes] != kk;
        evolv += fresh;
    }
    return jatam_neighbourhood_t{robust, evolv};
}

__global__ __launch_bounds__(kNbLanes) void neighbourhood_kernel(
    const jatam_result_t* __restrict__ own, const jatam_result_t* __restrict__ mut, uint64_t n,
    int nbits, jatam_neighbourhood_t* __restrict__ out)
{
    __shared__ uint64_t keys[64 * kNbLanes];
    const uint64_t i = (uint64_t)blockIdx.x * kNbLanes + threadIdx.x;
    if (i >= n)
        return;
    uint64_t* lk = keys + threadIdx.x;
    for (int k = 0; k < nbits; ++k)
        lk[k * kNbLanes] = phenotype_key(mut[i * (uint64_t)nbits + k]);
    out[i] = count_neighbourhood(lk, phenotype_key(own[i]), nbits);
}

__global__ __launch_bounds__(kNbLanes) void neighbourhood_space_kernel(
    const jatam_result_t* __restrict__ space, uint64_t first, uint64_t n, int nbits,
    jatam_neighbourhood_t* __restrict__ out)
{
    __shared__ uint64_t keys[64 * kNbLanes];
    const uint64_t i = (uint64_t)blockIdx.x * kNbLanes + threadIdx.x;
    if (i >= n)
        return;
    const uint64_t g = first + i;
    uint64_t* lk = keys + threadIdx.x;
    for (int k = 0; k < nbits; ++k)
        lk[k * kNbLanes] = phenotype_key(space[g ^ (1ull << k)]);
    out[i] = count_neighbourhood(lk, phenotype_key(space[g]), nbits);
}

int launch_mutants(const uint64_t* genomes, uint64_t first, int64_t n, int nbits, uint64_t* out,
                   hipStream_t s)
{
    const uint64_t total = (uint64_t)n * (uint64_t)nbits;
    for (uint64_t at = 0; at < total;) {
        // whole genotypes per launch, at most 2^31 elements
        const uint64_t per = ((1ull << 31) / (uint64_t)nbits) * (uint64_t)nbits;
        const uint64_t e = total - at < per ? total - at : per;
        const uint64_t gi = at / (uint64_t)nbits;
        hipLaunchKernelGGL(mutants_kernel, dim3((unsigned)((e + 255) / 256)), dim3(256), 0, s,
                           genomes != nullptr ? genomes + gi : nullptr, first + gi,
                           e / (uint64_t)nbits, nbits, out + at);
        at += e;
    }
    return hipGetLastError() == hipSuccess ? JATAM_OK : JATAM_E_HIP;
}

int launch_neighbourhood(const jatam_result_t* own, const jatam_result_t* mut, int64_t n,
                         int nbits, jatam_neighbourhood_t* out, hipStream_t s)
{
    for (int64_t at = 0; at < n; at += (int64_t)1 << 30) {
        const int64_t k = n - at < ((int64_t)1 << 30) ? n - at : ((int64_t)1 << 30);
        hipLaunchKernelGGL(neighbourhood_kernel, dim3((unsigned)((k + kNbLanes - 1) / kNbLanes)),
                           dim3(kNbLanes), 0, s, own + at, mut + at * nbits, (uint64_t)k, nbits,
                           out + at);
    }
    return hipGetLastError() == hipSuccess ? JATAM_OK : JATAM_E_HIP;
}

int launch_neighbourhood_space(const jatam_result_t* space, uint64_t first, int64_t n, int nbits,
                               jatam_neighbourhood_t* out, hipStream_t s)
{
    for (int64_t at = 0; at < n; at += (int64_t)1 << 30) {
        const int64_t k = n - at < ((int64_t)1 << 30) ? n - at : ((int64_t)1 << 30);
        hipLaunchKernelGGL(neighbourhood_space_kernel,
                           dim3((unsigned)((k + kNbLanes - 1) / kNbLanes)), dim3(kNbLanes), 0, s,
                           space, first + (uint64_t)at, (uint64_t)k, nbits, out + at);
    }
    return hipGetLastError() == hipSuccess ? JATAM_OK : JATAM_E_HIP;
}

}  // namespace jatam

extern "C" {

// Bits of a genome of t tiles over c colours, or -1 if (t, c) is invalid.
static int genome_bits(int t, int c)
{
    jatam::Params p;
    return jatam::make_params(t, c, 16, 1, 1, &p) == JATAM_OK ? p.genome_bits : -1;
}

int jatam_single_mutants(const uint64_t* genotypes, uint64_t first, int64_t n, int t, int c,
                         uint64_t* mutants, void* stream)
{
    const int nbits = genome_bits(t, c);
    if (nbits < 0 || n < 0 || (n > 0 && mutants == nullptr))
        return JATAM_E_INVALID_ARG;
    if (n == 0)
        return JATAM_OK;
    if (genotypes == nullptr) {
        const uint64_t last = first + (uint64_t)(n - 1);
        if (last < first || (nbits < 64 && (last >> nbits) != 0))
            return JATAM_E_INVALID_ARG;
    }
    return jatam::launch_mutants(genotypes, first, n, nbits, mutants, (hipStream_t)stream);
}

int jatam_neighbourhood(const jatam_result_t* own, const jatam_result_t* mutant_records,
                        int64_t n, int t, int c, jatam_neighbourhood_t* out, void* stream)
{
    const int nbits = genome_bits(t, c);
    if (nbits < 0 || n < 0 ||
        (n > 0 && (own == nullptr || mutant_records == nullptr || out == nullptr)))
        return JATAM_E_INVALID_ARG;
    if (n == 0)
        return JATAM_OK;
    return jatam::launch_neighbourhood(own, mutant_records, n, nbits, out, (hipStream_t)stream);
}

int jatam_neighbourhood_space(const jatam_result_t* space, uint64_t first, int64_t n, int t,
                              int c, jatam_neighbourhood_t* out, void* stream)
{
    const int nbits = genome_bits(t, c);
    if (nbits < 0 || nbits > 32 || n < 0 || (n > 0 && (space == nullptr || out == nullptr)))
        return JATAM_E_INVALID_ARG;
    if (n == 0)
        return JATAM_OK;
    const uint64_t last = first + (uint64_t)(n - 1);
    if (last < first || (last >> nbits) != 0)
        return JATAM_E_INVALID_ARG;
    return jatam::launch_neighbourhood_space(space, first, n, nbits, out, (hipStream_t)stream);
}

}  // extern "C"
