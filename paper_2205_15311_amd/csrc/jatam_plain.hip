// jatam_plain.hip - plain classification kernel: one lane per genotype.
//
// Each lane decodes its genotype, makes up to R assembly runs in sequence and
// writes one 16-byte record (§3.2, §3.3).  The grid of a lane lives in LDS
// (jatam_assembly.hpp).  A wave lasts as long as its slowest genotype.
#include "jatam_assembly.hpp"
#include "jatam_internal.hpp"

namespace jatam {

// Full classification of one genotype (§3.2): up to R runs, first witness
// in run order decides.  kVariant: JATAM_VARIANT_* flags (C4 hash, movelist
// traversal with the lane's stack in `stk`).
template <int W, int B, int TM, int kVariant = 0>
__device__ jatam_result_t classify_genotype(LaneGrid<W, B>& g, RunState& st, uint64_t genome,
                                            uint64_t rng_id, const Params& prm,
                                            LaneStack<B> stk = LaneStack<B>{nullptr})
{
    using Geo = Geometry<W>;
    const ModelSource<TM> m{build_model<TM>(genome, prm.t, prm.bits, prm.c)};
    const uint32_t rid_lo = (uint32_t)rng_id, rid_hi = (uint32_t)(rng_id >> 32);
    uint32_t occ0[Geo::kWords];
    int size0 = 0;
    int work = 0;
    for (int r = 0; r < prm.runs; ++r) {
        int ev;
        if constexpr ((kVariant & JATAM_VARIANT_LIFO) != 0)
            ev = run_assembly_lifo(m, g, stk, st, prm.grid, r, prm.key0, prm.key1, rid_lo,
                                   rid_hi);
        else
            ev = run_assembly(m, g, st, prm.grid, r, prm.key0, prm.key1, rid_lo, rid_hi);
        work += st.steps;
        if (ev == kEvCorrupt)
            return jatam_result_t{JATAM_INVALID, 0, 0u, 0};
        if (ev != kEvNone)
            return jatam_result_t{ev == kEvUnbound ? JATAM_UNBOUND : JATAM_ND_SITE, st.size, 0u,
                                  work};
        if (r == 0) {
#pragma unroll
            for (int w = 0; w < Geo::kWords; ++w)
                occ0[w] = (st.osum >> w) & 1u ? g.occ(w) : 0u;
            size0 = st.size;
            if (!st.choice)
                break;   // no draw was ever made: every run is this run
        } else {
            bool same = true;
#pragma unroll
            for (int w = 0; w < Geo::kWords; ++w)
                same = same && (((st.osum >> w) & 1u ? g.occ(w) : 0u) == occ0[w]);
            if (!same)
                return jatam_result_t{JATAM_ND_RUNS, st.size, 0u, work};
        }
    }
    uint32_t hash;
    if constexpr ((kVariant & JATAM_VARIANT_C4) != 0)
        hash = shape_hash_c4(g, prm.grid);
    else
        hash = shape_hash(g, prm.grid);
    return jatam_result_t{JATAM_DET, size0, hash, work};
}

template <int W, int B, int TM>
__global__ __launch_bounds__(B) void classify_plain_kernel(const uint64_t* __restrict__ genomes,
                                                           uint64_t first, int64_t n, Params prm,
                                                           jatam_result_t* __restrict__ out)
{
    using Geo = Geometry<W>;
    __shared__ uint32_t smem[Geo::kLaneWords * B];
    const int64_t i = (int64_t)blockIdx.x * B + threadIdx.x;
    if (i >= n)
        return;
    LaneGrid<W, B> g{smem + threadIdx.x};
    g.clear_all();
    RunState st{0, 0, 0, 0, 0, false};

    const uint64_t genome = genomes ? genomes[i] : first + (uint64_t)i;
    jatam_result_t rec;
    if (prm.genome_bits < 64 && (genome >> prm.genome_bits) != 0) {
        rec = jatam_result_t{JATAM_INVALID, 0, 0u, 0};
    } else {
        const uint64_t rng_id = genome | ((uint64_t)(uint32_t)prm.t << 56);
        rec = classify_genotype<W, B, TM>(g, st, genome, rng_id, prm);
    }
    out[i] = rec;
}

// The plain kernel with a classification variant: the lane's movelist stack
// (kStackWords words) follows the grid words of all lanes in LDS.
template <int W, int B, int TM, int kVariant>
__global__ __launch_bounds__(B) void classify_variant_kernel(const uint64_t* __restrict__ genomes,
                                                             uint64_t first, int64_t n,
                                                             Params prm,
                                                             jatam_result_t* __restrict__ out)
{
    using Geo = Geometry<W>;
    constexpr int kStack = (kVariant & JATAM_VARIANT_LIFO) != 0 ? kStackWords : 0;
    __shared__ uint32_t smem[(Geo::kLaneWords + kStack) * B];
    const int64_t i = (int64_t)blockIdx.x * B + threadIdx.x;
    if (i >= n)
        return;
    LaneGrid<W, B> g{smem + threadIdx.x};
    g.clear_all();
    LaneStack<B> stk{smem + Geo::kLaneWords * B + threadIdx.x};
    RunState st{0, 0, 0, 0, 0, false};
    const uint64_t genome = genomes ? genomes[i] : first + (uint64_t)i;
    jatam_result_t rec;
    if (prm.genome_bits < 64 && (genome >> prm.genome_bits) != 0) {
        rec = jatam_result_t{JATAM_INVALID, 0, 0u, 0};
    } else {
        const uint64_t rng_id = genome | ((uint64_t)(uint32_t)prm.t << 56);
        rec = classify_genotype<W, B, TM, kVariant>(g, st, genome, rng_id, prm, stk);
    }
    out[i] = rec;
}

template <int W, int B, int TM, int kVariant>
static void launch_variant_t(const uint64_t* genomes, uint64_t first, int64_t n,
                             const Params& prm, jatam_result_t* out, hipStream_t stream)
{
    const int64_t blocks = (n + B - 1) / B;
    hipLaunchKernelGGL((classify_variant_kernel<W, B, TM, kVariant>), dim3((unsigned)blocks),
                       dim3(B), 0, stream, genomes, first, n, prm, out);
}

template <int kVariant>
static void launch_variant_v(const uint64_t* genomes, uint64_t first, int64_t n,
                             const Params& prm, jatam_result_t* out, hipStream_t stream)
{
    const bool small = prm.t <= 2;
    if (prm.grid <= 16) {
        if (small)
            launch_variant_t<16, 64, 2, kVariant>(genomes, first, n, prm, out, stream);
        else
            launch_variant_t<16, 64, 4, kVariant>(genomes, first, n, prm, out, stream);
    } else if constexpr ((kVariant & JATAM_VARIANT_LIFO) == 0) {
        if (small)
            launch_variant_t<32, 64, 2, kVariant>(genomes, first, n, prm, out, stream);
        else
            launch_variant_t<32, 64, 4, kVariant>(genomes, first, n, prm, out, stream);
    }
}

int launch_variant(const uint64_t* genomes, uint64_t first, int64_t n, const Params& prm,
                   int variant, jatam_result_t* out, hipStream_t stream)
{
    if (n == 0)
        return JATAM_OK;
    if ((variant & JATAM_VARIANT_LIFO) != 0 && prm.grid > 16)
        return JATAM_E_UNSUPPORTED;
    switch (variant) {
    case 0: launch_variant_v<0>(genomes, first, n, prm, out, stream); break;
    case 1: launch_variant_v<1>(genomes, first, n, prm, out, stream); break;
    case 2: launch_variant_v<2>(genomes, first, n, prm, out, stream); break;
    case 3: launch_variant_v<3>(genomes, first, n, prm, out, stream); break;
    default: return JATAM_E_INVALID_ARG;
    }
    return hipGetLastError() == hipSuccess ? JATAM_OK : JATAM_E_HIP;
}

template <int W, int B, int TM>
static void launch_plain_t(const uint64_t* genomes, uint64_t first, int64_t n, const Params& prm,
                           jatam_result_t* out, hipStream_t stream)
{
    const int64_t blocks = (n + B - 1) / B;
    hipLaunchKernelGGL((classify_plain_kernel<W, B, TM>), dim3((unsigned)blocks), dim3(B), 0,
                       stream, genomes, first, n, prm, out);
}

int launch_plain(const uint64_t* genomes, uint64_t first, int64_t n, const Params& prm,
                 jatam_result_t* out, hipStream_t stream)
{
    if (n == 0)
        return JATAM_OK;
    const bool small = prm.t <= 2;
    if (prm.grid <= 16) {
        if (small)
            launch_plain_t<16, 256, 2>(genomes, first, n, prm, out, stream);
        else
            launch_plain_t<16, 256, 4>(genomes, first, n, prm, out, stream);
    } else {
        if (small)
            launch_plain_t<32, 64, 2>(genomes, first, n, prm, out, stream);
        else
            launch_plain_t<32, 64, 4>(genomes, first, n, prm, out, stream);
    }
    return hipGetLastError() == hipSuccess ? JATAM_OK : JATAM_E_HIP;
}

}  // namespace jatam
