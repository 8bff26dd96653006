// jatam_truth.hip - the true class of a genotype: every growth order followed.
//
// The k runs of §3.2 sample growth orders, so a genotype whose every sampled
// run ends in one shape can still have an order that meets an ambiguous site
// or ends in another shape; the paper measures how this misclassification
// falls as k grows (§4.1).  The true class needs every order:
//   DET  every order ends in one shape without an event (size, D4 hash),
//   ND   some order meets an event (a bondable ring site, an ambiguous
//        site) or ends in a second shape (occupancy, without rotation).
//
// Two stages.
//   first<W>    one lane per genotype makes one run (any order will do).  An
//               event in it is reachable: ND.  A run that never chose
//               between two sites is the only order: DET.  A guarded shape
//               (no conflicting neighbour can be placed before the cell it
//               conflicts with, so every order places the same tiles) is
//               DET.  Anything else is queued.
//   explore<W>  one wave per queued genotype, breadth first over the event-
//               free states (sets of placed (cell, tile) pairs), level by
//               level (a state of level L has L + 1 tiles, so states of one
//               level are only ever reached from the level before).  Each
//               lane takes a state, rebuilds its grid in LDS and checks every
//               occupied cell's empty neighbours from scratch (the isotropic
//               check of §3.2); an event ends the search (ND), an empty
//               frontier is a terminal shape, compared with the first one
//               found.  Successors are deduplicated in a per-wave open-
//               addressing table whose 64-bit slots hold a 32-bit state hash
//               and the successor itself (parent index, cell, tile), so
//               equal hashes are settled by comparing the two states exactly
//               and no lane ever waits for another.  More than `cap` states:
//               undecided.
#include <new>

#include "jatam_assembly.hpp"
#include "jatam_internal.hpp"

namespace jatam {

namespace {

// Words of one stored state: occupancy bitmap, 4-bit tiles of the occupied
// cells (zero elsewhere), and the state's hash.
template <int W>
struct StateLayout {
    using Geo = Geometry<W>;
    static constexpr int kOcc = 0;
    static constexpr int kPend = Geo::kWords;
    static constexpr int kHash = Geo::kWords + Geo::kPendWords;
    static constexpr int kWords = kHash + 1;
};

// Hash of one placed (cell, tile) pair; a state's hash is the XOR over its
// pairs, so a successor's hash is its parent's XOR one term.
__device__ __forceinline__ uint32_t pair_mix(uint32_t cell, uint32_t tile)
{
    uint32_t h = (cell * 16u + tile) * 0x9E3779B1u + 0x7F4A7C15u;
    h ^= h >> 16;
    h *= 0x85EBCA6Bu;
    h ^= h >> 13;
    h *= 0xC2B2AE35u;
    h ^= h >> 16;
    return h;
}

// Packed successor: parent index (bits 14..31), cell (4..13), tile (0..3).

__device__ __forceinline__ uint32_t succ_pack(uint32_t parent, uint32_t cell, uint32_t tile)
{
    return (parent << 14) | (cell << 4) | tile;   // parent < kMaxTruthLevel = 2^18
}

template <int W>
__device__ __forceinline__ uint32_t state_word(const uint32_t* parent, int w, uint32_t cell,
                                               uint32_t tile)
{
    using L = StateLayout<W>;
    uint32_t v = parent[w];
    if (w == L::kOcc + (int)(cell >> 5))
        v |= 1u << (cell & 31u);
    if (w == L::kPend + (int)(cell >> 3))
        v |= tile << ((cell & 7u) * 4u);
    return v;
}

// Whether parent_a + (cell_a, tile_a) and parent_b + (cell_b, tile_b) are the
// same set of pairs.
template <int W>
__device__ bool same_state(const uint32_t* level, uint32_t a, uint32_t b)
{
    using L = StateLayout<W>;
    const uint32_t pa = a >> 14, pb = b >> 14;
    if (pa == pb)
        return a == b;
    const uint32_t* sa = level + (size_t)pa * L::kWords;
    const uint32_t* sb = level + (size_t)pb * L::kWords;
    const uint32_t ca = (a >> 4) & 1023u, cb = (b >> 4) & 1023u;
    for (int w = 0; w < L::kHash; ++w)
        if (state_word<W>(sa, w, ca, a & 15u) != state_word<W>(sb, w, cb, b & 15u))
            return false;
    return true;
}

// Genotype i of the call.
__device__ __forceinline__ uint64_t truth_genome(const TruthArgs& a, uint64_t i)
{
    return a.genomes != nullptr ? a.genomes[i] : a.first + i;
}

__device__ __forceinline__ bool genome_ok(const TruthArgs& a, uint64_t g)
{
    return a.genome_bits == 64 || (g >> a.genome_bits) == 0;
}

}  // namespace

// ---------------------------------------------------------------------------
// Stage 1: one run per genotype; events and proofs decide, the rest queue.
// ---------------------------------------------------------------------------
template <int W, int B, int TM>
__global__ __launch_bounds__(B) void truth_first_kernel(TruthArgs a)
{
    using Geo = Geometry<W>;
    __shared__ uint32_t smem[Geo::kLaneWords * B];
    const uint64_t i = (uint64_t)blockIdx.x * B + threadIdx.x;
    bool queue = false;
    if (i < (uint64_t)a.n) {
        LaneGrid<W, B> g{smem + threadIdx.x};
        g.clear_all();
        RunState st{0, 0, 0, 0, 0, false};
        const uint64_t genome = truth_genome(a, i);
        jatam_result_t rec{JATAM_INVALID, 0, 0u, 0};
        if (genome_ok(a, genome)) {
            const ModelSource<TM> m{build_model<TM>(genome, a.t, a.bits, a.c)};
            const uint64_t rid = genome | ((uint64_t)(uint32_t)a.t << 56);
            const int ev = run_assembly(m, g, st, a.grid, 0, a.key0, a.key1, (uint32_t)rid,
                                        (uint32_t)(rid >> 32));
            if (ev == kEvCorrupt) {
                rec = jatam_result_t{JATAM_INVALID, 0, 0u, 0};
            } else if (ev != kEvNone) {
                rec = jatam_result_t{JATAM_ND_SITE, 0, 0u, 0};
            } else if (!st.choice || shape_is_guarded(m, g, st, a.grid)) {
                rec = jatam_result_t{JATAM_DET, st.size, shape_hash(g, a.grid), 0};
            } else {
                queue = true;
            }
        }
        if (!queue)
            a.out[i] = rec;
    }
    const uint64_t qm = __ballot(queue);
    if (qm != 0) {
        const int lane = (int)__lane_id();
        uint32_t base = 0;
        if (lane == __builtin_ctzll(qm))
            base = atomicAdd(a.counters + 0, (uint32_t)__popcll(qm));
        base = (uint32_t)__shfl((int)base, __builtin_ctzll(qm));
        if (queue)
            a.queue[base + (uint32_t)__popcll(qm & ((1ull << lane) - 1))] = (uint32_t)i;
    }
}

// ---------------------------------------------------------------------------
// Stage 2: exhaustive exploration, one wave per queued genotype.
// ---------------------------------------------------------------------------
template <int W, int TM>
__global__ __launch_bounds__(64) void truth_explore_kernel(TruthArgs a)
{
    using Geo = Geometry<W>;
    using L = StateLayout<W>;
    __shared__ uint32_t smem[Geo::kLaneWords * 64];
    __shared__ uint32_t s_next, s_terms, s_flags;   // flags: 1 event/second shape, 2 overflow
    __shared__ uint32_t s_ref[Geo::kWords];         // the first terminal shape
    const int lane = (int)threadIdx.x;
    LaneGrid<W, 64> g{smem + lane};
    const uint32_t maxw = a.max_level;
    uint32_t* const level0 = a.arena + (size_t)blockIdx.x * 2 * maxw * L::kWords;
    uint32_t* const level1 = level0 + (size_t)maxw * L::kWords;
    uint32_t* const list = a.lists + (size_t)blockIdx.x * maxw;
    uint32_t* const terms = a.terms + (size_t)blockIdx.x * maxw;
    unsigned long long* const table = a.tables + ((size_t)blockIdx.x << a.table_log2);
    const uint32_t tmask = (1u << a.table_log2) - 1u;

    for (;;) {
        uint32_t k = 0;
        if (lane == 0)
            k = atomicAdd(a.counters + 1, 1u);
        k = (uint32_t)__shfl((int)k, 0);
        if (k >= a.counters[0])
            break;
        const uint32_t i = a.queue[k];
        const uint64_t genome = truth_genome(a, i);
        const ModelSource<TM> m{build_model<TM>(genome, a.t, a.bits, a.c)};
        const int G = a.grid;
        const int seed = (G / 2 - 1) * W + (G / 2 - 1);
        // level 0: the seed alone (tile id 0: tile 0 unrotated)
        for (int w = lane; w < L::kWords; w += 64) {
            uint32_t v = 0;
            if (w == L::kOcc + (seed >> 5))
                v = 1u << (seed & 31);
            if (w == L::kHash)
                v = pair_mix((uint32_t)seed, 0u);
            level0[w] = v;
        }
        uint32_t* cur = level0;
        uint32_t* nxt = level1;
        uint32_t width = 1;
        int64_t total = 1;
        bool have_ref = false;
        int ref_size = 0;
        int verdict = -2;   // undecided until the search ends
        if (lane == 0)
            s_flags = 0;
        __syncthreads();
        for (;;) {
            if (lane == 0) {
                s_next = 0;
                s_terms = 0;
            }
            __syncthreads();
            // -- analyse the level's states, insert their successors --------
            for (uint32_t s = (uint32_t)lane; s < width; s += 64) {
                const uint32_t* src = cur + (size_t)s * L::kWords;
                RunState st{0, 0, 0, 0, 0, false};
                for (int w = 0; w < Geo::kWords; ++w) {
                    const uint32_t o = src[L::kOcc + w];
                    g.occ(w) = o;
                    g.fr(w) = 0;
                    st.osum |= (o != 0 ? 1u : 0u) << w;
                    st.size += __popc(o);
                }
                for (int w = 0; w < Geo::kPendWords; ++w)
                    g.word(Geo::kPend + w) = src[L::kPend + w];
                int ev = kEvNone;
                for (uint32_t os = st.osum; os != 0; os &= os - 1) {
                    const int w = __builtin_ctz(os);
                    for (uint32_t cells = g.occ(w); cells != 0; cells &= cells - 1) {
                        const int p = (w << 5) | __builtin_ctz(cells);
                        const uint32_t id =
                            (g.pend_word(p) >> ((uint32_t)(p & 7) * 4u)) & 15u;
                        const int e = update_site(m, g, st, G, p, m.oriented((int)id));
                        ev = e != kEvNone ? e : ev;
                    }
                }
                if (ev != kEvNone) {
                    atomicOr(&s_flags, 1u);
                } else if (st.nf == 0) {
                    const uint32_t pos = atomicAdd(&s_terms, 1u);
                    terms[pos] = s;
                } else {
                    const uint32_t h0 = src[L::kHash];
                    for (uint32_t fs = st.fsum; fs != 0; fs &= fs - 1) {
                        const int w = __builtin_ctz(fs);
                        for (uint32_t cells = g.fr(w); cells != 0; cells &= cells - 1) {
                            const uint32_t q = (uint32_t)((w << 5) | __builtin_ctz(cells));
                            const uint32_t tile = (g.pend_word((int)q) >> ((q & 7u) * 4u)) & 15u;
                            const uint32_t succ = succ_pack(s, q, tile);
                            const uint32_t h = h0 ^ pair_mix(q, tile);
                            const unsigned long long key =
                                ((unsigned long long)(h | 1u) << 32) | succ;
                            uint32_t slot = h & tmask;
                            for (uint32_t probe = 0;; ++probe) {
                                if (probe > tmask) {   // table full
                                    atomicOr(&s_flags, 2u);
                                    break;
                                }
                                const unsigned long long old = atomicCAS(&table[slot], 0ull, key);
                                if (old == 0ull) {
                                    const uint32_t pos = atomicAdd(&s_next, 1u);
                                    if (pos < maxw)
                                        list[pos] = slot;
                                    else
                                        atomicOr(&s_flags, 2u);
                                    break;
                                }
                                if ((old >> 32) == (key >> 32) &&
                                    same_state<W>(cur, (uint32_t)old, succ))
                                    break;   // already inserted by another path
                                slot = (slot + 1u) & tmask;
                            }
                        }
                    }
                }
            }
            __syncthreads();
            const uint32_t flags = s_flags;
            const uint32_t nnext = s_next < maxw ? s_next : maxw;
            const uint32_t nterms = s_terms;
            // -- terminal shapes: the first one is the reference ------------
            if (flags == 0 && nterms > 0) {
                if (!have_ref) {
                    const uint32_t* r = cur + (size_t)terms[0] * L::kWords;
                    for (int w = lane; w < Geo::kWords; w += 64)
                        s_ref[w] = r[L::kOcc + w];
                    __syncthreads();
                    have_ref = true;
                    ref_size = 0;
                    for (int w = 0; w < Geo::kWords; ++w)
                        ref_size += __popc(s_ref[w]);
                }
                for (uint32_t j = (uint32_t)lane; j < nterms; j += 64) {
                    const uint32_t* r = cur + (size_t)terms[j] * L::kWords;
                    bool same = true;
                    for (int w = 0; w < Geo::kWords; ++w)
                        same = same && r[L::kOcc + w] == s_ref[w];
                    if (!same)
                        atomicOr(&s_flags, 1u);
                }
                __syncthreads();
            }
            const uint32_t flags2 = s_flags;
            bool stop = false;
            if (flags2 & 1u) {
                verdict = JATAM_ND_SITE;
                stop = true;
            } else if ((flags2 & 2u) || total + (int64_t)nnext > a.cap) {
                verdict = -2;
                stop = true;
            } else if (nnext == 0) {
                verdict = have_ref ? JATAM_DET : -2;
                stop = true;
            }
            if (stop) {
                // leave the table empty for the next genotype
                if (flags2 & 2u) {
                    for (uint32_t j = (uint32_t)lane; j <= tmask; j += 64)
                        table[j] = 0ull;
                } else {
                    for (uint32_t j = (uint32_t)lane; j < nnext; j += 64)
                        table[list[j]] = 0ull;
                }
                __syncthreads();
                break;
            }
            // -- the next level's states, written out; table emptied ----------
            for (uint32_t j = (uint32_t)lane; j < nnext; j += 64) {
                const uint32_t slot = list[j];
                const uint32_t succ = (uint32_t)table[slot];
                table[slot] = 0ull;
                const uint32_t* src = cur + (size_t)(succ >> 14) * L::kWords;
                const uint32_t cell = (succ >> 4) & 1023u, tile = succ & 15u;
                uint32_t* dst = nxt + (size_t)j * L::kWords;
                for (int w = 0; w < L::kHash; ++w)
                    dst[w] = state_word<W>(src, w, cell, tile);
                dst[L::kHash] = src[L::kHash] ^ pair_mix(cell, tile);
            }
            __syncthreads();
            uint32_t* tmp = cur;
            cur = nxt;
            nxt = tmp;
            width = nnext;
            total += nnext;
        }
        if (lane == 0) {
            jatam_result_t rec{verdict, 0, 0u, (int32_t)(total < 0x7FFFFFFF ? total : 0x7FFFFFFF)};
            if (verdict == JATAM_DET)
                rec.size = ref_size;
            a.out[i] = rec;
        }
        if (verdict == JATAM_DET) {
            // the D4 hash of the reference shape, on lane 0's LDS grid
            if (lane == 0) {
                for (int w = 0; w < Geo::kWords; ++w)
                    g.occ(w) = s_ref[w];
                a.out[i].hash = shape_hash(g, G);
            }
        }
        __syncthreads();
    }
}

__global__ void truth_reset_kernel(uint32_t* counters)
{
    if (threadIdx.x < 2)
        counters[threadIdx.x] = 0;
}

template <int W, int TM>
static void launch_truth_t(const TruthArgs& a, int blocks, hipStream_t s)
{
    constexpr int B = W == 16 ? 256 : 64;
    const uint64_t nb = ((uint64_t)a.n + B - 1) / B;
    if (nb > 0)
        hipLaunchKernelGGL((truth_first_kernel<W, B, TM>), dim3((unsigned)nb), dim3(B), 0, s, a);
    hipLaunchKernelGGL((truth_explore_kernel<W, TM>), dim3(blocks), dim3(64), 0, s, a);
}

int launch_truth(const TruthArgs& a, int blocks, hipStream_t s)
{
    if (a.max_level > kMaxTruthLevel || a.max_level == 0)
        return JATAM_E_INVALID_ARG;
    hipLaunchKernelGGL(truth_reset_kernel, dim3(1), dim3(64), 0, s, a.counters);
    const bool small = a.t <= 2;
    if (a.grid <= 16) {
        if (small)
            launch_truth_t<16, 2>(a, blocks, s);
        else
            launch_truth_t<16, 4>(a, blocks, s);
    } else {
        if (small)
            launch_truth_t<32, 2>(a, blocks, s);
        else
            launch_truth_t<32, 4>(a, blocks, s);
    }
    return hipGetLastError() == hipSuccess ? JATAM_OK : JATAM_E_HIP;
}

}  // namespace jatam

// ---------------------------------------------------------------------------
// C ABI.
// ---------------------------------------------------------------------------
struct jatam_truth {
    int64_t max_n;
    uint32_t max_level;
    int waves;
    int table_log2;
    void* region;
    jatam::TruthArgs a;   // workspace pointers
};

namespace {

int truth_launch(jatam_truth_t* w, const uint64_t* genotypes, uint64_t first, int64_t n, int t,
                 int c, int grid_limit, int64_t cap, jatam_result_t* out, void* stream)
{
    if (w == nullptr || n < 0 || n > w->max_n || cap < 1 || (n > 0 && out == nullptr))
        return JATAM_E_INVALID_ARG;
    jatam::Params p;
    const int rc = jatam::make_params(t, c, grid_limit, 1, 1, &p);
    if (rc != JATAM_OK)
        return rc;
    if (n == 0)
        return JATAM_OK;
    jatam::TruthArgs a = w->a;
    a.genomes = genotypes;
    a.first = first;
    a.n = n;
    a.t = p.t;
    a.c = p.c;
    a.bits = p.bits;
    a.genome_bits = p.genome_bits;
    a.grid = p.grid;
    a.key0 = p.key0;
    a.key1 = p.key1;
    a.cap = cap;
    a.out = out;
    return jatam::launch_truth(a, w->waves, (hipStream_t)stream);
}

}  // namespace

extern "C" {

int jatam_truth_create(int64_t max_n, int32_t max_level, int32_t waves, jatam_truth_t** out)
{
    if (out == nullptr)
        return JATAM_E_INVALID_ARG;
    *out = nullptr;
    if (max_n < 1 || max_n > (int64_t(1) << 32) || max_level < 1 ||
        (uint32_t)max_level > jatam::kMaxTruthLevel || waves < 1 || waves > 4096)
        return JATAM_E_INVALID_ARG;
    jatam_truth_t* w = new (std::nothrow) jatam_truth_t();
    if (w == nullptr)
        return JATAM_E_HIP;
    w->max_n = max_n;
    w->max_level = (uint32_t)max_level;
    w->waves = waves;
    int tl = 1;
    while ((int64_t(1) << tl) < 2 * (int64_t)max_level)
        ++tl;
    w->table_log2 = tl;
    // both grid classes fit the 32 x 32 state size
    const size_t sw = (size_t)jatam::truth_state_words(32);
    const size_t counters = 256;
    const size_t queue = ((size_t)max_n * 4 + 255) / 256 * 256;
    const size_t arena = (size_t)waves * 2 * max_level * sw * 4;
    const size_t lists = ((size_t)waves * max_level * 4 + 255) / 256 * 256;
    const size_t tables = (size_t)waves * (size_t(1) << tl) * 8;
    const size_t total = counters + queue + 2 * lists + arena + tables;
    uint8_t* base = nullptr;
    if (hipMalloc((void**)&base, total) != hipSuccess) {
        delete w;
        return JATAM_E_HIP;
    }
    // the tables start empty and every call leaves them empty
    if (hipMemset(base, 0, total) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
        (void)hipFree(base);
        delete w;
        return JATAM_E_HIP;
    }
    w->region = base;
    jatam::TruthArgs& a = w->a;
    a = jatam::TruthArgs{};
    size_t off = 0;
    a.counters = (uint32_t*)(base + off);
    off += counters;
    a.tables = (unsigned long long*)(base + off);
    off += tables;
    a.queue = (uint32_t*)(base + off);
    off += queue;
    a.lists = (uint32_t*)(base + off);
    off += lists;
    a.terms = (uint32_t*)(base + off);
    off += lists;
    a.arena = (uint32_t*)(base + off);
    a.max_level = (uint32_t)max_level;
    a.table_log2 = tl;
    *out = w;
    return JATAM_OK;
}

int jatam_truth_destroy(jatam_truth_t* w)
{
    if (w == nullptr)
        return JATAM_OK;
    const hipError_t e = hipFree(w->region);
    delete w;
    return e == hipSuccess ? JATAM_OK : JATAM_E_HIP;
}

int jatam_true_class(jatam_truth_t* w, const uint64_t* genotypes, int64_t n, int t, int c,
                     int grid_limit, int64_t cap, jatam_result_t* out, void* stream)
{
    if (n > 0 && genotypes == nullptr)
        return JATAM_E_INVALID_ARG;
    return truth_launch(w, genotypes, 0, n, t, c, grid_limit, cap, out, stream);
}

int jatam_true_class_range(jatam_truth_t* w, uint64_t first, int64_t n, int t, int c,
                           int grid_limit, int64_t cap, jatam_result_t* out, void* stream)
{
    if (n > 0) {
        jatam::Params p;
        const int rc = jatam::make_params(t, c, grid_limit, 1, 1, &p);
        if (rc != JATAM_OK)
            return rc;
        const uint64_t last = first + (uint64_t)(n - 1);
        if (last < first || (p.genome_bits < 64 && (last >> p.genome_bits) != 0))
            return JATAM_E_INVALID_ARG;
    }
    return truth_launch(w, nullptr, first, n, t, c, grid_limit, cap, out, stream);
}

}  // extern "C"
