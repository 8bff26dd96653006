// jatam_batched.hip - pipelined classification without global queues.
//
// The plain kernel gives each lane a whole genotype, so a wave lasts as long
// as its slowest genotype: on S_{2,8} the sum over waves of the slowest lane's
// work is ~7x the total work.  Here the classification is split by what the
// work actually is, into three stages per grid class (W = 16 or 32):
//
//   first_run<W>  persistent waves over 64-genotype input chunks: a share of
//                 the chunks is dealt out (chunk k to wave k mod the grid),
//                 the rest are claimed a few at a time from device counters
//                 by the waves that run out of work first.  A wave screens a
//                 chunk (decode, bond options of the seed: an ambiguous seed
//                 neighbour is ND_SITE, a seed with nothing to bond is a DET
//                 monomer; ~59% of S_{2,8}) and keeps the survivors in an LDS
//                 ring.  Each lane runs the
//                 first run of one survivor; a lane that finishes takes the
//                 next survivor at once, so lanes stay busy while run lengths
//                 differ.  A first run ending in an event or without ever
//                 drawing a random word is final; one that drew and ended
//                 cleanly makes the genotype a DET candidate, staged with its
//                 size and its packed run-0 shape in the wave's own segment.
//   size sort     a counting sort of the candidates by run-0 size, largest
//                 first (all runs of a deterministic genotype have that size,
//                 so this orders the later work by its exact cost): per
//                 segment histograms counted in LDS by the first-run waves
//                 as they stage, one scan, scatter with LDS cursors that
//                 moves each packed shape beside its candidate.
//   prove<W>      one lane per candidate checks whether its run-0 shape is
//                 guarded (every growth order ends in it), from the packed
//                 shape or, where the shape did not pack, a replay: then the
//                 record is final.
//   repeat<W>     R lanes per candidate, lane r making run r; the first
//                 witness in run order (an event or a shape different from
//                 run 0's) is found in LDS, and for DET genotypes the 8
//                 orientation hashes are split across the group's lanes.
//                 By default in two passes (runs 0-3, then the rest for the
//                 candidates without a witness); then the proof and the
//                 first pass share one kernel (prove_repeat), each wave
//                 claiming chunks of the sorted queue one at a time and
//                 running the repeat rounds of the candidates it failed to
//                 prove.  Or in one pass, or (repeat_seq) one lane per
//                 candidate making its runs in turn and stopping at the
//                 first witness, both after a separate proof and compaction.
//
// Global atomics on shared counters are few: the first-run claims, a few
// chunks at a time by waves that have finished their dealt-out share, and
// the fused kernel's chunk claims, one atomic per chunk, each spread over
// eight counters in separate 256-byte blocks (atomics on one address from
// every wave serialise); and the second repeat queue's counter, one atomic
// per wave and round of the first pass.  Every other queue is a per-wave
// segment or a scan.  Records are identical
// to the plain kernel's: each is a pure function of the genotype, never of
// the schedule.
#include "jatam_assembly.hpp"
#include "jatam_internal.hpp"

namespace jatam {

// ---------------------------------------------------------------------------
// Inputs: a range, an array of genomes, or an array of mixed items.
// ---------------------------------------------------------------------------
struct Geno {
    uint64_t genome;
    uint64_t rng_id;
    int t;
    int grid;
    bool valid;
};

// `first`: the range mode's first genotype of this call (a.first, moved by
// the slice counter of a replayed enumeration).
__device__ __forceinline__ Geno fetch_geno(const BatchArgs& a, uint64_t first, uint32_t i)
{
    Geno g;
    if (a.items != nullptr) {
        const jatam_item_t it = a.items[i];
        g.genome = it.genome;
        g.rng_id = it.rng_id;
        g.t = it.t;
        g.grid = it.grid;
        const int gbits = 4 * g.t * a.bits;
        g.valid = g.t >= 1 && g.t <= 4 && gbits <= 64 && g.grid >= 8 && g.grid <= 32 &&
                  (g.grid & 1) == 0 && (gbits == 64 || (g.genome >> gbits) == 0);
    } else {
        g.genome = a.genomes != nullptr ? a.genomes[i] : first + (uint64_t)i;
        g.t = a.t;
        g.grid = a.grid;
        g.rng_id = g.genome | ((uint64_t)(uint32_t)a.t << 56);
        const int gbits = 4 * a.t * a.bits;
        g.valid = gbits == 64 || (g.genome >> gbits) == 0;
    }
    return g;
}

// Input modes, as a compile-time choice for the first-run kernel: a range
// (genome = first + i, no loads), a genome list, or items.  With the mode
// fixed, a range call has no global loads in its loop, and so no waits
// (the vector memory counter also counts the loop's record stores).
enum { kInRange = 0, kInList = 1, kInItems = 2, kInRuntime = 3 };

template <int kIn>
__device__ __forceinline__ Geno fetch_geno_in(const BatchArgs& a, uint64_t first, uint32_t i)
{
    if constexpr (kIn == kInRuntime) {
        return fetch_geno(a, first, i);
    } else if constexpr (kIn == kInItems) {
        Geno g;
        const jatam_item_t it = a.items[i];
        g.genome = it.genome;
        g.rng_id = it.rng_id;
        g.t = it.t;
        g.grid = it.grid;
        const int gbits = 4 * g.t * a.bits;
        g.valid = g.t >= 1 && g.t <= 4 && gbits <= 64 && g.grid >= 8 && g.grid <= 32 &&
                  (g.grid & 1) == 0 && (gbits == 64 || (g.genome >> gbits) == 0);
        return g;
    } else {
        Geno g;
        g.genome = kIn == kInList ? a.genomes[i] : first + (uint64_t)i;
        g.t = a.t;
        g.grid = a.grid;
        g.rng_id = g.genome | ((uint64_t)(uint32_t)a.t << 56);
        const int gbits = 4 * a.t * a.bits;
        g.valid = gbits == 64 || (g.genome >> gbits) == 0;
        return g;
    }
}

// The genotype as the kernels of a grid class run it: in the 16 x 16 layout
// an item of G > 16 runs in a window of G = 16 around the seed.  Up to the
// first placement that exposes a bondable site on the window's ring, such a
// run is the run in its own G x G grid (same cells relative to the seed,
// same row-major order, same draws); a run that reaches the window's ring
// ends UNBOUND here and the item is run again in its own grid (see
// overflow_count_kernel).
template <int W, int kIn = kInRuntime>
__device__ __forceinline__ Geno run_geno(const BatchArgs& a, uint64_t first, uint32_t i)
{
    Geno g = fetch_geno_in<kIn>(a, first, i);
    if constexpr (W == 16)
        g.grid = g.grid < 16 ? g.grid : 16;
    return g;
}

// A graph-replayed enumeration reads its slice s from the device: the call
// covers genotypes first + s*n .. and writes records at out + s*n if asked.
// (The kernel argument block is left untouched: a modified copy would live
// in scratch memory.)
__device__ __forceinline__ uint64_t slice_first(const BatchArgs& a)
{
    return a.slice != nullptr ? a.first + (uint64_t)*a.slice * (uint64_t)a.n : a.first;
}

__device__ __forceinline__ jatam_result_t* slice_out(const BatchArgs& a)
{
    return a.slice != nullptr && a.out_per_slice ? a.out + (uint64_t)*a.slice * (uint64_t)a.n
                                                 : a.out;
}

__global__ void slice_reset_kernel(uint32_t* counter) { counter[0] = 0; }
__global__ void slice_advance_kernel(uint32_t* counter) { counter[0] += 1; }

int launch_slice_reset(uint32_t* counter, hipStream_t stream)
{
    hipLaunchKernelGGL(slice_reset_kernel, dim3(1), dim3(1), 0, stream, counter);
    return hipGetLastError() == hipSuccess ? JATAM_OK : JATAM_E_HIP;
}

int launch_slice_advance(uint32_t* counter, hipStream_t stream)
{
    hipLaunchKernelGGL(slice_advance_kernel, dim3(1), dim3(1), 0, stream, counter);
    return hipGetLastError() == hipSuccess ? JATAM_OK : JATAM_E_HIP;
}

// Grid class of a genotype: 0 = the 16 x 16 layout, 1 = the 32 x 32 layout.
__device__ __forceinline__ int grid_class(const BatchArgs& a, int grid)
{
    return grid <= a.narrow_max ? 0 : 1;
}

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

__device__ __forceinline__ uint64_t lanes_below() { return (1ull << lane_id()) - 1; }

// Per-wave class counts, flushed with one atomic per class at the end.
struct WaveTally {
    uint32_t n[4];
    __device__ __forceinline__ void add(bool done, int cls)
    {
#pragma unroll
        for (int k = 0; k < 4; ++k)
            n[k] += (uint32_t)__popcll(__ballot(done && cls == k));
    }
    __device__ __forceinline__ void flush(unsigned long long* tally) const
    {
        if (tally != nullptr && lane_id() == 0)
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (n[k])
                    atomicAdd(&tally[k], (unsigned long long)n[k]);
    }
};

// LDS entries of the per-wave shape-hash cache.
constexpr int kShapeCache = 32;
using WaveShapeCache = ShapeCache<kShapeCache>;

// D4 hash of the DET shape in a lane's OCC, for lanes with `want` (called by
// the whole wave).  A monomer and a domino have one shape each up to D4:
// their hashes are computed once per workspace (small_hash_kernel).  Shapes
// that fit 8 x 8 go through the wave's cache; a miss hashes the bitmap and
// fills the cache.
// small0/small1: the monomer's and the domino's hashes, read once per kernel
// (a load in the loop would make the wave wait for all its record stores).
template <int W>
__device__ __forceinline__ uint32_t det_hash(LaneGrid<W, 64>& g, uint32_t small0, uint32_t small1,
                                             WaveShapeCache& cache, bool want, int size, int grid)
{
    uint32_t h = 0;
    bool miss = false;
    uint64_t key = 0;
    if (want) {
        if (size <= 2) {
            h = size <= 1 ? small0 : small1;
        } else if (shape_key8(g, grid, key)) {
            if (!cache.lookup(key, h)) {
                h = bitmap8_shape_hash(key);
                miss = true;
            }
        } else {
            h = shape_hash(g, grid);
        }
    }
    cache.insert(miss, key, h, lane_id());
    return h;
}

// D4 hash of a shape given as its anchored 8 x 8 bitmap, for lanes with
// `want` (called by the whole wave), through the wave's cache.
__device__ __forceinline__ uint32_t packed_hash(uint64_t key, uint32_t small0, uint32_t small1,
                                                WaveShapeCache& cache, bool want, int size)
{
    uint32_t h = 0;
    bool miss = false;
    if (want) {
        if (size <= 2) {
            h = size <= 1 ? small0 : small1;
        } else if (!cache.lookup(key, h)) {
            h = bitmap8_shape_hash(key);
            miss = true;
        }
    }
    cache.insert(miss, key, h, lane_id());
    return h;
}

// ---------------------------------------------------------------------------
// first_run<W>: screen + first runs with lane refill.
// ---------------------------------------------------------------------------
constexpr int kRing = 128;   // LDS survivor ring per wave (>= 2 chunks)

// Size-sort bucket of a run-0 size: 64 buckets, exact up to 47 cells, then
// 64 cells wide; the largest sizes get the smallest keys.
__device__ __forceinline__ uint32_t size_key(uint32_t size)
{
    const uint32_t b = size < 48 ? size : 48 + min(15u, (size - 48) >> 6);
    return kSizeBuckets - 1 - b;
}

template <int W, int TM, int kIn>
__global__ __launch_bounds__(64) void first_run_kernel(const BatchArgs a, int klass)
{
    const uint32_t small0 = a.small0, small1 = a.small1;
    using Geo = Geometry<W>;
    const uint64_t first = slice_first(a);
    jatam_result_t* const out = slice_out(a);
    __shared__ uint32_t smem[Geo::kLaneWords * 64];
    __shared__ uint32_t ring[kRing];       // survivor indices
    __shared__ uint32_t ring_opt[kRing];   // their seeds' four site codes
    __shared__ uint4 cache_mem[kShapeCache];
    __shared__ uint32_t size_hist[kSizeBuckets];   // sizes this wave staged, by bucket
    LaneGrid<W, 64> g{smem + threadIdx.x};
    g.clear_all();
    WaveShapeCache cache{cache_mem};
    cache.clear(lane_id());
    static_assert(kSizeBuckets == 64, "one bucket per lane");
    size_hist[lane_id()] = 0;
    __syncthreads();
    RunState st{0, 0, 0, 0, 0, false};
    DrawPair dc;
    dc.reset();

    const uint32_t wave = blockIdx.x, nwaves = gridDim.x;
    if (wave == 0) {
        // counters of the later stages of this class (the previous call's
        // kernels are done, and these are first used after the size sort)
        if (lane_id() == 0)
            a.ws.counters[kCntRepeat2 + klass] = 0;   // the second repeat queue, empty
        if (lane_id() < kClaimCounters)               // the fused kernel's chunk claims
            a.ws.queue_claim[(klass * kClaimCounters + lane_id()) * kClaimStride] = 0;
    }
    const uint32_t n_items = a.n_dev != nullptr ? *a.n_dev : (uint32_t)a.n;
    const uint32_t nchunks = (n_items + 63) / 64;
    // Chunks below static_end are dealt out: this wave owns wave + k*nwaves.
    // The rest are claimed a few at a time by the waves that run out of
    // work first, which evens out the waves' end times.  They are split
    // into eight contiguous parts with a counter each (one atomic per claim
    // on one address from every wave serialises): a wave starts at part
    // (wave mod 8), its XCD's under the round-robin dispatch of workgroups,
    // and moves on to the next part when one runs dry, so the parts even
    // out among themselves too.  A claim is made only while the wave's
    // candidate segment can hold every item it has in flight plus the claim
    // (a wave that cannot claim with nothing in flight has staged more than
    // its dealt share of slots, so not all waves can be in that state while
    // chunks are left; any wave can take any part's chunks).
    // Claims are made only where every wave gets at least 16 chunks (with a
    // chunk or two per wave there is nothing to even out), of up to
    // claim_chunks chunks, fewer while a large claim would leave most waves
    // without one.
    const uint32_t per_wave = nchunks / (16u * nwaves);
    const uint32_t static_end =
        per_wave < 1u ? nchunks
                      : nchunks - (uint32_t)((uint64_t)nchunks * (uint32_t)a.dyn16 / 16u);
    const uint32_t claim_size = per_wave < (uint32_t)a.claim_chunks ? per_wave
                                                                    : (uint32_t)a.claim_chunks;
    uint32_t next_chunk = wave;
    uint32_t claim_next = 0, claim_end = 0;   // chunks claimed, not yet screened
    bool claims_left = static_end < nchunks;
    const uint32_t claim_blocks =
        claim_size == 0 ? 0u : (nchunks - static_end + claim_size - 1) / claim_size;
    const uint32_t part_blocks = (claim_blocks + kClaimCounters - 1) / kClaimCounters;
    uint32_t* const claim_ctr = a.ws.run_claim + klass * kClaimCounters * kClaimStride;
    uint32_t part = wave % (uint32_t)kClaimCounters, parts_dry = 0;
    uint32_t head = 0, queued = 0;            // survivor ring (wave-uniform)
    uint32_t staged = 0;                      // candidates in this wave's segment
    uint32_t* seg_idx = a.ws.cand_idx[klass] + (size_t)wave * a.seg_cap;
    uint16_t* seg_size = a.ws.cand_size[klass] + (size_t)wave * a.seg_cap;
    uint4* seg_shape = a.ws.cand_shape + (size_t)wave * a.seg_cap;
    WaveTally tally{{0, 0, 0, 0}};

    bool busy = false;
    bool starved = false;                     // the last refill found no chunk left
    uint32_t idx = 0;
    Geno gd{0, 0, 0, 0, false};
    ModelSource<TM> m;
    int ev = kEvNone;

    for (;;) {
        // -- lanes whose first run is over: records, hashes, staging ----------
        const bool finish = busy && run_over(ev, st, gd.grid);
        if (__ballot(finish) != 0) {
            bool done = false, candidate = false, det = false;
            int cls = 0;
            jatam_result_t rec{0, 0, 0u, 0};
            if (finish) {
                done = true;
                if (ev == kEvCorrupt) {
                    rec = jatam_result_t{JATAM_INVALID, 0, 0u, 0};
                    cls = JATAM_INVALID;
                } else if (ev != kEvNone) {
                    cls = ev == kEvUnbound ? JATAM_UNBOUND : JATAM_ND_SITE;
                    rec = jatam_result_t{cls, st.size, 0u, st.steps};
                } else if (!st.choice || a.runs == 1) {
                    // no random word was drawn: every run would be this run
                    cls = JATAM_DET;
                    det = true;
                    rec = jatam_result_t{JATAM_DET, st.size, 0u, st.steps};
                } else {
                    done = false;
                    candidate = true;
                }
            }
            if (__ballot(det) != 0)
                rec.hash = det_hash(g, small0, small1, cache, det, st.size, gd.grid);
            if (finish) {
                if (done)
                    out[idx] = rec;
                busy = false;
            }
            tally.add(done, cls);
            const uint64_t cm = __ballot(candidate);
            if (candidate) {
                const uint32_t pos = staged + (uint32_t)__popcll(cm & lanes_below());
                seg_idx[pos] = idx;
                seg_size[pos] = (uint16_t)st.size;
                // the shape, for the proof stage to check without a replay
                seg_shape[pos] = pack_shape(g, gd.grid, st.size);
                atomicAdd(&size_hist[size_key((uint32_t)st.size)], 1u);
            }
            staged += (uint32_t)__popcll(cm);
        }
        // -- refill idle lanes once enough of them wait -----------------------
        const uint64_t idle = __ballot(!busy);
        const uint32_t nidle = (uint32_t)__popcll(idle);
        if (nidle >= (uint32_t)a.refill || nidle == 64) {
            starved = false;
            while (queued < nidle) {
                uint32_t chunk;
                if (next_chunk < static_end) {
                    chunk = next_chunk;
                    next_chunk += nwaves;
                } else {
                    if (claim_next == claim_end) {
                        if (!claims_left ||
                            staged + (64u - nidle) + queued + claim_size * 64u > a.seg_cap) {
                            starved = true;
                            break;
                        }
                        uint32_t base = nchunks;
                        while (parts_dry < (uint32_t)kClaimCounters) {
                            uint32_t q = 0;
                            if (lane_id() == 0)
                                q = atomicAdd(claim_ctr + part * kClaimStride, 1u);
                            const uint32_t blk = part * part_blocks + (uint32_t)__shfl((int)q, 0);
                            if (blk < min((part + 1u) * part_blocks, claim_blocks)) {
                                base = static_end + blk * claim_size;
                                break;
                            }
                            part = (part + 1u) % (uint32_t)kClaimCounters;
                            ++parts_dry;
                        }
                        if (base >= nchunks) {
                            claims_left = false;
                            starved = true;
                            break;
                        }
                        claim_next = base;
                        claim_end = min(base + claim_size, nchunks);
                    }
                    chunk = claim_next++;
                }
                // screen one chunk of the input (§3.2: what the seed decides)
                const uint32_t pos = chunk * 64 + (uint32_t)lane_id();
                uint32_t i = pos;
                bool in_range = pos < n_items;
                if (in_range && a.order != nullptr) {
                    i = a.order[pos];
                    in_range = i < (uint64_t)a.n;   // an entry out of range is skipped
                }
                bool done = false, keep = false;
                int cls = 0;
                uint32_t opts = 0;
                if (in_range) {
                    const Geno s = fetch_geno_in<kIn>(a, first, i);
                    if (!s.valid) {
                        // exactly one launched pass reports an invalid item:
                        // its grid's class, or with the window on (the
                        // 32 x 32 class then reruns listed items only) the
                        // 16 x 16 class
                        if (a.narrow_max > 16 ? klass == 0 : grid_class(a, s.grid) == klass)
                            out[i] = jatam_result_t{JATAM_INVALID, 0, 0u, 0};
                    } else if (grid_class(a, s.grid) == klass) {
                        const Model<TM> sm = build_model<TM>(s.genome, s.t, a.bits, a.c);
                        const uint32_t seed = seed_tile(sm);
                        bool ambiguous = false, bonds = false;
#pragma unroll
                        for (int d = 0; d < 4; ++d) {
                            const uint32_t opt = site_options(sm, seed, d);
                            ambiguous = ambiguous || (opt >> 4) >= 2;
                            bonds = bonds || opt != 0;
                            opts |= opt << (8 * d);
                        }
                        if (ambiguous) {
                            out[i] = jatam_result_t{JATAM_ND_SITE, 1, 0u, 0};
                            done = true;
                            cls = JATAM_ND_SITE;
                        } else if (!bonds) {
                            out[i] = jatam_result_t{JATAM_DET, 1, small0, 0};
                            done = true;
                            cls = JATAM_DET;
                        } else {
                            keep = true;
                        }
                    }
                }
                tally.add(done, cls);
                const uint64_t km = __ballot(keep);
                if (keep) {
                    const uint32_t slot = (head + queued + (uint32_t)__popcll(km & lanes_below())) % kRing;
                    ring[slot] = i;
                    ring_opt[slot] = opts;
                }
                queued += (uint32_t)__popcll(km);
            }
            wave_lds_sync();   // ring writes visible to the whole wave
            const uint32_t take = queued < nidle ? queued : nidle;
            if (!busy) {
                const uint32_t rank = (uint32_t)__popcll(idle & lanes_below());
                if (rank < take) {
                    const uint32_t slot = (head + rank) % kRing;
                    idx = ring[slot];
                    gd = run_geno<W, kIn>(a, first, idx);
                    m.m = build_model<TM>(gd.genome, gd.t, a.bits, a.c);
                    ev = run_start_known(g, st, dc, gd.grid, ring_opt[slot]);
                    busy = true;
                }
            }
            head = (head + take) % kRing;
            queued -= take;
            wave_lds_sync();   // ring slots read before they are refilled
        }
        if (__ballot(busy) == 0) {
            // with every lane idle the refill took the whole ring, so the
            // ring is empty exactly when no chunk was left to screen
            if (queued == 0 && starved)
                break;
            continue;
        }
        // -- steps until enough lanes wait for a refill (every lane, once no
        // chunk is left), at least one step: finished lanes keep their run's
        // state until the finish pass above takes them, so records, hashes
        // and staging are done once per refill rather than at every step ---
        const uint32_t enough = queued == 0 && starved ? 65u : (uint32_t)a.refill;
        for (;;) {
            const bool stepping = busy && !run_over(ev, st, gd.grid);
            if (__ballot(stepping) == 0)
                break;
            prefetch_draws(dc, stepping, st, 0, a.key0, a.key1, (uint32_t)gd.rng_id,
                           (uint32_t)(gd.rng_id >> 32));
            if (stepping) {
                // prefetch_draws above made the block of every stepping
                // lane's next draw present
                PrefetchedDraws pd{dc};
                ev = run_step(m, g, st, pd, gd.grid, 0, a.key0, a.key1, (uint32_t)gd.rng_id,
                              (uint32_t)(gd.rng_id >> 32));
            }
            const uint64_t waiting = __ballot(!busy || run_over(ev, st, gd.grid));
            if ((uint32_t)__popcll(waiting) >= enough)
                break;
        }
    }
    if (lane_id() == 0)
        a.ws.seg_count[klass][wave] = staged;
    wave_lds_sync();   // every staged size counted
    a.ws.seg_hist[klass][(uint32_t)lane_id() * nwaves + wave] = size_hist[lane_id()];
    tally.flush(a.tally);
}

// ---------------------------------------------------------------------------
// Size sort: 64 buckets, exact up to 47 cells, then 64 cells wide; largest
// first.  Each first-run wave counts the sizes it stages (its segment's
// histogram, stored bucket-major); the sort scans the histograms and
// scatters.
// ---------------------------------------------------------------------------

// Exclusive scan of the bucket-major histogram in three coalesced passes:
// each block scans kScanBlock entries in place and writes its total; one
// block scans the totals (and stores the candidate count); the scatter adds
// the block offsets.
__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t v)
{
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t u = __shfl_up(v, off);
        v += lane_id() >= off ? u : 0u;
    }
    return v;
}

// Exclusive scan of kScanBlock values across a 1024-thread block; *total
// receives their sum.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* wsum,
                                                         uint32_t* total)
{
    const uint32_t w = threadIdx.x >> 6, l = lane_id();
    const uint32_t incl = wave_inclusive_scan(v);
    if (l == 63)
        wsum[w] = incl;
    __syncthreads();
    if (w == 0) {
        const uint32_t x = l < kScanBlock / 64 ? wsum[l] : 0u;
        const uint32_t xi = wave_inclusive_scan(x);
        if (l < kScanBlock / 64)
            wsum[l] = xi - x;
        if (l == kScanBlock / 64 - 1)
            wsum[kScanBlock / 64] = xi;
    }
    __syncthreads();
    *total = wsum[kScanBlock / 64];
    return wsum[w] + incl - v;
}

// In-place exclusive scan of h[0..total) in blocks of kScanBlock; block b's
// total goes to sums[b].  With `items` given, only the first
// ceil(*items / 64) entries (the chunks of *items queue positions) are read
// and scanned; the rest count as zero.
__global__ __launch_bounds__(kScanBlock) void scan_blocks_kernel(uint32_t* h, uint32_t total,
                                                                 uint32_t* sums,
                                                                 const uint32_t* items)
{
    __shared__ uint32_t wsum[kScanBlock / 64 + 1];
    const uint32_t n = items != nullptr ? min(total, (*items + 63u) / 64u) : total;
    const uint32_t i = blockIdx.x * kScanBlock + threadIdx.x;
    const uint32_t v = i < n ? h[i] : 0u;
    uint32_t sum;
    const uint32_t excl = block_exclusive_scan(v, wsum, &sum);
    if (i < n)
        h[i] = excl;
    if (threadIdx.x == 0)
        sums[blockIdx.x] = sum;
}

// In-place exclusive scan of the block totals (one block, any count: each
// thread takes a run of them); *total_out receives their sum.
__global__ __launch_bounds__(kScanBlock) void scan_sums_kernel(uint32_t* sums, uint32_t nblocks,
                                                               uint32_t* total_out)
{
    __shared__ uint32_t wsum[kScanBlock / 64 + 1];
    const uint32_t per = (nblocks + kScanBlock - 1) / kScanBlock;
    const uint32_t lo = threadIdx.x * per, hi = min(nblocks, lo + per);
    uint32_t v = 0;
    for (uint32_t b = lo; b < hi; ++b)
        v += sums[b];
    uint32_t total;
    uint32_t run = block_exclusive_scan(v, wsum, &total);
    for (uint32_t b = lo; b < hi; ++b) {
        const uint32_t x = sums[b];
        sums[b] = run;
        run += x;
    }
    if (threadIdx.x == 0)
        *total_out = total;
}

static void exclusive_scan(uint32_t* h, uint32_t total, uint32_t* sums, uint32_t* total_out,
                           hipStream_t stream, const uint32_t* items = nullptr)
{
    const uint32_t blocks = (total + kScanBlock - 1) / kScanBlock;
    hipLaunchKernelGGL(scan_blocks_kernel, dim3(blocks), dim3(kScanBlock), 0, stream, h, total,
                       sums, items);
    hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(kScanBlock), 0, stream, sums, blocks,
                       total_out);
}

// One block per segment: place its candidates with LDS cursors per bucket.
__global__ __launch_bounds__(256) void sort_scatter_kernel(BatchArgs a, int klass)
{
    __shared__ uint32_t cursor[kSizeBuckets];
    const uint32_t seg = blockIdx.x, nseg = gridDim.x;
    if (threadIdx.x < kSizeBuckets) {
        const uint32_t e = threadIdx.x * nseg + seg;
        cursor[threadIdx.x] = a.ws.seg_hist[klass][e] + a.ws.scan_sums[klass][e / kScanBlock];
    }
    __syncthreads();
    const uint32_t n = a.ws.seg_count[klass][seg];
    const uint16_t* sz = a.ws.cand_size[klass] + (size_t)seg * a.seg_cap;
    const uint32_t* ix = a.ws.cand_idx[klass] + (size_t)seg * a.seg_cap;
    const uint4* sh = a.ws.cand_shape + (size_t)seg * a.seg_cap;
    for (uint32_t i = threadIdx.x; i < n; i += 256) {
        const uint32_t pos = atomicAdd(&cursor[size_key(sz[i])], 1u);
        a.ws.sorted[klass][pos] = ix[i];
        a.ws.sorted_shape[pos] = sh[i];
    }
}

// ---------------------------------------------------------------------------
// prove<W>: one lane per candidate (in size order) takes its run-0 shape as
// the first-run stage packed it (the sort moved it beside the candidate), or
// replays run 0 where it did not fit, and checks whether the shape is guarded
// (shape_is_guarded; forced shapes are the case without conflicts): then
// every run ends in it and the record is final without the repeat runs --
// DET, run 0's size and hash, (size - 1) * R placements.  The other
// candidates are kept,
// in queue order, for the repeat runs: keep[pos] holds the candidate or
// kNoCandidate, and chunk_cnt[c] the kept count of queue chunk c (64
// positions; every chunk that holds a candidate is written, and the scan
// and the compaction read no other).
// ---------------------------------------------------------------------------
constexpr uint32_t kNoCandidate = 0xFFFFFFFFu;

// The proof of the candidate at queue position pos of the size-sorted queue
// (lanes with `active`): a guarded shape gets its record here; otherwise
// the candidate is kept (the return value) for the repeat runs.  Called by
// the whole wave.
template <int W, int TM>
__device__ __forceinline__ bool prove_one(const BatchArgs& a, uint64_t first,
                                          jatam_result_t* out, LaneGrid<W, 64>& g, RunState& st,
                                          WaveShapeCache& cache, WaveTally& tally, int klass,
                                          bool active, uint32_t pos, uint32_t& idx)
{
    bool forced = false, packed = false;
    int size = 0;
    uint64_t key = 0;
    Geno gd{0, 0, 0, 0, false};
    idx = 0;
    if (active) {
        idx = a.ws.sorted[klass][pos];
        gd = run_geno<W>(a, first, idx);
        const ModelSource<TM> src{build_model<TM>(gd.genome, gd.t, a.bits, a.c)};
        const uint4 sh = a.ws.sorted_shape[pos];
        packed = packed_shape_valid(sh);
        if (packed) {
            // the first-run stage packed the shape: no replay
            key = ((uint64_t)sh.y << 32) | sh.x;
            size = __popcll(key);
            forced = packed_shape_is_guarded(src, sh);
        } else {
            const int ev = run_assembly(src, g, st, gd.grid, 0, a.key0, a.key1,
                                        (uint32_t)gd.rng_id, (uint32_t)(gd.rng_id >> 32));
            size = st.size;
            forced = ev == kEvNone && shape_is_guarded(src, g, st, gd.grid);
        }
    }
    // hashes: a packed shape's from its bitmap, a replayed one's from the grid
    uint32_t h = det_hash(g, a.small0, a.small1, cache, forced && !packed, size, gd.grid);
    const uint32_t hp = packed_hash(key, a.small0, a.small1, cache, forced && packed, size);
    h = packed ? hp : h;
    if (forced)
        out[idx] = jatam_result_t{JATAM_DET, size, h, (size - 1) * a.runs};
    tally.add(forced, JATAM_DET);
    return active && !forced;
}

template <int W, int TM>
__global__ __launch_bounds__(64) void prove_kernel(const BatchArgs a, int klass)
{
    using Geo = Geometry<W>;
    const uint64_t first = slice_first(a);
    jatam_result_t* const out = slice_out(a);
    __shared__ uint32_t smem[Geo::kLaneWords * 64];
    __shared__ uint4 cache_mem[kShapeCache];
    LaneGrid<W, 64> g{smem + threadIdx.x};
    g.clear_all();
    WaveShapeCache cache{cache_mem};
    cache.clear(lane_id());
    __syncthreads();
    RunState st{0, 0, 0, 0, 0, false};
    WaveTally tally{{0, 0, 0, 0}};
    const uint32_t count = a.ws.counters[kCntCand + klass];
    uint32_t* keep = a.ws.cand_idx[klass];
    uint32_t* chunk_cnt = a.ws.chunk_cnt[klass];
    const uint32_t qchunks = (count + 63) / 64;   // queue chunks holding candidates
    for (uint32_t c = blockIdx.x; c < qchunks; c += gridDim.x) {
        const uint32_t pos = c * 64 + (uint32_t)lane_id();
        const bool active = pos < count;
        uint32_t idx;
        const bool kept =
            prove_one<W, TM>(a, first, out, g, st, cache, tally, klass, active, pos, idx);
        if (active)
            keep[pos] = kept ? idx : kNoCandidate;
        const uint32_t kc = (uint32_t)__popcll(__ballot(kept));
        if (lane_id() == 0)
            chunk_cnt[c] = kc;
    }
    if (blockIdx.x == 0 && lane_id() == 0) {
        // the candidate count, kept for the compaction (the scan of the kept
        // counts overwrites kCntCand)
        a.ws.counters[kCntCandAll + klass] = count;
    }
    tally.flush(a.tally);
}

// Kept candidates to the front of the queue, in order: a grid-stride loop
// over the queue chunks that hold candidates, a wave per chunk at a time.
__global__ __launch_bounds__(256) void compact_kernel(const BatchArgs a, int klass)
{
    const uint32_t count = a.ws.counters[kCntCandAll + klass];
    const uint32_t span = (count + 63) / 64 * 64;   // whole chunks: every wave ballots
    for (uint32_t pos = blockIdx.x * 256 + threadIdx.x; pos < span; pos += gridDim.x * 256) {
        const uint32_t c = pos >> 6;
        const uint32_t v = pos < count ? a.ws.cand_idx[klass][pos] : kNoCandidate;
        const bool kept = v != kNoCandidate;
        const uint64_t m = __ballot(kept);
        if (kept) {
            const uint32_t base =
                a.ws.chunk_cnt[klass][c] + a.ws.chunk_sums[klass][c / kScanBlock];
            a.ws.sorted[klass][base + (uint32_t)__popcll(m & lanes_below())] = v;
        }
    }
}

// ---------------------------------------------------------------------------
// The 16 x 16 window (items of G > 16 classified in the 16 x 16 layout, see
// run_geno).  An item whose record came out UNBOUND there exposed a bondable
// site on the window's ring in some run up to the deciding one; every other
// item's record is exact: no run up to the deciding one left the window, so
// those runs equal the runs in the item's own grid.  The items that left are
// listed, in queue order, for a rerun of the pipeline in 32 x 32 grids: one
// wave per chunk of 64 queue positions counts them, a scan places them.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool left_window(const BatchArgs& a, uint64_t first,
                                            const jatam_result_t* out, uint32_t pos,
                                            uint32_t& i)
{
    i = pos;
    if (pos >= (uint64_t)a.n)
        return false;
    if (a.order != nullptr) {
        i = a.order[pos];
        if (i >= (uint64_t)a.n)
            return false;
    }
    const Geno s = fetch_geno(a, first, i);
    return s.valid && s.grid > 16 && grid_class(a, s.grid) == 0 && out[i].cls == JATAM_UNBOUND;
}

__global__ __launch_bounds__(256) void overflow_count_kernel(const BatchArgs a)
{
    const uint32_t c = blockIdx.x * 4 + threadIdx.x / 64;   // one chunk per wave
    if (c >= (uint32_t)((a.n + 63) / 64))
        return;
    uint32_t i;
    const bool left = left_window(a, slice_first(a), slice_out(a), c * 64 + (uint32_t)lane_id(), i);
    const uint64_t m = __ballot(left);
    if (lane_id() == 0)
        a.ws.chunk_cnt[1][c] = (uint32_t)__popcll(m);
}

__global__ __launch_bounds__(256) void overflow_scatter_kernel(const BatchArgs a)
{
    if (blockIdx.x == 0 && threadIdx.x == 0 && a.tally != nullptr) {
        // the window pass counted these items UNBOUND; the rerun counts them
        atomicAdd(&a.tally[JATAM_UNBOUND],
                  0ull - (unsigned long long)a.ws.counters[kCntOverflow]);
    }
    const uint32_t c = blockIdx.x * 4 + threadIdx.x / 64;
    if (c >= (uint32_t)((a.n + 63) / 64))
        return;
    uint32_t i;
    const bool left = left_window(a, slice_first(a), slice_out(a), c * 64 + (uint32_t)lane_id(), i);
    const uint64_t m = __ballot(left);
    if (left) {
        const uint32_t base = a.ws.chunk_cnt[1][c] + a.ws.chunk_sums[1][c / kScanBlock];
        a.ws.overflow[base + (uint32_t)__popcll(m & lanes_below())] = i;
    }
}

// ---------------------------------------------------------------------------
// repeat<W>: all R runs of a candidate at once, one lane per run.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int wave_inclusive_sum(int v)
{
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int u = __shfl_up(v, off);
        v += lane_id() >= off ? u : 0;
    }
    return v;
}

//
// With rpass < R (the first of two passes) a group of rpass lanes makes runs
// 0 .. rpass-1 of its candidate: a witness among them decides the record as
// above; a candidate without one goes to queue_out (count_out counts them)
// for the second pass, rpass = R, which makes the rest of its runs.  Most
// non-deterministic candidates are decided by run 1, 2 or 3, so the first
// pass spares most of the runs a single pass would make.
//
// A candidate left undecided by runs 0 .. k-1 ended all of them in run 0's
// occupancy, with size0 - 1 placements each.  In the 16 x 16 layout the
// first pass stores that occupancy (8 words at the candidate's queue_out
// position: words 0-3 in cand_shape, free after the size sort, 4-7 in
// occ_hi), and the second pass (skip = k) then makes runs k .. R-1 only,
// each compared with the stored words.
__device__ __forceinline__ uint32_t* occ_word(uint4* lo, uint4* hi, uint32_t slot, int w)
{
    // words 0..3 of a slot in lo[slot], words 4..7 in hi[slot]
    return w < 4 ? (uint32_t*)&lo[slot] + w : (uint32_t*)&hi[slot] + (w - 4);
}

// The LDS and the per-lane layout of the R-lanes-per-candidate repeat runs:
// runs skip .. rpass-1 of each candidate, lane jr of group grp making run
// skip + jr.  round() runs one candidate per group (active groups only) to
// its record, or (a first pass without a witness) to the second queue.
template <int W, int TM, bool kTable>
struct RepeatWave {
    using Geo = Geometry<W>;
    const BatchArgs& a;
    uint64_t first;
    jatam_result_t* out;
    LaneGrid<W, 64> g;       // this lane's grid
    LaneGrid<W, 64> g0;      // the group's lead lane's grid
    uint32_t (*orient)[64];  // per group: bond table words, then orientation hashes
    WaveShapeCache& cache;
    RunState& st;
    WaveTally& tally;
    int skip;
    bool store_occ, all_runs;
    int R, groups, lane, grp, jr, run, lead, tail;
    uint64_t gmask;
    uint32_t* queue_out;
    uint32_t* count_out;

    __device__ RepeatWave(const BatchArgs& a_, uint32_t* smem, uint32_t (*orient_)[64],
                          WaveShapeCache& cache_, RunState& st_, WaveTally& tally_, int rpass,
                          int skip_, bool store_occ_, uint32_t* queue_out_, uint32_t* count_out_)
        : a(a_), first(slice_first(a_)), out(slice_out(a_)), g{smem + threadIdx.x},
          g0{smem}, orient(orient_), cache(cache_), st(st_), tally(tally_), skip(skip_),
          store_occ(store_occ_), all_runs(rpass >= a_.runs), R(rpass - skip_),
          groups(64 / (rpass - skip_)), lane((int)threadIdx.x), grp(0), jr(0), run(0), lead(0),
          tail(0), gmask(0), queue_out(queue_out_), count_out(count_out_)
    {
        grp = lane / R;
        jr = lane - grp * R;
        run = skip + jr;
        lead = grp * R;            // lane making run `skip`
        tail = lead + R - 1;       // lane making run rpass-1
        gmask = R == 64 ? ~0ull : ((1ull << R) - 1);
        g0 = LaneGrid<W, 64>{smem + lead};
    }

    // `active`: this lane's group has candidate idx (wave-uniform per group);
    // `slot`: its position in the input queue (where a first pass stored
    // run 0's occupancy, read when skip > 0).  Called by the whole wave.
    __device__ void round(bool active, uint32_t idx, uint32_t slot)
    {
        Geno gd{0, 0, 0, 0, false};
        int ev = kEvNone;
        if constexpr (kTable) {
            // the group builds its genotype's bond table together (word j by
            // lane j of the group), shared through the orientation slots
            TableSource<TM> src;
            if (active) {
                gd = run_geno<W>(a, first, idx);
                src.m = build_model<TM>(gd.genome, gd.t, a.bits, a.c);
                for (int j = jr; j < 8; j += R)
                    orient[j][grp] = bond_table_word(src.m, j);
            }
            wave_lds_sync();
            if (active) {
#pragma unroll
                for (int d = 0; d < 4; ++d)
                    src.side[d] = ((uint64_t)orient[2 * d + 1][grp] << 32) | orient[2 * d][grp];
                ev = run_assembly(src, g, st, gd.grid, run, a.key0, a.key1, (uint32_t)gd.rng_id,
                                  (uint32_t)(gd.rng_id >> 32));
            }
        } else {
            if (active) {
                gd = run_geno<W>(a, first, idx);
                const ModelSource<TM> src{build_model<TM>(gd.genome, gd.t, a.bits, a.c)};
                ev = run_assembly(src, g, st, gd.grid, run, a.key0, a.key1, (uint32_t)gd.rng_id,
                                  (uint32_t)(gd.rng_id >> 32));
            }
        }
        wave_lds_sync();   // every run's grid is final (and the table slots read)
        // a witness is a later run that hit an event or ended in another
        // shape than run 0 (the lead lane's, or the stored one)
        bool same = true;
        int stored_size = 0;                          // run 0's size, from the store
        if constexpr (W == 16) {
            if (skip > 0 && active) {
                uint4* const lo = a.ws.cand_shape;
                uint4* const hi = a.ws.occ_hi;
#pragma unroll
                for (int w = 0; w < Geo::kWords; ++w) {
                    const uint32_t o = *occ_word(lo, hi, slot, w);
                    stored_size += __popc(o);
                    same = same && g.occ(w) == o;
                }
            }
        }
        if (skip == 0 && active && jr > 0 && ev == kEvNone) {
#pragma unroll
            for (int w = 0; w < Geo::kWords; ++w)
                same = same && g.occ(w) == g0.occ(w);
        }
        const bool witness = active && (skip > 0 || jr > 0) && (ev != kEvNone || !same);
        const uint64_t wm = (__ballot(witness) >> lead) & gmask;
        const int fw = wm ? (int)__builtin_ctzll(wm) : R;      // R: no witness
        const int wl = lead + (fw < R ? fw : 0);
        const int w_ev = __shfl(ev, wl);
        const int w_size = __shfl(st.size, wl);
        const int lead_ev = __shfl(ev, lead);
        int cls;
        if (lead_ev == kEvCorrupt || (fw < R && w_ev == kEvCorrupt))
            cls = JATAM_INVALID;
        else if (fw == R)
            cls = JATAM_DET;
        else
            cls = w_ev == kEvUnbound ? JATAM_UNBOUND
                : w_ev == kEvAmbig   ? JATAM_ND_SITE
                                     : JATAM_ND_RUNS;
        // placements summed over runs 0..first witness (all R runs if DET);
        // the skipped runs made size0 - 1 each
        const int last = fw < R ? fw : R - 1;
        const int incl = wave_inclusive_sum(active && jr <= last ? st.steps : 0);
        const int steps = __shfl(incl, tail) - __shfl(incl, lead) + __shfl(st.steps, lead) +
                          skip * (__shfl(stored_size, lead) - 1);
        // without a witness in a first pass the candidate waits for the second
        const bool undecided = active && fw == R && !all_runs && cls == JATAM_DET;
        const uint64_t um = __ballot(undecided && jr == 0);
        if (um != 0) {
            uint32_t at = 0;
            if (lane == 0)
                at = atomicAdd(count_out, (uint32_t)__popcll(um));
            at = (uint32_t)__shfl((int)at, 0);
            const uint32_t qslot = at + (uint32_t)__popcll(um & lanes_below());
            if (undecided && jr == 0)
                queue_out[qslot] = idx;
            if constexpr (W == 16) {
                // every run of the group ended in run 0's occupancy: lane jr
                // stores words jr, jr + R, ... of its own
                const uint32_t gslot = (uint32_t)__shfl((int)qslot, lead);
                if (store_occ && undecided) {
                    for (int w = jr; w < Geo::kWords; w += R)
                        *occ_word(a.ws.cand_shape, a.ws.occ_hi, gslot, w) = g.occ(w);
                }
            }
        }
        const bool det = active && cls == JATAM_DET && !undecided;
        const int size0 = __shfl(st.size, lead);
        // run 0's shape: from the wave's cache, else the group's lanes share
        // its 8 orientation hashes
        uint64_t key = 0;
        bool small = false, hit = false;
        uint32_t cached = 0;
        if (det && size0 > 2) {
            small = shape_key8(g0, gd.grid, key);
            hit = small && cache.lookup(key, cached);
            if (!hit) {
                if (small) {
                    int w8, h8;
                    bitmap8_dims(key, w8, h8);
                    for (int k = jr; k < 8; k += R)
                        orient[k][grp] = bitmap_hash8(image8(key, w8, h8, k));
                } else {
                    const ShapeBox bx = crop(g0, gd.grid);
                    for (int k = jr; k < 8; k += R)
                        orient[k][grp] = orientation_hash(g0, bx, k);
                }
            }
        }
        wave_lds_sync();
        const bool done = active && jr == 0 && !undecided;
        uint32_t h = 0;
        if (done) {
            jatam_result_t rec;
            if (det) {
                if (size0 <= 2) {
                    h = size0 <= 1 ? a.small0 : a.small1;
                } else if (hit) {
                    h = cached;
                } else {
                    uint32_t hs[8];
#pragma unroll
                    for (int k = 0; k < 8; ++k)
                        hs[k] = orient[k][grp];
                    h = combine_orientations(hs);
                }
                rec = jatam_result_t{JATAM_DET, size0, h, steps};
            } else if (cls == JATAM_INVALID) {
                rec = jatam_result_t{JATAM_INVALID, 0, 0u, 0};
            } else {
                rec = jatam_result_t{cls, w_size, 0u, steps};
            }
            out[idx] = rec;
        }
        tally.add(done, cls);
        cache.insert(done && det && small && !hit, key, h, lane);
        wave_lds_sync();   // orientation slots and grids reused next round
    }
};

template <int W, int TM, bool kTable>
__global__ __launch_bounds__(64) void repeat_kernel(const BatchArgs a, int klass, int rpass,
                                                    int skip, bool store_occ,
                                                    const uint32_t* queue_in,
                                                    const uint32_t* count_in,
                                                    uint32_t* queue_out, uint32_t* count_out)
{
    using Geo = Geometry<W>;
    __shared__ uint32_t smem[Geo::kLaneWords * 64];
    __shared__ uint32_t orient[8][64];
    __shared__ uint4 cache_mem[kShapeCache];
    LaneGrid<W, 64> lg{smem + threadIdx.x};
    lg.clear_all();
    WaveShapeCache cache{cache_mem};
    cache.clear(lane_id());
    __syncthreads();
    RunState st{0, 0, 0, 0, 0, false};
    WaveTally tally{{0, 0, 0, 0}};
    RepeatWave<W, TM, kTable> rw(a, smem, orient, cache, st, tally, rpass, skip, store_occ,
                                 queue_out, count_out);
    const uint32_t count = *count_in;
    const uint32_t groups = (uint32_t)rw.groups, grp = (uint32_t)rw.grp;
    const uint32_t stride = gridDim.x * groups;

    // static round-robin over the size-sorted queue; the next entry is
    // fetched one iteration ahead
    uint32_t base = blockIdx.x * groups;
    uint32_t next_idx = 0;
    if (grp < groups && base + grp < count)
        next_idx = queue_in[base + grp];
    for (; base < count; base += stride) {
        const bool active = grp < groups && base + grp < count;
        const uint32_t idx = next_idx;
        if (grp < groups && base + stride + grp < count)
            next_idx = queue_in[base + stride + grp];
        rw.round(active, idx, base + grp);
    }
    tally.flush(a.tally);
}

// ---------------------------------------------------------------------------
// prove_repeat<W>: the proof and the first repeat pass in one kernel.  A
// wave proves 64 positions of the size-sorted queue at a time (prove_one)
// and keeps its unproven candidates in LDS; whenever they fill its repeat
// groups (64 / rpass of them) it makes their runs 0 .. rpass-1
// (RepeatWave::round).  The proof's steady integer work and the runs'
// latency-bound steps share the CUs, and no compaction or launch sits
// between them.  With rpass < R the candidates without a witness go to the
// second queue (count_out, cleared by the first-run kernel), in the 16 x 16 layout
// with run 0's occupancy stored.
// ---------------------------------------------------------------------------
template <int W, int TM, bool kTable>
__global__ __launch_bounds__(64) void prove_repeat_kernel(const BatchArgs a, int klass,
                                                          int rpass, uint32_t* queue_out,
                                                          uint32_t* count_out)
{
    using Geo = Geometry<W>;
    __shared__ uint32_t smem[Geo::kLaneWords * 64];
    __shared__ uint32_t orient[8][64];
    __shared__ uint4 cache_mem[kShapeCache];
    __shared__ uint32_t pend[128];   // unproven candidates waiting for a round
    LaneGrid<W, 64> lg{smem + threadIdx.x};
    lg.clear_all();
    WaveShapeCache cache{cache_mem};
    cache.clear(lane_id());
    __syncthreads();
    RunState st{0, 0, 0, 0, 0, false};
    WaveTally tally{{0, 0, 0, 0}};
    RepeatWave<W, TM, kTable> rw(a, smem, orient, cache, st, tally, rpass, 0, W == 16,
                                 queue_out, count_out);
    const uint32_t count = a.ws.counters[kCntCand + klass];
    const uint32_t qchunks = (count + 63) / 64;
    const uint32_t groups = (uint32_t)rw.groups, grp = (uint32_t)rw.grp;
    const uint32_t lane = (uint32_t)lane_id();
    uint32_t npend = 0;   // wave-uniform, below groups between chunks
    // one round on the first k waiting candidates, the rest moved down
    auto round_of = [&](uint32_t k) {
        const uint32_t pidx = grp < k ? pend[grp] : 0u;
        rw.round(grp < k, pidx, 0u);
        const uint32_t rest = npend - k;   // < 64
        const uint32_t v = lane < rest ? pend[k + lane] : 0u;
        wave_lds_sync();
        if (lane < rest)
            pend[lane] = v;
        wave_lds_sync();
        npend = rest;
    };
    // Chunks are claimed one at a time, so that waves end together however
    // the proofs and rounds of their chunks differ: counter x (x = the
    // block's index mod 8, its XCD under the round-robin dispatch of
    // workgroups) hands out chunks x, x + 8, x + 16, ... of the queue, so
    // each counter serves an even share of every part of the size-sorted
    // queue.  The counters are cleared by the first-run kernel.
    const uint32_t claimer = blockIdx.x % (uint32_t)kClaimCounters;
    uint32_t* const claim_ctr =
        a.ws.queue_claim + (klass * kClaimCounters + claimer) * kClaimStride;
    auto claim = [&]() -> uint32_t {
        uint32_t q = 0;
        if (lane == 0)
            q = atomicAdd(claim_ctr, 1u);
        return claimer + (uint32_t)kClaimCounters * (uint32_t)__shfl((int)q, 0);
    };
    for (uint32_t c = claim(); c < qchunks; c = claim()) {
        const uint32_t pos = c * 64 + lane;
        uint32_t idx;
        const bool kept = prove_one<W, TM>(a, rw.first, rw.out, lg, st, cache, tally, klass,
                                           pos < count, pos, idx);
        const uint64_t km = __ballot(kept);
        if (kept)
            pend[npend + (uint32_t)__popcll(km & lanes_below())] = idx;
        npend += (uint32_t)__popcll(km);
        wave_lds_sync();
        while (npend >= groups)
            round_of(groups);
    }
    while (npend > 0)
        round_of(npend < groups ? npend : groups);
    tally.flush(a.tally);
}

// ---------------------------------------------------------------------------
// repeat_seq<W>: one lane per candidate, its runs made in turn.  Run 0 is
// replayed and its occupancy kept beside the lane's grid (OCC0, the words it
// touched); each later run is compared with it as soon as it ends, and the
// first witness in run order (an event, or another occupancy) decides, so a
// non-deterministic candidate makes only the runs up to its first witness.
// A lane that is done takes the wave's next queue position: the wave owns
// chunks k, k + grid, ... of 64 positions of the size-sorted queue, handed to
// idle lanes in order once at least kSeqRefill of them wait.
// ---------------------------------------------------------------------------
constexpr int kSeqRefill = 8;

template <int W, int TM, bool kTable>
__global__ __launch_bounds__(64) void repeat_seq_kernel(const BatchArgs a, int klass)
{
    using Geo = Geometry<W>;
    using Src = typename std::conditional<kTable, TableSource<TM>, ModelSource<TM>>::type;
    const uint32_t small0 = a.small0, small1 = a.small1;
    const uint64_t first = slice_first(a);
    jatam_result_t* const out = slice_out(a);
    __shared__ uint32_t smem[Geo::kLaneWords * 64];
    __shared__ uint32_t occ0_mem[Geo::kWords * 64];   // lane j's word w at [w * 64 + j]
    __shared__ uint4 cache_mem[kShapeCache];
    LaneGrid<W, 64> g{smem + threadIdx.x};
    uint32_t* const occ0 = occ0_mem + threadIdx.x;
    g.clear_all();
    WaveShapeCache cache{cache_mem};
    cache.clear(lane_id());
    __syncthreads();
    RunState st{0, 0, 0, 0, 0, false};
    WaveTally tally{{0, 0, 0, 0}};
    DrawPair dc;
    dc.reset();

    const int R = a.runs;
    const uint32_t count = a.ws.counters[kCntCand + klass];
    const uint32_t* queue = a.ws.sorted[klass];
    const uint32_t nwaves = gridDim.x;
    uint32_t chunk = blockIdx.x, off = 0;   // the wave's next queue position (wave-uniform)
    bool busy = false;
    uint32_t idx = 0, osum0 = 0;
    int run = 0, ev = kEvNone, steps_sum = 0, size0 = 0;
    Geno gd{0, 0, 0, 0, false};
    Src src;

    for (;;) {
        const uint64_t idle = __ballot(!busy);
        const uint32_t nidle = (uint32_t)__popcll(idle);
        const bool left = chunk * 64u + off < count;
        if (left && (nidle >= (uint32_t)kSeqRefill || nidle == 64)) {
            if (!busy) {
                // idle lane of rank k takes the k-th next position (at most
                // one chunk ahead: off + k < 128)
                const uint32_t o = off + (uint32_t)__popcll(idle & lanes_below());
                const uint32_t pos = (o < 64u ? chunk : chunk + nwaves) * 64u + (o & 63u);
                if (pos < count) {
                    idx = queue[pos];
                    gd = run_geno<W>(a, first, idx);
                    src.m = build_model<TM>(gd.genome, gd.t, a.bits, a.c);
                    if constexpr (kTable) {
#pragma unroll
                        for (int d = 0; d < 4; ++d)
                            src.side[d] = ((uint64_t)bond_table_word(src.m, 2 * d + 1) << 32) |
                                          bond_table_word(src.m, 2 * d);
                    }
                    run = 0;
                    steps_sum = 0;
                    ev = run_start(src, g, st, dc, gd.grid);
                    busy = true;
                }
            }
            const uint32_t o = off + nidle;
            chunk = o < 64u ? chunk : chunk + nwaves;
            off = o & 63u;
        }
        if (__ballot(busy) == 0) {
            if (!left)
                break;
            continue;
        }
        const uint32_t rid_lo = (uint32_t)gd.rng_id, rid_hi = (uint32_t)(gd.rng_id >> 32);
        const bool stepping = busy && !run_over(ev, st, gd.grid);
        prefetch_draws(dc, stepping, st, run, a.key0, a.key1, rid_lo, rid_hi);
        if (stepping)
            ev = run_step(src, g, st, dc, gd.grid, run, a.key0, a.key1, rid_lo, rid_hi);
        const bool ended = busy && run_over(ev, st, gd.grid);
        bool done = false, det = false;
        int cls = 0;
        jatam_result_t rec{0, 0, 0u, 0};
        if (ended) {
            steps_sum += st.steps;
            if (ev == kEvCorrupt) {
                rec = jatam_result_t{JATAM_INVALID, 0, 0u, 0};
                cls = JATAM_INVALID;
                done = true;
            } else if (run == 0 && ev != kEvNone) {
                // (a candidate's run 0 ended cleanly in the first-run stage)
                cls = ev == kEvUnbound ? JATAM_UNBOUND : JATAM_ND_SITE;
                rec = jatam_result_t{cls, st.size, 0u, steps_sum};
                done = true;
            } else if (run == 0) {
                // keep run 0's occupancy: only its nonzero words are ever read
                for (uint32_t sw = st.osum; sw != 0; sw &= sw - 1) {
                    const int w = __builtin_ctz(sw);
                    occ0[w * 64] = g.occ(w);
                }
                osum0 = st.osum;
                size0 = st.size;
                run = 1;
                ev = run_start(src, g, st, dc, gd.grid);
            } else {
                // occupancy only grows within a run, so osum is exactly the
                // set of nonzero words
                bool same = ev == kEvNone && st.osum == osum0 && st.size == size0;
                for (uint32_t sw = osum0; same && sw != 0; sw &= sw - 1) {
                    const int w = __builtin_ctz(sw);
                    same = g.occ(w) == occ0[w * 64];
                }
                if (!same) {
                    cls = ev == kEvUnbound ? JATAM_UNBOUND
                        : ev == kEvAmbig   ? JATAM_ND_SITE
                                           : JATAM_ND_RUNS;
                    rec = jatam_result_t{cls, st.size, 0u, steps_sum};
                    done = true;
                } else if (run == R - 1) {
                    cls = JATAM_DET;
                    det = true;
                    rec = jatam_result_t{JATAM_DET, size0, 0u, steps_sum};
                    done = true;
                } else {
                    run += 1;
                    ev = run_start(src, g, st, dc, gd.grid);
                }
            }
        }
        // the grid holds run R-1's shape, which is run 0's
        if (__ballot(det) != 0)
            rec.hash = det_hash(g, small0, small1, cache, det, size0, gd.grid);
        if (done) {
            out[idx] = rec;
            busy = false;
        }
        tally.add(done, cls);
    }
    tally.flush(a.tally);
}

// ---------------------------------------------------------------------------
// Hashes of the two shapes that have a single D4 class per size.
// ---------------------------------------------------------------------------
__global__ void small_hash_kernel(uint32_t* out)
{
    __shared__ uint32_t smem[Geometry<16>::kLaneWords * 64];
    LaneGrid<16, 64> g{smem + threadIdx.x};
    if (threadIdx.x == 0) {
        for (int w = 0; w < Geometry<16>::kWords; ++w)
            g.occ(w) = 0;
        g.occ(0) = 1u;                  // one cell
        out[0] = shape_hash(g, 16);
        g.occ(0) = 3u;                  // two cells side by side
        out[1] = shape_hash(g, 16);
    }
}

// ---------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------
int batch_init_small_hash(uint32_t* small_hash, hipStream_t stream)
{
    hipLaunchKernelGGL(small_hash_kernel, dim3(1), dim3(64), 0, stream, small_hash);
    return hipGetLastError() == hipSuccess ? JATAM_OK : JATAM_E_HIP;
}

// One-wave workgroups of `kernel` that are resident on a CU at once.  The
// runtime's answer is capped by the CU's LDS as it is handed out on gfx950:
// in granules of 1,280 bytes, 128 per CU.  (Measured with spinning
// workgroups of a given dynamic LDS size: eleven of 14,080 bytes run
// together, eleven of 14,336 do not, nor ten of 15,744, while four of
// 39,680 and three of 52,480 do; the runtime reports eleven, eleven and ten
// for the first three.  A persistent grid sized above the true count leaves
// its last workgroups waiting for the first ones to finish.)
template <class K>
static int resident_per_cu(K kernel)
{
    constexpr size_t kLdsGranule = 1280, kLdsGranules = 128;
    int occ = 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kernel, 64, 0) != hipSuccess || occ < 1)
        occ = 1;
    hipFuncAttributes attr;
    if (hipFuncGetAttributes(&attr, reinterpret_cast<const void*>(kernel)) == hipSuccess &&
        attr.sharedSizeBytes > 0) {
        const size_t granules = (attr.sharedSizeBytes + kLdsGranule - 1) / kLdsGranule;
        const int fit = (int)(kLdsGranules / granules);
        occ = fit < occ ? (fit < 1 ? 1 : fit) : occ;
    }
    return occ;
}

template <int W, int TM>
static void occupancy_of(int out[3])
{
    out[0] = resident_per_cu(first_run_kernel<W, TM, kInRange>);
    // the repeat grid runs the proof + first pass kernel and the second pass
    const int repeat = resident_per_cu(repeat_kernel<W, TM, true>);
    const int fused = resident_per_cu(prove_repeat_kernel<W, TM, true>);
    out[1] = repeat < fused ? repeat : fused;
    out[2] = resident_per_cu(repeat_seq_kernel<W, TM, true>);
}

void batch_occupancy(int occ[2][2][3])
{
    occupancy_of<16, 2>(occ[0][0]);
    occupancy_of<16, 4>(occ[0][1]);
    occupancy_of<32, 2>(occ[1][0]);
    occupancy_of<32, 4>(occ[1][1]);
}

__global__ __launch_bounds__(256) void records_differ_kernel(const int4* __restrict__ x,
                                                             const int4* __restrict__ y,
                                                             uint64_t n, uint32_t* flag)
{
    bool differ = false;
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * 256) {
        const int4 u = x[i], v = y[i];
        differ = differ || u.x != v.x || u.y != v.y || u.z != v.z || u.w != v.w;
    }
    if (__ballot(differ) != 0 && lane_id() == 0)
        atomicOr(flag, 1u);
}

int launch_records_differ(const jatam_result_t* x, const jatam_result_t* y, uint64_t n,
                          uint32_t* flag, hipStream_t stream)
{
    if (n == 0)
        return JATAM_OK;
    const uint64_t want = (n + 255) / 256;
    const uint32_t blocks = (uint32_t)(want < 4096 ? want : 4096);
    hipLaunchKernelGGL(records_differ_kernel, dim3(blocks), dim3(256), 0, stream,
                       reinterpret_cast<const int4*>(x), reinterpret_cast<const int4*>(y), n,
                       flag);
    return hipGetLastError() == hipSuccess ? JATAM_OK : JATAM_E_HIP;
}

// Zeroes one counter word (a kernel rather than a memset: graph-safe).
// Clears the claim counters of one grid class (before its first-run kernel).
__global__ void clear_claims_kernel(uint32_t* ctr)
{
    if (threadIdx.x < kClaimCounters)
        ctr[threadIdx.x * kClaimStride] = 0u;
}

// The first-run kernel compiled for the call's input mode.
template <int W, int TM>
static void launch_first(const BatchArgs& a, uint32_t nb, hipStream_t stream, int klass)
{
    if (a.items != nullptr)
        hipLaunchKernelGGL((first_run_kernel<W, TM, kInItems>), dim3(nb), dim3(64), 0, stream, a,
                           klass);
    else if (a.genomes != nullptr)
        hipLaunchKernelGGL((first_run_kernel<W, TM, kInList>), dim3(nb), dim3(64), 0, stream, a,
                           klass);
    else
        hipLaunchKernelGGL((first_run_kernel<W, TM, kInRange>), dim3(nb), dim3(64), 0, stream, a,
                           klass);
}

// The R-lanes-per-candidate repeat kernel of grid class k for one pass.
template <int TM>
static void launch_repeat(const BatchArgs& a, int k, bool table, uint32_t rb, int rpass,
                          int skip, bool store_occ, const uint32_t* qin, const uint32_t* cin,
                          uint32_t* qout, uint32_t* cout, hipStream_t stream)
{
    if (k == 0 && table)
        hipLaunchKernelGGL((repeat_kernel<16, TM, true>), dim3(rb), dim3(64), 0, stream, a, 0,
                           rpass, skip, store_occ, qin, cin, qout, cout);
    else if (k == 0)
        hipLaunchKernelGGL((repeat_kernel<16, TM, false>), dim3(rb), dim3(64), 0, stream, a, 0,
                           rpass, skip, store_occ, qin, cin, qout, cout);
    else if (table)
        hipLaunchKernelGGL((repeat_kernel<32, TM, true>), dim3(rb), dim3(64), 0, stream, a, 1,
                           rpass, 0, false, qin, cin, qout, cout);
    else
        hipLaunchKernelGGL((repeat_kernel<32, TM, false>), dim3(rb), dim3(64), 0, stream, a, 1,
                           rpass, 0, false, qin, cin, qout, cout);
}

// The proof + first repeat pass kernel of grid class k.
template <int TM>
static void launch_prove_repeat(const BatchArgs& a, int k, bool table, uint32_t rb, int rpass,
                                uint32_t* qout, uint32_t* cout, hipStream_t stream)
{
    if (k == 0 && table)
        hipLaunchKernelGGL((prove_repeat_kernel<16, TM, true>), dim3(rb), dim3(64), 0, stream, a,
                           0, rpass, qout, cout);
    else if (k == 0)
        hipLaunchKernelGGL((prove_repeat_kernel<16, TM, false>), dim3(rb), dim3(64), 0, stream, a,
                           0, rpass, qout, cout);
    else if (table)
        hipLaunchKernelGGL((prove_repeat_kernel<32, TM, true>), dim3(rb), dim3(64), 0, stream, a,
                           1, rpass, qout, cout);
    else
        hipLaunchKernelGGL((prove_repeat_kernel<32, TM, false>), dim3(rb), dim3(64), 0, stream, a,
                           1, rpass, qout, cout);
}

template <int TM>
static void launch_stages(BatchArgs a, const bool classes[2], const StageLaunch launch[2],
                          hipStream_t stream, hipEvent_t* marks, uint8_t* launched)
{
    auto begin = [&](int s) {
        if (marks)
            (void)hipEventRecord(marks[2 * s], stream);
    };
    auto end = [&](int s) {
        if (marks) {
            (void)hipEventRecord(marks[2 * s + 1], stream);
            launched[s] = 1;
        }
    };
    for (int k = 0; k < 2; ++k) {
        if (!classes[k])
            continue;
        const uint32_t nb = (uint32_t)launch[k].first_blocks;
        const uint32_t rb = (uint32_t)launch[k].repeat_blocks;
        a.refill = launch[k].refill;
        const uint64_t nchunks = (uint64_t)(a.n + 63) / 64;
        a.dyn16 = launch[k].dyn16;
        a.claim_chunks = launch[k].claim_chunks;
        // a wave's segment holds its dealt-out share and one claim (the
        // first-run kernel's claim size, which is 0 where it makes none)
        const uint64_t per_wave = nchunks / (16u * (uint64_t)nb);
        const uint32_t claim = a.dyn16 <= 0 ? 0u
                               : per_wave < (uint64_t)a.claim_chunks ? (uint32_t)per_wave
                                                                      : (uint32_t)a.claim_chunks;
        a.seg_cap = (uint32_t)((nchunks + nb - 1) / nb * 64) + claim * 64u;
        begin(kStageFirst + kStagesPerClass * k);
        if (k == 1 && a.narrow_max > 16) {
            // the 32 x 32 class reruns only the items that left the window
            const uint32_t blocks = (uint32_t)((nchunks + 3) / 4);
            hipLaunchKernelGGL(overflow_count_kernel, dim3(blocks), dim3(256), 0, stream, a);
            exclusive_scan(a.ws.chunk_cnt[1], (uint32_t)nchunks, a.ws.chunk_sums[1],
                           a.ws.counters + kCntOverflow, stream);
            hipLaunchKernelGGL(overflow_scatter_kernel, dim3(blocks), dim3(256), 0, stream, a);
            a.order = a.ws.overflow;
            a.n_dev = a.ws.counters + kCntOverflow;
            a.narrow_max = 16;
        }
        if (a.dyn16 > 0)
            hipLaunchKernelGGL(clear_claims_kernel, dim3(1), dim3(64), 0, stream,
                               a.ws.run_claim + k * kClaimCounters * kClaimStride);
        if (k == 0)
            launch_first<16, TM>(a, nb, stream, 0);
        else
            launch_first<32, TM>(a, nb, stream, 1);
        end(kStageFirst + kStagesPerClass * k);
        begin(kStageSort + kStagesPerClass * k);
        exclusive_scan(a.ws.seg_hist[k], (uint32_t)kSizeBuckets * nb, a.ws.scan_sums[k],
                       a.ws.counters + kCntCand + k, stream);
        hipLaunchKernelGGL(sort_scatter_kernel, dim3(nb), dim3(256), 0, stream, a, k);
        end(kStageSort + kStagesPerClass * k);
        // the bond table holds colours 0..7
        const bool table = a.c <= 8;
        const int mapping = launch[k].repeat_mapping;
        if (mapping == 2 && a.runs > kRepeatFirstRuns) {
            // two passes: the proof and the first pass (runs 0 ..
            // kRepeatFirstRuns-1, a cheap round of 16 candidates per wave)
            // in one kernel on the repeat grid, the undecided candidates to
            // the staging array (free after the sort) for the second pass,
            // which in the 16 x 16 layout makes only runs kRepeatFirstRuns ..
            // R-1 (the 32 x 32 layout remakes all)
            uint32_t* q1 = a.ws.cand_idx[k];
            uint32_t* c1 = a.ws.counters + kCntRepeat2 + k;   // cleared by the first runs
            begin(kStageProve + kStagesPerClass * k);
            launch_prove_repeat<TM>(a, k, table, rb, kRepeatFirstRuns, q1, c1, stream);
            end(kStageProve + kStagesPerClass * k);
            begin(kStageRepeat + kStagesPerClass * k);
            launch_repeat<TM>(a, k, table, rb, a.runs, k == 0 ? kRepeatFirstRuns : 0, false, q1, c1,
                              nullptr, nullptr, stream);
            end(kStageRepeat + kStagesPerClass * k);
        } else {
            // forced shapes are final; the rest are compacted, in queue
            // order, for one pass of all R runs per candidate (mapping 0: a
            // round of 64 / R candidates is too costly to interleave with the
            // proof) or the one-lane-per-candidate repeat runs (mapping 1)
            begin(kStageProve + kStagesPerClass * k);
            if (k == 0)
                hipLaunchKernelGGL((prove_kernel<16, TM>), dim3(nb), dim3(64), 0, stream, a, 0);
            else
                hipLaunchKernelGGL((prove_kernel<32, TM>), dim3(nb), dim3(64), 0, stream, a, 1);
            const uint32_t qchunks = (uint32_t)nchunks;
            exclusive_scan(a.ws.chunk_cnt[k], qchunks, a.ws.chunk_sums[k],
                           a.ws.counters + kCntCand + k, stream, a.ws.counters + kCntCandAll + k);
            // a grid-stride loop over the candidates' chunks only (the count
            // is on the device)
            hipLaunchKernelGGL(compact_kernel, dim3(nb), dim3(256), 0, stream, a, k);
            end(kStageProve + kStagesPerClass * k);
            begin(kStageRepeat + kStagesPerClass * k);
            if (mapping != 1)
                launch_repeat<TM>(a, k, table, rb, a.runs, 0, false, a.ws.sorted[k],
                                  a.ws.counters + kCntCand + k, nullptr, nullptr, stream);
            else if (k == 0 && table)
                hipLaunchKernelGGL((repeat_seq_kernel<16, TM, true>), dim3(rb), dim3(64), 0, stream,
                                   a, 0);
            else if (k == 0)
                hipLaunchKernelGGL((repeat_seq_kernel<16, TM, false>), dim3(rb), dim3(64), 0,
                                   stream, a, 0);
            else if (table)
                hipLaunchKernelGGL((repeat_seq_kernel<32, TM, true>), dim3(rb), dim3(64), 0, stream,
                                   a, 1);
            else
                hipLaunchKernelGGL((repeat_seq_kernel<32, TM, false>), dim3(rb), dim3(64), 0,
                                   stream, a, 1);
            end(kStageRepeat + kStagesPerClass * k);
        }
    }
}

int launch_batched(const BatchArgs& a, const bool classes[2], const StageLaunch launch[2], int tm,
                   hipStream_t stream, hipEvent_t* marks, uint8_t* launched)
{
    if (launched)
        for (int s = 0; s < kStages; ++s)
            launched[s] = 0;
    if (a.n > 0) {
        if (tm == 2)
            launch_stages<2>(a, classes, launch, stream, marks, launched);
        else
            launch_stages<4>(a, classes, launch, stream, marks, launched);
    }
    return hipGetLastError() == hipSuccess ? JATAM_OK : JATAM_E_HIP;
}

}  // namespace jatam
