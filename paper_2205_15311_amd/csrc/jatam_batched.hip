// jatam_batched.hip - pipelined classification without global queues.
//
// The plain kernel gives each lane a whole genotype, so a wave lasts as long
// as its slowest genotype: on S_{2,8} the sum over waves of the slowest lane's
// work is ~7x the total work.  Here the classification is split by what the
// work actually is, into three stages per grid class (W = 16 or 32):
//
//   first_run<W>  persistent waves, each owning a fixed set of 64-genotype
//                 input chunks.  A wave screens a chunk (decode, bond options
//                 of the seed: an ambiguous seed neighbour is ND_SITE, a seed
//                 with nothing to bond is a DET monomer; ~59% of S_{2,8}) and
//                 keeps the survivors in an LDS ring.  Each lane runs the
//                 first run of one survivor; a lane that finishes takes the
//                 next survivor at once, so lanes stay busy while run lengths
//                 differ.  A first run ending in an event or without ever
//                 drawing a random word is final; one that drew and ended
//                 cleanly makes the genotype a DET candidate, staged with its
//                 size in the wave's own segment.
//   size sort     a counting sort of the candidates by run-0 size, largest
//                 first (all runs of a deterministic genotype have that size,
//                 so this orders the repeat work by its exact cost): per
//                 segment histograms in LDS, one scan, scatter with LDS
//                 cursors.
//   repeat<W>     R lanes per candidate, lane r making run r; the first
//                 witness in run order (an event or a shape different from
//                 run 0's) is found in LDS, and for DET genotypes the 8
//                 orientation hashes are split across the group's lanes.
//
// No stage uses a global atomic on a shared counter (on MI355X those
// serialise across the 8 XCDs): work is partitioned statically, queues are
// per-wave segments.  Records are identical to the plain kernel's: each is a
// pure function of the genotype, never of the schedule.
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

__device__ __forceinline__ Geno fetch_geno(const BatchArgs& a, uint32_t i)
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
        g.genome = a.genomes != nullptr ? a.genomes[i] : a.first + (uint64_t)i;
        g.t = a.t;
        g.grid = a.grid;
        g.rng_id = g.genome | ((uint64_t)(uint32_t)a.t << 56);
        const int gbits = 4 * a.t * a.bits;
        g.valid = gbits == 64 || (g.genome >> gbits) == 0;
    }
    return g;
}

__device__ __forceinline__ int grid_class(int grid) { return grid <= 16 ? 0 : 1; }

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

// A monomer and a domino have one shape each up to D4: their hashes are
// computed once per workspace (small_hash_kernel) by the general function.
template <int W>
__device__ __forceinline__ uint32_t det_hash(LaneGrid<W, 64>& g, const BatchArgs& a, int size,
                                             int grid)
{
    if (size <= 2)
        return a.ws.small_hash[size - 1];
    return shape_hash(g, grid);
}

// ---------------------------------------------------------------------------
// first_run<W>: screen + first runs with lane refill.
// ---------------------------------------------------------------------------
constexpr int kRing = 128;   // LDS survivor ring per wave (>= 2 chunks)

template <int W, int TM>
__global__ __launch_bounds__(64) void first_run_kernel(BatchArgs a, int klass)
{
    using Geo = Geometry<W>;
    __shared__ uint32_t smem[Geo::kLaneWords * 64];
    __shared__ uint32_t ring[kRing];
    LaneGrid<W, 64> g{smem + threadIdx.x};
    g.clear_all();
    RunState st{0, 0, 0, 0, 0, false};
    DrawCache dc;
    dc.block = 0xFFFFFFFFu;

    const uint32_t wave = blockIdx.x, nwaves = gridDim.x;
    const uint32_t nchunks = (uint32_t)((a.n + 63) / 64);
    uint32_t next_chunk = wave;               // this wave owns chunks wave + k*nwaves
    uint32_t head = 0, queued = 0;            // survivor ring (wave-uniform)
    uint32_t staged = 0;                      // candidates in this wave's segment
    uint32_t* seg_idx = a.ws.cand_idx[klass] + (size_t)wave * a.seg_cap;
    uint16_t* seg_size = a.ws.cand_size[klass] + (size_t)wave * a.seg_cap;
    WaveTally tally{{0, 0, 0, 0}};

    bool busy = false;
    uint32_t idx = 0;
    Geno gd{0, 0, 0, 0, false};
    Model<TM> m;
    int ev = kEvNone;

    for (;;) {
        // -- refill idle lanes once enough of them wait -----------------------
        const uint64_t idle = __ballot(!busy);
        const uint32_t nidle = (uint32_t)__popcll(idle);
        if (nidle >= (uint32_t)a.refill || nidle == 64) {
            while (queued < nidle && next_chunk < nchunks) {
                // screen one chunk of the input (§3.2: what the seed decides)
                const uint32_t i = next_chunk * 64 + (uint32_t)lane_id();
                bool done = false, keep = false;
                int cls = 0;
                if (i < (uint64_t)a.n) {
                    const Geno s = fetch_geno(a, i);
                    if (!s.valid) {
                        // exactly one launched pass reports an invalid item
                        if (grid_class(s.grid) == klass)
                            a.out[i] = jatam_result_t{JATAM_INVALID, 0, 0u, 0};
                    } else if (grid_class(s.grid) == klass) {
                        const Model<TM> sm = build_model<TM>(s.genome, s.t, a.bits, a.c);
                        const uint32_t seed = seed_tile(sm);
                        bool ambiguous = false, bonds = false;
#pragma unroll
                        for (int d = 0; d < 4; ++d) {
                            const uint32_t opt = site_options(sm, seed, d);
                            ambiguous = ambiguous || (opt >> 4) >= 2;
                            bonds = bonds || opt != 0;
                        }
                        if (ambiguous) {
                            a.out[i] = jatam_result_t{JATAM_ND_SITE, 1, 0u, 0};
                            done = true;
                            cls = JATAM_ND_SITE;
                        } else if (!bonds) {
                            a.out[i] = jatam_result_t{JATAM_DET, 1, a.ws.small_hash[0], 0};
                            done = true;
                            cls = JATAM_DET;
                        } else {
                            keep = true;
                        }
                    }
                }
                tally.add(done, cls);
                const uint64_t km = __ballot(keep);
                if (keep)
                    ring[(head + queued + (uint32_t)__popcll(km & lanes_below())) % kRing] = i;
                queued += (uint32_t)__popcll(km);
                next_chunk += nwaves;
            }
            __syncthreads();   // ring writes visible to the whole wave
            const uint32_t take = queued < nidle ? queued : nidle;
            if (!busy) {
                const uint32_t rank = (uint32_t)__popcll(idle & lanes_below());
                if (rank < take) {
                    idx = ring[(head + rank) % kRing];
                    gd = fetch_geno(a, idx);
                    m = build_model<TM>(gd.genome, gd.t, a.bits, a.c);
                    ev = run_start(m, g, st, dc, gd.grid);
                    busy = true;
                }
            }
            head = (head + take) % kRing;
            queued -= take;
            __syncthreads();   // ring slots read before they are refilled
        }
        if (__ballot(busy) == 0) {
            if (queued == 0 && next_chunk >= nchunks)
                break;
            continue;
        }
        // -- one step of every busy lane ---------------------------------------
        if (busy && !run_over(ev, st, gd.grid))
            ev = run_step(m, g, st, dc, gd.grid, 0, a.key0, a.key1, (uint32_t)gd.rng_id,
                          (uint32_t)(gd.rng_id >> 32));
        // -- lanes whose first run is over ----------------------------------
        const bool finish = busy && run_over(ev, st, gd.grid);
        bool done = false, candidate = false;
        int cls = 0;
        if (finish) {
            jatam_result_t rec;
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
                rec = jatam_result_t{JATAM_DET, st.size, det_hash(g, a, st.size, gd.grid),
                                     st.steps};
            } else {
                done = false;
                candidate = true;
            }
            if (done)
                a.out[idx] = rec;
            busy = false;
        }
        tally.add(done, cls);
        const uint64_t cm = __ballot(candidate);
        if (candidate) {
            const uint32_t pos = staged + (uint32_t)__popcll(cm & lanes_below());
            seg_idx[pos] = idx;
            seg_size[pos] = (uint16_t)st.size;
        }
        staged += (uint32_t)__popcll(cm);
    }
    if (lane_id() == 0)
        a.ws.seg_count[klass][wave] = staged;
    tally.flush(a.tally);
}

// ---------------------------------------------------------------------------
// Size sort: 64 buckets, exact up to 47 cells, then 64 cells wide; largest
// first.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t size_key(uint32_t size)
{
    const uint32_t b = size < 48 ? size : 48 + min(15u, (size - 48) >> 6);
    return kSizeBuckets - 1 - b;
}

// One block per segment: its bucket histogram, stored bucket-major.
__global__ __launch_bounds__(256) void sort_hist_kernel(BatchArgs a, int klass)
{
    __shared__ uint32_t hist[kSizeBuckets];
    const uint32_t seg = blockIdx.x, nseg = gridDim.x;
    if (threadIdx.x < kSizeBuckets)
        hist[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t n = a.ws.seg_count[klass][seg];
    const uint16_t* sz = a.ws.cand_size[klass] + (size_t)seg * a.seg_cap;
    for (uint32_t i = threadIdx.x; i < n; i += 256)
        atomicAdd(&hist[size_key(sz[i])], 1u);
    __syncthreads();
    if (threadIdx.x < kSizeBuckets)
        a.ws.seg_hist[klass][threadIdx.x * nseg + seg] = hist[threadIdx.x];
}

// Exclusive scan of the bucket-major histogram, in place; the total is the
// candidate count.
__global__ __launch_bounds__(1024) void sort_scan_kernel(BatchArgs a, int klass, uint32_t nseg)
{
    __shared__ uint32_t part[1024];
    uint32_t* h = a.ws.seg_hist[klass];
    const uint32_t total = kSizeBuckets * nseg;
    const uint32_t per = (total + 1023) / 1024;
    const uint32_t lo = threadIdx.x * per, hi = min(total, lo + per);
    uint32_t sum = 0;
    for (uint32_t i = lo; i < hi; ++i)
        sum += h[i];
    part[threadIdx.x] = sum;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const uint32_t add = (int)threadIdx.x >= off ? part[threadIdx.x - off] : 0u;
        __syncthreads();
        part[threadIdx.x] += add;
        __syncthreads();
    }
    uint32_t run = part[threadIdx.x] - sum;
    for (uint32_t i = lo; i < hi; ++i) {
        const uint32_t v = h[i];
        h[i] = run;
        run += v;
    }
    if (threadIdx.x == 1023)
        a.ws.counters[kCntCand + klass] = part[1023];
}

// One block per segment: place its candidates with LDS cursors per bucket.
__global__ __launch_bounds__(256) void sort_scatter_kernel(BatchArgs a, int klass)
{
    __shared__ uint32_t cursor[kSizeBuckets];
    const uint32_t seg = blockIdx.x, nseg = gridDim.x;
    if (threadIdx.x < kSizeBuckets)
        cursor[threadIdx.x] = a.ws.seg_hist[klass][threadIdx.x * nseg + seg];
    __syncthreads();
    const uint32_t n = a.ws.seg_count[klass][seg];
    const uint16_t* sz = a.ws.cand_size[klass] + (size_t)seg * a.seg_cap;
    const uint32_t* ix = a.ws.cand_idx[klass] + (size_t)seg * a.seg_cap;
    for (uint32_t i = threadIdx.x; i < n; i += 256) {
        const uint32_t pos = atomicAdd(&cursor[size_key(sz[i])], 1u);
        a.ws.sorted[klass][pos] = ix[i];
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

template <int W, int TM>
__global__ __launch_bounds__(64) void repeat_kernel(BatchArgs a, int klass)
{
    using Geo = Geometry<W>;
    __shared__ uint32_t smem[Geo::kLaneWords * 64];
    __shared__ uint32_t orient[8][64];   // per group: the 8 orientation hashes
    LaneGrid<W, 64> g{smem + threadIdx.x};
    g.clear_all();
    RunState st{0, 0, 0, 0, 0, false};
    WaveTally tally{{0, 0, 0, 0}};

    const int R = a.runs;
    const int groups = 64 / R;
    const int lane = (int)threadIdx.x;
    const int grp = lane / R, run = lane - grp * R;
    const int lead = grp * R;                         // lane making run 0
    const int tail = lead + R - 1;                    // lane making run R-1
    const uint64_t gmask = R == 64 ? ~0ull : ((1ull << R) - 1);
    LaneGrid<W, 64> g0{smem + lead};
    const uint32_t count = a.ws.counters[kCntCand + klass];
    const uint32_t* queue = a.ws.sorted[klass];
    const uint32_t stride = gridDim.x * (uint32_t)groups;

    // static round-robin over the size-sorted queue; the next entry is
    // fetched one iteration ahead
    uint32_t base = blockIdx.x * (uint32_t)groups;
    uint32_t next_idx = 0;
    if (grp < groups && base + (uint32_t)grp < count)
        next_idx = queue[base + grp];
    for (; base < count; base += stride) {
        const bool active = grp < groups && base + (uint32_t)grp < count;
        const uint32_t idx = next_idx;
        if (grp < groups && base + stride + (uint32_t)grp < count)
            next_idx = queue[base + stride + grp];
        Geno gd{0, 0, 0, 0, false};
        int ev = kEvNone;
        if (active) {
            gd = fetch_geno(a, idx);
            const Model<TM> m = build_model<TM>(gd.genome, gd.t, a.bits, a.c);
            ev = run_assembly(m, g, st, gd.grid, run, a.key0, a.key1, (uint32_t)gd.rng_id,
                              (uint32_t)(gd.rng_id >> 32));
        }
        __syncthreads();   // every run's grid is final
        // a witness is a later run that hit an event or ended in another shape
        bool same = true;
        if (active && run > 0 && ev == kEvNone) {
#pragma unroll
            for (int w = 0; w < Geo::kWords; ++w)
                same = same && g.occ(w) == g0.occ(w);
        }
        const bool witness = active && run > 0 && (ev != kEvNone || !same);
        const uint64_t wm = (__ballot(witness) >> lead) & gmask;
        const int first = wm ? (int)__builtin_ctzll(wm) : R;      // R: no witness
        const int wl = lead + (first < R ? first : 0);
        const int w_ev = __shfl(ev, wl);
        const int w_size = __shfl(st.size, wl);
        const int lead_ev = __shfl(ev, lead);
        int cls;
        if (lead_ev == kEvCorrupt || (first < R && w_ev == kEvCorrupt))
            cls = JATAM_INVALID;
        else if (first == R)
            cls = JATAM_DET;
        else
            cls = w_ev == kEvUnbound ? JATAM_UNBOUND
                : w_ev == kEvAmbig   ? JATAM_ND_SITE
                                     : JATAM_ND_RUNS;
        // placements summed over runs 0..first (all R runs if DET)
        const int last = first < R ? first : R - 1;
        const int incl = wave_inclusive_sum(active && run <= last ? st.steps : 0);
        const int steps = __shfl(incl, tail) - __shfl(incl, lead) + __shfl(st.steps, lead);
        const bool det = active && cls == JATAM_DET;
        const int size0 = __shfl(st.size, lead);
        // the group's lanes share the 8 orientation hashes of run 0's shape
        if (det && size0 > 2) {
            uint64_t m8;
            int w8, h8;
            const bool small = shape_bitmap8(g0, gd.grid, m8, w8, h8);
            for (int k = run; k < 8; k += R) {
                if (small) {
                    orient[k][grp] = bitmap_hash8(image8(m8, w8, h8, k));
                } else {
                    const ShapeBox bx = crop(g0, gd.grid);
                    orient[k][grp] = orientation_hash(g0, bx, k);
                }
            }
        }
        __syncthreads();
        const bool done = active && run == 0;
        if (done) {
            jatam_result_t rec;
            if (det) {
                uint32_t h;
                if (size0 <= 2) {
                    h = a.ws.small_hash[size0 - 1];
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
            a.out[idx] = rec;
        }
        tally.add(done, cls);
        __syncthreads();   // orientation slots and grids reused next round
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

template <int W, int TM>
static int blocks_for(int cus)
{
    int a = 0, b = 0;
    hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, first_run_kernel<W, TM>, 64, 0);
    hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, repeat_kernel<W, TM>, 64, 0);
    const int p = a < b ? a : b;
    return (p > 0 ? p : 1) * cus;
}

void batch_persistent_blocks(int cus, int blocks[2][2])
{
    blocks[0][0] = blocks_for<16, 2>(cus);
    blocks[0][1] = blocks_for<16, 4>(cus);
    blocks[1][0] = blocks_for<32, 2>(cus);
    blocks[1][1] = blocks_for<32, 4>(cus);
}

template <int TM>
static void launch_stages(BatchArgs a, const bool classes[2], const int blocks[2][2],
                          hipStream_t stream, hipEvent_t* marks, uint8_t* launched)
{
    constexpr int ti = TM == 2 ? 0 : 1;
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
        const uint32_t nb = (uint32_t)blocks[k][ti];
        const uint64_t nchunks = (uint64_t)(a.n + 63) / 64;
        a.seg_cap = (uint32_t)((nchunks + nb - 1) / nb * 64);
        begin(kStageFirst + 3 * k);
        if (k == 0)
            hipLaunchKernelGGL((first_run_kernel<16, TM>), dim3(nb), dim3(64), 0, stream, a, 0);
        else
            hipLaunchKernelGGL((first_run_kernel<32, TM>), dim3(nb), dim3(64), 0, stream, a, 1);
        end(kStageFirst + 3 * k);
        begin(kStageSort + 3 * k);
        hipLaunchKernelGGL(sort_hist_kernel, dim3(nb), dim3(256), 0, stream, a, k);
        hipLaunchKernelGGL(sort_scan_kernel, dim3(1), dim3(1024), 0, stream, a, k, nb);
        hipLaunchKernelGGL(sort_scatter_kernel, dim3(nb), dim3(256), 0, stream, a, k);
        end(kStageSort + 3 * k);
        begin(kStageRepeat + 3 * k);
        if (k == 0)
            hipLaunchKernelGGL((repeat_kernel<16, TM>), dim3(nb), dim3(64), 0, stream, a, 0);
        else
            hipLaunchKernelGGL((repeat_kernel<32, TM>), dim3(nb), dim3(64), 0, stream, a, 1);
        end(kStageRepeat + 3 * k);
    }
}

int launch_batched(const BatchArgs& a, const bool classes[2], const int blocks[2][2], int tm,
                   hipStream_t stream, hipEvent_t* marks, uint8_t* launched)
{
    if (launched)
        for (int s = 0; s < kStages; ++s)
            launched[s] = 0;
    if (a.n > 0) {
        if (tm == 2)
            launch_stages<2>(a, classes, blocks, stream, marks, launched);
        else
            launch_stages<4>(a, classes, blocks, stream, marks, launched);
    }
    return hipGetLastError() == hipSuccess ? JATAM_OK : JATAM_E_HIP;
}

}  // namespace jatam
