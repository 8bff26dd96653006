// jatam_assembly.hpp - one lane's assembly run on gfx950, shared by the plain
// and the pipelined classification kernels.
//
// A lane's grid lives in LDS as
//   OCC   occupancy bitmap, W*W bits
//   FR    frontier bitmap (sites with exactly one admissible tile), W*W bits
//   PEND  the pending tile of every frontier site, 4 bits per cell
// in a lane-interleaved layout (word k of the lane with thread index j at
// smem[k*B + j]), so a wave's 64 lanes always touch 64 consecutive dwords and
// never conflict in a bank, whatever cells they address.
//
// Grid layout.  The bounded (G-1)-square is stored at cells (x, y) in
// [0, G-2]^2 of a W x W torus (W = 16 or 32 >= G), cell index y*W + x.  Its
// ring - the sites just outside the box - is every cell with x >= G-1 or
// y >= G-1: stepping E or S off the box lands on x or y = G-1, and stepping W
// or N off it wraps (mod W*W) onto x or y = W-1.  Cell order y*W + x is the
// row-major frontier order.  Only the words a run touched are cleared for the
// next run (the paper finds 83% of its time in re-initialising grids and
// proposes exactly this, §5.2).
#pragma once

#include "jatam_device.hpp"

namespace jatam {

template <int W>
struct Geometry {
    static_assert(W == 16 || W == 32, "W must be 16 or 32");
    static constexpr int kLogW = W == 16 ? 4 : 5;
    static constexpr int kCells = W * W;
    static constexpr int kWords = kCells / 32;       // bitmap words
    static constexpr int kPendWords = kCells / 8;    // 4-bit cells
    static constexpr int kOcc = 0;
    static constexpr int kFr = kWords;
    static constexpr int kPend = 2 * kWords;
    static constexpr int kLaneWords = 2 * kWords + kPendWords;
};

// Per-lane view of the workgroup's LDS.
template <int W, int B>
struct LaneGrid {
    using Geo = Geometry<W>;
    uint32_t* base;   // &smem[threadIdx.x]

    __device__ __forceinline__ uint32_t& word(int k) { return base[k * B]; }
    __device__ __forceinline__ uint32_t& occ(int w) { return word(Geo::kOcc + w); }
    __device__ __forceinline__ uint32_t& fr(int w) { return word(Geo::kFr + w); }

    __device__ __forceinline__ bool occupied(int p) { return (occ(p >> 5) >> (p & 31)) & 1u; }
    __device__ __forceinline__ bool on_frontier(int p) { return (fr(p >> 5) >> (p & 31)) & 1u; }
    // every word of the lane's grid, PEND included (kernel start)
    __device__ __forceinline__ void clear_all()
    {
        for (int k = 0; k < Geo::kLaneWords; ++k)
            word(k) = 0;
    }
    __device__ __forceinline__ uint32_t& pend_word(int p) { return word(Geo::kPend + (p >> 3)); }
    // LDS atomic OR without return: sets bits with no read on the critical path
    __device__ __forceinline__ static void set_bits(uint32_t& w, uint32_t bits)
    {
        __hip_atomic_fetch_or(&w, bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    __device__ __forceinline__ uint32_t row(int y)
    {
        if constexpr (W == 32) {
            return occ(y);
        } else {
            return (occ(y >> 1) >> ((y & 1) * 16)) & 0xFFFFu;
        }
    }
};

enum { kEvNone = 0, kEvUnbound = 1, kEvAmbig = 2, kEvCorrupt = 3 };

// For one-wave workgroups: LDS writes made by the wave before this point are
// seen by its LDS reads after it.  A wave's LDS operations are performed in
// order, so only the compiler must not move accesses across the point: no
// s_barrier, and no wait for the wave's outstanding global stores, which the
// workgroup-scope fence of __syncthreads adds.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Assembly state of one run, in registers.
struct RunState {
    uint32_t nf;       // frontier size
    uint32_t fsum;     // bit w set: frontier word w may be nonzero
    uint32_t osum;     // bit w set: occupancy word w may be nonzero
    int size;
    int steps;
    bool choice;
    // 32 x 32 layout: frontier sites per group of four rows, 16-bit fields,
    // groups 0-3 in gca and 4-7 in gcb (the frontier select's first level)
    uint64_t gca = 0, gcb = 0;
};

// 32 x 32 layout: the frontier count of cell q's group of four rows goes up
// (add) or down by one.  Nothing in the 16 x 16 layout.
template <int W>
__device__ __forceinline__ void frontier_group_add(RunState& st, int q, bool add)
{
    if constexpr (W == 32) {
        const int grp = q >> 7;
        const uint64_t one = 1ull << (16 * (grp & 3));
        const uint64_t d = add ? one : 0ull - one;
        st.gca += grp < 4 ? d : 0ull;
        st.gcb += grp < 4 ? 0ull : d;
    }
}

// The tile `tuple` was just placed at p: check its empty neighbours (§3.2).
// A bondable site on the ring means the structure leaves the box; a site
// that two distinct tiles can fill is ambiguous; otherwise a free site with
// one admissible tile joins the frontier with that tile pending.  All reads
// of the four neighbours are issued before any of them is used.
//
// Invariant: the PEND nibble of a free cell is zero unless the cell is on
// the frontier, so a new pending tile is written with one LDS atomic OR.  An
// occupied cell keeps the tile placed there in its nibble.
//
// `added`, if given, receives bit d for every direction d whose site joined
// the frontier (the movelist traversal pushes those sites).
//
// The check only looks at the neighbours' own bits and nibbles, so the
// words holding them may be read before p itself is marked (NeighbourWords,
// read by the step together with p's pending word).
struct NeighbourWords {
    int q[4];                          // the cells N, E, S, W of p
    uint32_t ow[4], fw[4], pw[4];      // their occupancy, frontier, pending words
};

template <int W, int B>
__device__ __forceinline__ NeighbourWords read_neighbours(LaneGrid<W, B>& g, int p)
{
    constexpr int kMask = W * W - 1;
    NeighbourWords nw;
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        const int delta = d == 0 ? -W : d == 1 ? 1 : d == 2 ? W : -1;
        nw.q[d] = (p + delta) & kMask;
        nw.ow[d] = g.occ(nw.q[d] >> 5);
        nw.fw[d] = g.fr(nw.q[d] >> 5);
        nw.pw[d] = g.pend_word(nw.q[d]);
    }
    return nw;
}

template <int W, int B, class Src>
__device__ __forceinline__ int update_site(const Src& m, LaneGrid<W, B>& g, RunState& st,
                                           int G, int p, uint32_t tuple,
                                           const NeighbourWords& nw,
                                           uint32_t* added = nullptr)
{
    const int* const q = nw.q;
    const uint32_t* const ow = nw.ow;
    const uint32_t* const fw = nw.fw;
    const uint32_t* const pw = nw.pw;
    SiteOpts opt[4];
#pragma unroll
    for (int d = 0; d < 4; ++d)
        opt[d] = m.options_split(tuple, d);
    // p lies in the box ([0, G-2]^2), so a neighbour is on the ring exactly
    // when p is on the box's edge in that direction (N and W wrap round the
    // torus onto row or column W-1)
    const int px = p & (W - 1), py = p >> Geometry<W>::kLogW;
    bool unbound = false, ambiguous = false;
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        const bool ring = d == 0 ? py == 0 : d == 1 ? px == G - 2 : d == 2 ? py == G - 2 : px == 0;
        const uint32_t bit = (uint32_t)q[d] & 31u;
        const bool has = opt[d].has;
        const bool free = ((ow[d] >> bit) & 1u) == 0;
        const bool live = has && !ring && free;
        const uint32_t id = opt[d].id;
        const bool multi = opt[d].multi;
        const bool in_f = ((fw[d] >> bit) & 1u) != 0;
        const uint32_t sh = ((uint32_t)q[d] & 7u) * 4u;
        const uint32_t pending = (pw[d] >> sh) & 15u;
        // plain (not short-circuit) logic: every operand is at hand, and
        // lane masks combine with scalar instructions
        unbound = unbound | (has & ring);
        ambiguous = ambiguous | (live & (multi | (in_f & (pending != id))));
        if (live && !multi && !in_f) {
            LaneGrid<W, B>::set_bits(g.fr(q[d] >> 5), 1u << bit);
            LaneGrid<W, B>::set_bits(g.pend_word(q[d]), id << sh);
            st.fsum |= 1u << (q[d] >> 5);
            st.nf += 1;
            frontier_group_add<W>(st, q[d], true);
            if (added != nullptr)
                *added |= 1u << d;
        }
    }
    return unbound ? kEvUnbound : ambiguous ? kEvAmbig : kEvNone;
}

template <int W, int B, class Src>
__device__ __forceinline__ int update_site(const Src& m, LaneGrid<W, B>& g, RunState& st,
                                           int G, int p, uint32_t tuple,
                                           uint32_t* added = nullptr)
{
    return update_site(m, g, st, G, p, tuple, read_neighbours(g, p), added);
}

// Philox block cache of a run: the 4 words of counter block `block`.  Kept
// as four scalars, never an array: an array picked by a run-time index ends
// up in scratch memory, one memory round trip per step.
struct DrawCache {
    uint32_t block;
    uint32_t w0, w1, w2, w3;

    __device__ __forceinline__ void reset() { block = 0xFFFFFFFFu; }
    __device__ __forceinline__ void fill(const Words4& v)
    {
        w0 = v.w[0];
        w1 = v.w[1];
        w2 = v.w[2];
        w3 = v.w[3];
    }
    // word k (0..3) by two register selects
    __device__ __forceinline__ uint32_t word(uint32_t k) const
    {
        const uint32_t lo = (k & 1u) ? w1 : w0;
        const uint32_t hi = (k & 1u) ? w3 : w2;
        return (k & 2u) ? hi : lo;
    }
    // random word s of run `run`: word s mod 4 of counter block s / 4
    __device__ __forceinline__ uint32_t draw(uint32_t s, int run, uint32_t key0, uint32_t key1,
                                             uint32_t rid_lo, uint32_t rid_hi)
    {
        const uint32_t blk = s >> 2;
        if (blk != block) {
            fill(philox4x32_10(blk, (uint32_t)run, rid_lo, rid_hi, key0, key1));
            block = blk;
        }
        return word(s & 3u);
    }
};

// Two Philox blocks of a run, one of even and one of odd block index, so
// that a block can be computed before the run reaches it.  A wave whose
// lanes run out of phase computes blocks whenever any lane needs one; with
// one block per lane that happens on most steps with few lanes active.  With
// two, every lane fills the block it lacks (its current one, else the next)
// at each such point, so all lanes share one computation about every fourth
// step (see prefetch).  draw() still computes a missing block itself.
struct DrawPair {
    uint32_t te, to;                    // block index held (all ones: none)
    uint32_t e0, e1, e2, e3;            // the even block
    uint32_t o0, o1, o2, o3;            // the odd block

    // Members are only ever combined by value selects: choosing between two
    // members as lvalues (or storing through such a choice) makes the
    // compiler address the struct by a run-time offset, in scratch memory.
    __device__ __forceinline__ static uint32_t pick(bool c, uint32_t x, uint32_t y)
    {
        return c ? x : y;
    }
    __device__ __forceinline__ void reset()
    {
        te = 0xFFFFFFFFu;
        to = 0xFFFFFFFFu;
    }
    // te only ever holds an even index and to an odd one
    __device__ __forceinline__ bool has(uint32_t blk) const { return te == blk || to == blk; }
    __device__ __forceinline__ void put(uint32_t blk, const Words4& v)
    {
        const bool odd = (blk & 1u) != 0;
        to = pick(odd, blk, to);
        o0 = pick(odd, v.w[0], o0);
        o1 = pick(odd, v.w[1], o1);
        o2 = pick(odd, v.w[2], o2);
        o3 = pick(odd, v.w[3], o3);
        te = pick(odd, te, blk);
        e0 = pick(odd, e0, v.w[0]);
        e1 = pick(odd, e1, v.w[1]);
        e2 = pick(odd, e2, v.w[2]);
        e3 = pick(odd, e3, v.w[3]);
    }
    // the block this lane should compute now, given its next draw index s:
    // block s/4 if missing, else block s/4 + 1 if missing; false if neither
    __device__ __forceinline__ bool wanted(uint32_t s, uint32_t& blk) const
    {
        const uint32_t b = s >> 2;
        const bool cur = !has(b);
        blk = cur ? b : b + 1u;
        return cur || !has(b + 1u);
    }
    __device__ __forceinline__ uint32_t draw(uint32_t s, int run, uint32_t key0, uint32_t key1,
                                             uint32_t rid_lo, uint32_t rid_hi)
    {
        const uint32_t blk = s >> 2;
        if (!has(blk))
            put(blk, philox4x32_10(blk, (uint32_t)run, rid_lo, rid_hi, key0, key1));
        const bool odd = (blk & 1u) != 0;
        const uint32_t k = s & 3u;
        const uint32_t x0 = pick(odd, o0, e0), x1 = pick(odd, o1, e1);
        const uint32_t x2 = pick(odd, o2, e2), x3 = pick(odd, o3, e3);
        const uint32_t lo = pick((k & 1u) != 0, x1, x0);
        const uint32_t hi = pick((k & 1u) != 0, x3, x2);
        return pick((k & 2u) != 0, hi, lo);
    }
};

// A DrawPair whose caller runs prefetch_draws before every step: the block
// of the next draw is then always present, so draw() reads it without the
// fallback computation (and the step loop holds one copy of the generator).
struct PrefetchedDraws {
    DrawPair& dp;
    __device__ __forceinline__ uint32_t draw(uint32_t s, int, uint32_t, uint32_t, uint32_t,
                                             uint32_t) const
    {
        const uint32_t blk = s >> 2;
        const bool odd = (blk & 1u) != 0;
        const uint32_t k = s & 3u;
        const uint32_t x0 = DrawPair::pick(odd, dp.o0, dp.e0), x1 = DrawPair::pick(odd, dp.o1, dp.e1);
        const uint32_t x2 = DrawPair::pick(odd, dp.o2, dp.e2), x3 = DrawPair::pick(odd, dp.o3, dp.e3);
        const uint32_t lo = DrawPair::pick((k & 1u) != 0, x1, x0);
        const uint32_t hi = DrawPair::pick((k & 1u) != 0, x3, x2);
        return DrawPair::pick((k & 2u) != 0, hi, lo);
    }
};

// Wave-wide Philox fill for lanes that keep a DrawPair: when the next draw
// of any stepping lane lacks its block, every stepping lane computes the
// block it lacks, so one pass of the generator serves the whole wave.  Call
// with every lane of the wave present (it takes a ballot).
__device__ __forceinline__ void prefetch_draws(DrawPair& dp, bool stepping, const RunState& st,
                                               int run, uint32_t key0, uint32_t key1,
                                               uint32_t rid_lo, uint32_t rid_hi)
{
    const uint32_t s = (uint32_t)st.steps;
    const bool need = stepping && st.nf >= 2 && !dp.has(s >> 2);
    if (__ballot(need) == 0)
        return;
    uint32_t blk = 0;
    if (stepping && dp.wanted(s, blk))
        dp.put(blk, philox4x32_10(blk, (uint32_t)run, rid_lo, rid_hi, key0, key1));
}

// Clears what the previous run touched and places the seed (tile 0,
// unrotated) at the centre; returns the seed's cell.
template <int W, int B, class Draws>
__device__ __forceinline__ int run_clear(LaneGrid<W, B>& g, RunState& st, Draws& dc, int G)
{
    // occupied cells keep their tiles in PEND, and a run that ended on an
    // event leaves frontier cells (with their PEND nibbles) behind: clear all
    for (uint32_t s = st.osum; s; s &= s - 1) {
        const int w = __builtin_ctz(s);
        g.occ(w) = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k)
            g.word(Geometry<W>::kPend + 4 * w + k) = 0;
    }
    for (uint32_t s = st.fsum; s; s &= s - 1) {
        const int w = __builtin_ctz(s);
        g.fr(w) = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k)
            g.word(Geometry<W>::kPend + 4 * w + k) = 0;
    }
    st.nf = 0;
    st.fsum = 0;
    st.gca = 0;
    st.gcb = 0;
    st.size = 1;
    st.steps = 0;
    st.choice = false;
    dc.reset();
    const int seed_pos = (G / 2 - 1) * W + (G / 2 - 1);
    g.occ(seed_pos >> 5) = 1u << (seed_pos & 31);
    st.osum = 1u << (seed_pos >> 5);
    return seed_pos;
}

// Starts a run: clears what the previous run touched, places the seed
// (tile 0, unrotated) at the centre and checks its neighbours.
template <int W, int B, class Src, class Draws>
__device__ __forceinline__ int run_start(const Src& m, LaneGrid<W, B>& g, RunState& st,
                                         Draws& dc, int G)
{
    const int seed_pos = run_clear(g, st, dc, G);
    return update_site(m, g, st, G, seed_pos, m.seed());
}

// run_start for a seed whose four site codes are already known (byte d of
// `seed_opts` is the options code of the seed's site in direction d).  In
// the cleared grid every neighbour of the seed is free and off the
// frontier, so update_site reduces to the ring test and the frontier
// insertions: no grid reads, no options lookups.
template <int W, int B, class Draws>
__device__ __forceinline__ int run_start_known(LaneGrid<W, B>& g, RunState& st, Draws& dc,
                                               int G, uint32_t seed_opts)
{
    constexpr int kMask = W * W - 1;
    const int p = run_clear(g, st, dc, G);
    bool unbound = false, ambiguous = false;
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        const int delta = d == 0 ? -W : d == 1 ? 1 : d == 2 ? W : -1;
        const int q = (p + delta) & kMask;
        const uint32_t opt = (seed_opts >> (8 * d)) & 0x3Fu;
        const int qx = q & (W - 1), qy = q >> Geometry<W>::kLogW;
        const bool ring = qx >= G - 1 || qy >= G - 1;
        const bool has = opt != 0;
        const bool multi = (opt >> 4) >= 2;
        unbound = unbound || (has && ring);
        ambiguous = ambiguous || (has && !ring && multi);
        if (has && !ring && !multi) {
            const uint32_t sh = ((uint32_t)q & 7u) * 4u;
            LaneGrid<W, B>::set_bits(g.fr(q >> 5), 1u << (q & 31));
            LaneGrid<W, B>::set_bits(g.pend_word(q), (opt & 15u) << sh);
            st.fsum |= 1u << (q >> 5);
            st.nf += 1;
            frontier_group_add<W>(st, q, true);
        }
    }
    return unbound ? kEvUnbound : ambiguous ? kEvAmbig : kEvNone;
}

// A run is over once an event happened or the frontier is empty.  Every step
// fills a new cell of the box, so (G-1)^2 steps also end it (never reached).
__device__ __forceinline__ bool run_over(int ev, const RunState& st, int G)
{
    return ev != kEvNone || st.nf == 0 || st.steps >= (G - 1) * (G - 1);
}

// One step: draw the frontier site of rank floor(u*|F|/2^32) in row-major
// order (u = Philox word `steps` of this run's stream; no draw is needed with
// one site), place its pending tile and check the new neighbours.
template <int W, int B, class Src, class Draws>
__device__ __forceinline__ int run_step(const Src& m, LaneGrid<W, B>& g, RunState& st,
                                        Draws& dc, int G, int run, uint32_t key0,
                                        uint32_t key1, uint32_t rid_lo, uint32_t rid_hi)
{
    uint32_t j = 0;
    if (st.nf >= 2) {
        st.choice = true;
        j = __umulhi(dc.draw((uint32_t)st.steps, run, key0, key1, rid_lo, rid_hi), st.nf);
    }
    // the j-th frontier site in row-major order
    int w = 0;
    uint32_t fw = 0;
    if constexpr (W == 16) {
        // 8 frontier words, no loop: inclusive prefix counts p0..p7; the
        // word holding site j is the number of prefixes <= j; the word and
        // its exclusive prefix are picked by binary trees of selects on that
        // index (scalars throughout: an array picked at run time would go to
        // scratch memory)
        const uint32_t f0 = g.fr(0), f1 = g.fr(1), f2 = g.fr(2), f3 = g.fr(3);
        const uint32_t f4 = g.fr(4), f5 = g.fr(5), f6 = g.fr(6), f7 = g.fr(7);
        const uint32_t p0 = __popc(f0), p1 = p0 + __popc(f1), p2 = p1 + __popc(f2);
        const uint32_t p3 = p2 + __popc(f3), p4 = p3 + __popc(f4), p5 = p4 + __popc(f5);
        const uint32_t p6 = p5 + __popc(f6), p7 = p6 + __popc(f7);
        if (p7 != st.nf)
            return kEvCorrupt;   // nf disagrees with the bitmap: cannot happen
        // p_k <= j exactly when p_k - (j + 1) is negative (all values < 2^9):
        // sign bits summed, no compare-and-select chains
        const uint32_t j1 = j + 1u;
        const uint32_t wi = ((p0 - j1) >> 31) + ((p1 - j1) >> 31) + ((p2 - j1) >> 31) +
                            ((p3 - j1) >> 31) + ((p4 - j1) >> 31) + ((p5 - j1) >> 31) +
                            ((p6 - j1) >> 31);
        const bool b0 = (wi & 1u) != 0, b1 = (wi & 2u) != 0, b2 = (wi & 4u) != 0;
        const uint32_t fa = b0 ? f1 : f0, fb = b0 ? f3 : f2, fc = b0 ? f5 : f4, fd = b0 ? f7 : f6;
        const uint32_t ea = b0 ? p0 : 0u, eb = b0 ? p2 : p1, ec = b0 ? p4 : p3, ed = b0 ? p6 : p5;
        const uint32_t fab = b1 ? fb : fa, fcd = b1 ? fd : fc;
        const uint32_t eab = b1 ? eb : ea, ecd = b1 ? ed : ec;
        fw = b2 ? fcd : fab;
        j -= b2 ? ecd : eab;
        w = (int)wi;
    } else {
        // two levels, one round of LDS reads: the frontier counts of the 8
        // groups of four rows (registers, 16-bit fields) pick the group, its
        // four words the row.  Inclusive prefix sums of the group counts:
        uint64_t pa = st.gca;
        pa += pa << 16;
        pa += pa << 32;
        uint64_t pb = st.gcb;
        pb += pb << 16;
        pb += pb << 32;
        pb += (pa >> 48) * 0x0001000100010001ull;   // groups 4-7 follow groups 0-3
        if ((uint32_t)(pb >> 48) != st.nf)
            return kEvCorrupt;   // the counts disagree with nf: cannot happen
        // the group holding site j is the number of prefixes <= j: a field
        // p (< 2^15, as j + 1 is) has bit 15 of (p | 2^15) - (j + 1) set
        // exactly when p > j, with no borrow between fields
        constexpr uint64_t kHigh = 0x8000800080008000ull;
        const uint64_t jj = (uint64_t)(j + 1u) * 0x0001000100010001ull;
        const uint32_t grp = 8u - (uint32_t)__popcll(((pa | kHigh) - jj) & kHigh) -
                             (uint32_t)__popcll(((pb | kHigh) - jj) & kHigh);
        const uint32_t gm = (grp - 1u) & 7u;   // the group before, if any
        const uint64_t below = gm < 4u ? pa : pb;
        j -= grp == 0u ? 0u : (uint32_t)(below >> (16u * (gm & 3u))) & 0xFFFFu;
        const int w0 = (int)grp * 4;
        const uint32_t f0 = g.fr(w0), f1 = g.fr(w0 + 1), f2 = g.fr(w0 + 2), f3 = g.fr(w0 + 3);
        const uint32_t c0 = __popc(f0), c1 = c0 + __popc(f1), c2 = c1 + __popc(f2);
        const uint32_t j1 = j + 1u;
        const uint32_t wi = ((c0 - j1) >> 31) + ((c1 - j1) >> 31) + ((c2 - j1) >> 31);
        const bool b0 = (wi & 1u) != 0, b1 = (wi & 2u) != 0;
        fw = b1 ? (b0 ? f3 : f2) : (b0 ? f1 : f0);
        j -= b1 ? (b0 ? c2 : c1) : (b0 ? c0 : 0u);
        w = w0 + (int)wi;
        if (j >= (uint32_t)__popc(fw))
            return kEvCorrupt;   // the counts disagree with the bitmap: cannot happen
    }
    // the j-th set bit of the word: j is below the word's frontier count,
    // nearly always 0..2, so clearing the lowest bit j times beats a
    // fixed binary search
    uint32_t rest = fw;
    for (uint32_t k = 0; k < j; ++k)
        rest &= rest - 1u;
    const int bit = __builtin_ctz(rest);
    const int p = (w << 5) | bit;
    // p's pending word and its neighbours' words in one round of LDS reads,
    // issued before p leaves the frontier and is marked occupied (the
    // neighbour check does not look at p's bits)
    const uint32_t pw = g.pend_word(p);
    const NeighbourWords nw = read_neighbours(g, p);
    fw &= ~(1u << bit);
    g.fr(w) = fw;
    if (fw == 0)
        st.fsum &= ~(1u << w);
    st.nf -= 1;
    frontier_group_add<W>(st, p, false);

    // place the pending tile (its nibble stays: the cell keeps its tile)
    const uint32_t sh = ((uint32_t)p & 7u) * 4u;
    const uint32_t tuple = m.oriented((int)((pw >> sh) & 15u));
    LaneGrid<W, B>::set_bits(g.occ(w), 1u << bit);
    st.osum |= 1u << w;
    st.size += 1;
    st.steps += 1;
    return update_site(m, g, st, G, p, tuple, nw);
}

// One run from the seed to completion or to an event.
template <int W, int B, class Src>
__device__ __forceinline__ int run_assembly(const Src& m, LaneGrid<W, B>& g, RunState& st, int G,
                                            int run,
                            uint32_t key0, uint32_t key1, uint32_t rid_lo, uint32_t rid_hi)
{
    DrawCache dc;
    int ev = run_start(m, g, st, dc, G);
    while (!run_over(ev, st, G))
        ev = run_step(m, g, st, dc, G, run, key0, key1, rid_lo, rid_hi);
    return ev;
}

// True if the shape held in OCC (tiles in PEND) is forced: at every occupied
// cell, the tiles that its occupied neighbours bond to are exactly that
// cell's own tile.  For the final shape of a run that ended without an
// event this means every growth order places the same tile in every cell
// of the shape and nowhere else (a site outside the shape that any shape
// cell bonds to would have stayed on the frontier, or ended the run as
// UNBOUND), and never meets an ambiguous site: every run ends in this shape.
// The seed cell's nibble is 0, the id of the unrotated seed tile.
template <int W, int B, class Src>
__device__ __forceinline__ bool shape_is_forced(const Src& m, LaneGrid<W, B>& g,
                                                const RunState& st)
{
    constexpr int kMask = W * W - 1;
    bool forced = true;
    for (uint32_t s = st.osum; s != 0 && forced; s &= s - 1) {
        const int w = __builtin_ctz(s);
        for (uint32_t cells = g.occ(w); cells != 0 && forced; cells &= cells - 1) {
            const int p = (w << 5) | __builtin_ctz(cells);
            const uint32_t id = (g.pend_word(p) >> ((uint32_t)(p & 7) * 4u)) & 15u;
#pragma unroll
            for (int d = 0; d < 4; ++d) {
                const int delta = d == 0 ? -W : d == 1 ? 1 : d == 2 ? W : -1;
                const int q = (p + delta) & kMask;
                if (!g.occupied(q))
                    continue;
                const uint32_t nq = (g.pend_word(q) >> ((uint32_t)(q & 7) * 4u)) & 15u;
                // options of the site in direction d + 2 of q's tile: cell p
                const SiteOpts o = m.options_split(m.oriented((int)nq), (d + 2) & 3);
                if (o.has && (o.multi || o.id != id))
                    forced = false;
            }
        }
    }
    return forced;
}

// Bounding box of the shape held in OCC (cropping, App. F.6).
struct ShapeBox {
    int xmin, ymin, w, h;
};

template <int W, int B>
__device__ __forceinline__ ShapeBox crop(LaneGrid<W, B>& g, int G)
{
    int ymin = W, ymax = -1;
    uint32_t cols = 0;
    for (int y = 0; y < G - 1; ++y) {
        const uint32_t r = g.row(y);
        if (r) {
            ymin = y < ymin ? y : ymin;
            ymax = y;
            cols |= r;
        }
    }
    const int xmin = __builtin_ctz(cols);
    const int xmax = 31 - __builtin_clz(cols);
    return ShapeBox{xmin, ymin, xmax - xmin + 1, ymax - ymin + 1};
}

// True if the shape held in OCC (tiles in PEND), left by a run that ended
// without an event, is guarded: every run ends in it.  Call an edge from an
// occupied cell q to an occupied neighbour p good when q's tile admits
// exactly p's tile at p, and a conflict when it admits anything else there.
// The shape is guarded when, for every conflict q -> p with p not the seed,
// every path of good edges from the seed to q passes through p.
//
// Why that suffices: in any growth order a tile is placed only from the
// frontier, where it arrived over an edge from a tile placed before it.  By
// induction over the placements, every tile so far is the shape's own tile
// in a cell of the shape, reached from the seed over good edges through
// cells placed before it; so a conflicting q is never placed while p is
// empty, and q's wrong option at p never counts.  No site outside the shape
// can be bonded to (run 0 would have grown there or met an event), so the
// run places the shape exactly, never meets an event, and places all of it
// (every cell of the shape has a good edge from a cell placed before it in
// run 0).  With no conflicts this is shape_is_forced.
//
// The flood fills run on 64-bit bitmaps of the shape's bounding box, which
// must fit 8 x 8; a larger shape is tested with shape_is_forced instead.
template <int W, int B, class Src>
__device__ __forceinline__ bool shape_is_guarded(const Src& m, LaneGrid<W, B>& g,
                                                 const RunState& st, int G)
{
    constexpr int kMask = W * W - 1;
    const ShapeBox bx = crop(g, G);
    if (bx.w > 8 || bx.h > 8)
        return shape_is_forced(m, g, st);
    // per cell p of the 8 x 8 frame, bit (y - ymin) * 8 + (x - xmin):
    // good_d / conf_d: the edge into p from its neighbour in direction d
    uint64_t shape = 0, good0 = 0, good1 = 0, good2 = 0, good3 = 0;
    uint64_t conf0 = 0, conf1 = 0, conf2 = 0, conf3 = 0;
    for (uint32_t s = st.osum; s != 0; s &= s - 1) {
        const int w = __builtin_ctz(s);
        for (uint32_t cells = g.occ(w); cells != 0; cells &= cells - 1) {
            const int p = (w << 5) | __builtin_ctz(cells);
            const int fx = (p & (W - 1)) - bx.xmin, fy = (p >> Geometry<W>::kLogW) - bx.ymin;
            const uint64_t bit = 1ull << (fy * 8 + fx);
            shape |= bit;
            const uint32_t id = (g.pend_word(p) >> ((uint32_t)(p & 7) * 4u)) & 15u;
#pragma unroll
            for (int d = 0; d < 4; ++d) {
                const int delta = d == 0 ? -W : d == 1 ? 1 : d == 2 ? W : -1;
                const int q = (p + delta) & kMask;
                if (!g.occupied(q))
                    continue;
                const uint32_t nq = (g.pend_word(q) >> ((uint32_t)(q & 7) * 4u)) & 15u;
                // options of the site in direction d + 2 of q's tile: cell p
                const SiteOpts o = m.options_split(m.oriented((int)nq), (d + 2) & 3);
                const bool good = o.has & !o.multi & (o.id == id);
                const bool conf = o.has & !good;
                const uint64_t gb = good ? bit : 0ull, cb = conf ? bit : 0ull;
                if (d == 0) { good0 |= gb; conf0 |= cb; }
                else if (d == 1) { good1 |= gb; conf1 |= cb; }
                else if (d == 2) { good2 |= gb; conf2 |= cb; }
                else { good3 |= gb; conf3 |= cb; }
            }
        }
    }
    const int seed = (G / 2 - 1) * W + (G / 2 - 1);
    const uint64_t seed_bit =
        1ull << (((seed >> Geometry<W>::kLogW) - bx.ymin) * 8 + ((seed & (W - 1)) - bx.xmin));
    // conflicts into the seed never count: the seed is placed first
    uint64_t todo = (conf0 | conf1 | conf2 | conf3) & ~seed_bit;
    bool guarded = true;
    for (; todo != 0 && guarded; todo &= todo - 1) {
        const uint64_t pb = todo & (~todo + 1);
        // the conflicting neighbours of p: N is 8 bits down, S 8 up, E 1 up, W 1 down
        const uint64_t src = ((conf0 & pb) >> 8) | ((conf2 & pb) << 8) | ((conf1 & pb) << 1) |
                             ((conf3 & pb) >> 1);
        const uint64_t allowed = shape & ~pb;
        uint64_t reach = seed_bit, prev = 0;
        while (reach != prev && (reach & src) == 0) {
            prev = reach;
            reach |= (((reach << 8) & good0) | ((reach >> 1) & good1) | ((reach >> 8) & good2) |
                      ((reach << 1) & good3)) & allowed;
        }
        guarded = (reach & src) == 0;
    }
    return guarded;
}

// One-at-a-time hash of the cropped shape in orientation k of the dihedral
// group: bit 2 transposes, bit 0 mirrors x, bit 1 mirrors y.  Cells are
// listed in row-major order of the oriented frame, each as the bytes x, y
// (§3.3, App. F.4).
template <int W, int B>
__device__ __forceinline__ uint32_t orientation_hash(LaneGrid<W, B>& g, const ShapeBox& bx, int k)
{
    const bool transpose = k & 4, flip_x = k & 1, flip_y = k & 2;
    const int wt = transpose ? bx.h : bx.w, ht = transpose ? bx.w : bx.h;
    uint32_t hv = 0;
    for (int yp = 0; yp < ht; ++yp) {
        for (int xp = 0; xp < wt; ++xp) {
            int u = transpose ? yp : xp;
            int v = transpose ? xp : yp;
            u = flip_x ? bx.w - 1 - u : u;
            v = flip_y ? bx.h - 1 - v : v;
            if ((g.row(bx.ymin + v) >> (bx.xmin + u)) & 1u) {
                hv = oaat_add(hv, (uint32_t)xp);
                hv = oaat_add(hv, (uint32_t)yp);
            }
        }
    }
    return oaat_finish(hv);
}

// The 8 orientation hashes sorted ascending, hashed again as 32
// little-endian bytes: the same value for every image of the shape.
__device__ __forceinline__ uint32_t combine_orientations(uint32_t hs[8])
{
#pragma unroll
    for (int pass = 0; pass < 8; ++pass) {
#pragma unroll
        for (int i = pass & 1; i + 1 < 8; i += 2) {
            const uint32_t a = hs[i], b = hs[i + 1];
            hs[i] = a < b ? a : b;
            hs[i + 1] = a < b ? b : a;
        }
    }
    uint32_t hv = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int b = 0; b < 4; ++b)
            hv = oaat_add(hv, (hs[i] >> (8 * b)) & 0xFFu);
    return oaat_finish(hv);
}

// ---------------------------------------------------------------------------
// Register-only D4 hash for shapes whose bounding box fits 8 x 8: the cropped
// shape is a 64-bit bitmap, bit 8*y + x, so row-major cell order is ascending
// bit order.  The 8 images are the 4 mirror combinations of the shape and of
// its transpose, each re-anchored at (0, 0).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t bytes_reversed(uint64_t v)
{
    const uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
    return ((uint64_t)__builtin_bswap32(lo) << 32) | __builtin_bswap32(hi);
}

// Mirror x: reverse the bits of every byte, then shift the shape back to x=0.
__device__ __forceinline__ uint64_t mirror_x8(uint64_t v, int w)
{
    const uint32_t lo = __builtin_bitreverse32((uint32_t)v);
    const uint32_t hi = __builtin_bitreverse32((uint32_t)(v >> 32));
    // bit-reversing each half also reversed byte order: undo that
    const uint64_t r = ((uint64_t)__builtin_bswap32(hi) << 32) | __builtin_bswap32(lo);
    return r >> (8 - w);
}

// Mirror y: reverse the row order, then shift the shape back to y=0.
__device__ __forceinline__ uint64_t mirror_y8(uint64_t v, int h)
{
    return bytes_reversed(v) >> (8 * (8 - h));
}

// Transpose of an 8 x 8 bit matrix (bit 8*y + x -> bit 8*x + y).
__device__ __forceinline__ uint64_t transpose8(uint64_t x)
{
    uint64_t t;
    t = (x ^ (x >> 7)) & 0x00AA00AA00AA00AAull;
    x = x ^ t ^ (t << 7);
    t = (x ^ (x >> 14)) & 0x0000CCCC0000CCCCull;
    x = x ^ t ^ (t << 14);
    t = (x ^ (x >> 28)) & 0x00000000F0F0F0F0ull;
    x = x ^ t ^ (t << 28);
    return x;
}

// OAAT over (x, y) of every set cell in ascending bit (row-major) order.
__device__ __forceinline__ uint32_t bitmap_hash8(uint64_t v)
{
    uint32_t h = 0;
    while (v != 0) {
        const uint32_t b = (uint32_t)__builtin_ctzll(v);
        v &= v - 1;
        h = oaat_add(h, b & 7u);
        h = oaat_add(h, b >> 3);
    }
    return oaat_finish(h);
}

// Image k (0..7) of the w x h shape m: bit 2 transposes, bit 0 mirrors x,
// bit 1 mirrors y (in the transposed frame when transposed).
__device__ __forceinline__ uint64_t image8(uint64_t m, int w, int h, int k)
{
    uint64_t v = m;
    int ww = w, hh = h;
    if (k & 4) {
        v = transpose8(v);
        ww = h;
        hh = w;
    }
    if (k & 1)
        v = mirror_x8(v, ww);
    if (k & 2)
        v = mirror_y8(v, hh);
    return v;
}

// The cropped shape held in OCC as an 8 x 8 bitmap; false if it does not fit.
template <int W, int B>
__device__ __forceinline__ bool shape_bitmap8(LaneGrid<W, B>& g, int G, uint64_t& m, int& w,
                                              int& h)
{
    const ShapeBox bx = crop(g, G);
    w = bx.w;
    h = bx.h;
    if (bx.w > 8 || bx.h > 8)
        return false;
    m = 0;
    for (int y = 0; y < bx.h; ++y)
        m |= (uint64_t)((g.row(bx.ymin + y) >> bx.xmin) & 0xFFu) << (8 * y);
    return true;
}

// Width and height of an anchored 8 x 8 bitmap (not empty).
__device__ __forceinline__ void bitmap8_dims(uint64_t m, int& w, int& h)
{
    uint32_t x = (uint32_t)m | (uint32_t)(m >> 32);
    x |= x >> 16;
    x |= x >> 8;
    w = 32 - __builtin_clz(x & 0xFFu);
    h = (63 - __builtin_clzll(m)) / 8 + 1;
}

// The cropped shape as an anchored 8 x 8 bitmap for W = 16, from the 8 OCC
// words at once: row masks and the column union give the bounding box; each
// word (two rows) is shifted to xmin and packed to two bytes; the 8-row
// window at ymin is cut from the 16 packed rows.  False if the box exceeds
// 8 x 8.
template <int B>
__device__ __forceinline__ bool shape_bitmap8_w16(LaneGrid<16, B>& g, uint64_t& m, int& x0,
                                                  int& y0)
{
    uint32_t o[8];
#pragma unroll
    for (int k = 0; k < 8; ++k)
        o[k] = g.occ(k);
    uint32_t rows = 0, cols = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        rows |= (uint32_t)((o[k] & 0xFFFFu) != 0) << (2 * k);
        rows |= (uint32_t)((o[k] >> 16) != 0) << (2 * k + 1);
        cols |= o[k];
    }
    cols = (cols | (cols >> 16)) & 0xFFFFu;
    const int ymin = __builtin_ctz(rows), ymax = 31 - __builtin_clz(rows);
    const int xmin = __builtin_ctz(cols), xmax = 31 - __builtin_clz(cols);
    x0 = xmin;
    y0 = ymin;
    if (xmax - xmin >= 8 || ymax - ymin >= 8)
        return false;
    uint32_t r[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint32_t a = (o[2 * q] >> xmin) & 0x00FF00FFu;
        const uint32_t b = (o[2 * q + 1] >> xmin) & 0x00FF00FFu;
        r[q] = ((a | (a >> 8)) & 0xFFFFu) | (((b | (b >> 8)) & 0xFFFFu) << 16);
    }
    // bytes ymin .. ymin+7 of r[0..3] (rows past 15 are empty)
    const int q = ymin >> 2, sh = 8 * (ymin & 3);
    const uint32_t a0 = q == 0 ? r[0] : q == 1 ? r[1] : q == 2 ? r[2] : r[3];
    const uint32_t a1 = q == 0 ? r[1] : q == 1 ? r[2] : q == 2 ? r[3] : 0u;
    const uint32_t a2 = q == 0 ? r[2] : q == 1 ? r[3] : 0u;
    const uint32_t lo = (uint32_t)((((uint64_t)a1 << 32) | a0) >> sh);
    const uint32_t hi = (uint32_t)((((uint64_t)a2 << 32) | a1) >> sh);
    m = ((uint64_t)hi << 32) | lo;
    return true;
}

template <int B>
__device__ __forceinline__ bool shape_bitmap8_w16(LaneGrid<16, B>& g, uint64_t& m)
{
    int x0, y0;
    return shape_bitmap8_w16(g, m, x0, y0);
}

// The cropped shape as an anchored 8 x 8 bitmap, whatever W.
template <int W, int B>
__device__ __forceinline__ bool shape_key8(LaneGrid<W, B>& g, int G, uint64_t& m)
{
    if constexpr (W == 16) {
        return shape_bitmap8_w16(g, m);
    } else {
        int w, h;
        return shape_bitmap8(g, G, m, w, h);
    }
}

// ---------------------------------------------------------------------------
// A run's final shape packed into 16 bytes, for the proof stage to check
// without replaying the run: .x/.y the anchored 8 x 8 bitmap (bit 8y + x),
// .z/.w a 64-bit word holding the tile nibble of every cell in ascending bit
// order (at most kPackedCells cells) and, in bits 58..63, the seed's bit.
// All ones in .z/.w: the shape does not fit (larger box or more cells).
// ---------------------------------------------------------------------------
constexpr int kPackedCells = 14;

__device__ __forceinline__ bool packed_shape_valid(const uint4& v)
{
    return !(v.z == 0xFFFFFFFFu && v.w == 0xFFFFFFFFu);
}

template <int W, int B>
__device__ __forceinline__ uint4 pack_shape(LaneGrid<W, B>& g, int G, int size)
{
    const uint4 none = make_uint4(0u, 0u, 0xFFFFFFFFu, 0xFFFFFFFFu);
    if (size > kPackedCells)
        return none;
    if constexpr (W == 16) {
        // the bitmap from the OCC words in registers; then the two PEND words
        // of each of the box's rows, all reads issued before any is used
        uint64_t m;
        int x0, y0;
        if (!shape_bitmap8_w16(g, m, x0, y0))
            return none;
        uint32_t lo[8], hi[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int y = y0 + r < 16 ? y0 + r : 15;
            lo[r] = g.word(Geometry<16>::kPend + 2 * y);
            hi[r] = g.word(Geometry<16>::kPend + 2 * y + 1);
        }
        uint64_t tiles = 0;
        int k = 0;
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            // the row's 8 nibbles from column x0 on
            const uint32_t row = (uint32_t)((((uint64_t)hi[r] << 32) | lo[r]) >> (4 * x0));
            for (uint32_t bits = (uint32_t)(m >> (8 * r)) & 0xFFu; bits != 0;
                 bits &= bits - 1, ++k) {
                const int x = __builtin_ctz(bits);
                tiles |= (uint64_t)((row >> (4 * x)) & 15u) << (4 * k);
            }
        }
        const int sc = G / 2 - 1;
        tiles |= (uint64_t)((sc - y0) * 8 + (sc - x0)) << 58;
        return make_uint4((uint32_t)m, (uint32_t)(m >> 32), (uint32_t)tiles,
                          (uint32_t)(tiles >> 32));
    }
    const ShapeBox bx = crop(g, G);
    if (bx.w > 8 || bx.h > 8)
        return none;
    uint64_t m = 0;
    for (int y = 0; y < bx.h; ++y)
        m |= (uint64_t)((g.row(bx.ymin + y) >> bx.xmin) & 0xFFu) << (8 * y);
    uint64_t tiles = 0;
    int k = 0;
    for (uint64_t cells = m; cells != 0; cells &= cells - 1, ++k) {
        const int b = __builtin_ctzll(cells);
        const int p = (bx.ymin + (b >> 3)) * W + bx.xmin + (b & 7);
        const uint64_t nib = (g.pend_word(p) >> ((uint32_t)(p & 7) * 4u)) & 15u;
        tiles |= nib << (4 * k);
    }
    const int sc = G / 2 - 1;
    tiles |= (uint64_t)((sc - bx.ymin) * 8 + (sc - bx.xmin)) << 58;
    return make_uint4((uint32_t)m, (uint32_t)(m >> 32), (uint32_t)tiles,
                      (uint32_t)(tiles >> 32));
}

// shape_is_guarded for a packed shape (same edges, same test), from
// registers: cell b's tile is nibble popcount(m below b) of the tile word.
template <class Src>
__device__ __forceinline__ bool packed_shape_is_guarded(const Src& src, const uint4& v)
{
    const uint64_t shape = ((uint64_t)v.y << 32) | v.x;
    const uint64_t word = ((uint64_t)v.w << 32) | v.z;
    const uint64_t tiles = word & ((1ull << 56) - 1);
    const uint64_t seed_bit = 1ull << (int)(word >> 58);
    uint64_t good0 = 0, good1 = 0, good2 = 0, good3 = 0;
    uint64_t conf0 = 0, conf1 = 0, conf2 = 0, conf3 = 0;
    for (uint64_t cells = shape; cells != 0; cells &= cells - 1) {
        const int b = __builtin_ctzll(cells);
        const uint64_t bit = 1ull << b;
        const uint32_t id = (uint32_t)(tiles >> (4 * __popcll(shape & (bit - 1)))) & 15u;
        const int x = b & 7, y = b >> 3;
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            const bool inside = d == 0 ? y > 0 : d == 1 ? x < 7 : d == 2 ? y < 7 : x > 0;
            const int qb = b + (d == 0 ? -8 : d == 1 ? 1 : d == 2 ? 8 : -1);
            if (!inside || ((shape >> (qb & 63)) & 1ull) == 0ull)
                continue;
            const uint32_t nq =
                (uint32_t)(tiles >> (4 * __popcll(shape & ((1ull << qb) - 1)))) & 15u;
            // options of the site in direction d + 2 of q's tile: cell b
            const SiteOpts o = src.options_split(src.oriented((int)nq), (d + 2) & 3);
            const bool good = o.has & !o.multi & (o.id == id);
            const bool conf = o.has & !good;
            const uint64_t gb = good ? bit : 0ull, cb = conf ? bit : 0ull;
            if (d == 0) { good0 |= gb; conf0 |= cb; }
            else if (d == 1) { good1 |= gb; conf1 |= cb; }
            else if (d == 2) { good2 |= gb; conf2 |= cb; }
            else { good3 |= gb; conf3 |= cb; }
        }
    }
    uint64_t todo = (conf0 | conf1 | conf2 | conf3) & ~seed_bit;
    bool guarded = true;
    for (; todo != 0 && guarded; todo &= todo - 1) {
        const uint64_t pb = todo & (~todo + 1);
        const uint64_t src_bits = ((conf0 & pb) >> 8) | ((conf2 & pb) << 8) |
                                  ((conf1 & pb) << 1) | ((conf3 & pb) >> 1);
        const uint64_t allowed = shape & ~pb;
        uint64_t reach = seed_bit, prev = 0;
        while (reach != prev && (reach & src_bits) == 0) {
            prev = reach;
            reach |= (((reach << 8) & good0) | ((reach >> 1) & good1) | ((reach >> 8) & good2) |
                      ((reach << 1) & good3)) & allowed;
        }
        guarded = (reach & src_bits) == 0;
    }
    return guarded;
}

// D4 hash of a shape given as an anchored 8 x 8 bitmap, by one lane.
__device__ __forceinline__ uint32_t bitmap8_shape_hash(uint64_t m)
{
    int w, h;
    bitmap8_dims(m, w, h);
    uint32_t hs[8];
#pragma unroll
    for (int k = 0; k < 8; ++k)
        hs[k] = bitmap_hash8(image8(m, w, h, k));
    return combine_orientations(hs);
}

// Per-wave cache of D4 hashes in LDS, keyed by the exact anchored 8 x 8
// bitmap of a shape (which determines the shape, so a hit returns exactly
// the hash the shape has).  N entries {bitmap lo, bitmap hi, hash, 0},
// direct mapped; an all-zero key marks an empty entry (no shape is empty).
// Lanes read it freely; entries are written one lane at a time.  For
// workgroups of one wave (insert synchronises the workgroup).
template <int N>
struct ShapeCache {
    static_assert((N & (N - 1)) == 0, "N must be a power of two");
    uint4* e;

    __device__ __forceinline__ static uint32_t slot(uint64_t m)
    {
        const uint32_t x = (uint32_t)m * 0x9E3779B1u ^ (uint32_t)(m >> 32) * 0x85EBCA77u;
        return (x ^ (x >> 15)) & (N - 1);
    }
    __device__ __forceinline__ void clear(int lane)
    {
        for (int i = lane; i < N; i += 64)
            e[i] = make_uint4(0u, 0u, 0u, 0u);
    }
    __device__ __forceinline__ bool lookup(uint64_t m, uint32_t& hash) const
    {
        const uint4 v = e[slot(m)];
        hash = v.z;
        return v.x == (uint32_t)m && v.y == (uint32_t)(m >> 32);
    }
    // Called by the whole wave of a one-wave workgroup: every lane with
    // `want` stores its entry, in lane order (a later lane with the same
    // slot overwrites), then the wave's later lookups see the entries.
    __device__ __forceinline__ void insert(bool want, uint64_t m, uint32_t hash, int lane)
    {
        uint64_t pending = __ballot(want);
        if (pending == 0)
            return;
        for (; pending != 0; pending &= pending - 1) {
            if (lane == __builtin_ctzll(pending))
                e[slot(m)] = make_uint4((uint32_t)m, (uint32_t)(m >> 32), hash, 0u);
        }
        wave_lds_sync();
    }
};

// The 4 rotation hashes sorted ascending, hashed again as 16 little-endian
// bytes (§3.3's rotation-invariant hash).
__device__ __forceinline__ uint32_t combine_rotations(uint32_t hs[4])
{
#pragma unroll
    for (int pass = 0; pass < 4; ++pass) {
#pragma unroll
        for (int i = pass & 1; i + 1 < 4; i += 2) {
            const uint32_t a = hs[i], b = hs[i + 1];
            hs[i] = a < b ? a : b;
            hs[i + 1] = a < b ? b : a;
        }
    }
    uint32_t hv = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int b = 0; b < 4; ++b)
            hv = oaat_add(hv, (hs[i] >> (8 * b)) & 0xFFu);
    return oaat_finish(hv);
}

// C4-invariant hash of the shape held in OCC: orientations 0 (identity),
// 3 (both mirrors: the half turn), 5 and 6 (a transpose and one mirror: the
// quarter turns) of the dihedral images, computed by one lane.
template <int W, int B>
__device__ uint32_t shape_hash_c4(LaneGrid<W, B>& g, int G)
{
    constexpr int kRot[4] = {0, 3, 5, 6};
    uint32_t hs[4];
    uint64_t m;
    int w, h;
    if (shape_bitmap8(g, G, m, w, h)) {
#pragma unroll
        for (int k = 0; k < 4; ++k)
            hs[k] = bitmap_hash8(image8(m, w, h, kRot[k]));
    } else {
        const ShapeBox bx = crop(g, G);
#pragma unroll
        for (int k = 0; k < 4; ++k)
            hs[k] = orientation_hash(g, bx, kRot[k]);
    }
    return combine_rotations(hs);
}

// ---------------------------------------------------------------------------
// The movelist traversal (§3.2): the frontier sites on a LIFO stack of cell
// indices (bytes, after the lane's grid words, 16 x 16 layout only).  A site
// that joins the frontier (directions N, E, S, W of each update) goes to slot
// floor(u (len + 1) / 2^32) counted from the bottom of the len sites on the
// stack, u the run's next word (word d for its d-th draw; none while the
// stack is empty); every step places the site on top.
// ---------------------------------------------------------------------------
constexpr int kStackWords = 64;   // 256 one-byte entries >= the 225 cells of the box

template <int B>
struct LaneStack {
    uint32_t* base;   // the lane's first stack word (word k at base[k * B])

    __device__ __forceinline__ uint8_t* byte(int i)
    {
        return reinterpret_cast<uint8_t*>(base + (i >> 2) * B) + (i & 3);
    }
    __device__ __forceinline__ int get(int i) { return *byte(i); }
    __device__ __forceinline__ void set(int i, int v) { *byte(i) = (uint8_t)v; }
};

// Pushes the sites of the directions in `added` (in order N, E, S, W) next to
// p; len is the stack's length before them.  Returns the new length.
template <int W, int B, class Draws>
__device__ __forceinline__ uint32_t movelist_push(LaneStack<B>& stk, uint32_t len, int p,
                                                  uint32_t added, Draws& dc, uint32_t& draws,
                                                  bool& choice, int run, uint32_t key0,
                                                  uint32_t key1, uint32_t rid_lo, uint32_t rid_hi)
{
    constexpr int kMask = W * W - 1;
    for (int d = 0; d < 4; ++d) {
        if (((added >> d) & 1u) == 0u)
            continue;
        const int delta = d == 0 ? -W : d == 1 ? 1 : d == 2 ? W : -1;
        const int q = (p + delta) & kMask;
        uint32_t pos = 0;
        if (len > 0u) {
            pos = __umulhi(dc.draw(draws, run, key0, key1, rid_lo, rid_hi), len + 1u);
            draws += 1;
            choice = true;
        }
        for (uint32_t i = len; i > pos; --i)
            stk.set((int)i, stk.get((int)i - 1));
        stk.set((int)pos, q);
        len += 1;
    }
    return len;
}

// One run with the movelist traversal, from the seed to completion or an
// event (st.nf is the stack's length throughout).
template <int W, int B, class Src>
__device__ __forceinline__ int run_assembly_lifo(const Src& m, LaneGrid<W, B>& g,
                                                 LaneStack<B>& stk, RunState& st, int G, int run,
                                                 uint32_t key0, uint32_t key1, uint32_t rid_lo,
                                                 uint32_t rid_hi)
{
    DrawCache dc;
    const int seed_pos = run_clear(g, st, dc, G);
    uint32_t draws = 0, added = 0;
    bool choice = false;
    int ev = update_site(m, g, st, G, seed_pos, m.seed(), &added);
    movelist_push<W>(stk, 0u, seed_pos, added, dc, draws, choice, run, key0, key1, rid_lo,
                     rid_hi);
    while (ev == kEvNone && st.nf > 0 && st.steps < (G - 1) * (G - 1)) {
        const int p = stk.get((int)st.nf - 1);
        st.nf -= 1;
        const int w = p >> 5;
        const uint32_t fw = g.fr(w) & ~(1u << (p & 31));
        g.fr(w) = fw;
        if (fw == 0)
            st.fsum &= ~(1u << w);
        const uint32_t pw = g.pend_word(p);
        const uint32_t sh = ((uint32_t)p & 7u) * 4u;
        const uint32_t tuple = m.oriented((int)((pw >> sh) & 15u));
        LaneGrid<W, B>::set_bits(g.occ(w), 1u << (p & 31));
        st.osum |= 1u << w;
        st.size += 1;
        st.steps += 1;
        const uint32_t len = st.nf;
        added = 0;
        ev = update_site(m, g, st, G, p, tuple, &added);
        movelist_push<W>(stk, len, p, added, dc, draws, choice, run, key0, key1, rid_lo, rid_hi);
    }
    st.choice = choice;
    return ev;
}

// D4-invariant hash of the shape held in OCC, computed by one lane.
template <int W, int B>
__device__ uint32_t shape_hash(LaneGrid<W, B>& g, int G)
{
    uint32_t hs[8];
    uint64_t m;
    int w, h;
    if (shape_bitmap8(g, G, m, w, h)) {
#pragma unroll
        for (int k = 0; k < 8; ++k)
            hs[k] = bitmap_hash8(image8(m, w, h, k));
    } else {
        const ShapeBox bx = crop(g, G);
#pragma unroll
        for (int k = 0; k < 8; ++k)
            hs[k] = orientation_hash(g, bx, k);
    }
    return combine_orientations(hs);
}

}  // namespace jatam
