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
    __device__ __forceinline__ uint32_t pend(int p)
    {
        return (word(Geo::kPend + (p >> 3)) >> ((p & 7) * 4)) & 15u;
    }
    __device__ __forceinline__ void set_pend(int p, uint32_t id)
    {
        uint32_t& w = word(Geo::kPend + (p >> 3));
        const int sh = (p & 7) * 4;
        w = (w & ~(15u << sh)) | (id << sh);
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

// Position of the j-th (0-based) set bit of x, j < popcount(x).
__device__ __forceinline__ int select_bit(uint32_t x, uint32_t j)
{
    int pos = 0;
    uint32_t c = __popc(x & 0xFFFFu);
    if (j >= c) { j -= c; x >>= 16; pos += 16; }
    c = __popc(x & 0xFFu);
    if (j >= c) { j -= c; x >>= 8; pos += 8; }
    c = __popc(x & 0xFu);
    if (j >= c) { j -= c; x >>= 4; pos += 4; }
    c = __popc(x & 0x3u);
    if (j >= c) { j -= c; x >>= 2; pos += 2; }
    c = x & 1u;
    if (j >= c) { pos += 1; }
    return pos;
}

// Assembly state of one run, in registers.
struct RunState {
    uint32_t nf;       // frontier size
    uint32_t fsum;     // bit w set: frontier word w may be nonzero
    uint32_t osum;     // bit w set: occupancy word w may be nonzero
    int size;
    int steps;
    bool choice;
};

// The tile `tuple` was just placed at p: check its empty neighbours (§3.2).
template <int W, int B, int TM>
__device__ __forceinline__ int update_site(const Model<TM>& m, LaneGrid<W, B>& g, RunState& st,
                                           int G, int p, uint32_t tuple)
{
    constexpr int kMask = W * W - 1;
    bool unbound = false, ambiguous = false;
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        const uint32_t opt = site_options(m, tuple, d);
        if (opt == 0)
            continue;
        const int delta = d == 0 ? -W : d == 1 ? 1 : d == 2 ? W : -1;
        const int q = (p + delta) & kMask;
        const int qx = q & (W - 1), qy = q >> Geometry<W>::kLogW;
        if (qx >= G - 1 || qy >= G - 1) {
            unbound = true;              // bondable site outside the box
            continue;
        }
        if (g.occupied(q))
            continue;
        const uint32_t id = opt & 15u;
        if ((opt >> 4) >= 2) {
            ambiguous = true;            // two distinct tiles bond here
        } else if (g.on_frontier(q)) {
            ambiguous = ambiguous || g.pend(q) != id;
        } else {
            g.fr(q >> 5) |= 1u << (q & 31);
            g.set_pend(q, id);
            st.fsum |= 1u << (q >> 5);
            st.nf += 1;
        }
    }
    return unbound ? kEvUnbound : ambiguous ? kEvAmbig : kEvNone;
}

// Philox block cache of a run: the 4 words of counter block `block`.
struct DrawCache {
    uint32_t block;
    Words4 words;
};

// Starts a run: clears what the previous run touched, places the seed
// (tile 0, unrotated) at the centre and checks its neighbours.
template <int W, int B, int TM>
__device__ __forceinline__ int run_start(const Model<TM>& m, LaneGrid<W, B>& g, RunState& st,
                                         DrawCache& dc, int G)
{
    for (uint32_t s = st.osum; s; s &= s - 1)
        g.occ(__builtin_ctz(s)) = 0;
    for (uint32_t s = st.fsum; s; s &= s - 1)
        g.fr(__builtin_ctz(s)) = 0;
    st.nf = 0;
    st.fsum = 0;
    st.size = 1;
    st.steps = 0;
    st.choice = false;
    dc.block = 0xFFFFFFFFu;
    const int seed_pos = (G / 2 - 1) * W + (G / 2 - 1);
    g.occ(seed_pos >> 5) = 1u << (seed_pos & 31);
    st.osum = 1u << (seed_pos >> 5);
    return update_site(m, g, st, G, seed_pos, seed_tile(m));
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
template <int W, int B, int TM>
__device__ __forceinline__ int run_step(const Model<TM>& m, LaneGrid<W, B>& g, RunState& st,
                                        DrawCache& dc, int G, int run, uint32_t key0,
                                        uint32_t key1, uint32_t rid_lo, uint32_t rid_hi)
{
    uint32_t j = 0;
    if (st.nf >= 2) {
        st.choice = true;
        const uint32_t blk = (uint32_t)st.steps >> 2;
        if (blk != dc.block) {
            dc.words = philox4x32_10(blk, (uint32_t)run, rid_lo, rid_hi, key0, key1);
            dc.block = blk;
        }
        const int k = st.steps & 3;
        uint32_t u = dc.words.w[0];
        u = k == 1 ? dc.words.w[1] : u;
        u = k == 2 ? dc.words.w[2] : u;
        u = k == 3 ? dc.words.w[3] : u;
        j = __umulhi(u, st.nf);
    }
    // the j-th frontier site in row-major order
    uint32_t fs = st.fsum;
    int w = 0;
    uint32_t fw = 0;
    while (fs != 0) {
        w = __builtin_ctz(fs);
        fw = g.fr(w);
        const uint32_t c = __popc(fw);
        if (j < c)
            break;
        j -= c;
        fs &= fs - 1;
    }
    if (fs == 0)
        return kEvCorrupt;   // nf disagrees with the bitmap: cannot happen
    const int bit = select_bit(fw, j);
    const int p = (w << 5) | bit;
    fw &= ~(1u << bit);
    g.fr(w) = fw;
    if (fw == 0)
        st.fsum &= ~(1u << w);
    st.nf -= 1;

    const uint32_t tuple = oriented_tile(m, (int)g.pend(p));
    g.occ(w) |= 1u << bit;
    st.osum |= 1u << w;
    st.size += 1;
    st.steps += 1;
    return update_site(m, g, st, G, p, tuple);
}

// One run from the seed to completion or to an event.
template <int W, int B, int TM>
__device__ int run_assembly(const Model<TM>& m, LaneGrid<W, B>& g, RunState& st, int G, int run,
                            uint32_t key0, uint32_t key1, uint32_t rid_lo, uint32_t rid_hi)
{
    DrawCache dc;
    int ev = run_start(m, g, st, dc, G);
    while (!run_over(ev, st, G))
        ev = run_step(m, g, st, dc, G, run, key0, key1, rid_lo, rid_hi);
    return ev;
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

// D4-invariant hash of the shape held in OCC, computed by one lane.
template <int W, int B>
__device__ uint32_t shape_hash(LaneGrid<W, B>& g, int G)
{
    const ShapeBox bx = crop(g, G);
    uint32_t hs[8];
#pragma unroll
    for (int k = 0; k < 8; ++k)
        hs[k] = orientation_hash(g, bx, k);
    return combine_orientations(hs);
}

}  // namespace jatam
