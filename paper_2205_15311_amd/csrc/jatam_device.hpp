// jatam_device.hpp - device building blocks of JaTAM assembly on gfx950.
//
// Everything here is integer arithmetic in registers; nothing is shared with
// the CPU oracle.  The pieces:
//   philox4x32_10   counter-based generator (Salmon et al., SC'11) that
//                   replaces the paper's cuRAND XORWOW (§3)
//   oaat_*          Jenkins one-at-a-time hash (App. F.4), on unsigned bytes
//   Model           a decoded genotype: tiles, their rotations, duplicate /
//                   symmetric orientations merged (§3.2), and the bonding
//                   options of every oriented tile (interaction rule of
//                   App. B.2: colours bond in adjacent pairs 1-2, 3-4, ...)
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace jatam {

// ---------------------------------------------------------------------------
// Philox4x32-10: ten rounds of the published S-P network; the key is bumped
// by the two Weyl constants between rounds.
// ---------------------------------------------------------------------------
struct Words4 {
    uint32_t w[4];
};

__device__ __forceinline__ Words4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                                uint32_t c3, uint32_t k0, uint32_t k1)
{
    constexpr uint32_t kMul0 = 0xD2511F53u, kMul1 = 0xCD9E8D57u;
    constexpr uint32_t kWeyl0 = 0x9E3779B9u, kWeyl1 = 0xBB67AE85u;
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        // each 32 x 32 -> 64-bit product as one multiply (v_mad_u64_u32)
        // rather than separate high and low halves
        const uint64_t p0 = (uint64_t)kMul0 * c0, p1 = (uint64_t)kMul1 * c2;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        const uint32_t n0 = hi1 ^ c1 ^ k0;
        const uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += kWeyl0;
        k1 += kWeyl1;
    }
    return Words4{{c0, c1, c2, c3}};
}

// ---------------------------------------------------------------------------
// One-at-a-time hash, split into its per-byte mix and its final avalanche.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t oaat_add(uint32_t h, uint32_t byte)
{
    h += byte;
    h += h << 10;
    h ^= h >> 6;
    return h;
}

__device__ __forceinline__ uint32_t oaat_finish(uint32_t h)
{
    h += h << 3;
    h ^= h >> 11;
    h += h << 15;
    return h;
}

// ---------------------------------------------------------------------------
// A decoded genotype of at most TM tiles (TM = 2 or 4).
//
// Oriented tile k = 4*i + r is tile i turned clockwise by r quarter turns; it
// is held as a 16-bit word of four nibbles, side d (N=0, E=1, S=2, W=3) in
// bits 4d..4d+3.  For every side s the colours that all 4*TM oriented tiles
// show on s are packed as nibble k of side_col(s), so one SWAR comparison
// finds every oriented tile that shows a given colour there.  `reps` has bit
// 4k+3 set for each k that is the first oriented tile with its colour tuple:
// duplicates and symmetric orientations collapse onto that representative.
// With TM = 2 every word is 32 bits, with TM = 4 64 bits.
// ---------------------------------------------------------------------------
template <int TM>
struct Model {
    static_assert(TM == 2 || TM == 4, "TM must be 2 or 4");
    using Word = typename std::conditional<TM == 2, uint32_t, uint64_t>::type;
    static constexpr int kOriented = 4 * TM;
    static constexpr Word kOnes = (Word)0x1111111111111111ull;
    static constexpr Word kLow3 = (Word)0x7777777777777777ull;

    Word tiles;          // tile i in bits 16i..16i+15, nibble d = colour of side d
    // nibble k = colour oriented tile k shows on side s; four scalars rather
    // than an array, so that a side chosen at run time stays in registers
    Word cols0, cols1, cols2, cols3;
    Word reps;           // bit 4k+3 set for representative oriented tiles
    int c;               // colour count

    // by value selects: a choice between the members as lvalues lets the
    // compiler address the struct by a run-time offset, in scratch memory
    __device__ __forceinline__ static Word pick(bool c, Word x, Word y) { return c ? x : y; }
    __device__ __forceinline__ Word side_col(int s) const
    {
        return pick(s < 2, pick(s == 0, cols0, cols1), pick(s == 2, cols2, cols3));
    }
};

__device__ __forceinline__ uint32_t rotate_tile(uint32_t tile, int r)
{
    // side d shows the colour of side (d - r) mod 4: nibbles move up by r
    const uint32_t s = 4u * (uint32_t)r;
    return ((tile << s) | (tile >> ((16u - s) & 15u))) & 0xFFFFu;
}

// Nibbles of a 16-bit tile word in reverse order (side 3 first).
__device__ __forceinline__ uint32_t reverse_nibbles16(uint32_t t)
{
    return ((t & 0xFu) << 12) | ((t & 0xF0u) << 4) | ((t >> 4) & 0xF0u) | ((t >> 12) & 0xFu);
}

template <int TM>
__device__ __forceinline__ Model<TM> build_model(uint64_t genome, int t, int bits, int c)
{
    using M = Model<TM>;
    using Word = typename M::Word;
    M m;
    const uint32_t cmask = (uint32_t)c - 1u;
    uint32_t tile[TM];
#pragma unroll
    for (int i = 0; i < TM; ++i) {
        uint32_t w = 0;
        if (i < t) {
#pragma unroll
            for (int d = 0; d < 4; ++d) {
                const int shift = bits * (4 * t - 1 - (4 * i + d));
                w |= (uint32_t)((genome >> shift) & cmask) << (4 * d);
            }
        }
        tile[i] = w;
    }
    m.tiles = 0;
#pragma unroll
    for (int i = 0; i < TM; ++i)
        m.tiles |= (Word)tile[i] << (16 * i);
    // side s of rotation r shows colour (s - r) mod 4: over r = 0..3 that is
    // the tile's nibbles reversed, rotated by s + 1
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        Word col = 0;
#pragma unroll
        for (int i = 0; i < TM; ++i)
            col |= (Word)rotate_tile(reverse_nibbles16(tile[i]), (s + 1) & 3) << (16 * i);
        if (s == 0)
            m.cols0 = col;
        else if (s == 1)
            m.cols1 = col;
        else if (s == 2)
            m.cols2 = col;
        else
            m.cols3 = col;
    }
    // representatives: the first orientation of each distinct colour tuple.
    // Rotation r of a tile repeats rotation 0 iff the tile has r-fold symmetry;
    // a later tile in the orbit of an earlier one repeats all of its tuples.
    Word reps = 0;
#pragma unroll
    for (int i = 0; i < TM; ++i) {
        const uint32_t r1 = rotate_tile(tile[i], 1), r2 = rotate_tile(tile[i], 2);
        const bool sym4 = r1 == tile[i];
        const bool sym2 = r2 == tile[i];
        uint32_t own = sym4 ? 0x1u : sym2 ? 0x3u : 0xFu;     // rotations kept
        bool repeated = i >= t;
#pragma unroll
        for (int i2 = 0; i2 < i; ++i2) {
            const uint32_t u = tile[i2];
            repeated = repeated || (i2 < t && (tile[i] == u || r1 == u || r2 == u ||
                                               rotate_tile(tile[i], 3) == u));
        }
        own = repeated ? 0u : own;
        // bit 4k+3 for k = 4i + r, r in own
        const uint32_t bitsr = ((own & 1u) << 3) | ((own & 2u) << 6) | ((own & 4u) << 9) |
                               ((own & 8u) << 12);
        reps |= (Word)bitsr << (16 * i);
    }
    m.reps = reps;
    m.c = c;
    return m;
}

// Colour tuple of oriented tile k: a shift, never an indexed load.
template <int TM>
__device__ __forceinline__ uint32_t oriented_tile(const Model<TM>& m, int k)
{
    const uint32_t w = (uint32_t)(m.tiles >> (16 * (k >> 2))) & 0xFFFFu;
    return rotate_tile(w, k & 3);
}

// Colour tuple of the seed: tile 0, unrotated.
template <int TM>
__device__ __forceinline__ uint32_t seed_tile(const Model<TM>& m)
{
    return (uint32_t)m.tiles & 0xFFFFu;
}

// Colour k in every nibble of a model word (k < 16): the byte kk copied to
// all four bytes by a byte permute.  (Written as k * 0x11111111 it becomes a
// full 32-bit multiply, a quarter-rate instruction.)
template <class Word>
__device__ __forceinline__ Word nibble_splat(uint32_t k)
{
    const uint32_t b = k | (k << 4);
    const uint32_t w = __builtin_amdgcn_perm(b, b, 0u);   // selector 0: byte 0 everywhere
    if constexpr (sizeof(Word) == 8)
        return ((uint64_t)w << 32) | w;
    else
        return w;
}

// Bonding options of the empty site next to a placed tile (colour tuple
// `tuple`) in direction d: the distinct representatives that show the
// partner of the tile's side-d colour on their side facing back.  Returns
// min(count, 2) in bits 4..5 and the lowest representative id in bits 0..3
// (0 when nothing bonds).  No branches: a colour without a partner masks
// the match instead.
// The representatives behind site_options: bit 4k+3 of the result is set
// for each representative k that bonds.
template <int TM>
__device__ __forceinline__ typename Model<TM>::Word site_match(const Model<TM>& m, uint32_t tuple,
                                                               int d)
{
    using M = Model<TM>;
    using Word = typename M::Word;
    const int x = (int)((tuple >> (4 * d)) & 15u);
    // partner colour: 1<->2, 3<->4, ...; 0 and a last odd colour have none
    const int p = ((x + 1) ^ 1) - 1;
    const bool bonds = p >= 0 && p < m.c;
    const Word v = m.side_col((d + 2) & 3) ^ nibble_splat<Word>((uint32_t)p & 15u);
    // high bit of each nibble set iff the nibble is nonzero (no carries escape)
    const Word nonzero = v | ((v & M::kLow3) + M::kLow3);
    return bonds ? (~nonzero & m.reps) : (Word)0;
}

// site_options as its three parts, without packing them into a code: any
// representative bonds, two or more do, the lowest one's id (meaningless
// when none does).
struct SiteOpts {
    bool has, multi;
    uint32_t id;
};

template <int TM>
__device__ __forceinline__ SiteOpts site_options_split(const Model<TM>& m, uint32_t tuple, int d)
{
    const typename Model<TM>::Word match = site_match(m, tuple, d);
    SiteOpts o;
    o.has = match != 0;
    o.multi = (match & (match - 1)) != 0;
    // the top bit is representative 4 TM - 1's: or-ing it in changes no
    // lowest set bit and keeps the count of trailing zeros defined
    if constexpr (TM == 2)
        o.id = (uint32_t)__builtin_ctz((uint32_t)match | 0x80000000u) >> 2;
    else
        o.id = (uint32_t)__builtin_ctzll((uint64_t)match | (1ull << 63)) >> 2;
    return o;
}

template <int TM>
__device__ __forceinline__ uint32_t site_options(const Model<TM>& m, uint32_t tuple, int d)
{
    using Word = typename Model<TM>::Word;
    const Word match = site_match(m, tuple, d);
    const Word lowest = match != 0 ? match : (Word)1;   // ctz of 0 is undefined
    uint32_t id;
    if constexpr (TM == 2)
        id = (uint32_t)__builtin_ctz((uint32_t)lowest) >> 2;
    else
        id = (uint32_t)__builtin_ctzll((uint64_t)lowest) >> 2;
    const uint32_t count = (match & (match - 1)) ? 2u : 1u;
    return match != 0 ? ((count << 4) | id) : 0u;
}

// ---------------------------------------------------------------------------
// Sources of bond options for the assembly loop.  Both give, for a placed
// tile's colour tuple and a direction d, the options code of site_options;
// the seed's tuple; and the tuple of oriented tile k.
// ---------------------------------------------------------------------------
// Options found by the SWAR comparison on every call.
template <int TM>
struct ModelSource {
    Model<TM> m;

    __device__ __forceinline__ uint32_t options(uint32_t tuple, int d) const
    {
        return site_options(m, tuple, d);
    }
    __device__ __forceinline__ SiteOpts options_split(uint32_t tuple, int d) const
    {
        return site_options_split(m, tuple, d);
    }
    __device__ __forceinline__ uint32_t seed() const { return seed_tile(m); }
    __device__ __forceinline__ uint32_t oriented(int k) const { return oriented_tile(m, k); }
};

// Options read from the genotype's bond table (c <= 8): byte x of side[d]
// is site_options(m, x << 4d, d), the code of shown colour x on side d.  d
// is a compile-time constant at every call and x only selects a shift, so
// the table stays in registers (a run-time index into an array, or a choice
// between two of its elements, would put it in scratch memory).
template <int TM>
struct TableSource {
    Model<TM> m;
    uint64_t side[4];

    __device__ __forceinline__ uint32_t options(uint32_t tuple, int d) const
    {
        const uint32_t x = (tuple >> (4 * d)) & 7u;
        return (uint32_t)(side[d] >> (8u * x)) & 0x3Fu;
    }
    __device__ __forceinline__ SiteOpts options_split(uint32_t tuple, int d) const
    {
        const uint32_t code = options(tuple, d);
        return SiteOpts{code != 0, (code >> 4) >= 2, code & 15u};
    }
    __device__ __forceinline__ uint32_t seed() const { return seed_tile(m); }
    __device__ __forceinline__ uint32_t oriented(int k) const { return oriented_tile(m, k); }
};

// Word j (0..7) of the bond table: the low (j even) or high half of side[j / 2].
template <int TM>
__device__ __forceinline__ uint32_t bond_table_word(const Model<TM>& m, int j)
{
    const int d = j >> 1, x0 = 4 * (j & 1);
    uint32_t w = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b)
        w |= site_options(m, (uint32_t)(x0 + b) << (4 * d), d) << (8 * b);
    return w;
}

}  // namespace jatam
