// jatam_internal.hpp - launch parameters and device workspace shared by the
// library's kernels and its C-ABI layer (not part of the public header).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/jatam.h"

namespace jatam {

// Validated, pre-digested arguments of one classification call.
struct Params {
    int t;            // tiles per genotype
    int c;            // colours
    int bits;         // log2(c)
    int genome_bits;  // 4 * t * bits
    int grid;         // G
    int runs;         // R
    uint32_t key0;    // Philox key = seed
    uint32_t key1;
};

int launch_plain(const uint64_t* genomes, uint64_t first, int64_t n, const Params& prm,
                 jatam_result_t* out, hipStream_t stream);

// ---------------------------------------------------------------------------
// Pipelined path.  Grid class 0 = G <= 16 (16 x 16 torus), 1 = G <= 32.
// ---------------------------------------------------------------------------
enum {
    kCntCand = 0,     // [2] DET candidates per grid class (written by the sort)
    kCntWords = 16,
};
constexpr int kSizeBuckets = 64;    // run-0 size buckets of the repeat queue

// Device memory of a jatam_batch_t, sized for max_n genotypes per call and a
// persistent grid of at most max_blocks one-wave blocks.
struct DeviceWorkspace {
    uint32_t* counters;       // kCntWords
    uint32_t* seg_count[2];   // [max_blocks] candidates staged by each wave
    uint32_t* seg_hist[2];    // [kSizeBuckets * max_blocks] bucket-major counts
    uint32_t* cand_idx[2];    // [max_n + 64 * (max_blocks + 1)] per-wave segments
    uint16_t* cand_size[2];   // same layout: run-0 sizes
    uint32_t* sorted[2];      // [max_n] candidates, largest size first
    uint32_t* small_hash;     // [2]: D4 hash of the monomer and of the domino
};

struct BatchArgs {
    const uint64_t* genomes;        // list mode, or nullptr
    const jatam_item_t* items;      // item mode, or nullptr
    uint64_t first;                 // range mode: genome i = first + i
    int64_t n;
    int t, grid;                    // uniform t and G (range and list modes)
    int c, bits, runs;
    uint32_t key0, key1;
    int refill;                     // idle lanes that trigger a refill (1..64)
    uint32_t seg_cap;               // staging slots per wave (set per launch)
    jatam_result_t* out;
    unsigned long long* tally;      // nullptr or [4], accumulated
    DeviceWorkspace ws;
};

// Pipeline stages, in launch order (timing hook): three per grid class.
enum {
    kStageFirst = 0,    // + 3 * grid class
    kStageSort = 1,     // + 3 * grid class
    kStageRepeat = 2,   // + 3 * grid class
    kStages = 6,
};

// blocks[grid class][TM == 2 ? 0 : 1]: persistent grid of the stage kernels.
// When `marks` is not null, an event is recorded on the stream before stage
// s (marks[2s]) and after it (marks[2s+1]), and launched[s] is set.
int batch_init_small_hash(uint32_t* small_hash, hipStream_t stream);
void batch_persistent_blocks(int cus, int blocks[2][2]);
int launch_batched(const BatchArgs& a, const bool classes[2], const int blocks[2][2], int tm,
                   hipStream_t stream, hipEvent_t* marks, uint8_t* launched);

}  // namespace jatam
