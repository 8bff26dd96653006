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
int launch_variant(const uint64_t* genomes, uint64_t first, int64_t n, const Params& prm,
                   int variant, jatam_result_t* out, hipStream_t stream);

// ---------------------------------------------------------------------------
// Pipelined path.  Grid class 0 = G <= 16 (16 x 16 torus), 1 = G <= 32.
// ---------------------------------------------------------------------------
enum {
    kCntCand = 0,     // [2] DET candidates per grid class (written by the sort)
    kCntDiff = 2,     // record comparison flag of the autotuner
    kCntSlice = 3,    // slice counter of a graph-replayed enumeration
    kCntCandAll = 4,  // [2] candidates before the forced-shape proof
    kCntOverflow = 6, // items that left the 16 x 16 window (rerun in 32 x 32 grids)
    kCntRepeat2 = 9,  // [2] candidates left for the second repeat pass
    kCntWords = 16,
};
constexpr int kSizeBuckets = 64;    // run-0 size buckets of the repeat queue
constexpr int kMaxClaimChunks = 8;  // most 64-item chunks one first-run claim may take
constexpr int kRepeatFirstRuns = 4; // runs per candidate in the first of two repeat passes
constexpr int kScanBlock = 1024;    // histogram entries per block of the size scan
// Chunk claims of the first-run kernel and of the fused proof + first repeat
// pass kernel: eight counters per grid class and stage (one per XCD), each
// in a 256-byte block of its own (counters that share a block serialise
// their atomics).
constexpr int kClaimCounters = 8;
constexpr int kClaimStride = 64;   // words between two counters
constexpr int kMaxScanBlocks = 1024;

// Entries of the candidate staging arrays for calls of up to max_n items on
// at most max_blocks first-run waves: nb waves of ceil(chunks / nb) dealt-out
// chunks and one claim each, a claim being at most chunks / (16 nb) chunks
// (claims are made only where every wave gets at least 16 chunks), so at
// most 64 (chunks + nb) + 4 chunks <= max_n + max_n / 16 + 64 (max_blocks + 2).
inline size_t staging_entries(size_t max_n, size_t max_blocks)
{
    return max_n + max_n / 16 + 64 * (max_blocks + 2);
}

// Device memory of a jatam_batch_t, sized for max_n genotypes per call and a
// persistent grid of at most max_blocks one-wave blocks.
struct DeviceWorkspace {
    uint32_t* counters;       // kCntWords
    uint32_t* run_claim;      // [2 * kClaimCounters * kClaimStride]: first-run claim
                              // counter x of class k at word (k * 8 + x) * kClaimStride
    uint32_t* queue_claim;    // the same for the fused proof kernel's queue chunks
    uint32_t* seg_count[2];   // [max_blocks] candidates staged by each wave
    uint32_t* seg_hist[2];    // [kSizeBuckets * max_blocks] bucket-major counts
    uint32_t* scan_sums[2];   // [kMaxScanBlocks] block totals of the histogram scan
    uint32_t* chunk_cnt[2];   // [max_n / 64 + 1] kept candidates per queue chunk, and
                              // ([1]) items per input chunk that left the 16 x 16 window
    uint32_t* chunk_sums[2];  // [max_n / 64 / kScanBlock + 1] block totals of their scan
    uint32_t* cand_idx[2];    // [staging_entries(max_n, max_blocks)]: per-wave
                              // segments of the first-run grid, each its dealt-out
                              // share plus one claim of slack
    uint16_t* cand_size[2];   // same layout: run-0 sizes
    uint32_t* sorted[2];      // [max_n] candidates, largest size first
    uint32_t* overflow;       // [max_n] items to rerun in 32 x 32 grids
    uint4* cand_shape;        // same layout as cand_idx[k] (both classes in turn): the
                              // packed run-0 shape of each candidate (pack_shape)
    uint4* sorted_shape;      // [max_n] the same, in the order of sorted[k], for the
                              // proof stage
    uint4* occ_hi;            // [max_n] words 4-7 of the run-0 occupancy a first
                              // repeat pass stores for the second (words 0-3 go to
                              // cand_shape)
    uint32_t* small_hash;     // [2]: D4 hash of the monomer and of the domino
    jatam_result_t* records;  // [max_n] records of a GA generation
};

struct BatchArgs {
    const uint64_t* genomes;        // list mode, or nullptr
    const jatam_item_t* items;      // item mode, or nullptr
    uint64_t first;                 // range mode: genome i = first + i
    int64_t n;
    int t, grid;                    // uniform t and G (range and list modes)
    int c, bits, runs;
    uint32_t key0, key1;
    const uint32_t* order;          // nullptr, or queue position -> input index
    const uint32_t* slice;          // nullptr, or device slice counter s: the call
                                    // covers first + s*n .. (graph replays)
    int out_per_slice;              // with `slice`: records go to out + s*n
    int narrow_max;                 // largest G classified with the 16 x 16 layout;
                                    // above 16 the layout is a window (see
                                    // overflow_count_kernel)
    const uint32_t* n_dev;          // nullptr, or the item count on the device
                                    // (first-run stage; at most n)
    int refill;                     // idle lanes that trigger a refill (1..64, per class)
    int dyn16;                      // sixteenths of the first-run chunks claimed from
                                    // device counters rather than dealt out (0..16)
    int claim_chunks;               // most chunks one claim takes (1..kMaxClaimChunks)
    uint32_t seg_cap;               // staging slots per wave (set per launch)
    uint32_t small0, small1;        // D4 hashes of the monomer and the domino (the
                                    // workspace's small_hash, copied at creation)
    jatam_result_t* out;
    unsigned long long* tally;      // nullptr or [4], accumulated
    DeviceWorkspace ws;
};

// Pipeline stages, in launch order (timing hook): four per grid class.
enum {
    kStageFirst = 0,    // + kStagesPerClass * grid class
    kStageSort = 1,
    kStageProve = 2,
    kStageRepeat = 3,
    kStagesPerClass = 4,
    kStages = 8,
};

// Launch parameters of one grid class: first-run refill threshold and the
// persistent grids (one-wave blocks) of the first-run and repeat stages.
struct StageLaunch {
    int refill;
    int first_blocks;
    int repeat_blocks;
    int dyn16;
    int claim_chunks;
    int repeat_mapping;   // 0: R lanes per candidate; 1: one lane per candidate;
                          // 2: kRepeatFirstRuns lanes first, R lanes for the undecided
};

// occ[grid class][TM == 2 ? 0 : 1][0 first runs, 1 repeat runs (R lanes per
// candidate), 2 repeat runs (one lane per candidate)]: resident one-wave
// blocks per CU of the stage kernels.
void batch_occupancy(int occ[2][2][3]);
// Default launch parameters of a grid class.
jatam_tuning_t default_tuning(int klass);
// Largest first-run grid (one-wave blocks) over the classes and tile bounds.
int max_first_blocks(const int occ[2][2][3], int cus);
// Whether the size scan can cover that many first-run blocks.
bool scan_fits(int max_blocks);
// Lays out a DeviceWorkspace for calls of up to max_n genotypes and first-run
// grids of up to max_blocks blocks in one region at `base` (pieces aligned to
// 256 bytes); `records` includes the GA generation's record array.  Returns
// the region's size in bytes; with base == nullptr only the size.
size_t carve_workspace(uint8_t* base, size_t max_n, int max_blocks, bool records,
                       DeviceWorkspace* ws);
// Validates and digests the arguments shared by every classification call.
int make_params(int t, int c, int grid, int runs, uint64_t seed, Params* p);

// The paper's GA: roulette, single-point crossover, Poisson bit flips
// (jatam_roulette.hip).
constexpr int kPoissonMax = 64;     // flip-count thresholds T_0 .. T_L, L <= 64
constexpr int kFujiMaxPop = 1024;   // one lane per genome, one workgroup per simulation
constexpr int kFujiMaxRates = 8;    // mutation rates per Fujiyama launch

struct PoissonTable {
    uint32_t tm1[kPoissonMax + 1];  // T_j - 1 where T_j >= 1
    uint64_t zero;                  // bit j: T_j == 0
};

struct RouletteArgs {
    uint32_t key0, key1;            // Philox key = GA seed
    int length;                     // genome bits L
    int crossover;                  // 1: single-point crossover with a second parent
    PoissonTable poisson;
};

struct FujiyamaArgs {
    RouletteArgs r;                 // length and crossover (keys set per simulation)
    uint64_t seed;                  // simulation s uses GA seed seed + s
    int rates, sims, pop, target, cutoff;
    int32_t* discovery;             // [sims * rates], index s * rates + k
    int32_t* adaptation;
    uint64_t* final_pop;            // nullptr, or [sims * rates * pop]
    PoissonTable poisson[kFujiMaxRates];
};

int launch_roulette_offspring(const uint64_t* pop, const uint32_t* fit, uint32_t n,
                              const RouletteArgs& r, int32_t generation, uint32_t n_out,
                              uint32_t* sums, uint64_t* out, hipStream_t s);
int launch_fujiyama(const FujiyamaArgs& f, hipStream_t s);

// Robustness and evolvability (jatam_neighbourhood.hip).
int launch_mutants(const uint64_t* genomes, uint64_t first, int64_t n, int nbits, uint64_t* out,
                   hipStream_t s);
int launch_neighbourhood(const jatam_result_t* own, const jatam_result_t* mut, int64_t n,
                         int nbits, jatam_neighbourhood_t* out, hipStream_t s);
int launch_neighbourhood_space(const jatam_result_t* space, uint64_t first, int64_t n, int nbits,
                               jatam_neighbourhood_t* out, hipStream_t s);
// Arguments of a pipelined call over a workspace (range mode, no order).
BatchArgs batch_args_for(const Params& p, int64_t n, jatam_result_t* out, uint64_t* tally,
                         const DeviceWorkspace& ws, const uint32_t small_hash[2]);
// Launches the pipeline with launch parameters tn[grid class], capped by the
// residency limits occ on a device of `cus` compute units.  grid_limit: the
// call's uniform G, or 0 for mixed items (both classes).
int launch_tuned(const jatam_tuning_t tn[2], const int occ[2][2][3], int cus, BatchArgs a,
                 int grid_limit, int max_t, hipStream_t stream, hipEvent_t* marks,
                 uint8_t* launched);
int batch_init_small_hash(uint32_t* small_hash, hipStream_t stream);
// When `marks` is not null, an event is recorded on the stream before stage
// s (marks[2s]) and after it (marks[2s+1]), and launched[s] is set.
int launch_batched(const BatchArgs& a, const bool classes[2], const StageLaunch launch[2], int tm,
                   hipStream_t stream, hipEvent_t* marks, uint8_t* launched);
// Slice counter of a replayed enumeration: set to 0, or advanced by one.
int launch_slice_reset(uint32_t* counter, hipStream_t stream);
int launch_slice_advance(uint32_t* counter, hipStream_t stream);
// flag[0] |= 1 if the two record arrays differ anywhere.
int launch_records_differ(const jatam_result_t* x, const jatam_result_t* y, uint64_t n,
                          uint32_t* flag, hipStream_t stream);

// ---------------------------------------------------------------------------
// Genetic algorithm.
// ---------------------------------------------------------------------------
struct GaArgs {
    uint32_t key0, key1;   // Philox key = GA seed
    int32_t generation;
    int tournament;        // T
    int mut_num, mut_den;  // per-edge mutation probability
    int t, c, bits;
};

int launch_ga_offspring(const uint64_t* pop, const int32_t* fit, uint32_t n, const GaArgs& g,
                        uint32_t n_out, uint64_t* out, hipStream_t stream);
int launch_ga_fitness(const jatam_result_t* rec, uint32_t n, int32_t* fit, hipStream_t stream);

// ---------------------------------------------------------------------------
// Surrogate MLP: 96 -> 256 -> 256 -> 4.  Flat fp32 parameter order:
// w1 [96][256], b1 [256], w2 [256][256], b2 [256], w3 [256][4], b3 [4].
// ---------------------------------------------------------------------------
constexpr int kMlpEdges = 12, kMlpIn = 96, kMlpHidden = 256, kMlpOut = 4;
constexpr int kMlpOffW1 = 0;
constexpr int kMlpOffB1 = kMlpOffW1 + kMlpIn * kMlpHidden;
constexpr int kMlpOffW2 = kMlpOffB1 + kMlpHidden;
constexpr int kMlpOffB2 = kMlpOffW2 + kMlpHidden * kMlpHidden;
constexpr int kMlpOffW3 = kMlpOffB2 + kMlpHidden;
constexpr int kMlpOffB3 = kMlpOffW3 + kMlpHidden * kMlpOut;
constexpr int kMlpParams = kMlpOffB3 + kMlpOut;   // 91,652

struct MlpTensors {      // views into one flat fp32 vector
    float* flat;
    float *w1, *b1, *w2, *b2, *w3, *b3;
};

struct MlpArgs {
    MlpTensors p;        // fp32 master weights
    MlpTensors g;        // gradients of the last training step
    float* m;            // Adam first moments
    float* v;            // Adam second moments
    uint16_t* w1b;       // bf16 copies of the weights
    uint16_t* w2b;
    uint16_t* w3b;
    uint16_t* w2t;       // [256][256] bf16 W2 transposed (k contiguous)
    uint16_t* w3t;       // [16][256] bf16 W3 transposed, rows 4..15 zero
    uint16_t* x;         // [batch][96] one-hot inputs (bf16)
    uint16_t* h1;        // [batch][256] bf16
    uint16_t* h2;        // [batch][256] bf16
    uint16_t* dh2;       // [batch][256] bf16
    uint16_t* dh1;       // [batch][256] bf16
    float* dout;         // [batch][4]
    float* loss;         // [batch] per-sample loss
    float* partial;      // partial sums of the backward reductions
    int c, bits;
};

// Floats of MlpArgs::partial for batches of up to max_batch samples.
size_t mlp_partial_floats(size_t max_batch);
int mlp_launch_init(const MlpArgs& a, uint64_t seed, hipStream_t s);
int mlp_launch_score(const MlpArgs& a, const uint64_t* genomes, const uint8_t* tvec, int t_all,
                     uint32_t n, float* scores, int kind, hipStream_t s);
int mlp_launch_refresh(const MlpArgs& a, hipStream_t s);
int mlp_launch_forward(const MlpArgs& a, const uint64_t* genomes, const uint8_t* tvec, int t_all,
                       uint32_t n, uint32_t n_pad, const jatam_result_t* labels, float* out4,
                       hipStream_t s);
int mlp_launch_backward(const MlpArgs& a, uint32_t n, uint32_t n_pad, float* loss_out,
                        hipStream_t s);
int mlp_launch_adam(const MlpArgs& a, float lr, int step, hipStream_t s);

// ---------------------------------------------------------------------------
// Top-k selection (jatam_select.hip).
// ---------------------------------------------------------------------------
constexpr int kSelectState = 2 + 256;

struct SelectWork {
    uint32_t* state;     // [kSelectState]
    uint32_t* flag;      // [n]
    uint32_t* rank_eq;   // [n]
    uint32_t* pos;       // [n]
    uint32_t* sums;      // [n / 1024 + 1]
};

// Indices of the k best scores (descending, ties to the lower index, NaN
// last), in ascending index order, into out_idx[k].
int launch_select_top(const float* scores, uint32_t n, uint32_t k, uint32_t* out_idx,
                      const SelectWork& w, hipStream_t s);

int launch_gather(const uint64_t* src, const uint32_t* idx, uint32_t n, uint64_t* dst,
                  hipStream_t s);

// Queue order by predicted cost (descending score buckets) into order[n];
// work: order_work_words(n) words of device scratch.
uint64_t order_work_words(uint64_t n);
int launch_order_by_cost(const float* scores, uint32_t n, uint32_t* order, uint32_t* work,
                         hipStream_t s);

// ---------------------------------------------------------------------------
// True class by exhaustive exploration (jatam_truth.hip).
// ---------------------------------------------------------------------------
struct TruthArgs {
    const uint64_t* genomes;        // list mode, or nullptr: genome i = first + i
    uint64_t first;
    int64_t n;
    int t, c, bits, genome_bits, grid;
    uint32_t key0, key1;            // key of the one run of the first stage
    int64_t cap;                    // most states explored per genotype
    jatam_result_t* out;
    uint32_t* counters;             // [0] queued genotypes, [1] next one to explore
    uint32_t* queue;                // [n]
    uint32_t max_level;             // states per level (<= 2^18)
    int table_log2;                 // slots of each wave's table (>= 2 * max_level)
    uint32_t* arena;                // per wave: 2 levels of max_level states
    uint32_t* lists;                // per wave: max_level
    uint32_t* terms;                // per wave: max_level
    unsigned long long* tables;     // per wave: 2^table_log2, all zero between calls
};

// Words of one stored state in the exploration (occupancy, tiles, hash).
constexpr int truth_state_words(int W) { return W * W / 32 + W * W / 8 + 1; }
constexpr uint32_t kMaxTruthLevel = 1u << 18;   // states per level (18-bit parent index)
int launch_truth(const TruthArgs& a, int blocks, hipStream_t s);

// ---------------------------------------------------------------------------
// Shape histogram.
// ---------------------------------------------------------------------------
// slice: nullptr, or a device slice counter s: the records read are
// recs + s * n (graph replays of an enumeration).
int launch_shape_hist(const jatam_result_t* recs, uint64_t n, jatam_shape_count_t* table,
                      int log2cap, uint64_t* overflow, int cus, const uint32_t* slice,
                      hipStream_t stream);

}  // namespace jatam
