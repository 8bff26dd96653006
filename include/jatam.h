/*
 * jatam.h - C ABI of the MI355X (gfx950) JaTAM library.
 *
 * Stochastic assembly and classification of JaTAM genotypes (tile sets),
 * the data-parallel hot path of Schroeder de Witt, "Biological Evolution and
 * Genetic Algorithms - Exploring the Space of Abstract Tile Self-Assembly"
 * (arXiv 2205.15311).
 *
 * Model (§1.2, App. B.2, App. B.3):
 *   - A genotype is a set of t square tiles, tile 0 being the seed.  Its
 *     genome holds the tiles in order, each as its N, E, S, W edge colours,
 *     log2(c) bits per colour, most significant first: colour of tile i on
 *     side d is (genome >> (b*(4t-1-(4i+d)))) & (c-1), b = log2(c).
 *   - Colours bond in adjacent pairs 1-2, 3-4, ... (matrix M of App. B.2);
 *     colour 0 and colour c-1, whose partner c does not exist (7 at c=8),
 *     are inert.  Temperature 1: one bond suffices,
 *     mismatched neighbours neither help nor hinder.  Tiles rotate by
 *     quarter turns and never flip; duplicate and symmetric orientations
 *     count as one tile (§3.2).
 *   - A run grows the structure from the seed (unrotated) at the centre
 *     (G/2, G/2) of a G x G grid.  The bounded box is the (G-1)-square
 *     [1, G-1]^2; when a placement exposes a bondable site outside it the
 *     genotype is UNBOUND (App. B.2, "unbounded by d").  Every empty site
 *     next to the structure is checked isotropically: if the tiles that bond
 *     to its occupied neighbours are not all one tile, the genotype is
 *     non-deterministic (ND_SITE, §3.2).  Otherwise the run draws one 32-bit
 *     word u of Philox4x32-10 (key = seed, counter = (step/4, run,
 *     lo32(rng_id), hi32(rng_id)), word step%4) and places the pending tile
 *     of the frontier site of rank floor(u*|F|/2^32) in row-major order.
 *   - R runs are compared by occupancy without rotation (§3.2); the first
 *     witness in run order decides (UNBOUND, ND_SITE, or ND_RUNS for a
 *     different shape).  A run 0 that never had two frontier sites to choose
 *     from used no random word, so all runs equal it and the rest are
 *     skipped.  Otherwise the genotype is DET and its shape is hashed: crop
 *     to the bounding box, one-at-a-time hash (App. F.4) of the occupied
 *     cells' (x, y) bytes in row-major order for each of the 8 orientations
 *     of the dihedral group, sort the 8 hashes, hash their 32 little-endian
 *     bytes (§3.3 describes the four-rotation version).
 *   - rng_id defaults to genome | (uint64)t << 56.
 *
 * Calls are asynchronous on `stream` (a hipStream_t; NULL = the null
 * stream); the caller synchronises.  All array arguments are DEVICE pointers
 * owned by the caller; the library allocates nothing per call.  Every record
 * is a pure function of (genome, t, c, grid, runs, seed, rng_id): it does not
 * depend on the launch configuration, slice size or order of genotypes.
 *
 * Limits: 1 <= t <= 4, c in {2, 4, 8, 16} with 4*t*log2(c) <= 64, grid even
 * in [8, 64], 1 <= runs <= 64, n >= 0.  Grids above 32 are valid models that
 * this library does not run: calls return JATAM_E_UNSUPPORTED.  Each lane
 * keeps its run's grid in LDS (2 occupancy/frontier bits and a 4-bit pending
 * tile per cell of a W x W torus, W = 16 or 32); at W = 64 that is 3 KiB per
 * lane, 192 KiB for a wave of 64 runs, more than the 160 KiB of LDS a CU has.
 */
#ifndef JATAM_H
#define JATAM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* One classification record, 16 bytes, written as one 16-byte store. */
typedef struct {
    int32_t  cls;    /* JATAM_UNBOUND .. JATAM_DET, or JATAM_INVALID           */
    int32_t  size;   /* tiles in the deciding run when it ended (run 0 if DET) */
    uint32_t hash;   /* D4-invariant shape hash if DET, else 0                 */
    int32_t  steps;  /* placements summed over every run that was made         */
} jatam_result_t;

enum {
    JATAM_INVALID = -1, /* record of a genome with bits set above 4*t*log2(c)   */
    JATAM_UNBOUND = 0,  /* a bondable site appeared outside the bounded box     */
    JATAM_ND_SITE = 1,  /* a site admitted two distinct tiles                   */
    JATAM_ND_RUNS = 2,  /* a run ended in a shape different from run 0's        */
    JATAM_DET = 3,      /* every run ended in run 0's shape                     */
};

enum {
    JATAM_OK = 0,
    JATAM_E_INVALID_ARG = -1, /* argument outside the limits above             */
    JATAM_E_UNSUPPORTED = -2, /* valid model, not built for this grid size     */
    JATAM_E_HIP = -3,         /* a HIP launch or runtime call failed           */
    JATAM_E_MISMATCH = -4,    /* autotuning: a candidate's records differed    */
    JATAM_E_IO = -5,          /* a file could not be read or written           */
};

/*
 * Classifies n genotypes given as an array (§3.2, §3.3).
 *   genotypes  device, n x uint64, genome layout above; read once, coalesced
 *   n          number of genotypes (0: no launch)
 *   t, c       tiles per genotype and colour count
 *   grid_limit G, the grid side (bounded box = (G-1)-square)
 *   runs       R, independent runs per genotype
 *   seed       Philox key
 *   out        device, n x jatam_result_t, written once per genotype
 *   stream     hipStream_t or NULL
 * Returns JATAM_OK or a negative JATAM_E_* code; on error nothing is
 * launched and out is untouched.  A genome with bits above its 4*t*log2(c)
 * gets the record {JATAM_INVALID, 0, 0, 0}.
 */
int jatam_classify(const uint64_t* genotypes, int64_t n, int t, int c, int grid_limit,
                   int runs, uint64_t seed, jatam_result_t* out, void* stream);

/*
 * Same, for the contiguous lexicographic range genome_i = first + i of the
 * search space S_{t,c} (the enumerations of §4.1 and §4.3).  No input is
 * read.  JATAM_E_INVALID_ARG if first + n exceeds c^(4t).
 */
int jatam_classify_range(uint64_t first, int64_t n, int t, int c, int grid_limit,
                         int runs, uint64_t seed, jatam_result_t* out, void* stream);

/* ------------------------------------------------------------------------
 * Pipelined ("batched") classification.
 *
 * Same records as jatam_classify, produced by a pipeline that keeps lanes
 * busy: a screen of every genotype's seed, a device queue of first runs
 * drained by persistent waves, and the repeat runs of deterministic
 * candidates ordered by their exact cost (run-0 size), one lane per run (the
 * batching and asynchronous execution of §3.4, and the "as many assembly
 * processes in parallel" optimisation suggested in §4.1).  The queues live in
 * a workspace created once; no call allocates.  Calls sharing one workspace
 * must be serialised (same stream); calls on different workspaces may run
 * concurrently.
 * ------------------------------------------------------------------------ */

/* One entry of a shape histogram (jatam_shape_histogram): a deterministic
 * shape (its D4 hash and size) and how many DET records have it.  size == 0
 * marks an empty entry. */
typedef struct {
    uint32_t hash;
    int32_t  size;
    uint64_t count;
} jatam_shape_count_t;   /* 16 bytes */

/* One genotype of a mixed stream: its own tile count, grid and RNG stream. */
typedef struct {
    uint64_t genome;   /* genome layout above, t tiles                        */
    uint64_t rng_id;   /* Philox stream id (the default is genome | t << 56)  */
    uint8_t  t;        /* 1..4                                                 */
    uint8_t  grid;     /* G, even, 8..32                                       */
    uint8_t  pad[6];
} jatam_item_t;        /* 24 bytes */

typedef struct jatam_batch jatam_batch_t;

/*
 * Creates a workspace for calls of up to max_n (1 <= max_n < 2^32) genotypes
 * on the current HIP device: 28 bytes of device memory per genotype plus a
 * few KiB.  Blocks until the workspace is initialised.  *batch receives the
 * handle; JATAM_E_HIP if device memory runs out.
 */
int jatam_batch_create(int64_t max_n, jatam_batch_t** batch);

/* Frees a workspace (NULL is accepted).  Synchronises its device. */
int jatam_batch_destroy(jatam_batch_t* batch);

/*
 * Pipelined equivalents of jatam_classify / jatam_classify_range, and a
 * mixed-item call where every genotype carries its own t, grid and rng_id.
 *   batch  workspace from jatam_batch_create, same device, n <= its max_n
 *   tally  NULL, or device uint64[4] to which the number of UNBOUND,
 *          ND_SITE, ND_RUNS and DET records is ADDED (the caller zeroes it)
 * Other arguments and errors as for jatam_classify.  Items with t, grid or
 * genome outside the limits get JATAM_INVALID records.
 */
int jatam_batch_classify(jatam_batch_t* batch, const uint64_t* genotypes, int64_t n, int t,
                         int c, int grid_limit, int runs, uint64_t seed, jatam_result_t* out,
                         uint64_t* tally, void* stream);
int jatam_batch_classify_range(jatam_batch_t* batch, uint64_t first, int64_t n, int t, int c,
                               int grid_limit, int runs, uint64_t seed, jatam_result_t* out,
                               uint64_t* tally, void* stream);
int jatam_batch_classify_items(jatam_batch_t* batch, const jatam_item_t* items, int64_t n,
                               int c, int runs, uint64_t seed, jatam_result_t* out,
                               uint64_t* tally, void* stream);

/*
 * Enumeration of a lexicographic range in slices, with HIP graphs: the
 * pipeline of one slice of `slice` genotypes (and, if `shapes` is given, the
 * shape histogram of its records) is captured once into a graph whose
 * kernels read the slice number from a device counter, then the graph is
 * launched `slices` times on `stream`, the counter advancing by one per
 * replay.  Covers genotypes first .. first + slice*slices - 1 (§3.4: the
 * paper's slice-by-slice enumeration, here without host work per slice).
 *   out     device, slice*slices records in genotype order, or NULL to keep
 *           only the tally and the histogram (records of each slice then go
 *           to the workspace and are overwritten by the next slice)
 *   tally   NULL or device uint64[4], ADDED to (as jatam_batch_classify)
 *   shapes, shapes_capacity
 *           NULL, or a table as for jatam_shape_histogram, ADDED to
 * 1 <= slice <= the workspace's max_n.  The graph is kept in the workspace
 * until the next enumeration or destroy (which first wait for it); calls on
 * one workspace must be serialised as for every other call.
 */
int jatam_batch_enumerate(jatam_batch_t* batch, uint64_t first, int64_t slice, int64_t slices,
                          int t, int c, int grid_limit, int runs, uint64_t seed,
                          jatam_result_t* out, uint64_t* tally, jatam_shape_count_t* shapes,
                          int64_t shapes_capacity, void* stream);

/*
 * Mixed items taken in the order of a queue: position p of the queue holds
 * item order[p] (device, n x uint32, a permutation of 0..n-1; an entry >= n
 * is skipped).  Records stay indexed by item: out[i] is item i's record,
 * whatever the order, which only decides which wave takes which item (a
 * queue sorted by predicted cost, for instance).  Other arguments as for
 * jatam_batch_classify_items.
 */
int jatam_batch_classify_items_ordered(jatam_batch_t* batch, const jatam_item_t* items,
                                       const uint32_t* order, int64_t n, int c, int runs,
                                       uint64_t seed, jatam_result_t* out, uint64_t* tally,
                                       void* stream);

/*
 * Tuning of the first-run stage: a wave refills its idle lanes (screening
 * new genotypes and starting their first runs) once at least idle_lanes of
 * its 64 lanes are idle (1..64; default 24).  Sets both grid classes.
 * Records never depend on it.
 */
int jatam_batch_set_refill(jatam_batch_t* batch, int idle_lanes);

/*
 * Launch parameters of the pipeline for one grid class (G <= 16 or
 * 16 < G <= 32).  None of them changes a record.
 *   refill        first runs: a wave refills once this many of its 64 lanes
 *                 are idle, 1..64 (default 24)
 *   first_waves   persistent one-wave workgroups per CU of the first-run
 *                 stage, >= 1; capped at what fits in a CU (default: that)
 *   repeat_waves  the same for the repeat stage
 *   wide_layout   G <= 16 class: 1 classifies these genotypes with the
 *                 32 x 32 LDS layout (and the other class's parameters)
 *                 instead of the 16 x 16 one (default 0).
 *                 16 < G <= 32 class: 2 first classifies these genotypes
 *                 in a 16 x 16 window around the seed, with the G <= 16
 *                 class's parameters, and reruns in 32 x 32 grids (with
 *                 this class's parameters) only those whose record came out
 *                 UNBOUND there, since only a run that reaches the window's
 *                 ring can differ from the run in its own grid; 1 classifies
 *                 them in 32 x 32 grids directly; 0 (default) is 2 for calls
 *                 of at least 2^20 genotypes and 1 below.  The G <= 16
 *                 class at 1 turns the window off.
 *   claim_share   first runs: sixteenths of the input's 64-item chunks that
 *                 waves claim from device counters (eight, each for a
 *                 contiguous eighth of the claimed chunks; a wave moves to
 *                 the next counter when its own runs dry), up to four chunks
 *                 at a time (fewer when each wave gets few chunks; none when
 *                 each wave gets under 16, where all are dealt out),
 *                 once their dealt-out chunks are done (0..16; default 12).
 *                 The rest are dealt out in turn (chunk k to wave k mod the
 *                 grid).  Run lengths follow the genome's digits, so dealt-
 *                 out chunks leave some waves far more work than others;
 *                 claimed chunks go to the waves that finish first.
 *   claim_chunks  first runs: the most 64-item chunks one claim takes
 *                 (1..8; default 4): the work queue's chunk size.
 *   repeat_mapping  repeat runs of the candidates that run 0 leaves
 *                 undecided (default 2 for G <= 16, 0 above): 0 gives each
 *                 candidate R lanes of a
 *                 wave, lane r making run r; 1 gives each candidate one
 *                 lane that makes runs 1, 2, ... in turn and stops at the
 *                 first witness, a lane that finishes taking the next
 *                 candidate from the queue; 2 makes two passes, the first
 *                 with 4 lanes per candidate (runs 0..3: a witness among
 *                 them decides, in the same kernel as the forced-shape
 *                 proof), the second for the candidates the first left
 *                 undecided (G <= 16: R - 4 lanes making runs 4..R-1;
 *                 above: R lanes).
 */
typedef struct {
    int refill;
    int first_waves;
    int repeat_waves;
    int wide_layout;
    int claim_share;
    int claim_chunks;
    int repeat_mapping;
} jatam_tuning_t;

/*
 * jatam_batch_classify_range with a queue order: queue position p holds
 * genotype first + order[p] (order: device uint32[n], a permutation of
 * 0..n-1; an entry >= n is skipped).  Records stay indexed by genotype and
 * never depend on the order.  The order is how a cost prediction (e.g.
 * jatam_order_by_cost over surrogate scores) reaches the first-run queue.
 */
int jatam_batch_classify_range_ordered(jatam_batch_t* batch, uint64_t first, int64_t n, int t,
                                       int c, int grid_limit, int runs, uint64_t seed,
                                       const uint32_t* order, jatam_result_t* out,
                                       uint64_t* tally, void* stream);

/*
 * A queue order by predicted cost: order[0..n) lists 0..n-1 by descending
 * score, in 256 buckets of 16 log2(score + 2) (scores as jatam_mlp_score
 * gives them, the expected size of a deterministic structure; NaN last),
 * items of one bucket in no particular order.  work: device scratch of
 * jatam_order_work_words(n) uint32 words.  n < 2^32.
 */
int64_t jatam_order_work_words(int64_t n);
int jatam_order_by_cost(const float* scores, int64_t n, uint32_t* order, uint32_t* work,
                        void* stream);

/*
 * The batch classification of the problem statement (App. B.2: a tile set in,
 * its classified phenotype out) over a mixed stream in one call.
 *   batch   workspace from jatam_batch_create, n <= its max_n
 *   items   device, n x jatam_item_t (each item its own t, grid and rng_id)
 *   order   NULL (queue position p holds item p), or device uint32[n]: a
 *           permutation giving the queue order (see
 *           jatam_batch_classify_items_ordered)
 *   tune    NULL: the workspace's parameters (defaults, or what
 *           jatam_batch_autotune chose); else tune[0] (G <= 16) and
 *           tune[1] (16 < G <= 32) for this call only, validated as by
 *           jatam_batch_set_tuning
 *   out, tally, stream, errors: as jatam_batch_classify_items.
 * Records never depend on order or tune.
 */
int jatam_classify_batch(jatam_batch_t* batch, const jatam_item_t* items, int64_t n, int c,
                         int runs, uint64_t seed, const uint32_t* order,
                         const jatam_tuning_t* tune, jatam_result_t* out, uint64_t* tally,
                         void* stream);

/* The parameters used for grid_limit's class (8 <= grid_limit <= 32). */
int jatam_batch_get_tuning(const jatam_batch_t* batch, int grid_limit, jatam_tuning_t* tuning);
int jatam_batch_set_tuning(jatam_batch_t* batch, int grid_limit, const jatam_tuning_t* tuning);

/*
 * Autotuner: picks the parameters of grid_limit's class by timing the
 * pipeline on a lexicographic sample [first, first + n) (arguments as for
 * jatam_batch_classify_range, 1 <= n <= the workspace's max_n).  Starting
 * from the current parameters it tries, one field at a time, refill in
 * {8, 16, 24, 32, 48}, first_waves and repeat_waves at and below the
 * residency limit, every wide_layout value of the class, claim_share in
 * {0, 4, 8, 12, 16}, claim_chunks in {1, 2, 4, 8} and the three
 * repeat_mapping values, keeping a
 * value when the median of three timed calls improves by more than 1%
 * (less is within run-to-run noise).  Every candidate's records are
 * compared with the starting configuration's, bit for bit: a difference
 * stops the search with JATAM_E_MISMATCH.  The best parameters found are
 * set on the workspace and written to *best (if not NULL).
 *   scratch  device, 2n records, caller-owned, overwritten
 * Synchronises the stream; allocates nothing on the device.
 */
int jatam_batch_autotune(jatam_batch_t* batch, uint64_t first, int64_t n, int t, int c,
                         int grid_limit, int runs, uint64_t seed, jatam_result_t* scratch,
                         jatam_tuning_t* best, void* stream);

/*
 * jatam_batch_autotune with a cache file, so the search runs once per
 * device and workload class: the file holds one JSON object per line,
 *   {"key": "<gfx arch>|cu<CUs>|G<16|32>|t<t>|c<c>|R<runs>|abi<version>",
 *    "refill": .., "first_waves": .., "repeat_waves": .., "wide_layout": ..,
 *    "claim_share": .., "claim_chunks": .., "repeat_mapping": ..}
 * keyed by the device, grid_limit's class, t, c and runs.  A valid entry
 * for the key is applied (jatam_batch_set_tuning) and *from_cache = 1;
 * otherwise jatam_batch_autotune runs (arguments as there) and the file is
 * rewritten with the new entry added (other keys kept, a broken line of this
 * key dropped; written to path.tmp, then renamed), *from_cache = 0.
 * JATAM_E_IO if the file cannot be written.  Not thread-safe on one file.
 */
int jatam_batch_autotune_cached(jatam_batch_t* batch, const char* path, uint64_t first,
                                int64_t n, int t, int c, int grid_limit, int runs,
                                uint64_t seed, jatam_result_t* scratch, jatam_tuning_t* best,
                                int* from_cache, void* stream);

/* Entry i of the last autotune's log (the configuration and its median ms);
 * returns the number of entries (i < 0: only that). */
int jatam_batch_autotune_log(const jatam_batch_t* batch, int i, jatam_tuning_t* tuning,
                             double* ms);

/*
 * Timing hook of the pipeline, for measurement.  While enabled, every call on
 * `batch` records HIP events on its stream around each stage (one event pair
 * per stage and call; enabling or disabling synchronises the device and
 * forgets earlier events).  jatam_batch_stage_times waits for the recorded
 * calls and writes, per stage s < max_stages, the summed duration in ms over
 * those calls to ms[s] and, if calls is not NULL, how many calls ran it to
 * calls[s]; it returns the number of stages written.  Stage names:
 * jatam_batch_stage_name (0 first runs, 1 size sort, 2 forced-shape proof
 * and compaction, 3 repeat runs for G <= 16; 4-7 the same for G <= 32).
 * With two repeat passes (repeat_mapping 2 and runs > 4) stage 2 is the
 * proof together with the first repeat pass (one kernel) and stage 3 the
 * second pass.
 */
int jatam_batch_set_timing(jatam_batch_t* batch, int enable);
int jatam_batch_stage_times(jatam_batch_t* batch, double* ms, int* calls, int max_stages);
const char* jatam_batch_stage_name(int stage);

/* ------------------------------------------------------------------------
 * Genetic algorithm with assembly as fitness (§2.2, §3.1): one offspring per
 * lane, one launch per generation (the kernel boundary is the global
 * synchronisation the paper requires).
 *
 * Operators: tournament selection of `tournament` genomes drawn uniformly
 * with replacement (fittest wins, ties to the earliest draw); uniform
 * crossover per edge colour; per-edge mutation with probability
 * mut_num/mut_den to a colour drawn uniformly from the other c-1; no
 * elitism.  Offspring i of generation g draws Philox4x32-10 keyed by `seed`
 * at counter (i, g, block, 1 << 28), word q = word q%4 of block q/4: words
 * 0..T-1 parent A's tournament, T..2T-1 parent B's, 2T the crossover mask
 * (bit e: edge e from B), 2T+1+e edge e's mutation test (mutate iff
 * floor(w*den/2^32) < num), 2T+1+E+e its new colour r = floor(w*(c-1)/2^32),
 * taken as r if r < old else r+1 (E = 4t).
 * ------------------------------------------------------------------------ */
typedef struct {
    uint64_t seed;        /* Philox key of the GA's draws                   */
    int32_t  tournament;  /* T, 1..8                                         */
    int32_t  mut_num;     /* per-edge mutation probability mut_num/mut_den  */
    int32_t  mut_den;
    int32_t  pad;
} jatam_ga_params_t;

/*
 * n_out offspring of a population of n (1 <= n < 2^32) genomes of t tiles.
 *   pop, fit  device, n genomes and their int32 fitness
 *   out       device, n_out genomes
 */
int jatam_ga_offspring(const uint64_t* pop, const int32_t* fit, int64_t n, int t, int c,
                       const jatam_ga_params_t* p, int32_t generation, int64_t n_out,
                       uint64_t* out, void* stream);

/* ------------------------------------------------------------------------
 * Surrogate MLP (not from the paper, which has no learned part).  Predicts a
 * genotype's class and log(1 + size) from its edge colours so work can be
 * ordered and GA offspring screened; every reported class still comes from
 * exact assembly.
 *
 * x = one-hot of the 12 edge colours of up to 3 tiles (c <= 8; edge e of the
 * genome -> input e*8 + colour; edges of absent tiles are zero), h1 =
 * relu(x W1 + b1), h2 = relu(h1 W2 + b2), 256 wide, out = h2 W3 + b3 =
 * (logit UNBOUND, logit ND, logit DET, log1p(size)).  Loss = mean
 * cross-entropy (ND_SITE and ND_RUNS are one class) + mean squared error of
 * log1p(size).  Weights are fp32 masters used as bf16, activations and hidden
 * gradients are bf16, products accumulate in fp32 (bf16 MFMA), Adam
 * (beta 0.9 / 0.999, eps 1e-8) updates the masters.
 *
 * Parameters are one fp32 vector of 91,652: w1 [96][256], b1 [256],
 * w2 [256][256], b2 [256], w3 [256][4], b3 [4] (row-major).
 * ------------------------------------------------------------------------ */
typedef struct jatam_mlp jatam_mlp_t;

/* Creates a network on the current device (parameters initialised He-uniform
 * from seed 0x5eed), with activation buffers for training batches of up to
 * max_batch (1..2^24) samples; c is the colour count (2, 4 or 8). */
int jatam_mlp_create(int64_t max_batch, int c, jatam_mlp_t** mlp);
int jatam_mlp_destroy(jatam_mlp_t* mlp);

/* Re-initialises: w = (2u - 1) sqrt(6 / fan_in), u = Philox word / 2^32 with
 * key `seed` at counter (index, 0, 0, 3 << 28); biases and Adam state 0. */
int jatam_mlp_init(jatam_mlp_t* mlp, uint64_t seed, void* stream);

/* Copies parameters in (device fp32 [91652]; Adam state reset) or out; grads
 * receives the gradient of the last training step (either may be NULL). */
int jatam_mlp_set_params(jatam_mlp_t* mlp, const float* params, void* stream);
int jatam_mlp_get_params(jatam_mlp_t* mlp, float* params, float* grads, void* stream);

/* out4[i] = network output for genome i (device, n x 4 fp32).  t: per-genome
 * tile counts (device uint8) or NULL for t_all (1..3; JATAM_E_INVALID_ARG
 * otherwise).  A genome whose own t is outside 1..3 is read as having no
 * tiles (an all-zero input): the network sees at most 12 edges. */
int jatam_mlp_forward(jatam_mlp_t* mlp, const uint64_t* genomes, const uint8_t* t, int t_all,
                      int64_t n, float* out4, void* stream);

/* One step on a batch of n <= max_batch labelled genotypes (labels: their
 * jatam_result_t records): forward, loss, backward, then Adam with learning
 * rate lr (lr = 0: gradients only).  loss_out: NULL or device float[1]. */
int jatam_mlp_train_step(jatam_mlp_t* mlp, const uint64_t* genomes, const uint8_t* t, int t_all,
                         const jatam_result_t* labels, int64_t n, float lr, float* loss_out,
                         void* stream);

/* Screening score of each genome: P(DET) * exp(predicted log1p size) - 1,
 * the expected size of a deterministic structure (device float [n]).  One
 * fused pass (layer-1 gather, h1 W2 and the head on the matrix cores, 64
 * genomes per workgroup); n is not limited by max_batch and no activations
 * are kept. */
int jatam_mlp_score(jatam_mlp_t* mlp, const uint64_t* genomes, const uint8_t* t, int t_all,
                    int64_t n, float* scores, void* stream);

/* What jatam_mlp_predict writes per genome (o = the network's four outputs,
 * p = the softmax of the three class logits o0..o2: UNBOUND, ND, DET):
 *   SCREEN     p_DET * exp(o3) - 1, as jatam_mlp_score
 *   COST       exp(o3) - 1: the predicted size of the deciding run, which is
 *              what the first run costs in placements (plus one); the order
 *              of a queue by predicted cost
 *   P_UNBOUND  p_UNBOUND: for a network trained on classifications at G = 16,
 *              the predicted probability that a run leaves the 16 x 16
 *              window, i.e. that an item of 16 < G <= 32 needs its own grid */
enum { JATAM_PREDICT_SCREEN = 0, JATAM_PREDICT_COST = 1, JATAM_PREDICT_P_UNBOUND = 2 };

/* One of the predictions above for each genome (device float [n]); the same
 * fused pass as jatam_mlp_score.  JATAM_E_INVALID_ARG for an unknown kind. */
int jatam_mlp_predict(jatam_mlp_t* mlp, int kind, const uint64_t* genomes, const uint8_t* t,
                      int t_all, int64_t n, float* out, void* stream);

/* ------------------------------------------------------------------------
 * Surrogate-screened GA.  A generation draws oversample * n offspring
 * (offspring i exactly as jatam_ga_offspring draws it), scores them with the
 * surrogate, keeps the n best (score descending, ties to the lower offspring
 * index, NaN last; kept offspring in ascending index order), and classifies
 * only those exactly: fitness always comes from assembly.
 * ------------------------------------------------------------------------ */
typedef struct jatam_ga jatam_ga_t;

/* Workspace for up to max_candidates offspring per generation (about 24
 * bytes of device memory each). */
int jatam_ga_create(int64_t max_candidates, jatam_ga_t** ga);
int jatam_ga_destroy(jatam_ga_t* ga);

/* Indices (device uint32 [k], ascending) of the k best of n scores by the
 * rule above; n <= the workspace's max_candidates. */
int jatam_select_top(jatam_ga_t* ga, const float* scores, int64_t n, int64_t k, uint32_t* out_idx,
                     void* stream);

/* One screened generation (t <= 3, c the network's colour count). */
int jatam_ga_step_screened(jatam_ga_t* ga, jatam_batch_t* batch, jatam_mlp_t* mlp,
                           const uint64_t* pop, const int32_t* fit, int64_t n, int t, int c,
                           int grid_limit, int runs, uint64_t seed, const jatam_ga_params_t* p,
                           int32_t generation, int oversample, uint64_t* next_pop,
                           int32_t* next_fit, void* stream);

/* What screens a generation: the network, the candidate workspace (at least
 * oversample * n candidates) and the oversampling factor (>= 1). */
typedef struct {
    jatam_mlp_t* mlp;
    jatam_ga_t*  ga;
    int32_t      oversample;
    int32_t      pad;
} jatam_screen_t;

/*
 * One generation of the GA (§2.2, §3.1): n offspring (next_pop, distinct
 * from pop), classified by the pipelined path of `batch` (n <= its max_n; R
 * runs on grid_limit with assembly seed `seed`), and their fitness
 * next_fit[i] = size if DET else 0.
 *   surrogate  NULL: the plain GA (offspring i drawn as jatam_ga_offspring
 *              draws it); else the screened generation of
 *              jatam_ga_step_screened with surrogate->mlp, ->ga and
 *              ->oversample (t <= 3).  Fitness always comes from assembly.
 */
int jatam_ga_step(jatam_batch_t* batch, const uint64_t* pop, const int32_t* fit, int64_t n, int t,
                  int c, int grid_limit, int runs, uint64_t seed, const jatam_ga_params_t* p,
                  int32_t generation, const jatam_screen_t* surrogate, uint64_t* next_pop,
                  int32_t* next_fit, void* stream);

/* ------------------------------------------------------------------------
 * Shape histogram (§3.4: the paper histograms the shape hashes of every
 * slice, on the host, while the next slice is classified).  Kept on the
 * device here.
 * ------------------------------------------------------------------------ */

/*
 * Adds the DET records of recs[0..n) to a shape histogram.
 *   recs      device, n records (any call's output; non-DET records ignored)
 *   table     device, capacity entries, open addressing keyed by
 *             (hash, size); zero it before its first use; counts are ADDED,
 *             so one table can collect many slices.  Entry order is not
 *             meaningful.
 *   capacity  a power of two in [64, 2^24]
 *   overflow  NULL, or device uint64[1] to which the number of DET records
 *             that found no free entry is added (0 unless the table is full)
 * JATAM_E_INVALID_ARG for a bad capacity or n < 0.  Calls adding to one
 * table must be serialised (same stream).
 */
int jatam_shape_histogram(const jatam_result_t* recs, int64_t n, jatam_shape_count_t* table,
                          int64_t capacity, uint64_t* overflow, void* stream);

/* ------------------------------------------------------------------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * pipelined classification of jatam_batch_classify (same records, the
 * default launch parameters) with its queues in a static 32 MiB device array
 * of the library, one per GPU, held until the process ends, instead of a
 * jatam_batch_t.  n <= 2^18 (JATAM_E_INVALID_ARG above).  Every call on a
 * GPU shares that GPU's array: calls that overlap on one GPU race and must
 * be serialised (one stream).  The first call on each device sets up (the
 * array's address, a kernel and a copy on the null stream, synchronised), so
 * it must not be captured; later calls only launch kernels on `stream` and
 * call no allocating routine.  Other arguments as for jatam_batch_classify.
 * ------------------------------------------------------------------------ */
int jatam_classify_static(const uint64_t* genotypes, int64_t n, int t, int c, int grid_limit,
                          int runs, uint64_t seed, jatam_result_t* out, uint64_t* tally,
                          void* stream);

/* ------------------------------------------------------------------------
 * True class (§3.2, §4.1): the k runs of the classifier sample growth
 * orders and can miss an order that meets an ambiguous site or ends in
 * another shape, so a genotype they class DET may not be deterministic; the
 * paper measures how often as k grows.  These calls follow every order:
 *   cls  JATAM_DET      every order ends in one shape without an event;
 *                       size and hash of that shape
 *        JATAM_ND_SITE  some order meets an event (a bondable site outside
 *                       the box, or an ambiguous site) or ends in a second
 *                       shape (occupancy compared without rotation); size 0,
 *                       hash 0
 *        JATAM_UNDECIDED  the search would pass `cap` states (or a level
 *                       would pass the workspace's max_level); size 0, hash 0
 *        JATAM_INVALID  genome bits above 4*t*log2(c)
 *   steps  states explored (0 when one run decided: an event in it, no
 *          choice in it, or a guarded shape, whose every order places the
 *          same tiles).
 * The verdict does not depend on the order in which states are visited
 * (except where the search is cut off by cap).
 * ------------------------------------------------------------------------ */
enum { JATAM_UNDECIDED = -2 };

typedef struct jatam_truth jatam_truth_t;

/* Workspace for calls of up to max_n genotypes: the queue of genotypes one
 * run leaves open, and per exploring wave (waves in [1, 4096]) two levels of
 * max_level states (max_level in [1, 2^18]; 644 bytes per state) and a hash
 * table of 2 * max_level slots.  Allocates and zeroes device memory
 * (synchronises the device). */
int jatam_truth_create(int64_t max_n, int32_t max_level, int32_t waves, jatam_truth_t** out);
int jatam_truth_destroy(jatam_truth_t* w);

/* True class of n genotypes (device array) of t tiles on a grid of side
 * grid_limit; cap >= 1 limits the states explored per genotype.  out:
 * device, n records.  Calls on one workspace must be serialised (one
 * stream). */
int jatam_true_class(jatam_truth_t* w, const uint64_t* genotypes, int64_t n, int t, int c,
                     int grid_limit, int64_t cap, jatam_result_t* out, void* stream);
/* Same for the range genome_i = first + i. */
int jatam_true_class_range(jatam_truth_t* w, uint64_t first, int64_t n, int t, int c,
                           int grid_limit, int64_t cap, jatam_result_t* out, void* stream);

/* ------------------------------------------------------------------------
 * Classification variants, by the plain kernel (one lane per genotype):
 *   JATAM_VARIANT_C4    DET shapes hashed up to rotation only (§3.3 names the
 *                       four rotations): the four rotation hashes sorted
 *                       ascending and hashed again as 16 little-endian bytes
 *   JATAM_VARIANT_LIFO  the movelist traversal of §3.2: frontier sites on a
 *                       LIFO stack; a site that joins the frontier (in the
 *                       order N, E, S, W of each placement's checks) goes to
 *                       slot floor(u (len + 1) / 2^32) from the bottom of the
 *                       len sites on the stack, u the run's next random word
 *                       (word d of the run's stream for its d-th draw; no
 *                       draw into an empty stack); each step places the site
 *                       on top.  A run without a draw is the only run.
 *                       G <= 16 only (JATAM_E_UNSUPPORTED above).
 * The flags combine; 0 gives jatam_classify's records.  genotypes: device
 * array, or NULL for the range genotype_i = first + i.  Other arguments and
 * errors as jatam_classify.
 * ------------------------------------------------------------------------ */
enum { JATAM_VARIANT_C4 = 1, JATAM_VARIANT_LIFO = 2 };

int jatam_classify_variant(const uint64_t* genotypes, uint64_t first, int64_t n, int t, int c,
                           int grid_limit, int runs, uint64_t seed, int variant,
                           jatam_result_t* out, void* stream);

/* ------------------------------------------------------------------------
 * Robustness and evolvability (§1.1): robustness is the share of a
 * genotype's single mutations that keep its phenotype, evolvability the
 * number of different phenotypes its single mutations reach.  A single
 * mutation flips one genome bit (the bit-flip mutation of App. B.3), so a
 * genotype of t tiles over c colours has m = 4 t log2(c) single mutants;
 * mutant k has bit k flipped (bit 0 the lowest).  A phenotype is UNBOUND,
 * non-deterministic (ND_SITE or ND_RUNS, one phenotype) or a deterministic
 * shape (size and hash); records of other classes count as
 * non-deterministic.
 *   robust  mutants whose phenotype equals the genotype's (0..m)
 *   evolv   distinct phenotypes among the mutants, the genotype's own
 *           excluded (0..m)
 * ------------------------------------------------------------------------ */
typedef struct {
    int32_t robust;
    int32_t evolv;
} jatam_neighbourhood_t;

/* The single mutants of n genotypes: mutants[i * m + k] = genotype i with
 * bit k flipped.  genotypes: device array, or NULL for the range
 * genotype_i = first + i (which must lie in the space).  mutants: device,
 * n * m entries.  JATAM_E_INVALID_ARG for bad t, c or range. */
int jatam_single_mutants(const uint64_t* genotypes, uint64_t first, int64_t n, int t, int c,
                         uint64_t* mutants, void* stream);

/* Robustness and evolvability of n genotypes from their records (own[i])
 * and their mutants' records (mutant_records[i * m + k], the records of
 * jatam_single_mutants' output, classified by any call with the same c,
 * grid, runs and seed).  All device memory; out: n entries. */
int jatam_neighbourhood(const jatam_result_t* own, const jatam_result_t* mutant_records,
                        int64_t n, int t, int c, jatam_neighbourhood_t* out, void* stream);

/* The same for genotypes first .. first + n - 1 of a whole space whose
 * records are at hand: space[g] is the record of genotype g for every g of
 * the space (c^(4t) records, m <= 32), so every mutant's record is read,
 * none classified.  JATAM_E_INVALID_ARG if m > 32 or the range leaves the
 * space. */
int jatam_neighbourhood_space(const jatam_result_t* space, uint64_t first, int64_t n, int t,
                              int c, jatam_neighbourhood_t* out, void* stream);

/* ------------------------------------------------------------------------
 * The paper's own genetic algorithm (§2.2, §3.1, App. C.1, D.1, D.2):
 * global roulette wheel selection, single-point crossover and Poisson-
 * distributed bit-flip mutation, over genomes of L bits (the low L bits of a
 * uint64_t; bit-string position 0 is bit L-1).
 *   selection  a dart d = floor(u S / 2^32), S = sum of the fitness, lands on
 *              the first genome whose running fitness sum exceeds d (App.
 *              C.1's lookup); uniform when S = 0
 *   crossover  (crossover = 1) a second parent by a second dart, a point
 *              p = floor(u L / 2^32): positions 0..p-1 from the second parent
 *   mutation   k ~ Poisson(lambda) flips, k = the first j with u < T_j,
 *              T_j = floor(2^32 P(k <= j)) computed on the host in double
 *              precision (p_0 = exp(-lambda), p_j = p_(j-1) lambda / j), at
 *              most L; k distinct positions floor(u L / 2^32), a repeat drawn
 *              again (App. D.1), at most 1024 position draws
 *   words      offspring i of generation g: Philox4x32-10 keyed by seed, at
 *              counter (i, g, block, 4 << 28), word q = word q % 4 of block
 *              q / 4: 0 parent, 1 second parent, 2 point, 3 flip count,
 *              4.. positions
 * ------------------------------------------------------------------------ */
typedef struct {
    uint64_t seed;      /* GA seed (Philox key)                              */
    int32_t length;     /* genome bits L, 1..64                              */
    int32_t crossover;  /* 0: asexual, 1: single-point crossover             */
    double lambda;      /* mean flips per offspring, mu L, 0..64             */
} jatam_roulette_params_t;

/* Device words of the work array of jatam_roulette_offspring for n parents. */
int64_t jatam_roulette_work_words(int64_t n);

/* n_out offspring of generation `generation` from n parents (device pop[n],
 * fit[n] with every fitness below 2^16, 1 <= n <= 2^16).  work: device,
 * jatam_roulette_work_words(n) uint32 (the running fitness sums, the
 * paper's summation kernel).  out: device, n_out genomes.  The offspring's
 * fitness is the caller's (Hamming weight, DET size from jatam_classify,
 * ...).  JATAM_E_INVALID_ARG for bad parameters or sizes. */
int jatam_roulette_offspring(const uint64_t* pop, const uint32_t* fit, int64_t n,
                             const jatam_roulette_params_t* p, int32_t generation, int64_t n_out,
                             uint32_t* work, uint64_t* out, void* stream);

/* The Fujiyama test bed (§4.2): fitness = Hamming weight of the genome;
 * sims independent simulations at each of rates (1..8) mutation rates
 * lambdas[k] (host array), each from the all-zero population of pop genomes
 * (1..1024) and GA seed p->seed + s for simulation s, run in one launch
 * (one workgroup per simulation, the generation loop in the kernel).
 * Simulation s at rate k writes, at index s * rates + k of the device arrays
 * discovery and adaptation, the first generation with a genome of weight >=
 * target and the first with at least half the population there (generation
 * 0 is the initial population; -1 if not within cutoff generations); the
 * simulation stops once both are found or at the cut-off.  final_pop: NULL,
 * or device [sims * rates * pop]: the population when it stopped. */
int jatam_fujiyama(const jatam_roulette_params_t* p, const double* lambdas, int32_t rates,
                   int32_t sims, int32_t pop, int32_t target, int32_t cutoff, int32_t* discovery,
                   int32_t* adaptation, uint64_t* final_pop, void* stream);

/* Static description of an error code. */
const char* jatam_strerror(int code);

/* Library ABI version (increments on any change to this header). */
int jatam_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* JATAM_H */
