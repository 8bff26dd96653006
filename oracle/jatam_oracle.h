/*
 * jatam_oracle.h - plain CPU oracle for JaTAM stochastic assembly and
 * classification.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may include, link
 * or call this code: only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark do.  It shares no code, header, table or
 * constant with the HIP library; it follows the paper directly:
 *
 *   tile model, temperature 1, rotation without flips ........ §1.2, App. B.2
 *   interaction matrix M (colours bond in adjacent pairs) ..... App. B.2
 *   genome = tiles in order, seed first, colours N,E,S,W ...... §2.1, App. B.3
 *   movelist assembly on a bounded grid, unbound on the edge .. §1.2, §3.2
 *   isotropic check of every frontier site for ambiguity ...... §3.2
 *   duplicate / symmetric tiles eliminated from bond lists .... §3.2
 *   k independent runs compared without rotation .............. §3.2
 *   crop + one-at-a-time hash, made rotation invariant ........ §3.3, App. F.4, F.6
 *
 * Readings where the paper is silent (documented in the design notes):
 * colour 7 is inert at c=8; colours are MSB-first in the genome; rotation is
 * clockwise quarter turns; the seed sits at (G/2,G/2) and the bounded box is
 * the (G-1)-square [1,G-1]^2; a run ends UNBOUND as soon as a placement
 * exposes a bondable site on the ring outside the box; a site is ambiguous
 * when the tiles that bond to its occupied neighbours form >= 2 distinct
 * (N,E,S,W) colour tuples; frontier moves are drawn uniformly over the
 * frontier in row-major order with Philox4x32-10 (Salmon et al., SC'11)
 * keyed by (seed, step, run, rng_id); runs are compared by occupancy; the
 * shape hash is made invariant under the dihedral group D4.
 *
 * Parity pins: see tests/test_oracle_*.py (closed forms, brute force,
 * invariances, hand traces, rocRAND Philox).
 */
#ifndef JATAM_ORACLE_H
#define JATAM_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* One classification record, 16 bytes. */
typedef struct {
    int32_t  cls;    /* JREF_UNBOUND .. JREF_DET                                  */
    int32_t  size;   /* tiles in the deciding run when it ended (run 0 if DET)    */
    uint32_t hash;   /* D4-invariant shape hash if DET, else 0                    */
    int32_t  steps;  /* placements summed over every run that was executed        */
} jref_result_t;

enum { JREF_UNBOUND = 0, JREF_ND_SITE = 1, JREF_ND_RUNS = 2, JREF_DET = 3 };

/* One item of a mixed stream: genome with its own tile count and grid. */
typedef struct {
    uint64_t genome;
    uint64_t rng_id;
    uint8_t  t;
    uint8_t  grid;
    uint8_t  pad[6];
} jref_item_t;

enum {
    JREF_OK = 0,
    JREF_E_INVALID_ARG = -1,
};

/* Philox4x32-10 block function: out = bijection_key(ctr). */
void jref_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Jenkins one-at-a-time hash of n unsigned bytes (App. F.4). */
uint32_t jref_oaat(const uint8_t* bytes, int64_t n);

/* Default RNG stream id of a genotype: genome | t << 56. */
uint64_t jref_default_rng_id(uint64_t genome, int t);

/* D4-invariant hash of a shape given as a w*h row-major byte mask (nonzero =
 * occupied).  Returns 0 for an empty mask. */
uint32_t jref_shape_hash_d4(const uint8_t* mask, int w, int h);
/* The same over the four rotations only (C4). */
uint32_t jref_shape_hash_c4(const uint8_t* mask, int w, int h);

/* Classification variants (NEXT to the uniform traversal and the D4 hash):
 * JREF_VARIANT_C4 hashes DET shapes up to rotation only; JREF_VARIANT_LIFO
 * grows by the LIFO movelist with random insertion (§3.2). */
enum { JREF_VARIANT_C4 = 1, JREF_VARIANT_LIFO = 2 };

/* genomes, or NULL for the range first + i; variant flags as above. */
int jref_classify_variant(const uint64_t* genomes, uint64_t first, int64_t n, int t, int c,
                          int grid, int runs, uint64_t seed, int variant, jref_result_t* out,
                          int threads);

/* jref_trace_run with a traversal variant. */
int jref_trace_run_variant(uint64_t genome, uint64_t rng_id, int t, int c, int grid,
                           int run, uint64_t seed, int variant, int32_t* cells_out, int cap,
                           int* event, int* choice);

/* Checks the arguments of a classification call. */
int jref_check_args(int t, int c, int grid, int runs);

/* Classifies one genotype.  occ_out, if not NULL, receives the (G+1)*(G+1)
 * occupancy of the deciding run (run 0 for DET), row-major, 1 = occupied. */
int jref_classify_one(uint64_t genome, uint64_t rng_id, int t, int c, int grid,
                      int runs, uint64_t seed, jref_result_t* out,
                      uint8_t* occ_out);

/* Classifies n genotypes with the default rng_id, on `threads` host threads
 * (<= 0: all online cores). */
int jref_classify(const uint64_t* genomes, int64_t n, int t, int c, int grid,
                  int runs, uint64_t seed, jref_result_t* out, int threads);

/* Same with genome i = first + i. */
int jref_classify_range(uint64_t first, int64_t n, int t, int c, int grid,
                        int runs, uint64_t seed, jref_result_t* out, int threads);

/* Same over a mixed stream of items (own t, grid and rng_id each). */
int jref_classify_items(const jref_item_t* items, int64_t n, int c, int runs,
                        uint64_t seed, jref_result_t* out, int threads);

/* Same as jref_classify_range, also reporting the first run of every
 * genotype: its placements, its event (0 none, 1 unbound, 2 ambiguous),
 * whether it ever had two frontier sites to choose from, and in
 * run0_forced bit 0 whether its shape is forced, bit 1 whether it is
 * guarded.  Used to account the work of each stage of a pipelined
 * implementation and to pin the shortcuts such a pipeline takes. */
int jref_classify_range_run0(uint64_t first, int64_t n, int t, int c, int grid,
                             int runs, uint64_t seed, jref_result_t* out,
                             int32_t* run0_steps, int8_t* run0_event,
                             int8_t* run0_choice, int8_t* run0_forced, int threads);

/* Traces one run: writes the placed cells in placement order (y*(G+1)+x,
 * seed first) to cells_out (capacity cap) and returns the event code of the
 * run (0 none/done, 1 unbound, 2 ambiguous) through *event.  Returns the
 * number of cells written, or a negative error. */
int jref_trace_run(uint64_t genome, uint64_t rng_id, int t, int c, int grid,
                   int run, uint64_t seed, int32_t* cells_out, int cap,
                   int* event, int* choice);

/* True class of n genotypes of t tiles on a G-grid by exhaustive
 * exploration of every growth order, breadth first over the event-free
 * states ((cell, tile) sets), each visited once.  out[i]: cls JREF_DET (one
 * terminal shape and no event reachable; size and hash of that shape),
 * JREF_ND_SITE (an event or a second terminal shape is reachable; size and
 * hash 0), or -2 (more than cap states; undecided); steps = states visited
 * when the exploration stopped.  Single-threaded. */
int jref_true_class(const uint64_t* genomes, int64_t n, int t, int c, int grid, int64_t cap,
                    jref_result_t* out);

/* ---- genetic algorithm (jatam_ga_oracle.c) ---- */
typedef struct {
    uint64_t seed;        /* Philox key of the GA's draws                   */
    int tournament;       /* tournament size T, 1..8                         */
    int mut_num, mut_den; /* per-edge mutation probability mut_num/mut_den   */
} jref_ga_params_t;

int jref_ga_check_params(const jref_ga_params_t* p, int t, int c);

/* n_out offspring of generation `generation` from a population of n. */
int jref_ga_offspring(const uint64_t* pop, const int32_t* fit, int64_t n, int t, int c,
                      const jref_ga_params_t* p, int32_t generation, int64_t n_out,
                      uint64_t* out);

/* One generation: n offspring and their fitness (DET size, else 0). */
int jref_ga_step(const uint64_t* pop, const int32_t* fit, int64_t n, int t, int c, int grid,
                 int runs, uint64_t seed, const jref_ga_params_t* p, int32_t generation,
                 uint64_t* next_pop, int32_t* next_fit, int threads);

/* ---- the paper's GA: roulette, single-point crossover, Poisson bit flips
 *      (jatam_roulette_oracle.c) ---- */
typedef struct {
    uint64_t seed;     /* Philox key of the GA's draws                     */
    int32_t length;    /* genome bits L, 1..64                             */
    int32_t crossover; /* 1: single-point crossover with a second parent   */
    double lambda;     /* mean number of flipped bits per offspring, mu L  */
} jref_roulette_params_t;

/* App. C.1's lookup: the first index whose running sum of weights reaches
 * cutoff, or -1. */
int64_t jref_roulette_lookup(const uint32_t* weights, int64_t n, uint64_t cutoff);

/* thr[j] = floor(2^32 * P(k <= j)) for k Poisson(lambda), j = 0..length
 * (2^32 once the sum reaches 1). */
void jref_poisson_thresholds(double lambda, int length, uint64_t* thr);

int jref_roulette_check(const jref_roulette_params_t* p, int64_t n);

/* n_out offspring of generation `generation` from a population of n with
 * fitness fit (each below 2^16, n <= 2^16). */
int jref_roulette_offspring(const uint64_t* pop, const uint32_t* fit, int64_t n,
                            const jref_roulette_params_t* p, int32_t generation, int64_t n_out,
                            uint64_t* out);

/* One Fujiyama simulation from the all-zero population of n: discovery and
 * adaptation times of Hamming weight `target` (-1: not within cutoff
 * generations); final_pop (n entries, or NULL) the population at the end. */
int jref_fujiyama(const jref_roulette_params_t* p, int64_t n, int32_t target, int32_t cutoff,
                  int32_t* discovery, int32_t* adaptation, uint64_t* final_pop);

#ifdef __cplusplus
}
#endif

#endif /* JATAM_ORACLE_H */
