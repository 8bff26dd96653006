/*
 * jatam_ga_oracle.c - plain CPU oracle of one generation of the genetic
 * algorithm whose fitness is JaTAM assembly (§2.2, §3.1).
 *
 * TEST INFRASTRUCTURE ONLY (see jatam_oracle.h).  The paper's GA selects by
 * global roulette and mutates by Poisson-distributed bit flips; the
 * configuration built here fixes instead (documented readings):
 *   selection  tournament of T genomes drawn uniformly with replacement; the
 *              fittest wins, ties go to the earliest draw;
 *   crossover  uniform per edge: each of the 4t edge colours comes from
 *              parent B when bit e of a random word is set, else from A;
 *   mutation   each edge mutates with probability num/den to a colour drawn
 *              uniformly from the other c-1 colours; no elitism;
 *   fitness    size of the structure if the genotype is DET, else 0.
 * The random words of offspring i in generation g are the Philox4x32-10
 * stream keyed by the GA seed at counter (i, g, block, 1 << 28): word q is
 * word q % 4 of block q / 4.  Words 0..T-1 draw parent A's tournament,
 * T..2T-1 parent B's, 2T is the crossover mask, 2T+1+e the mutation test of
 * edge e and 2T+1+E+e its replacement colour (E = 4t edges).
 */
#include "jatam_oracle.h"

#include <stdlib.h>

static uint32_t ga_word(uint64_t seed, uint64_t i, int32_t generation, int q)
{
    const uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    const uint32_t ctr[4] = { (uint32_t)i, (uint32_t)generation, (uint32_t)(q / 4),
                              1u << 28 };
    uint32_t out[4];
    jref_philox4x32_10(ctr, key, out);
    return out[q % 4];
}

/* floor(u * n / 2^32): a uniform integer in [0, n) from a 32-bit word */
static uint32_t scale(uint32_t u, uint32_t n)
{
    return (uint32_t)(((uint64_t)u * n) >> 32);
}

static int64_t tournament(const int32_t* fit, int64_t n, uint64_t seed, uint64_t i,
                          int32_t generation, int first_word, int size)
{
    int64_t best = -1;
    for (int k = 0; k < size; ++k) {
        const int64_t d = (int64_t)(((uint64_t)ga_word(seed, i, generation, first_word + k) *
                                     (uint64_t)n) >> 32);
        if (best < 0 || fit[d] > fit[best])
            best = d;
    }
    return best;
}

int jref_ga_check_params(const jref_ga_params_t* p, int t, int c)
{
    if (!p || p->tournament < 1 || p->tournament > 8 || p->mut_den < 1 || p->mut_num < 0 ||
        p->mut_num > p->mut_den)
        return JREF_E_INVALID_ARG;
    return jref_check_args(t, c, 16, 1);
}

int jref_ga_offspring(const uint64_t* pop, const int32_t* fit, int64_t n, int t, int c,
                      const jref_ga_params_t* p, int32_t generation, int64_t n_out,
                      uint64_t* out)
{
    if (jref_ga_check_params(p, t, c) != JREF_OK || n < 1 || n > 0xFFFFFFFFll || n_out < 0 ||
        n_out > 0xFFFFFFFFll)
        return JREF_E_INVALID_ARG;
    int b = 0;
    while ((1 << b) < c)
        ++b;
    const int E = 4 * t, T = p->tournament;
    for (int64_t i = 0; i < n_out; ++i) {
        const uint64_t pa = pop[tournament(fit, n, p->seed, (uint64_t)i, generation, 0, T)];
        const uint64_t pb = pop[tournament(fit, n, p->seed, (uint64_t)i, generation, T, T)];
        const uint32_t mask = ga_word(p->seed, (uint64_t)i, generation, 2 * T);
        uint64_t child = 0;
        for (int e = 0; e < E; ++e) {
            const int shift = b * (E - 1 - e);
            const uint64_t src = (mask >> e) & 1u ? pb : pa;
            uint32_t colour = (uint32_t)((src >> shift) & (uint64_t)(c - 1));
            const uint32_t test = ga_word(p->seed, (uint64_t)i, generation, 2 * T + 1 + e);
            if (scale(test, (uint32_t)p->mut_den) < (uint32_t)p->mut_num) {
                const uint32_t r = scale(ga_word(p->seed, (uint64_t)i, generation,
                                                 2 * T + 1 + E + e), (uint32_t)(c - 1));
                colour = r < colour ? r : r + 1;
            }
            child |= (uint64_t)colour << shift;
        }
        out[i] = child;
    }
    return JREF_OK;
}

int jref_ga_step(const uint64_t* pop, const int32_t* fit, int64_t n, int t, int c, int grid,
                 int runs, uint64_t seed, const jref_ga_params_t* p, int32_t generation,
                 uint64_t* next_pop, int32_t* next_fit, int threads)
{
    int rc = jref_ga_offspring(pop, fit, n, t, c, p, generation, n, next_pop);
    if (rc != JREF_OK)
        return rc;
    jref_result_t* rec = (jref_result_t*)malloc((size_t)n * sizeof(jref_result_t));
    if (!rec)
        return JREF_E_INVALID_ARG;
    rc = jref_classify(next_pop, n, t, c, grid, runs, seed, rec, threads);
    if (rc == JREF_OK)
        for (int64_t i = 0; i < n; ++i)
            next_fit[i] = rec[i].cls == JREF_DET ? rec[i].size : 0;
    free(rec);
    return rc;
}
