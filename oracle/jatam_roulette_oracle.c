/*
 * jatam_roulette_oracle.c - plain CPU oracle of the paper's own genetic
 * algorithm: global roulette wheel selection, single-point crossover and
 * Poisson-distributed bit-flip mutation (§2.2, §3.1, App. C.1, App. D.1,
 * App. D.2), and its Fujiyama test bed (§4.2).
 *
 * TEST INFRASTRUCTURE ONLY (see jatam_oracle.h).  Readings where the paper
 * leaves a choice open:
 *   genome     L bits (1..64) in the low bits of a word; position 0 of the
 *              bit string is bit L-1 (the first bit of the first byte);
 *   fitness    non-negative integers, f_i < 2^16, population n <= 2^16, so
 *              the wheel's total S = sum f_i stays below 2^32;
 *   roulette   a dart d = floor(u S / 2^32) from a 32-bit word u lands in
 *              the area of the first genome whose running fitness sum
 *              exceeds d (App. C.1's lookup: the first index whose running
 *              sum reaches the cut-off d + 1); every area is proportional
 *              to f_i.  With S = 0 every genome has the same chance:
 *              floor(u n / 2^32);
 *   crossover  (when enabled) a second parent b by a second dart; a point
 *              p = floor(u L / 2^32) in [0, L); the child takes positions
 *              0..p-1 from b and the rest from a (App. D.2 copies the bytes
 *              before the crossover byte, and that byte's leading bits,
 *              from the other genome);
 *   mutation   the number of flipped bits k is Poisson with mean lambda
 *              (lambda = mu L, App. D.1): k = the first j with u < T_j,
 *              T_j = floor(2^32 cdf(j)) from the cumulative Poisson
 *              probabilities computed in double precision by the recurrence
 *              p_0 = exp(-lambda), p_j = p_(j-1) * lambda / j; at most L.
 *              Then k distinct positions, each floor(u L / 2^32) from the
 *              next word, a position already chosen being drawn again
 *              (App. D.1's retry), with at most 1024 position draws in all;
 *   words      offspring i of generation g draws from the Philox4x32-10
 *              stream keyed by the GA seed at counter (i, g, block, 4 << 28)
 *              (domain tag 4); word q is word q % 4 of block q / 4: word 0
 *              the dart of parent a, 1 the dart of parent b, 2 the crossover
 *              point, 3 the number of flips, 4.. the flipped positions.
 * Fujiyama (§4.2): fitness = Hamming weight of the genome; every simulation
 * starts from the all-zero population; its discovery time is the first
 * generation in which some genome reaches the target weight H, its
 * adaptation time the first in which at least half of the population has;
 * generation 0 is the initial population and a simulation stops at the
 * cut-off (-1 for a time not reached).  Simulation s of a batch uses GA
 * seed base_seed + s.
 */
#include "jatam_oracle.h"

#include <math.h>
#include <stdlib.h>

static uint32_t roulette_word(uint64_t seed, uint64_t i, int32_t generation, int q)
{
    const uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    const uint32_t ctr[4] = { (uint32_t)i, (uint32_t)generation, (uint32_t)(q / 4), 4u << 28 };
    uint32_t out[4];
    jref_philox4x32_10(ctr, key, out);
    return out[q % 4];
}

int64_t jref_roulette_lookup(const uint32_t* weights, int64_t n, uint64_t cutoff)
{
    uint64_t partsum = 0;
    for (int64_t i = 0; i < n; ++i) {
        partsum += weights[i];
        if (partsum >= cutoff)
            return i;
    }
    return -1;
}

void jref_poisson_thresholds(double lambda, int length, uint64_t* thr)
{
    double p = exp(-lambda);
    double cdf = p;
    for (int j = 0; j <= length; ++j) {
        if (j > 0) {
            p = p * lambda / (double)j;
            cdf = cdf + p;
        }
        const double scaled = cdf * 4294967296.0;
        thr[j] = scaled >= 4294967296.0 ? (uint64_t)1 << 32 : (uint64_t)floor(scaled);
    }
}

int jref_roulette_check(const jref_roulette_params_t* p, int64_t n)
{
    if (!p || p->length < 1 || p->length > 64 || p->crossover < 0 || p->crossover > 1 ||
        !(p->lambda >= 0.0 && p->lambda <= 64.0) || n < 1 || n > 65536)
        return JREF_E_INVALID_ARG;
    return JREF_OK;
}

static uint64_t bit_at(int length, int pos)
{
    return (uint64_t)1 << (length - 1 - pos);
}

/* The parent a dart lands on: roulette over the running sums of fit. */
static int64_t roulette_pick(const uint32_t* fit, int64_t n, uint64_t total, uint32_t u)
{
    if (total == 0)
        return (int64_t)(((uint64_t)u * (uint64_t)n) >> 32);
    const uint64_t dart = ((uint64_t)u * total) >> 32;
    return jref_roulette_lookup(fit, n, dart + 1);
}

int jref_roulette_offspring(const uint64_t* pop, const uint32_t* fit, int64_t n,
                            const jref_roulette_params_t* p, int32_t generation, int64_t n_out,
                            uint64_t* out)
{
    if (jref_roulette_check(p, n) != JREF_OK || n_out < 0 || n_out > 0xFFFFFFFFll)
        return JREF_E_INVALID_ARG;
    uint64_t total = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (fit[i] >= 65536u)
            return JREF_E_INVALID_ARG;
        total += fit[i];
    }
    const int L = p->length;
    const uint64_t mask = L == 64 ? ~(uint64_t)0 : (((uint64_t)1 << L) - 1);
    uint64_t thr[65];
    jref_poisson_thresholds(p->lambda, L, thr);
    for (int64_t i = 0; i < n_out; ++i) {
        const uint64_t id = (uint64_t)i;
        const uint64_t a = pop[roulette_pick(fit, n, total, roulette_word(p->seed, id,
                                                                            generation, 0))];
        uint64_t child = a & mask;
        if (p->crossover) {
            const uint64_t b = pop[roulette_pick(fit, n, total,
                                                 roulette_word(p->seed, id, generation, 1))];
            const int point = (int)(((uint64_t)roulette_word(p->seed, id, generation, 2) *
                                     (uint64_t)L) >> 32);
            for (int pos = 0; pos < point; ++pos) {
                const uint64_t bit = bit_at(L, pos);
                child = (child & ~bit) | (b & bit);
            }
        }
        const uint32_t uk = roulette_word(p->seed, id, generation, 3);
        int flips = L;
        for (int j = 0; j < L; ++j)
            if ((uint64_t)uk < thr[j]) {
                flips = j;
                break;
            }
        uint64_t chosen = 0;
        int done = 0;
        for (int q = 4; done < flips && q < 4 + 1024; ++q) {
            const int pos = (int)(((uint64_t)roulette_word(p->seed, id, generation, q) *
                                   (uint64_t)L) >> 32);
            if (chosen & bit_at(L, pos))
                continue;   /* drawn already: draw again */
            chosen |= bit_at(L, pos);
            ++done;
        }
        out[i] = child ^ chosen;
    }
    return JREF_OK;
}

static uint32_t hamming_weight(uint64_t x)
{
    uint32_t w = 0;
    for (; x; x &= x - 1)
        ++w;
    return w;
}

int jref_fujiyama(const jref_roulette_params_t* p, int64_t n, int32_t target, int32_t cutoff,
                  int32_t* discovery, int32_t* adaptation, uint64_t* final_pop)
{
    if (jref_roulette_check(p, n) != JREF_OK || cutoff < 0 || target < 0 || target > p->length)
        return JREF_E_INVALID_ARG;
    uint64_t* pop = (uint64_t*)calloc((size_t)n, sizeof(uint64_t));
    uint64_t* nxt = (uint64_t*)calloc((size_t)n, sizeof(uint64_t));
    uint32_t* fit = (uint32_t*)calloc((size_t)n, sizeof(uint32_t));
    if (!pop || !nxt || !fit) {
        free(pop);
        free(nxt);
        free(fit);
        return JREF_E_INVALID_ARG;
    }
    *discovery = -1;
    *adaptation = -1;
    for (int32_t g = 0; g <= cutoff; ++g) {
        int64_t reached = 0;
        for (int64_t i = 0; i < n; ++i) {
            fit[i] = hamming_weight(pop[i]);
            reached += fit[i] >= (uint32_t)target;
        }
        if (*discovery < 0 && reached > 0)
            *discovery = g;
        if (*adaptation < 0 && 2 * reached >= n)
            *adaptation = g;
        if ((*discovery >= 0 && *adaptation >= 0) || g == cutoff)
            break;
        jref_roulette_offspring(pop, fit, n, p, g, n, nxt);
        uint64_t* t = pop;
        pop = nxt;
        nxt = t;
    }
    if (final_pop)
        for (int64_t i = 0; i < n; ++i)
            final_pop[i] = pop[i];
    free(pop);
    free(nxt);
    free(fit);
    return JREF_OK;
}
