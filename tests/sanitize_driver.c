/*
 * Exercises every entry point of the CPU oracle in one process built with
 * AddressSanitizer and UndefinedBehaviorSanitizer (tests/test_oracle_
 * sanitizers.py builds and runs it).  Prints one line of FNV-1a checksums
 * of the results, which the test compares with the same calls through the
 * ordinary build.
 */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../oracle/jatam_oracle.h"

static uint64_t fnv(uint64_t h, const void* data, size_t n)
{
    const unsigned char* p = (const unsigned char*)data;
    for (size_t i = 0; i < n; ++i) {
        h ^= p[i];
        h *= 1099511628211ull;
    }
    return h;
}

int main(void)
{
    const uint64_t basis = 1469598103934665603ull;
    enum { N1 = 4096, N2 = 2000 };
    jref_result_t* rec = (jref_result_t*)calloc(N1, sizeof(jref_result_t));
    uint64_t* gen = (uint64_t*)calloc(N2, sizeof(uint64_t));
    uint64_t state = 88172645463325252ull;
    for (int i = 0; i < N2; ++i) {
        state ^= state << 13;
        state ^= state >> 7;
        state ^= state << 17;
        gen[i] = state & ((1ull << 36) - 1);
    }
    /* classification: S_1,8 at G = 16, three-tile genotypes at G = 32 */
    if (jref_classify_range(0, N1, 1, 8, 16, 20, 1, rec, 2) != JREF_OK)
        return 2;
    uint64_t h_s18 = fnv(basis, rec, N1 * sizeof(jref_result_t));
    if (jref_classify(gen, 500, 3, 8, 32, 20, 1, rec, 2) != JREF_OK)
        return 3;
    uint64_t h_t3 = fnv(basis, rec, 500 * sizeof(jref_result_t));
    /* variants: C4 hash and the LIFO movelist */
    if (jref_classify_variant(NULL, 0, N1, 1, 8, 16, 20, 1, JREF_VARIANT_C4 | JREF_VARIANT_LIFO,
                              rec, 2) != JREF_OK)
        return 4;
    uint64_t h_var = fnv(basis, rec, N1 * sizeof(jref_result_t));
    /* true class of two-tile genotypes */
    for (int i = 0; i < 300; ++i)
        gen[i] &= (1ull << 24) - 1;
    if (jref_true_class(gen, 300, 2, 8, 16, 1 << 16, rec) != JREF_OK)
        return 5;
    uint64_t h_true = fnv(basis, rec, 300 * sizeof(jref_result_t));
    /* the tournament GA and the roulette GA */
    int32_t fit[256];
    uint32_t ufit[256];
    uint64_t pop[256], nxt[256];
    for (int i = 0; i < 256; ++i) {
        pop[i] = gen[i] & ((1ull << 36) - 1);
        fit[i] = (int32_t)(gen[i] % 17);
        ufit[i] = (uint32_t)(gen[i] % 29);
    }
    jref_ga_params_t gp = { 5, 4, 1, 12 };
    int32_t nfit[256];
    if (jref_ga_step(pop, fit, 256, 3, 8, 32, 20, 1, &gp, 0, nxt, nfit, 2) != JREF_OK)
        return 6;
    uint64_t h_ga = fnv(fnv(basis, nxt, sizeof(nxt)), nfit, sizeof(nfit));
    jref_roulette_params_t rp = { 7, 36, 1, 1.5 };
    if (jref_roulette_offspring(pop, ufit, 256, &rp, 3, 256, nxt) != JREF_OK)
        return 7;
    uint64_t h_rou = fnv(basis, nxt, sizeof(nxt));
    int32_t d = 0, a = 0;
    rp.length = 24;
    rp.lambda = 0.5;
    if (jref_fujiyama(&rp, 128, 18, 300, &d, &a, nxt) != JREF_OK)
        return 8;
    uint64_t h_fuji = fnv(fnv(basis, &d, sizeof(d)), &a, sizeof(a));
    printf("%016llx %016llx %016llx %016llx %016llx %016llx %016llx\n",
           (unsigned long long)h_s18, (unsigned long long)h_t3, (unsigned long long)h_var,
           (unsigned long long)h_true, (unsigned long long)h_ga, (unsigned long long)h_rou,
           (unsigned long long)h_fuji);
    free(rec);
    free(gen);
    return 0;
}
