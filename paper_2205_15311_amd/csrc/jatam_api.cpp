// jatam_api.cpp - the extern "C" entry points of include/jatam.h: argument
// validation, parameter digestion and kernel launch.  No memory is allocated
// and no exception crosses the ABI.
#include <hip/hip_runtime.h>

#include "jatam_internal.hpp"

namespace {

int log2_exact(int c)
{
    switch (c) {
    case 2: return 1;
    case 4: return 2;
    case 8: return 3;
    case 16: return 4;
    default: return -1;
    }
}

int make_params(int t, int c, int grid, int runs, uint64_t seed, jatam::Params* p)
{
    const int bits = log2_exact(c);
    if (t < 1 || t > 4 || bits < 0 || 4 * t * bits > 64)
        return JATAM_E_INVALID_ARG;
    if (grid < 8 || grid > 64 || (grid & 1) || runs < 1 || runs > 64)
        return JATAM_E_INVALID_ARG;
    if (grid > 32)
        return JATAM_E_UNSUPPORTED;
    p->t = t;
    p->c = c;
    p->bits = bits;
    p->genome_bits = 4 * t * bits;
    p->grid = grid;
    p->runs = runs;
    p->key0 = (uint32_t)seed;
    p->key1 = (uint32_t)(seed >> 32);
    return JATAM_OK;
}

}  // namespace

extern "C" {

int jatam_abi_version(void) { return 1; }

const char* jatam_strerror(int code)
{
    switch (code) {
    case JATAM_OK: return "ok";
    case JATAM_E_INVALID_ARG: return "invalid argument";
    case JATAM_E_UNSUPPORTED: return "unsupported configuration";
    case JATAM_E_HIP: return "HIP runtime error";
    default: return "unknown error";
    }
}

int jatam_classify(const uint64_t* genotypes, int64_t n, int t, int c, int grid_limit, int runs,
                   uint64_t seed, jatam_result_t* out, void* stream)
{
    jatam::Params p;
    const int rc = make_params(t, c, grid_limit, runs, seed, &p);
    if (rc != JATAM_OK)
        return rc;
    if (n < 0 || (n > 0 && (genotypes == nullptr || out == nullptr)))
        return JATAM_E_INVALID_ARG;
    return jatam::launch_plain(genotypes, 0, n, p, out, (hipStream_t)stream);
}

int jatam_classify_range(uint64_t first, int64_t n, int t, int c, int grid_limit, int runs,
                         uint64_t seed, jatam_result_t* out, void* stream)
{
    jatam::Params p;
    const int rc = make_params(t, c, grid_limit, runs, seed, &p);
    if (rc != JATAM_OK)
        return rc;
    if (n < 0 || (n > 0 && out == nullptr))
        return JATAM_E_INVALID_ARG;
    if (n > 0) {
        // every genome of the range must fit in 4*t*log2(c) bits
        const uint64_t last = first + (uint64_t)(n - 1);
        if (last < first)
            return JATAM_E_INVALID_ARG;
        if (p.genome_bits < 64 && (last >> p.genome_bits) != 0)
            return JATAM_E_INVALID_ARG;
    }
    return jatam::launch_plain(nullptr, first, n, p, out, (hipStream_t)stream);
}

}  // extern "C"
