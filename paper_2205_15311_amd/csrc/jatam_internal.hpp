// jatam_internal.hpp - launch parameters shared by the library's kernels and
// its C-ABI layer (not part of the public header).
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

}  // namespace jatam
