// jatam_api.cpp - the extern "C" entry points of include/jatam.h: argument
// validation, parameter digestion and kernel launch.  Only jatam_batch_create
// allocates (its workspace); no exception crosses the ABI.
#include <hip/hip_runtime.h>

#include <new>
#include <vector>

#include "jatam_internal.hpp"

struct jatam_batch {
    int device;
    int64_t max_n;
    int blocks[2][2];              // persistent grid per grid class and tile bound
    jatam::DeviceWorkspace ws;
    void* allocations[16];
    int nalloc;
    // timing hook: one set of stage events per call made while enabled
    int refill;                    // idle lanes that trigger a first-run refill
    bool timing;
    std::vector<hipEvent_t> marks;        // 2 * kStages per recorded call
    std::vector<uint8_t> launched;        // kStages per recorded call
};

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

int jatam_abi_version(void) { return 2; }

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

// ---------------------------------------------------------------------------
// Pipelined path.
// ---------------------------------------------------------------------------
static void drop_marks(jatam_batch_t* b)
{
    for (hipEvent_t e : b->marks)
        (void)hipEventDestroy(e);
    b->marks.clear();
    b->launched.clear();
}

static void free_batch(jatam_batch_t* b)
{
    drop_marks(b);
    for (int i = 0; i < b->nalloc; ++i)
        (void)hipFree(b->allocations[i]);
    delete b;
}

// Events and launched flags for the next call when timing is on.
static int next_marks(jatam_batch_t* b, hipEvent_t** marks, uint8_t** launched)
{
    *marks = nullptr;
    *launched = nullptr;
    if (!b->timing)
        return JATAM_OK;
    for (int i = 0; i < 2 * jatam::kStages; ++i) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess)
            return JATAM_E_HIP;
        b->marks.push_back(e);
    }
    b->launched.resize(b->launched.size() + jatam::kStages, 0);
    *marks = b->marks.data() + b->marks.size() - 2 * jatam::kStages;
    *launched = b->launched.data() + b->launched.size() - jatam::kStages;
    return JATAM_OK;
}

static int launch_timed(jatam_batch_t* b, const jatam::BatchArgs& a, const bool classes[2],
                        int max_t, hipStream_t stream)
{
    hipEvent_t* marks;
    uint8_t* launched;
    const int rc = next_marks(b, &marks, &launched);
    if (rc != JATAM_OK)
        return rc;
    return jatam::launch_batched(a, classes, b->blocks, max_t <= 2 ? 2 : 4, stream, marks,
                                 launched);
}

static bool batch_alloc(jatam_batch_t* b, size_t bytes, void** out)
{
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess)
        return false;
    b->allocations[b->nalloc++] = p;
    *out = p;
    return true;
}

int jatam_batch_create(int64_t max_n, jatam_batch_t** batch)
{
    if (batch == nullptr || max_n < 1 || max_n > (int64_t)0xFFFFFFFFu)
        return JATAM_E_INVALID_ARG;
    *batch = nullptr;
    jatam_batch_t* b = new (std::nothrow) jatam_batch_t();
    if (b == nullptr)
        return JATAM_E_HIP;
    b->max_n = max_n;
    b->nalloc = 0;
    b->timing = false;
    b->refill = 24;
    hipDeviceProp_t prop;
    if (hipGetDevice(&b->device) != hipSuccess ||
        hipGetDeviceProperties(&prop, b->device) != hipSuccess) {
        delete b;
        return JATAM_E_HIP;
    }
    jatam::batch_persistent_blocks(prop.multiProcessorCount, b->blocks);
    int max_blocks = 1;
    for (int k = 0; k < 2; ++k)
        for (int i = 0; i < 2; ++i)
            max_blocks = b->blocks[k][i] > max_blocks ? b->blocks[k][i] : max_blocks;
    const size_t n = (size_t)max_n;
    const size_t staging = n + 64 * ((size_t)max_blocks + 1);
    jatam::DeviceWorkspace& ws = b->ws;
    bool ok = batch_alloc(b, jatam::kCntWords * sizeof(uint32_t), (void**)&ws.counters) &&
              batch_alloc(b, 2 * sizeof(uint32_t), (void**)&ws.small_hash);
    for (int k = 0; k < 2 && ok; ++k) {
        ok = batch_alloc(b, (size_t)max_blocks * sizeof(uint32_t), (void**)&ws.seg_count[k]) &&
             batch_alloc(b, (size_t)jatam::kSizeBuckets * max_blocks * sizeof(uint32_t),
                         (void**)&ws.seg_hist[k]) &&
             batch_alloc(b, staging * sizeof(uint32_t), (void**)&ws.cand_idx[k]) &&
             batch_alloc(b, staging * sizeof(uint16_t), (void**)&ws.cand_size[k]) &&
             batch_alloc(b, n * sizeof(uint32_t), (void**)&ws.sorted[k]);
    }
    if (!ok) {
        free_batch(b);
        return JATAM_E_HIP;
    }
    if (jatam::batch_init_small_hash(ws.small_hash, nullptr) != JATAM_OK ||
        hipDeviceSynchronize() != hipSuccess) {
        free_batch(b);
        return JATAM_E_HIP;
    }
    *batch = b;
    return JATAM_OK;
}

int jatam_batch_destroy(jatam_batch_t* batch)
{
    if (batch == nullptr)
        return JATAM_OK;
    int dev = 0;
    (void)hipGetDevice(&dev);
    (void)hipSetDevice(batch->device);
    const hipError_t e = hipDeviceSynchronize();
    free_batch(batch);
    (void)hipSetDevice(dev);
    return e == hipSuccess ? JATAM_OK : JATAM_E_HIP;
}

static int batch_check(jatam_batch_t* b, int64_t n, const void* out)
{
    if (b == nullptr || n < 0 || n > b->max_n || (n > 0 && out == nullptr))
        return JATAM_E_INVALID_ARG;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != b->device)
        return JATAM_E_INVALID_ARG;
    return JATAM_OK;
}

static jatam::BatchArgs batch_args(jatam_batch_t* b, const jatam::Params& p, int64_t n,
                                   jatam_result_t* out, uint64_t* tally)
{
    jatam::BatchArgs a;
    a.genomes = nullptr;
    a.items = nullptr;
    a.first = 0;
    a.n = n;
    a.t = p.t;
    a.grid = p.grid;
    a.c = p.c;
    a.bits = p.bits;
    a.runs = p.runs;
    a.key0 = p.key0;
    a.key1 = p.key1;
    a.refill = b->refill;
    a.seg_cap = 0;
    a.out = out;
    a.tally = reinterpret_cast<unsigned long long*>(tally);
    a.ws = b->ws;
    return a;
}

int jatam_batch_classify(jatam_batch_t* batch, const uint64_t* genotypes, int64_t n, int t,
                         int c, int grid_limit, int runs, uint64_t seed, jatam_result_t* out,
                         uint64_t* tally, void* stream)
{
    jatam::Params p;
    int rc = make_params(t, c, grid_limit, runs, seed, &p);
    if (rc != JATAM_OK)
        return rc;
    if ((rc = batch_check(batch, n, out)) != JATAM_OK)
        return rc;
    if (n > 0 && genotypes == nullptr)
        return JATAM_E_INVALID_ARG;
    jatam::BatchArgs a = batch_args(batch, p, n, out, tally);
    a.genomes = genotypes;
    const bool classes[2] = {grid_limit <= 16, grid_limit > 16};
    return launch_timed(batch, a, classes, t, (hipStream_t)stream);
}

int jatam_batch_classify_range(jatam_batch_t* batch, uint64_t first, int64_t n, int t, int c,
                               int grid_limit, int runs, uint64_t seed, jatam_result_t* out,
                               uint64_t* tally, void* stream)
{
    jatam::Params p;
    int rc = make_params(t, c, grid_limit, runs, seed, &p);
    if (rc != JATAM_OK)
        return rc;
    if ((rc = batch_check(batch, n, out)) != JATAM_OK)
        return rc;
    if (n > 0) {
        const uint64_t last = first + (uint64_t)(n - 1);
        if (last < first || (p.genome_bits < 64 && (last >> p.genome_bits) != 0))
            return JATAM_E_INVALID_ARG;
    }
    jatam::BatchArgs a = batch_args(batch, p, n, out, tally);
    a.first = first;
    const bool classes[2] = {grid_limit <= 16, grid_limit > 16};
    return launch_timed(batch, a, classes, t, (hipStream_t)stream);
}

int jatam_batch_classify_items(jatam_batch_t* batch, const jatam_item_t* items, int64_t n,
                               int c, int runs, uint64_t seed, jatam_result_t* out,
                               uint64_t* tally, void* stream)
{
    jatam::Params p;
    // t and grid are per item; validate the shared arguments with placeholders
    int rc = make_params(1, c, 16, runs, seed, &p);
    if (rc != JATAM_OK)
        return rc;
    if ((rc = batch_check(batch, n, out)) != JATAM_OK)
        return rc;
    if (n > 0 && items == nullptr)
        return JATAM_E_INVALID_ARG;
    jatam::BatchArgs a = batch_args(batch, p, n, out, tally);
    a.items = items;
    const bool classes[2] = {true, true};
    return launch_timed(batch, a, classes, 4, (hipStream_t)stream);
}

int jatam_batch_set_refill(jatam_batch_t* batch, int idle_lanes)
{
    if (batch == nullptr || idle_lanes < 1 || idle_lanes > 64)
        return JATAM_E_INVALID_ARG;
    batch->refill = idle_lanes;
    return JATAM_OK;
}

int jatam_batch_set_timing(jatam_batch_t* batch, int enable)
{
    if (batch == nullptr)
        return JATAM_E_INVALID_ARG;
    int dev = 0;
    (void)hipGetDevice(&dev);
    (void)hipSetDevice(batch->device);
    const hipError_t e = hipDeviceSynchronize();
    drop_marks(batch);
    batch->timing = enable != 0;
    (void)hipSetDevice(dev);
    return e == hipSuccess ? JATAM_OK : JATAM_E_HIP;
}

int jatam_batch_stage_times(jatam_batch_t* batch, double* ms, int* calls, int max_stages)
{
    if (batch == nullptr || ms == nullptr || max_stages < 0)
        return JATAM_E_INVALID_ARG;
    const int stages = max_stages < jatam::kStages ? max_stages : jatam::kStages;
    for (int s = 0; s < stages; ++s) {
        ms[s] = 0.0;
        if (calls)
            calls[s] = 0;
    }
    const size_t ncalls = batch->marks.size() / (2 * jatam::kStages);
    for (size_t c = 0; c < ncalls; ++c) {
        for (int s = 0; s < stages; ++s) {
            if (!batch->launched[c * jatam::kStages + s])
                continue;
            hipEvent_t a = batch->marks[(c * jatam::kStages + s) * 2];
            hipEvent_t b = batch->marks[(c * jatam::kStages + s) * 2 + 1];
            float t = 0.f;
            if (hipEventSynchronize(b) != hipSuccess || hipEventElapsedTime(&t, a, b) != hipSuccess)
                return JATAM_E_HIP;
            ms[s] += t;
            if (calls)
                calls[s] += 1;
        }
    }
    return stages;
}

const char* jatam_batch_stage_name(int stage)
{
    static const char* names[jatam::kStages] = {
        "first_run_kernel<16>", "size_sort<16>", "repeat_kernel<16>",
        "first_run_kernel<32>", "size_sort<32>", "repeat_kernel<32>"};
    return stage >= 0 && stage < jatam::kStages ? names[stage] : "";
}

}  // extern "C"
