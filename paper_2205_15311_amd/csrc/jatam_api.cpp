// jatam_api.cpp - the extern "C" entry points of include/jatam.h: argument
// validation, parameter digestion and kernel launch.  Only jatam_batch_create
// allocates (its workspace); no exception crosses the ABI.
#include <hip/hip_runtime.h>

#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "jatam_internal.hpp"

struct jatam_batch {
    int device;
    int64_t max_n;
    int cus;                       // compute units of the device
    int occ[2][2][3];              // resident blocks per CU [class][tile bound][stage]
    jatam_tuning_t tune[2];        // launch parameters per grid class
    uint32_t small_hash[2];        // host copy of the workspace's small_hash
    std::vector<std::pair<jatam_tuning_t, double>> tune_log;   // last autotune
    jatam::DeviceWorkspace ws;
    void* allocations[24];
    int nalloc;
    // graph of the last enumeration (kept until the next one or destroy)
    hipStream_t capture_stream;
    hipGraph_t graph;
    hipGraphExec_t graph_exec;
    hipStream_t graph_stream;
    // timing hook: one set of stage events per call made while enabled
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

// Launch parameters of the class of grid_limit within their limits.
bool tuning_valid(int grid_limit, const jatam_tuning_t* t)
{
    return t->refill >= 1 && t->refill <= 64 && t->first_waves >= 1 && t->repeat_waves >= 1 &&
           t->wide_layout >= 0 && t->wide_layout <= (grid_limit > 16 ? 2 : 1) &&
           t->claim_share >= 0 && t->claim_share <= 16 && t->claim_chunks >= 1 &&
           t->claim_chunks <= jatam::kMaxClaimChunks && t->repeat_mapping >= 0 &&
           t->repeat_mapping <= 2;
}

// Candidate values of one tuning field, around the residency limit `occ`.
std::vector<int> wave_choices(int occ)
{
    std::vector<int> v;
    for (int w : {occ, occ - 1, occ - 2, (occ + 1) / 2, (occ + 3) / 4})
        if (w >= 1 && std::find(v.begin(), v.end(), w) == v.end())
            v.push_back(w);
    return v;
}

}  // namespace

extern "C" {

int jatam_abi_version(void) { return 6; }

const char* jatam_strerror(int code)
{
    switch (code) {
    case JATAM_OK: return "ok";
    case JATAM_E_INVALID_ARG: return "invalid argument";
    case JATAM_E_UNSUPPORTED: return "unsupported configuration";
    case JATAM_E_HIP: return "HIP runtime error";
    case JATAM_E_MISMATCH: return "a launch configuration changed the records";
    case JATAM_E_IO: return "a file could not be read or written";
    default: return "unknown error";
    }
}

int jatam_classify(const uint64_t* genotypes, int64_t n, int t, int c, int grid_limit, int runs,
                   uint64_t seed, jatam_result_t* out, void* stream)
{
    jatam::Params p;
    const int rc = jatam::make_params(t, c, grid_limit, runs, seed, &p);
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
    const int rc = jatam::make_params(t, c, grid_limit, runs, seed, &p);
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

int jatam_classify_variant(const uint64_t* genotypes, uint64_t first, int64_t n, int t, int c,
                           int grid_limit, int runs, uint64_t seed, int variant,
                           jatam_result_t* out, void* stream)
{
    jatam::Params p;
    const int rc = jatam::make_params(t, c, grid_limit, runs, seed, &p);
    if (rc != JATAM_OK)
        return rc;
    if (n < 0 || (n > 0 && out == nullptr) ||
        (variant & ~(JATAM_VARIANT_C4 | JATAM_VARIANT_LIFO)) != 0)
        return JATAM_E_INVALID_ARG;
    if (n > 0 && genotypes == nullptr) {
        const uint64_t last = first + (uint64_t)(n - 1);
        if (last < first || (p.genome_bits < 64 && (last >> p.genome_bits) != 0))
            return JATAM_E_INVALID_ARG;
    }
    return jatam::launch_variant(genotypes, first, n, p, variant, out, (hipStream_t)stream);
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

static void drop_graph(jatam_batch_t* b)
{
    if (b->graph_exec != nullptr)
        (void)hipGraphExecDestroy(b->graph_exec);
    if (b->graph != nullptr)
        (void)hipGraphDestroy(b->graph);
    b->graph_exec = nullptr;
    b->graph = nullptr;
}

static void free_batch(jatam_batch_t* b)
{
    drop_marks(b);
    drop_graph(b);
    if (b->capture_stream != nullptr)
        (void)hipStreamDestroy(b->capture_stream);
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

// Launches the pipeline with the workspace's parameters, or `tune` for this
// call.  grid_limit: the uniform G of the call, or 0 for mixed items (both
// grid classes).  marks/launched: timing hook or nullptr.

static int launch_pipeline(jatam_batch_t* b, const jatam::BatchArgs& a, int grid_limit,
                           int max_t, hipStream_t stream, hipEvent_t* marks, uint8_t* launched,
                           const jatam_tuning_t* tune = nullptr)
{
    return jatam::launch_tuned(tune != nullptr ? tune : b->tune, b->occ, b->cus, a, grid_limit,
                               max_t, stream, marks, launched);
}

static int launch_timed(jatam_batch_t* b, const jatam::BatchArgs& a, int grid_limit, int max_t,
                        hipStream_t stream)
{
    hipEvent_t* marks;
    uint8_t* launched;
    const int rc = next_marks(b, &marks, &launched);
    if (rc != JATAM_OK)
        return rc;
    return launch_pipeline(b, a, grid_limit, max_t, stream, marks, launched);
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
    b->capture_stream = nullptr;
    b->graph = nullptr;
    b->graph_exec = nullptr;
    b->graph_stream = nullptr;
    for (int k = 0; k < 2; ++k)
        b->tune[k] = jatam::default_tuning(k);
    hipDeviceProp_t prop;
    if (hipGetDevice(&b->device) != hipSuccess ||
        hipGetDeviceProperties(&prop, b->device) != hipSuccess) {
        delete b;
        return JATAM_E_HIP;
    }
    b->cus = prop.multiProcessorCount;
    jatam::batch_occupancy(b->occ);
    // a stream of its own to capture enumeration graphs on (default priority)
    if (hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking) != hipSuccess) {
        b->capture_stream = nullptr;
        free_batch(b);
        return JATAM_E_HIP;
    }
    const int max_blocks = jatam::max_first_blocks(b->occ, b->cus);
    if (!jatam::scan_fits(max_blocks)) {
        free_batch(b);
        return JATAM_E_UNSUPPORTED;
    }
    // one region, laid out by carve_workspace
    const size_t bytes = jatam::carve_workspace(nullptr, (size_t)max_n, max_blocks, true, nullptr);
    uint8_t* base = nullptr;
    if (!batch_alloc(b, bytes, (void**)&base)) {
        free_batch(b);
        return JATAM_E_HIP;
    }
    jatam::carve_workspace(base, (size_t)max_n, max_blocks, true, &b->ws);
    if (jatam::batch_init_small_hash(b->ws.small_hash, nullptr) != JATAM_OK ||
        hipDeviceSynchronize() != hipSuccess ||
        hipMemcpy(b->small_hash, b->ws.small_hash, sizeof(b->small_hash),
                  hipMemcpyDeviceToHost) != hipSuccess) {
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
    return jatam::batch_args_for(p, n, out, tally, b->ws, b->small_hash);
}

int jatam_batch_classify(jatam_batch_t* batch, const uint64_t* genotypes, int64_t n, int t,
                         int c, int grid_limit, int runs, uint64_t seed, jatam_result_t* out,
                         uint64_t* tally, void* stream)
{
    jatam::Params p;
    int rc = jatam::make_params(t, c, grid_limit, runs, seed, &p);
    if (rc != JATAM_OK)
        return rc;
    if ((rc = batch_check(batch, n, out)) != JATAM_OK)
        return rc;
    if (n > 0 && genotypes == nullptr)
        return JATAM_E_INVALID_ARG;
    jatam::BatchArgs a = batch_args(batch, p, n, out, tally);
    a.genomes = genotypes;
    return launch_timed(batch, a, grid_limit, t, (hipStream_t)stream);
}

int jatam_batch_classify_range(jatam_batch_t* batch, uint64_t first, int64_t n, int t, int c,
                               int grid_limit, int runs, uint64_t seed, jatam_result_t* out,
                               uint64_t* tally, void* stream)
{
    jatam::Params p;
    int rc = jatam::make_params(t, c, grid_limit, runs, seed, &p);
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
    return launch_timed(batch, a, grid_limit, t, (hipStream_t)stream);
}

int jatam_batch_classify_range_ordered(jatam_batch_t* batch, uint64_t first, int64_t n, int t,
                                       int c, int grid_limit, int runs, uint64_t seed,
                                       const uint32_t* order, jatam_result_t* out,
                                       uint64_t* tally, void* stream)
{
    jatam::Params p;
    int rc = jatam::make_params(t, c, grid_limit, runs, seed, &p);
    if (rc != JATAM_OK)
        return rc;
    if ((rc = batch_check(batch, n, out)) != JATAM_OK)
        return rc;
    if (n > 0) {
        const uint64_t last = first + (uint64_t)(n - 1);
        if (last < first || (p.genome_bits < 64 && (last >> p.genome_bits) != 0) ||
            order == nullptr)
            return JATAM_E_INVALID_ARG;
    }
    jatam::BatchArgs a = batch_args(batch, p, n, out, tally);
    a.first = first;
    a.order = order;
    return launch_timed(batch, a, grid_limit, t, (hipStream_t)stream);
}

int64_t jatam_order_work_words(int64_t n)
{
    return n < 0 ? -1 : (int64_t)jatam::order_work_words((uint64_t)n);
}

int jatam_order_by_cost(const float* scores, int64_t n, uint32_t* order, uint32_t* work,
                        void* stream)
{
    if (n < 0 || n > ((int64_t)1 << 32) - 1 ||
        (n > 0 && (scores == nullptr || order == nullptr || work == nullptr)))
        return JATAM_E_INVALID_ARG;
    return jatam::launch_order_by_cost(scores, (uint32_t)n, order, work, (hipStream_t)stream);
}

int jatam_batch_classify_items(jatam_batch_t* batch, const jatam_item_t* items, int64_t n,
                               int c, int runs, uint64_t seed, jatam_result_t* out,
                               uint64_t* tally, void* stream)
{
    return jatam_batch_classify_items_ordered(batch, items, nullptr, n, c, runs, seed, out, tally,
                                              stream);
}

int jatam_batch_classify_items_ordered(jatam_batch_t* batch, const jatam_item_t* items,
                                       const uint32_t* order, int64_t n, int c, int runs,
                                       uint64_t seed, jatam_result_t* out, uint64_t* tally,
                                       void* stream)
{
    jatam::Params p;
    // t and grid are per item; validate the shared arguments with placeholders
    int rc = jatam::make_params(1, c, 16, runs, seed, &p);
    if (rc != JATAM_OK)
        return rc;
    if ((rc = batch_check(batch, n, out)) != JATAM_OK)
        return rc;
    if (n > 0 && items == nullptr)
        return JATAM_E_INVALID_ARG;
    jatam::BatchArgs a = batch_args(batch, p, n, out, tally);
    a.items = items;
    a.order = order;
    return launch_timed(batch, a, 0, 4, (hipStream_t)stream);
}

int jatam_classify_batch(jatam_batch_t* batch, const jatam_item_t* items, int64_t n, int c,
                         int runs, uint64_t seed, const uint32_t* order,
                         const jatam_tuning_t* tune, jatam_result_t* out, uint64_t* tally,
                         void* stream)
{
    jatam::Params p;
    int rc = jatam::make_params(1, c, 16, runs, seed, &p);
    if (rc != JATAM_OK)
        return rc;
    if ((rc = batch_check(batch, n, out)) != JATAM_OK)
        return rc;
    if ((n > 0 && items == nullptr) ||
        (tune != nullptr && (!tuning_valid(16, &tune[0]) || !tuning_valid(32, &tune[1]))))
        return JATAM_E_INVALID_ARG;
    jatam::BatchArgs a = batch_args(batch, p, n, out, tally);
    a.items = items;
    a.order = order;
    hipEvent_t* marks;
    uint8_t* launched;
    if ((rc = next_marks(batch, &marks, &launched)) != JATAM_OK)
        return rc;
    return launch_pipeline(batch, a, 0, 4, (hipStream_t)stream, marks, launched, tune);
}

int jatam_batch_enumerate(jatam_batch_t* batch, uint64_t first, int64_t slice, int64_t slices,
                          int t, int c, int grid_limit, int runs, uint64_t seed,
                          jatam_result_t* out, uint64_t* tally, jatam_shape_count_t* shapes,
                          int64_t shapes_capacity, void* stream)
{
    jatam::Params p;
    int rc = jatam::make_params(t, c, grid_limit, runs, seed, &p);
    if (rc != JATAM_OK)
        return rc;
    if (batch == nullptr || slice < 1 || slice > batch->max_n || slices < 1 ||
        slices > (int64_t)0xFFFFFFFFu)
        return JATAM_E_INVALID_ARG;
    if ((rc = batch_check(batch, slice, batch)) != JATAM_OK)
        return rc;
    const uint64_t total = (uint64_t)slice * (uint64_t)slices;
    if (total / (uint64_t)slices != (uint64_t)slice)
        return JATAM_E_INVALID_ARG;
    const uint64_t last = first + (total - 1);
    if (last < first || (p.genome_bits < 64 && (last >> p.genome_bits) != 0))
        return JATAM_E_INVALID_ARG;
    int log2cap = 0;
    if (shapes != nullptr) {
        if (shapes_capacity < 64 || shapes_capacity > (1 << 24) ||
            (shapes_capacity & (shapes_capacity - 1)) != 0)
            return JATAM_E_INVALID_ARG;
        while ((int64_t(1) << log2cap) < shapes_capacity)
            ++log2cap;
    }
    hipStream_t s = (hipStream_t)stream;
    // the previous enumeration's graph may still run: wait for it, then drop it
    if (batch->graph_exec != nullptr) {
        if (hipStreamSynchronize(batch->graph_stream) != hipSuccess)
            return JATAM_E_HIP;
        drop_graph(batch);
    }
    jatam::BatchArgs a = batch_args(batch, p, slice, out != nullptr ? out : batch->ws.records,
                                    tally);
    a.first = first;
    a.slice = batch->ws.counters + jatam::kCntSlice;
    a.out_per_slice = out != nullptr;
    // capture one slice: pipeline, shape histogram of its records, counter + 1
    hipStream_t cs = batch->capture_stream;
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return JATAM_E_HIP;
    rc = launch_pipeline(batch, a, grid_limit, t, cs, nullptr, nullptr);
    if (rc == JATAM_OK && shapes != nullptr)
        rc = jatam::launch_shape_hist(a.out, (uint64_t)slice, shapes, log2cap, nullptr,
                                      batch->cus, out != nullptr ? a.slice : nullptr, cs);
    if (rc == JATAM_OK)
        rc = jatam::launch_slice_advance(batch->ws.counters + jatam::kCntSlice, cs);
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(cs, &graph);
    if (rc != JATAM_OK || ec != hipSuccess || graph == nullptr) {
        if (graph != nullptr)
            (void)hipGraphDestroy(graph);
        return rc != JATAM_OK ? rc : JATAM_E_HIP;
    }
    batch->graph = graph;
    if (hipGraphInstantiate(&batch->graph_exec, graph, nullptr, nullptr, 0) != hipSuccess) {
        batch->graph_exec = nullptr;
        drop_graph(batch);
        return JATAM_E_HIP;
    }
    batch->graph_stream = s;
    // replay it once per slice, the counter starting at 0
    if (jatam::launch_slice_reset(batch->ws.counters + jatam::kCntSlice, s) != JATAM_OK)
        return JATAM_E_HIP;
    for (int64_t k = 0; k < slices; ++k)
        if (hipGraphLaunch(batch->graph_exec, s) != hipSuccess)
            return JATAM_E_HIP;
    return JATAM_OK;
}

int jatam_batch_set_refill(jatam_batch_t* batch, int idle_lanes)
{
    if (batch == nullptr || idle_lanes < 1 || idle_lanes > 64)
        return JATAM_E_INVALID_ARG;
    batch->tune[0].refill = idle_lanes;
    batch->tune[1].refill = idle_lanes;
    return JATAM_OK;
}

int jatam_batch_get_tuning(const jatam_batch_t* batch, int grid_limit, jatam_tuning_t* tuning)
{
    if (batch == nullptr || tuning == nullptr || grid_limit < 8 || grid_limit > 32)
        return JATAM_E_INVALID_ARG;
    *tuning = batch->tune[grid_limit <= 16 ? 0 : 1];
    return JATAM_OK;
}

int jatam_batch_set_tuning(jatam_batch_t* batch, int grid_limit, const jatam_tuning_t* tuning)
{
    if (batch == nullptr || tuning == nullptr || grid_limit < 8 || grid_limit > 32 ||
        !tuning_valid(grid_limit, tuning))
        return JATAM_E_INVALID_ARG;
    batch->tune[grid_limit <= 16 ? 0 : 1] = *tuning;
    return JATAM_OK;
}

int jatam_batch_autotune(jatam_batch_t* batch, uint64_t first, int64_t n, int t, int c,
                         int grid_limit, int runs, uint64_t seed, jatam_result_t* scratch,
                         jatam_tuning_t* best, void* stream)
{
    if (batch == nullptr || scratch == nullptr || n < 1 || n > batch->max_n)
        return JATAM_E_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    const int k = grid_limit <= 16 ? 0 : 1;
    const int ti = t <= 2 ? 0 : 1;
    jatam_result_t* ref = scratch;
    jatam_result_t* cand = scratch + n;
    uint32_t* flag = batch->ws.counters + jatam::kCntDiff;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess)
        return JATAM_E_HIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return JATAM_E_HIP;
    }
    batch->tune_log.clear();
    int rc = JATAM_OK;
    // median of three timed calls after one warm-up; records into `dst`
    auto measure = [&](jatam_result_t* dst, double* ms) -> int {
        float v[3];
        for (int r = 0; r < 4; ++r) {
            if (r > 0 && hipEventRecord(e0, s) != hipSuccess)
                return JATAM_E_HIP;
            const int q = jatam_batch_classify_range(batch, first, n, t, c, grid_limit, runs,
                                                     seed, dst, nullptr, stream);
            if (q != JATAM_OK)
                return q;
            if (r > 0) {
                if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                    hipEventElapsedTime(&v[r - 1], e0, e1) != hipSuccess)
                    return JATAM_E_HIP;
            }
        }
        std::sort(v, v + 3);
        *ms = v[1];
        return JATAM_OK;
    };
    // the records of a candidate must equal the reference's, bit for bit
    auto same = [&](bool* ok) -> int {
        uint32_t h = 0;
        if (hipMemsetAsync(flag, 0, sizeof(uint32_t), s) != hipSuccess ||
            jatam::launch_records_differ(ref, cand, (uint64_t)n, flag, s) != JATAM_OK ||
            hipMemcpyAsync(&h, flag, sizeof(uint32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return JATAM_E_HIP;
        *ok = h == 0;
        return JATAM_OK;
    };
    jatam_tuning_t cur = batch->tune[k];
    double cur_ms = 0;
    if ((rc = measure(ref, &cur_ms)) != JATAM_OK)
        goto done;
    batch->tune_log.push_back({cur, cur_ms});
    // one field at a time, keeping the best value of each: the repeat
    // stage's mapping before its grid (whose residency limit it sets)
    static const int order[7] = {0, 1, 6, 2, 3, 4, 5};
    for (int fi = 0; fi < 7 && rc == JATAM_OK; ++fi) {
        const int field = order[fi];
        const int rocc = batch->occ[k][ti][cur.repeat_mapping == 1 ? 2 : 1];
        std::vector<int> choices;
        if (field == 0)
            choices = {8, 16, 24, 32, 48};
        else if (field == 4)
            choices = {0, 4, 8, 12, 16};
        else if (field == 5)
            choices = {1, 2, 4, 8};
        else if (field == 6)
            choices = {0, 1, 2};
        else if (field == 1)
            choices = wave_choices(batch->occ[k][ti][0]);
        else if (field == 2)
            choices = wave_choices(rocc);
        else if (k == 0)
            choices = {0, 1};
        else
            choices = {0, 1, 2};
        for (int v : choices) {
            jatam_tuning_t trial = cur;
            int* slot = field == 0 ? &trial.refill : field == 1 ? &trial.first_waves
                      : field == 2 ? &trial.repeat_waves : field == 3 ? &trial.wide_layout
                      : field == 4 ? &trial.claim_share : field == 5 ? &trial.claim_chunks
                      : &trial.repeat_mapping;
            if (*slot == v || (field == 1 && v >= batch->occ[k][ti][0] && cur.first_waves >= v) ||
                (field == 2 && v >= rocc && cur.repeat_waves >= v))
                continue;
            *slot = v;
            batch->tune[k] = trial;
            double ms = 0;
            bool ok = false;
            if ((rc = measure(cand, &ms)) != JATAM_OK || (rc = same(&ok)) != JATAM_OK)
                break;
            if (!ok) {
                rc = JATAM_E_MISMATCH;
                break;
            }
            batch->tune_log.push_back({trial, ms});
            // a change must win by more than the run-to-run noise
            if (ms < 0.99 * cur_ms) {
                cur = trial;
                cur_ms = ms;
            }
        }
    }
done:
    batch->tune[k] = cur;
    if (best != nullptr)
        *best = cur;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}

// ---------------------------------------------------------------------------
// Autotune cache: one JSON object per line,
//   {"key": "<arch>|cu<n>|G<16|32>|t<t>|c<c>|R<runs>|abi<v>", "refill": .., ...}
// ---------------------------------------------------------------------------
namespace {

const char* const kTuningFields[7] = {"refill",      "first_waves",  "repeat_waves",
                                      "wide_layout", "claim_share",  "claim_chunks",
                                      "repeat_mapping"};

int* tuning_field(jatam_tuning_t* t, int i)
{
    int* const f[7] = {&t->refill,      &t->first_waves,  &t->repeat_waves, &t->wide_layout,
                       &t->claim_share, &t->claim_chunks, &t->repeat_mapping};
    return f[i];
}

std::string tuning_key(const jatam_batch_t* batch, int t, int c, int grid_limit, int runs)
{
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, batch->device) == hipSuccess)
        arch = prop.gcnArchName;
    for (char& ch : arch)
        if (ch == '"' || ch == '|' || ch == '\\' || (unsigned char)ch < 32)
            ch = '_';
    char buf[256];
    snprintf(buf, sizeof(buf), "%s|cu%d|G%d|t%d|c%d|R%d|abi%d", arch.c_str(), batch->cus,
             grid_limit <= 16 ? 16 : 32, t, c, runs, jatam_abi_version());
    return buf;
}

// The tuning stored under `key` in one line of the file, if the line holds it
// whole and valid.
bool parse_tuning_line(const char* line, const std::string& key, int grid_limit,
                       jatam_tuning_t* out)
{
    const std::string want = "\"key\": \"" + key + "\"";
    if (strstr(line, want.c_str()) == nullptr)
        return false;
    jatam_tuning_t t{};
    for (int i = 0; i < 7; ++i) {
        const std::string name = std::string("\"") + kTuningFields[i] + "\":";
        const char* at = strstr(line, name.c_str());
        if (at == nullptr)
            return false;
        char* end = nullptr;
        const long v = strtol(at + name.size(), &end, 10);
        if (end == at + name.size() || v < -1000000 || v > 1000000)
            return false;
        *tuning_field(&t, i) = (int)v;
    }
    if (!tuning_valid(grid_limit, &t))
        return false;
    *out = t;
    return true;
}

std::string tuning_line(const std::string& key, const jatam_tuning_t& t)
{
    std::string line = "{\"key\": \"" + key + "\"";
    jatam_tuning_t c = t;
    for (int i = 0; i < 7; ++i)
        line += std::string(", \"") + kTuningFields[i] + "\": " +
                std::to_string(*tuning_field(&c, i));
    return line + "}";
}

}  // namespace

int jatam_batch_autotune_log(const jatam_batch_t* batch, int i, jatam_tuning_t* tuning, double* ms)
{
    if (batch == nullptr)
        return JATAM_E_INVALID_ARG;
    const int count = (int)batch->tune_log.size();
    if (i < 0)
        return count;
    if (i >= count || tuning == nullptr || ms == nullptr)
        return JATAM_E_INVALID_ARG;
    *tuning = batch->tune_log[(size_t)i].first;
    *ms = batch->tune_log[(size_t)i].second;
    return count;
}

int jatam_batch_autotune_cached(jatam_batch_t* batch, const char* path, uint64_t first,
                                int64_t n, int t, int c, int grid_limit, int runs,
                                uint64_t seed, jatam_result_t* scratch, jatam_tuning_t* best,
                                int* from_cache, void* stream)
{
    if (batch == nullptr || path == nullptr || grid_limit < 8 || grid_limit > 32)
        return JATAM_E_INVALID_ARG;
    const std::string key = tuning_key(batch, t, c, grid_limit, runs);
    std::vector<std::string> lines;
    jatam_tuning_t found{};
    bool have = false;
    if (FILE* f = fopen(path, "r")) {
        char buf[1024];
        while (fgets(buf, sizeof(buf), f) != nullptr) {
            std::string line(buf);
            while (!line.empty() && (line.back() == '\n' || line.back() == '\r'))
                line.pop_back();
            if (line.empty())
                continue;
            if (!have && parse_tuning_line(line.c_str(), key, grid_limit, &found)) {
                have = true;
                continue;   // rewritten below
            }
            if (line.find("\"key\": \"" + key + "\"") == std::string::npos)
                lines.push_back(line);   // other keys are kept; a broken line of this key is not
        }
        fclose(f);
    }
    if (have) {
        const int rc = jatam_batch_set_tuning(batch, grid_limit, &found);
        if (rc != JATAM_OK)
            return rc;
        if (best != nullptr)
            *best = found;
        if (from_cache != nullptr)
            *from_cache = 1;
        return JATAM_OK;
    }
    jatam_tuning_t tuned{};
    const int rc = jatam_batch_autotune(batch, first, n, t, c, grid_limit, runs, seed, scratch,
                                        &tuned, stream);
    if (rc != JATAM_OK)
        return rc;
    lines.push_back(tuning_line(key, tuned));
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = fopen(tmp.c_str(), "w");
    if (f == nullptr)
        return JATAM_E_IO;
    bool ok = true;
    for (const std::string& line : lines)
        ok = ok && fprintf(f, "%s\n", line.c_str()) > 0;
    ok = fclose(f) == 0 && ok;
    if (!ok || rename(tmp.c_str(), path) != 0)
        return JATAM_E_IO;
    if (best != nullptr)
        *best = tuned;
    if (from_cache != nullptr)
        *from_cache = 0;
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
        "first_run_kernel<16>", "size_sort<16>", "prove_kernel<16>", "repeat_kernel<16>",
        "first_run_kernel<32>", "size_sort<32>", "prove_kernel<32>", "repeat_kernel<32>"};
    return stage >= 0 && stage < jatam::kStages ? names[stage] : "";
}

// ---------------------------------------------------------------------------
// Genetic algorithm.
// ---------------------------------------------------------------------------
static int ga_args(const jatam_ga_params_t* p, int t, int c, int32_t generation,
                   jatam::GaArgs* g)
{
    const int bits = log2_exact(c);
    if (p == nullptr || bits < 0 || t < 1 || t > 4 || 4 * t * bits > 64 || p->tournament < 1 ||
        p->tournament > 8 || p->mut_den < 1 || p->mut_num < 0 || p->mut_num > p->mut_den)
        return JATAM_E_INVALID_ARG;
    g->key0 = (uint32_t)p->seed;
    g->key1 = (uint32_t)(p->seed >> 32);
    g->generation = generation;
    g->tournament = p->tournament;
    g->mut_num = p->mut_num;
    g->mut_den = p->mut_den;
    g->t = t;
    g->c = c;
    g->bits = bits;
    return JATAM_OK;
}

int jatam_ga_offspring(const uint64_t* pop, const int32_t* fit, int64_t n, int t, int c,
                       const jatam_ga_params_t* p, int32_t generation, int64_t n_out,
                       uint64_t* out, void* stream)
{
    jatam::GaArgs g;
    const int rc = ga_args(p, t, c, generation, &g);
    if (rc != JATAM_OK)
        return rc;
    if (n < 1 || n > (int64_t)0xFFFFFFFFu || n_out < 0 || n_out > (int64_t)0xFFFFFFFFu ||
        pop == nullptr || fit == nullptr || (n_out > 0 && out == nullptr))
        return JATAM_E_INVALID_ARG;
    return jatam::launch_ga_offspring(pop, fit, (uint32_t)n, g, (uint32_t)n_out, out,
                                      (hipStream_t)stream);
}

int jatam_ga_step(jatam_batch_t* batch, const uint64_t* pop, const int32_t* fit, int64_t n, int t,
                  int c, int grid_limit, int runs, uint64_t seed, const jatam_ga_params_t* p,
                  int32_t generation, const jatam_screen_t* surrogate, uint64_t* next_pop,
                  int32_t* next_fit, void* stream)
{
    if (surrogate != nullptr)
        return jatam_ga_step_screened(surrogate->ga, batch, surrogate->mlp, pop, fit, n, t, c,
                                      grid_limit, runs, seed, p, generation,
                                      surrogate->oversample, next_pop, next_fit, stream);
    jatam::GaArgs g;
    int rc = ga_args(p, t, c, generation, &g);
    if (rc != JATAM_OK)
        return rc;
    if (batch == nullptr || n < 1 || n > batch->max_n || pop == nullptr || fit == nullptr ||
        next_pop == nullptr || next_fit == nullptr || next_pop == pop)
        return JATAM_E_INVALID_ARG;
    const hipStream_t s = (hipStream_t)stream;
    if ((rc = jatam::launch_ga_offspring(pop, fit, (uint32_t)n, g, (uint32_t)n, next_pop, s)) !=
        JATAM_OK)
        return rc;
    if ((rc = jatam_batch_classify(batch, next_pop, n, t, c, grid_limit, runs, seed,
                                   batch->ws.records, nullptr, stream)) != JATAM_OK)
        return rc;
    return jatam::launch_ga_fitness(batch->ws.records, (uint32_t)n, next_fit, s);
}

// ---------------------------------------------------------------------------
// Surrogate MLP.
// ---------------------------------------------------------------------------
}  // extern "C"

struct jatam_mlp {
    int device;
    int64_t max_batch;     // padded to a multiple of 32
    int step;              // Adam steps taken since the parameters were set
    jatam::MlpArgs a;
    void* allocations[24];
    int nalloc;
};

static void mlp_views(float* flat, jatam::MlpTensors* t)
{
    t->flat = flat;
    t->w1 = flat + jatam::kMlpOffW1;
    t->b1 = flat + jatam::kMlpOffB1;
    t->w2 = flat + jatam::kMlpOffW2;
    t->b2 = flat + jatam::kMlpOffB2;
    t->w3 = flat + jatam::kMlpOffW3;
    t->b3 = flat + jatam::kMlpOffB3;
}

static void mlp_free(jatam_mlp_t* m)
{
    for (int i = 0; i < m->nalloc; ++i)
        (void)hipFree(m->allocations[i]);
    delete m;
}

static bool mlp_alloc(jatam_mlp_t* m, size_t bytes, void** out)
{
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess)
        return false;
    m->allocations[m->nalloc++] = p;
    *out = p;
    return true;
}

static uint32_t pad32(int64_t n) { return (uint32_t)((n + 31) / 32 * 32); }

extern "C" {

int jatam_mlp_create(int64_t max_batch, int c, jatam_mlp_t** mlp)
{
    const int bits = log2_exact(c);
    if (mlp == nullptr || max_batch < 1 || max_batch > (1 << 24) || bits < 0 || c > 8)
        return JATAM_E_INVALID_ARG;
    *mlp = nullptr;
    jatam_mlp_t* m = new (std::nothrow) jatam_mlp_t();
    if (m == nullptr)
        return JATAM_E_HIP;
    m->nalloc = 0;
    m->step = 0;
    m->max_batch = pad32(max_batch);
    if (hipGetDevice(&m->device) != hipSuccess) {
        delete m;
        return JATAM_E_HIP;
    }
    const size_t P = jatam::kMlpParams, B = (size_t)m->max_batch, Hd = jatam::kMlpHidden;
    float *p, *g;
    jatam::MlpArgs& a = m->a;
    bool ok = mlp_alloc(m, P * 4, (void**)&p) && mlp_alloc(m, P * 4, (void**)&g) &&
              mlp_alloc(m, P * 4, (void**)&a.m) && mlp_alloc(m, P * 4, (void**)&a.v) &&
              mlp_alloc(m, (size_t)jatam::kMlpIn * Hd * 2, (void**)&a.w1b) &&
              mlp_alloc(m, Hd * Hd * 2, (void**)&a.w2b) &&
              mlp_alloc(m, Hd * jatam::kMlpOut * 2, (void**)&a.w3b) &&
              mlp_alloc(m, Hd * Hd * 2, (void**)&a.w2t) &&
              mlp_alloc(m, 16 * Hd * 2, (void**)&a.w3t) &&
              mlp_alloc(m, B * jatam::kMlpIn * 2, (void**)&a.x) &&
              mlp_alloc(m, B * Hd * 2, (void**)&a.h1) && mlp_alloc(m, B * Hd * 2, (void**)&a.h2) &&
              mlp_alloc(m, B * Hd * 2, (void**)&a.dh2) &&
              mlp_alloc(m, B * Hd * 2, (void**)&a.dh1) &&
              mlp_alloc(m, B * jatam::kMlpOut * 4, (void**)&a.dout) &&
              mlp_alloc(m, B * 4, (void**)&a.loss) &&
              mlp_alloc(m, jatam::mlp_partial_floats(B) * 4, (void**)&a.partial);
    if (!ok) {
        mlp_free(m);
        return JATAM_E_HIP;
    }
    mlp_views(p, &a.p);
    mlp_views(g, &a.g);
    a.c = c;
    a.bits = bits;
    // the padding rows of the transposed head weights stay zero
    if (hipMemset(a.w3t, 0, 16 * Hd * 2) != hipSuccess ||
        jatam::mlp_launch_init(a, 0x5eed, nullptr) != JATAM_OK ||
        hipDeviceSynchronize() != hipSuccess) {
        mlp_free(m);
        return JATAM_E_HIP;
    }
    *mlp = m;
    return JATAM_OK;
}

int jatam_mlp_destroy(jatam_mlp_t* mlp)
{
    if (mlp == nullptr)
        return JATAM_OK;
    const hipError_t e = hipDeviceSynchronize();
    mlp_free(mlp);
    return e == hipSuccess ? JATAM_OK : JATAM_E_HIP;
}

int jatam_mlp_init(jatam_mlp_t* mlp, uint64_t seed, void* stream)
{
    if (mlp == nullptr)
        return JATAM_E_INVALID_ARG;
    mlp->step = 0;
    return jatam::mlp_launch_init(mlp->a, seed, (hipStream_t)stream);
}

int jatam_mlp_set_params(jatam_mlp_t* mlp, const float* params, void* stream)
{
    if (mlp == nullptr || params == nullptr)
        return JATAM_E_INVALID_ARG;
    const hipStream_t s = (hipStream_t)stream;
    const size_t bytes = (size_t)jatam::kMlpParams * 4;
    if (hipMemcpyAsync(mlp->a.p.flat, params, bytes, hipMemcpyDeviceToDevice, s) != hipSuccess ||
        hipMemsetAsync(mlp->a.m, 0, bytes, s) != hipSuccess ||
        hipMemsetAsync(mlp->a.v, 0, bytes, s) != hipSuccess)
        return JATAM_E_HIP;
    mlp->step = 0;
    return jatam::mlp_launch_refresh(mlp->a, s);
}

int jatam_mlp_get_params(jatam_mlp_t* mlp, float* params, float* grads, void* stream)
{
    if (mlp == nullptr)
        return JATAM_E_INVALID_ARG;
    const hipStream_t s = (hipStream_t)stream;
    const size_t bytes = (size_t)jatam::kMlpParams * 4;
    if (params != nullptr &&
        hipMemcpyAsync(params, mlp->a.p.flat, bytes, hipMemcpyDeviceToDevice, s) != hipSuccess)
        return JATAM_E_HIP;
    if (grads != nullptr &&
        hipMemcpyAsync(grads, mlp->a.g.flat, bytes, hipMemcpyDeviceToDevice, s) != hipSuccess)
        return JATAM_E_HIP;
    return JATAM_OK;
}

int jatam_mlp_forward(jatam_mlp_t* mlp, const uint64_t* genomes, const uint8_t* t, int t_all,
                      int64_t n, float* out4, void* stream)
{
    if (mlp == nullptr || n < 0 || (n > 0 && (genomes == nullptr || out4 == nullptr)) ||
        (t == nullptr && (t_all < 1 || t_all > 3)))
        return JATAM_E_INVALID_ARG;
    const hipStream_t s = (hipStream_t)stream;
    for (int64_t at = 0; at < n; at += mlp->max_batch) {
        const int64_t k = n - at < mlp->max_batch ? n - at : mlp->max_batch;
        const int rc = jatam::mlp_launch_forward(mlp->a, genomes + at, t ? t + at : nullptr, t_all,
                                                 (uint32_t)k, pad32(k), nullptr,
                                                 out4 + at * jatam::kMlpOut, s);
        if (rc != JATAM_OK)
            return rc;
    }
    return JATAM_OK;
}

int jatam_mlp_train_step(jatam_mlp_t* mlp, const uint64_t* genomes, const uint8_t* t, int t_all,
                         const jatam_result_t* labels, int64_t n, float lr, float* loss_out,
                         void* stream)
{
    if (mlp == nullptr || n < 1 || n > mlp->max_batch || genomes == nullptr ||
        labels == nullptr || !(lr >= 0.f) ||
        (t == nullptr && (t_all < 1 || t_all > 3)))
        return JATAM_E_INVALID_ARG;
    const hipStream_t s = (hipStream_t)stream;
    int rc = jatam::mlp_launch_forward(mlp->a, genomes, t, t_all, (uint32_t)n, pad32(n), labels,
                                       nullptr, s);
    if (rc == JATAM_OK)
        rc = jatam::mlp_launch_backward(mlp->a, (uint32_t)n, pad32(n), loss_out, s);
    if (rc == JATAM_OK && lr > 0.f)
        rc = jatam::mlp_launch_adam(mlp->a, lr, ++mlp->step, s);
    return rc;
}

int jatam_mlp_predict(jatam_mlp_t* mlp, int kind, const uint64_t* genomes, const uint8_t* t,
                      int t_all, int64_t n, float* out, void* stream)
{
    if (mlp == nullptr || n < 0 || (n > 0 && (genomes == nullptr || out == nullptr)) ||
        (t == nullptr && (t_all < 1 || t_all > 3)) ||
        (kind != JATAM_PREDICT_SCREEN && kind != JATAM_PREDICT_COST &&
         kind != JATAM_PREDICT_P_UNBOUND))
        return JATAM_E_INVALID_ARG;
    const hipStream_t s = (hipStream_t)stream;
    // one fused pass, in pieces of at most 2^31 samples (no activations kept)
    for (int64_t at = 0; at < n; at += (int64_t)1 << 31) {
        const int64_t k = n - at < ((int64_t)1 << 31) ? n - at : ((int64_t)1 << 31);
        const int rc = jatam::mlp_launch_score(mlp->a, genomes + at, t ? t + at : nullptr, t_all,
                                               (uint32_t)k, out + at, kind, s);
        if (rc != JATAM_OK)
            return rc;
    }
    return JATAM_OK;
}

int jatam_mlp_score(jatam_mlp_t* mlp, const uint64_t* genomes, const uint8_t* t, int t_all,
                    int64_t n, float* scores, void* stream)
{
    return jatam_mlp_predict(mlp, JATAM_PREDICT_SCREEN, genomes, t, t_all, n, scores, stream);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Screened GA workspace and top-k selection.
// ---------------------------------------------------------------------------
struct jatam_ga {
    int device;
    int64_t max_cand;
    uint64_t* cand;          // offspring candidates
    float* scores;           // their surrogate scores
    uint32_t* idx;           // kept candidates
    jatam::SelectWork sel;
    void* allocations[8];
    int nalloc;
};

static void ga_free(jatam_ga_t* g)
{
    for (int i = 0; i < g->nalloc; ++i)
        (void)hipFree(g->allocations[i]);
    delete g;
}

static bool ga_alloc(jatam_ga_t* g, size_t bytes, void** out)
{
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess)
        return false;
    g->allocations[g->nalloc++] = p;
    *out = p;
    return true;
}

extern "C" {

int jatam_ga_create(int64_t max_candidates, jatam_ga_t** ga)
{
    if (ga == nullptr || max_candidates < 1 || max_candidates > (int64_t)0xFFFFFFFFu)
        return JATAM_E_INVALID_ARG;
    *ga = nullptr;
    jatam_ga_t* g = new (std::nothrow) jatam_ga_t();
    if (g == nullptr)
        return JATAM_E_HIP;
    g->nalloc = 0;
    g->max_cand = max_candidates;
    if (hipGetDevice(&g->device) != hipSuccess) {
        delete g;
        return JATAM_E_HIP;
    }
    const size_t n = (size_t)max_candidates;
    const bool ok = ga_alloc(g, n * 8, (void**)&g->cand) && ga_alloc(g, n * 4, (void**)&g->scores) &&
                    ga_alloc(g, n * 4, (void**)&g->idx) &&
                    ga_alloc(g, jatam::kSelectState * 4, (void**)&g->sel.state) &&
                    ga_alloc(g, n * 4, (void**)&g->sel.flag) &&
                    ga_alloc(g, n * 4, (void**)&g->sel.rank_eq) &&
                    ga_alloc(g, n * 4, (void**)&g->sel.pos) &&
                    ga_alloc(g, (n / 1024 + 2) * 4, (void**)&g->sel.sums);
    if (!ok) {
        ga_free(g);
        return JATAM_E_HIP;
    }
    *ga = g;
    return JATAM_OK;
}

int jatam_ga_destroy(jatam_ga_t* ga)
{
    if (ga == nullptr)
        return JATAM_OK;
    const hipError_t e = hipDeviceSynchronize();
    ga_free(ga);
    return e == hipSuccess ? JATAM_OK : JATAM_E_HIP;
}

int jatam_select_top(jatam_ga_t* ga, const float* scores, int64_t n, int64_t k, uint32_t* out_idx,
                     void* stream)
{
    if (ga == nullptr || scores == nullptr || n < 0 || n > ga->max_cand || k < 0 || k > n ||
        (k > 0 && out_idx == nullptr))
        return JATAM_E_INVALID_ARG;
    return jatam::launch_select_top(scores, (uint32_t)n, (uint32_t)k, out_idx, ga->sel,
                                    (hipStream_t)stream);
}

int jatam_ga_step_screened(jatam_ga_t* ga, jatam_batch_t* batch, jatam_mlp_t* mlp,
                           const uint64_t* pop, const int32_t* fit, int64_t n, int t, int c,
                           int grid_limit, int runs, uint64_t seed, const jatam_ga_params_t* p,
                           int32_t generation, int oversample, uint64_t* next_pop,
                           int32_t* next_fit, void* stream)
{
    jatam::GaArgs g;
    int rc = ga_args(p, t, c, generation, &g);
    if (rc != JATAM_OK)
        return rc;
    if (ga == nullptr || batch == nullptr || mlp == nullptr || n < 1 || oversample < 1 ||
        oversample > 1024 ||
        n * oversample > ga->max_cand || n > batch->max_n || pop == nullptr || fit == nullptr ||
        next_pop == nullptr || next_fit == nullptr || next_pop == pop || t > 3 ||
        c != (1 << mlp->a.bits))
        return JATAM_E_INVALID_ARG;
    const hipStream_t s = (hipStream_t)stream;
    const uint32_t m = (uint32_t)(n * oversample);
    if ((rc = jatam::launch_ga_offspring(pop, fit, (uint32_t)n, g, m, ga->cand, s)) != JATAM_OK)
        return rc;
    if ((rc = jatam_mlp_score(mlp, ga->cand, nullptr, t, m, ga->scores, stream)) != JATAM_OK)
        return rc;
    if ((rc = jatam::launch_select_top(ga->scores, m, (uint32_t)n, ga->idx, ga->sel, s)) !=
        JATAM_OK)
        return rc;
    if ((rc = jatam::launch_gather(ga->cand, ga->idx, (uint32_t)n, next_pop, s)) != JATAM_OK)
        return rc;
    if ((rc = jatam_batch_classify(batch, next_pop, n, t, c, grid_limit, runs, seed,
                                   batch->ws.records, nullptr, stream)) != JATAM_OK)
        return rc;
    return jatam::launch_ga_fitness(batch->ws.records, (uint32_t)n, next_fit, s);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Shape histogram.
// ---------------------------------------------------------------------------
extern "C" int jatam_shape_histogram(const jatam_result_t* recs, int64_t n,
                                     jatam_shape_count_t* table, int64_t capacity,
                                     uint64_t* overflow, void* stream)
{
    if (n < 0 || capacity < 64 || capacity > (1 << 24) || (capacity & (capacity - 1)) != 0 ||
        table == nullptr || (n > 0 && recs == nullptr))
        return JATAM_E_INVALID_ARG;
    int log2cap = 0;
    while ((int64_t(1) << log2cap) < capacity)
        ++log2cap;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return JATAM_E_HIP;
    return jatam::launch_shape_hist(recs, (uint64_t)n, table, log2cap, overflow, cus, nullptr,
                                    (hipStream_t)stream);
}

// ---------------------------------------------------------------------------
// Workspace layout and launch parameters, shared by the workspace calls and
// the call without a workspace.
// ---------------------------------------------------------------------------
namespace jatam {

// Class 0 (G <= 16) makes its repeat runs in two passes (on S_2,8 most
// candidates left after the proofs are non-deterministic and decided by run
// 1, 2 or 3); class 1 in one (large deterministic shapes need every run).
jatam_tuning_t default_tuning(int klass)
{
    return jatam_tuning_t{24, 64, 64, 0, 12, 4, klass == 0 ? 2 : 0};
}

int max_first_blocks(const int occ[2][2][3], int cus)
{
    int m = 1;
    for (int k = 0; k < 2; ++k)
        for (int i = 0; i < 2; ++i)
            m = occ[k][i][0] * cus > m ? occ[k][i][0] * cus : m;
    return m;
}

bool scan_fits(int max_blocks)
{
    // the size scan covers kSizeBuckets * max_blocks histogram entries in at
    // most kMaxScanBlocks blocks
    return (size_t)kSizeBuckets * max_blocks <= (size_t)kScanBlock * kMaxScanBlocks;
}

size_t carve_workspace(uint8_t* base, size_t max_n, int max_blocks, bool records,
                       DeviceWorkspace* ws)
{
    size_t at = 0;
    auto take = [&](size_t bytes) -> void* {
        void* p = base != nullptr ? base + at : nullptr;
        at += (bytes + 255) / 256 * 256;
        return p;
    };
    const size_t n = max_n, mb = (size_t)max_blocks;
    // per wave: its share of the chunks, and room for one more claim
    const size_t staging = staging_entries(n, mb);
    DeviceWorkspace w;
    w.counters = (uint32_t*)take(kCntWords * sizeof(uint32_t));
    w.run_claim = (uint32_t*)take(2 * kClaimCounters * kClaimStride * sizeof(uint32_t));
    w.queue_claim = (uint32_t*)take(2 * kClaimCounters * kClaimStride * sizeof(uint32_t));
    w.small_hash = (uint32_t*)take(2 * sizeof(uint32_t));
    w.records = records ? (jatam_result_t*)take(n * sizeof(jatam_result_t)) : nullptr;
    for (int k = 0; k < 2; ++k) {
        w.seg_count[k] = (uint32_t*)take(mb * sizeof(uint32_t));
        w.seg_hist[k] = (uint32_t*)take((size_t)kSizeBuckets * mb * sizeof(uint32_t));
        w.scan_sums[k] = (uint32_t*)take((size_t)kMaxScanBlocks * sizeof(uint32_t));
        w.chunk_cnt[k] = (uint32_t*)take((n / 64 + 1) * sizeof(uint32_t));
        w.chunk_sums[k] = (uint32_t*)take((n / 64 / kScanBlock + 1) * sizeof(uint32_t));
        w.cand_idx[k] = (uint32_t*)take(staging * sizeof(uint32_t));
        w.cand_size[k] = (uint16_t*)take(staging * sizeof(uint16_t));
        w.sorted[k] = (uint32_t*)take(n * sizeof(uint32_t));
    }
    w.overflow = (uint32_t*)take(n * sizeof(uint32_t));
    w.cand_shape = (uint4*)take(staging * sizeof(uint4));
    w.sorted_shape = (uint4*)take(n * sizeof(uint4));
    w.occ_hi = (uint4*)take(n * sizeof(uint4));
    if (ws != nullptr)
        *ws = w;
    return at;
}

// Calls from this many items up take the 16 x 16 window for 16 < G <= 32 by
// default.  On smaller calls the window's extra stages and the reruns of the
// items that leave it (populations of large shapes) cost more than it saves.
constexpr int64_t kWindowMinItems = 1 << 20;

int launch_tuned(const jatam_tuning_t tn[2], const int occ[2][2][3], int cus, BatchArgs a,
                 int grid_limit, int max_t, hipStream_t stream, hipEvent_t* marks,
                 uint8_t* launched)
{
    const int tm = max_t <= 2 ? 2 : 4, ti = tm == 2 ? 0 : 1;
    // G <= narrow_max runs in the 16 x 16 layout; with the window on (the
    // default) that is every G <= 32, and the 32 x 32 class reruns only the
    // items of G > 16 that left the window
    const int w1 = tn[1].wide_layout;
    const bool window =
        !tn[0].wide_layout && (w1 == 2 || (w1 == 0 && a.n >= kWindowMinItems));
    a.narrow_max = tn[0].wide_layout ? 0 : window ? 32 : 16;
    const bool classes[2] = {grid_limit == 0 || grid_limit <= a.narrow_max,
                             grid_limit == 0 || grid_limit > (window ? 16 : a.narrow_max)};
    StageLaunch launch[2];
    for (int k = 0; k < 2; ++k) {
        const jatam_tuning_t& t = tn[k];
        const int rocc = occ[k][ti][t.repeat_mapping == 1 ? 2 : 1];
        const int fw = t.first_waves < occ[k][ti][0] ? t.first_waves : occ[k][ti][0];
        const int rw = t.repeat_waves < rocc ? t.repeat_waves : rocc;
        launch[k] = StageLaunch{t.refill,       fw * cus,       rw * cus,
                                t.claim_share, t.claim_chunks, t.repeat_mapping};
    }
    return launch_batched(a, classes, launch, tm, stream, marks, launched);
}

BatchArgs batch_args_for(const Params& p, int64_t n, jatam_result_t* out, uint64_t* tally,
                         const DeviceWorkspace& ws, const uint32_t small_hash[2])
{
    BatchArgs a;
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
    a.order = nullptr;
    a.slice = nullptr;
    a.out_per_slice = 0;
    a.narrow_max = 16;
    a.n_dev = nullptr;
    a.refill = 24;
    a.dyn16 = 0;
    a.claim_chunks = 1;
    a.seg_cap = 0;
    a.small0 = small_hash[0];
    a.small1 = small_hash[1];
    a.out = out;
    a.tally = reinterpret_cast<unsigned long long*>(tally);
    a.ws = ws;
    return a;
}

int make_params(int t, int c, int grid, int runs, uint64_t seed, Params* p)
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

}  // namespace jatam
