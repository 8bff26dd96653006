// jatam_static.hip - the pipelined classification for callers that cannot
// allocate device memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid hipMalloc): the pipeline's queues live in a static
// device array of the library instead of a jatam_batch_t workspace.
//
// `scratch` below is a host-side stand-in in host code: its device address
// is taken once per device with hipGetSymbolAddress (with that device
// current) and only that address is ever handed to kernels.  Every call on a
// device shares the device's copy of the array, so calls that overlap on one
// GPU race; the pipeline writes every queue entry and counter it reads
// (counters by kernels, never by a memset), so nothing carries over from the
// previous call.
#include <mutex>

#include "jatam_internal.hpp"

namespace {

constexpr int64_t kStaticMaxN = int64_t(1) << 18;   // genotypes per call
constexpr size_t kStaticBytes = size_t(32) << 20;   // 32 MiB per device
constexpr int kMaxDevices = 64;

struct StaticDevice {
    bool ready;
    int cus;
    int occ[2][2][3];
    uint32_t small_hash[2];
    jatam::DeviceWorkspace ws;
};

StaticDevice g_devices[kMaxDevices];
std::mutex g_setup;

}  // namespace

__device__ __align__(256) uint8_t scratch[kStaticBytes];

namespace {

// Set-up on the current device, once: the array's device address, the
// residency limits, the workspace layout and the two small-shape hashes (a
// kernel and a copy on the null stream, synchronised; so the first call on a
// device must not be under graph capture).
int static_setup(int dev, StaticDevice** out)
{
    std::lock_guard<std::mutex> lock(g_setup);
    StaticDevice& d = g_devices[dev];
    if (!d.ready) {
        uint8_t* ptr = nullptr;
        if (hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch)) != hipSuccess ||
            ptr == nullptr)
            return JATAM_E_HIP;
        if (hipDeviceGetAttribute(&d.cus, hipDeviceAttributeMultiprocessorCount, dev) !=
            hipSuccess)
            return JATAM_E_HIP;
        jatam::batch_occupancy(d.occ);
        const int max_blocks = jatam::max_first_blocks(d.occ, d.cus);
        if (!jatam::scan_fits(max_blocks) ||
            jatam::carve_workspace(nullptr, (size_t)kStaticMaxN, max_blocks, false, nullptr) >
                kStaticBytes)
            return JATAM_E_UNSUPPORTED;
        jatam::carve_workspace(ptr, (size_t)kStaticMaxN, max_blocks, false, &d.ws);
        if (jatam::batch_init_small_hash(d.ws.small_hash, nullptr) != JATAM_OK ||
            hipDeviceSynchronize() != hipSuccess ||
            hipMemcpy(d.small_hash, d.ws.small_hash, sizeof(d.small_hash),
                      hipMemcpyDeviceToHost) != hipSuccess)
            return JATAM_E_HIP;
        d.ready = true;
    }
    *out = &d;
    return JATAM_OK;
}

}  // namespace

extern "C" int jatam_classify_static(const uint64_t* genotypes, int64_t n, int t, int c,
                                     int grid_limit, int runs, uint64_t seed, jatam_result_t* out,
                                     uint64_t* tally, void* stream)
{
    jatam::Params p;
    const int rc = jatam::make_params(t, c, grid_limit, runs, seed, &p);
    if (rc != JATAM_OK)
        return rc;
    if (n < 0 || n > kStaticMaxN || (n > 0 && (genotypes == nullptr || out == nullptr)))
        return JATAM_E_INVALID_ARG;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0)
        return JATAM_E_HIP;
    if (dev >= kMaxDevices)
        return JATAM_E_UNSUPPORTED;
    StaticDevice* d = nullptr;
    const int sc = static_setup(dev, &d);
    if (sc != JATAM_OK)
        return sc;
    jatam::BatchArgs a = jatam::batch_args_for(p, n, out, tally, d->ws, d->small_hash);
    a.genomes = genotypes;
    const jatam_tuning_t tune[2] = {jatam::default_tuning(0), jatam::default_tuning(1)};
    return jatam::launch_tuned(tune, d->occ, d->cus, a, grid_limit, t, (hipStream_t)stream,
                               nullptr, nullptr);
}
