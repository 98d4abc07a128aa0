// fofse_extrapolate_batch_noalloc: the forward of fofse_extrapolate_batch for
// callers that cannot allocate device memory (code under HIP graph capture,
// tight serving loops, harnesses that forbid hipMalloc).
//
// The only memory the forward needs beyond the caller's inputs and outputs
// and the plan's tables (allocated by fofse_create) is the grouping workspace
// of the grouped organisation and of the DCT basis with per-block masks (a
// hash table of the support masks, per-block class and position, per-item
// block lists, counters).  Here it lives in a file-scope device array of fixed
// size; every device the library runs on holds its own copy until the process
// ends.  The hash table and counters are cleared by a kernel at the start of
// every call, so the contents a previous call left behind do not matter; two
// calls that overlap on one device share the array and race.

#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/fofse.h"
#include "fofse_kernel.h"

namespace {

// 5 MiB: the workspace of FOFSE_NOALLOC_MAX_BLOCKS blocks (262,144 hash slots
// of 20 B would exceed it; 131,072 slots x 20 B + 65,536 blocks x 32 B + 64 B
// = 4,718,656 B fit).
constexpr size_t kScratchBytes = (size_t)5 << 20;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

// Device address of each device's copy of `scratch`, looked up once per
// device with that device current.  In host code the array's name is only a
// host-side stand-in; kernels receive these addresses.
constexpr int kMaxDevices = 64;
void* g_scratch[kMaxDevices] = {};
std::mutex g_scratch_mutex;

hipError_t scratch_address(int device, void** out) {
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch[device]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch[device] = ptr;
    }
    *out = g_scratch[device];
    return hipSuccess;
}

}  // namespace

extern "C" fofse_status fofse_extrapolate_batch_noalloc(fofse_plan plan, int32_t n_blocks, const float* d_areas,
                                                        const uint8_t* d_known, const double* d_rho_gamma,
                                                        float* d_out, int32_t* d_sel, double* d_coef,
                                                        int32_t* d_status, void* stream) {
    static_assert(kScratchBytes >= (size_t)131072 * 20 + (size_t)FOFSE_NOALLOC_MAX_BLOCKS * 32 + 64,
                  "scratch must hold the workspace of the largest batch");
    if (!plan || n_blocks < 0) return FOFSE_ERR_ARG;
    if (n_blocks == 0) return FOFSE_OK;
    if (!d_areas || !d_rho_gamma || !d_out || !d_sel || !d_coef) return FOFSE_ERR_ARG;
    if (n_blocks > FOFSE_NOALLOC_MAX_BLOCKS) return FOFSE_ERR_LIMIT;
    const int device = fofse::plan_device(plan);
    if (device < 0 || device >= kMaxDevices) return FOFSE_ERR_UNSUPPORTED;
    int prev = -1;
    if (hipGetDevice(&prev) != hipSuccess || hipSetDevice(device) != hipSuccess) return FOFSE_ERR_DEVICE;
    void* base = nullptr;
    const hipError_t e = scratch_address(device, &base);
    (void)hipSetDevice(prev);
    if (e != hipSuccess) return FOFSE_ERR_DEVICE;
    const fofse::Workspace ws{base, kScratchBytes};
    return fofse::extrapolate_impl(plan, n_blocks, d_areas, d_known, d_rho_gamma, d_out, d_sel, d_coef, d_status,
                                   stream, &ws);
}
