// Host side of the FOFSE C ABI: argument validation, plan state, launches.
// Every entry point is declared in include/fofse.h.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/fofse.h"
#include "fofse_kernel.h"

struct fofse_plan_s {
    int device = 0;
    int M = 0, N = 0, T = 0, K = 0, nB = 0;
    uint8_t* d_target = nullptr;
    int32_t* d_bpix = nullptr;
    double2* d_twiddle = nullptr;
};

namespace {

bool fft_size_built(int T) { return T == 32 || T == 64; }

// Keeps the caller's current device across a library call.
struct DeviceGuard {
    int prev = -1;
    bool ok = false;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) return;
        ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

void free_plan(fofse_plan p) {
    if (!p) return;
    if (p->d_target) (void)hipFree(p->d_target);
    if (p->d_bpix) (void)hipFree(p->d_bpix);
    if (p->d_twiddle) (void)hipFree(p->d_twiddle);
    delete p;
}

}  // namespace

extern "C" {

const char* fofse_status_str(fofse_status s) {
    switch (s) {
        case FOFSE_OK: return "ok";
        case FOFSE_ERR_ARG: return "invalid argument";
        case FOFSE_ERR_UNSUPPORTED: return "unsupported configuration";
        case FOFSE_ERR_NOMEM: return "device allocation failed";
        case FOFSE_ERR_DEVICE: return "HIP runtime or launch failure";
    }
    return "unknown status";
}

fofse_status fofse_create(const fofse_geometry* g, int32_t device, fofse_plan* out) {
    if (!g || !out || !g->target_mask) return FOFSE_ERR_ARG;
    const int M = g->area_h, N = g->area_w, T = g->fft_size, K = g->iterations;
    if (M < 1 || N < 1 || T < 2 || (T & (T - 1)) != 0 || M > T || N > T) return FOFSE_ERR_ARG;
    if (K < 0 || K > 4096) return FOFSE_ERR_ARG;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess) return FOFSE_ERR_DEVICE;
    if (device < 0 || device >= ndev) return FOFSE_ERR_ARG;
    if (!fft_size_built(T)) return FOFSE_ERR_UNSUPPORTED;

    std::vector<int32_t> bpix;
    for (int i = 0; i < M * N; ++i)
        if (g->target_mask[i]) bpix.push_back(i);
    if (bpix.empty()) return FOFSE_ERR_ARG;
    if ((int)bpix.size() > fofse::max_target_samples(T)) return FOFSE_ERR_UNSUPPORTED;

    std::vector<uint8_t> target(M * N);
    for (int i = 0; i < M * N; ++i) target[i] = g->target_mask[i] ? 1 : 0;
    std::vector<double2> tw(T);
    for (int q = 0; q < T; ++q) {
        const double ang = 2.0 * M_PI * (double)q / (double)T;
        tw[q] = make_double2(std::cos(ang), -std::sin(ang));
    }

    DeviceGuard guard(device);
    if (!guard.ok) return FOFSE_ERR_DEVICE;
    fofse_plan p = new (std::nothrow) fofse_plan_s;
    if (!p) return FOFSE_ERR_NOMEM;
    p->device = device;
    p->M = M; p->N = N; p->T = T; p->K = K;
    p->nB = (int)bpix.size();
    if (hipMalloc(&p->d_target, M * N) != hipSuccess ||
        hipMalloc(&p->d_bpix, bpix.size() * sizeof(int32_t)) != hipSuccess ||
        hipMalloc(&p->d_twiddle, T * sizeof(double2)) != hipSuccess) {
        free_plan(p);
        return FOFSE_ERR_NOMEM;
    }
    if (hipMemcpy(p->d_target, target.data(), M * N, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(p->d_bpix, bpix.data(), bpix.size() * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(p->d_twiddle, tw.data(), T * sizeof(double2), hipMemcpyHostToDevice) != hipSuccess) {
        free_plan(p);
        return FOFSE_ERR_DEVICE;
    }
    *out = p;
    return FOFSE_OK;
}

int32_t fofse_target_count(fofse_plan p) { return p ? p->nB : 0; }

fofse_status fofse_extrapolate_batch(fofse_plan p, int32_t n_blocks, const float* d_areas,
                                     const uint8_t* d_known, const double* d_rho_gamma,
                                     float* d_out, int32_t* d_sel, double* d_coef,
                                     int32_t* d_status, void* stream) {
    if (!p || n_blocks < 0) return FOFSE_ERR_ARG;
    if (n_blocks == 0) return FOFSE_OK;
    if (!d_areas || !d_rho_gamma || !d_out) return FOFSE_ERR_ARG;
    DeviceGuard guard(p->device);
    if (!guard.ok) return FOFSE_ERR_DEVICE;
    fofse::KParams k{};
    k.n_blocks = n_blocks;
    k.T = p->T; k.M = p->M; k.N = p->N; k.K = p->K; k.nB = p->nB;
    k.areas = d_areas;
    k.known = d_known;
    k.target = p->d_target;
    k.bpix = p->d_bpix;
    k.rho_gamma = d_rho_gamma;
    k.twiddle = p->d_twiddle;
    k.out = d_out;
    k.sel = d_sel;
    k.coef = d_coef;
    k.status = d_status;
    hipError_t e = fofse::launch_forward(k, (hipStream_t)stream);
    return e == hipSuccess ? FOFSE_OK : FOFSE_ERR_DEVICE;
}

void fofse_destroy(fofse_plan p) {
    if (!p) return;
    DeviceGuard guard(p->device);
    free_plan(p);
}

}  // extern "C"
