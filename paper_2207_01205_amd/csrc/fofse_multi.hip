// Blocks of several geometries in one call (the problem statement of Section
// 2 for areas of different sizes, missing areas and FFT sizes, Section 3):
// fofse_create_multi, fofse_extrapolate_multi, fofse_destroy_multi.
//
// The blocks are sorted by geometry on the device, each geometry's areas are
// gathered from the caller's packed buffer (per-block element offsets) into
// plan-owned staging, run through that geometry's plan (every organisation
// and setting of fofse_extrapolate_batch), and g on the missing area is
// scattered back into the caller's output buffer at the same offsets.  The
// host reads the per-geometry counts (a few bytes) before it launches the
// per-geometry kernels.

#include <hip/hip_runtime.h>

#include <cstring>
#include <new>
#include <vector>

#include "../../include/fofse.h"
#include "fofse_kernel.h"

namespace {

struct GeomStage {
    int M = 0, N = 0, nB = 0;
    int32_t* d_bpix = nullptr;        // [nB] flat indices of B in the area, row-major
    size_t cap = 0;                   // staging capacity in blocks
    float* d_areas = nullptr;         // [cap][M N]
    uint8_t* d_known = nullptr;       // [cap][M N]
    float* d_out = nullptr;           // [cap][nB]
    int32_t* d_status = nullptr;      // [cap]
};

}  // namespace

struct fofse_multi_plan_s {
    int device = 0;
    std::vector<fofse_plan> plans;
    std::vector<GeomStage> st;
    int* d_counts = nullptr;          // [n_geoms] counts, [n_geoms] cursors, [1] bad id flag
    int* h_counts = nullptr;          // pinned copy of the counts and the flag
    size_t list_cap = 0;
    int* d_list = nullptr;            // blocks sorted by geometry
    std::vector<void*> retired;       // replaced staging, kept until destroy
};

namespace {

struct DevGuard {
    int prev = -1;
    bool ok = false;
    explicit DevGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) return;
        ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DevGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

__global__ void k_multi_clear(int* counts, int n) {
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i < n) counts[i] = 0;
}

__global__ void k_multi_count(const int32_t* geom, int n, int n_geoms, int* counts) {
    const int b = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (b >= n) return;
    const int g = geom[b];
    if (g < 0 || g >= n_geoms) atomicOr(&counts[2 * n_geoms], 1);
    else atomicAdd(&counts[g], 1);
}

struct Offsets {
    int v[FOFSE_MULTI_MAX_GEOMS];
};

__global__ void k_multi_fill(const int32_t* geom, int n, int n_geoms, int* counts, Offsets off, int* list) {
    const int b = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (b >= n) return;
    const int g = geom[b];
    const int pos = atomicAdd(&counts[n_geoms + g], 1);
    list[off.v[g] + pos] = b;
}

// staging[j][s] = areas[area_off[list[j]] + s] (and the known mask)
__global__ void k_multi_gather(const int* list, int count, int MN, const int64_t* area_off, const float* areas,
                               const uint8_t* known, float* s_areas, uint8_t* s_known) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (size_t)count * MN) return;
    const int j = (int)(i / MN), s = (int)(i - (size_t)j * MN);
    const size_t src = (size_t)area_off[list[j]] + s;
    s_areas[i] = areas[src];
    if (known) s_known[i] = known[src];
}

// out[area_off[list[j]] + bpix[q]] = staging_out[j][q]; status[list[j]] = staging_status[j]
__global__ void k_multi_scatter(const int* list, int count, int nB, const int32_t* bpix, const int64_t* area_off,
                                const float* s_out, const int32_t* s_status, float* out, int32_t* status) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (size_t)count * nB) return;
    const int j = (int)(i / nB), q = (int)(i - (size_t)j * nB);
    const int b = list[j];
    out[(size_t)area_off[b] + bpix[q]] = s_out[i];
    if (q == 0 && status) status[b] = s_status[j];
}

bool capturing(hipStream_t st) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    return hipStreamIsCapturing(st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone;
}

template <class X>
fofse_status grow(fofse_multi_plan mp, X** buf, size_t elems) {
    X* q = nullptr;
    if (hipMalloc(&q, elems * sizeof(X)) != hipSuccess) return FOFSE_ERR_NOMEM;
    if (*buf) mp->retired.push_back(*buf);
    *buf = q;
    return FOFSE_OK;
}

void free_multi(fofse_multi_plan mp) {
    for (fofse_plan p : mp->plans) fofse_destroy(p);
    for (GeomStage& s : mp->st) {
        if (s.d_bpix) (void)hipFree(s.d_bpix);
        if (s.d_areas) (void)hipFree(s.d_areas);
        if (s.d_known) (void)hipFree(s.d_known);
        if (s.d_out) (void)hipFree(s.d_out);
        if (s.d_status) (void)hipFree(s.d_status);
    }
    if (mp->d_counts) (void)hipFree(mp->d_counts);
    if (mp->h_counts) (void)hipHostFree(mp->h_counts);
    if (mp->d_list) (void)hipFree(mp->d_list);
    for (void* q : mp->retired) (void)hipFree(q);
    delete mp;
}

}  // namespace

extern "C" {

fofse_status fofse_create_multi(const fofse_geometry* geoms, int32_t n_geoms, int32_t device,
                                fofse_multi_plan* out) {
    if (!geoms || !out || n_geoms < 1 || n_geoms > FOFSE_MULTI_MAX_GEOMS) return FOFSE_ERR_ARG;
    fofse_multi_plan mp = new (std::nothrow) fofse_multi_plan_s;
    if (!mp) return FOFSE_ERR_NOMEM;
    mp->device = device;
    for (int g = 0; g < n_geoms; ++g) {
        fofse_plan p = nullptr;
        const fofse_status s = fofse_create(&geoms[g], device, &p);
        if (s != FOFSE_OK) {
            free_multi(mp);
            return s;
        }
        mp->plans.push_back(p);
        GeomStage gs;
        gs.M = geoms[g].area_h;
        gs.N = geoms[g].area_w;
        mp->st.push_back(gs);
    }
    DevGuard guard(device);
    if (!guard.ok) {
        free_multi(mp);
        return FOFSE_ERR_DEVICE;
    }
    for (int g = 0; g < n_geoms; ++g) {
        GeomStage& gs = mp->st[g];
        std::vector<int32_t> bpix;
        for (int i = 0; i < gs.M * gs.N; ++i)
            if (geoms[g].target_mask[i]) bpix.push_back(i);
        gs.nB = (int)bpix.size();
        if (hipMalloc(&gs.d_bpix, bpix.size() * sizeof(int32_t)) != hipSuccess) {
            free_multi(mp);
            return FOFSE_ERR_NOMEM;
        }
        if (hipMemcpy(gs.d_bpix, bpix.data(), bpix.size() * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess) {
            free_multi(mp);
            return FOFSE_ERR_DEVICE;
        }
    }
    if (hipMalloc(&mp->d_counts, (2 * FOFSE_MULTI_MAX_GEOMS + 1) * sizeof(int)) != hipSuccess ||
        hipHostMalloc(&mp->h_counts, (2 * FOFSE_MULTI_MAX_GEOMS + 1) * sizeof(int)) != hipSuccess) {
        free_multi(mp);
        return FOFSE_ERR_NOMEM;
    }
    *out = mp;
    return FOFSE_OK;
}

fofse_plan fofse_multi_geometry_plan(fofse_multi_plan mp, int32_t geom) {
    if (!mp || geom < 0 || geom >= (int)mp->plans.size()) return nullptr;
    return mp->plans[geom];
}

fofse_status fofse_extrapolate_multi(fofse_multi_plan mp, int32_t n_blocks, const int32_t* d_geom_id,
                                     const float* d_areas, const int64_t* d_area_off, const uint8_t* d_known,
                                     const double* d_rho_gamma, float* d_out, int32_t* d_status, void* stream) {
    if (!mp || n_blocks < 0) return FOFSE_ERR_ARG;
    if (n_blocks == 0) return FOFSE_OK;
    if (!d_geom_id || !d_areas || !d_area_off || !d_rho_gamma || !d_out) return FOFSE_ERR_ARG;
    hipStream_t st = (hipStream_t)stream;
    if (capturing(st)) return FOFSE_ERR_UNSUPPORTED;       // the counts are read on the host
    DevGuard guard(mp->device);
    if (!guard.ok) return FOFSE_ERR_DEVICE;
    const int G = (int)mp->plans.size();
    constexpr int TB = 256;
    const int nb = (n_blocks + TB - 1) / TB;
    hipLaunchKernelGGL(k_multi_clear, dim3(1), dim3(TB), 0, st, mp->d_counts, 2 * G + 1);
    hipLaunchKernelGGL(k_multi_count, dim3(nb), dim3(TB), 0, st, d_geom_id, n_blocks, G, mp->d_counts);
    if (hipGetLastError() != hipSuccess) return FOFSE_ERR_DEVICE;
    if (hipMemcpyAsync(mp->h_counts, mp->d_counts, (2 * G + 1) * sizeof(int), hipMemcpyDeviceToHost, st) !=
            hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return FOFSE_ERR_DEVICE;
    if (mp->h_counts[2 * G] != 0) return FOFSE_ERR_ARG;    // a geometry id out of range: nothing run
    Offsets off{};
    int total = 0;
    for (int g = 0; g < G; ++g) {
        off.v[g] = total;
        total += mp->h_counts[g];
    }
    if ((size_t)n_blocks > mp->list_cap) {
        const fofse_status s = grow(mp, &mp->d_list, (size_t)n_blocks);
        if (s != FOFSE_OK) return s;
        mp->list_cap = (size_t)n_blocks;
    }
    hipLaunchKernelGGL(k_multi_fill, dim3(nb), dim3(TB), 0, st, d_geom_id, n_blocks, G, mp->d_counts, off,
                       mp->d_list);
    if (hipGetLastError() != hipSuccess) return FOFSE_ERR_DEVICE;
    for (int g = 0; g < G; ++g) {
        const int c = mp->h_counts[g];
        if (c == 0) continue;
        GeomStage& gs = mp->st[g];
        const size_t MN = (size_t)gs.M * gs.N;
        if ((size_t)c > gs.cap) {
            const size_t cap = (size_t)c > 2 * gs.cap ? (size_t)c : 2 * gs.cap;
            fofse_status s = grow(mp, &gs.d_areas, cap * MN);
            if (s == FOFSE_OK) s = grow(mp, &gs.d_known, cap * MN);
            if (s == FOFSE_OK) s = grow(mp, &gs.d_out, cap * (size_t)gs.nB);
            if (s == FOFSE_OK) s = grow(mp, &gs.d_status, cap);
            if (s != FOFSE_OK) return s;
            gs.cap = cap;
        }
        const int* list = mp->d_list + off.v[g];
        const size_t ng = (size_t)c * MN;
        hipLaunchKernelGGL(k_multi_gather, dim3((unsigned)((ng + TB - 1) / TB)), dim3(TB), 0, st, list, c, (int)MN,
                           d_area_off, d_areas, d_known, gs.d_areas, gs.d_known);
        if (hipGetLastError() != hipSuccess) return FOFSE_ERR_DEVICE;
        const fofse_status s = fofse_extrapolate_batch(mp->plans[g], c, gs.d_areas, d_known ? gs.d_known : nullptr,
                                                       d_rho_gamma, gs.d_out, nullptr, nullptr, gs.d_status, stream);
        if (s != FOFSE_OK) return s;
        const size_t no = (size_t)c * gs.nB;
        hipLaunchKernelGGL(k_multi_scatter, dim3((unsigned)((no + TB - 1) / TB)), dim3(TB), 0, st, list, c, gs.nB,
                           gs.d_bpix, d_area_off, gs.d_out, gs.d_status, d_out, d_status);
        if (hipGetLastError() != hipSuccess) return FOFSE_ERR_DEVICE;
    }
    return FOFSE_OK;
}

void fofse_destroy_multi(fofse_multi_plan mp) {
    if (!mp) return;
    DevGuard guard(mp->device);
    free_multi(mp);
}

}  // extern "C"
