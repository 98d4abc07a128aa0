// Host side of the FOFSE C ABI: argument validation, plan state, launches.
// Every entry point is declared in include/fofse.h.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/fofse.h"
#include "dct_kernel.h"
#include "fofse_kernel.h"

struct fofse_plan_s {
    int device = 0;
    int n_cu = 0;
    int path = FOFSE_PATH_AUTO;
    int waves = 0;                  // split path: wavefronts per block (0 = default)
    int occupancy = 0;              // grouped path: workgroups per compute unit (0 = default)
    int basis = FOFSE_BASIS_DFT;
    int comp = FOFSE_COMP_CONSTANT;
    double* d_dct_cos = nullptr;    // DCT basis: cos(pi k (2m+1) / (2T)) at [m * T + k]
    int M = 0, N = 0, T = 0, K = 0, nB = 0;
    uint8_t* d_target = nullptr;
    int32_t* d_bpix = nullptr;
    int32_t* d_bidx = nullptr;      // [M*N] index in the B list, -1 off B
    int b_m0 = 0, b_n0 = 0, b_h = 0, b_w = 0;
    double2* d_twiddle = nullptr;
    double2* d_htw = nullptr;       // [2T] exp(-j pi q / T)
    double* d_wtab = nullptr;       // rho_hat ** dist per sample, refreshed per call
    double* d_dwtab = nullptr;      // its derivative in rho_hat (adjoint only)
    // per-block gradients when the caller passes no d_grad_block
    size_t gblk_bytes = 0;
    double* d_gblk = nullptr;
    // grouped-path workspace, grown on demand (capacity in blocks)
    int ws_blocks = 0;
    size_t ws_bytes = 0;
    void* d_ws = nullptr;
    // buffers replaced by larger ones: kept until fofse_destroy, since a graph
    // captured before the growth still refers to them
    std::vector<void*> retired;
    // profiling: event pairs around the main kernel of the last kRing calls
    bool timing = false;
    hipEvent_t ev_start[256] = {};
    hipEvent_t ev_stop[256] = {};
    long long n_timed = 0;
    // selection record used when the caller passes no d_sel / d_coef
    size_t rec_sel_bytes = 0, rec_coef_bytes = 0;
    int32_t* d_rec_sel = nullptr;
    double* d_rec_coef = nullptr;
};

namespace {

// Below this many blocks per compute unit the split path (several waves per
// block) finishes sooner than the grouped path (one wave per block).
constexpr int kGroupedMinBlocksPerCu = 8;

bool fft_size_built(int T) { return T == 16 || T == 32 || T == 64 || T == 128; }

// The 128-point kernel keeps a 64 x 64 staging tile of the area.
bool geometry_built(int M, int N, int T) { return fft_size_built(T) && (T != 128 || (M <= 64 && N <= 64)); }

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

constexpr int kRing = 256;

void free_events(fofse_plan p) {
    for (int i = 0; i < kRing; ++i) {
        if (p->ev_start[i]) (void)hipEventDestroy(p->ev_start[i]);
        if (p->ev_stop[i]) (void)hipEventDestroy(p->ev_stop[i]);
        p->ev_start[i] = p->ev_stop[i] = nullptr;
    }
}

void free_plan(fofse_plan p) {
    if (!p) return;
    free_events(p);
    if (p->d_ws) (void)hipFree(p->d_ws);
    if (p->d_rec_sel) (void)hipFree(p->d_rec_sel);
    if (p->d_rec_coef) (void)hipFree(p->d_rec_coef);
    if (p->d_target) (void)hipFree(p->d_target);
    if (p->d_bpix) (void)hipFree(p->d_bpix);
    if (p->d_bidx) (void)hipFree(p->d_bidx);
    if (p->d_twiddle) (void)hipFree(p->d_twiddle);
    if (p->d_htw) (void)hipFree(p->d_htw);
    if (p->d_wtab) (void)hipFree(p->d_wtab);
    if (p->d_dwtab) (void)hipFree(p->d_dwtab);
    if (p->d_gblk) (void)hipFree(p->d_gblk);
    if (p->d_dct_cos) (void)hipFree(p->d_dct_cos);
    for (void* q : p->retired) (void)hipFree(q);
    delete p;
}

// Grouped path: T = 64 (four blocks of one mask per workgroup) and T = 128
// (two blocks of one mask per workgroup, areas up to 64 x 64).
bool grouped_supported(const fofse_plan_s* p) {
    return (p->T == 64 || p->T == 128) && p->nB <= fofse::group_max_target_samples() && p->M <= 64 &&
           p->N <= 64;
}

// True when the stream is being captured into a graph (no allocation may be
// recorded then).
bool capturing(hipStream_t st) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    return hipStreamIsCapturing(st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone;
}

// Grows a plan-owned device buffer to at least `bytes` (to twice its capacity
// at least, so that growth is rare).  The replaced buffer stays allocated until
// fofse_destroy: a graph captured before the growth still refers to it.  Under
// stream capture no buffer is allocated: FOFSE_ERR_UNSUPPORTED.
fofse_status grow_buffer(fofse_plan p, void** buf, size_t* cap, size_t bytes, hipStream_t st) {
    if (bytes <= *cap) return FOFSE_OK;
    if (capturing(st)) return FOFSE_ERR_UNSUPPORTED;
    const size_t nb = bytes > 2 * *cap ? bytes : 2 * *cap;
    void* q = nullptr;
    if (hipMalloc(&q, nb) != hipSuccess) return FOFSE_ERR_NOMEM;
    if (*buf) p->retired.push_back(*buf);
    *buf = q;
    *cap = nb;
    return FOFSE_OK;
}

int hash_slots(int n) {
    int hsize = 64;
    while (hsize < 2 * n) hsize <<= 1;
    return hsize;
}

// Workspace of the grouped path for a capacity of n blocks: hash table of
// hsize slots (key 8 B, representative, count, first item: 4 B each), per-block
// class and position, per-item block list, size and class, the single-mask
// count and up to twelve counters.
size_t workspace_bytes_for(int n) {
    return (size_t)hash_slots(n) * 20 + (size_t)n * (8 + 4 * fofse::kGroup + 8) + 64;
}

// Lays the workspace for a capacity of cap blocks out from base (256-byte
// aligned).
void carve_workspace(void* base, int cap, fofse::GroupArgs& g) {
    const int hsize = hash_slots(cap);
    char* c = (char*)base;
    g.hsize = hsize;
    g.hmask = (uint32_t)(hsize - 1);
    g.ht_key = (unsigned long long*)c; c += (size_t)hsize * 8;
    g.ht_rep = (int*)c; c += (size_t)hsize * 4;
    g.ht_cnt = (int*)c; c += (size_t)hsize * 4;
    g.item_start = (int*)c; c += (size_t)hsize * 4;
    g.cls = (int*)c; c += (size_t)cap * 4;
    g.pos = (int*)c; c += (size_t)cap * 4;
    g.item_blk = (int*)c; c += (size_t)cap * 4 * fofse::kGroup;
    g.item_n = (int*)c; c += (size_t)cap * 4;
    g.item_cls = (int*)c; c += (size_t)cap * 4;
    g.n_single = (int*)c; c += 16;
    g.counts = (int*)c;
}

// The grouping workspace for n blocks: the caller's (ws), else the plan's,
// grown on demand.
fofse_status ensure_workspace(fofse_plan p, int n, fofse::GroupArgs& g, const fofse::Workspace* ws,
                              hipStream_t st) {
    if (ws) {
        if (workspace_bytes_for(n) > ws->bytes) return FOFSE_ERR_LIMIT;
        carve_workspace(ws->base, n, g);
        return FOFSE_OK;
    }
    if (n > p->ws_blocks) {
        const int cap = n > 2 * p->ws_blocks ? n : 2 * p->ws_blocks;
        if (capturing(st)) return FOFSE_ERR_UNSUPPORTED;
        void* q = nullptr;
        if (hipMalloc(&q, workspace_bytes_for(cap)) != hipSuccess) return FOFSE_ERR_NOMEM;
        if (p->d_ws) p->retired.push_back(p->d_ws);
        p->d_ws = q;
        p->ws_blocks = cap;
        p->ws_bytes = workspace_bytes_for(cap);
    }
    carve_workspace(p->d_ws, p->ws_blocks, g);
    return FOFSE_OK;
}

// Record of n blocks (K keys, K coefficients each) owned by the plan.
fofse_status ensure_record(fofse_plan p, int n, hipStream_t st) {
    const size_t k = p->K > 0 ? (size_t)p->K : 1;
    fofse_status s = grow_buffer(p, (void**)&p->d_rec_sel, &p->rec_sel_bytes, (size_t)n * k * sizeof(int32_t), st);
    if (s != FOFSE_OK) return s;
    return grow_buffer(p, (void**)&p->d_rec_coef, &p->rec_coef_bytes, (size_t)n * k * 2 * sizeof(double), st);
}

}  // namespace

namespace fofse {

// fofse_extrapolate_batch with an optional caller-supplied grouping workspace
// (ws; the record must then be the caller's).  Without one, plan-owned
// buffers are grown on demand.
fofse_status extrapolate_impl(fofse_plan p, int32_t n_blocks, const float* d_areas, const uint8_t* d_known,
                              const double* d_rho_gamma, float* d_out, int32_t* d_sel, double* d_coef,
                              int32_t* d_status, void* stream, const Workspace* ws) {
    if (!p || n_blocks < 0) return FOFSE_ERR_ARG;
    if (n_blocks == 0) return FOFSE_OK;
    if (!d_areas || !d_rho_gamma || !d_out) return FOFSE_ERR_ARG;
    DeviceGuard guard(p->device);
    if (!guard.ok) return FOFSE_ERR_DEVICE;
    KParams k{};
    k.n_blocks = n_blocks;
    k.T = p->T; k.M = p->M; k.N = p->N; k.K = p->K; k.nB = p->nB;
    k.areas = d_areas;
    k.known = d_known;
    k.target = p->d_target;
    k.bpix = p->d_bpix;
    k.bidx = p->d_bidx;
    k.b_m0 = p->b_m0; k.b_n0 = p->b_n0; k.b_h = p->b_h; k.b_w = p->b_w;
    k.rho_gamma = d_rho_gamma;
    k.twiddle = p->d_twiddle;
    k.htw = p->d_htw;
    k.wtab = p->d_wtab;
    k.out = d_out;
    k.sel = d_sel;
    k.coef = d_coef;
    k.status = d_status;
    k.waves = p->waves;
    hipStream_t st = (hipStream_t)stream;
    if (!d_sel || !d_coef) {
        if (ws) return FOFSE_ERR_ARG;            // a caller-supplied workspace holds no record
        const fofse_status rs = ensure_record(p, n_blocks, st);
        if (rs != FOFSE_OK) return rs;
        if (!d_sel) k.sel = p->d_rec_sel;
        if (!d_coef) k.coef = p->d_rec_coef;
    }
    if (p->basis == FOFSE_BASIS_DCT && p->comp != FOFSE_COMP_CONSTANT) return FOFSE_ERR_UNSUPPORTED;
    if (p->basis == FOFSE_BASIS_DCT) {
        Timing tm{};
        if (p->timing) {
            const int i = (int)(p->n_timed % kRing);
            tm.start = p->ev_start[i];
            tm.stop = p->ev_stop[i];
            ++p->n_timed;
        }
        GroupArgs g{};
        g.MN = p->M * p->N;
        g.known = d_known;
        g.target = p->d_target;
        g.direct = d_known == nullptr;
        g.vec16 = (p->M * p->N) % 16 == 0 && ((uintptr_t)d_known & 15) == 0;
        g.wg_per_cu = p->occupancy;
        if (!g.direct) {
            const fofse_status wst = ensure_workspace(p, n_blocks, g, ws, st);
            if (wst != FOFSE_OK) return wst;
            if (launch_clear(g, st) != hipSuccess) return FOFSE_ERR_DEVICE;
        }
        const hipError_t e = launch_dct(k, g, p->d_dct_cos, p->n_cu, st, tm);
        return e == hipSuccess ? FOFSE_OK : FOFSE_ERR_DEVICE;
    }
    // the full compensation: grouped organisation at T = 64, one wavefront per
    // block at T = 16 and 32
    const bool full = p->comp == FOFSE_COMP_FULL;
    bool grouped = full && p->T == 64;
    if (p->path == FOFSE_PATH_GROUPED) grouped = true;
    else if (p->path == FOFSE_PATH_AUTO)
        grouped = grouped || (grouped_supported(p) && n_blocks >= kGroupedMinBlocksPerCu * p->n_cu);
    hipError_t e;
    Timing tm{};
    if (p->timing) {
        const int i = (int)(p->n_timed % kRing);
        tm.start = p->ev_start[i];
        tm.stop = p->ev_stop[i];
        ++p->n_timed;
    }
    if (grouped) {
        GroupArgs g{};
        g.MN = p->M * p->N;
        g.known = d_known;
        g.target = p->d_target;
        g.direct = d_known == nullptr;
        g.vec16 = (p->M * p->N) % 16 == 0 && ((uintptr_t)d_known & 15) == 0;
        g.wg_per_cu = p->occupancy;
        if (!g.direct) {
            const fofse_status wst = ensure_workspace(p, n_blocks, g, ws, st);
            if (wst != FOFSE_OK) return wst;
            e = launch_clear(g, st);
            if (e != hipSuccess) return FOFSE_ERR_DEVICE;
        }
        e = p->T == 128 ? launch_grouped128(k, g, p->n_cu, st, tm)
                        : launch_grouped(k, g, p->n_cu, st, tm, full);
    } else {
        e = launch_forward(k, st, tm, full);
    }
    return e == hipSuccess ? FOFSE_OK : FOFSE_ERR_DEVICE;
}

int plan_device(fofse_plan p) { return p ? p->device : -1; }

size_t grouping_workspace_bytes(int n_blocks) { return workspace_bytes_for(n_blocks); }

}  // namespace fofse

extern "C" {

const char* fofse_status_str(fofse_status s) {
    switch (s) {
        case FOFSE_OK: return "ok";
        case FOFSE_ERR_ARG: return "invalid argument";
        case FOFSE_ERR_UNSUPPORTED: return "unsupported configuration";
        case FOFSE_ERR_NOMEM: return "device allocation failed";
        case FOFSE_ERR_DEVICE: return "HIP runtime or launch failure";
        case FOFSE_ERR_LIMIT: return "batch exceeds the fixed scratch of the no-allocation entry point";
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
    if (!geometry_built(M, N, T)) return FOFSE_ERR_UNSUPPORTED;

    std::vector<int32_t> bpix;
    for (int i = 0; i < M * N; ++i)
        if (g->target_mask[i]) bpix.push_back(i);
    if (bpix.empty()) return FOFSE_ERR_ARG;
    if ((int)bpix.size() > fofse::max_target_samples(T)) return FOFSE_ERR_UNSUPPORTED;

    std::vector<int32_t> bidx(M * N, -1);
    int m0 = M, m1 = -1, n0 = N, n1 = -1;
    for (size_t q = 0; q < bpix.size(); ++q) {
        const int i = bpix[q], m = i / N, n = i % N;
        bidx[i] = (int32_t)q;
        m0 = m < m0 ? m : m0; m1 = m > m1 ? m : m1;
        n0 = n < n0 ? n : n0; n1 = n > n1 ? n : n1;
    }
    std::vector<uint8_t> target(M * N);
    for (int i = 0; i < M * N; ++i) target[i] = g->target_mask[i] ? 1 : 0;
    std::vector<double2> tw(T), htw(2 * T);
    for (int q = 0; q < T; ++q) {
        const double ang = 2.0 * M_PI * (double)q / (double)T;
        tw[q] = make_double2(std::cos(ang), -std::sin(ang));
    }
    for (int q = 0; q < 2 * T; ++q) {
        const double ang = M_PI * (double)q / (double)T;
        htw[q] = make_double2(std::cos(ang), -std::sin(ang));
    }

    DeviceGuard guard(device);
    if (!guard.ok) return FOFSE_ERR_DEVICE;
    int n_cu = 0;
    if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
        return FOFSE_ERR_DEVICE;
    fofse_plan p = new (std::nothrow) fofse_plan_s;
    if (!p) return FOFSE_ERR_NOMEM;
    p->device = device;
    p->n_cu = n_cu;
    p->M = M; p->N = N; p->T = T; p->K = K;
    p->nB = (int)bpix.size();
    p->b_m0 = m0; p->b_n0 = n0; p->b_h = m1 - m0 + 1; p->b_w = n1 - n0 + 1;
    if (hipMalloc(&p->d_target, M * N) != hipSuccess ||
        hipMalloc(&p->d_bpix, bpix.size() * sizeof(int32_t)) != hipSuccess ||
        hipMalloc(&p->d_bidx, (size_t)M * N * sizeof(int32_t)) != hipSuccess ||
        hipMalloc(&p->d_twiddle, T * sizeof(double2)) != hipSuccess ||
        hipMalloc(&p->d_htw, 2 * T * sizeof(double2)) != hipSuccess ||
        hipMalloc(&p->d_wtab, (size_t)M * N * sizeof(double)) != hipSuccess ||
        hipMalloc(&p->d_dwtab, (size_t)M * N * sizeof(double)) != hipSuccess) {
        free_plan(p);
        return FOFSE_ERR_NOMEM;
    }
    if (hipMemcpy(p->d_target, target.data(), M * N, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(p->d_bpix, bpix.data(), bpix.size() * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(p->d_bidx, bidx.data(), (size_t)M * N * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(p->d_twiddle, tw.data(), T * sizeof(double2), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(p->d_htw, htw.data(), 2 * T * sizeof(double2), hipMemcpyHostToDevice) != hipSuccess) {
        free_plan(p);
        return FOFSE_ERR_DEVICE;
    }
    *out = p;
    return FOFSE_OK;
}

int32_t fofse_target_count(fofse_plan p) { return p ? p->nB : 0; }

fofse_status fofse_set_path(fofse_plan p, int32_t path) {
    if (!p || path < FOFSE_PATH_AUTO || path > FOFSE_PATH_GROUPED) return FOFSE_ERR_ARG;
    if (path == FOFSE_PATH_GROUPED && !grouped_supported(p)) return FOFSE_ERR_UNSUPPORTED;
    p->path = path;
    return FOFSE_OK;
}

fofse_status fofse_set_basis(fofse_plan p, int32_t basis) {
    if (!p || (basis != FOFSE_BASIS_DFT && basis != FOFSE_BASIS_DCT)) return FOFSE_ERR_ARG;
    if (basis == FOFSE_BASIS_DCT) {
        if (!fofse::dct_size_supported(p->T)) return FOFSE_ERR_UNSUPPORTED;
        if (!p->d_dct_cos) {
            const int T = p->T;
            std::vector<double> c((size_t)T * T);
            for (int m = 0; m < T; ++m)
                for (int k = 0; k < T; ++k)
                    c[(size_t)m * T + k] = std::cos(M_PI * (double)k * (2.0 * m + 1.0) / (2.0 * T));
            DeviceGuard guard(p->device);
            if (!guard.ok) return FOFSE_ERR_DEVICE;
            double* d = nullptr;
            if (hipMalloc(&d, c.size() * sizeof(double)) != hipSuccess) return FOFSE_ERR_NOMEM;
            if (hipMemcpy(d, c.data(), c.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
                (void)hipFree(d);
                return FOFSE_ERR_DEVICE;
            }
            p->d_dct_cos = d;
        }
    }
    p->basis = basis;
    return FOFSE_OK;
}

fofse_status fofse_set_compensation(fofse_plan p, int32_t mode) {
    if (!p || (mode != FOFSE_COMP_CONSTANT && mode != FOFSE_COMP_FULL)) return FOFSE_ERR_ARG;
    if (mode == FOFSE_COMP_FULL && !(p->T == 16 || p->T == 32 || (p->T == 64 && grouped_supported(p))))
        return FOFSE_ERR_UNSUPPORTED;
    p->comp = mode;
    return FOFSE_OK;
}

fofse_status fofse_set_occupancy(fofse_plan p, int32_t wg_per_cu) {
    if (!p || wg_per_cu < 0) return FOFSE_ERR_ARG;
    if (wg_per_cu > (p->T == 64 ? 2 : 1)) return FOFSE_ERR_UNSUPPORTED;
    p->occupancy = wg_per_cu;
    return FOFSE_OK;
}

fofse_status fofse_set_waves(fofse_plan p, int32_t waves) {
    if (!p || waves < 0) return FOFSE_ERR_ARG;
    if (!fofse::split_waves_built(p->T, waves)) return FOFSE_ERR_UNSUPPORTED;
    p->waves = waves;
    return FOFSE_OK;
}

fofse_status fofse_set_timing(fofse_plan p, int32_t enable) {
    if (!p) return FOFSE_ERR_ARG;
    DeviceGuard guard(p->device);
    if (!guard.ok) return FOFSE_ERR_DEVICE;
    if (enable) {
        for (int i = 0; i < kRing; ++i) {
            if (!p->ev_start[i] && hipEventCreate(&p->ev_start[i]) != hipSuccess) return FOFSE_ERR_DEVICE;
            if (!p->ev_stop[i] && hipEventCreate(&p->ev_stop[i]) != hipSuccess) return FOFSE_ERR_DEVICE;
        }
        p->n_timed = 0;
        p->timing = true;
    } else {
        p->timing = false;
    }
    return FOFSE_OK;
}

int32_t fofse_kernel_times(fofse_plan p, float* ms_out, int32_t max) {
    if (!p || !ms_out || max <= 0 || !p->timing) return 0;
    DeviceGuard guard(p->device);
    if (!guard.ok) return 0;
    long long n = p->n_timed < kRing ? p->n_timed : kRing;
    if (n > max) n = max;
    int32_t w = 0;
    for (long long c = p->n_timed - n; c < p->n_timed; ++c) {
        const int i = (int)(c % kRing);
        float ms = 0.0f;
        if (hipEventSynchronize(p->ev_stop[i]) != hipSuccess ||
            hipEventElapsedTime(&ms, p->ev_start[i], p->ev_stop[i]) != hipSuccess)
            return w;
        ms_out[w++] = ms;
    }
    return w;
}

fofse_status fofse_extrapolate_batch(fofse_plan p, int32_t n_blocks, const float* d_areas,
                                     const uint8_t* d_known, const double* d_rho_gamma,
                                     float* d_out, int32_t* d_sel, double* d_coef,
                                     int32_t* d_status, void* stream) {
    return fofse::extrapolate_impl(p, n_blocks, d_areas, d_known, d_rho_gamma, d_out, d_sel, d_coef, d_status,
                                   stream, nullptr);
}

fofse_status fofse_backward(fofse_plan p, int32_t n_blocks, const float* d_areas,
                            const uint8_t* d_known, const double* d_rho_gamma,
                            const int32_t* d_sel, const double* d_coef, const float* d_grad_out,
                            float* d_grad_areas, double* d_grad_rho_gamma, double* d_grad_block,
                            void* stream) {
    if (!p || n_blocks < 0) return FOFSE_ERR_ARG;
    if (n_blocks == 0) return FOFSE_OK;
    if (!d_areas || !d_rho_gamma || !d_sel || !d_coef || !d_grad_out) return FOFSE_ERR_ARG;
    if (p->K > (p->T == 128 ? fofse::kBackwardMaxK128 : fofse::kBackwardMaxK) || p->basis != FOFSE_BASIS_DFT ||
        p->comp != FOFSE_COMP_CONSTANT)
        return FOFSE_ERR_UNSUPPORTED;
    DeviceGuard guard(p->device);
    if (!guard.ok) return FOFSE_ERR_DEVICE;
    hipStream_t st = (hipStream_t)stream;
    double* blk = d_grad_block;
    if (!blk) {
        const fofse_status gs = grow_buffer(p, (void**)&p->d_gblk, &p->gblk_bytes,
                                            (size_t)n_blocks * 2 * sizeof(double), st);
        if (gs != FOFSE_OK) return gs;
        blk = p->d_gblk;
    }
    fofse::KParams wp{};
    wp.T = p->T; wp.M = p->M; wp.N = p->N; wp.K = p->K; wp.nB = p->nB;
    wp.rho_gamma = d_rho_gamma;
    wp.wtab = p->d_wtab;
    wp.dwtab = p->d_dwtab;
    fofse::BParams b{};
    b.n_blocks = n_blocks;
    b.T = p->T; b.M = p->M; b.N = p->N; b.K = p->K; b.nB = p->nB;
    b.areas = d_areas;
    b.known = d_known;
    b.target = p->d_target;
    b.bpix = p->d_bpix;
    b.rho_gamma = d_rho_gamma;
    b.wtab = p->d_wtab;
    b.dwtab = p->d_dwtab;
    b.twiddle = p->d_twiddle;
    b.sel = d_sel;
    b.coef = d_coef;
    b.grad_out = d_grad_out;
    b.grad_areas = d_grad_areas;
    b.grad_block = blk;
    b.bidx = p->d_bidx;
    b.b_m0 = p->b_m0; b.b_n0 = p->b_n0; b.b_h = p->b_h; b.b_w = p->b_w;
    fofse::Timing tm{};
    if (p->timing) {
        const int i = (int)(p->n_timed % kRing);
        tm.start = p->ev_start[i];
        tm.stop = p->ev_stop[i];
        ++p->n_timed;
    }
    // grouped adjoint: same rule as the forward, for K up to its register capacity
    const bool grouped_ok = p->T == 64 && grouped_supported(p) && p->K <= fofse::kGroupBackwardMaxK;
    bool grouped = false;
    if (p->path == FOFSE_PATH_GROUPED) grouped = grouped_ok;
    else if (p->path == FOFSE_PATH_AUTO) grouped = grouped_ok && n_blocks >= kGroupedMinBlocksPerCu * p->n_cu;
    hipError_t e;
    if (grouped) {
        fofse::GroupArgs g{};
        g.MN = p->M * p->N;
        g.known = d_known;
        g.target = p->d_target;
        g.direct = d_known == nullptr;
        g.vec16 = (p->M * p->N) % 16 == 0 && ((uintptr_t)d_known & 15) == 0;
        g.wg_per_cu = p->occupancy;
        if (!g.direct) {
            const fofse_status wst = ensure_workspace(p, n_blocks, g, nullptr, st);
            if (wst != FOFSE_OK) return wst;
            e = fofse::launch_clear(g, st);
            if (e != hipSuccess) return FOFSE_ERR_DEVICE;
        }
        e = fofse::launch_backward_grouped(wp, b, g, p->n_cu, d_grad_rho_gamma, st, tm);
    } else {
        e = fofse::launch_backward(wp, b, d_grad_rho_gamma, st, tm);
    }
    return e == hipSuccess ? FOFSE_OK : FOFSE_ERR_DEVICE;
}

void fofse_destroy(fofse_plan p) {
    if (!p) return;
    DeviceGuard guard(p->device);
    free_plan(p);
}

}  // extern "C"
