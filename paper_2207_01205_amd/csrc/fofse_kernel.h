// Internal interface between the C-ABI host code and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/fofse.h"

namespace fofse {

// Waves per workgroup (one workgroup = one block) for each FFT size.
constexpr int kWaves64 = 4;
constexpr int kWaves32 = 2;
constexpr int kWaves16 = 1;

struct KParams {
    int n_blocks;
    int T;                   // FFT size
    int M, N;                // area size
    int K;                   // iterations
    int nB;                  // samples of the missing area
    const float* areas;      // [n][M*N]
    const uint8_t* known;    // [n][M*N] or null (complement of B)
    const uint8_t* target;   // [M*N], non-zero on B
    const int32_t* bpix;     // [nB] flat indices m*N+n of B, row-major
    const double* rho_gamma; // [2]
    double* wtab;            // [M*N] rho_hat ** dist(centre), filled by k_weights
    double* dwtab;           // [M*N] d/drho_hat of wtab, or null (not needed)
    const double2* twiddle;  // [T] exp(-j 2 pi q / T)
    const double2* htw;      // [2T] exp(-j pi q / T) (centring phase of a symmetric w)
    float* out;              // [n][nB]
    int32_t* sel;            // [n][K] selection record (caller's or plan workspace)
    double* coef;            // [n][K][2] coefficient record
    int32_t* status;         // [n] or null
    int waves;               // split path: wavefronts per block (0 = default)
    const int32_t* bidx;     // [M*N] index of the sample in B's list, -1 off B
    int b_m0, b_n0, b_h, b_w; // bounding box of B (first row, first column, rows, columns)
};

// Wavefronts per block the split path is built for, per FFT size.
bool split_waves_built(int T, int waves);

// Arguments of the adjoint (backward) kernels.
struct BParams {
    int n_blocks;
    int T, M, N, K, nB;
    const float* areas;      // [n][M*N]
    const uint8_t* known;    // [n][M*N] or null
    const uint8_t* target;   // [M*N]
    const int32_t* bpix;     // [nB]
    const double* rho_gamma; // [2]
    const double* wtab;      // [M*N] rho_hat ** dist
    const double* dwtab;     // [M*N] dist * rho_hat ** (dist - 1)
    const double2* twiddle;  // [T] exp(-j 2 pi q / T)
    const int32_t* sel;      // [n][K] forward record: class keys
    const double* coef;      // [n][K][2] forward record: coefficients
    const float* grad_out;   // [n][nB] dL/dg on B
    float* grad_areas;       // [n][M*N] dL/df, or null
    double* grad_block;      // [n][2] per-block (dL/drho_hat, dL/dgamma)
    const int32_t* bidx;     // [M*N] index of the sample in B's list, -1 off B
    int b_m0, b_n0, b_h, b_w; // bounding box of B
};

// Largest K the adjoint kernel holds in LDS (FFT sizes 16-64, and 128).
constexpr int kBackwardMaxK = 2048;
constexpr int kBackwardMaxK128 = 512;

// Blocks per workgroup in the grouped path (they share one W).
constexpr int kGroup = 4;
constexpr int kGroupShift = 2;

// Largest K of the grouped adjoint (K / 64 rows per lane in registers).
constexpr int kGroupBackwardMaxK = 256;

// Device workspace and arguments of the grouped path.
struct GroupArgs {
    int direct;                       // 1: every block has the complement of B as support
    int gsize;                        // blocks per work item (1, 2 or kGroup)
    int gshift;                       // log2(gsize)
    int vec16;                        // MN % 16 == 0 and known 16-byte aligned: masks read 16 bytes at a time
    int n_wg;                         // workgroups of the persistent main kernel
    int wg_per_cu;                    // resident workgroups per compute unit asked for (0: the kernel's default)
    int MN;                           // samples per area
    const uint8_t* known;             // [n][MN] or null
    const uint8_t* target;            // [MN]
    uint32_t hmask;                   // hash table size - 1 (power of two)
    int hsize;
    unsigned long long* ht_key;       // [hsize] mask hash | 1, 0 = empty
    int* ht_rep;                      // [hsize] first block of the class
    int* ht_cnt;                      // [hsize] blocks in the class
    int* item_start;                  // [hsize] first work item of the class
    int* cls;                         // [n] class slot, -1 for a singleton
    int* pos;                         // [n] position inside the class / singleton index
    int* n_single;                    // [1]
    int* counts;                      // [2] grouped items, all items
    int* item_blk;                    // [n][kGroup] blocks of a work item (first gsize used)
    int* item_n;                      // [n] blocks in the item
    int* item_cls;                    // [n] class of the item
};

// Device memory a caller lends to a call for the grouping workspace (the
// no-allocation entry point's fixed scratch).
struct Workspace {
    void* base;          // 256-byte aligned device address
    size_t bytes;        // capacity
};

// fofse_extrapolate_batch with an optional workspace in place of the plan's
// (ws non-null: d_sel and d_coef are required, nothing is allocated).
fofse_status extrapolate_impl(fofse_plan p, int32_t n_blocks, const float* d_areas, const uint8_t* d_known,
                              const double* d_rho_gamma, float* d_out, int32_t* d_sel, double* d_coef,
                              int32_t* d_status, void* stream, const Workspace* ws);
// HIP device of a plan (-1 for NULL).
int plan_device(fofse_plan p);
// Bytes of grouping workspace a batch of n blocks uses.
size_t grouping_workspace_bytes(int n_blocks);

// Optional events recorded on the stream right before and after the main
// iteration kernel (null: not recorded).
struct Timing {
    hipEvent_t start = nullptr;
    hipEvent_t stop = nullptr;
};

// Largest number of samples of B a workgroup can hold for FFT size T.
int max_target_samples(int T);
int group_max_target_samples();

// Per-block organisation (T = 16, 32, 64, 128).  full: the full compensation
// (eqs. 10-13), built for T = 16 and 32 with one wavefront per block.
hipError_t launch_forward(const KParams& p, hipStream_t stream, const Timing& tm, bool full = false);
hipError_t launch_synthesis(const KParams& p, hipStream_t stream);
hipError_t launch_weights(const KParams& p, hipStream_t stream);
// full: the full orthogonality deficiency compensation (eqs. 10-13) instead of
// the constant factor of eq. 14.
hipError_t launch_grouped(const KParams& p, const GroupArgs& g, int n_cu, hipStream_t stream,
                          const Timing& tm, bool full = false);
hipError_t launch_clear(const GroupArgs& g, hipStream_t stream);
hipError_t launch_fwd128(const KParams& p, hipStream_t stream);
hipError_t launch_grouped128(const KParams& p, const GroupArgs& g, int n_cu, hipStream_t stream,
                             const Timing& tm);
hipError_t launch_backward(const KParams& wp, const BParams& p, double* d_sum, hipStream_t stream,
                           const Timing& tm);
// Mask classes and work items of n blocks (grouped forward and adjoint).
hipError_t launch_grouping(const GroupArgs& g, int n, hipStream_t stream);
hipError_t launch_backward_grouped(const KParams& wp, const BParams& p, const GroupArgs& g, int n_cu,
                                   double* d_sum, hipStream_t stream, const Timing& tm);
hipError_t launch_bwd_sum(const BParams& p, double* d_sum, hipStream_t stream);
hipError_t launch_bwd128(const BParams& p, hipStream_t stream);

}  // namespace fofse
