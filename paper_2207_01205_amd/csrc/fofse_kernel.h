// Internal interface between the C-ABI host code and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/fofse.h"

namespace fofse {

// Waves per workgroup (one workgroup = one block) for each FFT size.
constexpr int kWaves64 = 4;
constexpr int kWaves32 = 2;

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
    const double2* twiddle;  // [T] exp(-j 2 pi q / T)
    float* out;              // [n][nB]
    int32_t* sel;            // [n][K] or null
    double* coef;            // [n][K][2] or null
    int32_t* status;         // [n] or null
};

// Largest number of samples of B a workgroup can hold for FFT size T.
int max_target_samples(int T);

hipError_t launch_forward(const KParams& p, hipStream_t stream);

}  // namespace fofse
