// Synthesis of the model on the missing area (eqs. 1 and 2) as FP64 matrix
// products on the matrix cores.
//
// g[m, n] = sum_nu Re(c'_nu exp(+j 2 pi (k_nu m + l_nu n) / T)) with
// c' = 2 c for a conjugate pair and c for a self-conjugate class.  For a 16 x 16
// tile of B's bounding box this is one real product of a 16 x 2K matrix and a
// 2K x 16 matrix:
//     A[m, (nu, 0)] = Re(c'_nu a_nu[m]),  A[m, (nu, 1)] = -Im(c'_nu a_nu[m]),
//     B[(nu, 0), n] = Re b_nu[n],         B[(nu, 1), n] = Im b_nu[n],
// with a_nu[m] = exp(+j 2 pi k_nu m / T) and b_nu[n] = exp(+j 2 pi l_nu n / T),
// so that (A B)[m, n] = sum_nu Re(c'_nu a_nu[m] b_nu[n]) = g[m, n].  Each step of
// v_mfma_f64_16x16x4f64 takes two iterations (four columns of A).  One
// wavefront per (block, tile); the record is staged through LDS per wavefront.
//
// Operand layout of v_mfma_f64_16x16x4f64 (checked on the device): lane L holds
// A[L % 16][L / 16] and B[L / 16][L % 16]; result register r of lane L holds
// D[4 r + L / 16][L % 16].

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fofse_kernel.h"
#include "device_common.hpp"

namespace fofse {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kSynWaves = 4;
constexpr int kSynChunk = 128;         // record entries staged per pass (even)

template <int T>
__global__ __launch_bounds__(64 * kSynWaves) void k_synthesize_mfma(KParams p) {
    constexpr int LOG2 = T == 128 ? 7 : T == 64 ? 6 : T == 32 ? 5 : 4;
    __shared__ double2 tw[T];
    __shared__ double2 rc[kSynWaves][kSynChunk];
    __shared__ int rk[kSynWaves][kSynChunk];
    const int tid = (int)__builtin_amdgcn_workitem_id_x();
    const int lane = tid & 63, wave = tid >> 6;
    for (int i = tid; i < T; i += 64 * kSynWaves) tw[i] = p.twiddle[i];
    __syncthreads();
    const int tiles_c = (p.b_w + 15) >> 4, ntile = ((p.b_h + 15) >> 4) * tiles_c;
    const int item = (int)__builtin_amdgcn_workgroup_id_x() * kSynWaves + wave;
    if (item >= p.n_blocks * ntile) return;          // no barrier follows
    const int b = item / ntile, t = item - b * ntile;
    const int tr = t / tiles_c, tc = t - tr * tiles_c;
    const int row0 = p.b_m0 + 16 * tr, col0 = p.b_n0 + 16 * tc;
    const int m = row0 + (lane & 15);                // row of A for this lane
    const int n = col0 + (lane & 15);                // column of B for this lane
    const int kk = lane >> 4, half = kk >> 1, part = kk & 1;
    const int K = p.K;
    const int32_t* sel = p.sel + (size_t)b * K;
    const double2* coef = (const double2*)(p.coef + 2 * (size_t)b * K);
    double2* wrc = rc[wave];
    int* wrk = rk[wave];
    d4 acc = {0.0, 0.0, 0.0, 0.0};
    for (int c0 = 0; c0 < K; c0 += kSynChunk) {
        const int cnt = min(kSynChunk, K - c0);
        const int cnt2 = (cnt + 1) & ~1;
        // stage this wavefront's entries (its own LDS rows: lanes of one
        // wavefront see each other's LDS writes in program order)
        __builtin_amdgcn_wave_barrier();
        for (int i = lane; i < cnt2; i += 64) {
            double2 c = make_double2(0.0, 0.0);
            int kl = 0;
            if (i < cnt) {
                const int key = sel[c0 + i];
                const int k = (key >> LOG2) & (T - 1), l = key & (T - 1);
                const bool selfc = ((k & (T / 2 - 1)) == 0) && ((l & (T / 2 - 1)) == 0);
                const double mult = selfc ? 1.0 : 2.0;
                const double2 cv = coef[c0 + i];
                c = make_double2(mult * cv.x, mult * cv.y);
                kl = (k << 8) | l;
            }
            wrc[i] = c;
            wrk[i] = kl;
        }
        __builtin_amdgcn_wave_barrier();
        for (int s = 0; s < cnt2; s += 2) {
            const int i = s + half;
            const double2 c = wrc[i];
            const int kl = wrk[i];
            const double2 ta = tw[((kl >> 8) * m) & (T - 1)];     // exp(-j 2 pi k m / T)
            const double2 tb = tw[((kl & 255) * n) & (T - 1)];    // exp(-j 2 pi l n / T)
            // c' exp(+j theta): cos = ta.x, sin = -ta.y
            const double are = c.x * ta.x + c.y * ta.y;
            const double aim = c.y * ta.x - c.x * ta.y;
            const double av = part ? -aim : are;
            const double bv = part ? -tb.y : tb.x;
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
        }
    }
    const int rmax = p.b_m0 + p.b_h, cmax = p.b_n0 + p.b_w;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int mm = row0 + 4 * r + (lane >> 4), nn = col0 + (lane & 15);
        if (mm < rmax && nn < cmax) {
            const int q = p.bidx[mm * p.N + nn];
            if (q >= 0) p.out[(size_t)b * p.nB + q] = (float)acc[r];
        }
    }
}

template <int T>
hipError_t launch_t(const KParams& p, hipStream_t stream) {
    const int ntile = ((p.b_h + 15) >> 4) * ((p.b_w + 15) >> 4);
    const long long items = (long long)p.n_blocks * ntile;
    const int grid = (int)((items + kSynWaves - 1) / kSynWaves);
    hipLaunchKernelGGL(k_synthesize_mfma<T>, dim3(grid), dim3(64 * kSynWaves), 0, stream, p);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_synthesis(const KParams& p, hipStream_t stream) {
    switch (p.T) {
        case 16: return launch_t<16>(p, stream);
        case 32: return launch_t<32>(p, stream);
        case 64: return launch_t<64>(p, stream);
        case 128: return launch_t<128>(p, stream);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace fofse
