// FOFSE forward kernel for gfx950 (MI355X).
//
// Seiler & Kaup, fast orthogonality deficiency compensated frequency selective
// extrapolation: Section 2 (eqs. 1-9 and 14) with the 2-D DFT basis handled
// entirely in the transform domain (Section 2, last paragraph before the
// compensation; Section 3 names the T x T FFT).
//
// One workgroup extrapolates one block.  Per block:
//   1. w = a * rho_hat^dist (eqs. 4, 15) and z = w + j*(w*f) are formed on a
//      T x T grid in LDS; one complex 2-D FFT of z yields both W = DFT(w) and
//      R = DFT(w*f) (eqs. 7, 8), separated by Hermitian symmetry.
//   2. The area is placed transposed on the grid, so grid row r is the class
//      index l and grid column c is k of the basis phi_{k,l}[m,n] =
//      exp(+j 2 pi (k m + l n) / T); the stored half l in [0, T/2] is then the
//      representative half of the conjugate classes.  R (grid rows 0..T/2, all
//      T columns, IEEE double) stays in VGPRs: lane = grid column, register
//      slot = grid row.  W is written to an LDS "window" of rows
//      -T/4 .. 3T/4 (T+1 rows), so that for every register slot the two shifted
//      reads W[k-u, l-v] and W[k+u, l+v] are a per-lane base address plus a
//      compile-time row offset (rows below T/4 read the first term through
//      W[k-u] = conj(W[u-k]); rows above T/4 read the second through
//      W[k+u] = conj(W[-k-u])).
//   3. K iterations: argmax of |R| over the conjugate classes (eq. 9) by a
//      lane scan, a wavefront reduction and one LDS exchange between the waves
//      of the workgroup; c = gamma R[u]/W0 (eqs. 5, 14); every stored bin gets
//      R[k] -= c W[k-u] + conj(c) W[k+u] (eq. 3 via the DFT shift theorem);
//      the selection record (class key and c of every iteration) is written,
//      and the synthesis kernel builds the model on the missing area from it
//      (eqs. 1, 2).
//   A compile-time variant (FULL, one wavefront per block, T = 16 and 32)
//   takes c from the full compensation of eqs. 10-13 instead of eq. 14.
//
// No MFMA: the update is a shifted rank-2 update, not a contraction.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fofse_kernel.h"
#include "device_common.hpp"
#include "iterate.hpp"

namespace fofse {

// ---------------------------------------------------------------------------
// kernel
// ---------------------------------------------------------------------------

// R of this wave's rows from the transform Z = W + jR sitting in LDS in the
// FFT's output order, then the residual iteration.  Contains the two barriers
// that turn the LDS grid into the W window (all waves reach them).
template <int T, int NW, int WI, int WPT, bool FULL>
__device__ __forceinline__ void wave_body(double2* win, Xchg<NW>* xchg, const KParams& p, int b,
                                          int tid, int lane, const double2* wv, double gW0,
                                          int flags_pre, int* s_flags) {
    using L = Layout<T, NW>;
    using WR = WaveRows<T, NW, WI>;
    constexpr int S = WR::S;
    constexpr int NT = L::NT;
    constexpr int WROWS = L::WROWS;
    RegSpec<S> R;
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const int k = WR::k0 + s;
        double a_re = 0.0, a_im = 0.0;
        if (lane < T) {
            const double2 a = win[FftPlan<T>::perm(k) * T + FftPlan<T>::perm(lane)];
            const double2 c = win[FftPlan<T>::perm((-k) & (T - 1)) * T + FftPlan<T>::perm((-lane) & (T - 1))];
            a_re = 0.5 * (a.y + c.y);
            a_im = 0.5 * (c.x - a.x);
        }
        R.set(s, a_re, a_im);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < WPT; ++j) {
        const int e = tid + j * NT;
        if (e < WROWS * T) win[e] = wv[j];
    }
    __syncthreads();
    const int flags = *s_flags | flags_pre;
    if (flags == 0)
        run_wave<T, NW, WI, FULL>(R, win, xchg, p, b, lane, gW0);
}

// Every wave of the workgroup runs wave_body with its own compile-time row
// range (each wave takes the same barriers in it).
template <int T, int NW, int WI, int WPT, bool FULL>
__device__ __forceinline__ void dispatch_wave(int wave, double2* win, Xchg<NW>* xchg, const KParams& p, int b,
                                              int tid, int lane, const double2* wv, double gW0, int flags_pre,
                                              int* s_flags) {
    if (wave == WI) wave_body<T, NW, WI, WPT, FULL>(win, xchg, p, b, tid, lane, wv, gW0, flags_pre, s_flags);
    if constexpr (WI + 1 < NW)
        dispatch_wave<T, NW, WI + 1, WPT, FULL>(wave, win, xchg, p, b, tid, lane, wv, gW0, flags_pre, s_flags);
}

// FULL: the full compensation of eqs. 10-13 instead of eq. 14 (one wavefront
// per block; gamma is not used).
template <int T, int NW, bool FULL = false>
__global__ __launch_bounds__(NW * 64, 2) void fofse_fwd_kernel(KParams p) {
    using L = Layout<T, NW>;
    constexpr int NT = L::NT;
    constexpr int Q = L::Q;
    constexpr int WROWS = L::WROWS;
    constexpr int WPT = (WROWS * T + NT - 1) / NT;    // window entries per thread
    __shared__ double2 win[WROWS * T];
    __shared__ double2 tw[T];
    __shared__ Xchg<NW> xchg[2];
    __shared__ int s_flags;

    const int tid = (int)__builtin_amdgcn_workitem_id_x();
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int b = (int)__builtin_amdgcn_workgroup_id_x();
    const int M = p.M, N = p.N, K = p.K;
    const double rho = p.rho_gamma[0];
    const double gamma = p.rho_gamma[1];

    for (int i = tid; i < T; i += NT) tw[i] = p.twiddle[i];
    for (int i = tid; i < T * T; i += NT) win[i] = make_double2(0.0, 0.0);
    const bool params_ok = param_ok(rho) && (FULL || param_ok(gamma));
    if (tid == 0) s_flags = params_ok ? 0 : FOFSE_BLOCK_BAD_PARAM;
    __syncthreads();

    // eqs. 4, 15: w = rho_hat^dist on A;  z = w + j w f, placed transposed
    const size_t area_base = (size_t)b * M * N;
    for (int i = tid; i < M * N; i += NT) {
        const int m = i / N, n = i - m * N;
        bool a = p.target[i] == 0;
        if (p.known) a = a && (p.known[area_base + i] != 0);
        double w = 0.0, wf = 0.0;
        if (a) {
            const uint32_t fb = sample_bits(p.areas, area_base + i);
            if (nonfinite_bits(fb)) {
                atomicOr(&s_flags, FOFSE_BLOCK_NONFINITE);
            } else {
                w = p.wtab[i];
                wf = w * (double)__uint_as_float(fb);
            }
        }
        win[n * T + m] = make_double2(w, wf);
    }
    __syncthreads();

    // eqs. 7, 8: 2-D DFT of z (grid rows N..T-1 are zero before the row pass)
    fft_stage_a<T, NT>(win, tw, N, T, 1, tid);
    __syncthreads();
    fft_stage_b<T, NT>(win, N, T, 1, tid);
    __syncthreads();
    fft_stage_a<T, NT>(win, tw, T, 1, T, tid);
    __syncthreads();
    fft_stage_b<T, NT>(win, T, 1, T, tid);
    __syncthreads();

    // Z[kr][kc] sits at win[perm(kr) * T + perm(kc)].  W = (Z + conj Z(-k)) / 2
    // goes to the window: window row i holds grid row (i - T/4) mod T.
    auto zat = [&](int kr, int kc) -> double2 {
        return win[FftPlan<T>::perm(kr & (T - 1)) * T + FftPlan<T>::perm(kc & (T - 1))];
    };
    const double W0 = win[0].x;
    const int flags_pre = (!params_ok || W0 > 0.0) ? 0 : FOFSE_BLOCK_NO_SUPPORT;
    const double gW0 = gamma / W0;
    double2 wv[WPT];
#pragma unroll
    for (int j = 0; j < WPT; ++j) {
        const int e = tid + j * NT;
        wv[j] = make_double2(0.0, 0.0);
        if (e < WROWS * T) {
            const int i = e / T, c = e - i * T;
            const int r = i - Q;
            const double2 a = zat(r, c), z2 = zat(-r, -c);
            wv[j] = make_double2(0.5 * (a.x + z2.x), 0.5 * (a.y - z2.y));
        }
    }

    dispatch_wave<T, NW, 0, WPT, FULL>(wave, win, xchg, p, b, tid, lane, wv, gW0, flags_pre, &s_flags);

    // parameters out of range: that flag alone (as on every other path)
    const int flags = params_ok ? (s_flags | flags_pre) : FOFSE_BLOCK_BAD_PARAM;
    if (flags != 0) {          // empty record: the synthesised model is 0
        for (int it = tid; it < K; it += NT) {
            p.sel[(size_t)b * K + it] = 0;
            p.coef[2 * ((size_t)b * K + it)] = 0.0;
            p.coef[2 * ((size_t)b * K + it) + 1] = 0.0;
        }
    }
    if (p.status && tid == 0) p.status[b] = flags;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

template <int T, int NW, bool FULL = false>
static hipError_t launch_fwd(const KParams& p, hipStream_t stream) {
    hipLaunchKernelGGL((fofse_fwd_kernel<T, NW, FULL>), dim3(p.n_blocks), dim3(NW * 64), 0, stream, p);
    return hipGetLastError();
}

int max_target_samples(int T) { return T * T; }

bool split_waves_built(int T, int waves) {
    if (waves == 0) return true;
    switch (T) {
        case 16: return waves == 1 || waves == 2;
        case 32: return waves == 1 || waves == 2 || waves == 4;
        case 64: return waves == 2 || waves == 4 || waves == 8;
        case 128: return waves == 8 || waves == 16;
        default: return false;
    }
}

// eq. 15: isotropic model rho_hat ** dist((m, n), ((M-1)/2, (N-1)/2)) for every
// sample of the area (the mask of eq. 4 is applied where it is used).  Kept out
// of the main kernels so that they contain no library calls.
__global__ __launch_bounds__(256) void k_weights(KParams p) {
    const int i = (int)__builtin_amdgcn_workgroup_id_x() * 256 + (int)__builtin_amdgcn_workitem_id_x();
    if (i >= p.M * p.N) return;
    const int m = i / p.N, n = i - m * p.N;
    const double dm = m - 0.5 * (p.M - 1), dn = n - 0.5 * (p.N - 1);
    const double rho = p.rho_gamma[0];
    const bool ok = param_ok(rho);
    const double d = sqrt(dm * dm + dn * dn);
    p.wtab[i] = ok ? pow(rho, d) : 0.0;
    // derivative d rho^(d-1) for the adjoint (0 at the centre sample, d = 0)
    if (p.dwtab) p.dwtab[i] = ok && d > 0.0 ? d * pow(rho, d - 1.0) : 0.0;
}

hipError_t launch_weights(const KParams& p, hipStream_t stream) {
    hipLaunchKernelGGL(k_weights, dim3((p.M * p.N + 255) / 256), dim3(256), 0, stream, p);
    return hipGetLastError();
}

hipError_t launch_forward(const KParams& p, hipStream_t stream, const Timing& tm, bool full) {
    if (p.T != 128 && p.T != 64 && p.T != 32 && p.T != 16) return hipErrorInvalidValue;
    if (full && p.T != 32 && p.T != 16) return hipErrorInvalidValue;
    hipError_t e = launch_weights(p, stream);
    if (e != hipSuccess) return e;
    if (tm.start && hipEventRecord(tm.start, stream) != hipSuccess) return hipErrorUnknown;
    const int nw = p.waves;
    if (full) e = p.T == 32 ? launch_fwd<32, 1, true>(p, stream) : launch_fwd<16, 1, true>(p, stream);
    else if (p.T == 128) e = launch_fwd128(p, stream);
    else if (p.T == 64) e = nw == 2 ? launch_fwd<64, 2>(p, stream) : nw == 8 ? launch_fwd<64, 8>(p, stream)
                                    : launch_fwd<64, kWaves64>(p, stream);
    else if (p.T == 32) e = nw == 1 ? launch_fwd<32, 1>(p, stream) : nw == 4 ? launch_fwd<32, 4>(p, stream)
                                    : launch_fwd<32, kWaves32>(p, stream);
    else e = nw == 2 ? launch_fwd<16, 2>(p, stream) : launch_fwd<16, kWaves16>(p, stream);
    if (e != hipSuccess) return e;
    if (tm.stop && hipEventRecord(tm.stop, stream) != hipSuccess) return hipErrorUnknown;
    return launch_synthesis(p, stream);
}

}  // namespace fofse
