// Adjoint (reverse-mode derivative) of the FOFSE forward pass, for gfx950.
//
// With the class u_nu of every iteration fixed (the selection record of a
// forward call), the forward pass is
//   w = a rho_hat^d (eqs. 4, 15);  R0 = DFT(w f), W = DFT(w), W0 = sum w (eqs. 7, 8)
//   s_nu = R_{nu-1}[u_nu],  c_nu = gamma s_nu / W0  (real part for a
//          self-conjugate class; eqs. 5, 14)
//   R_nu = R_{nu-1} - c_nu W[. - u_nu] - conj(c_nu) W[. + u_nu]   (eq. 3, DFT domain)
//   g = sum_nu mult_nu Re(c_nu phi_{u_nu}) on B                 (eqs. 1, 2)
// Summing the updates, s_nu = R0[u_nu] - sum_{mu<nu} (c_mu W[u_nu - u_mu] +
// conj(c_mu) W[u_nu + u_mu]): the coefficients solve a K x K lower-triangular
// recurrence whose entries are samples of W.  Because the record holds every
// c_nu, the reverse pass needs neither the residual spectra nor their
// recovery; it is the transposed recurrence:
//   cbar_nu   = mult Gbar[u_nu]           (Gbar = DFT of dL/dg on B)
//               - sum_{mu>nu} (sbar_mu conj(W[u_mu - u_nu]) + conj(sbar_mu) W[u_mu + u_nu])
//   sbar_nu   = gamma / W0 * cbar_nu      (Re of cbar for a self-conjugate class)
// and the gradients follow from sbar and cbar (complex adjoints are written
// zbar = dL/dRe z + j dL/dIm z):
//   dL/dgamma = sum_nu Re(cbar_nu conj(c_nu)) / gamma
//   dL/dW0    = -sum_nu Re(cbar_nu conj(c_nu)) / W0
//   Rbar0[k]  = sum_{nu: u_nu = k} sbar_nu,  (w f)bar = Re sum_k Rbar0[k] phi_k
//   dL/df     = w (w f)bar on A
//   dL/drho   = sum_x dw/drho [f (w f)bar + W0bar]
//               - sum_{mu<nu} Re(sbar_nu conj(c_mu D[u_nu - u_mu]) + sbar_nu conj(conj(c_mu) D[u_nu + u_mu]))
// with D = DFT(dw/drho): the derivative through W never forms the adjoint
// spectrum of W, it pairs each of its K(K-1) entries with D directly.
//
// One workgroup per block.  W and D come from one complex FFT of
// z = w + j dw/drho in LDS (separated by Hermitian symmetry at each read); the
// recurrence runs in panels of 64 iterations: one wavefront resolves a panel
// serially (lane = iteration, the finished adjoint is broadcast with
// readlane), then all waves apply the panel to the earlier iterations and
// accumulate the rho terms.  (w f)bar comes from one more 2-D FFT.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fofse_kernel.h"
#include "device_common.hpp"

namespace fofse {

namespace {

// grid index of frequency (k, l), natural order and FFT output order
template <int T>
__device__ __forceinline__ int zi(int k, int l) {
    return ((k & (T - 1)) * T) | (l & (T - 1));
}
template <int T>
__device__ __forceinline__ int zp(int k, int l) {
    return FftPlan<T>::perm(k & (T - 1)) * T + FftPlan<T>::perm(l & (T - 1));
}

template <int T>
struct Key {
    static constexpr int LOG2 = T == 64 ? 6 : 5;
    __device__ static int k(int key) { return (key >> LOG2) & (T - 1); }
    __device__ static int l(int key) { return key & (T - 1); }
    __device__ static bool pair(int k, int l) {
        return !(((k & (T / 2 - 1)) == 0) && ((l & (T / 2 - 1)) == 0));
    }
};

// W[k] = (Z[k] + conj Z[-k]) / 2 from Z = W + j D (FFT output order in LDS)
template <int T>
__device__ __forceinline__ double2 w_at(const double2* Z, int k, int l) {
    const double2 a = Z[zp<T>(k, l)], b = Z[zp<T>(-k, -l)];
    return make_double2(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));
}

// W[k] and D[k] = (Z[k] - conj Z[-k]) / (2j)
template <int T>
__device__ __forceinline__ void wd_at(const double2* Z, int k, int l, double2& W, double2& D) {
    const double2 a = Z[zp<T>(k, l)], b = Z[zp<T>(-k, -l)];
    W = make_double2(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));
    D = make_double2(0.5 * (a.y + b.y), 0.5 * (b.x - a.x));
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

}  // namespace

template <int T, int KMAX>
__global__ __launch_bounds__(256, 2) void fofse_bwd_kernel(BParams p) {
    constexpr int NT = 256;
    constexpr int CH = 256;                 // samples of B staged per pass
    using KY = Key<T>;
    __shared__ double2 buf[T * T];
    __shared__ double2 tw[T];
    __shared__ int keyL[KMAX];
    __shared__ double2 cL[KMAX];
    __shared__ double2 cbL[KMAX];
    __shared__ float gq[CH];
    __shared__ int mnq[CH];
    __shared__ double red[2][NT / 64];
    __shared__ int s_flags;

    const int tid = (int)__builtin_amdgcn_workitem_id_x();
    const int lane = tid & 63, wave = tid >> 6;
    const int b = (int)__builtin_amdgcn_workgroup_id_x();
    const int M = p.M, N = p.N, K = p.K, MN = M * N, nB = p.nB;
    const double rho = p.rho_gamma[0];
    const double gamma = p.rho_gamma[1];
    const bool params_ok = param_ok(rho) && param_ok(gamma);

    for (int i = tid; i < T; i += NT) tw[i] = p.twiddle[i];
    for (int i = tid; i < T * T; i += NT) buf[i] = make_double2(0.0, 0.0);
    const size_t rb = (size_t)b * K;
    for (int i = tid; i < K; i += NT) {
        keyL[i] = p.sel[rb + i];
        cL[i] = make_double2(p.coef[2 * (rb + i)], p.coef[2 * (rb + i) + 1]);
    }
    if (tid == 0) s_flags = params_ok ? 0 : FOFSE_BLOCK_BAD_PARAM;
    __syncthreads();

    // z = w + j dw/drho on the T x T grid, area at the origin (row m, column n)
    const size_t ab = (size_t)b * MN;
    for (int i = tid; i < MN; i += NT) {
        const int m = i / N, n = i - m * N;
        bool a = p.target[i] == 0;
        if (p.known) a = a && p.known[ab + i] != 0;
        double w = 0.0, dw = 0.0;
        if (a) {
            const float fv = p.areas[ab + i];
            if ((__float_as_uint(fv) & 0x7f800000u) == 0x7f800000u) {
                atomicOr(&s_flags, FOFSE_BLOCK_NONFINITE);
            } else {
                w = p.wtab[i];
                dw = p.dwtab[i];
            }
        }
        buf[m * T + n] = make_double2(w, dw);
    }
    __syncthreads();
    fft_stage_a<T, NT>(buf, tw, M, T, 1, tid);
    __syncthreads();
    fft_stage_b<T, NT>(buf, M, T, 1, tid);
    __syncthreads();
    fft_stage_a<T, NT>(buf, tw, T, 1, T, tid);
    __syncthreads();
    fft_stage_b<T, NT>(buf, T, 1, T, tid);
    __syncthreads();
    const double W0 = buf[0].x, dW0 = buf[0].y;
    int flags = s_flags;
    if (params_ok && !(W0 > 0.0)) flags |= FOFSE_BLOCK_NO_SUPPORT;
    if (flags != 0) {            // the forward output of such a block is 0
        if (p.grad_areas)
            for (int i = tid; i < MN; i += NT) p.grad_areas[ab + i] = 0.0f;
        if (tid == 0) {
            p.grad_block[2 * b] = 0.0;
            p.grad_block[2 * b + 1] = 0.0;
        }
        return;
    }
    const double gW = gamma / W0;

    // cbar0_nu = mult Gbar[u_nu], Gbar[k] = sum_B gbar[x] exp(-j 2 pi <k, x> / T)
    for (int nu0 = 0; nu0 < K; nu0 += NT) {
        const int nu = nu0 + tid;
        int k = 0, l = 0;
        if (nu < K) {
            const int key = keyL[nu];
            k = KY::k(key);
            l = KY::l(key);
        }
        double ar = 0.0, ai = 0.0;
        for (int q0 = 0; q0 < nB; q0 += CH) {
            const int cnt = min(CH, nB - q0);
            __syncthreads();
            for (int i = tid; i < cnt; i += NT) {
                const int flat = p.bpix[q0 + i];
                const int m = flat / N, n = flat - m * N;
                gq[i] = p.grad_out[(size_t)b * nB + q0 + i];
                mnq[i] = (m << 16) | n;
            }
            __syncthreads();
            for (int i = 0; i < cnt; ++i) {
                const int mn = mnq[i];
                const double2 t = tw[(k * (mn >> 16) + l * (mn & 0xFFFF)) & (T - 1)];
                const double g = (double)gq[i];
                ar = fma(g, t.x, ar);
                ai = fma(g, t.y, ai);
            }
        }
        if (nu < K)
            cbL[nu] = KY::pair(k, l) ? make_double2(2.0 * ar, 2.0 * ai) : make_double2(ar, 0.0);
    }
    __syncthreads();

    // transposed recurrence, panels of 64 iterations from the last
    double racc = 0.0;
    for (int pn = (K - 1) >> 6; pn >= 0; --pn) {
        const int base = pn << 6, cnt = min(64, K - base), hi = base + cnt;
        if (wave == 0) {
            const int nu = base + lane;
            const bool valid = lane < cnt;
            int ku = 0, lu = 0;
            bool pr = false;
            double2 cb = make_double2(0.0, 0.0);
            if (valid) {
                const int key = keyL[nu];
                ku = KY::k(key);
                lu = KY::l(key);
                pr = KY::pair(ku, lu);
                cb = cbL[nu];
            }
            for (int j = cnt - 1; j >= 0; --j) {
                const int keyj = keyL[base + j];
                const int kj = KY::k(keyj), lj = KY::l(keyj);
                const double cr = readlane_f64(cb.x, j);
                const double ci = KY::pair(kj, lj) ? readlane_f64(cb.y, j) : 0.0;
                if (lane == j) cb = make_double2(cr, ci);          // final adjoint of c_j
                const double sr = gW * cr, si = gW * ci;           // sbar_j
                if (lane < j) {
                    const double2 wd = w_at<T>(buf, kj - ku, lj - lu);
                    cb.x -= sr * wd.x + si * wd.y;                  // sbar conj(W[u_j - u_i])
                    cb.y -= si * wd.x - sr * wd.y;
                    if (pr) {
                        const double2 ws = w_at<T>(buf, kj + ku, lj + lu);
                        cb.x -= sr * ws.x + si * ws.y;              // conj(sbar) W[u_j + u_i]
                        cb.y -= sr * ws.y - si * ws.x;
                    }
                }
            }
            if (valid) cbL[nu] = cb;
        }
        __syncthreads();
        // the panel's sbar into the earlier iterations, and the rho terms of
        // every pair (mu < nu) with nu in this panel
        for (int mu = tid; mu < hi; mu += NT) {
            const int key = keyL[mu];
            const int ku = KY::k(key), lu = KY::l(key);
            const bool pr = KY::pair(ku, lu);
            const bool cross = mu < base;
            const double2 c = cL[mu];
            double ar = 0.0, ai = 0.0, rr = 0.0;
            for (int nu = max(base, mu + 1); nu < hi; ++nu) {
                const int key2 = keyL[nu];
                const int kn = KY::k(key2), ln = KY::l(key2);
                const double2 cbn = cbL[nu];
                const double sr = gW * cbn.x, si = gW * cbn.y;
                double2 Wd, Dd;
                wd_at<T>(buf, kn - ku, ln - lu, Wd, Dd);
                if (cross) {
                    ar -= sr * Wd.x + si * Wd.y;
                    ai -= si * Wd.x - sr * Wd.y;
                }
                {   // -Re(sbar conj(c D[u_nu - u_mu]))
                    const double qr = c.x * Dd.x - c.y * Dd.y, qi = c.x * Dd.y + c.y * Dd.x;
                    rr -= sr * qr + si * qi;
                }
                if (pr) {
                    double2 Ws, Ds;
                    wd_at<T>(buf, kn + ku, ln + lu, Ws, Ds);
                    if (cross) {
                        ar -= sr * Ws.x + si * Ws.y;
                        ai -= sr * Ws.y - si * Ws.x;
                    }
                    // -Re(sbar conj(conj(c) D[u_nu + u_mu]))
                    const double qr = c.x * Ds.x + c.y * Ds.y, qi = c.x * Ds.y - c.y * Ds.x;
                    rr -= sr * qr + si * qi;
                }
            }
            if (cross) {
                const double2 o = cbL[mu];
                cbL[mu] = make_double2(o.x + ar, o.y + ai);
            }
            racc += rr;
        }
        __syncthreads();
    }

    // sum_nu Re(cbar_nu conj(c_nu)): gives dL/dgamma and dL/dW0
    double tacc = 0.0;
    for (int nu = tid; nu < K; nu += NT) {
        const double2 cb = cbL[nu], c = cL[nu];
        tacc += cb.x * c.x + cb.y * c.y;
    }

    // Rbar0 on the grid (conjugated, so that the forward FFT gives
    // conj of sum_k Rbar0[k] exp(+j ...), whose real part is (w f)bar).
    // Repeated classes are summed in iteration order by their first occurrence.
    for (int i = tid; i < T * T; i += NT) buf[i] = make_double2(0.0, 0.0);
    __syncthreads();
    for (int nu = tid; nu < K; nu += NT) {
        const int key = keyL[nu];
        const int kk = zi<T>(KY::k(key), KY::l(key));
        bool first = true;
        for (int j = 0; j < nu; ++j)
            if (zi<T>(KY::k(keyL[j]), KY::l(keyL[j])) == kk) {
                first = false;
                break;
            }
        if (first) {
            double sr = 0.0, si = 0.0;
            for (int j = nu; j < K; ++j)
                if (zi<T>(KY::k(keyL[j]), KY::l(keyL[j])) == kk) {
                    sr += cbL[j].x;
                    si += cbL[j].y;
                }
            buf[kk] = make_double2(gW * sr, -gW * si);
        }
    }
    __syncthreads();
    fft_stage_a<T, NT>(buf, tw, T, T, 1, tid);
    __syncthreads();
    fft_stage_b<T, NT>(buf, T, T, 1, tid);
    __syncthreads();
    fft_stage_a<T, NT>(buf, tw, T, 1, T, tid);
    __syncthreads();
    fft_stage_b<T, NT>(buf, T, 1, T, tid);
    __syncthreads();

    // dL/df = w (w f)bar on A; rho term of R0 = DFT(w f)
    for (int i = tid; i < MN; i += NT) {
        const int m = i / N, n = i - m * N;
        bool a = p.target[i] == 0;
        if (p.known) a = a && p.known[ab + i] != 0;
        double gv = 0.0;
        if (a) {
            const double wfb = buf[FftPlan<T>::perm(m) * T + FftPlan<T>::perm(n)].x;
            gv = p.wtab[i] * wfb;
            racc += p.dwtab[i] * (double)p.areas[ab + i] * wfb;
        }
        if (p.grad_areas) p.grad_areas[ab + i] = (float)gv;
    }

    racc = wave_sum(racc);
    tacc = wave_sum(tacc);
    if (lane == 0) {
        red[0][wave] = racc;
        red[1][wave] = tacc;
    }
    __syncthreads();
    if (tid == 0) {
        double r = 0.0, t = 0.0;
#pragma unroll
        for (int w = 0; w < NT / 64; ++w) {
            r += red[0][w];
            t += red[1][w];
        }
        const double W0bar = -t / W0;
        p.grad_block[2 * b] = r + W0bar * dW0;       // W0 = sum w: dW0/drho = sum dw
        p.grad_block[2 * b + 1] = t / gamma;
    }
}

// Sum of the per-block gradients in a fixed order (deterministic).
__global__ __launch_bounds__(256) void k_bwd_sum(const double* blk, int n, double* out) {
    __shared__ double s[2][256];
    const int tid = (int)__builtin_amdgcn_workitem_id_x();
    double r = 0.0, t = 0.0;
    for (int i = tid; i < n; i += 256) {
        r += blk[2 * i];
        t += blk[2 * i + 1];
    }
    s[0][tid] = r;
    s[1][tid] = t;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (tid < st) {
            s[0][tid] += s[0][tid + st];
            s[1][tid] += s[1][tid + st];
        }
        __syncthreads();
    }
    if (tid == 0) {
        out[0] = s[0][0];
        out[1] = s[1][0];
    }
}

template <int T, int KMAX>
static hipError_t launch_bwd(const BParams& p, hipStream_t stream) {
    hipLaunchKernelGGL((fofse_bwd_kernel<T, KMAX>), dim3(p.n_blocks), dim3(256), 0, stream, p);
    return hipGetLastError();
}

hipError_t launch_backward(const KParams& wp, const BParams& p, double* d_sum, hipStream_t stream,
                           const Timing& tm) {
    if ((p.T != 64 && p.T != 32) || p.K > kBackwardMaxK) return hipErrorInvalidValue;
    hipError_t e = launch_weights(wp, stream);
    if (e != hipSuccess) return e;
    if (tm.start && hipEventRecord(tm.start, stream) != hipSuccess) return hipErrorUnknown;
    if (p.T == 64) e = p.K <= 256 ? launch_bwd<64, 256>(p, stream) : launch_bwd<64, kBackwardMaxK>(p, stream);
    else e = p.K <= 256 ? launch_bwd<32, 256>(p, stream) : launch_bwd<32, kBackwardMaxK>(p, stream);
    if (e != hipSuccess) return e;
    if (tm.stop && hipEventRecord(tm.stop, stream) != hipSuccess) return hipErrorUnknown;
    if (d_sum) {
        hipLaunchKernelGGL(k_bwd_sum, dim3(1), dim3(256), 0, stream, (const double*)p.grad_block,
                           p.n_blocks, d_sum);
        e = hipGetLastError();
    }
    return e;
}

}  // namespace fofse
