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
//      the model is accumulated directly on the missing area (eqs. 1, 2).
//
// No MFMA: the update is a shifted rank-2 update, not a contraction.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fofse_kernel.h"

namespace fofse {

// ---------------------------------------------------------------------------
// small complex helpers (double2 = re, im)
// ---------------------------------------------------------------------------

__device__ __forceinline__ double2 c_add(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 c_sub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 c_mul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 c_mulmj(double2 a) { return make_double2(a.y, -a.x); }  // -j * a

// Forward DFTs of length 2, 4, 8 (kernel exp(-j 2 pi n k / R)), in place.
__device__ __forceinline__ void dft2(double2* x) {
    double2 a = x[0], b = x[1];
    x[0] = c_add(a, b);
    x[1] = c_sub(a, b);
}

__device__ __forceinline__ void dft4(double2* x) {
    double2 a = c_add(x[0], x[2]), b = c_sub(x[0], x[2]);
    double2 c = c_add(x[1], x[3]), d = c_mulmj(c_sub(x[1], x[3]));
    x[0] = c_add(a, c);
    x[2] = c_sub(a, c);
    x[1] = c_add(b, d);
    x[3] = c_sub(b, d);
}

__device__ __forceinline__ void dft8(double2* x) {
    double2 e[4] = {x[0], x[2], x[4], x[6]};
    double2 o[4] = {x[1], x[3], x[5], x[7]};
    dft4(e);
    dft4(o);
    const double r = 0.70710678118654752440084436210485;   // 1/sqrt(2)
    // twiddles exp(-j pi k / 4), k = 0..3
    double2 t1 = make_double2(r * (o[1].x + o[1].y), r * (o[1].y - o[1].x));
    double2 t2 = c_mulmj(o[2]);
    double2 t3 = make_double2(r * (o[3].y - o[3].x), -r * (o[3].x + o[3].y));
    x[0] = c_add(e[0], o[0]);
    x[4] = c_sub(e[0], o[0]);
    x[1] = c_add(e[1], t1);
    x[5] = c_sub(e[1], t1);
    x[2] = c_add(e[2], t2);
    x[6] = c_sub(e[2], t2);
    x[3] = c_add(e[3], t3);
    x[7] = c_sub(e[3], t3);
}

template <int R>
__device__ __forceinline__ void dft(double2* x) {
    if constexpr (R == 2) dft2(x);
    else if constexpr (R == 4) dft4(x);
    else dft8(x);
}

// ---------------------------------------------------------------------------
// T-point FFT along lines of a T x T LDS grid, as R1 x 8 (four-step):
// n = 8 n1 + n2, k = k1 + R1 k2.  Stage A: per (line, n2) a length-R1 DFT over
// n1, then twiddle exp(-j 2 pi n2 k1 / T), stored in place at 8 k1 + n2.
// Stage B: per (line, k1) a length-8 DFT over n2, X[k1 + R1 k2] stored in place
// at 8 k1 + k2.  The output of a line is therefore at position perm(k).
// ---------------------------------------------------------------------------

template <int T>
struct FftPlan {
    static constexpr int R1 = T / 8;
    __host__ __device__ static constexpr int perm(int k) { return 8 * (k % R1) + k / R1; }
};

template <int T, int NT>
__device__ __forceinline__ void fft_stage_a(double2* buf, const double2* tw, int nlines,
                                            int line_stride, int elem_stride, int tid) {
    constexpr int R1 = FftPlan<T>::R1;
    for (int task = tid; task < nlines * 8; task += NT) {
        const int line = task >> 3, n2 = task & 7;
        double2* base = buf + line * line_stride;
        double2 x[R1];
#pragma unroll
        for (int n1 = 0; n1 < R1; ++n1) x[n1] = base[(8 * n1 + n2) * elem_stride];
        dft<R1>(x);
#pragma unroll
        for (int k1 = 0; k1 < R1; ++k1) {
            double2 v = k1 ? c_mul(x[k1], tw[(n2 * k1) & (T - 1)]) : x[k1];
            base[(8 * k1 + n2) * elem_stride] = v;
        }
    }
}

template <int T, int NT>
__device__ __forceinline__ void fft_stage_b(double2* buf, int nlines, int line_stride,
                                            int elem_stride, int tid) {
    constexpr int R1 = FftPlan<T>::R1;
    for (int task = tid; task < nlines * R1; task += NT) {
        const int line = task / R1, k1 = task - line * R1;
        double2* base = buf + line * line_stride + 8 * k1 * elem_stride;
        double2 x[8];
#pragma unroll
        for (int n2 = 0; n2 < 8; ++n2) x[n2] = base[n2 * elem_stride];
        dft8(x);
#pragma unroll
        for (int k2 = 0; k2 < 8; ++k2) base[k2 * elem_stride] = x[k2];
    }
}

// ---------------------------------------------------------------------------
// wavefront helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ double readlane_f64(double v, int lane) {
    int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

// Maximum of an unsigned value over the 64 lanes (DPP within rows of 16, then
// row broadcasts); the result is uniform.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, ROW_MASK, 0xF, false);
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
    v = max(v, dpp_u32<0xB1, 0xF>(v));    // quad_perm [1,0,3,2]
    v = max(v, dpp_u32<0x4E, 0xF>(v));    // quad_perm [2,3,0,1]
    v = max(v, dpp_u32<0x141, 0xF>(v));   // row_half_mirror
    v = max(v, dpp_u32<0x140, 0xF>(v));   // row_mirror
    v = max(v, dpp_u32<0x142, 0xA>(v));   // row_bcast:15 into rows 1 and 3
    v = max(v, dpp_u32<0x143, 0xC>(v));   // row_bcast:31 into rows 2 and 3
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

// Candidate of one wave: selection key (see below) and the value R[u].
struct Cand {
    uint32_t hi, lo;
    double re, im;
};

// ---------------------------------------------------------------------------
// the per-wave iteration loop
// ---------------------------------------------------------------------------

template <int T, int NW>
struct Layout {
    static constexpr int H = T / 2;
    static constexpr int Q = T / 4;
    static constexpr int NROWS = H + 1;
    static constexpr int WROWS = T + 1;               // window rows -Q .. 3Q
    static constexpr int NT = NW * 64;
    // grid rows [begin(w), begin(w+1)) live in wave w
    __host__ __device__ static constexpr int begin(int w) { return (w * NROWS + NW - 1) / NW; }
    static constexpr int SMAX = begin(1) - begin(0);
};

// Row bookkeeping of wave WI: its rows and, for each of the four read forms,
// the reference row whose window offset is zero (smallest row for a direct
// form, largest for a mirrored one, so every per-slot offset is >= 0).
template <int T, int NW, int WI>
struct WaveRows {
    using L = Layout<T, NW>;
    static constexpr int k0 = L::begin(WI);
    static constexpr int S = L::begin(WI + 1) - k0;
    static constexpr int k1 = k0 + S - 1;
    static constexpr int Q = L::Q, H = L::H;
    static constexpr int r1d = (k1 >= Q) ? (k0 > Q ? k0 : Q) : Q;
    static constexpr int r1m = (k0 < Q) ? (k1 < Q - 1 ? k1 : Q - 1) : 0;
    static constexpr int r2d = (k0 <= Q) ? k0 : 0;
    static constexpr int r2m = (k1 > Q) ? k1 : H;
};

// Selection key of a bin: the IEEE bits of |R|^2 with the low 12 mantissa bits
// replaced by (63 - column) * 64 + (63 - row).  As doubles, keys order by
// magnitude first (the 12 bits change |R|^2 by < 2^-40 relative) and, between
// equal magnitudes, put the smaller class key column*T + row first -- the
// oracle's tie rule.  Unused bins get key 0.
template <int T, int NW, int WI, int PIX>
__device__ __forceinline__ void run_wave(
        double __attribute__((ext_vector_type(WaveRows<T, NW, WI>::S))) & Rre,
        double __attribute__((ext_vector_type(WaveRows<T, NW, WI>::S))) & Rim,
        const double2* win, const double2* tw, Cand (*xchg)[NW], const KParams& p, int b,
        int lane, double gW0, const int* pix_m, const int* pix_n, double* gacc, int npix_t) {
    using L = Layout<T, NW>;
    using WR = WaveRows<T, NW, WI>;
    constexpr int S = WR::S;
    constexpr int H = L::H;
    constexpr int Q = L::Q;
    const int K = p.K;
    const bool lane_ok = lane < T;
    const bool lane_edge_ok = lane <= H;   // rows 0, T/2: columns 0..T/2 represent the classes
    const uint32_t lane_bits = (uint32_t)(63 - lane) << 6;
    int u = 0, v = 0;
    double ca = 0.0, cb = 0.0;

    for (int it = 0; it < K; ++it) {
        if (it > 0) {
            const int l = lane;
            const int cA = (l - v) & (T - 1), cB = (v - l) & (T - 1);
            const int cC = (l + v) & (T - 1), cD = (-l - v) & (T - 1);
            const double2* b1d = win + (WR::r1d - u + Q) * T + cA;
            const double2* b1m = win + (u - WR::r1m + Q) * T + cB;
            const double2* b2d = win + (WR::r2d + u + Q) * T + cC;
            const double2* b2m = win + (T - WR::r2m - u + Q) * T + cD;
#pragma unroll
            for (int s = 0; s < S; ++s) {
                const int k = WR::k0 + s;
                double2 x1, x2;
                if (k >= Q) x1 = b1d[(k - WR::r1d) * T];
                else        x1 = b1m[(WR::r1m - k) * T];
                if (k <= Q) x2 = b2d[(k - WR::r2d) * T];
                else        x2 = b2m[(WR::r2m - k) * T];
                // R -= c W1 + conj(c) W2 with W1 = x1 or conj(x1), W2 = x2 or conj(x2)
                double re = Rre[s], im = Rim[s];
                const double sre = x1.x + x2.x;
                const double dre = x1.x - x2.x;
                if (k < Q) {            // W1 = conj(x1), W2 = x2
                    const double sim = x1.y + x2.y, dim = x2.y - x1.y;
                    re = fma(-ca, sre, re); re = fma(-cb, sim, re);
                    im = fma(-ca, dim, im); im = fma(-cb, dre, im);
                } else if (k == Q) {    // W1 = x1, W2 = x2
                    const double sim = x1.y + x2.y, dim = x1.y - x2.y;
                    re = fma(-ca, sre, re); re = fma(cb, dim, re);
                    im = fma(-ca, sim, im); im = fma(-cb, dre, im);
                } else {                // W1 = x1, W2 = conj(x2)
                    const double sim = x1.y + x2.y, dim = x1.y - x2.y;
                    re = fma(-ca, sre, re); re = fma(cb, sim, re);
                    im = fma(-ca, dim, im); im = fma(-cb, dre, im);
                }
                Rre[s] = re;
                Rim[s] = im;
            }
        }
        // eq. 9: largest |R| over this lane's classes, ties to the smallest key
        double best = 0.0;
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int k = WR::k0 + s;
            const double m2 = fma(Rim[s], Rim[s], Rre[s] * Rre[s]);
            const uint32_t lo = (__double2loint(m2) & 0xFFFFF000u) | (lane_bits | (uint32_t)(63 - k));
            double key = __hiloint2double(__double2hiint(m2), (int)lo);
            bool ok = lane_ok;
            if (k == 0 || k == H) ok = ok && lane_edge_ok;
            if (!ok) key = 0.0;
            best = fmax(best, key);
        }
        // wavefront maximum of the keys: high words by DPP, low words among ties
        const uint32_t bhi = (uint32_t)__double2hiint(best), blo = (uint32_t)__double2loint(best);
        const uint32_t mhi = wave_max_u32(bhi);
        uint64_t hits = __ballot(bhi == mhi);
        int wl = __builtin_ctzll(hits);
        uint32_t mlo = (uint32_t)__builtin_amdgcn_readlane((int)blo, wl);
        hits &= hits - 1;
        while (hits) {                       // equal high words in several lanes (rare)
            const int ln = __builtin_ctzll(hits);
            hits &= hits - 1;
            const uint32_t l2 = (uint32_t)__builtin_amdgcn_readlane((int)blo, ln);
            if (l2 > mlo) { mlo = l2; wl = ln; }
        }
        mlo = (uint32_t)__builtin_amdgcn_readfirstlane((int)mlo);
        wl = __builtin_amdgcn_readfirstlane(wl);
        // every wave owns at least one valid bin and valid keys have non-zero
        // low bits, so the winner is a bin of this wave; the clamp only guards
        // the register index
        int wslot = __builtin_amdgcn_readfirstlane((int)(63 - (mlo & 63u)) - WR::k0);
        wslot = wslot < 0 ? 0 : (wslot >= S ? S - 1 : wslot);
        const double wre = readlane_f64(Rre[wslot], wl);
        const double wim = readlane_f64(Rim[wslot], wl);
        Cand wc;
        if constexpr (NW > 1) {
            if (lane == 0) xchg[it & 1][WI] = Cand{mhi, mlo, wre, wim};
            __syncthreads();
            wc = xchg[it & 1][0];
#pragma unroll
            for (int w = 1; w < NW; ++w) {
                const Cand c = xchg[it & 1][w];
                if (c.hi > wc.hi || (c.hi == wc.hi && c.lo > wc.lo)) wc = c;
            }
        } else {
            wc = Cand{mhi, mlo, wre, wim};
        }
        // selected bin: grid row u (the class index l), grid column v (index k)
        u = 63 - (int)(wc.lo & 63u);
        v = (63 - (int)((wc.lo >> 6) & 63u)) & (T - 1);
        u = u > H ? H : u;
        // eqs. 5 and 14: c = gamma R[u] / W0; a self-conjugate class keeps Re c
        const bool selfc = (u == 0 || u == H) && (v == 0 || v == H);
        const double cre = wc.re * gW0;
        const double cim = selfc ? 0.0 : wc.im * gW0;
        if (WI == 0 && lane == 0) {
            const size_t r = (size_t)b * K + it;
            if (p.sel) p.sel[r] = v * T + u;
            if (p.coef) { p.coef[2 * r] = cre; p.coef[2 * r + 1] = cim; }
        }
        // a self-conjugate class is applied as two half terms (W[k+u] = W[k-u])
        ca = selfc ? 0.5 * cre : cre;
        cb = cim;
        // eqs. 1, 2: accumulate 2 Re(c phi) on the pixels of B owned here
#pragma unroll
        for (int j = 0; j < PIX; ++j) {
            if (PIX == 1 || j < npix_t) {
                const double2 t = tw[(v * pix_m[j] + u * pix_n[j]) & (T - 1)];
                gacc[j] = fma(2.0 * ca, t.x, fma(2.0 * cb, t.y, gacc[j]));
            }
        }
    }
}

// ---------------------------------------------------------------------------
// kernel
// ---------------------------------------------------------------------------

// R of this wave's rows from the transform Z = W + jR sitting in LDS in the
// FFT's output order, then the residual iteration.  Contains the two barriers
// that turn the LDS grid into the W window (all waves reach them).
template <int T, int NW, int WI, int PIX, int WPT>
__device__ __forceinline__ void wave_body(double2* win, const double2* tw, Cand (*xchg)[NW],
                                          const KParams& p, int b, int tid, int lane,
                                          const double2* wv, double gW0, int flags_pre,
                                          int* s_flags, const int* pix_m, const int* pix_n,
                                          double* gacc, int npix_t) {
    using L = Layout<T, NW>;
    using WR = WaveRows<T, NW, WI>;
    constexpr int S = WR::S;
    constexpr int NT = L::NT;
    constexpr int WROWS = L::WROWS;
    typedef double dvec __attribute__((ext_vector_type(S)));
    dvec Rre, Rim;
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const int k = WR::k0 + s;
        Rre[s] = 0.0;
        Rim[s] = 0.0;
        if (lane < T) {
            const double2 a = win[FftPlan<T>::perm(k) * T + FftPlan<T>::perm(lane)];
            const double2 c = win[FftPlan<T>::perm((-k) & (T - 1)) * T + FftPlan<T>::perm((-lane) & (T - 1))];
            Rre[s] = 0.5 * (a.y + c.y);
            Rim[s] = 0.5 * (c.x - a.x);
        }
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
        run_wave<T, NW, WI, PIX>(Rre, Rim, win, tw, xchg, p, b, lane, gW0, pix_m, pix_n, gacc, npix_t);
}

template <int T, int NW, int PIX>
__global__ __launch_bounds__(NW * 64, 2) void fofse_fwd_kernel(KParams p) {
    using L = Layout<T, NW>;
    constexpr int NT = L::NT;
    constexpr int Q = L::Q;
    constexpr int WROWS = L::WROWS;
    constexpr int WPT = (WROWS * T + NT - 1) / NT;    // window entries per thread
    __shared__ double2 win[WROWS * T];
    __shared__ double2 tw[T];
    __shared__ Cand xchg[2][NW];
    __shared__ int s_flags;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int b = blockIdx.x;
    const int M = p.M, N = p.N, K = p.K;
    const double rho = p.rho_gamma[0];
    const double gamma = p.rho_gamma[1];

    for (int i = tid; i < T; i += NT) tw[i] = p.twiddle[i];
    for (int i = tid; i < T * T; i += NT) win[i] = make_double2(0.0, 0.0);
    if (tid == 0) s_flags = (rho > 0.0 && rho <= 1.0 && gamma > 0.0 && gamma <= 1.0) ? 0 : FOFSE_BLOCK_BAD_PARAM;
    __syncthreads();

    // eqs. 4, 15: w = rho_hat^dist on A;  z = w + j w f, placed transposed
    const double cm = 0.5 * (M - 1), cn = 0.5 * (N - 1);
    const size_t area_base = (size_t)b * M * N;
    for (int i = tid; i < M * N; i += NT) {
        const int m = i / N, n = i - m * N;
        bool a = p.target[i] == 0;
        if (p.known) a = a && (p.known[area_base + i] != 0);
        double w = 0.0, wf = 0.0;
        if (a) {
            const float fv = p.areas[area_base + i];
            if (!isfinite(fv)) {
                atomicOr(&s_flags, FOFSE_BLOCK_NONFINITE);
            } else {
                const double dm = m - cm, dn = n - cn;
                w = pow(rho, sqrt(dm * dm + dn * dn));
                wf = w * (double)fv;
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
    const int flags_pre = (W0 > 0.0) ? 0 : FOFSE_BLOCK_NO_SUPPORT;
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

    // pixels of B owned by this thread
    int pix_m[PIX], pix_n[PIX];
    double gacc[PIX];
    int npix_t = 0;
#pragma unroll
    for (int j = 0; j < PIX; ++j) {
        const int q = tid + j * NT;
        pix_m[j] = 0;
        pix_n[j] = 0;
        gacc[j] = 0.0;
        if (q < p.nB) {
            const int flat = p.bpix[q];
            pix_m[j] = flat / N;
            pix_n[j] = flat - pix_m[j] * N;
            npix_t = j + 1;
        }
    }

    if (wave == 0) wave_body<T, NW, 0, PIX, WPT>(win, tw, xchg, p, b, tid, lane, wv, gW0, flags_pre, &s_flags, pix_m, pix_n, gacc, npix_t);
    if constexpr (NW > 1) if (wave == 1) wave_body<T, NW, 1, PIX, WPT>(win, tw, xchg, p, b, tid, lane, wv, gW0, flags_pre, &s_flags, pix_m, pix_n, gacc, npix_t);
    if constexpr (NW > 2) if (wave == 2) wave_body<T, NW, 2, PIX, WPT>(win, tw, xchg, p, b, tid, lane, wv, gW0, flags_pre, &s_flags, pix_m, pix_n, gacc, npix_t);
    if constexpr (NW > 3) if (wave == 3) wave_body<T, NW, 3, PIX, WPT>(win, tw, xchg, p, b, tid, lane, wv, gW0, flags_pre, &s_flags, pix_m, pix_n, gacc, npix_t);

    const int flags = s_flags | flags_pre;
    if (flags != 0 && tid == 0) {
        for (int it = 0; it < K; ++it) {
            if (p.sel) p.sel[(size_t)b * K + it] = 0;
            if (p.coef) { p.coef[2 * ((size_t)b * K + it)] = 0.0; p.coef[2 * ((size_t)b * K + it) + 1] = 0.0; }
        }
    }
#pragma unroll
    for (int j = 0; j < PIX; ++j) {
        if (j < npix_t) p.out[(size_t)b * p.nB + tid + j * NT] = (float)gacc[j];
    }
    if (p.status && tid == 0) p.status[b] = flags;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

template <int T, int NW, int PIX>
static hipError_t launch_fwd(const KParams& p, hipStream_t stream) {
    hipLaunchKernelGGL((fofse_fwd_kernel<T, NW, PIX>), dim3(p.n_blocks), dim3(NW * 64), 0, stream, p);
    return hipGetLastError();
}

int max_target_samples(int T) {
    if (T == 64) return 4 * kWaves64 * 64;
    if (T == 32) return 4 * kWaves32 * 64;
    return 0;
}

hipError_t launch_forward(const KParams& p, hipStream_t stream) {
    if (p.T == 64) {
        if (p.nB <= kWaves64 * 64) return launch_fwd<64, kWaves64, 1>(p, stream);
        return launch_fwd<64, kWaves64, 4>(p, stream);
    }
    if (p.T == 32) {
        if (p.nB <= kWaves32 * 64) return launch_fwd<32, kWaves32, 1>(p, stream);
        return launch_fwd<32, kWaves32, 4>(p, stream);
    }
    return hipErrorInvalidValue;
}

}  // namespace fofse
