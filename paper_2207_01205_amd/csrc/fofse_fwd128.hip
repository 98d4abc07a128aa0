// FOFSE forward kernel for the 128 x 128 DFT (areas up to 64 x 64), gfx950.
//
// The iteration is that of the other kernels (Section 2: eq. 9 selection, eqs.
// 5 and 14 coefficient, eq. 3 carried to the DFT domain); what differs is the
// storage, because a 128 x 128 spectrum in FP64 (256 KB) exceeds the LDS:
//
//   * Placement: area row m -> grid column (index k), area column n -> grid row
//     (index l), as in the other kernels, so the representative half of the
//     conjugate classes is grid rows l = 0..64.
//   * Initial transforms (eqs. 7, 8): for x = w f (then x = w), a direct DFT
//     over n evaluated only for l = 0..64 (the real input makes the other rows
//     redundant), then 128-point FFTs over m for each of those 65 rows.  The
//     result, the row half of the spectrum, occupies 65 x 128 x 16 B = 133 KB.
//   * R (rows 0..64) lives in registers: 8 or 16 wavefronts share the rows,
//     every lane holds columns lane and lane + 64.
//   * W stays in LDS as its row half.  A read W[r][c] with r outside 0..64 is
//     conj(W[-r][-c]) (w is real); for every register slot the choice between
//     the direct and the mirrored read is uniform (it depends on the slot's row
//     and the selected u only); the conjugation flips the sign bit of the read's
//     imaginary part.
//   * After the transforms each wavefront puts its rows in natural column order,
//     so that neighbouring lanes read neighbouring entries of W.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fofse_kernel.h"
#include "device_common.hpp"
#include "iterate.hpp"

namespace fofse {

namespace {

constexpr int T128 = 128;
constexpr int H128 = 64;
constexpr int ROWS128 = H128 + 1;

template <int NW>
__host__ __device__ constexpr int row_begin128(int w) { return (w * ROWS128 + NW - 1) / NW; }

// A wave's rows of R, one register pair per slot: the first 16 slots in one
// vector, the rest in a second (no padding slot: a 17-row wave has no
// registers to spare).
template <int S>
struct RowRegs {
    static constexpr int CA = S > 16 ? 16 : S;
    static constexpr int CB = S > 16 ? S - 16 : 1;
    static_assert(S <= 32, "at most two chunks");
    typedef double va __attribute__((ext_vector_type(CA)));
    typedef double vb __attribute__((ext_vector_type(CB)));
    va re0, im0;
    vb re1, im1;
    __device__ __forceinline__ double gr(int s) const { return s < CA ? re0[s] : re1[s - CA]; }
    __device__ __forceinline__ double gi(int s) const { return s < CA ? im0[s] : im1[s - CA]; }
    __device__ __forceinline__ void set(int s, double a, double c) {
        if (s < CA) { re0[s] = a; im0[s] = c; } else { re1[s - CA] = a; im1[s - CA] = c; }
    }
    // (re, im) of slot s (uniform) in lane `lane` (uniform)
    __device__ __forceinline__ double2 fetch(int s, int lane) const {
        double a, c;
        if (S <= 16 || s < CA) { a = readlane_f64(re0[s], lane); c = readlane_f64(im0[s], lane); }
        else { a = readlane_f64(re1[s - CA], lane); c = readlane_f64(im1[s - CA], lane); }
        return make_double2(a, c);
    }
};

__device__ __forceinline__ int perm128(int k) { return FftPlan<T128>::perm(k & (T128 - 1)); }

__device__ __forceinline__ double neg_if(bool c, double x) { return c ? -x : x; }

template <int NW>
struct Shared128 {
    double2 spec[ROWS128 * T128];   // row half of a spectrum, natural column order
    double2 tw[T128];
    Xchg<NW> xchg[2];
    int flags;
};

// Spectrum rows l = 0..64 of x (area values from ``val``, transposed placement)
// into sh.spec: direct DFT over n for l <= 64, then 128-point FFTs over m.
// ``val(i)`` gives the value of area sample i = m * N + n (0 outside A).
template <int NT, class F>
__device__ __forceinline__ void row_half_spectrum(double2* spec, const double2* tw, int M, int N, int tid,
                                                  F val, int* asym = nullptr) {
    constexpr int NW = NT / 64;
    constexpr int NJ = (ROWS128 + NW - 1) / NW;             // output rows per thread
    double* xs = reinterpret_cast<double*>(spec);         // staging xs[n * 64 + m]
    for (int i = tid; i < 64 * 64; i += NT) xs[i] = 0.0;
    __syncthreads();
    for (int i = tid; i < M * N; i += NT) {
        const int m = i / N, n = i - m * N;
        xs[n * 64 + m] = val(i);
    }
    __syncthreads();
    if (asym) {     // is x symmetric about the area's centre?  (reads only)
        bool a = false;
        for (int i = tid; i < M * N; i += NT) {
            const int m = i / N, n = i - m * N;
            a = a || xs[(N - 1 - n) * 64 + (M - 1 - m)] != xs[n * 64 + m];
        }
        if (a) *asym = 1;
    }
    // X1[l][m] = sum_n x[m][n] exp(-j 2 pi l n / 128) for l = 0..64, in two
    // steps with n = 8 n1 + n2 (x[m][n] = 0 for n >= 64):
    //   Y[n2][k][m] = sum_n1 x[m][8 n1 + n2] exp(-j 2 pi k n1 / 16), k = l mod 16,
    //   a 16-point DFT of 8 samples (even k: DFT8 of x, odd k: DFT8 of x
    //   exp(-j 2 pi n1 / 16)), one (m, n2) per thread;
    //   X1[l][m] = sum_n2 exp(-j 2 pi l n2 / 128) Y[n2][l mod 16][m].
    // Summing over n directly read a twiddle per (l, n) for every lane of a
    // wave, and that broadcast traffic bounded the transform.
    {
        const int m1 = tid & 63, n2 = (tid >> 6) & 7;
        const bool act = tid < 512;
        double xv[8];
#pragma unroll
        for (int n1 = 0; n1 < 8; ++n1) xv[n1] = act ? xs[(8 * n1 + n2) * 64 + m1] : 0.0;
        __syncthreads();                                    // staging consumed
        if (act) {
            double2* Y = spec + n2 * 16 * 64 + m1;          // Y[(n2 16 + k) 64 + m]
            double2 y[8];
#pragma unroll
            for (int n1 = 0; n1 < 8; ++n1) y[n1] = make_double2(xv[n1], 0.0);
            dft8(y);
#pragma unroll
            for (int q = 0; q < 8; ++q) Y[(2 * q) * 64] = y[q];
#pragma unroll
            for (int n1 = 0; n1 < 8; ++n1) {
                const double2 w = tw[8 * n1];               // exp(-j 2 pi n1 / 16)
                y[n1] = make_double2(xv[n1] * w.x, xv[n1] * w.y);
            }
            dft8(y);
#pragma unroll
            for (int q = 0; q < 8; ++q) Y[(2 * q + 1) * 64] = y[q];
        }
        __syncthreads();
    }
    const int m = tid & 63, lg = tid >> 6;
    double2 acc[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) acc[j] = make_double2(0.0, 0.0);
#pragma unroll 1
    for (int n2 = 0; n2 < 8; ++n2) {
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            const int l = min(lg + NW * j, H128);         // rows beyond 64 are not stored
            const double2 t = tw[(l * n2) & (T128 - 1)];
            const double2 y = spec[(n2 * 16 + (l & 15)) * 64 + m];
            acc[j].x = fma(t.x, y.x, fma(-t.y, y.y, acc[j].x));
            acc[j].y = fma(t.x, y.y, fma(t.y, y.x, acc[j].y));
        }
    }
    __syncthreads();                                        // Y consumed
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        const int l = lg + NW * j;
        if (l <= H128) {
            spec[l * T128 + m] = acc[j];
            spec[l * T128 + 64 + m] = make_double2(0.0, 0.0);
        }
    }
    __syncthreads();
    fft_stage_a<T128, NT>(spec, tw, ROWS128, T128, 1, tid);
    __syncthreads();
    fft_stage_b<T128, NT>(spec, ROWS128, T128, 1, tid);
    __syncthreads();
    // FFT output order -> natural column order, one row per wavefront: all lanes
    // read the row before any lane writes it (a wavefront's LDS operations run
    // in program order), so no barrier is needed inside a row
    const int lane = tid & 63;
    for (int r = tid >> 6; r < ROWS128; r += NW) {
        double2* row = spec + r * T128;
        const double2 a = row[perm128(lane)], c = row[perm128(lane + 64)];
        row[lane] = a;
        row[lane + 64] = c;
    }
    __syncthreads();
}

// One wavefront's rows [k0, k0 + S) of the K iterations of one block; the NW
// wavefronts of the block exchange their candidates through ``xchg`` (two
// buffers) and meet at a workgroup barrier every iteration.  ``live`` = false
// runs the same barriers and writes nothing (a missing or flagged block that
// shares the workgroup with a live one).
template <int NW, int WI>
__device__ __forceinline__ void run_wave128(RowRegs<row_begin128<NW>(WI + 1) - row_begin128<NW>(WI)>& R0,
                                            RowRegs<row_begin128<NW>(WI + 1) - row_begin128<NW>(WI)>& R1,
                                            const double2* Wb, Xchg<NW>* xchg, const KParams& p, int b,
                                            int lane, double gW0, bool live = true) {
    constexpr int k0 = row_begin128<NW>(WI);
    constexpr int S = row_begin128<NW>(WI + 1) - k0;
    const int K = p.K;
    int u = 0, v = 0;
    double cr = 0.0, ci = 0.0;
    const int c0 = lane, c1 = lane + 64;
    // With eight or more waves per block, the block's maximum key is taken by
    // 64-bit LDS atomics into one of three slots (the first words of xchg[0]):
    // slot it % 3 collects iteration it, and slot (it + 1) % 3, last read
    // before the previous barrier, is cleared for the next iteration.  With
    // four waves the candidates are compared after the barrier.
    constexpr bool kAtomicMax = NW >= 8;
    unsigned long long* keys = reinterpret_cast<unsigned long long*>(&xchg[0].hi[0]);
    if constexpr (kAtomicMax) {
        if (WI == 0 && lane == 0) keys[0] = 0ull;
        __syncthreads();
    }
    int ks = 0;
    for (int it = 0; it < K; ++it) {
        // column indices of the four read forms for both columns
        const int dA0 = (c0 - v) & (T128 - 1), mA0 = (v - c0) & (T128 - 1);
        const int dB0 = (c0 + v) & (T128 - 1), mB0 = (-c0 - v) & (T128 - 1);
        const int dA1 = (c1 - v) & (T128 - 1), mA1 = (v - c1) & (T128 - 1);
        const int dB1 = (c1 + v) & (T128 - 1), mB1 = (-c1 - v) & (T128 - 1);
        // The reads of a slot depend only on its row and on (u, v): chunks of CH
        // slots, the reads of chunk q + 1 issued before chunk q is computed.
        constexpr int CH = 2;
        constexpr int NC = (S + CH - 1) / CH;
        double2 xa[2][CH][2], xb[2][CH][2];     // [buffer][slot of the chunk][column half]
        auto load = [&](int q, int bf) {
#pragma unroll
            for (int j = 0; j < CH; ++j) {
                const int s = q * CH + j;
                if (s < S) {
                    const int k = k0 + s;
                    // uniform rows, kept in scalar registers
                    const int rowA = __builtin_amdgcn_readfirstlane(k - u);
                    const int rowB = __builtin_amdgcn_readfirstlane(k + u);
                    const bool mirA = rowA < 0, mirB = rowB > H128;
                    const double2* pA = Wb + (mirA ? -rowA : rowA) * T128;
                    const double2* pB = Wb + (mirB ? T128 - rowB : rowB) * T128;
                    xa[bf][j][0] = pA[mirA ? mA0 : dA0];
                    xa[bf][j][1] = pA[mirA ? mA1 : dA1];
                    xb[bf][j][0] = pB[mirB ? mB0 : dB0];
                    xb[bf][j][1] = pB[mirB ? mB1 : dB1];
                }
            }
        };
        load(0, 0);
        double best = 0.0;
#pragma unroll
        for (int q = 0; q < NC; ++q) {
            if (q + 1 < NC) load(q + 1, (q + 1) & 1);
#pragma unroll
            for (int j = 0; j < CH; ++j) {
                const int s = q * CH + j;
                if (s >= S) break;
                const int k = k0 + s;
                // R -= c W1 + conj(c) W2 with W1 = xa or conj(xa), W2 = xb or conj(xb):
                // a mirrored read is conjugated by flipping the sign bit of its
                // imaginary part in place (uniform masks, one integer op per read)
                const uint32_t sgA = __builtin_amdgcn_readfirstlane(k - u) < 0 ? 0x80000000u : 0u;
                const uint32_t sgB = __builtin_amdgcn_readfirstlane(k + u) > H128 ? 0x80000000u : 0u;
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const double2 x1 = xa[q & 1][j][h], x2 = xb[q & 1][j][h];
                    const double y1 = __hiloint2double(__double2hiint(x1.y) ^ (int)sgA, __double2loint(x1.y));
                    const double y2 = __hiloint2double(__double2hiint(x2.y) ^ (int)sgB, __double2loint(x2.y));
                    double re = h ? R1.gr(s) : R0.gr(s), im = h ? R1.gi(s) : R0.gi(s);
                    const double sr = x1.x + x2.x, dr = x1.x - x2.x;
                    re = fma(-cr, sr, re);
                    re = fma(ci, y1, re);
                    re = fma(-ci, y2, re);
                    im = fma(-ci, dr, im);
                    im = fma(-cr, y1, im);
                    im = fma(-cr, y2, im);
                    if (h) R1.set(s, re, im); else R0.set(s, re, im);
                    // eq. 9 key: |R|^2, then column half (0 first), then smaller row
                    const double m2 = sq_add(im, re * re);
                    uint32_t lo = (__double2loint(m2) & 0xFFFFFF00u) | ((uint32_t)(1 - h) << 7) | (uint32_t)(127 - k);
                    int hi = __double2hiint(m2);
                    if (k == 0 || k == H128) {
                        // rows 0 and 64 represent columns 0..64 only
                        const bool ok = h == 0 || lane == 0;
                        hi = ok ? hi : 0;
                        lo = ok ? lo : 0u;
                    }
                    best = max_f64(best, __hiloint2double(hi, (int)lo));
                }
            }
            if constexpr (NC > 1) __builtin_amdgcn_sched_barrier(0);
        }
        // wavefront maximum (see run_wave): magnitude and column half, then
        // the smallest lane, then (inside the lane) the smallest row
        const uint32_t bhi = (uint32_t)__double2hiint(best), blo = (uint32_t)__double2loint(best);
        const uint32_t mhi = wave_max_u32(bhi);
        uint64_t hits = __ballot(bhi == mhi);
        int wl = __builtin_ctzll(hits);
        uint32_t mlo = (uint32_t)__builtin_amdgcn_readlane((int)blo, wl);
        hits &= hits - 1;
        while (hits) {
            const int ln = __builtin_ctzll(hits);
            hits &= hits - 1;
            const uint32_t l2 = (uint32_t)__builtin_amdgcn_readlane((int)blo, ln);
            if ((l2 & 0xFFFFFF80u) > (mlo & 0xFFFFFF80u)) { mlo = l2; wl = ln; }
        }
        mlo = (uint32_t)__builtin_amdgcn_readfirstlane((int)mlo);
        wl = __builtin_amdgcn_readfirstlane(wl);
        int wslot = (int)(127 - (mlo & 127u)) - k0;
        wslot = __builtin_amdgcn_readfirstlane(wslot < 0 ? 0 : (wslot >= S ? S - 1 : wslot));
        const bool whalf = ((mlo >> 7) & 1u) == 0u;
        // the winner's value, read from its column half only (a uniform branch)
        double2 wvh;
        if (whalf) wvh = R1.fetch(wslot, wl);
        else wvh = R0.fetch(wslot, wl);
        Xchg<NW>& x = xchg[it & 1];
        const uint32_t mkey = (mlo & 0xFFFFC000u) | (((mlo >> 7) & 1u) << 13) | ((uint32_t)(63 - wl) << 7) | (mlo & 127u);
        int bw = 0;
        uint32_t wlo;
        if constexpr (kAtomicMax) {
            const int kn = ks == 2 ? 0 : ks + 1;
            if (lane == 0) {
                atomicMax(&keys[ks], ((unsigned long long)mhi << 32) | mkey);
                x.val[WI] = wvh;
                if (WI == 0) keys[kn] = 0ull;
            }
            __syncthreads();
            wlo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)keys[ks]);
            ks = kn;
            // the wave holding the winner's row
            const int wrow = 127 - (int)(wlo & 127u);
#pragma unroll
            for (int w = 1; w < NW; ++w) bw += wrow >= row_begin128<NW>(w) ? 1 : 0;
        } else {
            if (lane == 0) {
                x.hi[WI] = mhi;
                x.lo[WI] = mkey;
                x.val[WI] = wvh;
            }
            __syncthreads();
            uint32_t chi[NW], clo[NW];
#pragma unroll
            for (int w = 0; w < NW; ++w) { chi[w] = x.hi[w]; clo[w] = x.lo[w]; }
            uint32_t whi = chi[0];
            wlo = clo[0];
#pragma unroll
            for (int w = 1; w < NW; ++w) {
                const bool gt = chi[w] > whi || (chi[w] == whi && clo[w] > wlo);
                bw = gt ? w : bw;
                whi = gt ? chi[w] : whi;
                wlo = gt ? clo[w] : wlo;
            }
            bw = __builtin_amdgcn_readfirstlane(bw);
            wlo = (uint32_t)__builtin_amdgcn_readfirstlane((int)wlo);
        }
        const double2 wv = x.val[bw];
        // selected class: grid row u (index l), grid column v (index k)
        u = 127 - (int)(wlo & 127u);
        u = u > H128 ? H128 : u;
        v = (63 - (int)((wlo >> 7) & 63u)) + (((wlo >> 13) & 1u) ? 0 : 64);
        const bool selfc = (u == 0 || u == H128) && (v == 0 || v == H128);
        const double cre = wv.x * gW0;
        const double cim = selfc ? 0.0 : wv.y * gW0;
        if (live && WI == 0 && lane == 0) {
            const size_t r = (size_t)b * K + it;
            p.sel[r] = v * T128 + u;
            p.coef[2 * r] = cre;
            p.coef[2 * r + 1] = cim;
        }
        // a self-conjugate class is applied as two half terms (W[k+u] = W[k-u])
        cr = selfc ? 0.5 * cre : cre;
        ci = cim;
    }
}

// ---------------------------------------------------------------------------
// point-symmetric w: the real-table iteration (as run_wave_sym for T <= 64)
// ---------------------------------------------------------------------------
//
// W[a][b] = P(a, b) V(a, b) with P(a, b) = exp(-j pi (a R0 + b C0) / 128) and V
// real (R0, C0: grid rows and columns of the area - 1), so with Rt = conj(P) R
// the update is Rt[k] -= ct V(k - u) + conj(ct) V(k + u), ct = gamma Rt[u] / W0.
// The table V is stored for rows -32 .. 96 (window row = a + 32), 128 columns,
// 8 bytes each (132 KB, in place of the complex row half).  A slot k >= 32 reads
// V(k - u) directly and k < 32 through V(u - k, v - l); k <= 32 reads V(k + u)
// directly and k > 32 through (-1)^R0 V(128 - k - u, -l - v): the form depends
// on the slot's row only.  Column wraps give per-lane signs, folded into the
// coefficients.  ht holds exp(-j pi q / 128), q < 256.
constexpr int Q128 = 32;
constexpr int VROWS128 = 3 * Q128 + 1 + Q128;     // rows -32 .. 96

// The V window from the row half of W (natural column order) in spec, in place.
// Pass 1 computes rows a = -32 and a = 32 .. 96, which read W rows 32 .. 64
// only, and writes a = 32 .. 96 (the bytes of W rows 32 .. 64); pass 2 computes
// a = -31 .. 31 from W rows 0 .. 31 and writes a = -32 .. 31.
template <int NT>
__device__ __forceinline__ void build_v128(double2* spec, const double2* ht, int R0, int C0, int tid) {
    double* vw = reinterpret_cast<double*>(spec);
    auto vval = [&](int a, int b) -> double {
        // W[a mod 128][b] from the row half; rows beyond 64 or below 0 by W[-k] = conj W[k]
        double2 w;
        if (a >= 0 && a <= H128) w = spec[a * T128 + b];
        else {
            const int r = a < 0 ? -a : T128 - a;
            const double2 x = spec[r * T128 + ((-b) & (T128 - 1))];
            w = make_double2(x.x, -x.y);
        }
        const double2 P = ht[(a * R0 + b * C0) & (2 * T128 - 1)];
        return P.x * w.x + P.y * w.y;             // Re(conj(P) W)
    };
    // pass 1: a = 32 .. 96 (65 rows) and a = -32 (kept for pass 2)
    constexpr int N1 = 65 * T128, E1 = (N1 + NT - 1) / NT;
    constexpr int E0 = (T128 + NT - 1) / NT;
    double v1[E1], v0[E0];
#pragma unroll
    for (int e = 0; e < E1; ++e) {
        const int idx = tid + e * NT;
        if (idx < N1) v1[e] = vval(32 + idx / T128, idx & (T128 - 1));
    }
#pragma unroll
    for (int e = 0; e < E0; ++e) {
        const int idx = tid + e * NT;
        if (idx < T128) v0[e] = vval(-Q128, idx);
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E1; ++e) {
        const int idx = tid + e * NT;
        if (idx < N1) vw[(32 + Q128) * T128 + idx] = v1[e];
    }
    __syncthreads();
    // pass 2: a = -31 .. 31 (63 rows), W rows 0 .. 31 are intact
    constexpr int N2 = 63 * T128, E2 = (N2 + NT - 1) / NT;
    double v2[E2];
#pragma unroll
    for (int e = 0; e < E2; ++e) {
        const int idx = tid + e * NT;
        if (idx < N2) v2[e] = vval(-31 + idx / T128, idx & (T128 - 1));
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E2; ++e) {
        const int idx = tid + e * NT;
        if (idx < N2) vw[T128 + idx] = v2[e];          // rows a = -31 .. 31 start at window row 1
    }
#pragma unroll
    for (int e = 0; e < E0; ++e) {
        const int idx = tid + e * NT;
        if (idx < T128) vw[idx] = v0[e];                // window row 0 = a = -32
    }
    __syncthreads();
}

template <int NW, int WI>
__device__ __forceinline__ void run_wave128_sym(RowRegs<row_begin128<NW>(WI + 1) - row_begin128<NW>(WI)>& R0,
                                                RowRegs<row_begin128<NW>(WI + 1) - row_begin128<NW>(WI)>& R1,
                                                const double* vw, const double2* ht, Xchg<NW>* xchg,
                                                const KParams& p, int b, int lane, double gW0, bool live) {
    constexpr int k0 = row_begin128<NW>(WI);
    constexpr int S = row_begin128<NW>(WI + 1) - k0;
    constexpr int Q = Q128;
    const int K = p.K;
    const int RR = p.N - 1, CC = p.M - 1;       // transposed placement
    const bool odd_r = (RR & 1) != 0, odd_c = (CC & 1) != 0;
    // reference slots of the four read forms (see rd below)
    constexpr int r1d = k0 > Q ? k0 : Q;                  // V1 direct: slots k >= Q
    constexpr int r1m = k0 + S - 1 < Q - 1 ? k0 + S - 1 : Q - 1;   // V1 mirrored: k < Q
    constexpr int r2d = k0;                               // V2 direct: k <= Q
    constexpr int r2m = k0 + S - 1;                       // V2 mirrored: k > Q
    int u = 0, v = 0;
    double ca = 0.0, cb = 0.0;
    // window rows: W1 direct a = k - u, mirrored u - k; W2 direct k + u,
    // mirrored 128 - k - u (window row = a + 32).  Each read form has one
    // base per column half at the wave's slot of lowest row (the smallest k
    // for a direct form, the largest for a mirrored one), so that every
    // slot reads at a compile-time offset above it.
    const double* bs1d[2], *bs1m[2], *bs2d[2], *bs2m[2];
    auto set_bases = [&](int uu, int vv) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int c = lane + 64 * h;
            bs1d[h] = vw + (r1d - uu + Q) * T128 + ((c - vv) & (T128 - 1));
            bs1m[h] = vw + (uu - r1m + Q) * T128 + ((vv - c) & (T128 - 1));
            bs2d[h] = vw + (r2d + uu + Q) * T128 + ((c + vv) & (T128 - 1));
            bs2m[h] = vw + (T128 - r2m - uu + Q) * T128 + ((-c - vv) & (T128 - 1));
        }
    };
    auto rd = [&](int k, int h, double& V1, double& V2) {
        V1 = k >= Q ? bs1d[h][(k - r1d) * T128] : bs1m[h][(r1m - k) * T128];
        V2 = k <= Q ? bs2d[h][(k - r2d) * T128] : bs2m[h][(r2m - k) * T128];
    };
    constexpr int CH = 2;
    constexpr int NC = (S + CH - 1) / CH;
    double xv[2][CH][2][2];                      // [buffer][slot][half][V1, V2]
    auto load = [&](int q, int bf) {
#pragma unroll
        for (int j = 0; j < CH; ++j) {
            const int s = q * CH + j;
            if (s < S) {
#pragma unroll
                for (int h = 0; h < 2; ++h) rd(k0 + s, h, xv[bf][j][h][0], xv[bf][j][h][1]);
            }
        }
    };
    set_bases(0, 0);
    load(0, 0);
    // the block's maximum key, taken by LDS atomics into one of three 64-bit
    // slots (the first words of xchg[0]): slot it % 3 collects iteration it,
    // and slot (it + 1) % 3, last read before the previous barrier, is cleared
    // for the next iteration
    unsigned long long* keys = reinterpret_cast<unsigned long long*>(&xchg[0].hi[0]);
    if (WI == 0 && lane == 0) keys[0] = 0ull;
    __syncthreads();
    int ks = 0;
    for (int it = 0; it < K; ++it) {
        // per column half h (column c = lane + 64 h): the signs of the wraps
        // of the four read forms
        double A1d[2], B1d[2], A1m[2], B1m[2], A2d[2], B2d[2], A2m[2], B2m[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int c = lane + 64 * h;
            const bool n1d = odd_c && c < v;
            const bool n1m = odd_c && c > v;
            const bool n2d = odd_c && c + v >= T128;
            const bool n2m = odd_r != (odd_c && c + v > 0 && c + v <= T128);
            A1d[h] = n1d ? ca : -ca; B1d[h] = n1d ? cb : -cb;
            A1m[h] = n1m ? ca : -ca; B1m[h] = n1m ? cb : -cb;
            A2d[h] = n2d ? ca : -ca; B2d[h] = n2d ? -cb : cb;
            A2m[h] = n2m ? ca : -ca; B2m[h] = n2m ? -cb : cb;
        }
        double best = 0.0;
#pragma unroll
        for (int q = 0; q < NC; ++q) {
            if (q + 1 < NC) load(q + 1, (q + 1) & 1);
#pragma unroll
            for (int j = 0; j < CH; ++j) {
                const int s = q * CH + j;
                if (s >= S) break;
                const int k = k0 + s;
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const double V1 = xv[q & 1][j][h][0], V2 = xv[q & 1][j][h][1];
                    const double a1 = k >= Q ? A1d[h] : A1m[h], b1 = k >= Q ? B1d[h] : B1m[h];
                    const double a2 = k <= Q ? A2d[h] : A2m[h], b2 = k <= Q ? B2d[h] : B2m[h];
                    double re = h ? R1.gr(s) : R0.gr(s), im = h ? R1.gi(s) : R0.gi(s);
                    re = fma(a1, V1, re);
                    re = fma(a2, V2, re);
                    im = fma(b1, V1, im);
                    im = fma(b2, V2, im);
                    if (h) R1.set(s, re, im); else R0.set(s, re, im);
                    // eq. 9 key: |R|^2, then column half (0 first), then smaller row
                    const double m2 = sq_add(im, re * re);
                    uint32_t lo = (__double2loint(m2) & 0xFFFFFF00u) | ((uint32_t)(1 - h) << 7) | (uint32_t)(127 - k);
                    int hi = __double2hiint(m2);
                    if (k == 0 || k == H128) {
                        // rows 0 and 64 represent columns 0..64 only
                        const bool ok = h == 0 || lane == 0;
                        hi = ok ? hi : 0;
                        lo = ok ? lo : 0u;
                    }
                    best = max_f64(best, __hiloint2double(hi, (int)lo));
                }
            }
            if constexpr (NC > 1) __builtin_amdgcn_sched_barrier(0);
        }
        // wavefront maximum (as run_wave128); the block's maximum over its
        // wavefronts by the atomic key slots above, each wave publishing its
        // winner's value in the exchange record
        const uint32_t bhi = (uint32_t)__double2hiint(best), blo = (uint32_t)__double2loint(best);
        const uint32_t mhi = wave_max_u32(bhi);
        uint64_t hits = __ballot(bhi == mhi);
        int wl = __builtin_ctzll(hits);
        uint32_t mlo = (uint32_t)__builtin_amdgcn_readlane((int)blo, wl);
        hits &= hits - 1;
        while (hits) {
            const int ln = __builtin_ctzll(hits);
            hits &= hits - 1;
            const uint32_t l2 = (uint32_t)__builtin_amdgcn_readlane((int)blo, ln);
            if ((l2 & 0xFFFFFF80u) > (mlo & 0xFFFFFF80u)) { mlo = l2; wl = ln; }
        }
        mlo = (uint32_t)__builtin_amdgcn_readfirstlane((int)mlo);
        wl = __builtin_amdgcn_readfirstlane(wl);
        int wslot = (int)(127 - (mlo & 127u)) - k0;
        wslot = __builtin_amdgcn_readfirstlane(wslot < 0 ? 0 : (wslot >= S ? S - 1 : wslot));
        const bool whalf = ((mlo >> 7) & 1u) == 0u;
        // the winner's value, read from its column half only (a uniform branch)
        double2 wvh;
        if (whalf) wvh = R1.fetch(wslot, wl);
        else wvh = R0.fetch(wslot, wl);
        Xchg<NW>& x = xchg[it & 1];
        const int kn = ks == 2 ? 0 : ks + 1;
        if (lane == 0) {
            const uint32_t lo = (mlo & 0xFFFFC000u) | (((mlo >> 7) & 1u) << 13) | ((uint32_t)(63 - wl) << 7) | (mlo & 127u);
            atomicMax(&keys[ks], ((unsigned long long)mhi << 32) | lo);
            x.val[WI] = wvh;
            if (WI == 0) keys[kn] = 0ull;
        }
        __syncthreads();
        const uint32_t wlo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)keys[ks]);
        ks = kn;
        // the wave holding the winner's row
        const int wrow = 127 - (int)(wlo & 127u);
        int bw = 0;
#pragma unroll
        for (int w = 1; w < NW; ++w) bw += wrow >= row_begin128<NW>(w) ? 1 : 0;
        const double2 wv = x.val[bw];            // Rt[u]
        u = 127 - (int)(wlo & 127u);
        u = u > H128 ? H128 : u;
        v = (63 - (int)((wlo >> 7) & 63u)) + (((wlo >> 13) & 1u) ? 0 : 64);
        // the next iteration's first table reads go out ahead of the coefficient
        set_bases(u, v);
        load(0, 0);
        // eqs. 5, 14 in the rotated frame: ct = gamma Rt[u] / W0, c = ct P(u);
        // a self-conjugate class keeps Re c
        const bool selfc = (u == 0 || u == H128) && (v == 0 || v == H128);
        const double2 P = ht[(u * RR + v * CC) & (2 * T128 - 1)];
        double ctr = wv.x * gW0, cti = wv.y * gW0;
        double cre = ctr * P.x - cti * P.y;
        double cim = ctr * P.y + cti * P.x;
        if (selfc) {
            cim = 0.0;
            ctr = cre * P.x;
            cti = -cre * P.y;
        }
        if (live && WI == 0 && lane == 0) {
            const size_t r = (size_t)b * K + it;
            p.sel[r] = v * T128 + u;
            p.coef[2 * r] = cre;
            p.coef[2 * r + 1] = cim;
        }
        // a self-conjugate class is applied as two half terms
        ca = selfc ? 0.5 * ctr : ctr;
        cb = selfc ? 0.5 * cti : cti;
    }
}

// One wavefront: take its rows of R from the LDS spectrum into registers,
// join the W transform (all waves run the same barriers), then iterate.
template <int NW, int WI, class FW>
__device__ __forceinline__ void wave128(Shared128<NW>& sh, const KParams& p, int b, int tid, int lane,
                                        double gamma, int flags_pre, FW wval) {
    constexpr int k0 = row_begin128<NW>(WI);
    constexpr int S = row_begin128<NW>(WI + 1) - k0;
    RowRegs<S> R0, R1;
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const double2* row = sh.spec + (k0 + s) * T128;
        const double2 a = row[lane], c = row[lane + 64];
        R0.set(s, a.x, a.y);
        R1.set(s, c.x, c.y);
    }
    __syncthreads();                                        // every wave has its rows
    row_half_spectrum<NW * 64>(sh.spec, sh.tw, p.M, p.N, tid, wval);   // W, row half, in LDS
    const double W0 = sh.spec[0].x;
    int flags = sh.flags | flags_pre;
    if (flags == 0 && !(W0 > 0.0)) flags = FOFSE_BLOCK_NO_SUPPORT;
    if (flags == 0) run_wave128<NW, WI>(R0, R1, sh.spec, sh.xchg, p, b, lane, gamma / W0);
}

// dispatch wave w to its specialised instance
template <int NW, int WI, class FW>
__device__ __forceinline__ void wave128_dispatch(int w, Shared128<NW>& sh, const KParams& p, int b, int tid,
                                                 int lane, double gamma, int flags_pre, FW wval) {
    if constexpr (WI < NW) {
        if (w == WI) wave128<NW, WI>(sh, p, b, tid, lane, gamma, flags_pre, wval);
        else wave128_dispatch<NW, WI + 1>(w, sh, p, b, tid, lane, gamma, flags_pre, wval);
    }
}

}  // namespace

template <int NW>
__global__ __launch_bounds__(NW * 64, 1) void fofse_fwd128_kernel(KParams p) {
    constexpr int NT = NW * 64;
    __shared__ Shared128<NW> sh;
    const int tid = (int)__builtin_amdgcn_workitem_id_x();
    const int lane = tid & 63, wave = tid >> 6;
    const int b = (int)__builtin_amdgcn_workgroup_id_x();
    const int M = p.M, N = p.N, K = p.K;
    const double rho = p.rho_gamma[0], gamma = p.rho_gamma[1];
    const bool params_ok = param_ok(rho) && param_ok(gamma);
    for (int i = tid; i < T128; i += NT) sh.tw[i] = p.twiddle[i];
    if (tid == 0) sh.flags = params_ok ? 0 : FOFSE_BLOCK_BAD_PARAM;
    __syncthreads();
    const size_t ab = (size_t)b * M * N;
    auto support = [&](int i) -> bool {
        bool a = p.target[i] == 0;
        if (p.known) a = a && p.known[ab + i] != 0;
        return a;
    };
    // eqs. 4, 7, 8: R from w f (a non-finite known sample flags the block)
    row_half_spectrum<NT>(sh.spec, sh.tw, M, N, tid, [&](int i) -> double {
        if (!support(i)) return 0.0;
        const uint32_t fb = sample_bits(p.areas, ab + i);
        if (nonfinite_bits(fb)) {
            atomicOr(&sh.flags, FOFSE_BLOCK_NONFINITE);
            return 0.0;
        }
        return p.wtab[i] * (double)__uint_as_float(fb);
    });
    const int flags_pre = sh.flags;
    auto wval = [&](int i) -> double { return support(i) ? p.wtab[i] : 0.0; };
    wave128_dispatch<NW, 0>(wave, sh, p, b, tid, lane, gamma, flags_pre, wval);
    // flags are final after the W transform (all waves passed its barriers)
    int flags = params_ok ? sh.flags : FOFSE_BLOCK_BAD_PARAM;   // out-of-range parameters: that flag alone
    const double W0 = sh.spec[0].x;
    if (flags == 0 && !(W0 > 0.0)) flags = FOFSE_BLOCK_NO_SUPPORT;
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
// grouped T = 128: two blocks of one support mask per workgroup share the row
// half of W in LDS (eqs. 4 and 15 depend on the mask only); each block has
// kWaves128G wavefronts, so a compute unit iterates two blocks at once
// ---------------------------------------------------------------------------

namespace {

constexpr int kBlocks128G = 2;
constexpr int kWaves128G = 4;

struct Shared128G {
    double2 spec[ROWS128 * T128];       // row half of a spectrum, or the V window of a symmetric w
    double2 tw[T128];
    double2 ht[2 * T128];               // exp(-j pi q / 128), q < 256
    Xchg<kWaves128G> xchg[kBlocks128G][2];
    int flags[kBlocks128G];
    int asym;                           // the item's w is not point-symmetric
    int next;                           // next work item of the workgroup (queue)
};
static_assert(VROWS128 * T128 * sizeof(double) <= ROWS128 * T128 * sizeof(double2), "V window fits the row half");
static_assert(2 * sizeof(Xchg<kBlocks128G * kWaves128G>) <= sizeof(Shared128G::xchg), "eight-wave records fit");

// The exchange records of block slot jb: its own pair, or, with eight waves
// on one block, both slots' pairs as one pair of eight-wave records.
template <int NW>
__device__ __forceinline__ Xchg<NW>* xchg_of(Shared128G& sh, int jb) {
    if constexpr (NW == kWaves128G) return sh.xchg[jb];
    else return reinterpret_cast<Xchg<NW>*>(&sh.xchg[0][0]);
}

// One work item as seen by wave WI of block slot jb, NW waves per block: four
// for an item of two blocks, all eight (jb = 0) for an item of one block.
// Every wave of the workgroup runs the same sequence of barriers.
template <int NW, int WI>
__device__ __forceinline__ void item128(Shared128G& sh, const KParams& p, const GroupArgs& g, int item, int tid,
                                        int lane, int jb, bool params_ok, double gamma) {
    static_assert(NW == kWaves128G || NW == kBlocks128G * kWaves128G, "four waves per block, or all eight");
    constexpr int NT = kBlocks128G * kWaves128G * 64;
    constexpr int k0 = row_begin128<NW>(WI);
    constexpr int S = row_begin128<NW>(WI + 1) - k0;
    const int M = p.M, N = p.N, MN = M * N, K = p.K;
    int nblk, b0, b1;
    if (g.direct) {
        nblk = min(kBlocks128G, p.n_blocks - item * kBlocks128G);
        b0 = item * kBlocks128G;
        b1 = b0 + 1;
    } else {
        nblk = g.item_n[item];
        b0 = g.item_blk[(size_t)item * kGroup];
        b1 = g.item_blk[(size_t)item * kGroup + 1];
    }
    const size_t rep = (size_t)b0 * MN;          // every block of the item has this mask
    const bool present = jb < nblk;
    const int bj = present ? (jb == 0 ? b0 : b1) : 0;
    auto support = [&](int i) -> bool {
        bool a = p.target[i] == 0;
        if (p.known) a = a && p.known[rep + i] != 0;
        return a;
    };
    // the thread index as an opaque per-item value: keeps the compiler from
    // hoisting every per-thread index of the item's transforms out of the item
    // loop (they would be spilled for the whole kernel and reloaded per item)
    asm volatile("" : "+v"(tid), "+v"(lane));
    __syncthreads();                              // previous item done with LDS
    if (tid < kBlocks128G) sh.flags[tid] = params_ok ? 0 : FOFSE_BLOCK_BAD_PARAM;
    if (tid == 0) sh.asym = 0;

    // eqs. 4, 7, 8: R of each block by its own transform; its waves take their rows
    RowRegs<S> R0, R1;
#pragma unroll
    for (int s = 0; s < S; ++s) {
        R0.set(s, 0.0, 0.0);
        R1.set(s, 0.0, 0.0);
    }
    for (int j = 0; j < kBlocks128G; ++j) {
        if (j >= nblk) break;                     // uniform over the workgroup
        const size_t ab = (size_t)(j == 0 ? b0 : b1) * MN;
        row_half_spectrum<NT>(sh.spec, sh.tw, M, N, tid, [&](int i) -> double {
            if (!support(i)) return 0.0;
            const uint32_t fb = sample_bits(p.areas, ab + i);
            if (nonfinite_bits(fb)) {
                atomicOr(&sh.flags[j], FOFSE_BLOCK_NONFINITE);
                return 0.0;
            }
            return p.wtab[i] * (double)__uint_as_float(fb);
        });
        if (jb == j) {
#pragma unroll
            for (int s = 0; s < S; ++s) {
                const double2* row = sh.spec + (k0 + s) * T128;
                const double2 a = row[lane], c = row[lane + 64];
                R0.set(s, a.x, a.y);
                R1.set(s, c.x, c.y);
            }
        }
        __syncthreads();                          // rows taken before the next transform
    }
    row_half_spectrum<NT>(sh.spec, sh.tw, M, N, tid,
                          [&](int i) -> double { return support(i) ? p.wtab[i] : 0.0; }, &sh.asym);
    const double W0 = sh.spec[0].x;
    int flags = params_ok ? sh.flags[jb] : FOFSE_BLOCK_BAD_PARAM;   // out-of-range parameters: that flag alone
    if (flags == 0 && !(W0 > 0.0)) flags = FOFSE_BLOCK_NO_SUPPORT;
    const bool live = present && flags == 0;
    const bool sym = sh.asym == 0;                // uniform over the workgroup
    if (sym) {
        build_v128<NT>(sh.spec, sh.ht, N - 1, M - 1, tid);
        // Rt = conj(P) R on this wave's slots, both column halves
#pragma unroll
        for (int s = 0; s < S; ++s) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const double2 P = sh.ht[((k0 + s) * (N - 1) + (lane + 64 * h) * (M - 1)) & (2 * T128 - 1)];
                const double re = h ? R1.gr(s) : R0.gr(s), im = h ? R1.gi(s) : R0.gi(s);
                const double nr = re * P.x + im * P.y, ni = im * P.x - re * P.y;
                if (h) R1.set(s, nr, ni); else R0.set(s, nr, ni);
            }
        }
        run_wave128_sym<NW, WI>(R0, R1, reinterpret_cast<const double*>(sh.spec), sh.ht, xchg_of<NW>(sh, jb), p, bj,
                                lane, live ? gamma / W0 : 0.0, live);
    } else {
        run_wave128<NW, WI>(R0, R1, sh.spec, xchg_of<NW>(sh, jb), p, bj, lane, live ? gamma / W0 : 0.0, live);
    }
    if (present && !live) {                       // empty record: the synthesised model is 0
        for (int it = WI * 64 + lane; it < K; it += NW * 64) {
            p.sel[(size_t)bj * K + it] = 0;
            p.coef[2 * ((size_t)bj * K + it)] = 0.0;
            p.coef[2 * ((size_t)bj * K + it) + 1] = 0.0;
        }
    }
    if (present && p.status && WI == 0 && lane == 0) p.status[bj] = flags;
}

}  // namespace

// Clears the list of lone items and its queue counter before the grouped
// T = 128 launches.  The grouping's counters are g.counts[0] (grouped items),
// [1] (all items) and [2] (the first launch's queue); [3] counts the listed
// lone items and [4] is the second launch's queue (the workspace holds twelve).
__global__ void k_fwd128_lone_clear(GroupArgs g) {
    if (__builtin_amdgcn_workitem_id_x() == 0) {
        g.counts[3] = 0;
        g.counts[4] = 0;
    }
}

// LONE = false: the work items of two blocks, four waves per block.  An item
// of one block (a mask no other block has, or the last of an odd class) is
// appended to a list in g.cls (free once the grouping has filled the items)
// and left to the LONE = true launch, which runs each listed item on all
// eight waves; the row partition does not change the arithmetic of any class.
// With every block of one mask (no grouping) the last item of an odd count
// stays in the first launch.
template <bool LONE>
__global__ __launch_bounds__(kBlocks128G * kWaves128G * 64, 1) void fofse_fwd128_group_kernel(KParams p,
                                                                                               GroupArgs g) {
    constexpr int NT = kBlocks128G * kWaves128G * 64;
    __shared__ Shared128G sh;
    const int tid = (int)__builtin_amdgcn_workitem_id_x();
    const int lane = tid & 63, wave = tid >> 6;
    // wave WI of a block holds rows row_begin128(WI)..: 17, 16, 16, 16.  The
    // second block's row ranges are rotated by one wave so that the two
    // 17-row waves do not share a SIMD (the waves of a workgroup are spread
    // over the SIMDs in turn; the barrier waits for the busiest SIMD)
    const int jb = wave / kWaves128G, wi = (wave + jb) % kWaves128G;
    const double rho = p.rho_gamma[0], gamma = p.rho_gamma[1];
    const bool params_ok = param_ok(rho) && param_ok(gamma);
    for (int i = tid; i < T128; i += NT) sh.tw[i] = p.twiddle[i];
    for (int i = tid; i < 2 * T128; i += NT) sh.ht[i] = p.htw[i];
    // work items: contiguous ranges when every block has the same support
    // (every item costs the same), else a queue, since point-symmetric items
    // run a cheaper iteration (the counter zeroed by the grouping; the next
    // index is fetched while the current item runs)
    static_assert(kWaves128G == 4, "one instance per wave of a block");
    if constexpr (LONE) {
        const int n_lone = g.counts[3];
        if (n_lone == 0) return;                 // uniform: no barrier is left waiting
        if (tid == 0) sh.next = atomicAdd(&g.counts[4], 1);
        __syncthreads();
        int li = sh.next;
        while (li < n_lone) {
            int nxt = 0;
            if (tid == 0) nxt = atomicAdd(&g.counts[4], 1);
            const int item = g.cls[li];
            constexpr int W8 = kBlocks128G * kWaves128G;
            if (wave == 0) item128<W8, 0>(sh, p, g, item, tid, lane, 0, params_ok, gamma);
            else if (wave == 1) item128<W8, 1>(sh, p, g, item, tid, lane, 0, params_ok, gamma);
            else if (wave == 2) item128<W8, 2>(sh, p, g, item, tid, lane, 0, params_ok, gamma);
            else if (wave == 3) item128<W8, 3>(sh, p, g, item, tid, lane, 0, params_ok, gamma);
            else if (wave == 4) item128<W8, 4>(sh, p, g, item, tid, lane, 0, params_ok, gamma);
            else if (wave == 5) item128<W8, 5>(sh, p, g, item, tid, lane, 0, params_ok, gamma);
            else if (wave == 6) item128<W8, 6>(sh, p, g, item, tid, lane, 0, params_ok, gamma);
            else item128<W8, 7>(sh, p, g, item, tid, lane, 0, params_ok, gamma);
            if (tid == 0) sh.next = nxt;        // every read of the last index preceded the item's barriers
            __syncthreads();
            li = sh.next;
        }
        return;
    }
    // work items: contiguous ranges when every block has the same support
    // (every item costs the same), else a queue, since point-symmetric items
    // run a cheaper iteration (the counter zeroed by the grouping; the next
    // index is fetched while the current item runs)
    const int n_items = g.direct ? (p.n_blocks + kBlocks128G - 1) / kBlocks128G : g.counts[1];
    const int per = (n_items + g.n_wg - 1) / g.n_wg;
    const int i0 = (int)__builtin_amdgcn_workgroup_id_x() * per;
    const int i1 = g.direct ? min(n_items, i0 + per) : n_items;
    int item = i0;
    if (!g.direct) {
        if (tid == 0) sh.next = atomicAdd(&g.counts[2], 1);
        __syncthreads();
        item = sh.next;
    }
    while (item < i1) {
        int nxt = 0;
        if (!g.direct && tid == 0) nxt = atomicAdd(&g.counts[2], 1);
        if (!g.direct && g.item_n[item] == 1) {
            if (tid == 0) g.cls[atomicAdd(&g.counts[3], 1)] = item;
            __syncthreads();                     // every thread has read the index before it is replaced
        } else {
            constexpr int W4 = kWaves128G;
            if (wi == 0) item128<W4, 0>(sh, p, g, item, tid, lane, jb, params_ok, gamma);
            else if (wi == 1) item128<W4, 1>(sh, p, g, item, tid, lane, jb, params_ok, gamma);
            else if (wi == 2) item128<W4, 2>(sh, p, g, item, tid, lane, jb, params_ok, gamma);
            else item128<W4, 3>(sh, p, g, item, tid, lane, jb, params_ok, gamma);
        }
        if (g.direct) {
            ++item;
        } else {
            if (tid == 0) sh.next = nxt;        // every read of the last index preceded the item's barriers
            __syncthreads();
            item = sh.next;
        }
    }
}

hipError_t launch_grouped128(const KParams& p, const GroupArgs& g, int n_cu, hipStream_t stream,
                             const Timing& tm) {
    if (p.T != 128 || p.M > 64 || p.N > 64) return hipErrorInvalidValue;
    hipError_t e = launch_weights(p, stream);
    if (e != hipSuccess) return e;
    GroupArgs ga = g;
    static_assert(kBlocks128G == 2, "item size 2 = 1 << 1");
    ga.gsize = kBlocks128G;
    ga.gshift = 1;
    if (!g.direct) {
        e = launch_grouping(ga, p.n_blocks, stream);
        if (e != hipSuccess) return e;
    }
    const int max_items = g.direct ? (p.n_blocks + kBlocks128G - 1) / kBlocks128G : p.n_blocks;
    int grid = n_cu;
    if (grid > max_items) grid = max_items;
    ga.n_wg = grid;
    if (!g.direct) {
        hipLaunchKernelGGL(k_fwd128_lone_clear, dim3(1), dim3(64), 0, stream, ga);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (tm.start && hipEventRecord(tm.start, stream) != hipSuccess) return hipErrorUnknown;
    hipLaunchKernelGGL(fofse_fwd128_group_kernel<false>, dim3(grid), dim3(kBlocks128G * kWaves128G * 64), 0,
                       stream, p, ga);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (!g.direct) {
        hipLaunchKernelGGL(fofse_fwd128_group_kernel<true>, dim3(grid), dim3(kBlocks128G * kWaves128G * 64), 0,
                           stream, p, ga);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (tm.stop && hipEventRecord(tm.stop, stream) != hipSuccess) return hipErrorUnknown;
    return launch_synthesis(p, stream);
}

hipError_t launch_fwd128(const KParams& p, hipStream_t stream) {
    if (p.waves == 16)
        hipLaunchKernelGGL(fofse_fwd128_kernel<16>, dim3(p.n_blocks), dim3(16 * 64), 0, stream, p);
    else
        hipLaunchKernelGGL(fofse_fwd128_kernel<8>, dim3(p.n_blocks), dim3(8 * 64), 0, stream, p);
    return hipGetLastError();
}

}  // namespace fofse
