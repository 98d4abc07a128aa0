// The FOFSE iteration for one block whose grid rows 0..T/2 are spread over NW
// wavefronts (lane = grid column, register slot = grid row), with W in an LDS
// window; shared by the per-block and the grouped kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_common.hpp"
#include "fofse_kernel.h"

namespace fofse {

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
// Residual spectrum of S register slots (re, im per slot) held as chunks of at
// most 16 doubles, so that a slot chosen at run time (uniform) can be read with
// GPU register indexing.
template <int S>
struct RegSpec {
    static constexpr int NCH = (S + 15) / 16;
    static constexpr int CS = (S + NCH - 1) / NCH;
    typedef double chunk __attribute__((ext_vector_type(CS)));
    chunk re[NCH], im[NCH];
    __device__ __forceinline__ double gr(int s) const { return re[s / CS][s % CS]; }
    __device__ __forceinline__ double gi(int s) const { return im[s / CS][s % CS]; }
    __device__ __forceinline__ void set(int s, double a, double c) { re[s / CS][s % CS] = a; im[s / CS][s % CS] = c; }
    // (re, im) of slot s (uniform) in lane `lane` (uniform)
    __device__ __forceinline__ double2 fetch(int s, int lane) const {
        const int ch = s / CS, ix = s - ch * CS;
        double a = 0.0, c = 0.0;
#pragma unroll
        for (int q = 0; q < NCH; ++q)
            if (q == ch) { a = readlane_f64(re[q][ix], lane); c = readlane_f64(im[q][ix], lane); }
        return make_double2(a, c);
    }
};

// Sum over every bin l of the block's full T x T spectrum of R_l W[u - l]: the
// convolution (R (*) W)[u] of the full orthogonality deficiency compensation
// (eqs. 10-13 with the DFT basis: sum_l p_l Khat_{u,l} = (p (*) W)[u] / W0).
// For a wavefront that holds a whole block (rows 0..T/2, lane = column): a
// stored row k in 1..T/2-1 stands for itself and for its conjugate row T - k
// (R_{-l} = conj(R_l), W[u + l] read as in the update), rows 0 and T/2 are
// stored whole and count once.  The window reads are those of the update.
template <int T, int WI>
__device__ __forceinline__ double2 conv_at(const RegSpec<WaveRows<T, 1, WI>::S>& R, const double2* win,
                                           int u, int v, int lane) {
    using L = Layout<T, 1>;
    using WR = WaveRows<T, 1, WI>;
    constexpr int S = WR::S;
    constexpr int H = L::H;
    constexpr int Q = L::Q;
    const int l = lane;
    const int cA = (l - v) & (T - 1), cB = (v - l) & (T - 1);
    const int cC = (l + v) & (T - 1), cD = (-l - v) & (T - 1);
    const double2* b1d = win + (WR::r1d - u + Q) * T + cA;
    const double2* b1m = win + (u - WR::r1m + Q) * T + cB;
    const double2* b2d = win + (WR::r2d + u + Q) * T + cC;
    const double2* b2m = win + (T - WR::r2m - u + Q) * T + cD;
    double sr = 0.0, si = 0.0;
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const int k = WR::k0 + s;
        const double2 x1 = (k >= Q) ? b1d[(k - WR::r1d) * T] : b1m[(WR::r1m - k) * T];
        const double2 x2 = (k <= Q) ? b2d[(k - WR::r2d) * T] : b2m[(WR::r2m - k) * T];
        // W1 = W[k - u], W2 = W[k + u] (a mirrored read is the conjugate)
        const double w1r = x1.x, w1i = k < Q ? -x1.y : x1.y;
        const double w2r = x2.x, w2i = k > Q ? -x2.y : x2.y;
        const double rr = R.gr(s), ri = R.gi(s);
        sr = fma(rr, w1r, sr);            // R conj(W1)
        sr = fma(ri, w1i, sr);
        si = fma(ri, w1r, si);
        si = fma(-rr, w1i, si);
        if (k != 0 && k != H) {           // conj(R) W2 for the conjugate row
            sr = fma(rr, w2r, sr);
            sr = fma(ri, w2i, sr);
            si = fma(rr, w2i, si);
            si = fma(-ri, w2r, si);
        }
    }
    if (!(lane < T)) sr = si = 0.0;
    return make_double2(wave_sum_f64(sr), wave_sum_f64(si));
}

// One wave's share of the K iterations of one block.  The selection record
// (class key and coefficient of every iteration) goes to p.sel / p.coef; the
// model on B is synthesised from it by the synthesis kernel.  ``live`` = false runs the
// same barriers without writing (a wave of a missing or flagged block in a
// workgroup whose waves synchronise every iteration).
//
// FULL = false: the constant compensation of eq. 14, c = gamma R[u] / W0
// (gW0 = gamma / W0).  FULL = true (one wavefront per block): the full
// compensation of eqs. 10-13, c = gamma_u p_u = R[u]^2 / (R (*) W)[u], 0 when
// either factor is 0; gW0 is unused.
template <int T, int NW, int WI, bool FULL = false>
__device__ __forceinline__ void run_wave(RegSpec<WaveRows<T, NW, WI>::S>& R,
        const double2* win, Xchg<NW>* xchg, const KParams& p, int b, int lane, double gW0,
        bool live = true) {
    static_assert(!FULL || NW == 1, "the full compensation is built for one wavefront per block");
    using L = Layout<T, NW>;
    using WR = WaveRows<T, NW, WI>;
    constexpr int S = WR::S;
    constexpr int H = L::H;
    constexpr int Q = L::Q;
    const int K = p.K;
    const bool lane_ok = lane < T;
    const bool edge_ok = lane_ok && lane <= H;   // rows 0 and T/2: columns 0..T/2 represent
    int u = 0, v = 0;
    double ca = 0.0, cb = 0.0;

    for (int it = 0; it < K; ++it) {
        // R -= c W[k-u] + conj(c) W[k+u] for every slot, then the slot's key.
        // Iteration 0 runs with c = 0, which leaves R unchanged.  The window reads
        // go in chunks of CH slots; the reads of chunk q + 1 are issued before
        // chunk q is computed (all at once when the wave has few rows).
        const int l = lane;
        const int cA = (l - v) & (T - 1), cB = (v - l) & (T - 1);
        const int cC = (l + v) & (T - 1), cD = (-l - v) & (T - 1);
        const double2* b1d = win + (WR::r1d - u + Q) * T + cA;
        const double2* b1m = win + (u - WR::r1m + Q) * T + cB;
        const double2* b2d = win + (WR::r2d + u + Q) * T + cC;
        const double2* b2m = win + (T - WR::r2m - u + Q) * T + cD;
        constexpr int CH = S <= 9 ? S : 2;
        constexpr int NC = (S + CH - 1) / CH;
        double2 x1c[CH], x2c[CH], x1n[CH], x2n[CH];
#pragma unroll
        for (int j = 0; j < CH; ++j) {
            const int k = WR::k0 + j;
            if (j < S) {
                x1c[j] = (k >= Q) ? b1d[(k - WR::r1d) * T] : b1m[(WR::r1m - k) * T];
                x2c[j] = (k <= Q) ? b2d[(k - WR::r2d) * T] : b2m[(WR::r2m - k) * T];
            }
        }
        double best = 0.0;
#pragma unroll
        for (int q = 0; q < NC; ++q) {
#pragma unroll
            for (int j = 0; j < CH; ++j) {
                const int s = (q + 1) * CH + j;
                const int k = WR::k0 + s;
                if (q + 1 < NC && s < S) {
                    x1n[j] = (k >= Q) ? b1d[(k - WR::r1d) * T] : b1m[(WR::r1m - k) * T];
                    x2n[j] = (k <= Q) ? b2d[(k - WR::r2d) * T] : b2m[(WR::r2m - k) * T];
                }
            }
#pragma unroll
            for (int j = 0; j < CH; ++j) {
                const int s = q * CH + j;
                if (s >= S) break;
                const int k = WR::k0 + s;
                const double2 x1 = x1c[j], x2 = x2c[j];
                // W1 = x1 or conj(x1), W2 = x2 or conj(x2) (mirrored reads)
                double re = R.gr(s), im = R.gi(s);
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
                R.set(s, re, im);
                // eq. 9: largest |R| over this lane's classes, ties to the smallest row
                const double m2 = sq_add(im, re * re);
                uint32_t lo = (__double2loint(m2) & 0xFFFFFFC0u) | (uint32_t)(63 - k);
                int hi = __double2hiint(m2);
                if (k == 0 || k == H) { hi = edge_ok ? hi : 0; lo = edge_ok ? lo : 0u; }
                else if (T < 64)      { hi = lane_ok ? hi : 0; lo = lane_ok ? lo : 0u; }
                best = max_f64(best, __hiloint2double(hi, (int)lo));
            }
#pragma unroll
            for (int j = 0; j < CH; ++j) { x1c[j] = x1n[j]; x2c[j] = x2n[j]; }
            if constexpr (NC > 1) __builtin_amdgcn_sched_barrier(0);
        }
        // wavefront maximum: high words by DPP; among lanes with equal high words
        // the larger magnitude bits of the low word, then the smallest lane
        // (column) -- together with the per-lane row bits this is the order of
        // the class key column * T + row
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
            if ((l2 & 0xFFFFFFC0u) > (mlo & 0xFFFFFFC0u)) { mlo = l2; wl = ln; }
        }
        mlo = (uint32_t)__builtin_amdgcn_readfirstlane((int)mlo);
        wl = __builtin_amdgcn_readfirstlane(wl);
        // every wave owns at least one valid bin and valid keys have non-zero
        // low bits, so the winner is a bin of this wave; the clamp only guards
        // the register index
        int wslot = (int)(63 - (mlo & 63u)) - WR::k0;
        wslot = __builtin_amdgcn_readfirstlane(wslot < 0 ? 0 : (wslot >= S ? S - 1 : wslot));
        const double2 wrv = R.fetch(wslot, wl);
        const double wre = wrv.x, wim = wrv.y;
        double2 wv;
        uint32_t whi, wlo;
        if constexpr (NW > 1) {
            Xchg<NW>& x = xchg[it & 1];
            if (lane == 0) {
                x.hi[WI] = mhi;
                // magnitude bits, then (63 - column) and (63 - row) as tie bits
                x.lo[WI] = (mlo & 0xFFFFF000u) | ((uint32_t)(63 - wl) << 6) | (mlo & 63u);
                x.val[WI] = make_double2(wre, wim);
            }
            __syncthreads();
            // the candidates of all waves in one broadcast read
            uint32_t chi[NW], clo[NW];
#pragma unroll
            for (int w = 0; w < NW; ++w) { chi[w] = x.hi[w]; clo[w] = x.lo[w]; }
            int bw = 0;
            whi = chi[0];
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
            wv = x.val[bw];
        } else {
            wlo = (mlo & 0xFFFFF000u) | ((uint32_t)(63 - wl) << 6) | (mlo & 63u);
            wv = make_double2(wre, wim);
        }
        // selected bin: grid row u (the class index l), grid column v (index k)
        u = 63 - (int)(wlo & 63u);
        v = (63 - (int)((wlo >> 6) & 63u)) & (T - 1);
        u = u > H ? H : u;
        // eqs. 5 and 14: c = gamma R[u] / W0; a self-conjugate class keeps Re c
        const bool selfc = (u == 0 || u == H) && (v == 0 || v == H);
        double cre, cim;
        if constexpr (FULL) {
            // eqs. 10-13: c = R[u]^2 / (R (*) W)[u]
            const double2 cv = conv_at<T, WI>(R, win, u, v, lane);
            const double den = cv.x * cv.x + cv.y * cv.y;
            const double nr = wv.x * wv.x - wv.y * wv.y, ni = 2.0 * wv.x * wv.y;
            const bool ok = den > 0.0 && (wv.x != 0.0 || wv.y != 0.0);
            cre = ok ? (nr * cv.x + ni * cv.y) / den : 0.0;
            cim = ok && !selfc ? (ni * cv.x - nr * cv.y) / den : 0.0;
        } else {
            cre = wv.x * gW0;
            cim = selfc ? 0.0 : wv.y * gW0;
        }
        if (live && WI == 0 && lane == 0) {
            const size_t r = (size_t)b * K + it;
            p.sel[r] = v * T + u;
            p.coef[2 * r] = cre;
            p.coef[2 * r + 1] = cim;
        }
        // a self-conjugate class is applied as two half terms (W[k+u] = W[k-u])
        ca = selfc ? 0.5 * cre : cre;
        cb = cim;
    }
}


// ---------------------------------------------------------------------------
// the iteration for a point-symmetric weighting function (one wavefront per
// block)
// ---------------------------------------------------------------------------
//
// When w is symmetric about the area's centre, w[R0 - r][C0 - c] = w[r][c] on
// the grid (R0 = grid rows of the area - 1, C0 = grid columns - 1), its
// transform is a real function times a linear phase:
//   W[a][b] = P(a, b) V(a, b),  P(a, b) = exp(-j pi (a R0 + b C0) / T),
//   V(a, b) = sum w[r][c] cos(2 pi (a (r - R0/2) + b (c - C0/2)) / T)   (real),
// for integer a, b (not reduced mod T): V(-a, -b) = V(a, b), and a shift of a
// or b by T multiplies V by (-1)^R0 or (-1)^C0.  With the residual spectrum
// rotated, Rt = conj(P) R, the update of eq. 3 in the DFT domain becomes
//   Rt[k] -= ct V(k - u) + conj(ct) V(k + u),   ct = c conj(P(u)) = gamma Rt[u] / W0,
// a real table and two real multiply-adds per part, and |Rt| = |R| leaves the
// selection (eq. 9) unchanged.  The window holds the real table as pairs:
// entry i (row i, column b) = (V(i - Q, b), V(i - Q + 1, b)), rows -Q .. 3Q + 1,
// so one 16-byte read serves two neighbouring register slots.  Slot pairs
// (2p, 2p + 1) read W[k - u] directly from row k - u when k >= Q and mirrored
// (V(u - k, v - l)) when k < Q; W[k + u] directly from row k + u when
// k <= Q + 1 and mirrored (V(T - k - u, -l - v) times (-1)^R0) otherwise;
// column wraps give per-lane signs folded into per-lane coefficients.  ht
// holds exp(-j pi q / T) for q in [0, 2T).
// Slot pairs whose window reads are in flight ahead of the pair being updated.
constexpr int kSymPrefetch = 2;

template <int T>
__device__ __forceinline__ void run_wave_sym(RegSpec<WaveRows<T, 1, 0>::S>& R, const double2* win,
                                             const double2* ht, const KParams& p, int b, int lane,
                                             double gW0) {
    using L = Layout<T, 1>;
    constexpr int S = WaveRows<T, 1, 0>::S;      // T/2 + 1 slots, rows 0 .. T/2
    constexpr int H = L::H;
    constexpr int Q = L::Q;
    static_assert(S == H + 1 && (Q & 1) == 0 && (H & 1) == 0, "one wavefront holds rows 0 .. T/2");
    const int K = p.K;
    const int R0 = p.N - 1, C0 = p.M - 1;        // transposed placement: grid rows = area columns
    const bool odd_r = (R0 & 1) != 0, odd_c = (C0 & 1) != 0;
    const bool lane_ok = lane < T;
    const bool edge_ok = lane_ok && lane <= H;
    const int l = lane;
    int u = 0, v = 0;
    double ca = 0.0, cb = 0.0;
    // window pointers of a selection (u, v): pair entry rows (window row =
    // grid row + Q); every base row lies in the window and every per-slot
    // offset is a non-negative constant
    const double2 *p1d, *p1m, *p2d, *p2m;
    auto set_ptrs = [&](int uu, int vv) {
        p1d = win + (2 * Q - uu) * T + ((l - vv) & (T - 1));      // + (k - Q) T,     k >= Q
        p1m = win + (uu + 1) * T + ((vv - l) & (T - 1));          // + (Q - 2 - k) T, k < Q even
        p2d = win + (uu + Q) * T + ((l + vv) & (T - 1));          // + k T,           k <= Q even
        p2m = win + (T + Q - 1 - uu - H) * T + ((-l - vv) & (T - 1));   // + (H - k) T, k > Q + 1 even
    };
    auto rd1 = [&](int k) -> double2 { return k >= Q ? p1d[(k - Q) * T] : p1m[(Q - 2 - k) * T]; };
    auto rd2 = [&](int k) -> double2 { return k <= Q + 1 ? p2d[k * T] : p2m[(H - k) * T]; };
    constexpr int NP = (S + 1) / 2;              // slot pairs (the last holds slot T/2 alone)
    constexpr int D = kSymPrefetch < NP ? kSymPrefetch : NP;
    double2 x1[NP], x2[NP];                      // fully unrolled: registers of the pairs in flight
    set_ptrs(0, 0);
#pragma unroll
    for (int q = 0; q < D; ++q) { x1[q] = rd1(2 * q); x2[q] = rd2(2 * q); }
    for (int it = 0; it < K; ++it) {
        // per-lane signs of the column wraps (and the row shift of the mirrored
        // second read) of the selection being applied, folded into the coefficients
        const bool n1d = odd_c && l < v;
        const bool n1m = odd_c && l > v;
        const bool n2d = odd_c && l + v >= T;
        const bool n2m = odd_r != (odd_c && l + v > 0 && l + v <= T);
        const double a1d = n1d ? ca : -ca, b1d = n1d ? cb : -cb;
        const double a1m = n1m ? ca : -ca, b1m = n1m ? cb : -cb;
        const double a2d = n2d ? ca : -ca, b2d = n2d ? -cb : cb;
        const double a2m = n2m ? ca : -ca, b2m = n2m ? -cb : cb;
        double best = 0.0;
        // slot pairs; the first D pairs' reads were issued with the selection,
        // pair q + D is read before pair q is used
#pragma unroll
        for (int q = 0; q < NP; ++q) {
            const int k = 2 * q;
            if (q + D < NP) { x1[q + D] = rd1(k + 2 * D); x2[q + D] = rd2(k + 2 * D); }
            // V1, V2 of slot k and (when present) slot k + 1
            const double v1k  = k >= Q ? x1[q].x : x1[q].y;
            const double v1k1 = k >= Q ? x1[q].y : x1[q].x;
            const double v2k  = k <= Q + 1 ? x2[q].x : x2[q].y;
            const double v2k1 = k <= Q + 1 ? x2[q].y : x2[q].x;
            const double A1 = k >= Q ? a1d : a1m, B1 = k >= Q ? b1d : b1m;
            const double A2 = k <= Q + 1 ? a2d : a2m, B2 = k <= Q + 1 ? b2d : b2m;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int s = k + h;
                if (s >= S) break;
                const double V1 = h ? v1k1 : v1k, V2 = h ? v2k1 : v2k;
                double re = R.gr(s), im = R.gi(s);
                re = fma(A1, V1, re);
                re = fma(A2, V2, re);
                im = fma(B1, V1, im);
                im = fma(B2, V2, im);
                R.set(s, re, im);
                const double m2 = sq_add(im, re * re);
                uint32_t lo = (__double2loint(m2) & 0xFFFFFFC0u) | (uint32_t)(63 - s);
                int hi = __double2hiint(m2);
                if (s == 0 || s == H) { hi = edge_ok ? hi : 0; lo = edge_ok ? lo : 0u; }
                else if (T < 64)      { hi = lane_ok ? hi : 0; lo = lane_ok ? lo : 0u; }
                best = max_f64(best, __hiloint2double(hi, (int)lo));
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        // wavefront maximum, ties to the smallest class key (as run_wave)
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
            if ((l2 & 0xFFFFFFC0u) > (mlo & 0xFFFFFFC0u)) { mlo = l2; wl = ln; }
        }
        mlo = (uint32_t)__builtin_amdgcn_readfirstlane((int)mlo);
        wl = __builtin_amdgcn_readfirstlane(wl);
        int wslot = (int)(63 - (mlo & 63u));
        wslot = __builtin_amdgcn_readfirstlane(wslot >= S ? S - 1 : wslot);
        u = wslot > H ? H : wslot;
        v = wl & (T - 1);
        // the next iteration's first window reads and the phase P(u) go out now,
        // ahead of the coefficient
        const double2 P = ht[(u * R0 + v * C0) & (2 * T - 1)];
        set_ptrs(u, v);
#pragma unroll
        for (int q = 0; q < D; ++q) { x1[q] = rd1(2 * q); x2[q] = rd2(2 * q); }
        const double2 wv = R.fetch(wslot, wl);             // Rt[u]
        // eqs. 5, 14 in the rotated frame: ct = gamma Rt[u] / W0, c = ct P(u);
        // a self-conjugate class keeps Re c
        const bool selfc = (u == 0 || u == H) && (v == 0 || v == H);
        double ctr = wv.x * gW0, cti = wv.y * gW0;
        double cre = ctr * P.x - cti * P.y;
        double cim = ctr * P.y + cti * P.x;
        if (selfc) {             // c real; ct = c conj(P(u))
            cim = 0.0;
            ctr = cre * P.x;
            cti = -cre * P.y;
        }
        if (lane == 0) {
            const size_t r = (size_t)b * K + it;
            p.sel[r] = v * T + u;
            p.coef[2 * r] = cre;
            p.coef[2 * r + 1] = cim;
        }
        // a self-conjugate class is applied as two half terms
        ca = selfc ? 0.5 * ctr : ctr;
        cb = selfc ? 0.5 * cti : cti;
    }
}

// Rt = conj(P) R on the slots of a wavefront holding rows 0 .. T/2 (lane =
// grid column): the rotation into the frame of run_wave_sym.
template <int T>
__device__ __forceinline__ void rotate_rows(RegSpec<WaveRows<T, 1, 0>::S>& R, const double2* ht, int R0, int C0,
                                           int lane) {
    constexpr int S = WaveRows<T, 1, 0>::S;
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const double2 P = ht[(s * R0 + lane * C0) & (2 * T - 1)];
        const double re = R.gr(s), im = R.gi(s);
        // conj(P) (re + j im)
        R.set(s, re * P.x + im * P.y, im * P.x - re * P.y);
    }
}

}  // namespace fofse
