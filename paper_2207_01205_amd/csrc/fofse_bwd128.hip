// Adjoint of the FOFSE forward pass for FFT size 128, for gfx950.
//
// The derivative is the one of the smaller sizes (fofse_bwd.hip): with the
// record's classes fixed, the coefficients solve a K x K lower-triangular
// recurrence whose entries are samples of W = DFT(w) (eq. 3 in the DFT domain,
// eqs. 5, 14), and the reverse pass is the transposed recurrence
//   cbar_nu = mult Gbar[u_nu] - sum_{mu>nu} (sbar_mu conj(W[u_mu - u_nu]) + conj(sbar_mu) W[u_mu + u_nu])
//   sbar_nu = gamma / W0 * cbar_nu
// followed by the rho terms, which pair every sbar_nu with c_mu D[u_nu -+ u_mu]
// for mu < nu (D = DFT(dw/drho)), and one more 2-D transform for dL/df.
//
// What changes at T = 128 is storage: the complex spectrum of w + j dw/drho
// the smaller sizes keep in LDS would take 256 KB.  w and dw/drho are real, so
// W and D are Hermitian (X[-k] = conj X[k]) and the half plane X[k][l],
// l in [0, 64], holds all of either: 128 x 65 x 16 B = 133,120 B.  The
// workgroup keeps W there while it solves the recurrence, then replaces it
// with D for the rho terms, then uses the same storage for the last transform,
// whose output is real.  Each of the three 2-D transforms is real-in or
// real-out: two real rows share one complex 128-point FFT, and a Hermitian
// pair of rows becomes one complex row for the real-out direction.
//
// One workgroup of eight wavefronts per block, one workgroup per compute unit
// (the half plane and the record fill the LDS).

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fofse_kernel.h"
#include "device_common.hpp"
#include "adjoint.hpp"

namespace fofse {
namespace {

constexpr int T = 128;
constexpr int HL = T / 2 + 1;          // columns of the half plane, l in [0, 64]
constexpr int PS = 2 * HL;             // stride of a pair of rows
constexpr int NT = 512;                // threads per workgroup
constexpr int KM = kBackwardMaxK128;   // largest K held in LDS
static_assert(KM <= NT, "one thread per iteration in the last scatter");
constexpr int NSPLIT = (T / 2 * HL + NT - 1) / NT;
constexpr int NSPLIT_LOW = (T / 4 * HL + NT - 1) / NT;

using KY = Key<T>;
using FP = FftPlan<T>;

// X[k][l] of a Hermitian spectrum stored on the half plane after the column
// transform: X[k][l] at H[perm(k) * 65 + l] for l <= 64, conj X[-k][-l]
// otherwise.  half_idx gives the entry and whether it is to be conjugated.
__device__ __forceinline__ int half_idx(int k, int l, bool& conj) {
    k &= T - 1;
    l &= T - 1;
    const bool up = l <= T / 2;
    conj = !up;
    const int kk = up ? k : (T - k) & (T - 1);
    const int ll = up ? l : T - l;
    return FP::perm(kk) * HL + ll;
}
__device__ __forceinline__ double2 conj_if(double2 v, bool c) { return make_double2(v.x, c ? -v.y : v.y); }
__device__ __forceinline__ double2 half_at(const double2* H, int k, int l) {
    bool c;
    const int i = half_idx(k, l, c);
    return conj_if(H[i], c);
}

// Sum of v over aligned groups of G adjacent lanes (G = 1, 2, 4, 8 or 16,
// uniform) by DPP exchanges within rows of 16; every lane of a group gets the
// same bits (each step adds a value and its partner's in either order).
__device__ __forceinline__ double group_sum(double v, int G) {
    if (G >= 2) v += dpp_f64<0xB1, 0xF>(v);      // quad_perm [1,0,3,2]
    if (G >= 4) v += dpp_f64<0x4E, 0xF>(v);      // quad_perm [2,3,0,1]
    if (G >= 8) v += dpp_f64<0x141, 0xF>(v);     // row_half_mirror
    if (G >= 16) v += dpp_f64<0x140, 0xF>(v);    // row_mirror
    return v;
}

// Update of the adjoint cbar_i of a class u_i by a later class u_n with
// finished adjoint cbar_n (sbar_n = g cbar_n, g = gamma / W0):
//   cbar_i -= sbar_n conj(Wd) + pr_i conj(sbar_n) Ws,  Wd = W[u_n - u_i], Ws = W[u_n + u_i],
// pr_i = 1 for a conjugate-pair class u_i, 0 for a self-conjugate one.  In
// real arithmetic, with (cr, ci) = cbar_n:
//   Re cbar_i -= g (cr a + ci b),  Im cbar_i -= g (ci c + cr d),
//   a = Re Wd + pr_i Re Ws, b = Im Wd + pr_i Im Ws,
//   c = Re Wd - pr_i Re Ws, d = pr_i Im Ws - Im Wd.
// upd_coef gives (a, b, c, d) for prf = pr_i as 0.0 or 1.0; the factor g is
// applied to a sum of updates, or folded into the coefficients (upd_scale).
struct Upd {
    double a, b, c, d;
};
__device__ __forceinline__ Upd upd_coef(double2 wd, double2 ws, double prf) {
    return {fma(prf, ws.x, wd.x), fma(prf, ws.y, wd.y), fma(-prf, ws.x, wd.x), fma(prf, ws.y, -wd.y)};
}
__device__ __forceinline__ Upd upd_scale(const Upd& u, double g) { return {g * u.a, g * u.b, g * u.c, g * u.d}; }
__device__ __forceinline__ void upd_apply(double2& cb, const Upd& u, double cr, double ci) {
    cb.x = fma(-cr, u.a, fma(-ci, u.b, cb.x));
    cb.y = fma(-ci, u.c, fma(-cr, u.d, cb.y));
}

// The area of a 128-point plan is at most 64 x 64, so in the grid of the
// transforms rows and columns 64..127 are zero.  The loaders fill lines
// p < 32 of the row pairs (rows 2p and 2p + 1 as H[p * 130 + n] = x[2p][n] +
// j x[2p + 1][n], zero for n >= 64); lines 32..63 are not used.  Every load
// goes out before the first test (out-of-area samples read index 0).
constexpr int LINES = T / 4;                  // row pairs that can hold samples
constexpr int LOADS = LINES * (T / 2) / NT;   // loaded entries per thread

// x = tab (w or dw/drho) on A, zero elsewhere.  With check_finite the known
// samples of f are tested and a non-finite one is reported in the return
// value (its weight is taken as 0, as in the forward).
__device__ __forceinline__ int load_row_pairs(double2* H, const BParams& p, const double* tab, size_t ab,
                                              bool check_finite, int tid) {
    const int M = p.M, N = p.N;
    int bad = 0;
#pragma unroll
    for (int s = 0; s < LOADS; ++s) {
        const int t = tid + s * NT;
        const int pr = t >> 6, n = t & (T / 2 - 1);
        double v[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int m = 2 * pr + h;
            const bool in = m < M && n < N;
            const int i = in ? m * N + n : 0;
            const uint8_t tg = p.target[i];
            const uint8_t kn = p.known ? p.known[ab + i] : (uint8_t)1;
            const uint32_t fb = check_finite ? sample_bits(p.areas, ab + i) : 0u;
            const double x = tab[i];
            const bool a = in && tg == 0 && kn != 0;
            const bool nf = a && nonfinite_bits(fb);
            bad |= nf;
            v[h] = a && !nf ? x : 0.0;
        }
        H[pr * PS + n] = make_double2(v[0], v[1]);
        H[pr * PS + T / 2 + n] = make_double2(0.0, 0.0);
    }
    return bad;
}

// dL/dg on B (zero elsewhere) as row pairs, like load_row_pairs.
__device__ __forceinline__ void load_grad_pairs(double2* H, const BParams& p, int b, int tid) {
    const int M = p.M, N = p.N;
    const float* go = p.grad_out + (size_t)b * p.nB;
    int q[LOADS][2];
#pragma unroll
    for (int s = 0; s < LOADS; ++s) {
        const int t = tid + s * NT;
        const int pr = t >> 6, n = t & (T / 2 - 1);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int m = 2 * pr + h;
            const bool in = m < M && n < N;
            const int qq = p.bidx[in ? m * N + n : 0];
            q[s][h] = in ? qq : -1;
        }
    }
#pragma unroll
    for (int s = 0; s < LOADS; ++s) {
        const int t = tid + s * NT;
        const int pr = t >> 6, n = t & (T / 2 - 1);
        double v[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const float g = go[q[s][h] >= 0 ? q[s][h] : 0];
            v[h] = q[s][h] >= 0 ? (double)g : 0.0;
        }
        H[pr * PS + n] = make_double2(v[0], v[1]);
        H[pr * PS + T / 2 + n] = make_double2(0.0, 0.0);
    }
}

// Stage A of the column FFTs when rows 64..127 of the input are zero: of the
// samples 8 n1 + n2 only n1 < 8 are read (writes cover every row).
__device__ __forceinline__ void column_stage_a_low(double2* H, const double2* tw, int tid) {
    constexpr int R1 = FP::R1;
    for (int task = tid; task < HL * 8; task += NT) {
        const bool main = task < (T / 2) * 8;
        const int line = main ? task & (T / 2 - 1) : T / 2;
        const int n2 = main ? task >> 6 : task - (T / 2) * 8;
        double2* base = H + line;
        double2 x[R1];
#pragma unroll
        for (int n1 = 0; n1 < R1; ++n1) x[n1] = n1 < R1 / 2 ? base[(8 * n1 + n2) * HL] : make_double2(0.0, 0.0);
        dft<R1>(x);
#pragma unroll
        for (int k1 = 0; k1 < R1; ++k1) {
            const double2 v = k1 ? c_mul(x[k1], tw[(n2 * k1) & (T - 1)]) : x[k1];
            base[(8 * k1 + n2) * HL] = v;
        }
    }
}

// 128-point FFTs along the 65 columns of the half plane (rows r at r * 65),
// output row k at perm(k) * 65.
__device__ __forceinline__ void column_fft(double2* H, const double2* tw, int tid) {
    fft_stage_a<T, NT>(H, tw, T / 2, 1, HL, tid);
    fft_stage_a<T, NT>(H + T / 2, tw, 1, 1, HL, tid);
    __syncthreads();
    fft_stage_b<T, NT>(H, T / 2, 1, HL, tid);
    fft_stage_b<T, NT>(H + T / 2, 1, 1, HL, tid);
    __syncthreads();
}

// Half spectrum of the real grid loaded by load_row_pairs: X[k][l], l <= 64,
// at H[perm(k) * 65 + l].
__device__ void real_fft2_half(double2* H, const double2* tw, int tid) {
    fft_stage_a<T, NT>(H, tw, LINES, PS, 1, tid);
    __syncthreads();
    fft_stage_b<T, NT>(H, LINES, PS, 1, tid);
    __syncthreads();
    // the FFT Z of line p holds the spectra of its two real rows:
    // X_2p[l] = (Z[l] + conj Z[-l]) / 2, X_2p+1[l] = (Z[l] - conj Z[-l]) / (2j)
    double2 a[NSPLIT_LOW], b[NSPLIT_LOW];
#pragma unroll
    for (int s = 0; s < NSPLIT_LOW; ++s) {
        const int t = tid + s * NT;
        a[s] = b[s] = make_double2(0.0, 0.0);
        if (t < LINES * HL) {
            const int pr = t / HL, l = t - pr * HL;
            const double2 z = H[pr * PS + FP::perm(l)];
            const double2 zm = H[pr * PS + FP::perm((T - l) & (T - 1))];
            a[s] = make_double2(0.5 * (z.x + zm.x), 0.5 * (z.y - zm.y));
            b[s] = make_double2(0.5 * (z.y + zm.y), 0.5 * (zm.x - z.x));
        }
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < NSPLIT_LOW; ++s) {
        const int t = tid + s * NT;
        if (t < LINES * HL) {
            const int pr = t / HL, l = t - pr * HL;
            H[pr * PS + l] = a[s];          // row 2p at (2p) * 65
            H[pr * PS + HL + l] = b[s];     // row 2p + 1 at (2p + 1) * 65
        }
    }
    __syncthreads();
    // rows 64..127 are zero: stage A reads rows 0..63 only and writes all
    column_stage_a_low(H, tw, tid);
    __syncthreads();
    fft_stage_b<T, NT>(H, T / 2, 1, HL, tid);
    fft_stage_b<T, NT>(H + T / 2, 1, 1, HL, tid);
    __syncthreads();
}

// y[m][n] = sum_{k,l} Y[k][l] exp(-j 2 pi (k m + l n) / T) for a Hermitian Y
// given on the half plane H[k * 65 + l] (natural row order); y is real.
// Output: y[m][n] is the real (q even) or imaginary (q odd) part of
// H[(q >> 1) * 130 + perm(n)] with q = perm(m).
__device__ void real_out_fft2_half(double2* H, const double2* tw, int tid) {
    column_fft(H, tw, tid);             // row q = perm(m) now holds Y1[m][l], Hermitian in l
    double2 a[NSPLIT], b[NSPLIT];
#pragma unroll
    for (int s = 0; s < NSPLIT; ++s) {
        const int t = tid + s * NT;
        a[s] = b[s] = make_double2(0.0, 0.0);
        if (t < T / 2 * HL) {
            const int pr = t / HL, l = t - pr * HL;
            a[s] = H[pr * PS + l];
            b[s] = H[pr * PS + HL + l];
        }
    }
    __syncthreads();
    // rows q = 2p and 2p + 1 as one complex line Z[l] = A[l] + j B[l] over the
    // whole period (A[-l] = conj A[l]); its FFT is y[m0] + j y[m1]
#pragma unroll
    for (int s = 0; s < NSPLIT; ++s) {
        const int t = tid + s * NT;
        if (t < T / 2 * HL) {
            const int pr = t / HL, l = t - pr * HL;
            H[pr * PS + l] = make_double2(a[s].x - b[s].y, a[s].y + b[s].x);
            if (l > 0 && l < T / 2) H[pr * PS + T - l] = make_double2(a[s].x + b[s].y, b[s].x - a[s].y);
        }
    }
    __syncthreads();
    fft_stage_a<T, NT>(H, tw, T / 2, PS, 1, tid);
    __syncthreads();
    fft_stage_b<T, NT>(H, T / 2, PS, 1, tid);
    __syncthreads();
}

__global__ __launch_bounds__(NT, 1) void fofse_bwd128_kernel(BParams p) {
    __shared__ double2 H[T / 2 * PS];       // half plane, 133,120 B
    __shared__ double2 tw[T];
    __shared__ __align__(16) int keyL[KM];  // keys, -1 past K
    __shared__ double2 cL[KM];
    __shared__ double2 cbL[KM];
    __shared__ Upd cfL[16 * 16];            // pair coefficients of the panel being solved
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
    const size_t rb = (size_t)b * K;
    for (int i = tid; i < KM; i += NT) {
        const int key = i < K ? p.sel[rb + i] & (T * T - 1) : -1;   // k * T + l, read modulo the grid
        keyL[i] = key;
        cbL[i] = make_double2(0.0, 0.0);
        if (i < K) {
            // a self-conjugate class has a real coefficient (the forward writes 0)
            const bool pr = KY::pair(KY::k(key), KY::l(key));
            cL[i] = make_double2(p.coef[2 * (rb + i)], pr ? p.coef[2 * (rb + i) + 1] : 0.0);
        }
    }
    if (tid == 0) s_flags = params_ok ? 0 : FOFSE_BLOCK_BAD_PARAM;

    // cbar0_nu = mult Gbar[u_nu], Gbar = DFT of dL/dg on B: one real 2-D FFT
    // while the half plane is still free
    load_grad_pairs(H, p, b, tid);
    __syncthreads();
    real_fft2_half(H, tw, tid);
    for (int nu = tid; nu < K; nu += NT) {
        const int key = keyL[nu];
        const int k = KY::k(key), l = KY::l(key);
        const double2 g = half_at(H, k, l);
        cbL[nu] = KY::pair(k, l) ? make_double2(2.0 * g.x, 2.0 * g.y) : make_double2(g.x, 0.0);
    }
    __syncthreads();

    const size_t ab = (size_t)b * MN;
    const int bad = load_row_pairs(H, p, p.wtab, ab, true, tid);
    __syncthreads();
    if (bad) atomicOr(&s_flags, FOFSE_BLOCK_NONFINITE);
    real_fft2_half(H, tw, tid);             // W on the half plane; ends with a barrier

    const double W0 = H[0].x;
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

    // Transposed recurrence in panels of P iterations, from the last panel,
    // two barriers per panel.  Step pn:
    //  1. all threads, one pair each: the contributions of panel pn + 1
    //     (finished in the previous step) into panel pn, summed over 16
    //     adjacent lanes in a fixed order, and the update coefficients of the
    //     pairs i < j within panel pn into cfL (j-major, so that lane i of
    //     wave 0 reads them without bank conflicts);
    //  2. wave 0 resolves panel pn serially (its lanes are the panel's
    //     iterations; the finished adjoint of iteration j reaches the earlier
    //     lanes by readlane) while waves 1-7 apply panel pn + 1 to every
    //     iteration before panel pn.
    constexpr int P = 16;
    const int NPAN = (K + P - 1) / P;
    for (int pn = NPAN - 1; pn >= 0; --pn) {
        const int base = pn * P;
        const int cnt = min(P, K - base);
        const int pbase = (pn + 1) * P;
        const int pcnt = pn + 1 < NPAN ? min(P, K - pbase) : 0;
        {
            const int i = (tid >> 4) & (P - 1), x = tid & (P - 1);
            const int keyi = keyL[base + min(i, cnt - 1)];
            const int ku = KY::k(keyi), lu = KY::l(keyi);
            const double prf = KY::pair(ku, lu) ? 1.0 : 0.0;
            if (tid < P * P) {
                // x: an iteration of panel pn + 1
                double2 acc = make_double2(0.0, 0.0);
                if (i < cnt && x < pcnt) {
                    const int kn = keyL[pbase + x];
                    const double2 cbn = cbL[pbase + x];
                    const Upd c = upd_coef(half_at(H, KY::k(kn) - ku, KY::l(kn) - lu),
                                           half_at(H, KY::k(kn) + ku, KY::l(kn) + lu), prf);
                    upd_apply(acc, c, cbn.x, cbn.y);
                }
                acc.x = group_sum(acc.x, P);
                acc.y = group_sum(acc.y, P);
                if (x == 0 && i < cnt && pcnt > 0) {
                    const double2 o = cbL[base + i];
                    cbL[base + i] = make_double2(fma(gW, acc.x, o.x), fma(gW, acc.y, o.y));
                }
            } else if (i < x && x < cnt) {
                // x: a later iteration j of panel pn
                const int kj = keyL[base + x];
                cfL[x * P + i] = upd_scale(upd_coef(half_at(H, KY::k(kj) - ku, KY::l(kj) - lu),
                                                    half_at(H, KY::k(kj) + ku, KY::l(kj) + lu), prf), gW);
            }
        }
        __syncthreads();
        if (wave == 0) {
            const bool valid = lane < cnt;
            const int key = valid ? keyL[base + lane] : 0;
            const bool pr = KY::pair(KY::k(key), KY::l(key));
            const uint64_t pmask = __ballot(pr);
            double2 cb = valid ? cbL[base + lane] : make_double2(0.0, 0.0);
            // coefficients 0 where lane >= j or j >= cnt: those updates change nothing
            Upd cf[P];
#pragma unroll
            for (int j = 0; j < P; ++j) cf[j] = lane < j && j < cnt ? cfL[j * P + lane] : Upd{0.0, 0.0, 0.0, 0.0};
            // lane j's adjoint is final once the later lanes have updated it;
            // its imaginary part counts only for a pair class
#pragma unroll
            for (int j = P - 1; j >= 0; --j) {
                const double cr = readlane_f64(cb.x, j);
                const double ci = (pmask >> j) & 1 ? readlane_f64(cb.y, j) : 0.0;
                upd_apply(cb, cf[j], cr, ci);
            }
            if (!pr) cb.y = 0.0;
            if (valid) cbL[base + lane] = cb;
        } else if (pcnt > 0 && base > 0) {
            // panel pn + 1 into the iterations mu < base; G adjacent lanes share
            // the panel's iterations of one mu and meet by butterfly shuffles
            constexpr int NT7 = NT - 64;
            const int G = base * 16 <= NT7 ? 16 : base * 8 <= NT7 ? 8 : base * 4 <= NT7 ? 4 : base * 2 <= NT7 ? 2 : 1;
            const int NQ = P / G;
            for (int t = tid - 64; t < base * G; t += NT7) {
                const int mu = t / G, g = t - mu * G;
                const int key = keyL[mu];
                const int ku = KY::k(key), lu = KY::l(key);
                const double prf = KY::pair(ku, lu) ? 1.0 : 0.0;
                double2 acc = make_double2(0.0, 0.0);
                for (int q0 = 0; q0 < NQ; q0 += 4) {
                    double cr[4], ci[4];
                    int id[8];
                    bool cj[8];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int nu = pbase + g + (q0 + q) * G;
                        const int v = min(nu, pbase + pcnt - 1);
                        const int key2 = keyL[v];
                        const double2 cbn = cbL[v];
                        const bool use = q0 + q < NQ && nu < pbase + pcnt;
                        cr[q] = use ? cbn.x : 0.0;
                        ci[q] = use ? cbn.y : 0.0;
                        id[2 * q] = half_idx(KY::k(key2) - ku, KY::l(key2) - lu, cj[2 * q]);
                        id[2 * q + 1] = half_idx(KY::k(key2) + ku, KY::l(key2) + lu, cj[2 * q + 1]);
                    }
                    double2 w[8];
#pragma unroll
                    for (int q = 0; q < 8; ++q) w[q] = H[id[q]];
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        upd_apply(acc, upd_coef(conj_if(w[2 * q], cj[2 * q]), conj_if(w[2 * q + 1], cj[2 * q + 1]), prf),
                                  cr[q], ci[q]);
                }
                acc.x = group_sum(acc.x, G);
                acc.y = group_sum(acc.y, G);
                if (g == 0) {
                    const double2 o = cbL[mu];
                    cbL[mu] = make_double2(fma(gW, acc.x, o.x), fma(gW, acc.y, o.y));
                }
            }
        }
        __syncthreads();
    }

    // D = DFT(dw/drho) replaces W on the half plane
    load_row_pairs(H, p, p.dwtab, ab, false, tid);
    __syncthreads();
    real_fft2_half(H, tw, tid);
    const double dW0 = H[0].x;              // sum of dw/drho over A

    // rho terms of the recurrence: -sum_{mu<nu} Re(sbar_nu conj(c_mu D[u_nu - u_mu])
    //                                + sbar_nu conj(conj(c_mu) D[u_nu + u_mu]))
    // Row mu of the pairs (nu = mu + 1 .. K - 1) and row K - 2 - mu hold K pairs
    // together, so the rows go in such couples (the middle row alone when K is
    // even) and slot (couple c, position q) of the C x K slots is a pair or
    // nothing; four slots per thread are in flight at a time.
    double racc = 0.0;
    {
        const int C = K / 2;
        const int total = C * K;
        const float rK = K > 0 ? 1.0f / (float)K : 0.0f;
        for (int i0 = tid; i0 < total; i0 += 4 * NT) {
            int mu[4], nu[4];
            bool ok[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int idx = i0 + q * NT;
                int c = (int)((float)idx * rK);
                c += (c + 1) * K <= idx ? 1 : 0;
                c -= c * K > idx ? 1 : 0;
                const int pos = idx - c * K;
                const int len0 = K - 1 - c;            // pairs of row c
                const int m2 = K - 2 - c;              // its partner row
                ok[q] = idx < total && (pos < len0 || m2 != c);
                mu[q] = pos < len0 ? c : m2;
                nu[q] = pos < len0 ? c + 1 + pos : m2 + 1 + (pos - len0);
                if (!ok[q]) mu[q] = nu[q] = 0;
            }
            int km[4], kn[4];
            double2 c[4], cbn[4], dd[4], ds[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                km[q] = keyL[mu[q]];
                kn[q] = keyL[nu[q]];
                c[q] = cL[mu[q]];
                cbn[q] = cbL[nu[q]];
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int ku = KY::k(km[q]), lu = KY::l(km[q]);
                dd[q] = half_at(H, KY::k(kn[q]) - ku, KY::l(kn[q]) - lu);
                ds[q] = half_at(H, KY::k(kn[q]) + ku, KY::l(kn[q]) + lu);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const double h = ok[q] ? gW : 0.0;
                const double sr = h * cbn[q].x, si = h * cbn[q].y;   // sbar_nu
                // -Re(sbar conj(c_mu D[u_nu - u_mu]))
                double qr = c[q].x * dd[q].x - c[q].y * dd[q].y, qi = c[q].x * dd[q].y + c[q].y * dd[q].x;
                racc -= sr * qr + si * qi;
                if (KY::pair(KY::k(km[q]), KY::l(km[q]))) {
                    // -Re(sbar conj(conj(c_mu) D[u_nu + u_mu]))
                    qr = c[q].x * ds[q].x + c[q].y * ds[q].y;
                    qi = c[q].x * ds[q].y - c[q].y * ds[q].x;
                    racc -= sr * qr + si * qi;
                }
            }
        }
    }

    // sum_nu Re(cbar_nu conj(c_nu)): gives dL/dgamma and dL/dW0
    double tacc = 0.0;
    for (int nu = tid; nu < K; nu += NT) {
        const double2 cb = cbL[nu], c = cL[nu];
        tacc += cb.x * c.x + cb.y * c.y;
    }
    __syncthreads();                        // every read of D done

    // (w f)bar = Re sum_k Rbar0[k] exp(+j 2 pi <k, x> / T) = F y_h with
    // y = conj(Rbar0) on the grid, Rbar0[k] = gamma / W0 * sum_{nu: u_nu = k} cbar_nu,
    // and y_h[k] = (y[k] + conj y[-k]) / 2 its Hermitian part, given on the
    // half plane.  An iteration reaches the bin (k, l) when l <= 64 and the
    // bin (-k, -l) when l = 0 or l >= 64 (once when the two coincide).
    // Every bin's 16 bytes first hold four counters: the first iteration that
    // reaches it (LDS atomic min), how many do (atomic add), and for a bin
    // reached several times the start of its list of iterations in `seg` and
    // that list's fill.  The lists are filled in any order; each member then
    // finds its rank (the number of smaller iterations in its list), so that
    // the first iteration sums the bin in iteration order.  Nothing here
    // depends on the order of the atomics.  A bin reached by none is cleared.
    int* Hi = reinterpret_cast<int*>(H);
    int* seg = reinterpret_cast<int*>(cfL);              // lists, then sorted lists
    constexpr int SEG = KM * 2;                          // room for every (iteration, bin)
    static_assert(2 * SEG * sizeof(int) <= sizeof(cfL), "lists fit in the panel coefficients");
    for (int i = tid; i < T * HL; i += NT) reinterpret_cast<int4*>(H)[i] = make_int4(K, 0, 0, 0);
    if (tid == 0) s_flags = 0;                          // reused: list space taken so far
    __syncthreads();
    int bin[2] = {-1, -1}, hkey[2] = {-2, -2}, nkey[2] = {-2, -2};
    double2 own[2] = {make_double2(0.0, 0.0), make_double2(0.0, 0.0)};
    const int nu = tid;                     // K <= NT: one iteration per thread
    if (nu < K) {
        const int key = keyL[nu];
        const int k = KY::k(key), l = KY::l(key);
        const int nk = (T - k) & (T - 1), nl = (T - l) & (T - 1);
        const double2 cbn = cbL[nu];
        if (l <= T / 2) {
            bin[0] = k * HL + l;
            hkey[0] = key;
            nkey[0] = nk * T + nl;
            // y / 2, and conj(y) / 2 as well for a bin that is its own negative
            own[0] = key == nkey[0] ? make_double2(cbn.x, 0.0) : make_double2(0.5 * cbn.x, -0.5 * cbn.y);
        }
        if ((l == 0 || l >= T / 2) && !(nk == k && nl == l)) {
            bin[1] = nk * HL + nl;
            hkey[1] = nk * T + nl;
            nkey[1] = key;
            own[1] = make_double2(0.5 * cbn.x, 0.5 * cbn.y);       // conj(y) / 2
        }
#pragma unroll
        for (int sd = 0; sd < 2; ++sd) {
            if (bin[sd] >= 0) {
                atomicMin(&Hi[4 * bin[sd]], nu);
                atomicAdd(&Hi[4 * bin[sd] + 1], 1);
            }
        }
    }
    __syncthreads();
    int first[2] = {K, K}, count[2] = {0, 0};
#pragma unroll
    for (int sd = 0; sd < 2; ++sd) {
        if (bin[sd] >= 0) {
            first[sd] = Hi[4 * bin[sd]];
            count[sd] = Hi[4 * bin[sd] + 1];
            if (first[sd] == nu && count[sd] > 1) Hi[4 * bin[sd] + 2] = atomicAdd(&s_flags, count[sd]);
        }
    }
    __syncthreads();
    int lbase[2] = {0, 0};
#pragma unroll
    for (int sd = 0; sd < 2; ++sd) {
        if (count[sd] > 1) {
            lbase[sd] = Hi[4 * bin[sd] + 2];
            seg[lbase[sd] + atomicAdd(&Hi[4 * bin[sd] + 3], 1)] = nu;
        }
    }
    __syncthreads();
#pragma unroll
    for (int sd = 0; sd < 2; ++sd) {
        if (count[sd] > 1) {
            int rank = 0;
            for (int q = 0; q < count[sd]; ++q) rank += seg[lbase[sd] + q] < nu ? 1 : 0;
            seg[SEG + lbase[sd] + rank] = nu;
        }
    }
    constexpr int BPT = (T * HL + NT - 1) / NT;
    bool unreached[BPT];
#pragma unroll
    for (int q = 0; q < BPT; ++q) {
        const int i = tid + q * NT;
        unreached[q] = i < T * HL && Hi[4 * i + 1] == 0;
    }
    __syncthreads();
#pragma unroll
    for (int sd = 0; sd < 2; ++sd) {
        if (first[sd] == nu && count[sd] > 1) {
            double sr = 0.0, si = 0.0;
            for (int q = 0; q < count[sd]; ++q) {
                const int j = seg[SEG + lbase[sd] + q];
                const int kj = keyL[j];
                const double2 cbj = cbL[j];
                if (kj == hkey[sd]) {   // y_j = conj(cbar_j) directly
                    sr += cbj.x;
                    si -= cbj.y;
                }
                if (kj == nkey[sd]) {   // conj(y_j) through -k
                    sr += cbj.x;
                    si += cbj.y;
                }
            }
            own[sd] = make_double2(0.5 * sr, 0.5 * si);
        }
    }
#pragma unroll
    for (int q = 0; q < BPT; ++q)
        if (unreached[q]) H[tid + q * NT] = make_double2(0.0, 0.0);
#pragma unroll
    for (int sd = 0; sd < 2; ++sd)
        if (first[sd] == nu) H[bin[sd]] = make_double2(gW * own[sd].x, gW * own[sd].y);
    __syncthreads();
    real_out_fft2_half(H, tw, tid);

    // dL/df = w (w f)bar on A; rho term of R0 = DFT(w f)
    for (int i = tid; i < MN; i += NT) {
        const int m = i / N, n = i - m * N;
        const uint8_t tg = p.target[i];
        const uint8_t kn = p.known ? p.known[ab + i] : (uint8_t)1;
        const double w = p.wtab[i], dw = p.dwtab[i];
        const float f = p.areas[ab + i];
        const int q = FP::perm(m);
        const double2 v = H[(q >> 1) * PS + FP::perm(n)];
        const double wfb = (q & 1) ? v.y : v.x;
        const bool a = tg == 0 && kn != 0;
        if (a) racc += dw * (double)f * wfb;
        if (p.grad_areas) p.grad_areas[ab + i] = a ? (float)(w * wfb) : 0.0f;
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

}  // namespace

hipError_t launch_bwd128(const BParams& p, hipStream_t stream) {
    if (p.T != T || p.K > KM || p.M > T || p.N > T) return hipErrorInvalidValue;
    hipLaunchKernelGGL(fofse_bwd128_kernel, dim3(p.n_blocks), dim3(NT), 0, stream, p);
    return hipGetLastError();
}

}  // namespace fofse
