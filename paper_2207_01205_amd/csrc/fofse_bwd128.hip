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
constexpr int NSPLIT = (T / 2 * HL + NT - 1) / NT;

using KY = Key<T>;
using FP = FftPlan<T>;

// X[k][l] of a Hermitian spectrum stored on the half plane after the column
// transform: X[k][l] at H[perm(k) * 65 + l] for l <= 64, conj X[-k][-l] otherwise.
__device__ __forceinline__ double2 half_at(const double2* H, int k, int l) {
    k &= T - 1;
    l &= T - 1;
    const bool up = l <= T / 2;
    const int kk = up ? k : (T - k) & (T - 1);
    const int ll = up ? l : T - l;
    const double2 v = H[FP::perm(kk) * HL + ll];
    return make_double2(v.x, up ? v.y : -v.y);
}

// x = tab (w or dw/drho) on A, zero elsewhere, written as complex lines of
// row pairs H[p * 130 + n] = x[2p][n] + j x[2p + 1][n].  With check_finite the
// known samples of f are tested and a non-finite one is reported in the
// return value (its weight is taken as 0, as in the forward).
__device__ __forceinline__ int load_row_pairs(double2* H, const BParams& p, const double* tab, size_t ab,
                                              bool check_finite, int tid) {
    const int M = p.M, N = p.N;
    int bad = 0;
#pragma unroll 4
    for (int t = tid; t < T / 2 * T; t += NT) {
        const int pr = t >> 7, n = t & (T - 1);
        double v[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int m = 2 * pr + h;
            v[h] = 0.0;
            if (m < M && n < N) {
                const int i = m * N + n;
                const bool a = p.target[i] == 0 && (!p.known || p.known[ab + i] != 0);
                if (a) {
                    bool nf = false;
                    if (check_finite) nf = nonfinite_bits(sample_bits(p.areas, ab + i));
                    bad |= nf;
                    v[h] = nf ? 0.0 : tab[i];
                }
            }
        }
        H[pr * PS + n] = make_double2(v[0], v[1]);
    }
    return bad;
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
    fft_stage_a<T, NT>(H, tw, T / 2, PS, 1, tid);
    __syncthreads();
    fft_stage_b<T, NT>(H, T / 2, PS, 1, tid);
    __syncthreads();
    // the FFT Z of line p holds the spectra of its two real rows:
    // X_2p[l] = (Z[l] + conj Z[-l]) / 2, X_2p+1[l] = (Z[l] - conj Z[-l]) / (2j)
    double2 a[NSPLIT], b[NSPLIT];
#pragma unroll
    for (int s = 0; s < NSPLIT; ++s) {
        const int t = tid + s * NT;
        a[s] = b[s] = make_double2(0.0, 0.0);
        if (t < T / 2 * HL) {
            const int pr = t / HL, l = t - pr * HL;
            const double2 z = H[pr * PS + FP::perm(l)];
            const double2 zm = H[pr * PS + FP::perm((T - l) & (T - 1))];
            a[s] = make_double2(0.5 * (z.x + zm.x), 0.5 * (z.y - zm.y));
            b[s] = make_double2(0.5 * (z.y + zm.y), 0.5 * (zm.x - z.x));
        }
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < NSPLIT; ++s) {
        const int t = tid + s * NT;
        if (t < T / 2 * HL) {
            const int pr = t / HL, l = t - pr * HL;
            H[pr * PS + l] = a[s];          // row 2p at (2p) * 65
            H[pr * PS + HL + l] = b[s];     // row 2p + 1 at (2p + 1) * 65
        }
    }
    __syncthreads();
    column_fft(H, tw, tid);
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
    constexpr int CH = 256;                 // samples of B staged per pass
    __shared__ double2 H[T / 2 * PS];       // half plane, 133,120 B
    __shared__ double2 tw[T];
    __shared__ int keyL[KM];
    __shared__ double2 cL[KM];
    __shared__ double2 cbL[KM];
    __shared__ int2 gm[CH];                 // (dL/dg as float bits, m << 16 | n)
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
    for (int i = tid; i < K; i += NT) {
        const int key = p.sel[rb + i] & (T * T - 1);   // k * T + l, read modulo the grid
        keyL[i] = key;
        // a self-conjugate class has a real coefficient (the forward writes 0)
        const bool pr = KY::pair(KY::k(key), KY::l(key));
        cL[i] = make_double2(p.coef[2 * (rb + i)], pr ? p.coef[2 * (rb + i) + 1] : 0.0);
    }
    if (tid == 0) s_flags = params_ok ? 0 : FOFSE_BLOCK_BAD_PARAM;
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

    // cbar0_nu = mult Gbar[u_nu], Gbar[k] = sum_B gbar[x] exp(-j 2 pi <k, x> / T);
    // the samples of B are staged through LDS (padded with zeros to a
    // multiple of 8)
    for (int nu0 = 0; nu0 < K; nu0 += NT) {
        const int nu = nu0 + tid;
        const int key = nu < K ? keyL[nu] : 0;
        const int k = KY::k(key), l = KY::l(key);
        double ar = 0.0, ai = 0.0;
        for (int q0 = 0; q0 < nB; q0 += CH) {
            const int cnt = min(CH, nB - q0);
            const int cnt8 = (cnt + 7) & ~7;
            __syncthreads();
            for (int i = tid; i < cnt8; i += NT) {
                int2 v = make_int2(0, 0);
                if (i < cnt) {
                    const int flat = p.bpix[q0 + i];
                    const int m = flat / N, n = flat - m * N;
                    v = make_int2(__float_as_int(p.grad_out[(size_t)b * nB + q0 + i]), (m << 16) | n);
                }
                gm[i] = v;
            }
            __syncthreads();
            for (int i = 0; i < cnt8; i += 8) {
                int2 v[8];
                double2 t[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) v[u] = gm[i + u];
#pragma unroll
                for (int u = 0; u < 8; ++u) t[u] = tw[(k * (v[u].y >> 16) + l * (v[u].y & 0xFFFF)) & (T - 1)];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const double g = (double)__int_as_float(v[u].x);
                    ar = fma(g, t[u].x, ar);
                    ai = fma(g, t[u].y, ai);
                }
            }
        }
        if (nu < K)
            cbL[nu] = KY::pair(k, l) ? make_double2(2.0 * ar, 2.0 * ai) : make_double2(ar, 0.0);
    }
    __syncthreads();

    // Transposed recurrence in panels of P iterations, from the last panel.
    // Step pn: wave 0 takes the contributions of panel pn + 1 (solved in the
    // previous step) into panel pn and resolves panel pn serially; at the same
    // time waves 1-7 apply panel pn + 1 to every iteration before panel pn.
    constexpr int P = 16;
    const int NPAN = (K + P - 1) / P;
    int kprev = 0;                       // wave 0: classes and finished adjoints of panel pn + 1
    double2 cprev = make_double2(0.0, 0.0);
    for (int pn = NPAN - 1; pn >= 0; --pn) {
        const int base = pn * P;
        const int cnt = min(P, K - base);
        const int pbase = (pn + 1) * P;
        const int pcnt = pn + 1 < NPAN ? min(P, K - pbase) : 0;
        if (wave == 0) {
            const bool valid = lane < cnt;
            const int key = valid ? keyL[base + lane] : 0;
            const int ku = KY::k(key), lu = KY::l(key);
            const bool pr = KY::pair(ku, lu);
            double2 cb = valid ? cbL[base + lane] : make_double2(0.0, 0.0);
            if (valid) {
                for (int u0 = 0; u0 < pcnt; u0 += 4) {
                    double sr[4], si[4];
                    double2 wd[4], ws[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int u = min(u0 + q, pcnt - 1);
                        const int kn = __builtin_amdgcn_readlane(kprev, u);
                        const double h = u0 + q < pcnt ? gW : 0.0;
                        sr[q] = h * readlane_f64(cprev.x, u);
                        si[q] = h * readlane_f64(cprev.y, u);
                        wd[q] = half_at(H, KY::k(kn) - ku, KY::l(kn) - lu);
                        ws[q] = half_at(H, KY::k(kn) + ku, KY::l(kn) + lu);
                    }
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        cb.x -= sr[q] * wd[q].x + si[q] * wd[q].y;     // sbar conj(W[u_n - u_i])
                        cb.y -= si[q] * wd[q].x - sr[q] * wd[q].y;
                        if (pr) {
                            cb.x -= sr[q] * ws[q].x + si[q] * ws[q].y; // conj(sbar) W[u_n + u_i]
                            cb.y -= sr[q] * ws[q].y - si[q] * ws[q].x;
                        }
                    }
                }
            }
            // serial sweep of panel pn: each lane first takes W at the sums and
            // differences with every later class of the panel into registers;
            // the finished adjoint of iteration j reaches the others by readlane
            double wr[P], wi[P], vr[P], vi[P];
            if (lane < P) {
#pragma unroll
                for (int j = 0; j < P; ++j) {
                    const int jj = min(j, cnt - 1);
                    const int kj = __builtin_amdgcn_readlane(ku, jj), lj = __builtin_amdgcn_readlane(lu, jj);
                    const double2 d = half_at(H, kj - ku, lj - lu);
                    const double2 s = half_at(H, kj + ku, lj + lu);
                    wr[j] = d.x;
                    wi[j] = d.y;
                    vr[j] = s.x;
                    vi[j] = s.y;
                }
            }
#pragma unroll
            for (int j = P - 1; j >= 0; --j) {
                if (j < cnt) {
                    const int keyj = __builtin_amdgcn_readlane(key, j);
                    const bool pj = KY::pair(KY::k(keyj), KY::l(keyj));
                    const double cr = readlane_f64(cb.x, j);
                    const double ci = pj ? readlane_f64(cb.y, j) : 0.0;
                    if (lane == j) cb = make_double2(cr, ci);  // final adjoint of c_j
                    const double sr = gW * cr, si = gW * ci;   // sbar_j
                    if (lane < j) {
                        cb.x -= sr * wr[j] + si * wi[j];
                        cb.y -= si * wr[j] - sr * wi[j];
                        if (pr) {
                            cb.x -= sr * vr[j] + si * vi[j];
                            cb.y -= sr * vi[j] - si * vr[j];
                        }
                    }
                }
            }
            if (valid) cbL[base + lane] = cb;
            kprev = key;
            cprev = cb;
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
                const bool pr = KY::pair(ku, lu);
                double ar = 0.0, ai = 0.0;
                for (int q0 = 0; q0 < NQ; q0 += 4) {
                    double sr[4], si[4];
                    double2 wd[4], ws[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int nu = pbase + g + (q0 + q) * G;
                        const int v = min(nu, pbase + pcnt - 1);
                        const int key2 = keyL[v];
                        const double2 cbn = cbL[v];
                        const double h = (q0 + q < NQ && nu < pbase + pcnt) ? gW : 0.0;
                        sr[q] = h * cbn.x;
                        si[q] = h * cbn.y;
                        wd[q] = half_at(H, KY::k(key2) - ku, KY::l(key2) - lu);
                        ws[q] = half_at(H, KY::k(key2) + ku, KY::l(key2) + lu);
                    }
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        ar -= sr[q] * wd[q].x + si[q] * wd[q].y;
                        ai -= si[q] * wd[q].x - sr[q] * wd[q].y;
                        if (pr) {
                            ar -= sr[q] * ws[q].x + si[q] * ws[q].y;
                            ai -= sr[q] * ws[q].y - si[q] * ws[q].x;
                        }
                    }
                }
                for (int o = 1; o < G; o <<= 1) {
                    ar += __shfl_xor(ar, o, 64);
                    ai += __shfl_xor(ai, o, 64);
                }
                if (g == 0) {
                    const double2 o = cbL[mu];
                    cbL[mu] = make_double2(o.x + ar, o.y + ai);
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
    double racc = 0.0;
    if (K > 0) {
        const int dmu = NT / K, dnu = NT - dmu * K;
        int mu = tid / K, nu = tid - mu * K;
        while (mu < K) {
            if (nu > mu) {
                const int km = keyL[mu], kn = keyL[nu];
                const int ku = KY::k(km), lu = KY::l(km);
                const double2 c = cL[mu];
                const double2 cbn = cbL[nu];
                const double sr = gW * cbn.x, si = gW * cbn.y;
                const double2 dd = half_at(H, KY::k(kn) - ku, KY::l(kn) - lu);
                double qr = c.x * dd.x - c.y * dd.y, qi = c.x * dd.y + c.y * dd.x;
                racc -= sr * qr + si * qi;
                if (KY::pair(ku, lu)) {
                    const double2 ds = half_at(H, KY::k(kn) + ku, KY::l(kn) + lu);
                    qr = c.x * ds.x + c.y * ds.y;
                    qi = c.x * ds.y - c.y * ds.x;
                    racc -= sr * qr + si * qi;
                }
            }
            mu += dmu;
            nu += dnu;
            if (nu >= K) {
                nu -= K;
                ++mu;
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
    // half plane.  Every bin is summed in iteration order by the first
    // iteration that reaches it (directly or through -k).
    for (int i = tid; i < T * HL; i += NT) H[i] = make_double2(0.0, 0.0);
    __syncthreads();
    for (int nu = tid; nu < K; nu += NT) {
        const int key = keyL[nu];
        const int k = KY::k(key), l = KY::l(key);
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            int hk = k, hl = l;
            if (side == 0) {
                if (l > T / 2) continue;
            } else {
                if (l != 0 && l < T / 2) continue;
                hk = (T - k) & (T - 1);
                hl = (T - l) & (T - 1);
                if (hk == k && hl == l) continue;       // same bin as side 0
            }
            const int hkey = hk * T + hl;
            const int nkey = ((T - hk) & (T - 1)) * T + ((T - hl) & (T - 1));
            int first = K;
            double sr = 0.0, si = 0.0;
            for (int j = 0; j < K; ++j) {       // same trip count everywhere: broadcast reads
                const int kj = keyL[j];
                const double2 cbj = cbL[j];
                const bool m1 = kj == hkey, m2 = kj == nkey;
                first = (m1 || m2) && j < first ? j : first;
                // y_j = conj(cbar_j) (times gamma / W0) directly, conj(y_j) through -k
                sr += m1 ? cbj.x : 0.0;
                si -= m1 ? cbj.y : 0.0;
                sr += m2 ? cbj.x : 0.0;
                si += m2 ? cbj.y : 0.0;
            }
            if (first == nu) H[hk * HL + hl] = make_double2(0.5 * gW * sr, 0.5 * gW * si);
        }
    }
    __syncthreads();
    real_out_fft2_half(H, tw, tid);

    // dL/df = w (w f)bar on A; rho term of R0 = DFT(w f)
    for (int i = tid; i < MN; i += NT) {
        const int m = i / N, n = i - m * N;
        const bool a = p.target[i] == 0 && (!p.known || p.known[ab + i] != 0);
        double gv = 0.0;
        if (a) {
            const int q = FP::perm(m);
            const double2 v = H[(q >> 1) * PS + FP::perm(n)];
            const double wfb = (q & 1) ? v.y : v.x;
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

}  // namespace

hipError_t launch_bwd128(const BParams& p, hipStream_t stream) {
    if (p.T != T || p.K > KM || p.M > T || p.N > T) return hipErrorInvalidValue;
    hipLaunchKernelGGL(fofse_bwd128_kernel, dim3(p.n_blocks), dim3(NT), 0, stream, p);
    return hipGetLastError();
}

}  // namespace fofse
