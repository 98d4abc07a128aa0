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
// One workgroup per block (the grouped adjoint in fofse_bwd_group.hip serves
// batches of blocks that share support masks).  W and D come from one complex
// FFT of z = w + j dw/drho in LDS (separated by Hermitian symmetry at each
// read); the recurrence runs in panels of 16 iterations: one wavefront
// resolves a panel serially (lane = iteration, the finished adjoint is
// broadcast with readlane) while the other waves apply the previous panel to
// the earlier iterations and accumulate the rho terms.  (w f)bar comes from
// one more 2-D FFT.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fofse_kernel.h"
#include "device_common.hpp"
#include "adjoint.hpp"

namespace fofse {

// Workgroups per CU: at T <= 32 the LDS of four fits and the kernel is bound by
// latency, so four (128 VGPRs, with some spilling) run faster than two.
template <int T, int KMAX>
__global__ __launch_bounds__(256, KMAX <= 256 ? (T <= 32 ? 4 : 2) : 1) void fofse_bwd_kernel(BParams p) {
    constexpr int NT = 256;
    constexpr int CH = 256;                 // samples of B staged per pass
    using KY = Key<T>;
    __shared__ double2 buf[T * T];
    __shared__ double2 tw[T];
    __shared__ int keyL[KMAX];
    __shared__ double2 cL[KMAX];
    __shared__ double2 cbL[KMAX];
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
    for (int i = tid; i < T * T; i += NT) buf[i] = make_double2(0.0, 0.0);
    const size_t rb = (size_t)b * K;
    for (int i = tid; i < K; i += NT) {
        const int key = p.sel[rb + i] & (T * T - 1);   // k * T + l, read modulo the grid
        keyL[i] = key;
        // a self-conjugate class has a real coefficient (the forward writes 0)
        const bool pr = KY::pair(KY::k(key), KY::l(key));
        cL[i] = make_double2(p.coef[2 * (rb + i)], pr ? p.coef[2 * (rb + i) + 1] : 0.0);
    }
    if (tid == 0) s_flags = params_ok ? 0 : FOFSE_BLOCK_BAD_PARAM;
    __syncthreads();

    // z = w + j dw/drho on the T x T grid, area at the origin (row m, column n);
    // all loads of a thread are issued before the first use
    constexpr int PPT = T * T / NT;         // samples per thread (M N <= T^2)
    const size_t ab = (size_t)b * MN;
    {
        bool a[PPT];
        uint32_t fb[PPT];
        double w[PPT], dw[PPT];
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            const int i = tid + j * NT;
            a[j] = false;
            fb[j] = 0u;
            w[j] = dw[j] = 0.0;
            if (i < MN) {
                a[j] = p.target[i] == 0 && (!p.known || p.known[ab + i] != 0);
                fb[j] = sample_bits(p.areas, ab + i);
                w[j] = p.wtab[i];
                dw[j] = p.dwtab[i];
            }
        }
        int bad = 0;
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            const int i = tid + j * NT;
            if (i < MN) {
                const int m = i / N, n = i - m * N;
                const bool nf = nonfinite_bits(fb[j]);
                bad |= a[j] && nf;
                const bool use = a[j] && !nf;
                buf[m * T + n] = use ? make_double2(w[j], dw[j]) : make_double2(0.0, 0.0);
            }
        }
        if (bad) atomicOr(&s_flags, FOFSE_BLOCK_NONFINITE);
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
    if constexpr (T == 64) {
        // FFT output order -> natural order.  For T = 64 the order swaps the
        // two octal digits of each index, an involution: one pass of swaps.
        for (int e = tid; e < T * T; e += NT) {
            const int pe = FftPlan<T>::perm(e / T) * T + FftPlan<T>::perm(e % T);
            if (pe > e) {
                const double2 x = buf[e], y = buf[pe];
                buf[e] = y;
                buf[pe] = x;
            }
        }
        __syncthreads();
    }
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

    // cbar0_nu = mult Gbar[u_nu], Gbar[k] = sum_B gbar[x] exp(-j 2 pi <k, x> / T);
    // the samples of B are staged through LDS (padded with zeros to a
    // multiple of 8, so the unrolled loop needs no tail)
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
    // Step pn: wave 0 takes the contributions of the panel solved in the
    // previous step (pn + 1) into panel pn and then resolves panel pn serially;
    // at the same time waves 1-3 apply panel pn + 1 to every iteration before
    // panel pn and accumulate the rho terms of all its pairs.  One barrier per
    // step; the last step (pn = -1) only finishes the rho terms of panel 0.
    constexpr int P = 16;
    const double hW = 0.5 * gW;         // sbar / 2 absorbs the halving in W = (Z + conj Z(-k)) / 2
    double racc = 0.0;
    const int NPAN = (K + P - 1) / P;
    int kprev = 0;                       // wave 0: classes and finished adjoints of panel pn + 1
    double2 cprev = make_double2(0.0, 0.0);
    for (int pn = NPAN - 1; pn >= -1; --pn) {
        const int base = pn >= 0 ? pn * P : 0;
        const int cnt = pn >= 0 ? min(P, K - base) : 0;
        const int pbase = (pn + 1) * P;
        const int pcnt = pn + 1 < NPAN ? min(P, K - pbase) : 0;
        const int phi = pbase + pcnt;
        if (wave == 0) {
            if (pn >= 0) {
                const bool valid = lane < cnt;
                const int key = valid ? keyL[base + lane] : 0;
                const int ku = KY::k(key), lu = KY::l(key);
                const bool pr = KY::pair(ku, lu);
                double2 cb = valid ? cbL[base + lane] : make_double2(0.0, 0.0);
                const ZOff<T> zo(ku, lu);
                // contributions of panel pn + 1 (lane u of kprev / cprev)
                if (valid) {
                    for (int u0 = 0; u0 < pcnt; u0 += 4) {
                        double sr[4], si[4];
                        double2 za[4], zb[4], zc[4], zd[4];
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const int u = min(u0 + q, pcnt - 1);
                            const int kn = __builtin_amdgcn_readlane(kprev, u);
                            const double h = u0 + q < pcnt ? hW : 0.0;
                            sr[q] = h * readlane_f64(cprev.x, u);
                            si[q] = h * readlane_f64(cprev.y, u);
                            int oa, ob, oc, od;
                            zo.get(KY::k(kn), KY::l(kn), oa, ob, oc, od);
                            za[q] = lds_at(buf, oa);
                            zb[q] = lds_at(buf, ob);
                            zc[q] = lds_at(buf, oc);
                            zd[q] = lds_at(buf, od);
                        }
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const double wdr = za[q].x + zb[q].x, wdi = za[q].y - zb[q].y;
                            cb.x -= sr[q] * wdr + si[q] * wdi;
                            cb.y -= si[q] * wdr - sr[q] * wdi;
                            if (pr) {
                                const double wsr = zc[q].x + zd[q].x, wsi = zc[q].y - zd[q].y;
                                cb.x -= sr[q] * wsr + si[q] * wsi;
                                cb.y -= sr[q] * wsi - si[q] * wsr;
                            }
                        }
                    }
                }
                // serial sweep of panel pn.  Each lane first takes the W samples
                // it needs from every later iteration of the panel into
                // registers; the sweep then touches no memory: the finished
                // adjoint of iteration j reaches the other lanes by readlane.
                double wr[P], wi[P], vr[P], vi[P];     // 2 W[u_j - u_i], 2 W[u_j + u_i]
                if (lane < P) {
#pragma unroll
                    for (int j = 0; j < P; ++j) {
                        const int jj = min(j, cnt - 1);
                        const int kj = __builtin_amdgcn_readlane(ku, jj), lj = __builtin_amdgcn_readlane(lu, jj);
                        int oa, ob, oc, od;
                        zo.get(kj, lj, oa, ob, oc, od);
                        const double2 za = lds_at(buf, oa), zb = lds_at(buf, ob);
                        const double2 zc = lds_at(buf, oc), zd = lds_at(buf, od);
                        wr[j] = za.x + zb.x;
                        wi[j] = za.y - zb.y;
                        vr[j] = zc.x + zd.x;
                        vi[j] = zc.y - zd.y;
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
                        const double sr = hW * cr, si = hW * ci;   // sbar_j / 2
                        if (lane < j) {
                            cb.x -= sr * wr[j] + si * wi[j];        // sbar conj(W[u_j - u_i])
                            cb.y -= si * wr[j] - sr * wi[j];
                            if (pr) {
                                cb.x -= sr * vr[j] + si * vi[j];    // conj(sbar) W[u_j + u_i]
                                cb.y -= sr * vi[j] - si * vr[j];
                            }
                        }
                    }
                }
                if (valid) cbL[base + lane] = cb;
                kprev = key;
                cprev = cb;
            }
        } else if (pcnt > 0) {
            // Waves 1-3: panel pn + 1 into the iterations mu < base, and the rho
            // terms of every pair mu < nu with nu in panel pn + 1.  G threads
            // (adjacent lanes) share the panel's iterations of one mu; their
            // partial sums meet by butterfly shuffles (fixed order).
            constexpr int NT3 = NT - 64;
            const int G = phi * 16 <= NT3 ? 16 : phi * 8 <= NT3 ? 8 : phi * 4 <= NT3 ? 4 : phi * 2 <= NT3 ? 2 : 1;
            const int NQ = P / G;
            for (int t = tid - 64; t < phi * G; t += NT3) {
                const int mu = t / G, g = t - mu * G;
                const int key = keyL[mu];
                const int ku = KY::k(key), lu = KY::l(key);
                const bool pr = KY::pair(ku, lu);
                const bool cross = mu < base && pn >= 0;
                const double2 c = cL[mu];
                const ZOff<T> zo(ku, lu);
                double ar = 0.0, ai = 0.0, rr = 0.0;
                for (int q0 = 0; q0 < NQ; q0 += 4) {
                    double sr[4], si[4];
                    double2 za[4], zb[4], zc[4], zd[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int nu = pbase + g + (q0 + q) * G;
                        const int v = min(nu, phi - 1);
                        const int key2 = keyL[v];
                        const int kn = KY::k(key2), ln = KY::l(key2);
                        const double2 cbn = cbL[v];
                        const double h = (q0 + q < NQ && nu < phi && nu > mu) ? hW : 0.0;
                        sr[q] = h * cbn.x;              // sbar / 2
                        si[q] = h * cbn.y;
                        int oa, ob, oc, od;
                        zo.get(kn, ln, oa, ob, oc, od);
                        za[q] = lds_at(buf, oa);
                        zb[q] = lds_at(buf, ob);
                        zc[q] = lds_at(buf, oc);
                        zd[q] = lds_at(buf, od);
                    }
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        // 2 W and 2 D (D = DFT(dw/drho)) at u_nu - u_mu and u_nu + u_mu
                        const double wdr = za[q].x + zb[q].x, wdi = za[q].y - zb[q].y;
                        const double ddr = za[q].y + zb[q].y, ddi = zb[q].x - za[q].x;
                        if (cross) {
                            ar -= sr[q] * wdr + si[q] * wdi;
                            ai -= si[q] * wdr - sr[q] * wdi;
                        }
                        {   // -Re(sbar conj(c D[u_nu - u_mu]))
                            const double qr = c.x * ddr - c.y * ddi, qi = c.x * ddi + c.y * ddr;
                            rr -= sr[q] * qr + si[q] * qi;
                        }
                        if (pr) {
                            const double wsr = zc[q].x + zd[q].x, wsi = zc[q].y - zd[q].y;
                            const double dsr = zc[q].y + zd[q].y, dsi = zd[q].x - zc[q].x;
                            if (cross) {
                                ar -= sr[q] * wsr + si[q] * wsi;
                                ai -= sr[q] * wsi - si[q] * wsr;
                            }
                            // -Re(sbar conj(conj(c) D[u_nu + u_mu]))
                            const double qr = c.x * dsr + c.y * dsi, qi = c.x * dsi - c.y * dsr;
                            rr -= sr[q] * qr + si[q] * qi;
                        }
                    }
                }
                for (int o = 1; o < G; o <<= 1) {
                    ar += __shfl_xor(ar, o, 64);
                    ai += __shfl_xor(ai, o, 64);
                }
                if (cross && g == 0) {
                    const double2 o = cbL[mu];
                    cbL[mu] = make_double2(o.x + ar, o.y + ai);
                }
                racc += rr;
            }
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
        const int kk = keyL[nu];
        int first = K;
        double sr = 0.0, si = 0.0;
        for (int j = 0; j < K; ++j) {       // same trip count everywhere: broadcast reads
            const bool m = keyL[j] == kk;
            const double2 cbj = cbL[j];
            first = m && j < first ? j : first;
            sr += m ? cbj.x : 0.0;
            si += m ? cbj.y : 0.0;
        }
        if (first == nu) buf[kk] = make_double2(gW * sr, -gW * si);
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
    {
        bool a[PPT];
        float fv[PPT];
        double w[PPT], dw[PPT];
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            const int i = tid + j * NT;
            a[j] = false;
            fv[j] = 0.0f;
            w[j] = dw[j] = 0.0;
            if (i < MN) {
                a[j] = p.target[i] == 0 && (!p.known || p.known[ab + i] != 0);
                fv[j] = p.areas[ab + i];
                w[j] = p.wtab[i];
                dw[j] = p.dwtab[i];
            }
        }
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            const int i = tid + j * NT;
            if (i < MN) {
                const int m = i / N, n = i - m * N;
                double gv = 0.0;
                if (a[j]) {
                    const double wfb = buf[FftPlan<T>::perm(m) * T + FftPlan<T>::perm(n)].x;
                    gv = w[j] * wfb;
                    racc += dw[j] * (double)fv[j] * wfb;
                }
                if (p.grad_areas) p.grad_areas[ab + i] = (float)gv;
            }
        }
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
    const bool t128 = p.T == 128;
    if ((p.T != 64 && p.T != 32 && p.T != 16 && !t128) || p.K > (t128 ? kBackwardMaxK128 : kBackwardMaxK))
        return hipErrorInvalidValue;
    hipError_t e = launch_weights(wp, stream);
    if (e != hipSuccess) return e;
    if (tm.start && hipEventRecord(tm.start, stream) != hipSuccess) return hipErrorUnknown;
    if (t128) e = launch_bwd128(p, stream);
    else if (p.T == 64) e = p.K <= 256 ? launch_bwd<64, 256>(p, stream) : launch_bwd<64, kBackwardMaxK>(p, stream);
    else if (p.T == 32) e = p.K <= 256 ? launch_bwd<32, 256>(p, stream) : launch_bwd<32, kBackwardMaxK>(p, stream);
    else e = p.K <= 256 ? launch_bwd<16, 256>(p, stream) : launch_bwd<16, kBackwardMaxK>(p, stream);
    if (e != hipSuccess) return e;
    if (tm.stop && hipEventRecord(tm.stop, stream) != hipSuccess) return hipErrorUnknown;
    return d_sum ? launch_bwd_sum(p, d_sum, stream) : hipSuccess;
}

hipError_t launch_bwd_sum(const BParams& p, double* d_sum, hipStream_t stream) {
    hipLaunchKernelGGL(k_bwd_sum, dim3(1), dim3(256), 0, stream, (const double*)p.grad_block, p.n_blocks,
                       d_sum);
    return hipGetLastError();
}

}  // namespace fofse
