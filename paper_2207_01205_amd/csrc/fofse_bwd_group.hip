// Grouped adjoint of the FOFSE forward pass for gfx950 (T = 64, K <= 256).
//
// The arithmetic is the transposed recurrence of the per-block adjoint
// (fofse_bwd.hip states it in full): with the selection record fixed,
//   cbar_nu = mult Gbar[u_nu]
//             - sum_{mu>nu} (sbar_mu conj(W[u_mu - u_nu]) + conj(sbar_mu) W[u_mu + u_nu])
//   sbar_nu = gamma / W0 cbar_nu       (real part for a self-conjugate class)
// plus the rho terms, which pair sbar with D = DFT(dw/drho), and one inverse
// transform of Rbar0 for dL/df (eqs. 1-5, 7, 8, 14, 15).
//
// Blocks whose support areas have the same known-sample mask share w, hence W
// and D (eqs. 4 and 15 depend on the mask only).  A workgroup takes the work
// items of the grouped forward (up to kGroup blocks of one mask), builds
// Z = W + j D once in LDS and gives each block one wavefront:
//   * the K iterations of a block live in registers, K / 64 per lane (row
//     mu = lane + 64 r) with class, coefficient and running adjoint;
//   * rows are resolved from the last chunk of 64 down: inside a chunk
//     serially (the finished adjoint of row j is broadcast with readlane and
//     applied to the rows below it), then the whole chunk is applied to every
//     lower chunk with all lanes busy;
//   * Gbar[u_nu] is separable over the rows of B's bounding box;
//   * Rbar0 is scattered, made Hermitian, so that its transform is real; the
//     even and odd columns of that real result come from one 64 x 32 complex
//     FFT per block (two blocks per 64 KB pass).  The scatter adds in 64-bit
//     fixed point (exact integer sums at a resolution of 2^-49 of the block's
//     largest value), so the result does not depend on the order in which the
//     atomic adds land, nor on the other blocks of the work item.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "adjoint.hpp"
#include "device_common.hpp"
#include "fofse_kernel.h"

namespace fofse {

namespace {

constexpr int kRC = kGroupBackwardMaxK / 64;   // row chunks per lane
constexpr int kBatch = 6;                      // samples per lane with loads in flight

// Z' is stored skewed: entry (k, l) at column (l + 13 k) mod 64 of row k, so
// that the LDS bank of an entry depends on k as well as l (the classes of a
// record cluster at low frequencies; unskewed, the gathers of a wave pile onto
// few banks; on frame records the multiplier 13 leaves about as many conflicts
// as random addresses would).  A class travels packed as k << 26 | s << 4 with
// s = (l + 13 k) mod 64: k << 10 in the high and s << 4 in the low 16-bit half.  The skew is
// additive, so one packed 16-bit add or subtract forms both coordinates of the
// skewed address of u_nu +- u_mu with no borrow between them; the high half
// wraps k modulo 64 by itself, the low half is masked, and (r >> 16) | (r & 0x3F0)
// is the byte offset in the 64 x 64 table.
constexpr int kSkew = 13;
__device__ __forceinline__ uint32_t pack_class(int k, int l) {
    return ((uint32_t)k << 26) | ((uint32_t)((l + kSkew * k) & 63) << 4);
}
__device__ __forceinline__ int class_k(uint32_t x) { return (int)(x >> 26); }
__device__ __forceinline__ int class_l(uint32_t x) { return (int)((x >> 4) - kSkew * (x >> 26)) & 63; }
// self-conjugate when k and l are 0 or 32 (with k a multiple of 32, s = l mod 32)
__device__ __forceinline__ bool packed_pair(uint32_t x) { return (x & ((31u << 26) | (31u << 4))) != 0; }

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pk_add(uint32_t a, uint32_t b) {
    return __builtin_bit_cast(uint32_t, __builtin_bit_cast(u16x2, a) + __builtin_bit_cast(u16x2, b));
}
__device__ __forceinline__ uint32_t pk_sub(uint32_t a, uint32_t b) {
    return __builtin_bit_cast(uint32_t, __builtin_bit_cast(u16x2, a) - __builtin_bit_cast(u16x2, b));
}
__device__ __forceinline__ int zoff(uint32_t r) { return (int)((r >> 16) | (r & 0x3F0u)); }

// exact power of two, -1022 <= n <= 1023
__device__ __forceinline__ double pow2(int n) { return __hiloint2double((n + 1023) << 20, 0); }

// The four samples of Z' a pair of classes needs: Z'[u_nu - u_mu],
// Z'[u_mu - u_nu], Z'[u_nu + u_mu], Z'[-u_nu - u_mu] for the packed classes x
// (uniform, nu; nx = -x) and y (per lane, mu).
struct ZQ {
    double2 a, b, c, d;
};

__device__ __forceinline__ ZQ zgather(const double2* Z, uint32_t x, uint32_t nx, uint32_t y) {
    const int oa = zoff(pk_sub(x, y));
    const int ob = zoff(pk_sub(y, x));
    const int oc = zoff(pk_add(x, y));
    const int od = zoff(pk_sub(nx, y));
    ZQ q;
    q.a = lds_at(Z, oa);
    q.b = lds_at(Z, ob);
    q.c = lds_at(Z, oc);
    q.d = lds_at(Z, od);
    return q;
}

// Row mu takes the finished iteration nu.  Z' = gamma / (2 W0) Z, so with
// (sr, si) = cbar_nu and 2 W[d] = Z[d] + conj Z[-d], 2 j D[d] = Z[d] - conj Z[-d]:
//   cbar_mu -= sbar conj(W[u_nu - u_mu]) + conj(sbar) W[u_nu + u_mu]
//   racc    -= Re(sbar conj(c_mu D[u_nu - u_mu])) + Re(sbar conj(conj(c_mu) D[u_nu + u_mu]))
// A self-conjugate mu takes the first term of each line only; as u_mu = -u_mu
// there, the second term equals the first (c_mu is real), so such a row runs
// the same formula on a doubled cbar_mu and a halved c_mu.
__device__ __forceinline__ void zapply(const ZQ& q, double sr, double si, double2 c, double2& cb,
                                       double& rr) {
    const double s1 = q.a.x + q.b.x, s2 = q.c.x + q.d.x;   // Re W[d], Re W[s] (scaled)
    const double d1 = q.a.y - q.b.y, d2 = q.c.y - q.d.y;   // Im W
    const double e1 = q.a.y + q.b.y, e2 = q.c.y + q.d.y;   // Re D
    const double f1 = q.b.x - q.a.x, f2 = q.d.x - q.c.x;   // Im D
    cb.x -= sr * (s1 + s2) + si * (d1 + d2);
    cb.y -= si * (s1 - s2) - sr * (d1 - d2);
    const double qr = c.x * (e1 + e2) - c.y * (f1 - f2);
    const double qi = c.x * (f1 + f2) + c.y * (e1 - e2);
    rr -= sr * qr + si * qi;
}

// The iterations of one block, row mu = lane + 64 r.
struct Rows {
    uint32_t x[kRC];   // class, packed
    bool pr[kRC];      // not self-conjugate (and a valid row)
    double2 c[kRC];    // forward coefficient c_mu (halved for a self-conjugate class)
    double2 cb[kRC];   // cbar_mu: running (doubled for a self-conjugate class), then final
};

struct BwdGroupShared {
    double2 buf[64 * 64];       // H tables, then Z', then the output grids
    double2 tw[64];             // exp(-j 2 pi q / 64)
    double2 tw32[32];           // exp(-j 2 pi q / 32)
    int expo[kGroup];
    int live[kGroup];           // block slot takes part (present, no flag)
    double rpart[kGroup][64];   // rho_hat terms of dL/df a helper wavefront found, per slot and lane
    int next;                   // next work item of the workgroup (queue)
    alignas(16) uint8_t mask[64 * 64];   // support mask of the work item's blocks
};

// Serial sweep of chunk r: row j (from the last) is final when reached; it is
// applied to the rows below it in the chunk.  The samples of the next step are
// gathered before the current step is computed.
template <int r>
__device__ __forceinline__ void sweep_chunk(Rows& R, const double2* Z, int lane, int nv, double& rr) {
    auto step = [&](int j, uint32_t x, const ZQ& q) {
        double cr = readlane_f64(R.cb[r].x, j), ci = 0.0;
        if (packed_pair(x)) ci = readlane_f64(R.cb[r].y, j);
        else cr *= 0.5;                   // a self-conjugate row runs doubled
        if (lane < j) zapply(q, cr, ci, R.c[r], R.cb[r], rr);
    };
    auto cls = [&](int j) { return (uint32_t)__builtin_amdgcn_readlane((int)R.x[r], j); };
    int j = nv - 1;
    uint32_t xa = cls(j);
    ZQ qa = zgather(Z, xa, pk_sub(0u, xa), R.x[r]);
    for (; j >= 1; j -= 2) {
        const uint32_t xb = cls(j - 1);
        const ZQ qb = zgather(Z, xb, pk_sub(0u, xb), R.x[r]);
        step(j, xa, qa);
        xa = cls(max(j - 2, 0));
        qa = zgather(Z, xa, pk_sub(0u, xa), R.x[r]);
        step(j - 1, xb, qb);
    }
    if (j == 0) step(0, xa, qa);
    // final adjoint of a self-conjugate class: real, back to scale
    if (!R.pr[r]) R.cb[r] = make_double2(0.5 * R.cb[r].x, 0.0);
}

// The finished chunk r applied to every lower chunk (all lanes, all rows valid).
template <int r>
__device__ __forceinline__ void cross_chunk(Rows& R, const double2* Z, int nv, double& rr) {
    for (int j = 0; j < nv; ++j) {
        const uint32_t x = (uint32_t)__builtin_amdgcn_readlane((int)R.x[r], j);
        const uint32_t nx = pk_sub(0u, x);
        const double cr = readlane_f64(R.cb[r].x, j);
        const double ci = readlane_f64(R.cb[r].y, j);
#pragma unroll
        for (int r2 = 0; r2 < r; ++r2) {
            const ZQ q = zgather(Z, x, nx, R.x[r2]);
            zapply(q, cr, ci, R.c[r2], R.cb[r2], rr);
        }
    }
}

template <int r>
__device__ __forceinline__ void chunk(Rows& R, const double2* Z, int lane, int K, double& rr) {
    const int nv = min(64, K - 64 * r);
    if (nv > 0) {
        sweep_chunk<r>(R, Z, lane, nv, rr);
        if constexpr (r > 0) cross_chunk<r>(R, Z, nv, rr);
    }
}

// cbar0_nu = mult Gbar[u_nu] with Gbar[k, l] = sum_B gbar[m, n] exp(-j 2 pi (k m + l n) / 64),
// separable over the rows of B's bounding box: H[m][l] = sum_n gbar[m, n] tw[l n]
// (lane = l, 16 box rows per pass, in this wave's 16 KB of LDS), then
// Gbar[k, l] = sum_m tw[k m] H[m][l] (lane = iteration).
__device__ __forceinline__ void cbar0_rows(const BParams& p, int bj, int lane, double2* H,
                                           const double2* tw, Rows& R, int K) {
    double2 acc[kRC];
#pragma unroll
    for (int r = 0; r < kRC; ++r) acc[r] = make_double2(0.0, 0.0);
    const int N = p.N;
    const float* go = p.grad_out + (size_t)bj * p.nB;
    for (int m0 = 0; m0 < p.b_h; m0 += 16) {
        // the 16 index loads, then the 16 value loads, each group in flight
        // together (indices clamped into the box, values outside it dropped)
        float gv[16];
        int qv[16];
        const int n = p.b_n0 + min(lane, p.b_w - 1);
#pragma unroll
        for (int i = 0; i < 16; ++i) qv[i] = p.bidx[(p.b_m0 + min(m0 + i, p.b_h - 1)) * N + n];
#pragma unroll
        for (int i = 0; i < 16; ++i) gv[i] = go[max(qv[i], 0)];
#pragma unroll
        for (int i = 0; i < 16; ++i)
            if (!(lane < p.b_w && m0 + i < p.b_h && qv[i] >= 0)) gv[i] = 0.0f;
        double2 h[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) h[i] = make_double2(0.0, 0.0);
        for (int c = 0; c < p.b_w; ++c) {
            const double2 t = tw[(lane * (p.b_n0 + c)) & 63];
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const double g = (double)__int_as_float(__builtin_amdgcn_readlane(__float_as_int(gv[i]), c));
                h[i].x = fma(g, t.x, h[i].x);
                h[i].y = fma(g, t.y, h[i].y);
            }
        }
        // this wavefront's LDS rows: its lanes see each other's writes in program order
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int i = 0; i < 16; ++i) H[i * 64 + lane] = h[i];
        __builtin_amdgcn_wave_barrier();
        const int rows = min(16, p.b_h - m0);
#pragma unroll
        for (int r = 0; r < kRC; ++r) {
            const int k = class_k(R.x[r]), l = class_l(R.x[r]);
            for (int i = 0; i < rows; ++i) {
                const double2 hv = H[i * 64 + l];
                const double2 t = tw[(k * (p.b_m0 + m0 + i)) & 63];
                acc[r].x += hv.x * t.x - hv.y * t.y;
                acc[r].y += hv.x * t.y + hv.y * t.x;
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
#pragma unroll
    for (int r = 0; r < kRC; ++r) {
        // mult Gbar (mult = 2 for a conjugate pair); a self-conjugate row runs doubled
        const bool valid = lane + 64 * r < K;
        R.cb[r] = valid ? make_double2(2.0 * acc[r].x, R.pr[r] ? 2.0 * acc[r].y : 0.0) : make_double2(0.0, 0.0);
    }
}

}  // namespace

template <int MAXPX>
__global__ __launch_bounds__(64 * kGroup, 2) void fofse_bwd_group_kernel(BParams p, GroupArgs g) {
    constexpr int T = 64, NT = 64 * kGroup;
    __shared__ BwdGroupShared sh;

    const int tid = (int)__builtin_amdgcn_workitem_id_x(), lane = tid & 63, wave = tid >> 6;
    const int M = p.M, N = p.N, MN = M * N, K = p.K;
    const double rho = p.rho_gamma[0], gamma = p.rho_gamma[1];
    const bool params_ok = param_ok(rho) && param_ok(gamma);
    for (int i = tid; i < T; i += NT) sh.tw[i] = p.twiddle[i];
    for (int i = tid; i < 32; i += NT) sh.tw32[i] = p.twiddle[2 * i];

    // work items: contiguous ranges when every block has the same support,
    // else a queue (the counter zeroed by the grouping; the next index is
    // fetched while the current item runs)
    const int n_items = g.direct ? (p.n_blocks + kGroup - 1) / kGroup : g.counts[1];
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
        int nblk, b0, b1, b2, b3;
        if (g.direct) {
            nblk = min(kGroup, p.n_blocks - item * kGroup);
            b0 = item * kGroup;
            b1 = b0 + 1;
            b2 = b0 + 2;
            b3 = b0 + 3;
        } else {
            const int* ib = g.item_blk + (size_t)item * kGroup;
            nblk = g.item_n[item];
            b0 = ib[0];
            b1 = ib[1];
            b2 = ib[2];
            b3 = ib[3];
        }
        static_assert(kGroup == 4, "one wavefront per block slot");
        const int b_rep = b0;                    // every block of the item has this mask
        const bool present = wave < nblk;
        const int bj = present ? __builtin_amdgcn_readfirstlane(wave == 0 ? b0 : wave == 1 ? b1 : wave == 2 ? b2 : b3)
                               : 0;
        const size_t ab = (size_t)bj * MN;
        // thread index as an opaque per-item value: keeps the compiler from
        // hoisting every per-thread address of the item's loops out of the
        // item loop (they would pin registers for the whole kernel)
        int tidv = tid;
        asm volatile("" : "+v"(tidv));
        __syncthreads();                         // previous item done with LDS
        // the item's support mask, once for all its blocks (every load issued
        // before any is used, indices clamped into the area)
        {
            uint8_t off[MAXPX];                  // on B or unknown
#pragma unroll
            for (int q = 0; q < MAXPX; ++q) off[q] = p.target[min(tidv + q * NT, MN - 1)];
            if (p.known) {
                uint8_t kn[MAXPX];
#pragma unroll
                for (int q = 0; q < MAXPX; ++q) kn[q] = p.known[(size_t)b_rep * MN + min(tidv + q * NT, MN - 1)];
#pragma unroll
                for (int q = 0; q < MAXPX; ++q) off[q] |= kn[q] == 0;
            }
#pragma unroll
            for (int q = 0; q < MAXPX; ++q) {
                const int i = tidv + q * NT;
                if (i < MN) sh.mask[i] = off[q] == 0 ? 1 : 0;
            }
        }
        __syncthreads();

        // per wavefront: flags, record, cbar0
        int flags = params_ok ? 0 : FOFSE_BLOCK_BAD_PARAM;
        if (present) {
            bool bad = false;
            if ((MN & 3) == 0 && (((uintptr_t)p.areas) & 15) == 0) {
                // four samples per 16-byte load, kQuad loads per lane in flight
                constexpr int kQuad = 12;
                const uint4* a4 = reinterpret_cast<const uint4*>(p.areas + ab);
                const uint32_t* m4 = reinterpret_cast<const uint32_t*>(sh.mask);
                const int nq = MN >> 2;
                for (int q0 = lane; q0 < nq; q0 += 64 * kQuad) {
                    uint4 x[kQuad];
#pragma unroll
                    for (int u = 0; u < kQuad; ++u) {
                        const int q = q0 + 64 * u;
                        x[u] = q < nq ? a4[q] : make_uint4(0u, 0u, 0u, 0u);
                    }
#pragma unroll
                    for (int u = 0; u < kQuad; ++u) {
                        const int q = q0 + 64 * u;
                        if (q < nq) {
                            const uint32_t mk = m4[q];    // the four mask bytes of these samples
                            bad |= (mk & 0xFFu) && nonfinite_bits(x[u].x);
                            bad |= (mk & 0xFF00u) && nonfinite_bits(x[u].y);
                            bad |= (mk & 0xFF0000u) && nonfinite_bits(x[u].z);
                            bad |= (mk & 0xFF000000u) && nonfinite_bits(x[u].w);
                        }
                    }
                }
            } else {
                // kBatch samples per lane in flight
                for (int i0 = lane; i0 < MN; i0 += 64 * kBatch) {
                    uint32_t x[kBatch];
#pragma unroll
                    for (int u = 0; u < kBatch; ++u) {
                        const int i = i0 + 64 * u;
                        x[u] = i < MN ? sample_bits(p.areas, ab + i) : 0u;
                    }
#pragma unroll
                    for (int u = 0; u < kBatch; ++u) {
                        const int i = i0 + 64 * u;
                        if (i < MN && sh.mask[i]) bad |= nonfinite_bits(x[u]);
                    }
                }
            }
            if (__any(bad)) flags |= FOFSE_BLOCK_NONFINITE;
        }
        Rows R;
#pragma unroll
        for (int r = 0; r < kRC; ++r) {
            const int nu = lane + 64 * r;
            const bool valid = present && nu < K;
            // loaded without a per-row branch (index clamped into the block's
            // record; an empty record, K = 0, is never read) so that the loads
            // of every row are in flight together
            int key_l = 0;
            double2 c_l = make_double2(0.0, 0.0);
            if (K > 0) {
                const size_t ri = (size_t)bj * K + min(nu, K - 1);
                key_l = p.sel[ri];
                c_l = make_double2(p.coef[2 * ri], p.coef[2 * ri + 1]);
            }
            const int key = valid ? key_l & (T * T - 1) : 0;
            double2 c = valid ? c_l : make_double2(0.0, 0.0);
            R.x[r] = pack_class(key >> 6, key & 63);
            R.pr[r] = valid && packed_pair(R.x[r]);
            // a self-conjugate class has a real coefficient (the forward writes 0
            // for its imaginary part); halved, see zapply
            R.c[r] = R.pr[r] ? c : make_double2(0.5 * c.x, 0.0);
            R.cb[r] = make_double2(0.0, 0.0);
        }
        if (present && flags == 0) cbar0_rows(p, bj, lane, sh.buf + wave * 1024, sh.tw, R, K);
        __syncthreads();                         // H tables done

        // Z = DFT(w + j dw/drho) of the item's mask, natural order: every sample
        // of the area is written (0 off the support), the rest of the grid is
        // cleared, and the table loads are all issued before any is used
        {
            double2 wz[MAXPX];
#pragma unroll
            for (int q = 0; q < MAXPX; ++q) {
                const int i = min(tidv + q * NT, MN - 1);
                wz[q] = make_double2(p.wtab[i], p.dwtab[i]);
            }
            for (int e = tidv; e < T * T; e += NT) {
                const int m = e >> 6, n = e & (T - 1);
                if (m >= M || n >= N) sh.buf[e] = make_double2(0.0, 0.0);
            }
#pragma unroll
            for (int q = 0; q < MAXPX; ++q) {
                const int i = tidv + q * NT;
                if (i < MN) {
                    const int m = i / N, n = i - m * N;
                    sh.buf[m * T + n] = sh.mask[i] ? wz[q] : make_double2(0.0, 0.0);
                }
            }
        }
        __syncthreads();
        fft_stage_a<T, NT>(sh.buf, sh.tw, M, T, 1, tidv);
        __syncthreads();
        fft_stage_b<T, NT>(sh.buf, M, T, 1, tidv);
        __syncthreads();
        fft_stage_a<T, NT>(sh.buf, sh.tw, T, 1, T, tidv);
        __syncthreads();
        fft_stage_b<T, NT>(sh.buf, T, 1, T, tidv);
        __syncthreads();
        // FFT output order -> natural order: for T = 64 the order swaps the two
        // octal digits of each index, an involution
        for (int e = tidv; e < T * T; e += NT) {
            const int pe = FftPlan<T>::perm(e / T) * T + FftPlan<T>::perm(e % T);
            if (pe > e) {
                const double2 x = sh.buf[e], y = sh.buf[pe];
                sh.buf[e] = y;
                sh.buf[pe] = x;
            }
        }
        __syncthreads();
        const double W0 = sh.buf[0].x, dW0 = sh.buf[0].y;
        __syncthreads();
        if (params_ok && !(W0 > 0.0)) flags |= FOFSE_BLOCK_NO_SUPPORT;
        const bool live = present && flags == 0;
        if (lane == 0) sh.live[wave] = live ? 1 : 0;     // read after the output pass's first barrier
        const double hW = (params_ok && W0 > 0.0) ? 0.5 * gamma / W0 : 0.0;
        // Z' = hW Z, each row k rotated by 13 k columns (the skewed layout above);
        // one wavefront per row: its lanes read the row before any writes it
        for (int r = (tidv >> 6); r < T; r += NT / 64) {
            const double2 z = sh.buf[r * T + lane];
            sh.buf[r * T + ((lane + kSkew * r) & (T - 1))] = make_double2(hW * z.x, hW * z.y);
        }
        __syncthreads();

        // the transposed recurrence of this wavefront's block
        double racc = 0.0, tacc = 0.0;
        if (live) {
            chunk<3>(R, sh.buf, lane, K, racc);
            chunk<2>(R, sh.buf, lane, K, racc);
            chunk<1>(R, sh.buf, lane, K, racc);
            chunk<0>(R, sh.buf, lane, K, racc);
#pragma unroll
            for (int r = 0; r < kRC; ++r)
                if (lane + 64 * r < K)
                    tacc += (R.pr[r] ? 1.0 : 2.0) * (R.cb[r].x * R.c[r].x + R.cb[r].y * R.c[r].y);
        }

        // (w f)bar = Re FFT(Y), Y = conj(gamma / W0 cbar) summed per class.  Made
        // Hermitian, Yh = (Y(k) + conj Y(-k)) / 2, its transform x is real, and the
        // even and odd columns of x travel as one 64 x 32 complex transform:
        //   z[m][n'] = x[m][2n'] + j x[m][2n'+1] = FFT(C)[m][n'],
        //   C[k][l'] = Yh[k][l'] + Yh[k][l'+32] + j (Yh[k][l'] - Yh[k][l'+32]) w^l'
        // (w = exp(-j 2 pi / 64)).  Each block has its own 32 KB grid (two blocks
        // per pass) and its own fixed-point scale, so its result does not depend on
        // the other blocks of the work item.
        const double gW = 2.0 * hW;
        unsigned long long* acc = (unsigned long long*)sh.buf;
        for (int pp = 0; pp < 2; ++pp) {
            if (2 * pp >= nblk) break;           // uniform over the workgroup
            const bool mine = (wave >> 1) == pp;
            const int grid = wave & 1;
            __syncthreads();                     // Z' or the previous grids no longer read
            for (int i = tidv; i < 2 * T * T; i += NT) acc[i] = 0ull;
            if (mine) {
                uint32_t eb = 0;
                if (live) {
#pragma unroll
                    for (int r = 0; r < kRC; ++r)
                        if (lane + 64 * r < K) {
                            const uint32_t ex = (uint32_t)(__double2hiint(gW * R.cb[r].x) >> 20) & 0x7FF;
                            const uint32_t ey = (uint32_t)(__double2hiint(gW * R.cb[r].y) >> 20) & 0x7FF;
                            eb = max(eb, max(ex, ey));
                        }
                }
                eb = wave_max_u32(eb);
                // 2^e exceeds every |component| of Y; tiny or empty blocks use -900
                const int e = max(-900, (int)eb - 1022);
                if (lane == 0) sh.expo[wave] = e;
            }
            __syncthreads();
            if (mine && live) {
                // a term Y / 2 (1 +- j w^l') has components below 2^(e + 1): at
                // S = 2^(49 - e) below 2^50, and at most 4 K <= 2^10 terms meet in an entry
                const double S = pow2(49 - sh.expo[wave]);
                unsigned long long* ga = acc + grid * 2 * 2048;
                auto put = [&](int kk, int ll, double vr, double vi) {
                    const int lp = ll & 31;
                    const double2 w = sh.tw[lp];
                    const double sg = ll < 32 ? 1.0 : -1.0;
                    const double fr = 1.0 - sg * w.y, fi = sg * w.x;      // 1 +- j w^l'
                    const long long qr = __double2ll_rn((vr * fr - vi * fi) * S);
                    const long long qi = __double2ll_rn((vr * fi + vi * fr) * S);
                    atomicAdd(&ga[2 * (kk * 32 + lp)], (unsigned long long)qr);
                    atomicAdd(&ga[2 * (kk * 32 + lp) + 1], (unsigned long long)qi);
                };
#pragma unroll
                for (int r = 0; r < kRC; ++r) {
                    if (lane + 64 * r < K) {
                        const double yr = 0.5 * gW * R.cb[r].x, yi = -0.5 * gW * R.cb[r].y;
                        const int k = class_k(R.x[r]), l = class_l(R.x[r]);
                        put(k, l, yr, yi);                       // Y / 2 at (k, l)
                        put((-k) & 63, (-l) & 63, yr, -yi);      // conj(Y) / 2 at (-k, -l)
                    }
                }
            }
            __syncthreads();
            for (int i = tidv; i < T * T; i += NT) {
                const double U = pow2(sh.expo[2 * pp + (i >> 11)] - 49);
                const long long a = (long long)acc[2 * i], b = (long long)acc[2 * i + 1];
                sh.buf[i] = make_double2((double)a * U, (double)b * U);
            }
            __syncthreads();
            // 32-point transforms along the rows of both grids, then 64-point
            // transforms along the columns of each
            fft_stage_a<32, NT>(sh.buf, sh.tw32, 2 * T, 32, 1, tidv);
            __syncthreads();
            fft_stage_b<32, NT>(sh.buf, 2 * T, 32, 1, tidv);
            __syncthreads();
            fft_stage_a<T, NT>(sh.buf, sh.tw, 32, 1, 32, tidv);
            fft_stage_a<T, NT>(sh.buf + 2048, sh.tw, 32, 1, 32, tidv);
            __syncthreads();
            fft_stage_b<T, NT>(sh.buf, 32, 1, 32, tidv);
            fft_stage_b<T, NT>(sh.buf + 2048, 32, 1, 32, tidv);
            __syncthreads();
            // dL/df = w (w f)bar on A and the rho term of R0 = DFT(w f) for the
            // two blocks of the pass, each by its own wavefront and one of the
            // other pass (every other group of 64 samples); the helper's rho
            // terms go to rpart.  kBatch samples per lane in flight.
            {
                const int slot = 2 * pp + (wave & 1);
                const int help = (wave >> 1) != pp ? 1 : 0;
                if (slot < nblk) {
                    const int bs = slot == 0 ? b0 : slot == 1 ? b1 : slot == 2 ? b2 : b3;
                    const size_t abs = (size_t)bs * MN;
                    const bool lv = sh.live[slot] != 0;
                    const double2* zg = sh.buf + (slot & 1) * 2048;
                    double rr = 0.0;
                    for (int i0 = lane + 64 * help; i0 < MN; i0 += 128 * kBatch) {
                        double w[kBatch], dw[kBatch];
                        float x[kBatch];
#pragma unroll
                        for (int u = 0; u < kBatch; ++u) {
                            const int i = i0 + 128 * u;
                            const bool in = lv && i < MN;
                            w[u] = in ? p.wtab[i] : 0.0;
                            dw[u] = in ? p.dwtab[i] : 0.0;
                            x[u] = in ? p.areas[abs + i] : 0.0f;
                        }
#pragma unroll
                        for (int u = 0; u < kBatch; ++u) {
                            const int i = i0 + 128 * u;
                            if (i < MN) {
                                float gv = 0.0f;
                                if (lv && sh.mask[i]) {
                                    const int m = i / N, n = i - m * N;
                                    const double2 v = zg[FftPlan<T>::perm(m) * 32 + FftPlan<32>::perm(n >> 1)];
                                    const double wfb = (n & 1) ? v.y : v.x;
                                    gv = (float)(w[u] * wfb);
                                    rr += dw[u] * (double)x[u] * wfb;
                                }
                                if (p.grad_areas) p.grad_areas[abs + i] = gv;
                            }
                        }
                    }
                    if (help) sh.rpart[slot][lane] = rr;
                    else racc += rr;
                }
            }
        }
        __syncthreads();                         // the helpers' rho terms are in rpart
        if (present) racc += sh.rpart[wave][lane];
        if (present) {
            racc = wave_sum(racc);
            tacc = wave_sum(tacc);
            if (lane == 0) {
                if (live) {
                    p.grad_block[2 * bj] = racc - tacc / W0 * dW0;   // W0 = sum w: dW0/drho = sum dw
                    p.grad_block[2 * bj + 1] = tacc / gamma;
                } else {
                    p.grad_block[2 * bj] = 0.0;
                    p.grad_block[2 * bj + 1] = 0.0;
                }
            }
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

hipError_t launch_backward_grouped(const KParams& wp, const BParams& p, const GroupArgs& g, int n_cu,
                                   double* d_sum, hipStream_t stream, const Timing& tm) {
    if (p.T != 64 || p.K > kGroupBackwardMaxK || p.M * p.N > 16 * 64 * kGroup) return hipErrorInvalidValue;
    hipError_t e = launch_weights(wp, stream);
    if (e != hipSuccess) return e;
    GroupArgs ga = g;
    ga.gsize = kGroup;
    ga.gshift = kGroupShift;
    if (!g.direct) {
        e = launch_grouping(ga, p.n_blocks, stream);
        if (e != hipSuccess) return e;
    }
    const int max_items = g.direct ? (p.n_blocks + kGroup - 1) / kGroup : p.n_blocks;
    int grid = (g.wg_per_cu > 0 ? g.wg_per_cu : 2) * n_cu;     // two fit per compute unit
    if (grid > max_items) grid = max_items;
    ga.n_wg = grid;
    constexpr int NT = 64 * kGroup;
    if (tm.start && hipEventRecord(tm.start, stream) != hipSuccess) return hipErrorUnknown;
    if (p.M * p.N <= 9 * NT)
        hipLaunchKernelGGL((fofse_bwd_group_kernel<9>), dim3(grid), dim3(NT), 0, stream, p, ga);
    else
        hipLaunchKernelGGL((fofse_bwd_group_kernel<16>), dim3(grid), dim3(NT), 0, stream, p, ga);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (tm.stop && hipEventRecord(tm.stop, stream) != hipSuccess) return hipErrorUnknown;
    return d_sum ? launch_bwd_sum(p, d_sum, stream) : hipSuccess;
}

}  // namespace fofse
