// FOFSE with the two-dimensional DCT as its set of basis functions: the
// variant that, like the DFT one, runs entirely in the transform domain
// (Section 2, after eq. 9).
//
// Basis phi_{k,l}[m,n] = a_k a_l C(k, m) C(l, n), C(a, m) = cos(pi a (2m+1) /
// (2T)), a_0 = sqrt(1/T), a_k = sqrt(2/T): the orthonormal DCT-II of the T x T
// grid (T = 16, 32 or 64), the area at its origin.  Per block:
//   R = DCT(w f)                                          (eqs. 7, 8)
//   K times: u = argmax |R|, ties to the smallest k*T + l  (eq. 9)
//            c = gamma R[u] / <phi_u, phi_u>_w             (eqs. 5, 14)
//            R[k] -= c <w phi_u, phi_k> for every k        (eq. 3)
//   g on B = sum of c phi_u                                (eqs. 1, 2)
//
// Gram entries from one table.  cos x cos y = (cos(x - y) + cos(x + y)) / 2 in
// each dimension gives
//   <w phi_u, phi_k> = a_k1 a_k2 a_u1 a_u2 / 4 * sum_{s1,s2 = +-1} Wc[k1 + s1 u1][k2 + s2 u2]
// with Wc[a][b] = sum_A w C(a, m) C(b, n).  As C(-a) = C(a), C(2T - a) = -C(a)
// and C(T) = 0, every index in (-T, 2T) folds into [0, T] with a sign, so the
// table holds Wc on [0, T] x [0, T] (row and column T are zero).
//
// Organisation.  One wavefront per block: lane = column index l, register slot
// = row index k (T doubles per lane; lanes T..63 idle for T < 64).  Blocks with one support mask share w
// and so the table; a workgroup of eight wavefronts takes up to eight of them
// (one or two work items of the device-side grouping) and builds the table
// once.  Per iteration a lane needs four table entries per slot: two columns
// (|l - v| and the fold of l + v, fixed for the lane) in two rows (k - u and
// k + u, uniform for the slot).  The table is stored row-extended (rows -T ..
// 2T - 1, the row fold and its sign applied), so that both rows advance with the
// slot: every read is at a compile-time offset from four per-iteration
// addresses, and a row's 64 columns are consecutive doubles (8-byte reads
// without bank conflicts).  The iteration loop has no barrier.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dct_kernel.h"
#include "device_common.hpp"

namespace fofse {

namespace {

constexpr int kWv = 8;                      // wavefronts (blocks) per workgroup
constexpr int kNT = 64 * kWv;
constexpr int kAhead = 6;                   // slots whose table reads are in flight
static_assert(2 * kGroup == kWv, "a workgroup takes two work items of the grouping");

typedef double d16 __attribute__((ext_vector_type(16)));

// Sizes for grid size T, and the normalisation a_0 = sqrt(1/T), a_k = sqrt(2/T).
template <int T> struct Dct;
template <> struct Dct<16> { static constexpr double a0 = 0.25, a1 = 0.3535533905932738; static constexpr int lg = 4; };
template <> struct Dct<32> { static constexpr double a0 = 0.1767766952966369, a1 = 0.25; static constexpr int lg = 5; };
template <> struct Dct<64> { static constexpr double a0 = 0.125, a1 = 0.1767766952966369; static constexpr int lg = 6; };

template <int T>
struct DctSize {
    static constexpr int RW = T / kWv;      // rows per wavefront in the transforms
    static constexpr int TP = T + 1;        // row stride of the column pass
    static constexpr int BufLen = T * TP;   // >= T * T
    static constexpr int Rows = 3 * T;      // rows of the extended table (-T .. 2T - 1)
    static constexpr int CS = T + 1;        // row stride of the synthesis cosine table
    static constexpr int NCH = T / 16;      // register chunks of R
    static_assert(BufLen + T * T <= Rows * T, "column pass and staging fit in the table's space");
};

// E[a][b] = Wc[a][b] for 0 <= a < T, Wc[-a][b] for -T < a < 0, -Wc[2T - a][b]
// for T < a < 2T, 0 for a = +-T; columns b < T (column T is 0).  E[a][b] is
// ext[(a + T) * T + b].
template <int T>
struct DctShared {
    double ext[DctSize<T>::Rows * T];   // while the blocks are transformed: column pass + one block's R
    double cs[T * DctSize<T>::CS];      // C(u, m) at [u * CS + m], for the synthesis
    int flags[kWv];
};

template <int T>
__device__ __forceinline__ int ext_index(int a, int b) { return (a + T) * T + b; }

__device__ __forceinline__ bool known_sample(const uint8_t* known, const uint8_t* target, size_t base, int i) {
    return target[i] == 0 && (known == nullptr || known[base + i] != 0);
}

// P[n][k] = sum_m C(k, m) X[m][n] for n < N and the RW rows k of wave wv, with
// X = w on the support of the item's mask, times f of block b when b >= 0.
// Written to buf[n * TP + k].  A non-finite known sample of block b sets
// FOFSE_BLOCK_NONFINITE in *flag (its contribution is 0).
template <int T>
__device__ __forceinline__ void column_pass(double* buf, const KParams& p, const GroupArgs& g, size_t rep_base,
                                            int b, int* flag, const double* __restrict__ cosm, int wv, int lane) {
    constexpr int RW = DctSize<T>::RW, TP = DctSize<T>::TP;
    const int M = p.M, N = p.N, MN = M * N;
    const bool col = lane < N;
    double acc[RW];
#pragma unroll
    for (int j = 0; j < RW; ++j) acc[j] = 0.0;
    for (int m = 0; m < M; ++m) {
        double x = 0.0;
        if (col) {
            const int i = m * N + lane;
            if (known_sample(g.known, p.target, rep_base, i)) {
                const double w = p.wtab[i];
                if (b < 0) {
                    x = w;
                } else {
                    const uint32_t xb = sample_bits(p.areas, (size_t)b * MN + i);
                    if (nonfinite_bits(xb)) atomicOr(flag, FOFSE_BLOCK_NONFINITE);
                    else x = w * (double)__uint_as_float(xb);
                }
            }
        }
        const double* cr = cosm + m * T + RW * wv;        // C(RW wv + j, m), uniform
#pragma unroll
        for (int j = 0; j < RW; ++j) acc[j] = fma(cr[j], x, acc[j]);
    }
    if (col) {
#pragma unroll
        for (int j = 0; j < RW; ++j) buf[lane * TP + RW * wv + j] = acc[j];
    }
}

// acc[j] = sum_{n < N} P[n][RW wv + j] C(l, n) for the lane's column l < T.
template <int T>
__device__ __forceinline__ void row_pass(double (&acc)[DctSize<T>::RW], const double* buf, int N,
                                         const double* __restrict__ cosm, int wv, int lane) {
    constexpr int RW = DctSize<T>::RW, TP = DctSize<T>::TP;
#pragma unroll
    for (int j = 0; j < RW; ++j) acc[j] = 0.0;
    for (int n = 0; n < N; ++n) {
        const double c = lane < T ? cosm[n * T + lane] : 0.0;
        const double* pr = buf + n * TP + RW * wv;         // uniform: broadcast reads
#pragma unroll
        for (int j = 0; j < RW; ++j) acc[j] = fma(pr[j], c, acc[j]);
    }
}

// Selection key of slot k: |R| with its 6 lowest mantissa bits replaced by
// 63 - k (the magnitude changes by < 2^-46 relative); a larger key is a larger
// magnitude, or the same magnitude in a smaller row.
__device__ __forceinline__ double key_of(double r, int k) {
    const uint32_t lo = ((uint32_t)__double2loint(r) & 0xFFFFFFC0u) | (uint32_t)(63 - k);
    return __hiloint2double(__double2hiint(r), (int)lo);
}

// max(best, |key|) as one v_max_f64 with an absolute-value source modifier.
__device__ __forceinline__ double max_abs(double best, double key) {
    double r;
    asm("v_max_f64 %0, |%1|, %2" : "=v"(r) : "v"(key), "v"(best));
    return r;
}

// R of slot k (uniform) in lane `lane` (uniform), by a tree of uniform
// branches down to a plain register read (a run-time register index would put
// R in scratch memory).
template <int LO, int HI, int NCH>
__device__ __forceinline__ double fetch_slot(const d16 (&R)[NCH], int k, int lane) {
    if constexpr (HI - LO == 1) {
        return readlane_f64(R[LO >> 4][LO & 15], lane);
    } else {
        constexpr int MID = (LO + HI) / 2;
        if (k < MID) return fetch_slot<LO, MID, NCH>(R, k, lane);
        return fetch_slot<MID, HI, NCH>(R, k, lane);
    }
}

// R[k][l] -= q_k <Gram sum> for the T rows of column l = lane, and the largest
// key.  t[0..3] point at the entries of slot 0 (rows -u and u in the columns
// |l - v| and fold(l + v)); slot k reads T k doubles further on.
template <int T>
__device__ __forceinline__ double update_rows(d16 (&R)[DctSize<T>::NCH], const double* const (&t)[4], double sgnB,
                                              double q0, double q1) {
    constexpr int NB = kAhead + 1;
    double x[NB][4];
    auto load = [&](int k, double* y) {
#pragma unroll
        for (int q = 0; q < 4; ++q) y[q] = t[q][k * T];
    };
#pragma unroll
    for (int k = 0; k < kAhead; ++k) load(k, x[k]);
    double best = 0.0;
#pragma unroll
    for (int k = 0; k < T; ++k) {
        if (k + kAhead < T) load(k + kAhead, x[(k + kAhead) % NB]);
        const double* y = x[k % NB];
        const double s = fma(sgnB, y[1], y[0]) + fma(sgnB, y[3], y[2]);
        const double r = fma(k == 0 ? -q0 : -q1, s, R[k >> 4][k & 15]);
        R[k >> 4][k & 15] = r;
        best = max_abs(best, key_of(r, k));
        __builtin_amdgcn_sched_barrier(0);
    }
    return best;
}

// The K iterations of one block held by this wavefront (R: slot k of chunk
// k / 16 at element k % 16).  Writes the selection record of block b.  Lanes
// T..63 (T < 64) carry no column: they read column 0 and take no part in the
// selection.
template <int T>
__device__ __forceinline__ void dct_iterate(d16 (&R)[DctSize<T>::NCH], const double* e, const KParams& p, int b,
                                            int lane, double gamma) {
    constexpr double A0 = Dct<T>::a0, A1 = Dct<T>::a1;
    const int K = p.K;
    const bool col = lane < T;
    const double al = lane == 0 ? A0 : A1;
    int u = 0, v = 0;
    double q0 = 0.0, q1 = 0.0;          // update scale of row 0 and of rows 1..T-1 in this column
    for (int it = 0;; ++it) {
        // Pass 0 runs with c = 0 (R unchanged).
        const int cA = !col ? 0 : lane >= v ? lane - v : v - lane;
        const int sb = lane + v;
        const int cB = !col ? 0 : sb < T ? sb : (sb == T ? 0 : 2 * T - sb);
        const double sgnB = !col ? 0.0 : sb < T ? 1.0 : (sb == T ? 0.0 : -1.0);
        const double* t[4] = {e + ext_index<T>(-u, cA), e + ext_index<T>(-u, cB), e + ext_index<T>(u, cA),
                              e + ext_index<T>(u, cB)};
        double best = update_rows<T>(R, t, sgnB, q0, q1);
        if (!col) best = 0.0;
        if (it == K) break;

        // eq. 9 over the wavefront: the largest high word, then among those the
        // largest low word (magnitude bits and 63 - row), then the smallest lane
        const uint32_t bhi = (uint32_t)__double2hiint(best), blo = (uint32_t)__double2loint(best);
        const uint32_t mhi = wave_max_u32(bhi);
        const uint32_t mlo = wave_max_u32(bhi == mhi ? blo : 0u);
        const uint64_t hits = __ballot(bhi == mhi && blo == mlo);
        const int vl = __builtin_amdgcn_readfirstlane((int)__builtin_ctzll(hits));
        const int uk = __builtin_amdgcn_readfirstlane(63 - (int)(mlo & 63u));
        const double Ru = fetch_slot<0, T, DctSize<T>::NCH>(R, uk, vl);

        // eq. 5: <phi_u, phi_u>_w is the Gram entry at k = u (rows 0 and 2u,
        // columns 0 and 2v of Wc); eq. 14: c = gamma p
        const int d1 = 2 * uk, d2 = 2 * vl;
        const int f1 = d1 <= T ? d1 : 2 * T - d1, f2 = d2 <= T ? d2 : 2 * T - d2;
        const double s1 = d1 <= T ? 1.0 : -1.0, s2 = d2 <= T ? 1.0 : -1.0;
        const double w00 = e[ext_index<T>(0, 0)];
        const double w02 = f2 < T ? e[ext_index<T>(0, f2)] : 0.0;
        const double w10 = e[ext_index<T>(f1, 0)];              // row T of E is 0
        const double w12 = f2 < T ? e[ext_index<T>(f1, f2)] : 0.0;
        const double wsum = w00 + s2 * w02 + s1 * (w10 + s2 * w12);
        const double au1 = uk == 0 ? A0 : A1, au2 = vl == 0 ? A0 : A1;
        const double S = 0.25 * (au1 * au1) * (au2 * au2) * wsum;
        const double c = S > 0.0 ? gamma * Ru / S : 0.0;
        if (lane == 0) {
            const size_t r = (size_t)b * K + it;
            p.sel[r] = uk * T + vl;
            p.coef[2 * r] = c;
            p.coef[2 * r + 1] = 0.0;
        }
        const double q = 0.25 * c * au1 * au2;
        q0 = q * al * A0;
        q1 = q * al * A1;
        u = uk;
        v = vl;
    }
}

// g on B = sum_nu c_nu phi_{u_nu} from the record this wavefront wrote (read
// back with cache-bypassing loads after the release fence); cs holds C(u, m)
// at [u * CS + m], so that lanes of different pixels read different banks.
template <int T>
__device__ __forceinline__ void dct_synthesis(const double* cs, const KParams& p, int b, int lane) {
    constexpr int CS = DctSize<T>::CS, LG = Dct<T>::lg;
    constexpr double A0 = Dct<T>::a0, A1 = Dct<T>::a1;
    const int K = p.K, N = p.N, nB = p.nB;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    const volatile int32_t* sel = p.sel + (size_t)b * K;
    const volatile double* coef = p.coef + 2 * (size_t)b * K;
    for (int q0 = 0; q0 < nB; q0 += 64) {
        const int q = q0 + lane;
        const bool ok = q < nB;
        const int i = ok ? p.bpix[q] : 0;
        const int m = i / N, n = i - m * N;
        double acc = 0.0;
        for (int nu0 = 0; nu0 < K; nu0 += 64) {
            const int nu = nu0 + lane;
            int key = 0;
            double c = 0.0;
            if (nu < K) {
                key = sel[nu];
                c = coef[2 * nu];
            }
            const int cnt = K - nu0 < 64 ? K - nu0 : 64;
            for (int j = 0; j < cnt; ++j) {
                const int kj = __builtin_amdgcn_readlane(key, j);
                const double cj = readlane_f64(c, j);
                const int u1 = (kj >> LG) & (T - 1), u2 = kj & (T - 1);
                const double s = cj * (u1 == 0 ? A0 : A1) * (u2 == 0 ? A0 : A1);
                acc = fma(s, cs[u1 * CS + m] * cs[u2 * CS + n], acc);
            }
        }
        if (ok) p.out[(size_t)b * nB + q] = (float)acc;
    }
}

// Up to kWv blocks of one support mask, blk[0 .. nblk).
template <int T>
__device__ __forceinline__ void dct_item(DctShared<T>& sh, const KParams& p, const GroupArgs& g,
                                         const double* __restrict__ cosm, const int (&blk)[kWv], int nblk,
                                         int tid, int lane, int wv, bool params_ok, double gamma) {
    using Z = DctSize<T>;
    constexpr int RW = Z::RW, NCH = Z::NCH;
    constexpr double A0 = Dct<T>::a0, A1 = Dct<T>::a1;
    const int MN = p.M * p.N, N = p.N, K = p.K;
    const size_t rep_base = (size_t)blk[0] * MN;    // every block of the item has this mask
    double* buf = sh.ext;
    double* stage = buf + Z::BufLen;
    double* e = buf;
    __syncthreads();                                 // the previous item is done with the LDS
    if (tid < kWv) sh.flags[tid] = params_ok ? 0 : FOFSE_BLOCK_BAD_PARAM;
    __syncthreads();

    d16 R[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) R[c] = (d16)0.0;
    if (params_ok) {
        // R = DCT(w f) of each block (eqs. 7, 8), staged in the table's space
        const double al = lane == 0 ? A0 : A1;
        for (int j = 0; j < kWv; ++j) {
            if (j >= nblk) break;                    // uniform over the workgroup
            column_pass<T>(buf, p, g, rep_base, blk[j], &sh.flags[j], cosm, wv, lane);
            __syncthreads();
            double acc[RW];
            row_pass<T>(acc, buf, N, cosm, wv, lane);
            if (lane < T) {
#pragma unroll
                for (int jj = 0; jj < RW; ++jj) {
                    const int k = RW * wv + jj;
                    stage[k * T + lane] = acc[jj] * al * (k == 0 ? A0 : A1);
                }
            }
            __syncthreads();
            if (wv == j && lane < T) {
#pragma unroll
                for (int k = 0; k < T; ++k) R[k >> 4][k & 15] = stage[k * T + lane];
            }
        }
        // the table Wc of the item's w, written row-extended once every read
        // of the column pass and of the staging is done
        column_pass<T>(buf, p, g, rep_base, -1, nullptr, cosm, wv, lane);
        __syncthreads();
        double acc[RW];
        row_pass<T>(acc, buf, N, cosm, wv, lane);
        __syncthreads();
        if (lane < T) {
#pragma unroll
            for (int jj = 0; jj < RW; ++jj) {
                const int k = RW * wv + jj;
                e[ext_index<T>(k, lane)] = acc[jj];
                e[ext_index<T>(-k, lane)] = acc[jj];
                if (k > 0) e[ext_index<T>(2 * T - k, lane)] = -acc[jj];
            }
        }
        if (tid < T) {
            e[ext_index<T>(T, tid)] = 0.0;
            e[ext_index<T>(-T, tid)] = 0.0;
        }
        __syncthreads();
    }

    const bool present = wv < nblk;
    int flags = present ? sh.flags[wv] : 0;
    const double W0 = params_ok ? e[ext_index<T>(0, 0)] : 0.0;   // Wc[0][0] = sum of the weights
    if (params_ok && !(W0 > 0.0)) flags |= FOFSE_BLOCK_NO_SUPPORT;
    const bool live = present && flags == 0;
    int bj = blk[0];                                 // blk[wv] without a run-time register index
#pragma unroll
    for (int j = 1; j < kWv; ++j) bj = wv == j ? blk[j] : bj;
    if (live) {
        dct_iterate<T>(R, e, p, bj, lane, gamma);
        dct_synthesis<T>(sh.cs, p, bj, lane);
    } else if (present) {                            // empty record, model 0
        for (int it = lane; it < K; it += 64) {
            const size_t r = (size_t)bj * K + it;
            p.sel[r] = 0;
            p.coef[2 * r] = 0.0;
            p.coef[2 * r + 1] = 0.0;
        }
        for (int q = lane; q < p.nB; q += 64) p.out[(size_t)bj * p.nB + q] = 0.0f;
    }
    if (present && lane == 0 && p.status) p.status[bj] = flags;
}

// Each workgroup takes a contiguous range of the grouping's work items (up to
// kGroup blocks of one mask each) and runs them one at a time, or two at a
// time when the next item of the range has the same mask (then the first one
// is full: only the last item of a class can be partial).  Without a known
// array every block has the one mask and the items are kWv consecutive blocks.
template <int T>
__global__ __launch_bounds__(kNT, 1) void fofse_dct_kernel(KParams p, GroupArgs g,
                                                            const double* __restrict__ cosm) {
    __shared__ DctShared<T> sh;
    constexpr int CS = DctSize<T>::CS;
    const int tid = (int)__builtin_amdgcn_workitem_id_x(), lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const double rho = p.rho_gamma[0], gamma = p.rho_gamma[1];
    const bool params_ok = param_ok(rho) && param_ok(gamma);
    for (int i = tid; i < T * T; i += kNT)                          // visible after the first item's barrier
        sh.cs[(i & (T - 1)) * CS + (i >> Dct<T>::lg)] = cosm[i];
    const int n_items = g.direct ? (p.n_blocks + kWv - 1) / kWv : g.counts[1];
    const int per = (n_items + g.n_wg - 1) / g.n_wg;
    const int i0 = (int)__builtin_amdgcn_workgroup_id_x() * per;
    const int i1 = min(n_items, i0 + per);
    for (int item = i0; item < i1;) {
        int nblk, blk[kWv];
        if (g.direct) {
            nblk = min(kWv, p.n_blocks - item * kWv);
#pragma unroll
            for (int j = 0; j < kWv; ++j) blk[j] = item * kWv + (j < nblk ? j : 0);
            item += 1;
        } else {
            const int n0 = g.item_n[item];
            const int cls = g.item_cls[item];
            const bool two = item + 1 < i1 && n0 == kGroup && cls >= 0 && g.item_cls[item + 1] == cls;
            const int n1 = two ? g.item_n[item + 1] : 0;
            nblk = n0 + n1;
#pragma unroll
            for (int j = 0; j < kGroup; ++j) {
                blk[j] = g.item_blk[(size_t)item * kGroup + (j < n0 ? j : 0)];
                blk[kGroup + j] = two && j < n1 ? g.item_blk[(size_t)(item + 1) * kGroup + j] : blk[0];
            }
            item += two ? 2 : 1;
        }
        dct_item<T>(sh, p, g, cosm, blk, nblk, tid, lane, wv, params_ok, gamma);
    }
}

}  // namespace

bool dct_size_supported(int T) { return T == 16 || T == 32 || T == 64; }

hipError_t launch_dct(const KParams& p, const GroupArgs& g, const double* cosm, int n_cu, hipStream_t stream,
                      const Timing& tm) {
    if (!dct_size_supported(p.T) || p.M > p.T || p.N > p.T || !cosm) return hipErrorInvalidValue;
    const hipError_t ew = launch_weights(p, stream);
    if (ew != hipSuccess) return ew;
    GroupArgs ga = g;
    ga.gsize = kGroup;
    ga.gshift = kGroupShift;
    if (!g.direct) {
        const hipError_t eg = launch_grouping(ga, p.n_blocks, stream);
        if (eg != hipSuccess) return eg;
    }
    // one workgroup per compute unit
    const int max_items = g.direct ? (p.n_blocks + kWv - 1) / kWv : p.n_blocks;
    int grid = n_cu;
    if (grid > max_items) grid = max_items;
    ga.n_wg = grid;
    if (tm.start && hipEventRecord(tm.start, stream) != hipSuccess) return hipErrorUnknown;
    if (p.T == 64) hipLaunchKernelGGL(fofse_dct_kernel<64>, dim3(grid), dim3(kNT), 0, stream, p, ga, cosm);
    else if (p.T == 32) hipLaunchKernelGGL(fofse_dct_kernel<32>, dim3(grid), dim3(kNT), 0, stream, p, ga, cosm);
    else hipLaunchKernelGGL(fofse_dct_kernel<16>, dim3(grid), dim3(kNT), 0, stream, p, ga, cosm);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (tm.stop && hipEventRecord(tm.stop, stream) != hipSuccess) return hipErrorUnknown;
    return hipSuccess;
}

}  // namespace fofse
