// Grouped FOFSE forward for gfx950: blocks whose support areas have the same
// known-sample mask share one weighting function w, hence one W = DFT(w)
// (eq. 4 / eq. 15 depend only on the mask).  A workgroup takes up to kGroup
// such blocks, keeps ONE W window in LDS for all of them and gives each block a
// whole wavefront: lane = grid column, register slot = grid row 0..T/2.  The
// iteration (eqs. 3, 5, 9, 14 in the DFT domain; eqs. 1, 2 for the model) then
// runs with no cross-wave exchange at all.
//
// Grouping runs on the device:
//   k_mask_hash   64-bit hash of each block's mask, inserted into an open-address
//                 table (the first inserter becomes the class representative)
//   k_group_count exact byte comparison with the representative (blocks that
//                 differ from their representative on a hash collision become
//                 singletons)
//   k_group_pos   position of each block inside its class (one atomic per
//                 distinct class of a wavefront of blocks)
//   k_group_scan  work items per class (ceil(count / gsize)) -> item offsets
//   k_group_fill  item -> list of its blocks
// The main kernel is persistent: workgroup g processes a contiguous range of
// items, so consecutive items of one class land on the same workgroup.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_common.hpp"
#include "fofse_kernel.h"
#include "iterate.hpp"

namespace fofse {

// ---------------------------------------------------------------------------
// grouping kernels (one wavefront per block unless stated)
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    // splitmix64 finaliser
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ bool eff_known(const uint8_t* known, const uint8_t* target, size_t base, int i) {
    return target[i] == 0 && (known == nullptr || known[base + i] != 0);
}

// Support bits of 16 consecutive samples from 16 bytes of the known mask and 16
// of the target mask: bit j set when sample 16 c + j is known and off B.
__device__ __forceinline__ uint32_t nz_bytes(uint32_t x) {      // high bit of each non-zero byte
    return (((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | x) & 0x80808080u;
}
__device__ __forceinline__ uint32_t pack_hi_bits(uint32_t e) {  // bits 7, 15, 23, 31 -> 0..3
    return ((e >> 7) & 1u) | ((e >> 14) & 2u) | ((e >> 21) & 4u) | ((e >> 28) & 8u);
}
__device__ __forceinline__ uint32_t support_bits16(uint4 kn, uint4 tg) {
    return pack_hi_bits(nz_bytes(kn.x) & ~nz_bytes(tg.x)) | (pack_hi_bits(nz_bytes(kn.y) & ~nz_bytes(tg.y)) << 4) |
           (pack_hi_bits(nz_bytes(kn.z) & ~nz_bytes(tg.z)) << 8) | (pack_hi_bits(nz_bytes(kn.w) & ~nz_bytes(tg.w)) << 12);
}

__device__ __forceinline__ uint64_t wave_xor_u64(uint64_t v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, off, 64);
        const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), off, 64);
        v ^= ((uint64_t)hi << 32) | lo;
    }
    return v;
}

// grouping kernels run one wavefront per block, kHashBlocks blocks per workgroup
constexpr int kHashBlocks = 4;

__global__ __launch_bounds__(64 * kHashBlocks) void k_mask_hash(GroupArgs g, int n) {
    const int tid = (int)__builtin_amdgcn_workitem_id_x();
    const int b = (int)__builtin_amdgcn_workgroup_id_x() * kHashBlocks + (tid >> 6), lane = tid & 63;
    if (b >= n) return;
    const size_t base = (size_t)b * g.MN;
    uint64_t h = 0;
    if (g.vec16) {          // 16 samples per load: hash of (chunk index, support bits)
        const uint4* kn = reinterpret_cast<const uint4*>(g.known + base);
        const uint4* tg = reinterpret_cast<const uint4*>(g.target);
        for (int c = lane; c < (g.MN >> 4); c += 64)
            h ^= mix64(((uint64_t)c << 16) | support_bits16(kn[c], tg[c]));
    } else {
        for (int i = lane; i < g.MN; i += 64)
            if (eff_known(g.known, g.target, base, i)) h ^= mix64((uint64_t)i);
    }
    h = wave_xor_u64(h) | 1ull;          // 0 marks an empty table slot
    if (lane == 0) {
        uint32_t slot = (uint32_t)(h >> 17) & g.hmask;
        for (;;) {
            // most blocks find their class already inserted: a plain read first
            // keeps them off the atomic unit (a stale 0 just falls through to the
            // compare-and-swap, which decides)
            const unsigned long long seen =
                __hip_atomic_load(&g.ht_key[slot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (seen == h) break;
            if (seen == 0ull) {
                const unsigned long long prev = atomicCAS(&g.ht_key[slot], 0ull, (unsigned long long)h);
                if (prev == 0ull) { g.ht_rep[slot] = b; break; }
                if (prev == h) break;
            }
            slot = (slot + 1) & g.hmask;
        }
        g.cls[b] = (int)slot;
    }
}

__global__ __launch_bounds__(64 * kHashBlocks) void k_group_count(GroupArgs g, int n) {
    const int tid = (int)__builtin_amdgcn_workitem_id_x();
    const int b = (int)__builtin_amdgcn_workgroup_id_x() * kHashBlocks + (tid >> 6), lane = tid & 63;
    if (b >= n) return;
    const int slot = g.cls[b];
    const int rep = g.ht_rep[slot];
    const size_t base = (size_t)b * g.MN, rbase = (size_t)rep * g.MN;
    bool same = true;
    if (g.vec16) {
        const uint4* kb = reinterpret_cast<const uint4*>(g.known + base);
        const uint4* kr = reinterpret_cast<const uint4*>(g.known + rbase);
        const uint4* tg = reinterpret_cast<const uint4*>(g.target);
        for (int c = lane; c < (g.MN >> 4); c += 64) {
            const uint4 t = tg[c];
            same = same && support_bits16(kb[c], t) == support_bits16(kr[c], t);
        }
    } else {
        for (int i = lane; i < g.MN; i += 64)
            same = same && (eff_known(g.known, g.target, base, i) == eff_known(g.known, g.target, rbase, i));
    }
    same = __all(same);
    if (lane == 0 && !same) g.cls[b] = -1;
}

// One thread per block: its position inside its class (or among the
// singletons).  The lanes of a wavefront that share a class take consecutive
// positions from one atomic add.
__global__ __launch_bounds__(256) void k_group_pos(GroupArgs g, int n) {
    const int b = (int)__builtin_amdgcn_workgroup_id_x() * 256 + (int)__builtin_amdgcn_workitem_id_x();
    const int lane = (int)__builtin_amdgcn_workitem_id_x() & 63;
    const bool valid = b < n;
    const int slot = valid ? g.cls[b] : 0;
    uint64_t todo = __ballot(valid);
    int pos = 0;
    while (todo) {
        const int leader = (int)__builtin_ctzll(todo);
        const int s = __builtin_amdgcn_readlane(slot, leader);
        const uint64_t m = __ballot(valid && slot == s);
        int base = 0;
        if (lane == leader) base = atomicAdd(s >= 0 ? &g.ht_cnt[s] : g.n_single, (int)__popcll(m));
        base = __builtin_amdgcn_readlane(base, leader);
        if (valid && slot == s) pos = base + (int)__popcll(m & ((1ull << lane) - 1ull));
        todo &= ~m;
    }
    if (valid) g.pos[b] = pos;
}

__device__ __forceinline__ int wave_sum_i32(int v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// One workgroup of 1024 threads: items per slot and their exclusive prefix.
// Wave w owns the slots [w P, (w + 1) P), P = hsize / 16 (hsize is a power of
// two >= 64), read 64 at a time (coalesced): a first pass sums them, the wave
// offsets follow from the 16 sums, a second pass scans each group of 64.
__global__ __launch_bounds__(1024) void k_group_scan(GroupArgs g) {
    __shared__ int wtot[16];
    const int tid = (int)__builtin_amdgcn_workitem_id_x(), lane = tid & 63, w = tid >> 6;
    const int P = g.hsize >> 4;
    const int start = w * P, end = start + P;
    int tot = 0;
#pragma unroll 4
    for (int c = start + lane; c < end; c += 64) tot += (g.ht_cnt[c] + g.gsize - 1) >> g.gshift;
    tot = wave_sum_i32(tot);
    if (lane == 0) wtot[w] = tot;
    __syncthreads();
    int carry = 0, all = 0;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        carry += i < w ? wtot[i] : 0;
        all += wtot[i];
    }
    for (int c0 = start; c0 < end; c0 += 64) {
        const int c = c0 + lane;
        const int x = c < end ? (g.ht_cnt[c] + g.gsize - 1) >> g.gshift : 0;
        int incl = x;                                 // inclusive scan over the wavefront
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int y = __shfl_up(incl, off, 64);
            incl += lane >= off ? y : 0;
        }
        if (c < end) g.item_start[c] = carry + incl - x;
        carry += __builtin_amdgcn_readlane(incl, 63);
    }
    if (tid == 0) {
        g.counts[0] = all;                            // grouped items
        g.counts[1] = all + *g.n_single;              // all items
        g.counts[2] = 0;                              // next item of the main kernel's queue
    }
}

__global__ void k_group_fill(GroupArgs g, int n) {
    const int b = (int)__builtin_amdgcn_workgroup_id_x() * 256 + (int)__builtin_amdgcn_workitem_id_x();
    if (b >= n) return;
    const int slot = g.cls[b];
    const int pos = g.pos[b];
    int item, j, cnt;
    if (slot >= 0) {
        item = g.item_start[slot] + (pos >> g.gshift);
        j = pos & (g.gsize - 1);
        const int c = g.ht_cnt[slot] - ((pos >> g.gshift) << g.gshift);
        cnt = c < g.gsize ? c : g.gsize;
    } else {
        item = g.counts[0] + pos;
        j = 0;
        cnt = 1;
    }
    g.item_blk[(size_t)item * kGroup + j] = b;
    if (j == 0) {
        g.item_n[item] = cnt;
        g.item_cls[item] = slot;
    }
}

// ---------------------------------------------------------------------------
// last FFT stage of W written straight into the window layout
// ---------------------------------------------------------------------------

// The 64 stored columns of a 64-point transform split into two halves, each
// closed under the output permutation perm(c) = 8 (c % 8) + c / 8 (which swaps
// the octal digits of c): first 32 entries = half A, last 32 = half B.
__constant__ int kColHalves[64] = {
    0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 16, 17, 18, 19, 20, 24, 25, 26, 27,
    32, 33, 34, 40, 41, 48, 49, 56,
    15, 21, 22, 23, 28, 29, 30, 31, 35, 36, 37, 38, 39, 42, 43, 44, 45, 46, 47, 50, 51, 52,
    53, 54, 55, 57, 58, 59, 60, 61, 62, 63};

// Stage B of the column pass of a 64 x 64 FFT, written into the W window:
// window row i (0..64) holds grid row (i - 16) mod 64, columns in natural order.
// The outputs of stored column pc go to LDS column perm(pc), which lies in the
// same half as pc.  Each half is read into registers, then written after a
// barrier, so the in-place reshuffle never clobbers an unread input.
template <int NT>
__device__ __forceinline__ void fft64_stage_b_to_window(double2* win, int tid) {
    constexpr int T = 64, Q = 16;
    static_assert(NT == 256, "one stage-B task per thread and half");
#pragma unroll
    for (int half = 0; half < 2; ++half) {
        // half A first, then half B: the writes of a half only touch columns of
        // that half, whose inputs have all been read before the barrier
        // neighbouring lanes take different columns (different LDS banks)
        const int pc = kColHalves[(half << 5) | (tid & 31)];
        const int k1 = tid >> 5;
        double2 x[8];
#pragma unroll
        for (int n2 = 0; n2 < 8; ++n2) x[n2] = win[(8 * k1 + n2) * T + pc];
        dft8(x);
        __syncthreads();
        const int c = FftPlan<T>::perm(pc);
#pragma unroll
        for (int k2 = 0; k2 < 8; ++k2) {
            const int k = k1 + 8 * k2;                 // natural grid row
            win[((k + Q) & (T - 1)) * T + c] = x[k2];
            if (k == 3 * Q) win[T * T + c] = x[k2];    // window row 64 repeats grid row 48
        }
        __syncthreads();
    }
}

// The same last stage for a point-symmetric w: the window of real pairs of
// run_wave_sym.  Grid row k of W, column c, gives V(a, c) = Re(conj(P(a, c))
// W[k][c]) for each unreduced row a = k or k - T in -Q .. 3Q + 1, written as
// the first element of entry a + Q and the second of entry a + Q - 1 (only
// column c is written, so the two halves stay apart as above).
template <int NT>
__device__ __forceinline__ void fft64_stage_b_to_pairs(double2* win, const double2* ht, int R0, int C0, int tid) {
    constexpr int T = 64, Q = 16;
    static_assert(NT == 256, "one stage-B task per thread and half");
    double* wd = reinterpret_cast<double*>(win);
#pragma unroll
    for (int half = 0; half < 2; ++half) {
        const int pc = kColHalves[(half << 5) | (tid & 31)];
        const int k1 = tid >> 5;
        double2 x[8];
#pragma unroll
        for (int n2 = 0; n2 < 8; ++n2) x[n2] = win[(8 * k1 + n2) * T + pc];
        dft8(x);
        __syncthreads();
        const int c = FftPlan<T>::perm(pc);
#pragma unroll
        for (int k2 = 0; k2 < 8; ++k2) {
            const int k = k1 + 8 * k2;                 // natural grid row
#pragma unroll
            for (int wrap = 0; wrap < 2; ++wrap) {
                const int a = wrap ? k - T : k;
                if (a < -Q || a > 3 * Q + 1) continue;
                const double2 P = ht[(a * R0 + c * C0) & (2 * T - 1)];
                const double val = P.x * x[k2].x + P.y * x[k2].y;
                const int i = a + Q;
                if (i <= T) wd[2 * (i * T + c)] = val;
                if (i >= 1) wd[2 * ((i - 1) * T + c) + 1] = val;
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// persistent grouped kernel: kGroup blocks x kWavesG waves per workgroup
// ---------------------------------------------------------------------------

constexpr int kWavesG = 1;                  // waves per block in the grouped path

// A zero 16-byte LDS entry whose value is made where it is stored: a zero
// register tuple kept live across the transforms gets spilled, and its reload
// then waits for every global load in flight (loads complete in order).
__device__ __forceinline__ void store_zero16(double2* dst) {
    uint32_t z;
    asm volatile("v_mov_b32 %0, 0" : "=v"(z));
    *reinterpret_cast<uint4*>(dst) = make_uint4(z, z, z, z);
}

// Row stride (16-byte entries) of the per-block transform grid: one entry more
// than a row, so that entry (n, m) and (n + 1, m) lie on different LDS banks.
// 64 rows of 65 entries fill the window exactly.
constexpr int kGridStride64 = 65;

template <int T, int WI>
__device__ __forceinline__ void extract_rows(const double2* win, int lane,
                                             RegSpec<WaveRows<T, kWavesG, WI>::S>& R) {
    using WR = WaveRows<T, kWavesG, WI>;
    constexpr int S = kGridStride64;
#pragma unroll
    for (int s = 0; s < WR::S; ++s) {
        const int k = WR::k0 + s;
        double2 a = make_double2(0.0, 0.0);
        if (lane < T) a = win[FftPlan<T>::perm(k) * S + FftPlan<T>::perm(lane)];
        R.set(s, a.x, a.y);
    }
}

// Stage B of a 64-point FFT along contiguous lines of a grid with row stride
// kGridStride64: the eight lanes of a group take eight consecutive lines at
// the same k1, so their reads and writes fall on different banks (with a
// lane per k1 of one line they all met the same ones).  Lines run up to
// nlines rounded up to a multiple of 8; the extra lines must hold zeros.
template <int NT>
__device__ __forceinline__ void fft64_stage_b_rows(double2* buf, int nlines, int tid) {
    constexpr int S = kGridStride64;
    const int ntask = ((nlines + 7) & ~7) * 8;
    for (int task = tid; task < ntask; task += NT) {
        const int line = (task & 7) | ((task >> 6) << 3);
        const int k1 = (task >> 3) & 7;
        double2* base = buf + line * S + 8 * k1;
        double2 x[8];
#pragma unroll
        for (int n2 = 0; n2 < 8; ++n2) x[n2] = base[n2];
        dft8(x);
#pragma unroll
        for (int k2 = 0; k2 < 8; ++k2) base[k2] = x[k2];
    }
}

// LDS of the grouped kernel.
template <int T>
struct GroupShared {
    double2 win[(T + 1) * T];
    double2 tw[T];
    double2 ht[2 * T];                     // exp(-j pi q / T), q < 2T
    Xchg<kWavesG> xchg[kGroup][2];
    int flags[kGroup];
    int asym;                              // the item's w is not point-symmetric
    int next;                              // next work item of the workgroup
};

// One work item (up to kGroup blocks of one mask class) as seen by wave WI of
// its block.  Every wave of the workgroup runs the same sequence of barriers.
// FULL selects the full compensation of eqs. 10-13 (see run_wave).
template <int T, int WI, int MAXPX, bool FULL>
__device__ __forceinline__ void process_item(GroupShared<T>& sh, const KParams& p, const GroupArgs& g,
                                             int item, int tid, int lane, int jblk, int tib,
                                             bool params_ok, double rho, double gamma) {
    constexpr int NT = kGroup * kWavesG * 64;
    const int M = p.M, N = p.N, MN = M * N, K = p.K;
    double2* win = sh.win;
    int nblk, blk[kGroup];
    if (g.direct) {
        nblk = min(kGroup, p.n_blocks - item * kGroup);
#pragma unroll
        for (int j = 0; j < kGroup; ++j) blk[j] = item * kGroup + j;
    } else {
        nblk = g.item_n[item];
#pragma unroll
        for (int j = 0; j < kGroup; ++j) blk[j] = g.item_blk[(size_t)item * kGroup + j];
    }
    const int b_rep = blk[0];              // every block of the item has this mask
    // the thread index as an opaque per-item value: keeps the compiler from
    // hoisting every per-thread sample address of the item's loops out of the
    // item loop (they would be spilled for the whole kernel and reloaded per item)
    asm volatile("" : "+v"(tid), "+v"(lane));
    __syncthreads();                       // previous item done with LDS
    if (tid < kGroup) sh.flags[tid] = params_ok ? 0 : FOFSE_BLOCK_BAD_PARAM;
    if (tid == 0) sh.asym = 0;

    // weights of this thread's samples (eqs. 4, 15): identical for the item
    // (every load issued before any is used, indices clamped into the area)
    double wreg[MAXPX];
    {
        uint8_t off[MAXPX];                 // sample beyond the area, on B or unknown
#pragma unroll
        for (int q = 0; q < MAXPX; ++q) {
            const int i = min(tid + q * NT, MN - 1);
            wreg[q] = p.wtab[i];
            off[q] = p.target[i];
        }
        if (g.known) {
            uint8_t kn[MAXPX];
#pragma unroll
            for (int q = 0; q < MAXPX; ++q) kn[q] = g.known[(size_t)b_rep * MN + min(tid + q * NT, MN - 1)];
#pragma unroll
            for (int q = 0; q < MAXPX; ++q) off[q] |= kn[q] == 0;
        }
#pragma unroll
        for (int q = 0; q < MAXPX; ++q)
            if (tid + q * NT >= MN || off[q] != 0) wreg[q] = 0.0;
    }

    // R = DFT(w f) of each block by its own transform (eqs. 7, 8), so that a
    // block's result does not depend on which blocks share its work item.
    // The grid is transposed (entry (n, m) holds area sample (m, n)) with row
    // stride kGridStride64; rows n >= N and entries m >= M are zero.
    constexpr int S = kGridStride64;
    static_assert(T == 64 && S == T + 1, "the transform grid (T rows of T + 1 entries) fills the window");
    RegSpec<WaveRows<T, kWavesG, WI>::S> R;
#pragma unroll
    for (int j = 0; j < kGroup; ++j) {
        if (j >= nblk) break;                  // uniform over the workgroup
        // this thread's samples of the block, all loads issued before any is
        // used (indices clamped into the area, samples beyond it dropped)
        uint32_t xs[MAXPX];
#pragma unroll
        for (int q = 0; q < MAXPX; ++q) xs[q] = sample_bits(p.areas, (size_t)blk[j] * MN + min(tid + q * NT, MN - 1));
        __syncthreads();
        for (int e = tid; e < T * T; e += NT) {
            const int n = e >> 6, m = e & (T - 1);
            if (n >= N || m >= M) store_zero16(&win[e + n]);       // n S + m with S = T + 1
        }
#pragma unroll
        for (int q = 0; q < MAXPX; ++q) {
            const int i = tid + q * NT;
            if (i < MN) {
                const int m = i / N, n = i - m * N;
                double fw = 0.0;
                if (wreg[q] != 0.0) {
                    if (nonfinite_bits(xs[q])) atomicOr(&sh.flags[j], FOFSE_BLOCK_NONFINITE);
                    else fw = wreg[q] * (double)__uint_as_float(xs[q]);
                }
                win[n * S + m] = make_double2(fw, 0.0);
            }
        }
        __syncthreads();
        fft_stage_a<T, NT>(win, sh.tw, N, S, 1, tid);
        __syncthreads();
        fft64_stage_b_rows<NT>(win, N, tid);
        __syncthreads();
        fft_stage_a<T, NT>(win, sh.tw, T, 1, S, tid);
        __syncthreads();
        fft_stage_b<T, NT>(win, T, 1, S, tid);
        __syncthreads();
        if (jblk == j) extract_rows<T, WI>(win, lane, R);
    }

    // W = DFT(w) straight into the window (rows -T/4 .. 3T/4), from the
    // transposed grid with row stride T (rows n >= N and entries m >= M zero)
    __syncthreads();
    for (int e = tid; e < T * T; e += NT) {
        const int n = e >> 6, m = e & (T - 1);
        if (n >= N || m >= M) store_zero16(&win[e]);
    }
#pragma unroll
    for (int q = 0; q < MAXPX; ++q) {
        const int i = tid + q * NT;
        if (i < MN) {
            const int m = i / N, n = i - m * N;
            win[n * T + m] = make_double2(wreg[q], 0.0);
        }
    }
    __syncthreads();
    if constexpr (!FULL) {
        // is w symmetric about the area's centre?  (the weights of mirrored
        // samples are computed from the same distance, so they compare equal)
        bool asym = false;
#pragma unroll
        for (int q = 0; q < MAXPX; ++q) {
            const int i = tid + q * NT;
            if (i < MN) {
                const int m = i / N, n = i - m * N;
                asym = asym || win[(N - 1 - n) * T + (M - 1 - m)].x != wreg[q];
            }
        }
        if (asym) sh.asym = 1;
        __syncthreads();
    }
    fft_stage_a<T, NT>(win, sh.tw, N, T, 1, tid);
    __syncthreads();
    fft_stage_b<T, NT>(win, N, T, 1, tid);
    __syncthreads();
    fft_stage_a<T, NT>(win, sh.tw, T, 1, T, tid);
    __syncthreads();
    const bool sym = !FULL && sh.asym == 0;
    if (sym) fft64_stage_b_to_pairs<NT>(win, sh.ht, N - 1, M - 1, tid);
    else     fft64_stage_b_to_window<NT>(win, tid);
    const double W0 = win[16 * T].x;      // W[0, 0] (V(0, 0)) sits in window row 16

    // the K iterations: every wave runs them (and their barriers); waves of a
    // missing or flagged block compute on zeros and write nothing
    const bool present = jblk < nblk;
    int flags = present ? sh.flags[jblk] : 0;
    if (params_ok && !(W0 > 0.0)) flags |= FOFSE_BLOCK_NO_SUPPORT;
    const bool live = present && flags == 0;
    const int bj = blk[jblk];
    const double gW0 = live ? gamma / W0 : 0.0;
    if constexpr (kWavesG == 1 && !FULL) {
        if (live && sym) {
            rotate_rows<T>(R, sh.ht, N - 1, M - 1, lane);
            run_wave_sym<T>(R, win, sh.ht, p, bj, lane, gW0);
        } else if (live) {
            run_wave<T, kWavesG, WI, FULL>(R, win, sh.xchg[jblk], p, bj, lane, gW0, live);
        }
    } else if (kWavesG > 1 || live) {
        run_wave<T, kWavesG, WI, FULL>(R, win, sh.xchg[jblk], p, bj, lane, gW0, live);
    }
    if (present) {
        if (!live) {          // empty record: the synthesised model is 0
            for (int it = tib; it < K; it += kWavesG * 64) {
                p.sel[(size_t)bj * K + it] = 0;
                p.coef[2 * ((size_t)bj * K + it)] = 0.0;
                p.coef[2 * ((size_t)bj * K + it) + 1] = 0.0;
            }
        }
        if (p.status && tib == 0) p.status[bj] = flags;
    }
}

template <int T, int MAXPX, bool FULL = false>
__global__ __launch_bounds__(kGroup * kWavesG * 64, 2) void fofse_group_kernel(KParams p, GroupArgs g) {
    constexpr int NT = kGroup * kWavesG * 64;
    static_assert(T == 64, "the window stage is written for T = 64");
    __shared__ GroupShared<T> sh;

    const int tid = (int)__builtin_amdgcn_workitem_id_x(), lane = tid & 63, wave = tid >> 6;
    const int jblk = wave / kWavesG;             // block slot of this wave in the item
    const int wi = wave % kWavesG;               // wave index within the block
    const int tib = wi * 64 + lane;              // thread index within the block
    const double rho = p.rho_gamma[0], gamma = p.rho_gamma[1];
    const bool params_ok = param_ok(rho) && (FULL || param_ok(gamma));   // the full compensation has no gamma
    for (int i = tid; i < T; i += NT) sh.tw[i] = p.twiddle[i];
    for (int i = tid; i < 2 * T; i += NT) sh.ht[i] = p.htw[i];

    // work items: contiguous ranges when every block has the same support
    // (every item costs the same), else a queue, since items differ in cost (a
    // point-symmetric mask takes about two thirds of the time of another): the
    // counter is zeroed by the grouping, and the next index is fetched while
    // the current item runs
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
        if constexpr (kWavesG == 1) {
            process_item<T, 0, MAXPX, FULL>(sh, p, g, item, tid, lane, jblk, tib, params_ok, rho, gamma);
        } else {
            if (wi == 0) process_item<T, 0, MAXPX, FULL>(sh, p, g, item, tid, lane, jblk, tib, params_ok, rho, gamma);
            else         process_item<T, 1, MAXPX, FULL>(sh, p, g, item, tid, lane, jblk, tib, params_ok, rho, gamma);
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

// ---------------------------------------------------------------------------
// host-side launch sequence (all asynchronous on the stream)
// ---------------------------------------------------------------------------

int group_max_target_samples() { return 64 * 64; }

// Clears the hash table and counters with a kernel (no memset node when a
// caller captures the launch sequence in a graph).
__global__ void k_clear(GroupArgs g) {
    const int i = (int)__builtin_amdgcn_workgroup_id_x() * 256 + (int)__builtin_amdgcn_workitem_id_x();
    if (i < g.hsize) { g.ht_key[i] = 0ull; g.ht_cnt[i] = 0; }
    if (i == 0) *g.n_single = 0;
}

hipError_t launch_clear(const GroupArgs& g, hipStream_t stream) {
    hipLaunchKernelGGL(k_clear, dim3((g.hsize + 255) / 256), dim3(256), 0, stream, g);
    return hipGetLastError();
}

hipError_t launch_grouping(const GroupArgs& g, int n, hipStream_t stream) {
    const int nwg = (n + kHashBlocks - 1) / kHashBlocks;
    hipLaunchKernelGGL(k_mask_hash, dim3(nwg), dim3(64 * kHashBlocks), 0, stream, g, n);
    hipLaunchKernelGGL(k_group_count, dim3(nwg), dim3(64 * kHashBlocks), 0, stream, g, n);
    hipLaunchKernelGGL(k_group_pos, dim3((n + 255) / 256), dim3(256), 0, stream, g, n);
    hipLaunchKernelGGL(k_group_scan, dim3(1), dim3(1024), 0, stream, g);
    hipLaunchKernelGGL(k_group_fill, dim3((n + 255) / 256), dim3(256), 0, stream, g, n);
    return hipGetLastError();
}

hipError_t launch_grouped(const KParams& p, const GroupArgs& g, int n_cu, hipStream_t stream,
                          const Timing& tm, bool full) {
    if (p.T != 64) return hipErrorInvalidValue;
    const hipError_t ew = launch_weights(p, stream);
    if (ew != hipSuccess) return ew;
    GroupArgs ga = g;
    ga.gsize = kGroup;
    ga.gshift = kGroupShift;
    if (!g.direct) {
        const hipError_t eg = launch_grouping(ga, p.n_blocks, stream);
        if (eg != hipSuccess) return eg;
    }
    const int max_items = g.direct ? (p.n_blocks + kGroup - 1) / kGroup : p.n_blocks;
    int grid = (g.wg_per_cu > 0 ? g.wg_per_cu : 2) * n_cu;     // two fit per compute unit
    if (grid > max_items) grid = max_items;
    constexpr int NT = kGroup * kWavesG * 64;
    const int mn = p.M * p.N;
    ga.n_wg = grid;
    if (tm.start && hipEventRecord(tm.start, stream) != hipSuccess) return hipErrorUnknown;
    if (full) {
        if (mn <= 9 * NT) hipLaunchKernelGGL((fofse_group_kernel<64, 9, true>), dim3(grid), dim3(NT), 0, stream, p, ga);
        else              hipLaunchKernelGGL((fofse_group_kernel<64, 16, true>), dim3(grid), dim3(NT), 0, stream, p, ga);
    } else {
        if (mn <= 9 * NT) hipLaunchKernelGGL((fofse_group_kernel<64, 9>), dim3(grid), dim3(NT), 0, stream, p, ga);
        else              hipLaunchKernelGGL((fofse_group_kernel<64, 16>), dim3(grid), dim3(NT), 0, stream, p, ga);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (tm.stop && hipEventRecord(tm.stop, stream) != hipSuccess) return hipErrorUnknown;
    return launch_synthesis(p, stream);
}

}  // namespace fofse
