// Helpers shared by the adjoint kernels: class keys of the selection record,
// packed LDS offsets of the spectrum Z = W + j D at the sums and differences
// of two classes, wavefront sums.
#pragma once

#include <hip/hip_runtime.h>

#include "device_common.hpp"

namespace fofse {

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
    static constexpr int LOG2 = T == 128 ? 7 : T == 64 ? 6 : T == 32 ? 5 : 4;
    __device__ static int k(int key) { return (key >> LOG2) & (T - 1); }
    __device__ static int l(int key) { return key & (T - 1); }
    __device__ static bool pair(int k, int l) {
        return !(((k & (T / 2 - 1)) == 0) && ((l & (T / 2 - 1)) == 0));
    }
};

// Byte offsets of Z[u_j - u_i], Z[u_i - u_j], Z[u_j + u_i], Z[-u_j - u_i] in the
// LDS spectrum, for a per-lane class u_i = (ku, lu) and a uniform u_j.
// T = 64: Z in natural order; the two indices travel packed as k << 8 | l with
// a guard bit (128) that keeps the l field from borrowing, so each offset is
// one add or subtract and three bit operations.  Other T: FFT output order.
template <int T>
struct ZOff {
    int ku, lu;
    __device__ ZOff(int k, int l) : ku(k), lu(l) {}
    __device__ void get(int kj, int lj, int& a, int& b, int& c, int& d) const {
        a = 16 * zp<T>(kj - ku, lj - lu);
        b = 16 * zp<T>(ku - kj, lu - lj);
        c = 16 * zp<T>(kj + ku, lj + lu);
        d = 16 * zp<T>(-kj - ku, -lj - lu);
    }
};

template <>
struct ZOff<64> {
    int yd, ym;
    __device__ ZOff(int k, int l) : yd((k << 8) | l), ym((k << 8) | 128 | l) {}
    __device__ static int off(int r) { return ((r << 2) & 0xFC00) | ((r << 4) & 0x3F0); }
    __device__ void get(int kj, int lj, int& a, int& b, int& c, int& d) const {
        const int xs = (kj << 8) | lj;
        a = off((xs | 128) - yd);
        b = off(ym - xs);
        c = off(xs + yd);
        d = off(((64 << 8) | 128) - xs - yd);
    }
};

__device__ __forceinline__ double2 lds_at(const double2* base, int byte_off) {
    return *(const double2*)((const char*)base + byte_off);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

}  // namespace fofse
