// Device helpers shared by the FOFSE kernels: complex arithmetic, the in-LDS
// T x T FFT, wavefront reductions and parameter checks.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

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

// length 16 as two length-8 DFTs (even and odd samples) and twiddles
// exp(-j 2 pi k / 16)
__device__ __forceinline__ void dft16(double2* x) {
    double2 e[8], o[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        e[i] = x[2 * i];
        o[i] = x[2 * i + 1];
    }
    dft8(e);
    dft8(o);
    const double c1 = 0.92387953251128675613, s1 = 0.38268343236508977173;   // cos, sin(pi/8)
    const double r = 0.70710678118654752440;
    const double2 w[8] = {make_double2(1.0, 0.0), make_double2(c1, -s1), make_double2(r, -r),
                          make_double2(s1, -c1), make_double2(0.0, -1.0), make_double2(-s1, -c1),
                          make_double2(-r, -r), make_double2(-c1, -s1)};
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const double2 t = k ? c_mul(o[k], w[k]) : o[k];
        x[k] = c_add(e[k], t);
        x[k + 8] = c_sub(e[k], t);
    }
}

template <int R>
__device__ __forceinline__ void dft(double2* x) {
    if constexpr (R == 2) dft2(x);
    else if constexpr (R == 4) dft4(x);
    else if constexpr (R == 8) dft8(x);
    else dft16(x);
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

// Tasks go to threads so that the lanes of a wavefront touch different LDS banks:
// along contiguous lines (elem_stride 1) neighbouring lanes take neighbouring
// elements of one line; across lines (elem_stride > 1, nlines a power of two)
// neighbouring lanes take neighbouring lines (a lane-per-element mapping there
// would put the lanes of a line T entries apart, all in one bank).
template <int T, int NT>
__device__ __forceinline__ void fft_stage_a(double2* buf, const double2* tw, int nlines,
                                            int line_stride, int elem_stride, int tid) {
    constexpr int R1 = FftPlan<T>::R1;
    const bool across = elem_stride != 1;
    const int lsh = __builtin_ctz(nlines);          // across lines, nlines is a power of two
    for (int task = tid; task < nlines * 8; task += NT) {
        const int line = across ? task & (nlines - 1) : task >> 3;
        const int n2 = across ? task >> lsh : task & 7;
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
    const bool across = elem_stride != 1;
    const int lsh = __builtin_ctz(nlines);          // across lines, nlines is a power of two
    for (int task = tid; task < nlines * R1; task += NT) {
        const int line = across ? task & (nlines - 1) : task / R1;
        const int k1 = across ? task >> lsh : task - line * R1;
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

// A double moved across lanes by a DPP control, both 32-bit halves (0 in the
// rows the row mask leaves out).
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_f64(double x) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, ROW_MASK, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, ROW_MASK, 0xF, false);
    return __hiloint2double(hi, lo);
}

// Sum of a double over the 64 lanes by the exchanges of wave_max_u32 (quads,
// half rows, rows, then the row broadcasts into lane 63); the result is uniform.
__device__ __forceinline__ double wave_sum_f64(double v) {
    v += dpp_f64<0xB1, 0xF>(v);           // quad_perm [1,0,3,2]
    v += dpp_f64<0x4E, 0xF>(v);           // quad_perm [2,3,0,1]
    v += dpp_f64<0x141, 0xF>(v);          // row_half_mirror
    v += dpp_f64<0x140, 0xF>(v);          // row_mirror
    v += dpp_f64<0x142, 0xA>(v);          // row_bcast:15 into rows 1 and 3
    v += dpp_f64<0x143, 0xC>(v);          // row_bcast:31 into rows 2 and 3
    return readlane_f64(v, 63);
}

// max of two doubles as one v_max_f64 (the operands are finite keys; no
// operand canonicalisation or absolute value is wanted)
__device__ __forceinline__ double max_f64(double a, double b) {
    double r;
    asm("v_max_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

// a * a + c as one v_fma_f64 the compiler treats as opaque (so it does not
// add sign-bit operations to a value it knows is non-negative)
__device__ __forceinline__ double sq_add(double a, double c) {
    double r;
    asm("v_fma_f64 %0, %1, %1, %2" : "=v"(r) : "v"(a), "v"(c));
    return r;
}

// A float sample read as its bit pattern, and the test for an exponent of all
// ones (Inf or NaN) on those bits.  The library is compiled without NaN
// semantics; under them the compiler may rewrite a bit test on a float value
// into |x| == inf, which is false for NaN, so the test never sees a float.
__device__ __forceinline__ uint32_t sample_bits(const float* a, size_t i) {
    return reinterpret_cast<const uint32_t*>(a)[i];
}
__device__ __forceinline__ bool nonfinite_bits(uint32_t b) { return (b & 0x7f800000u) == 0x7f800000u; }

// 0 < x <= 1, false for NaN (tested on the bits, see the input check).
__device__ __forceinline__ bool param_ok(double x) {
    const uint64_t b = (uint64_t)__double_as_longlong(x);
    return b != 0 && b <= 0x3FF0000000000000ull;   // +0 < x <= 1.0 as ordered bit patterns
}

// Candidates of the waves of a workgroup: selection key (high and low word,
// see run_wave) and the value R[u] of each wave's best bin.
template <int NW>
struct Xchg {
    uint32_t hi[NW];
    uint32_t lo[NW];
    double2 val[NW];
};


}  // namespace fofse
