// Device-side helpers shared by the gfx950 kernels of the DMD hot path.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "dmdmi.h"

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef double doublex2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

#define DMD_WAVE 64

// ---------------------------------------------------------------- MFMA
// All three use the 16x16 output tile with the same lane layout:
//   A operand: lane l supplies A[i = l % 16][k-group l / 16]
//   B operand: lane l supplies B[k-group l / 16][j = l % 16]
//   D:         lane l holds D[acc_row(l, v)][l % 16], v = 0..3 (see acc_row)
// For f32 / f64 the k-group is one k index (depth 4); for bf16 it is 8
// consecutive k indices (depth 32).
__device__ __forceinline__ floatx4 mfma_f32(float a, float b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ doublex4 mfma_f64(double a, double b, doublex4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ floatx4 mfma_bf16(bf16x8 a, bf16x8 b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

template <typename T> struct Acc;
template <> struct Acc<float> { typedef floatx4 type; };
template <> struct Acc<double> { typedef doublex4 type; };

__device__ __forceinline__ floatx4 mfma(float a, float b, floatx4 c) { return mfma_f32(a, b, c); }
__device__ __forceinline__ doublex4 mfma(double a, double b, doublex4 c) { return mfma_f64(a, b, c); }

// Row (within the 16x16 tile) of accumulator element v held by `lane`.  The f32
// and bf16 16x16 instructions give lane l rows 4*(l/16)+v; the f64 16x16x4
// instruction gives rows l/16 + 4v (columns are l % 16 for all three).
template <typename V> __device__ __forceinline__ int acc_row(int lane, int v);
template <> __device__ __forceinline__ int acc_row<floatx4>(int lane, int v) { return 4 * (lane >> 4) + v; }
template <> __device__ __forceinline__ int acc_row<doublex4>(int lane, int v) { return (lane >> 4) + 4 * v; }

template <typename V> __device__ __forceinline__ V zero_acc() {
    V z;
    z[0] = 0; z[1] = 0; z[2] = 0; z[3] = 0;
    return z;
}

// ---------------------------------------------------------------- wave reductions
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, DMD_WAVE);
    return v;
}
// The same sum with the intra-row steps as DPP lane moves (quad permutations, half-row and
// row mirrors; no LDS round trip) and the four row sums combined from readlanes.  Every
// lane gets the bit-identical result (each step adds two equal-order partial sums).  All
// 64 lanes must be active.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double readlane_d(double v, int l) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double wave_sum_dpp(double v) {
    v += dpp_move<0xB1>(v);      // quad_perm [1, 0, 3, 2]
    v += dpp_move<0x4E>(v);      // quad_perm [2, 3, 0, 1]
    v += dpp_move<0x141>(v);     // row_half_mirror: the other quad of each 8 lanes
    v += dpp_move<0x140>(v);     // row_mirror: the other 8 lanes of each row
    return (readlane_d(v, 0) + readlane_d(v, 16)) + (readlane_d(v, 32) + readlane_d(v, 48));
}
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, DMD_WAVE);
    return v;
}

// Intra-wave ordering of LDS writes and later reads by other lanes of the same wave.
__device__ __forceinline__ void wave_sync_lds()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// First error wins: record a device-side status code.
__device__ __forceinline__ void set_status(int32_t* info, int32_t code) {
    if (info) atomicCAS(info, 0, code);
}

// ---------------------------------------------------------------- fast FP64 reciprocals
// 1/sqrt(s) for s > 0 and 1/s for s != 0 (normal range): the hardware estimates (about 23
// correct bits) refined by two Newton steps each, which leaves an error of a few ulp.
__device__ __forceinline__ double rsqrt_nr(double s)
{
    double r = __builtin_amdgcn_rsq(s);
    const double hs = 0.5 * s;
    r = r * fma(-hs * r, r, 1.5);
    r = r * fma(-hs * r, r, 1.5);
    return r;
}
__device__ __forceinline__ double rcp_nr(double s)
{
    double r = __builtin_amdgcn_rcp(s);
    r = fma(r, fma(-s, r, 1.0), r);
    r = fma(r, fma(-s, r, 1.0), r);
    return r;
}

// ---------------------------------------------------------------- complex (FP64)
struct cplx { double re, im; };
__device__ __forceinline__ cplx cmul(cplx a, cplx b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ cplx cadd(cplx a, cplx b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cplx csub(cplx a, cplx b) { return {a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ cplx cconj(cplx a) { return {a.re, -a.im}; }
__device__ __forceinline__ cplx cdiv(cplx a, cplx b) {
    // Smith's algorithm
    if (fabs(b.re) >= fabs(b.im)) {
        double r = b.im / b.re, d = b.re + b.im * r;
        return {(a.re + a.im * r) / d, (a.im - a.re * r) / d};
    } else {
        double r = b.re / b.im, d = b.re * r + b.im;
        return {(a.re * r + a.im) / d, (a.im * r - a.re) / d};
    }
}

// lambda^e on the principal branch, computed as exp(e * Log lambda) in FP64.
// 0^0 = 1 and 0^e = 0 for e > 0; 0^e for e < 0 gives +inf (non-finite).
__device__ __forceinline__ cplx cpow_real(cplx lam, double e) {
    double a = hypot(lam.re, lam.im);
    if (a == 0.0) {
        if (e == 0.0) return {1.0, 0.0};
        if (e > 0.0) return {0.0, 0.0};
        return {__builtin_inf(), 0.0};
    }
    double th = atan2(lam.im, lam.re);
    double mag = exp(e * log(a));
    double s, c;
    sincos(e * th, &s, &c);
    return {mag * c, mag * s};
}

// Status bits of a coefficient pass, or-ed into one device word that the host reads back
// (a power of lambda = 0 outside its domain; a coefficient beyond the output type's range).
constexpr int32_t COEF_DOMAIN = 1;
constexpr int32_t COEF_OVERFLOW = 2;

// ---------------------------------------------------------------- misc
__host__ __device__ __forceinline__ int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }
__host__ __device__ __forceinline__ int64_t ceil_div(int64_t x, int64_t m) { return (x + m - 1) / m; }
