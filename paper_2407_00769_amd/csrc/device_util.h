// Device helpers: complex word packing for the three storage forms, block
// reductions, and the launch descriptors the planner fills.
#pragma once

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cstdint>

#include "common.h"

namespace tnc {

// ------------------------------------------------------------------ storage words
struct HalfWord {
    uint32_t w;   // low 16 bits: re (IEEE binary16), high 16 bits: im
};
struct Bf16Word {
    uint32_t w;   // low 16 bits: re (bfloat16), high 16 bits: im
};

__device__ __forceinline__ float2 unpack(uint2 v) { return make_float2(__uint_as_float(v.x), __uint_as_float(v.y)); }
__device__ __forceinline__ float2 unpack(HalfWord v) {
    return make_float2(__half2float(__ushort_as_half((unsigned short)(v.w & 0xffffu))),
                       __half2float(__ushort_as_half((unsigned short)(v.w >> 16))));
}
__device__ __forceinline__ float2 unpack(Bf16Word v) {
    return make_float2(__uint_as_float(v.w << 16), __uint_as_float(v.w & 0xffff0000u));
}

// round-to-nearest-even float -> bfloat16 bits
__device__ __forceinline__ uint32_t f2bf_bits(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0u;   // NaN stays NaN
    u += 0x7fffu + ((u >> 16) & 1u);
    return u >> 16;
}
__device__ __forceinline__ uint32_t f2h_bits(float f) {
    __half h = __float2half_rn(f);
    return (uint32_t)__half_as_ushort(h);
}

template <typename W> struct Pack;
template <> struct Pack<uint2> {
    __device__ static uint2 make(float re, float im) { return make_uint2(__float_as_uint(re), __float_as_uint(im)); }
};
template <> struct Pack<HalfWord> {
    __device__ static HalfWord make(float re, float im) { return HalfWord{f2h_bits(re) | (f2h_bits(im) << 16)}; }
};
template <> struct Pack<Bf16Word> {
    __device__ static Bf16Word make(float re, float im) { return Bf16Word{f2bf_bits(re) | (f2bf_bits(im) << 16)}; }
};

template <typename W> __device__ __forceinline__ float word_absmax(W v) {
    float2 f = unpack(v);
    return fmaxf(fabsf(f.x), fabsf(f.y));
}
template <typename W> __device__ __forceinline__ double2 word_to_double2(W v) {
    float2 f = unpack(v);
    return make_double2((double)f.x, (double)f.y);
}

// Largest value of a block (result valid in thread 0).  NaN propagates as
// the largest value because fmaxf ignores NaN: callers pass |x| with NaN
// already mapped to +inf.
__device__ __forceinline__ float wave_max(float v) {
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ float block_max(float v) {
    __shared__ float red[16];
    v = wave_max(v);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int nw = (blockDim.x + 63) >> 6;
    __syncthreads();
    if (l == 0) red[w] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < nw; i++) v = fmaxf(v, red[i]);
    }
    return v;
}
// |x| with NaN mapped to +inf, so a NaN shows up as an overflow
__device__ __forceinline__ float absmax_nan(float a, float b) {
    float m = fmaxf(fabsf(a), fabsf(b));
    return (a != a || b != b) ? __builtin_inff() : m;
}

// ------------------------------------------------------------------ scale bookkeeping
// All 16-bit results are stored as value * 2^-shift with
//   shift = floor(log2 maxA) + floor(log2 maxB) + growth - kTargetLog2
// so that the largest stored component lands near 2^kTargetLog2.
constexpr int kTargetLog2 = kTargetLog2Host;

__device__ __forceinline__ int floor_log2_pos(float x) {
    int e;
    frexpf(x, &e);   // x = f * 2^e, f in [0.5, 1)
    return e - 1;
}

__device__ __forceinline__ int step_shift(const ScaleRefs &sc, int s) {
    float ma = __uint_as_float(sc.maxA[s * sc.mA]);
    float mb = __uint_as_float(sc.maxB[s * sc.mB]);
    if (!(ma > 0.f) || !(mb > 0.f) || !(ma <= 3.0e38f) || !(mb <= 3.0e38f)) return 0;
    return floor_log2_pos(ma) + floor_log2_pos(mb) + *sc.growth - kTargetLog2;
}

// First block of slice s records the output exponent and the shift.
__device__ __forceinline__ void record_exponent(const ScaleRefs &sc, int s, int shift) {
    double e = sc.expA[s * sc.eA] + sc.expB[s * sc.eB] + (double)shift;
    sc.expC[s] = e;
    if (sc.shift) sc.shift[s] = shift;
}

}  // namespace tnc
