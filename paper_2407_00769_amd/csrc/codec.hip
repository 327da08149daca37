// Low-precision exchange codec (paper Sec. 3.2, Eq. quantcal, Table
// quanttable): a group of real values y = sign(x)|x|^exp is mapped to
//     q = y * scale + zero,  scale = (q_max - q_min) / (max y - min y),
//                            zero  = (q_min max y - q_max min y) / (max y - min y)
// and, for the integer kinds, rounded half-to-even and clamped.  Kinds:
//     half  q in +-65504, exp 1, one group (the whole tensor), stored as FP16
//     int8  q in -128..127, exp 0.2, one group, stored as int8
//     int4  q in 0..15, exp 1, groups of G (default 128), two codes per byte
//           (entry 2j in the low nibble of byte j)
// A complex tensor is coded as the real array of its interleaved (re, im)
// values.  The integer decision is taken in float32 with the operations
// unfused (q = (y * scale) + zero, each rounded; this file is compiled with
// -ffp-contract=off).  The power 0.2 uses the hardware log2 and exp2 (a few
// ulp), so codes equal those of a float32 implementation with a correctly
// rounded power except for values within about 1e-4 of a rounding tie.
// Each thread moves 16 values with 16-byte loads and stores.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cstdint>
#include <mutex>

#include "common.h"

namespace tnc {

struct QKind {
    float qmin, qmax, exp, inv_exp;
    bool round;
};
__host__ __device__ inline QKind qkind(int kind) {
    switch (kind) {
        case 0: return {-65504.f, 65504.f, 1.f, 1.f, false};
        case 1: return {-128.f, 127.f, 0.2f, 5.f, true};
        default: return {0.f, 15.f, 1.f, 1.f, true};
    }
}

// sign(x)|x|^e for the coding side (e = 1 or 0.2): exp2(e log2|x|) on the
// hardware units for normal |x|, powf below that
__device__ __forceinline__ float qpow(float x, float e) {
    if (e == 1.f) return x;
    const float a = fabsf(x);
    const float r = a >= FLT_MIN ? __builtin_amdgcn_exp2f(__fmul_rn(e, __builtin_amdgcn_logf(a))) : powf(a, e);
    return copysignf(r, x);
}

// the inverse power on the decoding side (1/e = 1 or 5): y^5 as y^2 y^2 y,
// which keeps the sign and loses at most a few ulp
__device__ __forceinline__ float qpow_inv(float y, float inv_e) {
    if (inv_e == 1.f) return y;
    if (inv_e == 5.f) {
        const float y2 = __fmul_rn(y, y);
        return __fmul_rn(__fmul_rn(y2, y2), y);
    }
    return copysignf(powf(fabsf(y), inv_e), y);
}

// scale and zero of a group from the extremes of y, in the oracle's order
__device__ __forceinline__ void scale_zero(const QKind &k, float mn, float mx, float &scale, float &zero) {
    if (mx == mn) {
        scale = 1.f;
        zero = __fsub_rn(k.qmin, mn);
        return;
    }
    const float d = __fsub_rn(mx, mn);
    scale = __fdiv_rn(__fsub_rn(k.qmax, k.qmin), d);
    zero = __fdiv_rn(__fsub_rn(__fmul_rn(k.qmin, mx), __fmul_rn(k.qmax, mn)), d);
}

__device__ __forceinline__ float qcode(const QKind &k, float y, float scale, float zero) {
    float q = __fadd_rn(__fmul_rn(y, scale), zero);
    if (k.round) q = fminf(fmaxf(rintf(q), k.qmin), k.qmax);
    return q;
}

__device__ __forceinline__ float qdecode(const QKind &k, float q, float scale, float zero) {
    return qpow_inv(__fdiv_rn(__fsub_rn(q, zero), scale), k.inv_exp);
}

// ------------------------------------------------------------------ whole-tensor kinds

// partial (min, max) of x per block; the power is monotone, so the extremes
// of y are the powers of the extremes of x
__global__ void __launch_bounds__(256) minmax_partial_kernel(const float *__restrict__ x, int64_t n,
                                                             float2 *__restrict__ part) {
    float mn = FLT_MAX, mx = -FLT_MAX;
    const int64_t n4 = n / 4, stride = (int64_t)gridDim.x * blockDim.x;
    const float4 *x4 = (const float4 *)x;
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    // four 16-byte loads in flight per thread
    for (; i + 3 * stride < n4; i += 4 * stride) {
        const float4 v[4] = {x4[i], x4[i + stride], x4[i + 2 * stride], x4[i + 3 * stride]};
#pragma unroll
        for (int u = 0; u < 4; u++) {
            mn = fminf(fminf(fminf(mn, v[u].x), fminf(v[u].y, v[u].z)), v[u].w);
            mx = fmaxf(fmaxf(fmaxf(mx, v[u].x), fmaxf(v[u].y, v[u].z)), v[u].w);
        }
    }
    for (; i < n4; i += stride) {
        const float4 v = x4[i];
        mn = fminf(fminf(fminf(mn, v.x), fminf(v.y, v.z)), v.w);
        mx = fmaxf(fmaxf(fmaxf(mx, v.x), fmaxf(v.y, v.z)), v.w);
    }
    for (int64_t i = n4 * 4 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        mn = fminf(mn, x[i]);
        mx = fmaxf(mx, x[i]);
    }
    for (int o = 32; o > 0; o >>= 1) {
        mn = fminf(mn, __shfl_xor(mn, o, 64));
        mx = fmaxf(mx, __shfl_xor(mx, o, 64));
    }
    __shared__ float2 w[4];
    if ((threadIdx.x & 63) == 0) w[threadIdx.x >> 6] = make_float2(mn, mx);
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < (int)(blockDim.x >> 6); i++) {
            mn = fminf(mn, w[i].x);
            mx = fmaxf(mx, w[i].y);
        }
        part[blockIdx.x] = make_float2(mn, mx);
    }
}

// one wave: the extremes of the partials (min and max are exact in any order)
__global__ void scale_zero_kernel(const float2 *__restrict__ part, int np, int kind, float *scales, float *zeros) {
    float mn = FLT_MAX, mx = -FLT_MAX;
    for (int i = threadIdx.x; i < np; i += 64) {
        mn = fminf(mn, part[i].x);
        mx = fmaxf(mx, part[i].y);
    }
    for (int o = 32; o > 0; o >>= 1) {
        mn = fminf(mn, __shfl_xor(mn, o, 64));
        mx = fmaxf(mx, __shfl_xor(mx, o, 64));
    }
    if (threadIdx.x != 0) return;
    const QKind k = qkind(kind);
    float s, z;
    scale_zero(k, qpow(mn, k.exp), qpow(mx, k.exp), s, z);
    scales[0] = s;
    zeros[0] = z;
}

template <int KIND>
__global__ void __launch_bounds__(256) quantize_whole_kernel(const float *__restrict__ x, int64_t n,
                                                             const float *__restrict__ scales,
                                                             const float *__restrict__ zeros, void *__restrict__ codes) {
    const QKind k = qkind(KIND);
    const float scale = scales[0], zero = zeros[0];
    const int64_t n16 = n / 16;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n16; t += (int64_t)gridDim.x * blockDim.x) {
        float v[16];
#pragma unroll
        for (int c = 0; c < 4; c++) {
            float4 f = ((const float4 *)x)[4 * t + c];
            v[4 * c] = f.x; v[4 * c + 1] = f.y; v[4 * c + 2] = f.z; v[4 * c + 3] = f.w;
        }
        if constexpr (KIND == 0) {
            uint32_t h[8];
#pragma unroll
            for (int i = 0; i < 8; i++)
                h[i] = (uint32_t)__half_as_ushort(__float2half_rn(qcode(k, v[2 * i], scale, zero))) |
                       ((uint32_t)__half_as_ushort(__float2half_rn(qcode(k, v[2 * i + 1], scale, zero))) << 16);
            uint4 *o = (uint4 *)codes + 2 * t;
            o[0] = make_uint4(h[0], h[1], h[2], h[3]);
            o[1] = make_uint4(h[4], h[5], h[6], h[7]);
        } else {
            uint32_t b[4];
#pragma unroll
            for (int i = 0; i < 4; i++) {
                b[i] = 0;
#pragma unroll
                for (int j = 0; j < 4; j++) {
                    int q = (int)qcode(k, qpow(v[4 * i + j], k.exp), scale, zero);
                    b[i] |= ((uint32_t)q & 0xffu) << (8 * j);
                }
            }
            ((uint4 *)codes)[t] = make_uint4(b[0], b[1], b[2], b[3]);
        }
    }
    // tail
    for (int64_t i = n16 * 16 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        if constexpr (KIND == 0)
            ((__half *)codes)[i] = __float2half_rn(qcode(k, x[i], scale, zero));
        else
            ((int8_t *)codes)[i] = (int8_t)(int)qcode(k, qpow(x[i], k.exp), scale, zero);
    }
}

// Chunks of 4 values, lane-contiguous: in each of a thread's four rounds the
// 64 lanes of a wave decode 64 consecutive chunks, so every 16-byte store
// instruction writes one contiguous 1 KB run.
template <int KIND>
__global__ void __launch_bounds__(256) dequantize_whole_kernel(const void *__restrict__ codes, int64_t n,
                                                               const float *__restrict__ scales,
                                                               const float *__restrict__ zeros, float *__restrict__ x) {
    const QKind k = qkind(KIND);
    const float scale = scales[0], zero = zeros[0];
    const int64_t n4 = n / 4, step = (int64_t)gridDim.x * blockDim.x * 4;
    for (int64_t c0 = (int64_t)blockIdx.x * blockDim.x * 4 + threadIdx.x; c0 < n4; c0 += step) {
        float v[4][4];
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const int64_t c = c0 + (int64_t)u * blockDim.x;
            if (c >= n4) break;
            if constexpr (KIND == 0) {
                const uint2 h = ((const uint2 *)codes)[c];
                v[u][0] = __half2float(__ushort_as_half((unsigned short)(h.x & 0xffffu)));
                v[u][1] = __half2float(__ushort_as_half((unsigned short)(h.x >> 16)));
                v[u][2] = __half2float(__ushort_as_half((unsigned short)(h.y & 0xffffu)));
                v[u][3] = __half2float(__ushort_as_half((unsigned short)(h.y >> 16)));
            } else {
                const uint32_t b = ((const uint32_t *)codes)[c];
#pragma unroll
                for (int i = 0; i < 4; i++) v[u][i] = (float)(int8_t)((b >> (8 * i)) & 0xffu);
            }
        }
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const int64_t c = c0 + (int64_t)u * blockDim.x;
            if (c >= n4) break;
            ((float4 *)x)[c] = make_float4(qdecode(k, v[u][0], scale, zero), qdecode(k, v[u][1], scale, zero),
                                           qdecode(k, v[u][2], scale, zero), qdecode(k, v[u][3], scale, zero));
        }
    }
    for (int64_t i = n4 * 4 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        float q = KIND == 0 ? __half2float(((const __half *)codes)[i]) : (float)((const int8_t *)codes)[i];
        x[i] = qdecode(k, q, scale, zero);
    }
}

// ------------------------------------------------------------------ int4, groups of G = 16 T values
// A team of T lanes owns one group; lane j of the team holds values
// 16 j .. 16 j + 15 of it.  Entries past n are left out of the extremes and
// not stored.

template <int T>
__global__ void __launch_bounds__(256) quantize_int4_kernel(const float *__restrict__ x, int64_t n, int64_t n_groups,
                                                            float *__restrict__ scales, float *__restrict__ zeros,
                                                            uint8_t *__restrict__ codes) {
    constexpr int G = 16 * T;
    const QKind k = qkind(2);
    const int lane = threadIdx.x & 63, j = lane % T;
    const int64_t teams_per_block = blockDim.x / T;
    // the lanes of a team share gi, so a team enters and leaves the loop as a
    // whole and the shuffles below (offsets < T) stay inside it
    for (int64_t gi = blockIdx.x * teams_per_block + threadIdx.x / T; gi < n_groups;
         gi += (int64_t)gridDim.x * teams_per_block) {
        const int64_t base = gi * G + 16 * j;
        float v[16];
        float mn = FLT_MAX, mx = -FLT_MAX;
        if (base + 16 <= n) {
#pragma unroll
            for (int c = 0; c < 4; c++) {
                float4 f = ((const float4 *)(x + base))[c];
                v[4 * c] = f.x; v[4 * c + 1] = f.y; v[4 * c + 2] = f.z; v[4 * c + 3] = f.w;
            }
#pragma unroll
            for (int i = 0; i < 16; i++) {
                mn = fminf(mn, v[i]);
                mx = fmaxf(mx, v[i]);
            }
        } else {
#pragma unroll
            for (int i = 0; i < 16; i++) {
                const bool in = base + i < n;
                v[i] = in ? x[base + i] : 0.f;
                if (in) {
                    mn = fminf(mn, v[i]);
                    mx = fmaxf(mx, v[i]);
                }
            }
        }
#pragma unroll
        for (int o = 1; o < T; o <<= 1) {
            mn = fminf(mn, __shfl_xor(mn, o, 64));
            mx = fmaxf(mx, __shfl_xor(mx, o, 64));
        }
        float scale, zero;
        scale_zero(k, mn, mx, scale, zero);
        if (j == 0) {
            scales[gi] = scale;
            zeros[gi] = zero;
        }
        uint32_t w[2] = {0u, 0u};
#pragma unroll
        for (int i = 0; i < 16; i++) {
            uint32_t q = (uint32_t)(int)qcode(k, v[i], scale, zero);
            w[i / 8] |= q << (4 * (i % 8));
        }
        if (base + 16 <= n) {
            *(uint2 *)(codes + base / 2) = make_uint2(w[0], w[1]);
        } else {
            // a ragged end: whole bytes, the high nibble past the end left 0
            for (int i = 0; i < 16; i += 2)
                if (base + i < n)
                    codes[(base + i) / 2] = (uint8_t)((w[i / 8] >> (4 * (i % 8))) & (base + i + 1 < n ? 0xffu : 0x0fu));
        }
    }
}

// decoding is lane-contiguous like the whole-tensor kinds: chunk c holds
// values 4c..4c+3 (two bytes of codes), all in group 4c / G
template <int T>
__global__ void __launch_bounds__(256) dequantize_int4_kernel(const uint8_t *__restrict__ codes, int64_t n,
                                                              const float *__restrict__ scales,
                                                              const float *__restrict__ zeros, float *__restrict__ x) {
    constexpr int G = 16 * T;
    const QKind k = qkind(2);
    const int64_t n4 = n / 4, step = (int64_t)gridDim.x * blockDim.x * 4;
    for (int64_t c0 = (int64_t)blockIdx.x * blockDim.x * 4 + threadIdx.x; c0 < n4; c0 += step) {
        float v[4][4];
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const int64_t c = c0 + (int64_t)u * blockDim.x;
            if (c >= n4) break;
            const uint32_t b = ((const uint16_t *)codes)[c];
            const int64_t gi = (4 * c) / G;
            const float scale = scales[gi], zero = zeros[gi];
#pragma unroll
            for (int i = 0; i < 4; i++) v[u][i] = qdecode(k, (float)((b >> (4 * i)) & 15u), scale, zero);
        }
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const int64_t c = c0 + (int64_t)u * blockDim.x;
            if (c >= n4) break;
            ((float4 *)x)[c] = make_float4(v[u][0], v[u][1], v[u][2], v[u][3]);
        }
    }
    for (int64_t i = n4 * 4 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t b = codes[i / 2];
        const int64_t gi = i / G;
        x[i] = qdecode(k, (float)((b >> (4 * (i & 1))) & 15u), scales[gi], zeros[gi]);
    }
}

// ------------------------------------------------------------------ launches

static int grid_cap(int64_t work, int64_t per_block, int cap) {
    int64_t g = (work + per_block - 1) / per_block;
    return (int)(g < 1 ? 1 : (g > cap ? cap : g));
}

void launch_quantize(int kind, int64_t n, int group, const float *x, void *codes, float *scales, float *zeros,
                     float2 *part, hipStream_t st) {
    if (n <= 0) return;
    if (kind == 0 || kind == 1) {
        const int np = grid_cap(n, 256 * 64, kQuantPartials);   // partials: 512 float2 = a 4 KB buffer
        hipLaunchKernelGGL(minmax_partial_kernel, dim3(np), dim3(256), 0, st, x, n, part);
        hipLaunchKernelGGL(scale_zero_kernel, dim3(1), dim3(64), 0, st, (const float2 *)part, np, kind, scales, zeros);
        const int g = grid_cap(n / 16 + 1, 256, 8192);
        if (kind == 0)
            hipLaunchKernelGGL(quantize_whole_kernel<0>, dim3(g), dim3(256), 0, st, x, n, scales, zeros, codes);
        else
            hipLaunchKernelGGL(quantize_whole_kernel<1>, dim3(g), dim3(256), 0, st, x, n, scales, zeros, codes);
    } else {
        const int64_t ng = (n + group - 1) / group;
        const int T = group / 16;
        const int g = grid_cap(ng, 256 / T, 8192);
#define Q4(TV) hipLaunchKernelGGL(quantize_int4_kernel<TV>, dim3(g), dim3(256), 0, st, x, n, ng, scales, zeros, (uint8_t *)codes)
        switch (T) {
            case 1: Q4(1); break;
            case 2: Q4(2); break;
            case 4: Q4(4); break;
            case 8: Q4(8); break;
            case 16: Q4(16); break;
            case 32: Q4(32); break;
            default: Q4(64); break;
        }
#undef Q4
    }
    HIP_CHECK(hipGetLastError());
}

void launch_dequantize(int kind, int64_t n, int group, const void *codes, const float *scales, const float *zeros,
                       float *x, hipStream_t st) {
    if (n <= 0) return;
    const int g = grid_cap((n + 15) / 16, 256, 8192);
    if (kind == 0) {
        hipLaunchKernelGGL(dequantize_whole_kernel<0>, dim3(g), dim3(256), 0, st, codes, n, scales, zeros, x);
    } else if (kind == 1) {
        hipLaunchKernelGGL(dequantize_whole_kernel<1>, dim3(g), dim3(256), 0, st, codes, n, scales, zeros, x);
    } else {
        const int T = group / 16;
#define D4(TV) hipLaunchKernelGGL(dequantize_int4_kernel<TV>, dim3(g), dim3(256), 0, st, (const uint8_t *)codes, n, scales, zeros, x)
        switch (T) {
            case 1: D4(1); break;
            case 2: D4(2); break;
            case 4: D4(4); break;
            case 8: D4(8); break;
            case 16: D4(16); break;
            case 32: D4(32); break;
            default: D4(64); break;
        }
#undef D4
    }
    HIP_CHECK(hipGetLastError());
}

}  // namespace tnc

// ------------------------------------------------------------------ quantize without allocation
namespace tnc {

// The min/max partials of the whole-tensor kinds live in this array for
// tnc_quantize_noalloc: one copy per GPU, held until the process ends.  Host
// code reaches it only through the address hipGetSymbolAddress returns on
// each device (the array's name is a host-side stand-in there).
static __device__ __align__(256) float2 scratch[kQuantPartials];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float2 *g_scratch[kMaxDevices] = {};

// the array's device address on the current device, resolved once per device
float2 *scratch_on_current_device() {
    int dev = 0;
    HIP_CHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) TNC_THROW(TNC_EUNSUPPORTED, "device id above 63");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) TNC_THROW(TNC_EDEVICE, "hipGetSymbolAddress returned NULL for the codec scratch array");
        g_scratch[dev] = (float2 *)p;
    }
    return g_scratch[dev];
}
}  // namespace

}  // namespace tnc

extern "C" int tnc_quantize_noalloc(int32_t kind, int64_t n, const float *x, int32_t group, void *codes,
                                    float *scales, float *zeros, void *hip_stream) {
    using namespace tnc;
    try {
        if (n < 0) TNC_THROW(TNC_EINVAL, "negative length");
        const int g = codec_group(kind, group);
        if (n == 0) return TNC_OK;
        if (!x || !codes || !scales || !zeros) TNC_THROW(TNC_EINVAL, "NULL buffer");
        if (((uintptr_t)x & 15u) || ((uintptr_t)codes & 15u))
            TNC_THROW(TNC_EINVAL, "values and codes must be 16-byte aligned");
        // the whole-tensor kinds write one partial per block of the min/max
        // pass; that pass never launches more blocks than the array holds
        if ((kind == 0 || kind == 1) && grid_cap(n, 256 * 64, kQuantPartials) > kQuantPartials)
            TNC_THROW(TNC_EINVAL, "min/max pass needs more partials than the scratch array holds");
        float2 *part = scratch_on_current_device();
        launch_quantize(kind, n, g, x, codes, scales, zeros, part, (hipStream_t)hip_stream);
        return TNC_OK;
    } catch (const Error &e) {
        set_error(e.msg);
        return e.code;
    }
}
