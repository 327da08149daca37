// HIP kernels for gfx950: operand permutes, slice selection of the input
// tensors, batched complex GEMMs (complex64 on FP32 matrix cores; FP16/BF16
// 4M and 3M on 16-bit matrix cores with FP32 accumulation and a power-of-two
// output scale), and the FP64 cross-slice amplitude sum.
//
// Complex storage: C64 = float2 (re, im); 16-bit forms = one 32-bit word per
// entry, re in the low half, im in the high half (paper Sec. 3.3: complex-half
// as a real tensor with a trailing re/im mode).
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <algorithm>

#include "common.h"
#include "device_util.h"

namespace tnc {

// ===================================================================== small utilities

__global__ void fill_u32_kernel(uint32_t *p, uint32_t v, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void fill_f64_kernel(double *p, double v, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

static int grid_for(int64_t n, int threads, int cap = 65536) {
    int64_t g = (n + threads - 1) / threads;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

void launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(fill_u32_kernel, dim3(grid_for(n, 256)), dim3(256), 0, st, p, v, n);
    HIP_CHECK(hipGetLastError());
}
void launch_fill_f64(double *p, double v, int64_t n, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(fill_f64_kernel, dim3(grid_for(n, 256)), dim3(256), 0, st, p, v, n);
    HIP_CHECK(hipGetLastError());
}

// Operand stand-ins for the autotuner: each 32-bit word gets a hash of its
// index mapped to two 16-bit values (or one float) uniform in [-1, 1), so the
// timed kernels toggle their matrix cores as on real data (a loaded GPU's
// clock depends on it).
__global__ void fill_random_kernel(uint32_t *p, int64_t n_words, uint32_t seed, int kind) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n_words;
         i += (int64_t)gridDim.x * blockDim.x) {
        uint32_t h = (uint32_t)i * 0x9E3779B1u ^ (uint32_t)(i >> 32) * 0x85EBCA77u ^ seed;
        h ^= h >> 16;
        h *= 0x7FEB352Du;
        h ^= h >> 15;
        h *= 0x846CA68Bu;
        h ^= h >> 16;
        const float lo = (float)(h & 0xffffu) * (1.f / 32768.f) - 1.f, hi = (float)(h >> 16) * (1.f / 32768.f) - 1.f;
        if (kind == 0) p[i] = __float_as_uint((float)(h >> 8) * (1.f / 8388608.f) - 1.f);
        else if (kind == 1) p[i] = f2h_bits(lo) | (f2h_bits(hi) << 16);
        else p[i] = f2bf_bits(lo) | (f2bf_bits(hi) << 16);
    }
}

void launch_fill_random(Dtype dt, void *p, int64_t n_words, uint32_t seed, hipStream_t st) {
    if (n_words <= 0) return;
    const int kind = dt == Dtype::C64 ? 0 : (dt == Dtype::BF16 ? 2 : 1);
    hipLaunchKernelGGL(fill_random_kernel, dim3(grid_for(n_words, 256, 16384)), dim3(256), 0, st, (uint32_t *)p,
                       n_words, seed, kind);
    HIP_CHECK(hipGetLastError());
}

// ===================================================================== permute (bit permutation)
//
// dst[s][j] = src[s * src_slice_stride + slice_off[s] + sum_b bit_b(j) * stride[b]]
// The destination is written contiguously; reads follow the permutation.

template <typename W>
__global__ void permute_naive_kernel(const W *__restrict__ src, W *__restrict__ dst, PermuteDesc d,
                                     int64_t n_out, int64_t src_ss, const int64_t *__restrict__ soff,
                                     int64_t dst_ss) {
    const int s = blockIdx.y;
    const W *sp = src + s * src_ss + (soff ? soff[s] : 0);
    W *dp = dst + s * dst_ss;
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n_out;
         j += (int64_t)gridDim.x * blockDim.x) {
        int64_t o = 0;
        int64_t jj = j;
        for (int b = 0; b < d.rank; b++) {
            if (jj & 1) o += d.src_stride[b];
            jj >>= 1;
        }
        dp[j] = sp[o];
    }
}

// Tiled variant: a tile is every combination of the tile bits T (the w
// lowest destination bits and the destination bits holding the w lowest
// source bits, grown to 12 bits with further low bits of either side); the
// remaining bits select the tile.  The tile is read in
// source order and written in destination order through LDS, so both HBM
// streams are runs of at least 2^w entries; every thread moves 16-byte
// chunks (VEC entries, contiguous in the source when read and in the
// destination when written).  In-tile offsets depend only on the thread, so
// they are computed once; the LDS index is XOR-swizzled so both the scattered
// and the sequential accesses spread over the banks.
template <typename W, int VEC>
__global__ void __launch_bounds__(256) permute_tiled_kernel(const W *__restrict__ src, W *__restrict__ dst,
                                                            PermuteDesc d, int64_t n_tiles, int64_t src_ss,
                                                            const int64_t *__restrict__ soff, int64_t dst_ss,
                                                            TileBits tb) {
    typedef W Vec __attribute__((ext_vector_type(VEC)));
    constexpr int LV = VEC == 4 ? 2 : 1;
    constexpr int TE = 1 << kPermTileBits;
    constexpr int CPT = TE / VEC / 256;   // chunks per thread for the largest tile
    __shared__ W tile[TE];
    const int s = blockIdx.y;
    const W *sp = src + s * src_ss + (soff ? soff[s] : 0);
    W *dp = dst + s * dst_ss;
    const int te = 1 << tb.nt;
    const int nch = te >> LV;
    int64_t so_c[CPT], do_c[CPT];
    int li_q[CPT][VEC];
    for (int j = 0; j < CPT; j++) {
        const int c = threadIdx.x + j * 256;
        // read side: chunk c covers source-order indices c*VEC .. c*VEC+VEC-1
        int64_t so = 0;
        int li_c = 0;
        for (int i = LV; i < tb.nt; i++)
            if (((c << LV) >> i) & 1) {
                so += d.src_stride[tb.src_order[i]];
                li_c |= 1 << tb.lds_bit[i];
            }
        so_c[j] = so;
        for (int q = 0; q < VEC; q++) {
            int li = li_c;
            for (int i = 0; i < LV; i++)
                if ((q >> i) & 1) li |= 1 << tb.lds_bit[i];
            li_q[j][q] = li ^ ((li >> 5) & 31);
        }
        // write side: chunk c covers destination-order indices c*VEC .. +VEC-1
        int64_t dof = 0;
        for (int i = LV; i < tb.nt; i++)
            if (((c << LV) >> i) & 1) dof += (int64_t)1 << tb.dst_order[i];
        do_c[j] = dof;
    }
    for (int64_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
        int64_t dbase = 0, sbase = 0;
        int64_t tt = t;
        for (int i = 0; i < tb.n_rest; i++) {
            int b = tb.rest[i];
            if (tt & 1) {
                dbase += (int64_t)1 << b;
                sbase += d.src_stride[b];
            }
            tt >>= 1;
        }
#pragma unroll
        for (int j = 0; j < CPT; j++) {
            if (threadIdx.x + j * 256 < nch) {
                Vec v = *(const Vec *)(sp + sbase + so_c[j]);
#pragma unroll
                for (int q = 0; q < VEC; q++) tile[li_q[j][q]] = v[q];
            }
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < CPT; j++) {
            const int c = threadIdx.x + j * 256;
            if (c < nch) {
                Vec v;
#pragma unroll
                for (int q = 0; q < VEC; q++) {
                    int e = (c << LV) + q;
                    v[q] = tile[e ^ ((e >> 5) & 31)];
                }
                *(Vec *)(dp + dbase + do_c[j]) = v;
            }
        }
        __syncthreads();
    }
}

void launch_permute(Dtype dt, const void *src, void *dst, const PermuteDesc &d, int64_t n_out, int S,
                    int64_t src_ss, const int64_t *soff, int64_t dst_ss, hipStream_t st) {
    if (n_out <= 0 || S <= 0) return;
    TileBits tb;
    const int LW = 5;
    bool tiled = plan_tile_bits(d, LW, kPermTileBits, tb);
    if (tiled) {
        int64_t n_tiles = n_out >> tb.nt;
        int g = grid_for(n_tiles, 1, 8192);
        if (dt == Dtype::C64)
            hipLaunchKernelGGL((permute_tiled_kernel<unsigned long long, 2>), dim3(g, S), dim3(256), 0, st,
                               (const unsigned long long *)src, (unsigned long long *)dst, d, n_tiles, src_ss, soff,
                               dst_ss, tb);
        else
            hipLaunchKernelGGL((permute_tiled_kernel<uint32_t, 4>), dim3(g, S), dim3(256), 0, st,
                               (const uint32_t *)src, (uint32_t *)dst, d, n_tiles, src_ss, soff, dst_ss, tb);
    } else {
        int g = grid_for(n_out, 256, 1 << 20);
        if (dt == Dtype::C64)
            hipLaunchKernelGGL((permute_naive_kernel<uint2>), dim3(g, S), dim3(256), 0, st,
                               (const uint2 *)src, (uint2 *)dst, d, n_out, src_ss, soff, dst_ss);
        else
            hipLaunchKernelGGL((permute_naive_kernel<uint32_t>), dim3(g, S), dim3(256), 0, st,
                               (const uint32_t *)src, (uint32_t *)dst, d, n_out, src_ss, soff, dst_ss);
    }
    HIP_CHECK(hipGetLastError());
}

// ===================================================================== leaf selection (slicing)
//
// One launch gathers every input tensor of a slice group: block (leaf, slice)
// copies the sub-tensor of leaf i at the fixed label values of slice
// sigma = sigma0 + s (recomputed labels: the bits above the sliced ones,
// which a pass adds to the group's base) into the arena, in the order its first step wants, and
// records its largest component (16-bit forms) and a zero exponent.

template <typename W>
__global__ void gather_leaves_kernel(const LeafDesc *__restrict__ descs, const int64_t *__restrict__ params,
                                     const W *__restrict__ leafdata, uint8_t *__restrict__ arena,
                                     uint32_t *__restrict__ maxw, double *__restrict__ expw, int64_t group_base,
                                     const int64_t *__restrict__ spoff) {
    const LeafDesc &L = descs[blockIdx.x];
    const int s = blockIdx.y;
    const int d = blockIdx.z;   // sparse-state block (0 otherwise)
    if (s >= L.n_slices || d >= L.nd) return;
    const int64_t sigma = params[0] + group_base + s;
    int64_t so = L.src_off + L.closed_off + (spoff ? spoff[L.sp_base + d] : 0);
    for (int j = 0; j < L.n_sliced; j++)
        if ((sigma >> L.slice_bit[j]) & 1) so += L.slice_stride[j];
    const int64_t n = (int64_t)1 << L.rank;
    W *dp = (W *)(arena + L.dst_byte_off) + (int64_t)s * L.dst_slice_stride + (int64_t)d * n;
    float mx = 0.f;
    for (int64_t j = threadIdx.x; j < n; j += blockDim.x) {
        int64_t o = so;
        for (int b = 0; b < L.rank; b++)
            if ((j >> b) & 1) o += L.stride[b];
        W v = leafdata[o];
        dp[j] = v;
        mx = fmaxf(mx, word_absmax(v));
    }
    if (maxw) {
        mx = block_max(mx);
        if (threadIdx.x == 0) {
            atomicMax(&maxw[L.max_slot + s * L.slot_stride], __float_as_uint(mx));
            expw[L.max_slot + s * L.slot_stride] = 0.0;
        }
    }
}

void launch_gather_leaves_impl(Dtype dt, int n_leaves, const LeafDesc *d_desc, const int64_t *d_params,
                               const void *leafdata, uint8_t *arena, uint32_t *maxw, double *expw,
                               int64_t group_base, int S, hipStream_t st, const int64_t *spoff, int nd_max) {
    if (n_leaves <= 0) return;
    const dim3 grid(n_leaves, S, nd_max);
    if (dt == Dtype::C64)
        hipLaunchKernelGGL((gather_leaves_kernel<uint2>), grid, dim3(64), 0, st, d_desc, d_params,
                           (const uint2 *)leafdata, arena, (uint32_t *)nullptr, (double *)nullptr, group_base, spoff);
    else if (dt == Dtype::F16)
        hipLaunchKernelGGL((gather_leaves_kernel<HalfWord>), grid, dim3(64), 0, st, d_desc, d_params,
                           (const HalfWord *)leafdata, arena, maxw, expw, group_base, spoff);
    else
        hipLaunchKernelGGL((gather_leaves_kernel<Bf16Word>), grid, dim3(64), 0, st, d_desc, d_params,
                           (const Bf16Word *)leafdata, arena, maxw, expw, group_base, spoff);
    HIP_CHECK(hipGetLastError());
}

// ===================================================================== block copies (sparse state)
//
// Destination block j of slice s takes source block k = idx[j] - lo of that
// slice when lo <= idx[j] < hi; otherwise it is zeroed (fill) or left alone.
// Blocks hold `block` entries; each thread moves 16 bytes at a time.

template <typename W>
__global__ void __launch_bounds__(256) block_copy_kernel(const W *__restrict__ src, int64_t src_ss, W *__restrict__ dst,
                                                         int64_t dst_ss, const int32_t *__restrict__ idx, int64_t lo,
                                                         int64_t hi, int64_t block, int fill) {
    const int64_t j = blockIdx.y;
    const int s = blockIdx.z;
    const int64_t k = (int64_t)idx[j] - lo;
    const bool take = k >= 0 && k < hi - lo;
    if (!take && !fill) return;
    constexpr int V = 16 / sizeof(W);
    typedef uint32_t u4 __attribute__((ext_vector_type(4)));
    W *d = dst + s * dst_ss + j * block;
    const W *sp = src + s * src_ss + (take ? k : 0) * block;
    if (block % V == 0) {
        for (int64_t e = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) * V; e < block;
             e += (int64_t)gridDim.x * blockDim.x * V) {
            u4 v = {0u, 0u, 0u, 0u};
            if (take) v = *(const u4 *)(sp + e);
            *(u4 *)(d + e) = v;
        }
    } else {
        for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < block; e += (int64_t)gridDim.x * blockDim.x) {
            W v{};
            if (take) v = sp[e];
            d[e] = v;
        }
    }
}

void launch_block_copy(Dtype dt, const void *src, int64_t src_ss, void *dst, int64_t dst_ss, const int32_t *idx,
                       int64_t n_blocks, int64_t lo, int64_t hi, int64_t block, int S, bool fill, hipStream_t st) {
    if (n_blocks <= 0 || S <= 0) return;
    const int es = elem_bytes(dt);
    const int gx = (int)std::max<int64_t>(1, std::min<int64_t>((block * es / 16 + 255) / 256, 64));
    for (int64_t j0 = 0; j0 < n_blocks; j0 += 65535) {
        const int64_t nb = std::min<int64_t>(65535, n_blocks - j0);
        const dim3 grid(gx, (unsigned)nb, S);
        uint8_t *d = (uint8_t *)dst + j0 * block * es;
        if (dt == Dtype::C64)
            hipLaunchKernelGGL((block_copy_kernel<uint2>), grid, dim3(256), 0, st, (const uint2 *)src, src_ss, (uint2 *)d,
                               dst_ss, idx + j0, lo, hi, block, (int)fill);
        else
            hipLaunchKernelGGL((block_copy_kernel<uint32_t>), grid, dim3(256), 0, st, (const uint32_t *)src, src_ss,
                               (uint32_t *)d, dst_ss, idx + j0, lo, hi, block, (int)fill);
    }
    HIP_CHECK(hipGetLastError());
}

// ===================================================================== FP64 cross-slice sum
//
// acc[j] += 2^exp[s] * R[s][idx(x_j)] for s = 0..S-1 in order (deterministic).
// idx(x) takes bit b from qubit qubit_of_bit[b] of the bitstring.

template <typename W>
__global__ void accumulate_kernel(const W *__restrict__ R, int rank, int S, int64_t ss,
                                  const double *__restrict__ expR, int es, int64_t nbits,
                                  const uint64_t *__restrict__ bits, const int *__restrict__ qob,
                                  double *__restrict__ acc, const int32_t *__restrict__ map) {
    int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= nbits) return;
    int64_t idx = 0;
    if (map) {
        idx = map[j];   // sparse state: the root block of bitstring j
    } else {
        const uint64_t x = bits[j];
        for (int b = 0; b < rank; b++) idx |= (int64_t)((x >> qob[b]) & 1ull) << b;
    }
    double re = acc[2 * j], im = acc[2 * j + 1];
    for (int s = 0; s < S; s++) {
        double2 v = word_to_double2(R[s * ss + idx]);
        double e = expR ? expR[s * es] : 0.0;
        re += ldexp(v.x, (int)e);
        im += ldexp(v.y, (int)e);
    }
    acc[2 * j] = re;
    acc[2 * j + 1] = im;
}

void launch_accumulate(Dtype dt, const void *R, int rank, int S, int64_t ss, const double *expR, int es,
                       int64_t nbits, const uint64_t *d_bits, const int *d_qob, double *acc, hipStream_t st,
                       const int32_t *d_map) {
    if (nbits <= 0 || S <= 0) return;
    int g = (int)((nbits + 255) / 256);
    if (dt == Dtype::C64)
        hipLaunchKernelGGL((accumulate_kernel<uint2>), dim3(g), dim3(256), 0, st, (const uint2 *)R, rank, S, ss,
                           (const double *)nullptr, es, nbits, d_bits, d_qob, acc, d_map);
    else if (dt == Dtype::F16)
        hipLaunchKernelGGL((accumulate_kernel<HalfWord>), dim3(g), dim3(256), 0, st, (const HalfWord *)R, rank, S,
                           ss, expR, es, nbits, d_bits, d_qob, acc, d_map);
    else
        hipLaunchKernelGGL((accumulate_kernel<Bf16Word>), dim3(g), dim3(256), 0, st, (const Bf16Word *)R, rank, S,
                           ss, expR, es, nbits, d_bits, d_qob, acc, d_map);
    HIP_CHECK(hipGetLastError());
}

// ===================================================================== tensor max (for one-off contractions)

template <typename W>
__global__ void tensor_max_kernel(const W *__restrict__ x, int64_t n, int64_t ss, uint32_t *__restrict__ out) {
    const int s = blockIdx.y;
    float mx = 0.f;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        mx = fmaxf(mx, word_absmax(x[s * ss + i]));
    mx = block_max(mx);
    if (threadIdx.x == 0) atomicMax(&out[s], __float_as_uint(mx));
}

void launch_tensor_max(Dtype dt, const void *x, int64_t n, int S, int64_t ss, uint32_t *out, hipStream_t st) {
    int g = grid_for(n, 256, 4096);
    if (dt == Dtype::C64)
        hipLaunchKernelGGL((tensor_max_kernel<uint2>), dim3(g, S), dim3(256), 0, st, (const uint2 *)x, n, ss, out);
    else if (dt == Dtype::F16)
        hipLaunchKernelGGL((tensor_max_kernel<HalfWord>), dim3(g, S), dim3(256), 0, st, (const HalfWord *)x, n, ss, out);
    else
        hipLaunchKernelGGL((tensor_max_kernel<Bf16Word>), dim3(g, S), dim3(256), 0, st, (const Bf16Word *)x, n, ss, out);
    HIP_CHECK(hipGetLastError());
}

// ===================================================================== input conversion
// complex128 (interleaved doubles) -> storage words, round to nearest even.
template <typename W>
__global__ void convert_c128_kernel(const double *__restrict__ src, int64_t n, W *__restrict__ dst) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = Pack<W>::make((float)src[2 * i], (float)src[2 * i + 1]);
}

void launch_convert_c128(const double *src, int64_t n, Dtype dt, void *dst, hipStream_t st) {
    if (n <= 0) return;
    int g = grid_for(n, 256, 4096);
    if (dt == Dtype::C64)
        hipLaunchKernelGGL((convert_c128_kernel<uint2>), dim3(g), dim3(256), 0, st, src, n, (uint2 *)dst);
    else if (dt == Dtype::F16)
        hipLaunchKernelGGL((convert_c128_kernel<HalfWord>), dim3(g), dim3(256), 0, st, src, n, (HalfWord *)dst);
    else
        hipLaunchKernelGGL((convert_c128_kernel<Bf16Word>), dim3(g), dim3(256), 0, st, src, n, (Bf16Word *)dst);
    HIP_CHECK(hipGetLastError());
}

}  // namespace tnc
