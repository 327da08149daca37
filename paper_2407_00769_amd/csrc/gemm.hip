// Batched complex GEMM for one contraction step (paper Eq. contraction in
// its pure-GEMM form, Sec. 3.3):
//     C[s][b][m][n] = sum_k A[s][b][m][k] * B[s][b][n][k]
// A is the large operand, B the small one; both are K-contiguous, C is
// N-contiguous.  s is the slice in flight, b the inner batch.
//
// Forms:
//   4M   -- one real GEMM  C'[m][2n+d] = sum_{k'} A'[m][k'] B'[k'][2n+d], with
//           A' the interleaved (re, im) view of A (k' = 2k + c) and B' the
//           small operand padded on the fly to [B(re,-im), B(im,re)] (paper
//           Eq. eq_modified2); 8 real flops per complex multiply-add.
//   3M   -- T1 = Ar Br, T2 = Ai Bi, T3 = (Ar+Ai)(Br+Bi) with the sums rounded
//           once to the storage type; Cr = T1 - T2, Ci = T3 - T1 - T2.
// 16-bit results are stored as value * 2^-shift (see device_util.h).
#include <hip/hip_runtime.h>

#include <type_traits>

#include "common.h"
#include "device_util.h"

namespace tnc {

typedef _Float16 half8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <typename W> __device__ __forceinline__ float round_to_storage(float x);
template <> __device__ __forceinline__ float round_to_storage<HalfWord>(float x) {
    return __half2float(__float2half_rn(x));
}
template <> __device__ __forceinline__ float round_to_storage<Bf16Word>(float x) {
    return __uint_as_float(f2bf_bits(x) << 16);
}
template <> __device__ __forceinline__ float round_to_storage<uint2>(float x) { return x; }

// Store one output entry: scale, round, and return its largest component.
template <typename W, bool SCALE>
__device__ __forceinline__ float store_entry(W *p, float re, float im, float scale) {
    if (SCALE) {
        re *= scale;
        im *= scale;
    }
    W w = Pack<W>::make(re, im);
    *p = w;
    if (!SCALE) return 0.f;
    float2 f = unpack(w);
    return absmax_nan(f.x, f.y);
}

template <bool SCALE>
__device__ __forceinline__ void finish_max(const ScaleRefs &sc, int s, float mx) {
    if (!SCALE) return;
    mx = block_max(mx);
    if (threadIdx.x == 0) {
        atomicMax(&sc.maxC[s], __float_as_uint(mx));
        if (!(mx <= 3.0e38f) && sc.flag) atomicOr(sc.flag, 1u);   // rounded to inf, or NaN
    }
}

// exact 2^-shift as a float (shift is clamped to the normal range)
__device__ __forceinline__ float pow2_neg(int shift) {
    shift = shift > 126 ? 126 : (shift < -126 ? -126 : shift);
    return __uint_as_float((uint32_t)(127 - shift) << 23);
}

// ===================================================================== naive: thread per output

template <typename W, bool SCALE, bool M3>
__global__ void __launch_bounds__(256) gemm_naive_kernel(const W *__restrict__ A, const W *__restrict__ B,
                                                         W *__restrict__ C, GemmShape g, ScaleRefs sc) {
    const int s = blockIdx.z;
    const int64_t b = blockIdx.y;
    int shift = SCALE ? step_shift(sc, s) : 0;
    if (SCALE && blockIdx.x == 0 && b == 0 && threadIdx.x == 0) record_exponent(sc, s, shift);
    const float scale = pow2_neg(shift);
    const W *Ap = A + s * g.sA + b * g.bA;
    const W *Bp = B + s * g.sB + b * g.bB;
    W *Cp = C + s * g.sC + b * g.bC;
    float mx = 0.f;
    const int64_t total = g.M * g.N;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t m = i / g.N, n = i - m * g.N;
        const W *ar = Ap + m * g.K;
        const W *br = Bp + n * g.K;
        float re = 0.f, im = 0.f;
        if (!M3) {
            for (int64_t k = 0; k < g.K; k++) {
                float2 a = unpack(ar[k]), bb = unpack(br[k]);
                re = fmaf(a.x, bb.x, re);
                re = fmaf(-a.y, bb.y, re);
                im = fmaf(a.x, bb.y, im);
                im = fmaf(a.y, bb.x, im);
            }
        } else {
            float t1 = 0.f, t2 = 0.f, t3 = 0.f;
            for (int64_t k = 0; k < g.K; k++) {
                float2 a = unpack(ar[k]), bb = unpack(br[k]);
                t1 = fmaf(a.x, bb.x, t1);
                t2 = fmaf(a.y, bb.y, t2);
                t3 = fmaf(round_to_storage<W>(a.x + a.y), round_to_storage<W>(bb.x + bb.y), t3);
            }
            re = t1 - t2;
            im = t3 - t1 - t2;
        }
        mx = fmaxf(mx, store_entry<W, SCALE>(Cp + i, re, im, scale));
    }
    finish_max<SCALE>(sc, s, mx);
}

// ===================================================================== skinny: row per thread (VALU)
// Each thread owns one row m and NN consecutive columns; B's NN x KC chunk is
// staged in LDS.  For thin steps, which are bound by HBM traffic.

template <typename W, int NN, bool SCALE, bool M3>
__global__ void __launch_bounds__(256) gemm_skinny_kernel(const W *__restrict__ A, const W *__restrict__ B,
                                                          W *__restrict__ C, GemmShape g, ScaleRefs sc) {
    constexpr int KC = 64;
    __shared__ float2 Bs[NN][KC];
    __shared__ float Bsum[M3 ? NN : 1][KC];
    const int s = blockIdx.z;
    const int64_t nchunks = (g.N + NN - 1) / NN;
    const int64_t b = blockIdx.y / nchunks;
    const int64_t n0 = (blockIdx.y - b * nchunks) * NN;
    int shift = SCALE ? step_shift(sc, s) : 0;
    if (SCALE && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) record_exponent(sc, s, shift);
    const float scale = pow2_neg(shift);
    const W *Ap = A + s * g.sA + b * g.bA;
    const W *Bp = B + s * g.sB + b * g.bB;
    W *Cp = C + s * g.sC + b * g.bC;
    const int nn = (int)((g.N - n0) < NN ? (g.N - n0) : NN);
    const int64_t m = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const bool live = m < g.M;
    float2 acc[NN];
    float t3[M3 ? NN : 1];
#pragma unroll
    for (int j = 0; j < NN; j++) acc[j] = make_float2(0.f, 0.f);
#pragma unroll
    for (int j = 0; j < (M3 ? NN : 1); j++) t3[j] = 0.f;
    for (int64_t k0 = 0; k0 < g.K; k0 += KC) {
        const int kc = (int)((g.K - k0) < KC ? (g.K - k0) : KC);
        __syncthreads();
        for (int e = threadIdx.x; e < NN * KC; e += blockDim.x) {
            int j = e / KC, kk = e - j * KC;
            float2 v = make_float2(0.f, 0.f);
            if (j < nn && kk < kc) v = unpack(Bp[(n0 + j) * g.K + k0 + kk]);
            Bs[j][kk] = v;
            if constexpr (M3) Bsum[j][kk] = round_to_storage<W>(v.x + v.y);
        }
        __syncthreads();
        if (live) {
            const W *ar = Ap + m * g.K + k0;
            for (int kk = 0; kk < kc; kk++) {
                float2 a = unpack(ar[kk]);
                if constexpr (!M3) {
#pragma unroll
                    for (int j = 0; j < NN; j++) {
                        float2 bb = Bs[j][kk];
                        acc[j].x = fmaf(a.x, bb.x, acc[j].x);
                        acc[j].x = fmaf(-a.y, bb.y, acc[j].x);
                        acc[j].y = fmaf(a.x, bb.y, acc[j].y);
                        acc[j].y = fmaf(a.y, bb.x, acc[j].y);
                    }
                } else {
                    float as = round_to_storage<W>(a.x + a.y);
#pragma unroll
                    for (int j = 0; j < NN; j++) {
                        float2 bb = Bs[j][kk];
                        acc[j].x = fmaf(a.x, bb.x, acc[j].x);   // T1
                        acc[j].y = fmaf(a.y, bb.y, acc[j].y);   // T2
                        t3[j] = fmaf(as, Bsum[j][kk], t3[j]);   // T3
                    }
                }
            }
        }
    }
    float mx = 0.f;
    if (live) {
        W *cr = Cp + m * g.N + n0;
#pragma unroll
        for (int j = 0; j < NN; j++) {
            if (j < nn) {
                float re, im;
                if constexpr (!M3) {
                    re = acc[j].x;
                    im = acc[j].y;
                } else {
                    re = acc[j].x - acc[j].y;
                    im = t3[j] - acc[j].x - acc[j].y;
                }
                mx = fmaxf(mx, store_entry<W, SCALE>(cr + j, re, im, scale));
            }
        }
    }
    finish_max<SCALE>(sc, s, mx);
}

// ===================================================================== matrix cores, 16-bit 4M
//
// Block tile BM rows x BN complex columns, k-tile BK complex; WM x WN waves,
// each wave (BM/WM) x (2BN/WN) real outputs as 32x32 MFMA blocks.
// v_mfma_f32_32x32x16_{f16,bf16}: lane l holds A'[l%32][8(l/32)+0..7] and
// B'[8(l/32)+0..7][l%32]; result register r of lane l is row
// 8(r/4) + 4(l/32) + r%4, column l%32.

template <bool BF> __device__ __forceinline__ floatx16 mfma16(u32x4 a, u32x4 b, floatx16 c) {
    if constexpr (BF)
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8_t, a),
                                                       __builtin_bit_cast(bf16x8_t, b), c, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(half8_t, a),
                                                      __builtin_bit_cast(half8_t, b), c, 0, 0, 0);
}

__device__ __forceinline__ uint32_t swap_halves(uint32_t w) { return (w >> 16) | (w << 16); }

// XCD-aware order: consecutive tiles of one row block land on one XCD (8 per chip).
__device__ __forceinline__ int64_t xcd_tile(int64_t w, int64_t total) {
    if (total % 8) return w;
    return (w % 8) * (total / 8) + w / 8;
}

template <bool BF, int BM, int BN, int BK, int WM, int WN, bool SCALE>
__global__ void __launch_bounds__(64 * WM * WN)
    gemm_mfma_h4m_kernel(const uint32_t *__restrict__ A, const uint32_t *__restrict__ B, uint32_t *__restrict__ C,
                         GemmShape g, ScaleRefs sc) {
    using W = typename std::conditional<BF, Bf16Word, HalfWord>::type;
    constexpr int NT = 64 * WM * WN;
    constexpr int PAD = 4;
    constexpr int LDA = BK + PAD, LDB = BK + PAD;
    constexpr int WTM = BM / WM, WTN = 2 * BN / WN;   // wave tile: rows, real cols
    constexpr int FM = WTM / 32, FN = WTN / 32;
    static_assert(FM >= 1 && FN >= 1, "wave tile too small");
    constexpr int A_CHUNKS = BM * BK / 4, B_CHUNKS = BN * BK / 4;   // 16-byte chunks
    constexpr int A_PER = (A_CHUNKS + NT - 1) / NT, B_PER = (B_CHUNKS + NT - 1) / NT;
    constexpr int LDS_AB = 2 * (BM * LDA + BN * LDB);
    constexpr int LDS_C = BM * BN;
    __shared__ uint32_t lds[LDS_AB > LDS_C ? LDS_AB : LDS_C];
    auto As = [&](int buf) { return lds + buf * (BM * LDA); };
    auto Bs = [&](int buf) { return lds + 2 * BM * LDA + buf * (BN * LDB); };

    const int s = blockIdx.z;
    const int64_t b = blockIdx.y;
    const int64_t tiles_n = (g.N + BN - 1) / BN;
    const int64_t tiles_m = (g.M + BM - 1) / BM;
    const int64_t t = xcd_tile(blockIdx.x, tiles_m * tiles_n);
    const int64_t m0 = (t / tiles_n) * BM, n0 = (t % tiles_n) * BN;
    int shift = SCALE ? step_shift(sc, s) : 0;
    if (SCALE && blockIdx.x == 0 && b == 0 && threadIdx.x == 0) record_exponent(sc, s, shift);
    const float scale = pow2_neg(shift);

    const uint32_t *Ap = A + s * g.sA + b * g.bA;
    const uint32_t *Bp = B + s * g.sB + b * g.bB;
    uint32_t *Cp = C + s * g.sC + b * g.bC;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave / WN, wn = wave % WN;

    u32x4 ra[A_PER], rb[B_PER];
    auto gload = [&](int64_t k0) {
#pragma unroll
        for (int i = 0; i < A_PER; i++) {
            int c = tid + i * NT;
            u32x4 v = {0u, 0u, 0u, 0u};
            if (c < A_CHUNKS) {
                int row = c / (BK / 4), col = (c % (BK / 4)) * 4;
                int64_t gm = m0 + row, gk = k0 + col;
                if (gm < g.M && gk < g.K) v = *(const u32x4 *)(Ap + gm * g.K + gk);
            }
            ra[i] = v;
        }
#pragma unroll
        for (int i = 0; i < B_PER; i++) {
            int c = tid + i * NT;
            u32x4 v = {0u, 0u, 0u, 0u};
            if (c < B_CHUNKS) {
                int row = c / (BK / 4), col = (c % (BK / 4)) * 4;
                int64_t gn = n0 + row, gk = k0 + col;
                if (gn < g.N && gk < g.K) v = *(const u32x4 *)(Bp + gn * g.K + gk);
            }
            rb[i] = v;
        }
    };
    auto sstore = [&](int buf) {
#pragma unroll
        for (int i = 0; i < A_PER; i++) {
            int c = tid + i * NT;
            if (c < A_CHUNKS) {
                int row = c / (BK / 4), col = (c % (BK / 4)) * 4;
                *(u32x4 *)(As(buf) + row * LDA + col) = ra[i];
            }
        }
#pragma unroll
        for (int i = 0; i < B_PER; i++) {
            int c = tid + i * NT;
            if (c < B_CHUNKS) {
                int row = c / (BK / 4), col = (c % (BK / 4)) * 4;
                *(u32x4 *)(Bs(buf) + row * LDB + col) = rb[i];
            }
        }
    };

    floatx16 acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; i++)
#pragma unroll
        for (int j = 0; j < FN; j++)
#pragma unroll
            for (int r = 0; r < 16; r++) acc[i][j][r] = 0.f;

    const int64_t nk = (g.K + BK - 1) / BK;
    gload(0);
    sstore(0);
    __syncthreads();
    const int kq = (lane >> 5) * 4;     // this lane's 4 complex k within an 8-complex MFMA step
    const int d = lane & 1;             // B' column parity: 0 -> (br, -bi), 1 -> (bi, br)
    for (int64_t kt = 0; kt < nk; kt++) {
        const int buf = kt & 1;
        if (kt + 1 < nk) gload((kt + 1) * BK);
#pragma unroll
        for (int kk = 0; kk < BK / 8; kk++) {
            u32x4 af[FM], bf[FN];
#pragma unroll
            for (int i = 0; i < FM; i++) {
                int row = wm * WTM + i * 32 + (lane & 31);
                af[i] = *(const u32x4 *)(As(buf) + row * LDA + kk * 8 + kq);
            }
#pragma unroll
            for (int j = 0; j < FN; j++) {
                int ncol = (wn * WTN + j * 32 + (lane & 31)) >> 1;
                u32x4 v = *(const u32x4 *)(Bs(buf) + ncol * LDB + kk * 8 + kq);
                if (d == 0) {
                    v[0] ^= 0x80000000u; v[1] ^= 0x80000000u; v[2] ^= 0x80000000u; v[3] ^= 0x80000000u;
                } else {
                    v[0] = swap_halves(v[0]); v[1] = swap_halves(v[1]);
                    v[2] = swap_halves(v[2]); v[3] = swap_halves(v[3]);
                }
                bf[j] = v;
            }
#pragma unroll
            for (int i = 0; i < FM; i++)
#pragma unroll
                for (int j = 0; j < FN; j++) acc[i][j] = mfma16<BF>(af[i], bf[j], acc[i][j]);
        }
        __syncthreads();
        if (kt + 1 < nk) {
            sstore(buf ^ 1);
            __syncthreads();
        }
    }

    // epilogue: scale, round, stage the tile in LDS as complex words, write rows out
    uint16_t *Cs = (uint16_t *)lds;   // [BM][2*BN] halves
#pragma unroll
    for (int i = 0; i < FM; i++)
#pragma unroll
        for (int j = 0; j < FN; j++)
#pragma unroll
            for (int r = 0; r < 16; r++) {
                int row = wm * WTM + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                int col = wn * WTN + j * 32 + (lane & 31);   // real column 2n + part
                float v = acc[i][j][r];
                if (SCALE) v *= scale;
                uint32_t h = BF ? f2bf_bits(v) : f2h_bits(v);
                Cs[row * (2 * BN) + col] = (uint16_t)h;
            }
    __syncthreads();
    float mx = 0.f;
    constexpr int C_CHUNKS = BM * BN / 4;
    for (int c = tid; c < C_CHUNKS; c += NT) {
        int row = c / (BN / 4), col = (c % (BN / 4)) * 4;
        int64_t gm = m0 + row, gn = n0 + col;
        u32x4 v = *(const u32x4 *)(lds + row * BN + col);
        if (gm < g.M && gn < g.N) {
            *(u32x4 *)(Cp + gm * g.N + gn) = v;
            if (SCALE) {
#pragma unroll
                for (int q = 0; q < 4; q++) {
                    float2 f = unpack(W{v[q]});
                    mx = fmaxf(mx, absmax_nan(f.x, f.y));
                }
            }
        }
    }
    finish_max<SCALE>(sc, s, mx);
}

// ===================================================================== matrix cores, complex64 4M
// v_mfma_f32_32x32x2f32: lane l holds A'[l%32][l/32] and B'[l/32][l%32];
// one MFMA per complex k (k' = 2k + c).

template <int BM, int BN, int BK, int WM, int WN>
__global__ void __launch_bounds__(64 * WM * WN)
    gemm_mfma_c64_kernel(const float2 *__restrict__ A, const float2 *__restrict__ B, float2 *__restrict__ C,
                         GemmShape g) {
    constexpr int NT = 64 * WM * WN;
    constexpr int LDA = BK + 1, LDB = BK + 1;
    constexpr int WTM = BM / WM, WTN = 2 * BN / WN;
    constexpr int FM = WTM / 32, FN = WTN / 32;
    static_assert(FM >= 1 && FN >= 1, "wave tile too small");
    constexpr int A_CHUNKS = BM * BK / 2, B_CHUNKS = BN * BK / 2;   // 16-byte chunks (2 complex)
    constexpr int A_PER = (A_CHUNKS + NT - 1) / NT, B_PER = (B_CHUNKS + NT - 1) / NT;
    constexpr int LDS_AB = 2 * (BM * LDA + BN * LDB);
    constexpr int LDS_C = BM * BN;
    __shared__ float2 lds[LDS_AB > LDS_C ? LDS_AB : LDS_C];
    auto As = [&](int buf) { return lds + buf * (BM * LDA); };
    auto Bs = [&](int buf) { return lds + 2 * BM * LDA + buf * (BN * LDB); };

    const int s = blockIdx.z;
    const int64_t b = blockIdx.y;
    const int64_t tiles_n = (g.N + BN - 1) / BN;
    const int64_t tiles_m = (g.M + BM - 1) / BM;
    const int64_t t = xcd_tile(blockIdx.x, tiles_m * tiles_n);
    const int64_t m0 = (t / tiles_n) * BM, n0 = (t % tiles_n) * BN;
    const float2 *Ap = A + s * g.sA + b * g.bA;
    const float2 *Bp = B + s * g.sB + b * g.bB;
    float2 *Cp = C + s * g.sC + b * g.bC;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave / WN, wn = wave % WN;

    float4 ra[A_PER], rb[B_PER];
    auto gload = [&](int64_t k0) {
#pragma unroll
        for (int i = 0; i < A_PER; i++) {
            int c = tid + i * NT;
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (c < A_CHUNKS) {
                int row = c / (BK / 2), col = (c % (BK / 2)) * 2;
                int64_t gm = m0 + row, gk = k0 + col;
                if (gm < g.M && gk < g.K) v = *(const float4 *)(Ap + gm * g.K + gk);
            }
            ra[i] = v;
        }
#pragma unroll
        for (int i = 0; i < B_PER; i++) {
            int c = tid + i * NT;
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (c < B_CHUNKS) {
                int row = c / (BK / 2), col = (c % (BK / 2)) * 2;
                int64_t gn = n0 + row, gk = k0 + col;
                if (gn < g.N && gk < g.K) v = *(const float4 *)(Bp + gn * g.K + gk);
            }
            rb[i] = v;
        }
    };
    auto sstore = [&](int buf) {
#pragma unroll
        for (int i = 0; i < A_PER; i++) {
            int c = tid + i * NT;
            if (c < A_CHUNKS) {
                int row = c / (BK / 2), col = (c % (BK / 2)) * 2;
                As(buf)[row * LDA + col] = make_float2(ra[i].x, ra[i].y);
                As(buf)[row * LDA + col + 1] = make_float2(ra[i].z, ra[i].w);
            }
        }
#pragma unroll
        for (int i = 0; i < B_PER; i++) {
            int c = tid + i * NT;
            if (c < B_CHUNKS) {
                int row = c / (BK / 2), col = (c % (BK / 2)) * 2;
                Bs(buf)[row * LDB + col] = make_float2(rb[i].x, rb[i].y);
                Bs(buf)[row * LDB + col + 1] = make_float2(rb[i].z, rb[i].w);
            }
        }
    };

    floatx16 acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; i++)
#pragma unroll
        for (int j = 0; j < FN; j++)
#pragma unroll
            for (int r = 0; r < 16; r++) acc[i][j][r] = 0.f;

    const int64_t nk = (g.K + BK - 1) / BK;
    gload(0);
    sstore(0);
    __syncthreads();
    const int c = lane >> 5;        // k' parity this lane feeds: 0 = re, 1 = im
    const int d = lane & 1;         // output column parity
    for (int64_t kt = 0; kt < nk; kt++) {
        const int buf = kt & 1;
        if (kt + 1 < nk) gload((kt + 1) * BK);
#pragma unroll 4
        for (int kk = 0; kk < BK; kk++) {
            float af[FM], bf[FN];
#pragma unroll
            for (int i = 0; i < FM; i++) {
                float2 v = As(buf)[(wm * WTM + i * 32 + (lane & 31)) * LDA + kk];
                af[i] = c ? v.y : v.x;
            }
#pragma unroll
            for (int j = 0; j < FN; j++) {
                float2 v = Bs(buf)[((wn * WTN + j * 32 + (lane & 31)) >> 1) * LDB + kk];
                // B'[2k+c][2n+d]: (c,d) = (0,0) br, (1,0) -bi, (0,1) bi, (1,1) br
                bf[j] = (c == d) ? v.x : (c ? -v.y : v.y);
            }
#pragma unroll
            for (int i = 0; i < FM; i++)
#pragma unroll
                for (int j = 0; j < FN; j++)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[i], bf[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
        if (kt + 1 < nk) {
            sstore(buf ^ 1);
            __syncthreads();
        }
    }
    float *Cs = (float *)lds;   // [BM][2*BN]
#pragma unroll
    for (int i = 0; i < FM; i++)
#pragma unroll
        for (int j = 0; j < FN; j++)
#pragma unroll
            for (int r = 0; r < 16; r++) {
                int row = wm * WTM + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                int col = wn * WTN + j * 32 + (lane & 31);
                Cs[row * (2 * BN) + col] = acc[i][j][r];
            }
    __syncthreads();
    constexpr int C_CHUNKS = BM * BN / 2;
    for (int cc = tid; cc < C_CHUNKS; cc += NT) {
        int row = cc / (BN / 2), col = (cc % (BN / 2)) * 2;
        int64_t gm = m0 + row, gn = n0 + col;
        if (gm < g.M && gn < g.N) *(float4 *)(Cp + gm * g.N + gn) = *(const float4 *)(Cs + row * 2 * BN + 2 * col);
    }
}

// ===================================================================== dispatch

const char *kernel_name(int k) {
    switch (k) {
        case K_NAIVE: return "naive";
        case K_SKINNY_N: return "skinny";
        case K_MFMA_S: return "mfma_64x16";
        case K_MFMA_M: return "mfma_128x32";
        case K_MFMA_L: return "mfma_128x64";
        case K_MFMA_W: return "mfma_256x16";
        default: return "?";
    }
}

struct TileCfg {
    int BM, BN;
};
static TileCfg tile_of(int kid, Dtype dt) {
    if (dt == Dtype::C64) {
        switch (kid) {
            case K_MFMA_S: return {64, 16};
            case K_MFMA_M: return {128, 16};
            case K_MFMA_L: return {128, 32};
            case K_MFMA_W: return {256, 16};
        }
    }
    switch (kid) {
        case K_MFMA_S: return {64, 16};
        case K_MFMA_M: return {128, 32};
        case K_MFMA_L: return {128, 64};
        case K_MFMA_W: return {256, 16};
    }
    return {0, 0};
}

bool gemm_supported(int kid, Dtype dt, Algo al, const GemmShape &g) {
    if (g.M <= 0 || g.N <= 0 || g.K <= 0 || g.nb <= 0) return false;
    if (kid == K_NAIVE) return g.nb <= 65535;
    if (kid == K_SKINNY_N) {
        int64_t nn = g.N < 16 ? g.N : 16;
        return g.nb * ((g.N + nn - 1) / nn) <= 65535;
    }
    if (g.nb > 65535) return false;
    if (kid < 0 || kid >= K_COUNT) return false;
    if (al == Algo::M3) return false;           // 3M runs on the VALU kernels
    TileCfg t = tile_of(kid, dt);
    // matrix-core tiles need whole 16-byte chunks along K and whole tiles along M, N
    const int64_t kmin = dt == Dtype::C64 ? 2 : 8;
    if (g.K < kmin) return false;
    if (g.M < t.BM || g.N < t.BN) return false;
    return true;
}

template <typename W, bool SCALE>
static void launch_valu(int kid, Algo al, const void *A, const void *B, void *C, const GemmShape &g, int S,
                        const ScaleRefs &sc, hipStream_t st) {
    if (kid == K_NAIVE) {
        int64_t total = g.M * g.N;
        int gx = (int)std::min<int64_t>((total + 255) / 256, 1 << 16);
        dim3 grid(gx, (unsigned)g.nb, S);
        if (al == Algo::M3)
            hipLaunchKernelGGL((gemm_naive_kernel<W, SCALE, true>), grid, dim3(256), 0, st, (const W *)A,
                               (const W *)B, (W *)C, g, sc);
        else
            hipLaunchKernelGGL((gemm_naive_kernel<W, SCALE, false>), grid, dim3(256), 0, st, (const W *)A,
                               (const W *)B, (W *)C, g, sc);
        return;
    }
    // skinny: choose NN = min(N, 16) rounded to a power of two
    int64_t nn = g.N < 16 ? g.N : 16;
    int64_t nch = (g.N + nn - 1) / nn;
    dim3 grid((unsigned)((g.M + 255) / 256), (unsigned)(g.nb * nch), S);
#define SKINNY(NNV)                                                                                        \
    do {                                                                                                   \
        if (al == Algo::M3)                                                                                \
            hipLaunchKernelGGL((gemm_skinny_kernel<W, NNV, SCALE, true>), grid, dim3(256), 0, st,          \
                               (const W *)A, (const W *)B, (W *)C, g, sc);                                 \
        else                                                                                               \
            hipLaunchKernelGGL((gemm_skinny_kernel<W, NNV, SCALE, false>), grid, dim3(256), 0, st,         \
                               (const W *)A, (const W *)B, (W *)C, g, sc);                                 \
    } while (0)
    switch (nn) {
        case 1: SKINNY(1); break;
        case 2: SKINNY(2); break;
        case 4: SKINNY(4); break;
        case 8: SKINNY(8); break;
        default: SKINNY(16); break;
    }
#undef SKINNY
}

template <bool BF>
static void launch_h4m(int kid, const void *A, const void *B, void *C, const GemmShape &g, int S,
                       const ScaleRefs &sc, hipStream_t st) {
    TileCfg t = tile_of(kid, BF ? Dtype::BF16 : Dtype::F16);
    int64_t tiles = ((g.M + t.BM - 1) / t.BM) * ((g.N + t.BN - 1) / t.BN);
    dim3 grid((unsigned)tiles, (unsigned)g.nb, S);
    auto a = (const uint32_t *)A;
    auto b = (const uint32_t *)B;
    auto c = (uint32_t *)C;
    switch (kid) {
        case K_MFMA_S:
            hipLaunchKernelGGL((gemm_mfma_h4m_kernel<BF, 64, 16, 32, 2, 1, true>), grid, dim3(128), 0, st, a, b, c, g, sc);
            break;
        case K_MFMA_M:
            hipLaunchKernelGGL((gemm_mfma_h4m_kernel<BF, 128, 32, 32, 2, 2, true>), grid, dim3(256), 0, st, a, b, c, g, sc);
            break;
        case K_MFMA_L:
            hipLaunchKernelGGL((gemm_mfma_h4m_kernel<BF, 128, 64, 32, 2, 2, true>), grid, dim3(256), 0, st, a, b, c, g, sc);
            break;
        case K_MFMA_W:
            hipLaunchKernelGGL((gemm_mfma_h4m_kernel<BF, 256, 16, 32, 4, 1, true>), grid, dim3(256), 0, st, a, b, c, g, sc);
            break;
    }
}

static void launch_c64(int kid, const void *A, const void *B, void *C, const GemmShape &g, int S, hipStream_t st) {
    TileCfg t = tile_of(kid, Dtype::C64);
    int64_t tiles = ((g.M + t.BM - 1) / t.BM) * ((g.N + t.BN - 1) / t.BN);
    dim3 grid((unsigned)tiles, (unsigned)g.nb, S);
    auto a = (const float2 *)A;
    auto b = (const float2 *)B;
    auto c = (float2 *)C;
    switch (kid) {
        case K_MFMA_S:
            hipLaunchKernelGGL((gemm_mfma_c64_kernel<64, 16, 16, 2, 1>), grid, dim3(128), 0, st, a, b, c, g);
            break;
        case K_MFMA_M:
            hipLaunchKernelGGL((gemm_mfma_c64_kernel<128, 16, 16, 4, 1>), grid, dim3(256), 0, st, a, b, c, g);
            break;
        case K_MFMA_L:
            hipLaunchKernelGGL((gemm_mfma_c64_kernel<128, 32, 16, 2, 2>), grid, dim3(256), 0, st, a, b, c, g);
            break;
        case K_MFMA_W:
            hipLaunchKernelGGL((gemm_mfma_c64_kernel<256, 16, 16, 4, 1>), grid, dim3(256), 0, st, a, b, c, g);
            break;
    }
}

void launch_gemm(int kid, Dtype dt, Algo al, const void *A, const void *B, void *C, const GemmShape &g, int S,
                 const ScaleRefs *sc, hipStream_t st) {
    if (S <= 0) return;
    if (!gemm_supported(kid, dt, al, g)) TNC_THROW(TNC_EINVAL, std::string("kernel ") + kernel_name(kid) + " cannot run this shape");
    ScaleRefs none{};
    const ScaleRefs &s = sc ? *sc : none;
    if (kid == K_NAIVE || kid == K_SKINNY_N) {
        if (dt == Dtype::C64)
            launch_valu<uint2, false>(kid, al, A, B, C, g, S, s, st);
        else if (dt == Dtype::F16)
            launch_valu<HalfWord, true>(kid, al, A, B, C, g, S, s, st);
        else
            launch_valu<Bf16Word, true>(kid, al, A, B, C, g, S, s, st);
    } else if (dt == Dtype::C64) {
        launch_c64(kid, A, B, C, g, S, st);
    } else if (dt == Dtype::F16) {
        launch_h4m<false>(kid, A, B, C, g, S, s, st);
    } else {
        launch_h4m<true>(kid, A, B, C, g, S, s, st);
    }
    HIP_CHECK(hipGetLastError());
}

}  // namespace tnc
