// Batched complex GEMM for one contraction step (paper Eq. contraction in
// its pure-GEMM form, Sec. 3.3):
//     C[s][b][m][n] = sum_k A[s][b][m][k] * B[s][b][n][k]
// s is the slice in flight, b the inner batch.  Each operand is stored in
// either orientation (A as [m][k] or [k][m], B as [n][k] or [k][n]) and C is
// written as [m][n] or [n][m], so the planner can skip most permutes.
//
// Forms:
//   4M   -- one real GEMM  C'[m][2n+d] = sum_{k'} A'[m][k'] B'[k'][2n+d], with
//           A' the interleaved (re, im) view of A (k' = 2k + c) and B' the
//           small operand padded on the fly to [B(re,-im), B(im,re)] (paper
//           Eq. eq_modified2); 8 real flops per complex multiply-add.
//   3M   -- T1 = Ar Br, T2 = Ai Bi, T3 = (Ar+Ai)(Br+Bi) with the sums rounded
//           once to the storage type; Cr = T1 - T2, Ci = T3 - T1 - T2
//           (6 executed real flops per complex multiply-add).
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
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

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
        if (!(mx <= sc.flag_above) && sc.flag) atomicOr(sc.flag, 1u);   // too large, inf, or NaN
    }
}

// exact 2^-shift as a float (shift is clamped to the normal range)
__device__ __forceinline__ float pow2_neg(int shift) {
    shift = shift > 126 ? 126 : (shift < -126 ? -126 : shift);
    return __uint_as_float((uint32_t)(127 - shift) << 23);
}

__device__ __forceinline__ int64_t a_index(const GemmShape &g, int64_t m, int64_t k) {
    return seg_offset(g.am, m) + seg_offset(g.ak, k);
}
__device__ __forceinline__ int64_t b_index(const GemmShape &g, int64_t n, int64_t k) {
    return seg_offset(g.bn, n) + seg_offset(g.bk, k);
}
__device__ __forceinline__ int64_t c_index(const GemmShape &g, int64_t m, int64_t n) {
    return seg_offset(g.cm, m) + seg_offset(g.cn, n);
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
    const W *Ap = A + s * g.sA + a_block(g, b) * g.bA;
    const W *Bp = B + s * g.sB + b_block(g, b) * g.bB;
    W *Cp = C + s * g.sC + b * g.bC;
    float mx = 0.f;
    const int64_t total = g.M * g.N;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        // consecutive threads walk the contiguous dimension of C
        int64_t m, n;
        if (g.c_nc) {
            m = i / g.N;
            n = i - m * g.N;
        } else {
            n = i / g.M;
            m = i - n * g.M;
        }
        float re = 0.f, im = 0.f;
        if (!M3) {
            for (int64_t k = 0; k < g.K; k++) {
                float2 a = unpack(Ap[a_index(g, m, k)]), bb = unpack(Bp[b_index(g, n, k)]);
                re = fmaf(a.x, bb.x, re);
                re = fmaf(-a.y, bb.y, re);
                im = fmaf(a.x, bb.y, im);
                im = fmaf(a.y, bb.x, im);
            }
        } else {
            float t1 = 0.f, t2 = 0.f, t3 = 0.f;
            for (int64_t k = 0; k < g.K; k++) {
                float2 a = unpack(Ap[a_index(g, m, k)]), bb = unpack(Bp[b_index(g, n, k)]);
                t1 = fmaf(a.x, bb.x, t1);
                t2 = fmaf(a.y, bb.y, t2);
                t3 = fmaf(round_to_storage<W>(a.x + a.y), round_to_storage<W>(bb.x + bb.y), t3);
            }
            re = t1 - t2;
            im = t3 - t1 - t2;
        }
        mx = fmaxf(mx, store_entry<W, SCALE>(Cp + c_index(g, m, n), re, im, scale));
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
    const W *Ap = A + s * g.sA + a_block(g, b) * g.bA;
    const W *Bp = B + s * g.sB + b_block(g, b) * g.bB;
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
            int j, kk;
            if (g.b_kc) {
                j = e / KC;
                kk = e - j * KC;
            } else {
                kk = e / NN;
                j = e - kk * NN;
            }
            float2 v = make_float2(0.f, 0.f);
            if (j < nn && kk < kc) v = unpack(Bp[b_index(g, n0 + j, k0 + kk)]);
            Bs[j][kk] = v;
            if constexpr (M3) Bsum[j][kk] = round_to_storage<W>(v.x + v.y);
        }
        __syncthreads();
        if (live) {
            for (int kk = 0; kk < kc; kk++) {
                float2 a = unpack(Ap[a_index(g, m, k0 + kk)]);
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
                mx = fmaxf(mx, store_entry<W, SCALE>(Cp + c_index(g, m, n0 + j), re, im, scale));
            }
        }
    }
    finish_max<SCALE>(sc, s, mx);
}

// ===================================================================== thin: N <= 16, K <= 64 (VALU)
// HBM-bound steps (a wide operand times a few columns).  B's NN columns are
// staged in LDS once per block; the grid is capped and threads stride over
// row units.  A unit is one row whose k entries are read in 16-byte loads
// (MODE 0, A chunked along k) or V consecutive rows read with one 16-byte
// load per k (MODE 1, A chunked along m).  Results leave in 16-byte stores
// when the result is chunked along the index the unit spans.

template <typename W> struct alignas(16) Pack16 {
    static constexpr int N = 16 / sizeof(W);
    W w[N];
};

template <typename W, bool SCALE>
__device__ __forceinline__ W make_entry(float re, float im, float scale, float &mx) {
    if (SCALE) {
        re *= scale;
        im *= scale;
    }
    W w = Pack<W>::make(re, im);
    if (SCALE) {
        float2 f = unpack(w);
        mx = fmaxf(mx, absmax_nan(f.x, f.y));
    }
    return w;
}

template <typename W, int NN, int MODE, bool SCALE, bool M3>
__global__ void __launch_bounds__(256) gemm_thin_kernel(const W *__restrict__ A, const W *__restrict__ B,
                                                        W *__restrict__ C, GemmShape g, ScaleRefs sc) {
    constexpr int V = 16 / sizeof(W);
    constexpr int KMAX = 64;
    constexpr int R = MODE == 1 ? V : 1;   // rows per unit
    __shared__ float2 Bs[NN][KMAX];
    __shared__ float Bsum[M3 ? NN : 1][KMAX];
    const int s = blockIdx.z;
    const int64_t nchunks = g.N / NN;
    const int64_t b = blockIdx.y / nchunks;
    const int64_t n0 = (blockIdx.y - b * nchunks) * NN;
    int shift = SCALE ? step_shift(sc, s) : 0;
    if (SCALE && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) record_exponent(sc, s, shift);
    const float scale = pow2_neg(shift);
    const W *Ap = A + s * g.sA + a_block(g, b) * g.bA;
    const W *Bp = B + s * g.sB + b_block(g, b) * g.bB;
    W *Cp = C + s * g.sC + b * g.bC;
    const int K = (int)g.K;
    for (int e = threadIdx.x; e < NN * KMAX; e += blockDim.x) {
        const int j = e / KMAX, kk = e - j * KMAX;
        float2 v = make_float2(0.f, 0.f);
        if (kk < K) v = unpack(Bp[b_index(g, n0 + j, kk)]);
        Bs[j][kk] = v;
        if constexpr (M3) Bsum[j][kk] = round_to_storage<W>(v.x + v.y);
    }
    __syncthreads();
    // vector stores: along n (V consecutive columns of one row: MODE 0, and
    // MODE 1 row by row) or along m (the V rows of a MODE 1 unit)
    constexpr int LV = V == 4 ? 2 : 1;
    const bool n_vec = NN % V == 0 && g.cn.ls == 0 && g.cn.l >= LV && g.N >= V;
    const bool m_vec = MODE == 1 && g.cm.ls == 0 && g.cm.l >= LV;
    const bool vstore = MODE == 0 ? (g.c_nc && n_vec) : (!g.c_nc ? m_vec : n_vec);
    const int64_t units = g.M / R;
    float mx = 0.f;
    for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < units; u += (int64_t)gridDim.x * blockDim.x) {
        const int64_t m = u * R;
        float2 acc[R][NN];
        float t3[M3 ? R : 1][M3 ? NN : 1];
#pragma unroll
        for (int r = 0; r < R; r++)
#pragma unroll
            for (int j = 0; j < NN; j++) {
                acc[r][j] = make_float2(0.f, 0.f);
                if constexpr (M3) t3[r][j] = 0.f;
            }
        const W *ap = Ap + seg_offset(g.am, m);
        auto madd = [&](int r, float2 a, int k) {
            if constexpr (!M3) {
#pragma unroll
                for (int j = 0; j < NN; j++) {
                    float2 bb = Bs[j][k];
                    acc[r][j].x = fmaf(a.x, bb.x, acc[r][j].x);
                    acc[r][j].x = fmaf(-a.y, bb.y, acc[r][j].x);
                    acc[r][j].y = fmaf(a.x, bb.y, acc[r][j].y);
                    acc[r][j].y = fmaf(a.y, bb.x, acc[r][j].y);
                }
            } else {
                float as = round_to_storage<W>(a.x + a.y);
#pragma unroll
                for (int j = 0; j < NN; j++) {
                    float2 bb = Bs[j][k];
                    acc[r][j].x = fmaf(a.x, bb.x, acc[r][j].x);   // T1
                    acc[r][j].y = fmaf(a.y, bb.y, acc[r][j].y);   // T2
                    t3[r][j] = fmaf(as, Bsum[j][k], t3[r][j]);    // T3
                }
            }
        };
        if constexpr (MODE == 0) {
            for (int k0 = 0; k0 < K; k0 += V) {
                Pack16<W> v = *(const Pack16<W> *)(ap + seg_offset(g.ak, k0));
#pragma unroll
                for (int q = 0; q < V; q++) madd(0, unpack(v.w[q]), k0 + q);
            }
        } else {
            for (int k = 0; k < K; k++) {
                Pack16<W> v = *(const Pack16<W> *)(ap + seg_offset(g.ak, k));
#pragma unroll
                for (int q = 0; q < V; q++) madd(q, unpack(v.w[q]), k);
            }
        }
        auto value = [&](int r, int j, float &re, float &im) {
            if constexpr (!M3) {
                re = acc[r][j].x;
                im = acc[r][j].y;
            } else {
                re = acc[r][j].x - acc[r][j].y;
                im = t3[r][j] - acc[r][j].x - acc[r][j].y;
            }
        };
        if (vstore) {
            if constexpr (MODE == 0) {
#pragma unroll
                for (int j0 = 0; j0 < NN; j0 += V) {
                    Pack16<W> o;
#pragma unroll
                    for (int q = 0; q < V; q++) {
                        float re, im;
                        value(0, (j0 + q) % NN, re, im);
                        o.w[q] = make_entry<W, SCALE>(re, im, scale, mx);
                    }
                    *(Pack16<W> *)(Cp + c_index(g, m, n0 + j0)) = o;
                }
            } else if (!g.c_nc) {
#pragma unroll
                for (int j = 0; j < NN; j++) {
                    Pack16<W> o;
#pragma unroll
                    for (int q = 0; q < V; q++) {
                        float re, im;
                        value(q % R, j, re, im);
                        o.w[q] = make_entry<W, SCALE>(re, im, scale, mx);
                    }
                    *(Pack16<W> *)(Cp + c_index(g, m, n0 + j)) = o;
                }
            } else {
#pragma unroll
                for (int r = 0; r < R; r++)
#pragma unroll
                    for (int j0 = 0; j0 < NN; j0 += V) {
                        Pack16<W> o;
#pragma unroll
                        for (int q = 0; q < V; q++) {
                            float re, im;
                            value(r, (j0 + q) % NN, re, im);
                            o.w[q] = make_entry<W, SCALE>(re, im, scale, mx);
                        }
                        *(Pack16<W> *)(Cp + c_index(g, m + r, n0 + j0)) = o;
                    }
            }
        } else {
#pragma unroll
            for (int r = 0; r < R; r++)
#pragma unroll
                for (int j = 0; j < NN; j++) {
                    float re, im;
                    value(r, j, re, im);
                    Cp[c_index(g, m + r, n0 + j)] = make_entry<W, SCALE>(re, im, scale, mx);
                }
        }
    }
    finish_max<SCALE>(sc, s, mx);
}

// Which thin variant can run a shape (-1: none).
static int thin_mode(Dtype dt, const GemmShape &g) {
    const int lv = dt == Dtype::C64 ? 1 : 2;   // log2 of the entries in 16 bytes
    const int64_t v = (int64_t)1 << lv;
    if (g.K > 64 || g.N > 16 || g.nb * (g.N / std::min<int64_t>(g.N, 16)) > 65535) return -1;
    auto ok = [&](const Seg &sg, int64_t ext) { return sg.ls == 0 && seg_low_run(sg, ext) >= lv && ext % v == 0; };
    // the result is written with 16-byte stores where its layout allows, else entry by entry
    if (g.a_kc && ok(g.ak, g.K)) return 0;
    if (!g.a_kc && ok(g.am, g.M)) return 1;
    return -1;
}

// ===================================================================== matrix cores, 16-bit
//
// Block tile BM rows x BN complex columns, k-tile BK complex; WM x WN waves.
// v_mfma_f32_32x32x16_{f16,bf16}: lane l holds A[l%32][8(l/32)+0..7] and
// B[8(l/32)+0..7][l%32]; result register r of lane l is row
// 8(r/4) + 4(l/32) + r%4, column l%32.
//   4M: the real GEMM of the header (k' = 2k + c, columns 2n + d); a wave
//       owns (BM/WM) rows x (2BN/WN) real columns.
//   3M: three real GEMMs over k; a wave owns (BM/WM) rows x (BN/WN) complex
//       columns with three accumulators per 32x32 block.

template <bool BF> __device__ __forceinline__ floatx16 mfma16(u32x4 a, u32x4 b, floatx16 c) {
    if constexpr (BF)
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8_t, a),
                                                       __builtin_bit_cast(bf16x8_t, b), c, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(half8_t, a),
                                                      __builtin_bit_cast(half8_t, b), c, 0, 0, 0);
}


// 4M padding of B in registers, without branches: lane parity d picks
// (br, -bi) (d = 0: keep the halves, flip the sign of the high one) or
// (bi, br) (d = 1: swap the halves) through a byte permute and an XOR
struct Pad4M {
    uint32_t sel, mask;
    __device__ explicit Pad4M(int d) : sel(d ? 0x01000302u : 0x03020100u), mask(d ? 0u : 0x80000000u) {}
    __device__ __forceinline__ u32x4 operator()(u32x4 v) const {
#pragma unroll
        for (int q = 0; q < 4; q++) v[q] = __builtin_amdgcn_perm(v[q], v[q], sel) ^ mask;
        return v;
    }
};

// rounded re + im of a 16-bit complex word, as 16-bit bits
template <bool BF> __device__ __forceinline__ uint32_t sum_bits(uint32_t w) {
    if constexpr (BF) {
        float re = __uint_as_float(w << 16), im = __uint_as_float(w & 0xffff0000u);
        return f2bf_bits(re + im);
    } else {
        float re = __half2float(__ushort_as_half((unsigned short)(w & 0xffffu)));
        float im = __half2float(__ushort_as_half((unsigned short)(w >> 16)));
        return f2h_bits(re + im);
    }
}

// XCD-aware order: blocks are dispatched to the 8 XCDs round-robin, so block
// w is given tile (w % 8) * (total / 8) + w / 8 and each XCD works through a
// contiguous range of the tile order.
__device__ __forceinline__ int64_t xcd_tile(int64_t w, int64_t total) {
    if (total % 8) return w;
    return (w % 8) * (total / 8) + w / 8;
}

// Tile order in groups of GM row blocks: tile t covers row block
// g*GM + t % gm and column block (t / gm) % tiles_n of group g, so the ~32
// tiles an XCD runs at once form a GM x 8 patch whose operand strips are
// shared through its L2 (a 1 x 32 row would fetch 32 B strips).
template <int GM>
__device__ __forceinline__ void tile_coords(int64_t t, int64_t tiles_m, int64_t tiles_n, int64_t &mt, int64_t &nt) {
    const int64_t per_group = (int64_t)GM * tiles_n;
    const int64_t g = t / per_group, r = t - g * per_group;
    const int64_t gm = tiles_m - g * GM < GM ? tiles_m - g * GM : GM;
    mt = g * GM + r % gm;
    nt = r / gm;
}

template <bool BF, bool M3, int BM, int BN, int BK, int WM, int WN>
struct HTile {
    static constexpr int NT = 64 * WM * WN;
    // 4M: LDS holds complex words; 3M: three planes of 16-bit values
    static constexpr int PAD = M3 ? 8 : 4;                    // in elements of the LDS row type
    static constexpr int LDA = BK + PAD, LDB = BK + PAD;
    static constexpr int A_ELEMS = M3 ? 3 * BM * LDA : BM * LDA;   // halves (3M) or words (4M)
    static constexpr int B_ELEMS = M3 ? 3 * BN * LDB : BN * LDB;
    static constexpr int ESZ = M3 ? 2 : 4;
    static constexpr int AB_BYTES = 2 * (A_ELEMS + B_ELEMS) * ESZ;
    static constexpr int C_BYTES = BM * BN * 4;
    static constexpr int LDS_BYTES = AB_BYTES > C_BYTES ? AB_BYTES : C_BYTES;
    static constexpr int WTM = BM / WM;
    static constexpr int WTN = M3 ? BN / WN : 2 * BN / WN;    // complex (3M) or real (4M) columns
    static constexpr int FM = WTM / 32, FN = WTN / 32;
    static constexpr int KSTEP = M3 ? 16 : 8;                  // complex k per MFMA
    static constexpr int A_CHUNKS = BM * BK / 4, B_CHUNKS = BN * BK / 4;
    static constexpr int A_PER = (A_CHUNKS + NT - 1) / NT, B_PER = (B_CHUNKS + NT - 1) / NT;
    static_assert(FM >= 1 && FN >= 1, "wave tile too small");
    static_assert(BK % KSTEP == 0, "k tile");
    static_assert(LDS_BYTES <= 160 * 1024, "LDS");
};

template <bool BF, bool M3, int BM, int BN, int BK, int WM, int WN>
__global__ void __launch_bounds__(64 * WM * WN)
    gemm_mfma_h_kernel(const uint32_t *__restrict__ A, const uint32_t *__restrict__ B, uint32_t *__restrict__ C,
                       GemmShape g, ScaleRefs sc) {
    using Tl = HTile<BF, M3, BM, BN, BK, WM, WN>;
    using W = typename std::conditional<BF, Bf16Word, HalfWord>::type;
    constexpr int NT = Tl::NT, LDA = Tl::LDA, LDB = Tl::LDB, FM = Tl::FM, FN = Tl::FN;
    constexpr int WTM = Tl::WTM, WTN = Tl::WTN, ESZ = Tl::ESZ;
    extern __shared__ __align__(16) uint8_t smem[];

    const int s = blockIdx.z;
    const int64_t P = g.split;
    const int64_t b = blockIdx.y / P, part = blockIdx.y - b * P;
    const int64_t tiles_n = (g.N + BN - 1) / BN;
    const int64_t tiles_m = (g.M + BM - 1) / BM;
    const int64_t t = xcd_tile(blockIdx.x, tiles_m * tiles_n);
    int64_t mt, nt;
    tile_coords<4>(t, tiles_m, tiles_n, mt, nt);
    const int64_t m0 = mt * BM, n0 = nt * BN;
    float scale = 1.f;
    if (P == 1) {
        int shift = step_shift(sc, s);
        if (blockIdx.x == 0 && b == 0 && threadIdx.x == 0) record_exponent(sc, s, shift);
        scale = pow2_neg(shift);
    }

    const uint32_t *Ap = A + s * g.sA + a_block(g, b) * g.bA;
    const uint32_t *Bp = B + s * g.sB + b_block(g, b) * g.bB;
    uint32_t *Cp = C + s * g.sC + b * g.bC;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave / WN, wn = wave % WN;

    // ---- global loads: 16-byte chunks of 4 complex words
    u32x4 ra[Tl::A_PER], rb[Tl::B_PER];
    auto gload = [&](int64_t k0) {
#pragma unroll
        for (int i = 0; i < Tl::A_PER; i++) {
            int c = tid + i * NT;
            u32x4 v = {0u, 0u, 0u, 0u};
            if (c < Tl::A_CHUNKS) {
                if (g.a_kc) {
                    int row = c / (BK / 4), col = (c % (BK / 4)) * 4;
                    int64_t gm = m0 + row, gk = k0 + col;
                    if (gm < g.M && gk < g.K) v = *(const u32x4 *)(Ap + a_index(g, gm, gk));
                } else {
                    int kr = c / (BM / 4), mc = (c % (BM / 4)) * 4;
                    int64_t gk = k0 + kr, gm = m0 + mc;
                    if (gk < g.K && gm < g.M) v = *(const u32x4 *)(Ap + a_index(g, gm, gk));
                }
            }
            ra[i] = v;
        }
#pragma unroll
        for (int i = 0; i < Tl::B_PER; i++) {
            int c = tid + i * NT;
            u32x4 v = {0u, 0u, 0u, 0u};
            if (c < Tl::B_CHUNKS) {
                if (g.b_kc) {
                    int row = c / (BK / 4), col = (c % (BK / 4)) * 4;
                    int64_t gn = n0 + row, gk = k0 + col;
                    if (gn < g.N && gk < g.K) v = *(const u32x4 *)(Bp + b_index(g, gn, gk));
                } else {
                    int kr = c / (BN / 4), nc = (c % (BN / 4)) * 4;
                    int64_t gk = k0 + kr, gn = n0 + nc;
                    if (gk < g.K && gn < g.N) v = *(const u32x4 *)(Bp + b_index(g, gn, gk));
                }
            }
            rb[i] = v;
        }
    };
    // ---- LDS stores (row = m or n, col = k)
    auto a_base = [&](int buf) { return smem + buf * (Tl::A_ELEMS * ESZ); };
    auto b_base = [&](int buf) { return smem + 2 * Tl::A_ELEMS * ESZ + buf * (Tl::B_ELEMS * ESZ); };
    auto put = [&](uint8_t *base, int rows, int ld, int row, int col, uint32_t w) {
        if constexpr (M3) {
            uint16_t *p = (uint16_t *)base;
            p[row * ld + col] = (uint16_t)(w & 0xffffu);                    // re plane
            p[rows * ld + row * ld + col] = (uint16_t)(w >> 16);            // im plane
            p[2 * rows * ld + row * ld + col] = (uint16_t)sum_bits<BF>(w);  // sum plane
        } else {
            ((uint32_t *)base)[row * ld + col] = w;
        }
    };
    auto put4 = [&](uint8_t *base, int rows, int ld, int row, int col, u32x4 v) {
        if constexpr (M3) {
            uint16_t *p = (uint16_t *)base;
            u32x2 re = {(v[0] & 0xffffu) | (v[1] << 16), (v[2] & 0xffffu) | (v[3] << 16)};
            u32x2 im = {(v[0] >> 16) | (v[1] & 0xffff0000u), (v[2] >> 16) | (v[3] & 0xffff0000u)};
            u32x2 sm = {sum_bits<BF>(v[0]) | (sum_bits<BF>(v[1]) << 16), sum_bits<BF>(v[2]) | (sum_bits<BF>(v[3]) << 16)};
            *(u32x2 *)(p + row * ld + col) = re;
            *(u32x2 *)(p + rows * ld + row * ld + col) = im;
            *(u32x2 *)(p + 2 * rows * ld + row * ld + col) = sm;
        } else {
            *(u32x4 *)((uint32_t *)base + row * ld + col) = v;
        }
    };
    auto sstore = [&](int buf) {
        uint8_t *ab = a_base(buf), *bb = b_base(buf);
#pragma unroll
        for (int i = 0; i < Tl::A_PER; i++) {
            int c = tid + i * NT;
            if (c < Tl::A_CHUNKS) {
                if (g.a_kc) {
                    put4(ab, BM, LDA, c / (BK / 4), (c % (BK / 4)) * 4, ra[i]);
                } else {
                    int kr = c / (BM / 4), mc = (c % (BM / 4)) * 4;
#pragma unroll
                    for (int q = 0; q < 4; q++) put(ab, BM, LDA, mc + q, kr, ra[i][q]);
                }
            }
        }
#pragma unroll
        for (int i = 0; i < Tl::B_PER; i++) {
            int c = tid + i * NT;
            if (c < Tl::B_CHUNKS) {
                if (g.b_kc) {
                    put4(bb, BN, LDB, c / (BK / 4), (c % (BK / 4)) * 4, rb[i]);
                } else {
                    int kr = c / (BN / 4), nc = (c % (BN / 4)) * 4;
#pragma unroll
                    for (int q = 0; q < 4; q++) put(bb, BN, LDB, nc + q, kr, rb[i][q]);
                }
            }
        }
    };

    constexpr int NACC = M3 ? 3 : 1;
    floatx16 acc[NACC][FM][FN];
#pragma unroll
    for (int a = 0; a < NACC; a++)
#pragma unroll
        for (int i = 0; i < FM; i++)
#pragma unroll
            for (int j = 0; j < FN; j++)
#pragma unroll
                for (int r = 0; r < 16; r++) acc[a][i][j][r] = 0.f;

    // k tiles of this split part
    const int64_t nk_all = (g.K + BK - 1) / BK;
    const int64_t kt0 = nk_all * part / P, kt1 = nk_all * (part + 1) / P;
    const int64_t nk = kt1 - kt0;
    gload(kt0 * BK);
    sstore(0);
    __syncthreads();
    for (int64_t kt = 0; kt < nk; kt++) {
        const int buf = kt & 1;
        if (kt + 1 < nk) gload((kt0 + kt + 1) * BK);
        const uint8_t *ab = a_base(buf), *bb = b_base(buf);
#pragma unroll
        for (int kk = 0; kk < BK / Tl::KSTEP; kk++) {
            if constexpr (!M3) {
                const uint32_t *As = (const uint32_t *)ab, *Bs = (const uint32_t *)bb;
                const int kq = kk * 8 + (lane >> 5) * 4;
                const Pad4M pad(lane & 1);
                u32x4 af[FM], bf[FN];
#pragma unroll
                for (int i = 0; i < FM; i++) af[i] = *(const u32x4 *)(As + (wm * WTM + i * 32 + (lane & 31)) * LDA + kq);
#pragma unroll
                for (int j = 0; j < FN; j++) {
                    bf[j] = pad(*(const u32x4 *)(Bs + ((wn * WTN + j * 32 + (lane & 31)) >> 1) * LDB + kq));
                }
#pragma unroll
                for (int i = 0; i < FM; i++)
#pragma unroll
                    for (int j = 0; j < FN; j++) acc[0][i][j] = mfma16<BF>(af[i], bf[j], acc[0][i][j]);
            } else {
                const uint16_t *As = (const uint16_t *)ab, *Bs = (const uint16_t *)bb;
                const int kq = kk * 16 + (lane >> 5) * 8;
#pragma unroll
                for (int p = 0; p < 3; p++) {
                    u32x4 af[FM], bf[FN];
#pragma unroll
                    for (int i = 0; i < FM; i++)
                        af[i] = *(const u32x4 *)(As + p * BM * LDA + (wm * WTM + i * 32 + (lane & 31)) * LDA + kq);
#pragma unroll
                    for (int j = 0; j < FN; j++)
                        bf[j] = *(const u32x4 *)(Bs + p * BN * LDB + (wn * WTN + j * 32 + (lane & 31)) * LDB + kq);
#pragma unroll
                    for (int i = 0; i < FM; i++)
#pragma unroll
                        for (int j = 0; j < FN; j++) acc[p][i][j] = mfma16<BF>(af[i], bf[j], acc[p][i][j]);
                }
            }
        }
        __syncthreads();
        if (kt + 1 < nk) {
            sstore(buf ^ 1);
            __syncthreads();
        }
    }

    if (P > 1) {
        // split part: FP32 partial sums straight from the accumulators
        float *pp = (float *)(g.part + ((s * g.nb + b) * P + part) * g.M * g.N);
#pragma unroll
        for (int i = 0; i < FM; i++)
#pragma unroll
            for (int j = 0; j < FN; j++)
#pragma unroll
                for (int r = 0; r < 16; r++) {
                    int row = wm * WTM + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                    int col = wn * WTN + j * 32 + (lane & 31);
                    if constexpr (!M3) {
                        // real column 2n + part of the interleaved complex row
                        pp[(m0 + row) * 2 * g.N + 2 * n0 + col] = acc[0][i][j][r];
                    } else {
                        float t1 = acc[0][i][j][r], t2 = acc[1][i][j][r], t3 = acc[2][i][j][r];
                        ((float2 *)pp)[(m0 + row) * g.N + n0 + col] = make_float2(t1 - t2, t3 - t1 - t2);
                    }
                }
        return;
    }

    // ---- epilogue: scale, round, stage the tile as complex words [BM][BN], write out
    uint32_t *Cw = (uint32_t *)smem;
    if constexpr (!M3) {
        uint16_t *Ch = (uint16_t *)smem;
#pragma unroll
        for (int i = 0; i < FM; i++)
#pragma unroll
            for (int j = 0; j < FN; j++)
#pragma unroll
                for (int r = 0; r < 16; r++) {
                    int row = wm * WTM + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                    int col = wn * WTN + j * 32 + (lane & 31);   // real column 2n + part
                    float v = acc[0][i][j][r] * scale;
                    Ch[row * (2 * BN) + col] = (uint16_t)(BF ? f2bf_bits(v) : f2h_bits(v));
                }
    } else {
#pragma unroll
        for (int i = 0; i < FM; i++)
#pragma unroll
            for (int j = 0; j < FN; j++)
#pragma unroll
                for (int r = 0; r < 16; r++) {
                    int row = wm * WTM + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                    int col = wn * WTN + j * 32 + (lane & 31);   // complex column
                    float t1 = acc[0][i][j][r], t2 = acc[1][i][j][r], t3 = acc[2][i][j][r];
                    float re = (t1 - t2) * scale, im = (t3 - t1 - t2) * scale;
                    Cw[row * BN + col] = Pack<W>::make(re, im).w;
                }
    }
    __syncthreads();
    float mx = 0.f;
    constexpr int C_CHUNKS = BM * BN / 4;
    for (int c = tid; c < C_CHUNKS; c += NT) {
        u32x4 v;
        int64_t off;
        bool ok;
        if (g.c_nc) {
            int row = c / (BN / 4), col = (c % (BN / 4)) * 4;
            v = *(const u32x4 *)(Cw + row * BN + col);
            ok = (m0 + row) < g.M && (n0 + col) < g.N;
            off = c_index(g, m0 + row, n0 + col);
        } else {
            int col = c / (BM / 4), row = (c % (BM / 4)) * 4;
#pragma unroll
            for (int q = 0; q < 4; q++) v[q] = Cw[(row + q) * BN + col];
            ok = (m0 + row) < g.M && (n0 + col) < g.N;
            off = c_index(g, m0 + row, n0 + col);
        }
        if (ok) {
            *(u32x4 *)(Cp + off) = v;
#pragma unroll
            for (int q = 0; q < 4; q++) {
                float2 f = unpack(W{v[q]});
                mx = fmaxf(mx, absmax_nan(f.x, f.y));
            }
        }
    }
    finish_max<true>(sc, s, mx);
}

// ===================================================================== matrix cores, 16-bit 4M, LDS DMA
//
// The compute-bound steps: both operands chunked along k, whole tiles.  The
// operands go from global memory straight into a ring of STAGES LDS buffers
// (global_load_lds_dwordx4 writes lane j's 16 bytes at base + 16 j), so no
// registers stage them and up to STAGES-1 k-tiles are in flight while the
// matrix cores work on the oldest.  An LDS row is one operand row's 32
// complex k (128 bytes, 8 chunks); chunk q of row r sits in slot q ^ (r & 7),
// so the DMA (whole rows) and the fragment reads (8 rows, one chunk each) are
// both free of bank conflicts.
//
// 4M here keeps the real and the imaginary parts of C in separate
// accumulators: a B fragment is 32 complex columns (lane l: column l % 32,
// complex k 4(l/32)..+3), read once, and gives the real-part operand
// (br, -bi) by one XOR and the imaginary-part operand (bi, br) by one byte
// permute per register:
//     Re C = sum_k' A'[m][k'] (br, -bi)[k'],   Im C = sum_k' A'[m][k'] (bi, br)[k']
// with A' the interleaved (re, im) view of A (k' = 2k + c).

// s_waitcnt vmcnt(VM) lgkmcnt(0), expcnt untouched (gfx9 field layout), then
// s_barrier; a compiler barrier for memory on both sides
template <int VM> __device__ __forceinline__ void ring_wait() {
    static_assert(VM >= 0 && VM < 64, "vmcnt");
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt((VM & 15) | ((VM >> 4) << 14) | (7 << 4));
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

template <int BM, int BN, int WM, int WN, int STAGES>
struct DTile {
    static constexpr int NT = 64 * WM * WN;
    static constexpr int BK = 32;                               // complex k per stage
    static constexpr int A_BYTES = BM * 128, B_BYTES = BN * 128;
    static constexpr int STAGE_BYTES = A_BYTES + B_BYTES;
    static constexpr int RING_BYTES = STAGES * STAGE_BYTES;
    static constexpr int LDS_BYTES = RING_BYTES;                  // the result leaves from registers
    static constexpr int WTM = BM / WM, WTC = BN / WN;          // rows, complex columns per wave
    static constexpr int FM = WTM / 32, FC = WTC / 32;
    static constexpr int A_PER = BM / 8 / (NT / 64);             // 1 KB DMA blocks per wave and stage
    static constexpr int B_PER = BN / 8 / (NT / 64);
    static constexpr int LPT = A_PER + B_PER;                    // DMA loads per thread and stage
    // two-stage variants fit two blocks per CU in LDS; their registers are
    // sized for that (see the launch bounds of the kernel)
    static_assert(STAGES != 2 || LDS_BYTES <= 80 * 1024, "two blocks per CU");
    static_assert(FM >= 1 && FC >= 1, "wave tile too small");
    static_assert(A_PER >= 1 && B_PER >= 1 && A_PER * (NT / 64) * 8 == BM && B_PER * (NT / 64) * 8 == BN, "DMA split");
    static_assert(STAGES >= 2 && LPT * (STAGES - 2) < 64, "stages");
    static_assert(LDS_BYTES <= 160 * 1024, "LDS");
};

template <int VM_AHEAD, int LPT> __device__ __forceinline__ void ring_wait_for(int64_t ahead) {
    // stage kt is complete once at most `ahead` later stages are outstanding
    if constexpr (VM_AHEAD == 0) {
        ring_wait<0>();
    } else {
        if (ahead >= VM_AHEAD) ring_wait<VM_AHEAD * LPT>();
        else ring_wait_for<VM_AHEAD - 1, LPT>(ahead);
    }
}

// blocks per CU the register budget is sized for: two-stage tiles fit two
// blocks in LDS, except the 3M 128 x 128 tile, whose 64 x 64 wave tiles need
// three accumulator sets (192 registers) and so run one wave per SIMD
template <bool M3, int BM, int BN, int STAGES> constexpr int dma_min_blocks() {
    return (STAGES == 2 && !(M3 && BM == 128 && BN == 128)) ? 2 : 1;
}

// 3M from the same ring: a k-step covers 16 complex k; lane l's two chunks
// hold complex k 8(l/32)..+7 of its row as 8 words (re low, im high).  One
// byte permute per pair of words gives the real plane, one the imaginary
// plane, and a packed FP16 add their rounded sum:
//     T1 = Ar Br,  T2 = Ai Bi,  T3 = (Ar + Ai)(Br + Bi);  Re C = T1 - T2,  Im C = T3 - T1 - T2.
__device__ __forceinline__ void planes3m(const u32x4 &w0, const u32x4 &w1, u32x4 &re, u32x4 &im, u32x4 &sm) {
    typedef _Float16 h2 __attribute__((ext_vector_type(2)));
    re[0] = __builtin_amdgcn_perm(w0[1], w0[0], 0x05040100u);
    re[1] = __builtin_amdgcn_perm(w0[3], w0[2], 0x05040100u);
    re[2] = __builtin_amdgcn_perm(w1[1], w1[0], 0x05040100u);
    re[3] = __builtin_amdgcn_perm(w1[3], w1[2], 0x05040100u);
    im[0] = __builtin_amdgcn_perm(w0[1], w0[0], 0x07060302u);
    im[1] = __builtin_amdgcn_perm(w0[3], w0[2], 0x07060302u);
    im[2] = __builtin_amdgcn_perm(w1[1], w1[0], 0x07060302u);
    im[3] = __builtin_amdgcn_perm(w1[3], w1[2], 0x07060302u);
    // (the vector elements are copied to scalars first: a bit cast straight from
    // an element of an ext_vector was compiled as a cast of element 0)
#pragma unroll
    for (int q = 0; q < 4; q++) {
        const uint32_t r = re[q], i = im[q];
        const h2 sum = __builtin_bit_cast(h2, r) + __builtin_bit_cast(h2, i);
        sm[q] = __builtin_bit_cast(uint32_t, sum);
    }
}

// ---- result tile straight from the accumulators (no LDS)
// Register group q (r = 4q..4q+3) of a 32 x 32 accumulator block holds rows
// 8q + 4(l/32) + 0..3 of column l%32 in lane l.  With C chunked along m those
// four rows are one 16-byte run of C.  With C chunked along n, a 4 x 4
// transpose within each quad of lanes (two exchange rounds of DPP quad
// permutes) leaves lane l with row 8q + 4(l/32) + l%4 and columns
// 4((l%32)/4)..+3: again one 16-byte run, and one store instruction writes
// eight whole 128-byte lines.
template <int CTRL> __device__ __forceinline__ uint32_t quad_perm(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, CTRL, 0xF, 0xF, false);
}
__device__ __forceinline__ void quad_transpose(uint32_t (&w)[4], int lane) {
    const bool b1 = (lane & 2) != 0, b0 = (lane & 1) != 0;
    // swap the off-diagonal 2 x 2 blocks with the lane two over (quad_perm 2,3,0,1)
    const uint32_t t0 = quad_perm<0x4E>(w[0]), t1 = quad_perm<0x4E>(w[1]);
    const uint32_t t2 = quad_perm<0x4E>(w[2]), t3 = quad_perm<0x4E>(w[3]);
    const uint32_t a0 = b1 ? t2 : w[0], a1 = b1 ? t3 : w[1], a2 = b1 ? w[2] : t0, a3 = b1 ? w[3] : t1;
    // transpose each 2 x 2 block with the lane one over (quad_perm 1,0,3,2)
    const uint32_t u0 = quad_perm<0xB1>(a0), u1 = quad_perm<0xB1>(a1);
    const uint32_t u2 = quad_perm<0xB1>(a2), u3 = quad_perm<0xB1>(a3);
    w[0] = b0 ? u1 : a0;
    w[1] = b0 ? a1 : u0;
    w[2] = b0 ? u3 : a2;
    w[3] = b0 ? a3 : u2;
}

// Scales, rounds and stores a wave's FM x FC accumulator blocks (4M: real and
// imaginary sets; 3M: T1, T2, T3) whose first row and column are r0, c0 (r0 a
// multiple of 64, c0 of 32); returns the lane's largest stored |re|, |im|
// (NaN as +inf).  The row and column of an entry are sums of bit-disjoint
// parts (tile origin, block, group, lane), so its offset is one per-lane base
// plus a wave-uniform offset per group.
template <typename W, bool M3, int FM, int FC, int NACC>
__device__ __forceinline__ float store_tile(const floatx16 (&acc)[FM][FC][NACC], float scale, uint32_t *Cp,
                                            const GemmShape &g, int64_t r0, int64_t c0, int lane) {
    const bool nc = g.c_nc != 0;
    const int64_t lr = 4 * (lane >> 5) + (nc ? (lane & 3) : 0);
    const int64_t lc = nc ? (lane & 28) : (lane & 31);
    uint32_t *base = Cp + seg_offset(g.cm, r0 + lr) + seg_offset(g.cn, c0 + lc);
    float mx = 0.f;
#pragma unroll
    for (int i = 0; i < FM; i++)
#pragma unroll
        for (int j = 0; j < FC; j++)
#pragma unroll
            for (int q = 0; q < 4; q++) {
                uint32_t w[4];
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    const int r = 4 * q + e;
                    float re, im;
                    if constexpr (M3) {
                        re = acc[i][j][0][r] - acc[i][j][1][r];
                        im = acc[i][j][2][r] - acc[i][j][0][r] - acc[i][j][1][r];
                    } else {
                        re = acc[i][j][0][r];
                        im = acc[i][j][1][r];
                    }
                    w[e] = Pack<W>::make(re * scale, im * scale).w;
                }
                if (nc) quad_transpose(w, lane);
                u32x4 v;
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    v[e] = w[e];
                    const float2 f = unpack(W{w[e]});
                    mx = fmaxf(mx, absmax_nan(f.x, f.y));
                }
                const int64_t uo = seg_offset(g.cm, i * 32 + 8 * q) + seg_offset(g.cn, j * 32);
                *(u32x4 *)(base + uo) = v;
                // one group at a time: the compiler would otherwise interleave
                // all of them and run out of registers
                __builtin_amdgcn_sched_barrier(0);
            }
    return mx;
}

template <bool BF, bool M3, int BM, int BN, int WM, int WN, int STAGES>
__global__ void __launch_bounds__(64 * WM * WN, (dma_min_blocks<M3, BM, BN, STAGES>()))
    gemm_dma_h_kernel(const uint32_t *__restrict__ A, const uint32_t *__restrict__ B, uint32_t *__restrict__ C,
                      GemmShape g, ScaleRefs sc) {
    using Tl = DTile<BM, BN, WM, WN, STAGES>;
    using W = typename std::conditional<BF, Bf16Word, HalfWord>::type;
    constexpr int NT = Tl::NT, FM = Tl::FM, FC = Tl::FC, WTM = Tl::WTM, WTC = Tl::WTC, BK = Tl::BK;
    extern __shared__ __align__(16) uint8_t smem[];

    const int s = blockIdx.z;
    const int64_t P = g.split;
    const int64_t b = blockIdx.y / P, part = blockIdx.y - b * P;
    const int64_t tiles_n = g.N / BN, tiles_m = g.M / BM;
    const int64_t t = xcd_tile(blockIdx.x, tiles_m * tiles_n);
    int64_t mt, nt;
    tile_coords<4>(t, tiles_m, tiles_n, mt, nt);
    const int64_t m0 = mt * BM, n0 = nt * BN;
    float scale = 1.f;
    if (P == 1) {
        int shift = step_shift(sc, s);
        if (blockIdx.x == 0 && b == 0 && threadIdx.x == 0) record_exponent(sc, s, shift);
        scale = pow2_neg(shift);
    }
    const uint32_t *Ap = A + s * g.sA + a_block(g, b) * g.bA;
    const uint32_t *Bp = B + s * g.sB + b_block(g, b) * g.bB;
    uint32_t *Cp = C + s * g.sC + b * g.bC;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave / WN, wn = wave % WN;

    // DMA: wave w fills 1 KB blocks w, w + NT/64, ... of each operand; lane j
    // of a block writes row 8 * block + j / 8, slot j % 8, which holds chunk
    // q = (j % 8) ^ (j / 8) of that row.  For k0 a multiple of 32,
    // offset(k0 + 4q) = offset(k0) + offset(4q) (both runs of a Seg are at
    // least as aligned), so the lane part is folded into the row pointers and
    // each stage adds one uniform offset.
    const int dq = (lane & 7) ^ (lane >> 3);
    const uint32_t *pa[Tl::A_PER], *pb[Tl::B_PER];
#pragma unroll
    for (int i = 0; i < Tl::A_PER; i++)
        pa[i] = Ap + seg_offset(g.am, m0 + 8 * (wave + i * (NT / 64)) + (lane >> 3)) + seg_offset(g.ak, 4 * dq);
#pragma unroll
    for (int i = 0; i < Tl::B_PER; i++)
        pb[i] = Bp + seg_offset(g.bn, n0 + 8 * (wave + i * (NT / 64)) + (lane >> 3)) + seg_offset(g.bk, 4 * dq);
    const int nk_all = (int)(g.K / BK);
    const int kt0 = (int)(nk_all * part / P), kt1 = (int)(nk_all * (part + 1) / P);
    const int nk = kt1 - kt0;
    auto issue = [&](int kt) {
        uint8_t *base = smem + (kt % STAGES) * Tl::STAGE_BYTES;
        const int64_t k0 = (int64_t)(kt0 + kt) * BK;
        const int64_t ka = seg_offset(g.ak, k0), kb = seg_offset(g.bk, k0);
#pragma unroll
        for (int i = 0; i < Tl::A_PER; i++)
            __builtin_amdgcn_global_load_lds((const void *)(pa[i] + ka),
                                             (__attribute__((address_space(3))) void *)(base + (wave + i * (NT / 64)) * 1024),
                                             16, 0, 0);
#pragma unroll
        for (int i = 0; i < Tl::B_PER; i++)
            __builtin_amdgcn_global_load_lds((const void *)(pb[i] + kb),
                                             (__attribute__((address_space(3))) void *)(base + Tl::A_BYTES +
                                                                                        (wave + i * (NT / 64)) * 1024),
                                             16, 0, 0);
    };

    static_assert(!(M3 && BF), "the DMA 3M path is FP16 only");
    constexpr int NACC = M3 ? 3 : 2;
    floatx16 acc[FM][FC][NACC];
#pragma unroll
    for (int i = 0; i < FM; i++)
#pragma unroll
        for (int j = 0; j < FC; j++)
#pragma unroll
            for (int a = 0; a < NACC; a++)
#pragma unroll
                for (int r = 0; r < 16; r++) acc[i][j][a][r] = 0.f;
    // the complex result entry r of block (i, j)
    auto c_re = [&](int i, int j, int r) {
        if constexpr (M3) return acc[i][j][0][r] - acc[i][j][1][r];
        else return acc[i][j][0][r];
    };
    auto c_im = [&](int i, int j, int r) {
        if constexpr (M3) return acc[i][j][2][r] - acc[i][j][0][r] - acc[i][j][1][r];
        else return acc[i][j][1][r];
    };

    // fragment rows: wm*WTM + 32i + lane%32 (A) and wn*WTC + 32j + lane%32
    // (B); both have row & 7 = lane & 7, so the slot of chunk 2kk + lane/32
    // is (2kk) ^ (lane/32) ^ (lane & 7); offsets within a stage, per kk
    const int f_s0 = (lane >> 5) ^ (lane & 7);
    int a_off[BK / 8], b_off[BK / 8];
#pragma unroll
    for (int kk = 0; kk < BK / 8; kk++) {
        a_off[kk] = (wm * WTM + (lane & 31)) * 128 + ((kk << 1) ^ f_s0) * 16;
        b_off[kk] = Tl::A_BYTES + (wn * WTC + (lane & 31)) * 128 + ((kk << 1) ^ f_s0) * 16;
    }

    auto load = [&](const uint8_t *sb, int kk, u32x4 (&fa)[FM], u32x4 (&fb)[FC]) {
#pragma unroll
        for (int i = 0; i < FM; i++) fa[i] = *(const u32x4 *)(sb + a_off[kk] + i * 32 * 128);
#pragma unroll
        for (int j = 0; j < FC; j++) fb[j] = *(const u32x4 *)(sb + b_off[kk] + j * 32 * 128);
    };
    // B fragment -> real-part operand (br, -bi) and imaginary-part operand (bi, br)
    auto xform = [&](const u32x4 (&fb)[FC], u32x4 (&bre)[FC], u32x4 (&bim)[FC]) {
#pragma unroll
        for (int j = 0; j < FC; j++)
#pragma unroll
            for (int q = 0; q < 4; q++) {
                bre[j][q] = fb[j][q] ^ 0x80000000u;
                bim[j][q] = __builtin_amdgcn_perm(fb[j][q], fb[j][q], 0x01000302u);
            }
    };
    auto madd = [&](const u32x4 (&fa)[FM], const u32x4 (&bre)[FC], const u32x4 (&bim)[FC]) {
#pragma unroll
        for (int j = 0; j < FC; j++)
#pragma unroll
            for (int i = 0; i < FM; i++) {
                acc[i][j][0] = mfma16<BF>(fa[i], bre[j], acc[i][j][0]);
                acc[i][j][1] = mfma16<BF>(fa[i], bim[j], acc[i][j][1]);
            }
    };
    static_assert(BK / 8 == 4, "the k-step pipeline below is written for four steps per stage");

#pragma unroll
    for (int st = 0; st < STAGES - 1; st++)
        if (st < nk) issue(st);
    // 3M chunk offsets within a stage: step ks, chunk h2 of lane l's pair
    int a3_off[2][2], b3_off[2][2];
#pragma unroll
    for (int ks = 0; ks < 2; ks++)
#pragma unroll
        for (int h2 = 0; h2 < 2; h2++) {
            const int slot = ((4 * ks + 2 * (lane >> 5) + h2) ^ (lane & 7)) * 16;
            a3_off[ks][h2] = (wm * WTM + (lane & 31)) * 128 + slot;
            b3_off[ks][h2] = Tl::A_BYTES + (wn * WTC + (lane & 31)) * 128 + slot;
        }
    auto step3 = [&](const uint8_t *sb, int ks) {
        u32x4 ar[FM], ai[FM], as[FM], br[FC], bi[FC], bs[FC];
#pragma unroll
        for (int i = 0; i < FM; i++) {
            const u32x4 w0 = *(const u32x4 *)(sb + a3_off[ks][0] + i * 32 * 128);
            const u32x4 w1 = *(const u32x4 *)(sb + a3_off[ks][1] + i * 32 * 128);
            planes3m(w0, w1, ar[i], ai[i], as[i]);
        }
#pragma unroll
        for (int j = 0; j < FC; j++) {
            const u32x4 w0 = *(const u32x4 *)(sb + b3_off[ks][0] + j * 32 * 128);
            const u32x4 w1 = *(const u32x4 *)(sb + b3_off[ks][1] + j * 32 * 128);
            planes3m(w0, w1, br[j], bi[j], bs[j]);
        }
#pragma unroll
        for (int j = 0; j < FC; j++)
#pragma unroll
            for (int i = 0; i < FM; i++) {
                acc[i][j][0] = mfma16<false>(ar[i], br[j], acc[i][j][0]);
                acc[i][j][1] = mfma16<false>(ai[i], bi[j], acc[i][j][1]);
                acc[i][j][2] = mfma16<false>(as[i], bs[j], acc[i][j][2]);
            }
    };

    for (int kt = 0; kt < nk; kt++) {
        ring_wait_for<STAGES - 2, Tl::LPT>(nk - 1 - kt);
        if (kt + STAGES - 1 < nk) issue(kt + STAGES - 1);
        const uint8_t *sb = smem + (kt % STAGES) * Tl::STAGE_BYTES;
        if constexpr (M3) {
            step3(sb, 0);
            __builtin_amdgcn_sched_barrier(0);
            step3(sb, 1);
            continue;
        }
        // Two register sets of fragments: the reads of step kk+1 are issued
        // before the matrix-core work of step kk, and a set's first use (its
        // B transform) comes before the next reads, so each wait covers only
        // reads that had a whole step to land.  The scheduling barriers keep
        // the compiler from undoing that order.
        u32x4 fa0[FM], fb0[FC], re0[FC], im0[FC], fa1[FM], fb1[FC], re1[FC], im1[FC];
        load(sb, 0, fa0, fb0);
        xform(fb0, re0, im0);
        __builtin_amdgcn_sched_barrier(0);
        load(sb, 1, fa1, fb1);
        __builtin_amdgcn_sched_barrier(0);
        madd(fa0, re0, im0);
        __builtin_amdgcn_sched_barrier(0);
        xform(fb1, re1, im1);
        __builtin_amdgcn_sched_barrier(0);
        load(sb, 2, fa0, fb0);
        __builtin_amdgcn_sched_barrier(0);
        madd(fa1, re1, im1);
        __builtin_amdgcn_sched_barrier(0);
        xform(fb0, re0, im0);
        __builtin_amdgcn_sched_barrier(0);
        load(sb, 3, fa1, fb1);
        __builtin_amdgcn_sched_barrier(0);
        madd(fa0, re0, im0);
        __builtin_amdgcn_sched_barrier(0);
        xform(fb1, re1, im1);
        madd(fa1, re1, im1);
    }
    if (P > 1) {
        float2 *pp = g.part + ((s * g.nb + b) * P + part) * g.M * g.N;
#pragma unroll
        for (int i = 0; i < FM; i++)
#pragma unroll
            for (int j = 0; j < FC; j++)
#pragma unroll
                for (int r = 0; r < 16; r++) {
                    int row = wm * WTM + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                    int col = wn * WTC + j * 32 + (lane & 31);
                    pp[(m0 + row) * g.N + n0 + col] = make_float2(c_re(i, j, r), c_im(i, j, r));
                }
        return;
    }
    // epilogue: scale, round and store from the accumulators (the last
    // stage's wait left no DMA in flight, and LDS is not touched again)
    const float mx = store_tile<W, M3>(acc, scale, Cp, g, m0 + wm * WTM, n0 + wn * WTC, lane);
    finish_max<true>(sc, s, mx);
}

// ===================================================================== thin on the matrix cores: N = 4 .. 32
//
// The VALU thin kernel spends 4 FP32 FMAs per complex product (256 per row at
// N = K = 8), which holds it near the VALU rate instead of the memory rate.
// Here v_mfma_f32_16x16x16_{f16,bf16} does the products: lane l holds
// A'[l%16][4(l/16)..+3], i.e. complex k 2(l/16), 2(l/16)+1 of row l%16,
// B'[4(l/16)..+3][l%16], and the result rows 4(l/16)..+3 of real column
// l%16.  Real column 2n + d of the padded B' is (br, -bi) for d = 0 and
// (bi, br) for d = 1 (4M), so lanes 2n and 2n+1 hold Re and Im of complex
// column n and swap them with one DPP quad permute (columns n >= N are zero).
// A wave takes 64 rows per pass.  A chunked along k: one 8-byte load per
// lane reads 16 whole rows (K = 2 or 4 fill one k chunk in part: the lanes
// past K load nothing and hold zeros in A and B').  A chunked along m: the pass's K x 64 entries
// come in 16-byte chunks along m and go through an LDS region of the wave's
// own, read back k-major.  The next pass's A is loaded before this pass's
// result is staged (LDS, [row][n] words) and stored in 16-byte chunks, into
// the register buffer the matrix cores have just read (a second buffer only
// for N <= 8 with A chunked along k and K <= 16).

typedef _Float16 half4_t __attribute__((ext_vector_type(4)));
typedef short short4_t __attribute__((ext_vector_type(4)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

template <bool BF> __device__ __forceinline__ floatx4 mfma16x16(u32x2 a, u32x2 b, floatx4 c) {
    if constexpr (BF)
        return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(short4_t, a), __builtin_bit_cast(short4_t, b),
                                                         c, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_16x16x16f16(__builtin_bit_cast(half4_t, a), __builtin_bit_cast(half4_t, b), c, 0,
                                                     0, 0);
}

// wait for this wave's LDS traffic (its own region: no block barrier)
__device__ __forceinline__ void wave_lds_wait() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0), nothing else
    asm volatile("" ::: "memory");
}

template <bool BF, int NB, int KCM, bool AKC>
__global__ void __launch_bounds__(256) gemm_thinm_kernel(const uint32_t *__restrict__ A, const uint32_t *__restrict__ B,
                                                         uint32_t *__restrict__ C, GemmShape g, ScaleRefs sc) {
    using W = typename std::conditional<BF, Bf16Word, HalfWord>::type;
    // NS: staged words per result row; RW: rows per wave pass; KCM: k chunks of
    // 8 at most; AS: words per staged A row (64 m, padded against bank conflicts)
    constexpr int NS = 8 * NB, RW = 64, AS = RW + 4, NCH = AKC ? 1 : 2 * KCM;
    __shared__ __align__(16) uint32_t Cs[4][RW * NS];
    __shared__ __align__(16) uint32_t Asm[AKC ? 1 : 4][AKC ? 1 : 8 * KCM * AS];
    const int s = blockIdx.z;
    const int64_t b = blockIdx.y;
    const int shift = step_shift(sc, s);
    if (blockIdx.x == 0 && b == 0 && threadIdx.x == 0) record_exponent(sc, s, shift);
    const float scale = pow2_neg(shift);
    const uint32_t *Ap = A + s * g.sA + a_block(g, b) * g.bA;
    const uint32_t *Bp = B + s * g.sB + b_block(g, b) * g.bB;
    uint32_t *Cp = C + s * g.sC + b * g.bC;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // k chunks of 8 complex; K = 2 or 4 is one chunk whose lanes past K hold
    // zeros in both operands (lane l covers complex k 8t + 2(l/16), + 1)
    const int kk = (int)g.K, kc = (kk + 7) / 8, nn = (int)g.N;
    const bool klane = 2 * (lane >> 4) < kk;   // this lane's k pair exists in chunk 0
    const bool odd = (lane & 1) != 0;
    // padded B' operands of every k chunk and column block
    u32x2 bop[KCM][NB];
#pragma unroll
    for (int t = 0; t < KCM; t++)
#pragma unroll
        for (int q = 0; q < NB; q++) {
            u32x2 v = {0u, 0u};
            const int n = q * 8 + (lane & 15) / 2;
            if (t < kc && n < nn && (t > 0 || klane)) {
                const int64_t k = 8 * t + 2 * (lane >> 4);
#pragma unroll
                for (int e = 0; e < 2; e++) {
                    const uint32_t w = Bp[b_index(g, n, k + e)];
                    v[e] = odd ? __builtin_amdgcn_perm(w, w, 0x01000302u) : (w ^ 0x80000000u);
                }
            }
            bop[t][q] = v;
        }
    uint32_t *cs = Cs[wave];
    uint32_t *as = Asm[AKC ? 0 : wave];
    float mx = 0.f;
    const int64_t units = g.M / RW, step = (int64_t)gridDim.x * 4;
    // A of a 64-row pass as loaded: k-chunked, the MFMA operands themselves
    // (four groups of 16 rows); m-chunked, 16-byte chunks of 4 rows at one k
    struct Raw {
        u32x2 a[4][KCM];
        u32x4 c[NCH];
    };
    auto load_pass = [&](int64_t u, Raw &r) {
        const int64_t m0 = u * RW;
        if constexpr (AKC) {
#pragma unroll
            for (int gq = 0; gq < 4; gq++) {
                const uint32_t *ap = Ap + seg_offset(g.am, m0 + 16 * gq + (lane & 15));
#pragma unroll
                for (int t = 0; t < KCM; t++)
                    if (t < kc)
                        r.a[gq][t] = (t > 0 || klane) ? *(const u32x2 *)(ap + seg_offset(g.ak, 8 * t + 2 * (lane >> 4)))
                                                      : u32x2{0u, 0u};
            }
        } else {
            // chunk c: k = c / 16, rows 4 (c % 16)..+3
#pragma unroll
            for (int i = 0; i < NCH; i++) {
                const int c = i * 64 + lane, k = c >> 4, m4 = (c & 15) * 4;
                if (k < kk) r.c[i] = *(const u32x4 *)(Ap + seg_offset(g.am, m0 + m4) + seg_offset(g.ak, k));
            }
        }
    };
    // MFMA operands from a loaded pass (m-chunked A: through the LDS region)
    auto operands = [&](Raw &r) {
        if constexpr (!AKC) {
#pragma unroll
            for (int i = 0; i < NCH; i++) {
                const int c = i * 64 + lane, k = c >> 4, m4 = (c & 15) * 4;
                if (k < kk) *(u32x4 *)(as + k * AS + m4) = r.c[i];
            }
            wave_lds_wait();
#pragma unroll
            for (int gq = 0; gq < 4; gq++)
#pragma unroll
                for (int t = 0; t < KCM; t++)
                    if (t < kc) {
                        const int k = 8 * t + 2 * (lane >> 4), m = 16 * gq + (lane & 15);
                        r.a[gq][t] = (t > 0 || klane) ? u32x2{as[k * AS + m], as[(k + 1) * AS + m]} : u32x2{0u, 0u};
                    }
            wave_lds_wait();   // read out before the next pass writes
        }
    };
    auto pass = [&](int64_t u, Raw &cur, Raw &nxt) {
        const int64_t m0 = u * RW;
        operands(cur);
        floatx4 acc[4][NB];
#pragma unroll
        for (int gq = 0; gq < 4; gq++)
#pragma unroll
            for (int q = 0; q < NB; q++) {
                acc[gq][q] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int t = 0; t < KCM; t++)
                    if (t < kc) acc[gq][q] = mfma16x16<BF>(cur.a[gq][t], bop[t][q], acc[gq][q]);
            }
        if (u + step < units) load_pass(u + step, nxt);
        // Re/Im from the lane pair; even lanes stage rows e = 0, 1 of their
        // group, odd lanes rows 2, 3
#pragma unroll
        for (int gq = 0; gq < 4; gq++)
#pragma unroll
            for (int q = 0; q < NB; q++)
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    const float own = acc[gq][q][e];
                    const float other = __uint_as_float(quad_perm<0xB1>(__float_as_uint(own)));
                    const float re = odd ? other : own, im = odd ? own : other;
                    const int n = q * 8 + (lane & 15) / 2;
                    if ((e >> 1) == (int)odd && n < nn) {
                        const int row = 16 * gq + 4 * (lane >> 4) + e;
                        cs[row * NS + n] = Pack<W>::make(re * scale, im * scale).w;
                    }
                }
        wave_lds_wait();
        // 16-byte chunks: 64 rows x N words
        const int nq = nn / 4;
#pragma unroll
        for (int uq = 0; uq < NS / 4; uq++) {
            if (uq >= nq) break;
            const int c = uq * 64 + lane;
            u32x4 v;
            int64_t off;
            if (g.c_nc) {
                const int row = c / nq, n4 = (c % nq) * 4;
                v = *(const u32x4 *)(cs + row * NS + n4);
                off = c_index(g, m0 + row, n4);
            } else {
                const int n = c / (RW / 4), r4 = (c % (RW / 4)) * 4;
#pragma unroll
                for (int e = 0; e < 4; e++) v[e] = cs[(r4 + e) * NS + n];
                off = c_index(g, m0 + r4, n);
            }
            *(u32x4 *)(Cp + off) = v;
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const float2 f = unpack(W{v[e]});
                mx = fmaxf(mx, absmax_nan(f.x, f.y));
            }
        }
        wave_lds_wait();   // read out before the next pass writes
    };
    int64_t u = (int64_t)blockIdx.x * 4 + wave;
    if constexpr (!(NB == 1 && AKC && KCM == 2)) {
        // one buffer: the next pass loads into it once this pass's matrix-core
        // work has taken its operands, and the loads are in flight during the
        // epilogue either way.  Fewer registers, more waves per SIMD: with
        // N = 16 the K = 32..64 steps move 4.6-5.0 TB/s instead of 3.4-3.9, and
        // with A chunked along m the short-k steps gain 12-36%.  (The
        // smallest variant already runs four waves per SIMD and keeps two.)
        Raw r0;
        if (u < units) load_pass(u, r0);
        while (u < units) {
            pass(u, r0, r0);
            u += step;
        }
    } else {
        Raw r0, r1;
        if (u < units) load_pass(u, r0);
        while (u < units) {
            pass(u, r0, r1);
            u += step;
            if (u >= units) break;
            pass(u, r1, r0);
            u += step;
        }
    }
    finish_max<true>(sc, s, mx);
}

// ===================================================================== persistent LDS-DMA 4M (short k)
//
// The short-k steps (K = 2^6..2^9 complex) write a large C per tile, and a
// one-tile block fills its ring from empty once per tile.  Here two blocks
// per CU (two-stage rings) each walk a list of tiles (all slices and
// inner-batch entries of the launch) and the DMA ring runs on across tile
// boundaries: the first stage of tile j+1 is in flight while tile j's last
// stage is multiplied and its result is stored (straight from the
// accumulators), and the waits never cover the stores unless a later stage
// needs them to.  On 128 x 128 tiles, measured against the one-tile kernel
// on the same tile, it is level on K = 2^7 and 5-10% slower on K = 2^9.  On
// 256 x 64 tiles with four waves it serves the HBM-bound N = 64 steps, whose
// tiles hold two to four k-stages: 15-19% above the one-tile narrow kernels
// there (about 5 TB/s).  The autotuner picks.
//
// Vector-memory ordering: the ring wait counts every vector memory
// instruction issued after the awaited stage's loads -- the later stages'
// loads and, when a tile ended in between, that tile's stores -- relying on
// vmcnt retiring loads and stores in issue order.
//
// Tile order: block i (on XCD i % 8) takes items i, i + G, i + 2G, ...
// (G = blocks in the grid, a multiple of 8); within each window of G items
// the XCD's blocks take one run of G / 8 consecutive items, so the tiles an
// XCD holds at once form a patch of row and column blocks of one slice.

template <int BM, int BN, int WM, int WN, int STAGES>
struct PTile {
    using D = DTile<BM, BN, WM, WN, STAGES>;
    static constexpr int NT = D::NT, BK = D::BK;
    static constexpr int STAGE_BYTES = D::STAGE_BYTES;
    static constexpr int RING_BYTES = STAGES * STAGE_BYTES;
    static constexpr int LDS_BYTES = RING_BYTES;                 // the result leaves from registers
    static constexpr int NS = D::FM * D::FC * 4;                 // 16-byte stores per thread and tile
    static constexpr int LPT = D::LPT;
    // two blocks per CU when two rings fit in LDS
    static constexpr int BLOCKS_PER_CU = 2 * LDS_BYTES <= 160 * 1024 ? 2 : 1;
    static_assert((STAGES - 2) * LPT + NS < 64, "vmcnt range");
    static_assert(LDS_BYTES <= 160 * 1024, "LDS");
};

// wait until at most VM vector memory instructions are outstanding (VM = 63:
// no vector memory wait), LDS traffic done, then the block barrier
template <int STAGES, int LPT, int NS>
__device__ __forceinline__ void pring_wait(int ahead, bool epi) {
    // ahead in [0, STAGES - 2]
    if constexpr (STAGES == 2) {
        if (epi) ring_wait<NS>();
        else ring_wait<0>();
    } else if constexpr (STAGES == 3) {
        if (ahead == 1) {
            if (epi) ring_wait<LPT + NS>();
            else ring_wait<LPT>();
        } else {
            if (epi) ring_wait<NS>();
            else ring_wait<0>();
        }
    } else {
        static_assert(STAGES == 2 || STAGES == 3, "stages");
    }
}

template <bool BF, int BM, int BN, int WM, int WN, int STAGES>
__global__ void __launch_bounds__(64 * WM * WN, (PTile<BM, BN, WM, WN, STAGES>::BLOCKS_PER_CU))
    gemm_dmap_h_kernel(const uint32_t *__restrict__ A, const uint32_t *__restrict__ B, uint32_t *__restrict__ C,
                       GemmShape g, ScaleRefs sc, int S) {
    using Pt = PTile<BM, BN, WM, WN, STAGES>;
    using Tl = DTile<BM, BN, WM, WN, STAGES>;
    using W = typename std::conditional<BF, Bf16Word, HalfWord>::type;
    constexpr int NT = Pt::NT, FM = Tl::FM, FC = Tl::FC, WTM = Tl::WTM, WTC = Tl::WTC, BK = Pt::BK;
    constexpr int LPT = Pt::LPT, NS = Pt::NS;
    extern __shared__ __align__(16) uint8_t smem[];

    const int64_t tiles_n = g.N / BN, tiles_m = g.M / BM, tiles = tiles_m * tiles_n;
    const int64_t total = (int64_t)S * g.nb * tiles;
    const int64_t G = gridDim.x, bi = blockIdx.x;
    if (bi >= total) return;
    const int64_t n_items = (total - bi + G - 1) / G;
    const int nk = (int)(g.K / BK);
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave / WN, wn = wave % WN;
    const int dq = (lane & 7) ^ (lane >> 3);

    // item j of this block -> (slice, batch entry, tile origin)
    struct Item {
        int s;
        int64_t b, m0, n0;
    };
    auto item_of = [&](int64_t j) {
        const int64_t w0 = j * G;
        int64_t idx = w0 + bi;
        if (w0 + G <= total && (G & 7) == 0) idx = w0 + (bi & 7) * (G >> 3) + (bi >> 3);
        Item it;
        const int64_t t = idx % tiles, rest = idx / tiles;
        it.b = rest % g.nb;
        it.s = (int)(rest / g.nb);
        int64_t mt, nt;
        tile_coords<4>(t, tiles_m, tiles_n, mt, nt);
        it.m0 = mt * BM;
        it.n0 = nt * BN;
        return it;
    };
    // DMA row pointers of an item (lane part folded in, as in the one-tile kernel)
    struct Ptrs {
        const uint32_t *pa[Tl::A_PER], *pb[Tl::B_PER];
    };
    auto ptrs_of = [&](const Item &it) {
        Ptrs p;
        const uint32_t *Ap = A + it.s * g.sA + a_block(g, it.b) * g.bA;
        const uint32_t *Bp = B + it.s * g.sB + b_block(g, it.b) * g.bB;
#pragma unroll
        for (int i = 0; i < Tl::A_PER; i++)
            p.pa[i] = Ap + seg_offset(g.am, it.m0 + 8 * (wave + i * (NT / 64)) + (lane >> 3)) + seg_offset(g.ak, 4 * dq);
#pragma unroll
        for (int i = 0; i < Tl::B_PER; i++)
            p.pb[i] = Bp + seg_offset(g.bn, it.n0 + 8 * (wave + i * (NT / 64)) + (lane >> 3)) + seg_offset(g.bk, 4 * dq);
        return p;
    };
    auto issue = [&](const Ptrs &p, int slot, int kt) {
        uint8_t *base = smem + slot * Pt::STAGE_BYTES;
        const int64_t k0 = (int64_t)kt * BK;
        const int64_t ka = seg_offset(g.ak, k0), kb = seg_offset(g.bk, k0);
#pragma unroll
        for (int i = 0; i < Tl::A_PER; i++)
            __builtin_amdgcn_global_load_lds((const void *)(p.pa[i] + ka),
                                             (__attribute__((address_space(3))) void *)(base + (wave + i * (NT / 64)) * 1024),
                                             16, 0, 0);
#pragma unroll
        for (int i = 0; i < Tl::B_PER; i++)
            __builtin_amdgcn_global_load_lds((const void *)(p.pb[i] + kb),
                                             (__attribute__((address_space(3))) void *)(base + Tl::A_BYTES +
                                                                                        (wave + i * (NT / 64)) * 1024),
                                             16, 0, 0);
    };

    const int f_s0 = (lane >> 5) ^ (lane & 7);
    int a_off[BK / 8], b_off[BK / 8];
#pragma unroll
    for (int kk = 0; kk < BK / 8; kk++) {
        a_off[kk] = (wm * WTM + (lane & 31)) * 128 + ((kk << 1) ^ f_s0) * 16;
        b_off[kk] = Tl::A_BYTES + (wn * WTC + (lane & 31)) * 128 + ((kk << 1) ^ f_s0) * 16;
    }
    floatx16 acc[FM][FC][2];
    auto load = [&](const uint8_t *sb, int kk, u32x4 (&fa)[FM], u32x4 (&fb)[FC]) {
#pragma unroll
        for (int i = 0; i < FM; i++) fa[i] = *(const u32x4 *)(sb + a_off[kk] + i * 32 * 128);
#pragma unroll
        for (int j = 0; j < FC; j++) fb[j] = *(const u32x4 *)(sb + b_off[kk] + j * 32 * 128);
    };
    auto xform = [&](const u32x4 (&fb)[FC], u32x4 (&bre)[FC], u32x4 (&bim)[FC]) {
#pragma unroll
        for (int j = 0; j < FC; j++)
#pragma unroll
            for (int q = 0; q < 4; q++) {
                bre[j][q] = fb[j][q] ^ 0x80000000u;
                bim[j][q] = __builtin_amdgcn_perm(fb[j][q], fb[j][q], 0x01000302u);
            }
    };
    auto madd = [&](const u32x4 (&fa)[FM], const u32x4 (&bre)[FC], const u32x4 (&bim)[FC]) {
#pragma unroll
        for (int j = 0; j < FC; j++)
#pragma unroll
            for (int i = 0; i < FM; i++) {
                acc[i][j][0] = mfma16<BF>(fa[i], bre[j], acc[i][j][0]);
                acc[i][j][1] = mfma16<BF>(fa[i], bim[j], acc[i][j][1]);
            }
    };
    static_assert(BK / 8 == 4, "four k-steps per stage");

    Item cur = item_of(0);
    Ptrs pc = ptrs_of(cur), pn = pc;
    Item nxt = cur;
    if (n_items > 1) {
        nxt = item_of(1);
        pn = ptrs_of(nxt);
    }
    // stage counters in 32 bits (the launcher checks the range); ring slots
    // rotate without a division
    const int Q = (int)(n_items * nk);
#pragma unroll
    for (int st = 0; st < STAGES - 1; st++)
        if (st < Q) issue(pc, st, st);   // nk >= STAGES - 1: all in item 0
    int slot_r = 0, slot_w = STAGES - 1;   // ring slots of stages q and q + STAGES - 1

    float mx = 0.f;           // running max of the stored values of slice cur.s
    int mx_slice = cur.s;
    auto flush = [&]() {
        float v = wave_max(mx);
        if (lane == 0) {
            atomicMax(&sc.maxC[mx_slice], __float_as_uint(v));
            if (!(v <= sc.flag_above) && sc.flag) atomicOr(sc.flag, 1u);
        }
        mx = 0.f;
    };

    for (int64_t j = 0; j < n_items; j++) {
#pragma unroll
        for (int i = 0; i < FM; i++)
#pragma unroll
            for (int jj = 0; jj < FC; jj++)
#pragma unroll
                for (int r = 0; r < 16; r++) {
                    acc[i][jj][0][r] = 0.f;
                    acc[i][jj][1][r] = 0.f;
                }
        const int q0 = (int)j * nk;
        for (int kt = 0; kt < nk; kt++) {
            const int q = q0 + kt;
            {
                const int later = Q - 1 - q;
                const int ahead = (int)(later < STAGES - 2 ? later : STAGES - 2);
                // the previous tile's stores went out after this stage's loads
                const bool epi = j > 0 && kt <= STAGES - 2;
                pring_wait<STAGES, LPT, NS>(ahead, epi);
            }
            {
                if (q + STAGES - 1 < Q) {
                    const int kti = kt + STAGES - 1;
                    if (kti < nk) issue(pc, slot_w, kti);
                    else issue(pn, slot_w, kti - nk);
                }
            }
            const uint8_t *sb = smem + slot_r * Pt::STAGE_BYTES;
            slot_r = slot_r == STAGES - 1 ? 0 : slot_r + 1;
            slot_w = slot_w == STAGES - 1 ? 0 : slot_w + 1;
            u32x4 fa0[FM], fb0[FC], re0[FC], im0[FC], fa1[FM], fb1[FC], re1[FC], im1[FC];
            load(sb, 0, fa0, fb0);
            xform(fb0, re0, im0);
            __builtin_amdgcn_sched_barrier(0);
            load(sb, 1, fa1, fb1);
            __builtin_amdgcn_sched_barrier(0);
            madd(fa0, re0, im0);
            __builtin_amdgcn_sched_barrier(0);
            xform(fb1, re1, im1);
            __builtin_amdgcn_sched_barrier(0);
            load(sb, 2, fa0, fb0);
            __builtin_amdgcn_sched_barrier(0);
            madd(fa1, re1, im1);
            __builtin_amdgcn_sched_barrier(0);
            xform(fb0, re0, im0);
            __builtin_amdgcn_sched_barrier(0);
            load(sb, 3, fa1, fb1);
            __builtin_amdgcn_sched_barrier(0);
            madd(fa0, re0, im0);
            __builtin_amdgcn_sched_barrier(0);
            xform(fb1, re1, im1);
            madd(fa1, re1, im1);
        }
        // ---- tile done: scale and store (the stores drain under the next tile)
        const int shift = step_shift(sc, cur.s);
        if (cur.b == 0 && cur.m0 == 0 && cur.n0 == 0 && tid == 0) record_exponent(sc, cur.s, shift);
        const float scale = pow2_neg(shift);
        if (cur.s != mx_slice) {
            flush();
            mx_slice = cur.s;
        }
        uint32_t *Cp = C + cur.s * g.sC + cur.b * g.bC;
        mx = fmaxf(mx, store_tile<W, false>(acc, scale, Cp, g, cur.m0 + wm * WTM, cur.n0 + wn * WTC, lane));
        if (j + 1 < n_items) {
            cur = nxt;
            pc = pn;
            if (j + 2 < n_items) {
                nxt = item_of(j + 2);
                pn = ptrs_of(nxt);
            }
        }
    }
    flush();
}

// ===================================================================== matrix cores, complex64 4M
// v_mfma_f32_32x32x2f32: lane l holds A'[l%32][l/32] and B'[l/32][l%32];
// one MFMA per complex k (k' = 2k + c).

template <int BM, int BN, int BK, int WM, int WN>
struct CTile {
    static constexpr int NT = 64 * WM * WN;
    static constexpr int LDA = BK + 1, LDB = BK + 1;
    static constexpr int AB = 2 * (BM * LDA + BN * LDB) * 8;
    static constexpr int CB = BM * BN * 8;
    static constexpr int LDS_BYTES = AB > CB ? AB : CB;
    static constexpr int WTM = BM / WM, WTN = 2 * BN / WN;
    static constexpr int FM = WTM / 32, FN = WTN / 32;
    static constexpr int A_CHUNKS = BM * BK / 2, B_CHUNKS = BN * BK / 2;   // 16-byte chunks (2 complex)
    static constexpr int A_PER = (A_CHUNKS + NT - 1) / NT, B_PER = (B_CHUNKS + NT - 1) / NT;
    static_assert(FM >= 1 && FN >= 1, "wave tile too small");
    static_assert(LDS_BYTES <= 160 * 1024, "LDS");
};

template <int BM, int BN, int BK, int WM, int WN>
__global__ void __launch_bounds__(64 * WM * WN)
    gemm_mfma_c64_kernel(const float2 *__restrict__ A, const float2 *__restrict__ B, float2 *__restrict__ C,
                         GemmShape g) {
    using Tl = CTile<BM, BN, BK, WM, WN>;
    constexpr int NT = Tl::NT, LDA = Tl::LDA, LDB = Tl::LDB, FM = Tl::FM, FN = Tl::FN;
    constexpr int WTM = Tl::WTM, WTN = Tl::WTN;
    extern __shared__ __align__(16) uint8_t smem[];
    float2 *lds = (float2 *)smem;
    auto As = [&](int buf) { return lds + buf * (BM * LDA); };
    auto Bs = [&](int buf) { return lds + 2 * BM * LDA + buf * (BN * LDB); };

    const int s = blockIdx.z;
    const int64_t P = g.split;
    const int64_t b = blockIdx.y / P, part = blockIdx.y - b * P;
    const int64_t tiles_n = (g.N + BN - 1) / BN;
    const int64_t tiles_m = (g.M + BM - 1) / BM;
    const int64_t t = xcd_tile(blockIdx.x, tiles_m * tiles_n);
    int64_t mt, nt;
    tile_coords<4>(t, tiles_m, tiles_n, mt, nt);
    const int64_t m0 = mt * BM, n0 = nt * BN;
    const float2 *Ap = A + s * g.sA + a_block(g, b) * g.bA;
    const float2 *Bp = B + s * g.sB + b_block(g, b) * g.bB;
    float2 *Cp = C + s * g.sC + b * g.bC;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave / WN, wn = wave % WN;

    float4 ra[Tl::A_PER], rb[Tl::B_PER];
    auto gload = [&](int64_t k0) {
#pragma unroll
        for (int i = 0; i < Tl::A_PER; i++) {
            int c = tid + i * NT;
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (c < Tl::A_CHUNKS) {
                if (g.a_kc) {
                    int row = c / (BK / 2), col = (c % (BK / 2)) * 2;
                    int64_t gm = m0 + row, gk = k0 + col;
                    if (gm < g.M && gk < g.K) v = *(const float4 *)(Ap + a_index(g, gm, gk));
                } else {
                    int kr = c / (BM / 2), mc = (c % (BM / 2)) * 2;
                    int64_t gk = k0 + kr, gm = m0 + mc;
                    if (gk < g.K && gm < g.M) v = *(const float4 *)(Ap + a_index(g, gm, gk));
                }
            }
            ra[i] = v;
        }
#pragma unroll
        for (int i = 0; i < Tl::B_PER; i++) {
            int c = tid + i * NT;
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (c < Tl::B_CHUNKS) {
                if (g.b_kc) {
                    int row = c / (BK / 2), col = (c % (BK / 2)) * 2;
                    int64_t gn = n0 + row, gk = k0 + col;
                    if (gn < g.N && gk < g.K) v = *(const float4 *)(Bp + b_index(g, gn, gk));
                } else {
                    int kr = c / (BN / 2), nc = (c % (BN / 2)) * 2;
                    int64_t gk = k0 + kr, gn = n0 + nc;
                    if (gk < g.K && gn < g.N) v = *(const float4 *)(Bp + b_index(g, gn, gk));
                }
            }
            rb[i] = v;
        }
    };
    auto sstore = [&](int buf) {
        float2 *a = As(buf), *bb = Bs(buf);
#pragma unroll
        for (int i = 0; i < Tl::A_PER; i++) {
            int c = tid + i * NT;
            if (c < Tl::A_CHUNKS) {
                if (g.a_kc) {
                    int row = c / (BK / 2), col = (c % (BK / 2)) * 2;
                    a[row * LDA + col] = make_float2(ra[i].x, ra[i].y);
                    a[row * LDA + col + 1] = make_float2(ra[i].z, ra[i].w);
                } else {
                    int kr = c / (BM / 2), mc = (c % (BM / 2)) * 2;
                    a[mc * LDA + kr] = make_float2(ra[i].x, ra[i].y);
                    a[(mc + 1) * LDA + kr] = make_float2(ra[i].z, ra[i].w);
                }
            }
        }
#pragma unroll
        for (int i = 0; i < Tl::B_PER; i++) {
            int c = tid + i * NT;
            if (c < Tl::B_CHUNKS) {
                if (g.b_kc) {
                    int row = c / (BK / 2), col = (c % (BK / 2)) * 2;
                    bb[row * LDB + col] = make_float2(rb[i].x, rb[i].y);
                    bb[row * LDB + col + 1] = make_float2(rb[i].z, rb[i].w);
                } else {
                    int kr = c / (BN / 2), nc = (c % (BN / 2)) * 2;
                    bb[nc * LDB + kr] = make_float2(rb[i].x, rb[i].y);
                    bb[(nc + 1) * LDB + kr] = make_float2(rb[i].z, rb[i].w);
                }
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

    const int64_t nk_all = (g.K + BK - 1) / BK;
    const int64_t kt0 = nk_all * part / P, kt1 = nk_all * (part + 1) / P;
    const int64_t nk = kt1 - kt0;
    gload(kt0 * BK);
    sstore(0);
    __syncthreads();
    const int c = lane >> 5;        // k' parity this lane feeds: 0 = re, 1 = im
    const int d = lane & 1;         // output column parity
    for (int64_t kt = 0; kt < nk; kt++) {
        const int buf = kt & 1;
        if (kt + 1 < nk) gload((kt0 + kt + 1) * BK);
        const float2 *a = As(buf), *bb = Bs(buf);
#pragma unroll 4
        for (int kk = 0; kk < BK; kk++) {
            float af[FM], bf[FN];
#pragma unroll
            for (int i = 0; i < FM; i++) {
                float2 v = a[(wm * WTM + i * 32 + (lane & 31)) * LDA + kk];
                af[i] = c ? v.y : v.x;
            }
#pragma unroll
            for (int j = 0; j < FN; j++) {
                float2 v = bb[((wn * WTN + j * 32 + (lane & 31)) >> 1) * LDB + kk];
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
    if (P > 1) {
        float *pp = (float *)(g.part + ((s * g.nb + b) * P + part) * g.M * g.N);
#pragma unroll
        for (int i = 0; i < FM; i++)
#pragma unroll
            for (int j = 0; j < FN; j++)
#pragma unroll
                for (int r = 0; r < 16; r++) {
                    int row = wm * WTM + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                    int col = wn * WTN + j * 32 + (lane & 31);
                    pp[(m0 + row) * 2 * g.N + 2 * n0 + col] = acc[i][j][r];
                }
        return;
    }
    float *Cs = (float *)smem;   // [BM][2*BN]
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
        if (g.c_nc) {
            int row = cc / (BN / 2), col = (cc % (BN / 2)) * 2;
            int64_t gm = m0 + row, gn = n0 + col;
            if (gm < g.M && gn < g.N) *(float4 *)(Cp + c_index(g, gm, gn)) = *(const float4 *)(Cs + row * 2 * BN + 2 * col);
        } else {
            int col = cc / (BM / 2), row = (cc % (BM / 2)) * 2;
            int64_t gm = m0 + row, gn = n0 + col;
            if (gm < g.M && gn < g.N) {
                float2 v0 = *(const float2 *)(Cs + row * 2 * BN + 2 * col);
                float2 v1 = *(const float2 *)(Cs + (row + 1) * 2 * BN + 2 * col);
                *(float4 *)(Cp + c_index(g, gm, gn)) = make_float4(v0.x, v0.y, v1.x, v1.y);
            }
        }
    }
}

// ===================================================================== split-K reduction
// C[m][n] = sum over parts p = 0..P-1 of part[p][m][n], in that order; then the
// usual epilogue (scale, round, orientation, max, overflow flag).

template <typename W, bool SCALE>
__global__ void __launch_bounds__(256) splitk_reduce_kernel(W *__restrict__ C, GemmShape g, ScaleRefs sc) {
    const int s = blockIdx.z;
    const int64_t b = blockIdx.y;
    int shift = SCALE ? step_shift(sc, s) : 0;
    if (SCALE && blockIdx.x == 0 && b == 0 && threadIdx.x == 0) record_exponent(sc, s, shift);
    const float scale = pow2_neg(shift);
    const int64_t MN = g.M * g.N;
    const float2 *pp = g.part + (s * g.nb + b) * g.split * MN;
    W *Cp = C + s * g.sC + b * g.bC;
    float mx = 0.f;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < MN; i += (int64_t)gridDim.x * blockDim.x) {
        float re = 0.f, im = 0.f;
        for (int64_t p = 0; p < g.split; p++) {
            float2 v = pp[p * MN + i];
            re += v.x;
            im += v.y;
        }
        const int64_t m = i / g.N, n = i - m * g.N;
        mx = fmaxf(mx, store_entry<W, SCALE>(Cp + c_index(g, m, n), re, im, scale));
    }
    finish_max<SCALE>(sc, s, mx);
}

// ===================================================================== dispatch

const char *kernel_name(int k) {
    switch (k) {
        case K_NAIVE: return "naive";
        case K_SKINNY_N: return "skinny";
        case K_MFMA_S: return "mfma_s";
        case K_MFMA_M: return "mfma_m";
        case K_MFMA_L: return "mfma_l";
        case K_MFMA_W: return "mfma_w";
        case K_MFMA_XL: return "mfma_xl";
        case K_MFMA_L2: return "mfma_l2";
        case K_DMA_4: return "dma_4";
        case K_DMA_8: return "dma_8";
        case K_DMA_8W: return "dma_8w";
        case K_DMA_2: return "dma_2";
        case K_DMA_N64: return "dma_n64";
        case K_DMA_N32: return "dma_n32";
        case K_DMA3_N64: return "dma3_n64";
        case K_DMA3_2: return "dma3_2";
        case K_DMAP_2: return "dmap_2";
        case K_DMAP_N64: return "dmap_n64";
        case K_THINM: return "thinm";
        default: return "?";
    }
}

// block tile (rows, complex columns) of each matrix-core variant
struct TileCfg {
    int BM, BN;
};
static TileCfg tile_of(int kid, Dtype dt, Algo al) {
    if (dt == Dtype::C64) {
        switch (kid) {
            case K_MFMA_S: return {64, 16};
            case K_MFMA_M: return {128, 16};
            case K_MFMA_L: return {128, 32};
            case K_MFMA_W: return {256, 16};
            case K_MFMA_XL: return {128, 64};
            case K_MFMA_L2: return {256, 32};
        }
    } else if (al == Algo::M4) {
        switch (kid) {
            case K_MFMA_S: return {64, 16};
            case K_MFMA_M: return {128, 32};
            case K_MFMA_L: return {128, 64};
            case K_MFMA_W: return {256, 16};
            case K_MFMA_XL: return {256, 128};
            case K_MFMA_L2: return {128, 128};
            case K_DMA_4: return {256, 128};
            case K_DMA_8: return {256, 128};
            case K_DMA_8W: return {256, 128};
            case K_DMA_2: return {128, 128};
            case K_DMA_N64: return {256, 64};
            case K_DMA_N32: return {256, 32};
            case K_DMAP_2: return {128, 128};
            case K_DMAP_N64: return {256, 64};
            case K_THINM: return {64, 4};
        }
    } else {
        switch (kid) {
            case K_MFMA_S: return {64, 32};
            case K_MFMA_M: return {128, 64};
            case K_MFMA_L: return {128, 128};
            case K_MFMA_W: return {256, 32};
            case K_MFMA_XL: return {256, 64};
            case K_MFMA_L2: return {128, 32};
            case K_DMA3_N64: return {256, 64};
            case K_DMA3_2: return {128, 128};
        }
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
    if (dt == Dtype::C64 && al == Algo::M3) return false;
    if (kid >= K_DMA_4 && kid <= K_DMA_N32) {
        // 16-bit 4M, both operands chunked along k, whole tiles and k-tiles
        if (dt == Dtype::C64 || al != Algo::M4 || !g.a_kc || !g.b_kc) return false;
        if (g.K % 32) return false;
    }
    if (kid == K_THINM) {
        // thin on the matrix cores: 4M, N = 4, 8 or 16, K = 2, 4 or a multiple
        // of 8 up to 64 (16 when A is chunked along m); N = 32 with K up to
        // 16; whole 64-row passes
        if (dt == Dtype::C64 || al != Algo::M4) return false;
        if (!(g.N == 4 || g.N == 8 || g.N == 16 || g.N == 32) || g.M % 64) return false;
        if (g.K % 8 && g.K != 2 && g.K != 4) return false;
        if (g.K > (g.a_kc && g.N <= 16 ? 64 : 16)) return false;
        // its own access rules: A in 8-byte pairs of k (chunked along k) or
        // 16-byte chunks of m, B entry by entry, C in 16-byte chunks
        auto run = [&](const Seg &sg, int64_t ext, int lo) { return sg.ls == 0 && seg_low_run(sg, ext) >= lo; };
        if (!(g.a_kc ? run(g.ak, g.K, 1) : run(g.am, g.M, 2))) return false;
        return g.c_nc ? run(g.cn, g.N, 2) : run(g.cm, g.M, 2);
    }
    if (kid == K_DMAP_2 || kid == K_DMAP_N64) {
        // the persistent tile loop: as the DMA kernels (a two-stage ring spans
        // two tiles at most for any whole number of k-tiles)
        if (dt == Dtype::C64 || al != Algo::M4 || !g.a_kc || !g.b_kc) return false;
        if (g.K % 32) return false;
    }
    if (kid == K_DMA3_N64 || kid == K_DMA3_2) {
        // FP16 3M, the same operand conditions
        if (dt != Dtype::F16 || al != Algo::M3 || !g.a_kc || !g.b_kc) return false;
        if (g.K % 32) return false;
    }
    TileCfg t = tile_of(kid, dt, al);
    // whole 16-byte chunks along every chunked index (its low run starts at
    // bit 0 and holds at least one chunk), whole tiles along M and N
    const int64_t q = dt == Dtype::C64 ? 2 : 4;
    const int lq = dt == Dtype::C64 ? 1 : 2;
    if (g.K < q || g.K % q) return false;
    auto chunked = [&](const Seg &sg, int64_t ext) { return sg.ls == 0 && seg_low_run(sg, ext) >= lq; };
    if (!(g.a_kc ? chunked(g.ak, g.K) : chunked(g.am, g.M))) return false;
    if (!(g.b_kc ? chunked(g.bk, g.K) : chunked(g.bn, g.N))) return false;
    if (!(g.c_nc ? chunked(g.cn, g.N) : chunked(g.cm, g.M))) return false;
    if (dt != Dtype::C64 && g.K < 8) return false;
    if (g.M < t.BM || g.N < t.BN) return false;
    if (g.M % t.BM || g.N % t.BN) return false;
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
    int64_t nn = g.N < 16 ? g.N : 16;
    int64_t nch = (g.N + nn - 1) / nn;
    const Dtype dt = sizeof(W) == 8 ? Dtype::C64 : Dtype::F16;
    const int mode = thin_mode(dt, g);
    if (mode >= 0) {
        // about 4096 blocks in all (two rounds of eight per CU): each thread
        // then walks many row units, so the B columns a block stages in LDS
        // serve many rows
        const int64_t units = mode == 0 ? g.M : g.M / (16 / (int64_t)sizeof(W));
        const int64_t others = g.nb * nch * (int64_t)S;
        const int64_t gx = std::max<int64_t>(1, std::min<int64_t>({(units + 255) / 256, 2048, (4096 + others - 1) / others}));
        dim3 tg((unsigned)gx, (unsigned)(g.nb * nch), S);
#define THIN(NNV)                                                                                          \
    do {                                                                                                   \
        if (mode == 0) {                                                                                   \
            if (al == Algo::M3)                                                                            \
                hipLaunchKernelGGL((gemm_thin_kernel<W, NNV, 0, SCALE, true>), tg, dim3(256), 0, st,       \
                                   (const W *)A, (const W *)B, (W *)C, g, sc);                             \
            else                                                                                           \
                hipLaunchKernelGGL((gemm_thin_kernel<W, NNV, 0, SCALE, false>), tg, dim3(256), 0, st,      \
                                   (const W *)A, (const W *)B, (W *)C, g, sc);                             \
        } else {                                                                                           \
            if (al == Algo::M3)                                                                            \
                hipLaunchKernelGGL((gemm_thin_kernel<W, NNV, 1, SCALE, true>), tg, dim3(256), 0, st,       \
                                   (const W *)A, (const W *)B, (W *)C, g, sc);                             \
            else                                                                                           \
                hipLaunchKernelGGL((gemm_thin_kernel<W, NNV, 1, SCALE, false>), tg, dim3(256), 0, st,      \
                                   (const W *)A, (const W *)B, (W *)C, g, sc);                             \
        }                                                                                                  \
    } while (0)
        switch (nn) {
            case 1: THIN(1); break;
            case 2: THIN(2); break;
            case 4: THIN(4); break;
            case 8: THIN(8); break;
            default: THIN(16); break;
        }
#undef THIN
        return;
    }
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

template <bool BF, bool M3, int BM, int BN, int BK, int WM, int WN>
static void launch_h_cfg(const void *A, const void *B, void *C, const GemmShape &g, int S, const ScaleRefs &sc,
                         hipStream_t st) {
    using Tl = HTile<BF, M3, BM, BN, BK, WM, WN>;
    auto kern = gemm_mfma_h_kernel<BF, M3, BM, BN, BK, WM, WN>;
    static bool attr = false;
    if (!attr) {
        HIP_CHECK(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, Tl::LDS_BYTES));
        attr = true;
    }
    int64_t tiles = (g.M / BM) * (g.N / BN);
    dim3 grid((unsigned)tiles, (unsigned)(g.nb * g.split), S);
    hipLaunchKernelGGL(kern, grid, dim3(Tl::NT), Tl::LDS_BYTES, st, (const uint32_t *)A, (const uint32_t *)B,
                       (uint32_t *)C, g, sc);
}

template <bool BF, int BM, int BN, int WM, int WN, int STAGES, bool M3 = false>
static void launch_dma_cfg(const void *A, const void *B, void *C, const GemmShape &g, int S, const ScaleRefs &sc,
                           hipStream_t st) {
    using Tl = DTile<BM, BN, WM, WN, STAGES>;
    auto kern = gemm_dma_h_kernel<BF, M3, BM, BN, WM, WN, STAGES>;
    static bool attr = false;
    if (!attr) {
        HIP_CHECK(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, Tl::LDS_BYTES));
        attr = true;
    }
    int64_t tiles = (g.M / BM) * (g.N / BN);
    dim3 grid((unsigned)tiles, (unsigned)(g.nb * g.split), S);
    hipLaunchKernelGGL(kern, grid, dim3(Tl::NT), Tl::LDS_BYTES, st, (const uint32_t *)A, (const uint32_t *)B,
                       (uint32_t *)C, g, sc);
}

// One or two blocks per CU (as many as their rings fit in LDS), each walking
// its share of the launch's S x nb x tiles items (the grid a multiple of 8 so
// that the XCD patches line up).
template <bool BF, int BM, int BN, int WM, int WN, int STAGES>
static void launch_dmap_cfg(const void *A, const void *B, void *C, const GemmShape &g, int S, const ScaleRefs &sc,
                            hipStream_t st) {
    using Pt = PTile<BM, BN, WM, WN, STAGES>;
    auto kern = gemm_dmap_h_kernel<BF, BM, BN, WM, WN, STAGES>;
    static bool attr = false;
    if (!attr) {
        HIP_CHECK(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, Pt::LDS_BYTES));
        attr = true;
    }
    static int n_cu = 0;
    if (!n_cu) {
        int dev = 0;
        HIP_CHECK(hipGetDevice(&dev));
        HIP_CHECK(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
        if (n_cu < 1) n_cu = 1;
    }
    if (g.split != 1) TNC_THROW(TNC_EINVAL, "internal: the persistent tile loop takes no split-K");
    const int64_t total = (int64_t)S * g.nb * (g.M / BM) * (g.N / BN);
    int64_t G = std::min<int64_t>(total, (int64_t)n_cu * Pt::BLOCKS_PER_CU);
    if (G >= 8) G &= ~(int64_t)7;
    // a block's stage counter (items x k-tiles) runs in 32 bits
    if ((total + G - 1) / G * (g.K / Pt::BK) >= ((int64_t)1 << 31))
        TNC_THROW(TNC_EINVAL, "internal: too many tiles per block for the persistent tile loop");
    hipLaunchKernelGGL(kern, dim3((unsigned)G), dim3(Pt::NT), Pt::LDS_BYTES, st, (const uint32_t *)A,
                       (const uint32_t *)B, (uint32_t *)C, g, sc, S);
}

template <bool BF>
static void launch_h(int kid, Algo al, const void *A, const void *B, void *C, const GemmShape &g, int S,
                     const ScaleRefs &sc, hipStream_t st) {
    if (kid == K_DMAP_2) return launch_dmap_cfg<BF, 128, 128, 2, 2, 2>(A, B, C, g, S, sc, st);
    if (kid == K_DMAP_N64) return launch_dmap_cfg<BF, 256, 64, 2, 2, 2>(A, B, C, g, S, sc, st);
    if (kid == K_THINM) {
        // about 4096 blocks in all; each wave walks 64-row passes
        const int64_t units = g.M / 64, others = g.nb * (int64_t)S;
        const int64_t gx = std::max<int64_t>(1, std::min<int64_t>((units + 3) / 4, (4096 + others - 1) / others));
        dim3 grid((unsigned)gx, (unsigned)g.nb, S);
        auto args = [&](auto kern) {
            hipLaunchKernelGGL(kern, grid, dim3(256), 0, st, (const uint32_t *)A, (const uint32_t *)B, (uint32_t *)C, g,
                               sc);
        };
        const bool short_k = g.K <= 16;   // the double-buffered A of a pass fits few registers
        if (!g.a_kc) {
            if (g.N <= 8) args(gemm_thinm_kernel<BF, 1, 2, false>);
            else if (g.N <= 16) args(gemm_thinm_kernel<BF, 2, 2, false>);
            else args(gemm_thinm_kernel<BF, 4, 2, false>);
        } else if (g.N == 32) {
            args(gemm_thinm_kernel<BF, 4, 2, true>);
        } else if (g.N <= 8) {
            if (short_k) args(gemm_thinm_kernel<BF, 1, 2, true>);
            else args(gemm_thinm_kernel<BF, 1, 8, true>);
        } else {
            if (short_k) args(gemm_thinm_kernel<BF, 2, 2, true>);
            else args(gemm_thinm_kernel<BF, 2, 8, true>);
        }
        return;
    }
    if (kid == K_DMA_4) return launch_dma_cfg<BF, 256, 128, 2, 2, 3>(A, B, C, g, S, sc, st);
    if (kid == K_DMA_8) return launch_dma_cfg<BF, 256, 128, 4, 2, 3>(A, B, C, g, S, sc, st);
    if (kid == K_DMA_8W) return launch_dma_cfg<BF, 256, 128, 2, 4, 3>(A, B, C, g, S, sc, st);
    if (kid == K_DMA_2) return launch_dma_cfg<BF, 128, 128, 2, 2, 2>(A, B, C, g, S, sc, st);
    if (kid == K_DMA_N64) return launch_dma_cfg<BF, 256, 64, 4, 2, 2>(A, B, C, g, S, sc, st);
    if (kid == K_DMA_N32) return launch_dma_cfg<BF, 256, 32, 4, 1, 2>(A, B, C, g, S, sc, st);
    if constexpr (!BF) {
        if (kid == K_DMA3_N64) return launch_dma_cfg<false, 256, 64, 4, 2, 2, true>(A, B, C, g, S, sc, st);
        if (kid == K_DMA3_2) return launch_dma_cfg<false, 128, 128, 2, 2, 2, true>(A, B, C, g, S, sc, st);
    }
    if (al == Algo::M4) {
        switch (kid) {
            case K_MFMA_S: launch_h_cfg<BF, false, 64, 16, 32, 2, 1>(A, B, C, g, S, sc, st); break;
            case K_MFMA_M: launch_h_cfg<BF, false, 128, 32, 32, 2, 2>(A, B, C, g, S, sc, st); break;
            case K_MFMA_L: launch_h_cfg<BF, false, 128, 64, 32, 2, 2>(A, B, C, g, S, sc, st); break;
            case K_MFMA_W: launch_h_cfg<BF, false, 256, 16, 32, 4, 1>(A, B, C, g, S, sc, st); break;
            case K_MFMA_XL: launch_h_cfg<BF, false, 256, 128, 32, 4, 2>(A, B, C, g, S, sc, st); break;
            case K_MFMA_L2: launch_h_cfg<BF, false, 128, 128, 32, 2, 2>(A, B, C, g, S, sc, st); break;
        }
    } else {
        switch (kid) {
            case K_MFMA_S: launch_h_cfg<BF, true, 64, 32, 32, 2, 1>(A, B, C, g, S, sc, st); break;
            case K_MFMA_M: launch_h_cfg<BF, true, 128, 64, 32, 2, 2>(A, B, C, g, S, sc, st); break;
            case K_MFMA_L: launch_h_cfg<BF, true, 128, 128, 32, 2, 2>(A, B, C, g, S, sc, st); break;
            case K_MFMA_W: launch_h_cfg<BF, true, 256, 32, 32, 4, 1>(A, B, C, g, S, sc, st); break;
            case K_MFMA_XL: launch_h_cfg<BF, true, 256, 64, 32, 4, 1>(A, B, C, g, S, sc, st); break;
            case K_MFMA_L2: launch_h_cfg<BF, true, 128, 32, 32, 4, 1>(A, B, C, g, S, sc, st); break;
        }
    }
}

template <int BM, int BN, int BK, int WM, int WN>
static void launch_c_cfg(const void *A, const void *B, void *C, const GemmShape &g, int S, hipStream_t st) {
    using Tl = CTile<BM, BN, BK, WM, WN>;
    auto kern = gemm_mfma_c64_kernel<BM, BN, BK, WM, WN>;
    static bool attr = false;
    if (!attr) {
        HIP_CHECK(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, Tl::LDS_BYTES));
        attr = true;
    }
    int64_t tiles = (g.M / BM) * (g.N / BN);
    dim3 grid((unsigned)tiles, (unsigned)(g.nb * g.split), S);
    hipLaunchKernelGGL(kern, grid, dim3(Tl::NT), Tl::LDS_BYTES, st, (const float2 *)A, (const float2 *)B,
                       (float2 *)C, g);
}

static void launch_c64(int kid, const void *A, const void *B, void *C, const GemmShape &g, int S, hipStream_t st) {
    switch (kid) {
        case K_MFMA_S: launch_c_cfg<64, 16, 16, 2, 1>(A, B, C, g, S, st); break;
        case K_MFMA_M: launch_c_cfg<128, 16, 16, 4, 1>(A, B, C, g, S, st); break;
        case K_MFMA_L: launch_c_cfg<128, 32, 16, 2, 2>(A, B, C, g, S, st); break;
        case K_MFMA_W: launch_c_cfg<256, 16, 16, 4, 1>(A, B, C, g, S, st); break;
        case K_MFMA_XL: launch_c_cfg<128, 64, 16, 2, 2>(A, B, C, g, S, st); break;
        case K_MFMA_L2: launch_c_cfg<256, 32, 16, 2, 2>(A, B, C, g, S, st); break;
    }
}

int64_t splitk_factor(int kid, Dtype dt, Algo al, const GemmShape &g, int S) {
    if (kid < K_MFMA_S || kid >= K_COUNT || !gemm_supported(kid, dt, al, g)) return 1;
    if (kid == K_DMAP_2 || kid == K_DMAP_N64 || kid == K_THINM) return 1;
    TileCfg t = tile_of(kid, dt, al);
    const int64_t bk = dt == Dtype::C64 ? 16 : 32;
    const int64_t blocks = (g.M / t.BM) * (g.N / t.BN) * g.nb * (int64_t)S;
    const int64_t ktiles = g.K / bk;
    if (blocks >= 512 || ktiles < 16) return 1;
    int64_t p = 1;
    while (p * 2 * blocks <= 1024 && p * 2 <= ktiles / 4 && g.nb * p * 2 <= 65535) p *= 2;
    return p;
}

int64_t splitk_bytes(int kid, Dtype dt, Algo al, const GemmShape &g, int S) {
    int64_t p = splitk_factor(kid, dt, al, g, S);
    return p > 1 ? p * (int64_t)S * g.nb * g.M * g.N * (int64_t)sizeof(float2) : 0;
}

void launch_gemm(int kid, Dtype dt, Algo al, const void *A, const void *B, void *C, const GemmShape &g_in, int S,
                 const ScaleRefs *sc, hipStream_t st) {
    if (S <= 0) return;
    if (!gemm_supported(kid, dt, al, g_in)) TNC_THROW(TNC_EINVAL, std::string("kernel ") + kernel_name(kid) + " cannot run this shape");
    {
        // The batch runs on grid.y, times the column chunks of the VALU
        // kernels or the split-K parts (at most 64 when it applies); a
        // batch too large for that (sparse-state steps have one per block)
        // goes out in several launches.
        const int64_t fac = std::max<int64_t>(64, (g_in.N + 15) / 16);
        if (g_in.nb * fac > 65535) {
            const int64_t chunk = std::max<int64_t>(1, 65535 / fac);
            const int64_t es = elem_bytes(dt);
            for (int64_t b0 = 0; b0 < g_in.nb; b0 += chunk) {
                GemmShape g = g_in;
                g.nb = std::min(chunk, g_in.nb - b0);
                const uint8_t *pa = (const uint8_t *)A, *pb = (const uint8_t *)B;
                if (g.ia) g.ia += b0;
                else pa += b0 * g.bA * es;
                if (g.ib) g.ib += b0;
                else pb += b0 * g.bB * es;
                launch_gemm(kid, dt, al, pa, pb, (uint8_t *)C + b0 * g.bC * es, g, S, sc, st);
            }
            return;
        }
    }
    ScaleRefs s = sc ? *sc : ScaleRefs{};
    if (dt != Dtype::C64 && !sc) TNC_THROW(TNC_EINVAL, "16-bit forms need scale bookkeeping");
    s.flag_above = dt == Dtype::F16 ? kF16FlagAbove : 3.0e38f;
    GemmShape g = g_in;
    const int64_t split_s = g.split_slices > 0 ? g.split_slices : S;
    if (S > split_s) TNC_THROW(TNC_EINVAL, "launch covers more slices than its split-K buffer was sized for");
    g.split = g.part ? splitk_factor(kid, dt, al, g, (int)split_s) : 1;
    if (g.split > 1) {
        // the parts of this launch: split x S slices x batch x M x N (re, im) pairs
        const int64_t need = g.split * (int64_t)S * g.nb * g.M * g.N * (int64_t)sizeof(float2);
        if (need > g.part_cap)
            TNC_THROW(TNC_EINVAL, "internal: split-K partial sums need " + std::to_string(need) + " bytes, buffer has " +
                                      std::to_string(g.part_cap));
    }
    if (g.split > 1) {
        if (dt == Dtype::C64)
            launch_c64(kid, A, B, C, g, S, st);
        else if (dt == Dtype::F16)
            launch_h<false>(kid, al, A, B, C, g, S, s, st);
        else
            launch_h<true>(kid, al, A, B, C, g, S, s, st);
        HIP_CHECK(hipGetLastError());
        const int64_t MN = g.M * g.N;
        dim3 grid((unsigned)std::min<int64_t>((MN + 255) / 256, 4096), (unsigned)g.nb, S);
        if (dt == Dtype::C64)
            hipLaunchKernelGGL((splitk_reduce_kernel<uint2, false>), grid, dim3(256), 0, st, (uint2 *)C, g, s);
        else if (dt == Dtype::F16)
            hipLaunchKernelGGL((splitk_reduce_kernel<HalfWord, true>), grid, dim3(256), 0, st, (HalfWord *)C, g, s);
        else
            hipLaunchKernelGGL((splitk_reduce_kernel<Bf16Word, true>), grid, dim3(256), 0, st, (Bf16Word *)C, g, s);
        HIP_CHECK(hipGetLastError());
        return;
    }
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
        launch_h<false>(kid, al, A, B, C, g, S, s, st);
    } else {
        launch_h<true>(kid, al, A, B, C, g, S, s, st);
    }
    HIP_CHECK(hipGetLastError());
}

}  // namespace tnc
