// Internal declarations shared by the host planner, the executor and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/tnc.h"

namespace tnc {

// ------------------------------------------------------------------ errors
void set_error(const std::string &msg);

struct Error {
    int code;
    std::string msg;
};

#define TNC_THROW(code, msg)                                  \
    do {                                                      \
        throw ::tnc::Error{(code), std::string(msg)};         \
    } while (0)

#define HIP_CHECK(expr)                                                                        \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                  \
            throw ::tnc::Error{TNC_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)}; \
    } while (0)

// ------------------------------------------------------------------ element kinds
enum class Dtype : int { C64 = 0, F16 = 1, BF16 = 2 };
enum class Algo : int { M4 = 0, M3 = 1 };

inline Dtype dtype_of(tnc_precision p) {
    switch (p) {
        case TNC_C64: return Dtype::C64;
        case TNC_F16_4M:
        case TNC_F16_3M: return Dtype::F16;
        default: return Dtype::BF16;
    }
}
inline Algo algo_of(tnc_precision p) {
    return (p == TNC_F16_3M || p == TNC_BF16_3M) ? Algo::M3 : Algo::M4;
}
inline int elem_bytes(Dtype d) { return d == Dtype::C64 ? 8 : 4; }

// ------------------------------------------------------------------ network (host)
struct Network {
    int n_tensors = 0;
    std::vector<std::vector<int>> labels;      // per tensor, first label slowest
    std::vector<std::vector<double>> data;     // per tensor, interleaved complex128
    int n_qubits = 0;
    std::vector<int> output_labels;            // per qubit
    int n_labels = 0;                          // 1 + max label id
    bool hyperedges = false;                   // some label is held by three or more tensors
};

// ------------------------------------------------------------------ kernel launch descriptors

// Bit permutation of a batch of tensors.  Destination element j of slice s
// reads source element  src_base(s) + sum_b bit_b(j) * src_stride[b].
constexpr int kMaxRank = 48;
struct PermuteDesc {
    int rank;                   // destination rank
    int64_t src_stride[kMaxRank];  // element stride in the source for destination bit b (bit 0 = fastest)
};

// Placement of one GEMM index in memory.  The index's labels lie in at most
// two runs of consecutive bits: x = (hi << l) | lo with lo < 2^l, and
//     offset(x) = (hi << hs) + (lo << ls)      (in entries).
// A single run has l = 62 (hi is always 0).
struct Seg {
    int32_t l = 62, ls = 0, hs = 0;
};
__host__ __device__ inline int64_t seg_offset(const Seg &s, int64_t x) {
    return ((x >> s.l) << s.hs) + ((x & (((int64_t)1 << s.l) - 1)) << s.ls);
}
// length of the run that holds index bit 0 (the run chunks are taken along)
inline int seg_low_run(const Seg &s, int64_t extent) {
    int b = 0;
    while (((int64_t)1 << (b + 1)) <= extent) b++;
    return s.l < b ? s.l : b;
}

// Everything one step needs at run time.  Sizes are complex entries.
// Chunk direction: A is read in 16-byte chunks along k (a_kc = 1) or along m;
// B along k (b_kc = 1) or along n; C is written along n (c_nc = 1) or along m.
// Where each index lives is given by its Seg (am, ak, bn, bk, cm, cn); the
// chunked index's low run must start at bit 0 (ls = 0).
struct GemmShape {
    int64_t M, N, K, nb;        // rows, cols, reduced, inner batch
    int64_t sA, sB, sC;         // slice strides (0 = shared by every slice)
    int64_t bA, bB, bC;         // inner-batch strides
    int a_kc = 1, b_kc = 1, c_nc = 1, pad_ = 0;
    Seg am, ak, bn, bk, cm, cn;
    // split-K: the reduced range is cut into `split` parts; each part's FP32
    // partial result goes to part[((s * nb + b) * split + p)][m][n] (re, im
    // pairs) and a second kernel sums the parts in order
    int64_t split = 1;
    float2 *part = nullptr;
    int64_t part_cap = 0;       // bytes available at `part` (checked on the host before a split launch)
    // the split factor is chosen for this many slices per launch, the count
    // the partial buffer was sized for (0: the launch's own count); a launch
    // over fewer slices keeps that factor, so it never needs more buffer
    int64_t split_slices = 0;
    // sparse state: batch b reads block ia[b] of A and ib[b] of B (device
    // arrays; NULL = block b); C's block is always b
    const int32_t *ia = nullptr, *ib = nullptr;
};
__host__ __device__ inline int64_t a_block(const GemmShape &g, int64_t b) { return g.ia ? (int64_t)g.ia[b] : b; }
__host__ __device__ inline int64_t b_block(const GemmShape &g, int64_t b) { return g.ib ? (int64_t)g.ib[b] : b; }

// Scale bookkeeping of the 16-bit forms, per tensor and slice.
struct ScaleRefs {
    const uint32_t *maxA; int mA;   // max |re|,|im| (float bits); index s*mA
    const uint32_t *maxB; int mB;
    uint32_t *maxC;                 // written with atomicMax, index s
    const double *expA; int eA;     // power-of-two exponents, index s*eA
    const double *expB; int eB;
    double *expC;                   // index s
    int *shift;                     // per slice (written), may be null
    const int *growth;              // device int: expected log2 growth of this step
    uint32_t *flag;                 // set nonzero on range overflow
    // a stored maximum above this flags the step (set by launch_gemm from the
    // storage type): FP16 results must stay below half the FP16 range so that
    // a consumer's 3M sum plane (re + im) stays finite
    float flag_above = 3.0e38f;
};

// Target exponent of the largest stored 16-bit component (see device_util.h).
constexpr int kTargetLog2Host = 13;
// Largest FP16 stored component a step may leave: half of 65504, so that the
// sum re + im a 3M consumer forms is at most the largest finite FP16 value.
constexpr float kF16FlagAbove = 32752.0f;

// Exchange codec: the group size a kind uses (group 0 = the kind's default);
// throws TNC_EINVAL for an unknown kind or group size.
int codec_group(int32_t kind, int32_t group);
// Partials of the codec's whole-tensor min/max pass (one float2 per block).
constexpr int kQuantPartials = 512;

// Kernel variant ids (autotuned per step).
enum KernelId : int {
    K_NAIVE = 0,      // thread per output entry; any shape
    K_SKINNY_N = 1,   // row per thread, N <= 16, VALU
    K_MFMA_S = 2,     // matrix-core tiles (rows x complex cols; see tile_of)
    K_MFMA_M = 3,
    K_MFMA_L = 4,
    K_MFMA_W = 5,     // tall thin tile
    K_MFMA_XL = 6,    // large tiles for compute-bound steps
    K_MFMA_L2 = 7,
    K_DMA_4 = 8,      // 16-bit 4M, operands streamed into LDS by DMA; 4 waves
    K_DMA_8 = 9,      // the same with 8 waves (4 x 2)
    K_DMA_8W = 10,    // 8 waves as 2 x 4 (wider wave tiles along n)
    K_DMA_2 = 11,     // 128 x 128 tile, two stages: two blocks per CU (short k)
    K_DMA_N64 = 12,   // 256 x 64 tile, two stages, two blocks per CU (narrow n, HBM-bound)
    K_DMA_N32 = 13,   // 256 x 32 tile, the same
    K_DMA3_N64 = 14,  // FP16 3M from the DMA ring: 256 x 64 tile, two stages, two blocks per CU
    K_DMA3_2 = 15,    // FP16 3M, 128 x 128 tile, two stages, one wave per SIMD
    K_DMAP_2 = 16,    // 16-bit 4M, 128 x 128 tile, persistent over the launch's tiles, two stages
    K_THINM = 17,     // 16-bit 4M thin steps (N = 4 .. 32) on 16 x 16 x 16 matrix-core tiles
    K_DMAP_N64 = 18,  // the same on a 256 x 64 tile (2 x 2 waves, two blocks per CU): HBM-bound narrow steps
    K_COUNT = 19
};
const char *kernel_name(int k);
// Segments of the plain layouts ([m][k] or [k][m] etc., as the chunk flags
// say); M, N, K must be powers of two.
void set_plain_segs(GemmShape &g);

// Launch wrappers (kernels.hip).
void launch_permute(Dtype dt, const void *src, void *dst, const PermuteDesc &d, int64_t n_out,
                    int S, int64_t src_slice_stride, const int64_t *d_slice_offsets,
                    int64_t dst_slice_stride, hipStream_t st);
bool gemm_supported(int kid, Dtype dt, Algo al, const GemmShape &g);
// split-K factor the launch of kernel kid would use for S slices (1 = none),
// and the partial-result bytes it needs
int64_t splitk_factor(int kid, Dtype dt, Algo al, const GemmShape &g, int S);
int64_t splitk_bytes(int kid, Dtype dt, Algo al, const GemmShape &g, int S);
void launch_gemm(int kid, Dtype dt, Algo al, const void *A, const void *B, void *C,
                 const GemmShape &g, int S, const ScaleRefs *sc, hipStream_t st);
void launch_convert_c128(const double *src, int64_t n, Dtype dt, void *dst, hipStream_t st);
// Sparse state: destination block j (of `block` entries, per slice) takes
// source block idx[j] - lo when that lies in [0, hi - lo), else is zeroed
// (fill) or left as it is.
void launch_block_copy(Dtype dt, const void *src, int64_t src_ss, void *dst, int64_t dst_ss, const int32_t *idx,
                       int64_t n_blocks, int64_t lo, int64_t hi, int64_t block, int S, bool fill, hipStream_t st);
void launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t st);
void launch_fill_f64(double *p, double v, int64_t n, hipStream_t st);
void launch_fill_random(Dtype dt, void *p, int64_t n_words, uint32_t seed, hipStream_t st);
void launch_tensor_max(Dtype dt, const void *x, int64_t n, int S, int64_t slice_stride,
                       uint32_t *max_out, hipStream_t st);
void launch_accumulate(Dtype dt, const void *R, int rank, int S, int64_t slice_stride,
                       const double *expR, int n_exp_stride, int64_t nbits, const uint64_t *d_bits,
                       const int *d_qubit_of_bit, double *acc, hipStream_t st, const int32_t *d_map = nullptr);

// Bits of an LDS-tiled permute.  The tile is the union T of the w lowest
// destination bits and the destination bits that hold the w lowest source
// bits, grown to nt_max bits (or the whole rank) with further low destination
// and source bits in turn; src_order lists T's destination bits by source position, dst_order by
// destination position, lds_bit[i] is the position of src_order[i] in
// dst_order; rest lists the destination bits outside T.
struct TileBits {
    int nt;
    int src_order[16];
    int dst_order[16];
    int lds_bit[16];
    int rest[kMaxRank];
    int n_rest;
};
bool plan_tile_bits(const PermuteDesc &d, int lw, int nt_max, TileBits &tb);
constexpr int kPermTileBits = 12;   // 4096 entries per LDS tile

// Slice selection of one input tensor (see gather_leaves_kernel).
constexpr int kMaxLeafRank = 16;
struct LeafDesc {
    int64_t src_off;            // element offset of the full tensor in the leaf buffer
    int64_t closed_off;         // element offset from the closed-qubit values of this call
    int64_t dst_byte_off;       // arena byte offset of slice 0
    int64_t dst_slice_stride;   // elements between consecutive slices
    int64_t stride[kMaxLeafRank];        // source stride of destination bit b
    int64_t slice_stride[kMaxLeafRank];  // source stride of sliced label j
    int slice_bit[kMaxLeafRank];         // bit of the slice id that sets sliced label j
    int rank, n_sliced, n_slices, max_slot, slot_stride, pad_;
    // sparse state: nd blocks, block d taken at element offset spoff[sp_base + d]
    int64_t sp_base;
    int nd, pad2_;
};
void launch_gather_leaves_impl(Dtype dt, int n_leaves, const LeafDesc *d_desc, const int64_t *d_params,
                               const void *leafdata, uint8_t *arena, uint32_t *maxw, double *expw,
                               int64_t group_base, int S, hipStream_t st, const int64_t *spoff = nullptr,
                               int nd_max = 1);

}  // namespace tnc
