// Host planner: turns (network, path, sliced labels, open qubits) into the
// steps one slice runs, the memory layout of every tensor, and the arena.
#pragma once

#include <map>
#include <memory>
#include <vector>

#include "common.h"

namespace tnc {

struct TensorRec {
    std::vector<int> labels;    // storage order, first = slowest
    bool dep = false;           // depends on the slice id
    bool inner = false;         // holds a recomputed label in its sub-tree (computed once per pass)
    // sparse state: the qubits whose output labels this tensor holds, and the
    // number of their distinct value combinations among the requested
    // bitstrings; the tensor is stored as nd dense blocks [d][labels]
    uint64_t sp_mask = 0;
    int64_t nd = 1;
    bool leaf = false;
    int producer = -1;          // step index, or -1 for an input tensor
    int consumer = -1;          // step index, or -1 for the root
    int64_t off = -1;           // arena byte offset (slice 0)
    int rank() const { return (int)labels.size(); }
};

struct StepRec {
    int x = -1, y = -1, z = -1;       // operand and result tensor ids (SSA)
    int a = -1, b = -1;               // tensor ids used as A (large side) and B
    std::vector<int> beta, m, n, k;   // label groups, each in storage order
    bool perm_a = false, perm_b = false;
    int64_t scr_a = -1, scr_b = -1;   // arena offsets of the permuted operands
    std::vector<int> a_from, b_from;  // operand orders before the permute
    int64_t M = 1, N = 1, K = 1, nb = 1;
    int a_kc = 1, b_kc = 1, c_nc = 1;  // operand / result chunk direction (see GemmShape)
    Seg am, ak, bn, bk, cm, cn;        // where each GEMM index lives in A, B and the result
    bool hoist_a = false, hoist_b = false;   // permute of an invariant operand, done once per call
    bool dep = false;
    bool inner = false;               // runs once per recomputation pass
    // sparse state: which dense block of A and B each result block d reads:
    // mode 0 the same d, 1 block 0 for every d, 2 the index array
    int a_mode = 0, b_mode = 0;
    std::vector<int32_t> a_idx, b_idx;
    // second indexing scheme (the padded two-dimensional index): when many
    // result blocks read the same A block, A is used as stored, one GEMM per
    // A block against B_P, the B blocks of its mr result blocks side by side
    // (index -1: a zero block), and C is taken out of the product C_P;
    // A blocks are processed `chunk` at a time through scratch buffers
    int scheme = 1;
    int64_t mr = 1, chunk = 0;
    std::vector<int32_t> bp_idx;      // per (A block, r): the B block, or -1
    std::vector<int32_t> cp_idx;      // per result block: its block of C_P (A block * mr + r)
    int64_t scr_bp = -1, scr_cp = -1; // arena offsets of the B_P and C_P chunks
    int kernel = K_NAIVE;
    double flops = 0;                 // per slice (or once, if invariant)
    double bytes = 0;                 // GEMM bytes per slice
    double perm_bytes = 0;            // permute bytes per slice
};

struct Analysis {
    std::vector<TensorRec> tensors;   // leaves 0..n-1, then step results
    std::vector<StepRec> steps;
    std::vector<int> fixed;           // per label: -1 free, 0 sliced, 1 closed output
    std::vector<int> slice_bit;       // per label: bit of the slice id (sliced labels)
    std::vector<int> open_qubit_of_label;
    int root = -1;
    int n_sliced = 0;                 // sliced labels (slice ids 0 .. 2^n_sliced - 1)
    int n_recompute = 0;              // recomputed labels: 2^n_recompute passes per slice
    // sparse state (uncorrelated bitstrings): every output label is replaced
    // by a block index over the distinct values of the tensor's qubits
    bool sparse = false;
    std::vector<std::vector<uint64_t>> leaf_keys;   // per input tensor: its blocks' qubit values
    std::vector<int32_t> root_map;                  // per requested bitstring: its block of the root
    int max_rank = 0;
    Dtype dt = Dtype::C64;
    Algo al = Algo::M4;
};

// Validate and analyse; throws tnc::Error.  Recomputed labels (paper Sec.
// 3.4.1) are fixed like sliced ones, but per pass: their values are the slice
// id bits n_sliced + j of a pass, and the steps whose sub-tree holds one of
// them (the suffix) run once per pass while the rest (the prefix) run once
// per slice.
//
// Sparse state (paper Sec. 3.4.2): with `sparse_bits`, the amplitudes of
// those n_sparse bitstrings are computed together whatever bits they share.
// Every output label leaves the dense labels; a tensor holding the output
// labels of qubit set Q is stored as one dense block per distinct value of
// the bitstrings restricted to Q, and a step forms each result block from the
// operand blocks with the matching values (a gathered multi-pair GEMM).
Analysis analyze(const Network &net, int n_steps, const int32_t *ssa, int n_sliced, const int32_t *sliced,
                 int n_open, const int32_t *open_q, tnc_precision prec, int n_recompute = 0,
                 const int32_t *recompute = nullptr, int64_t n_sparse = 0, const uint64_t *sparse_bits = nullptr);

// Execution class of a tensor or step: 0 slice-invariant (once per call),
// 1 slice prefix (once per slice group), 2 recomputed suffix (once per pass).
inline int exec_class(bool dep, bool inner) { return !dep ? 0 : (inner ? 2 : 1); }

// Byte offsets of every tensor and scratch buffer for S slices in flight;
// returns the arena peak in bytes.
int64_t plan_memory(Analysis &an, int S, bool assign);

// Segment of the GEMM index whose labels are `idx` (most significant first)
// in a tensor stored in `order`; false if they are not in at most two runs.
bool derive_seg(const std::vector<int> &order, const std::vector<int> &idx, Seg &out);

// GEMM descriptor of a step (slice strides zero).
GemmShape step_gemm(const StepRec &st);
// The GEMM the step actually launches: step_gemm, or for a step on the
// second sparse-state scheme the per-A-block product with B_P (nb = chunk).
GemmShape step_gemm_exec(const StepRec &st);

// Default kernel choice for a step shape.
int choose_kernel(Dtype dt, Algo al, const GemmShape &g);

PermuteDesc make_permute(const std::vector<int> &from, const std::vector<int> &to);

void fill_stats(const Analysis &an, tnc_plan_stats &st);

// Host FP64 pre-contraction (simplify.cpp): the steps of a path whose operands
// are input tensors or results of such steps, one of them of rank <= 2, and
// whose result is no larger than the larger operand and has at most
// `max_rank` labels (fixed labels included), are contracted on the host in
// complex128; `net` and `ssa` are the device's leaves and path.
constexpr int kDefaultHostRank = 10;
constexpr int kMaxHostRank = 14;
struct Simplified {
    Network net;
    std::vector<int32_t> ssa;
    std::vector<int> plan_step_of;   // per step of the given path: device step, or -1 (host)
    int host_steps = 0;
};
// rank cap of host steps: TNC_HOST_RANK if set (0 switches the pass off), else kDefaultHostRank
int host_rank_cap();
Simplified presimplify(const Network &net, int n_steps, const int32_t *ssa, int n_sliced, const int32_t *sliced,
                       int n_open, const int32_t *open_q, int max_rank, int n_recompute = 0,
                       const int32_t *recompute = nullptr);

}  // namespace tnc
