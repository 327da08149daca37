// Engine objects behind the C handles.
#pragma once

#include <map>
#include <tuple>
#include <vector>

#include "common.h"
#include "planner.h"

struct tnc_network {
    tnc::Network net;
};

namespace tnc {
struct Mlp;   // learned step-cost model (mlp.hip)
void mlp_free(Mlp *m);
}

namespace tnc {
void launch_quantize(int kind, int64_t n, int group, const float *x, void *codes, float *scales, float *zeros,
                     float2 *part, hipStream_t st);
void launch_dequantize(int kind, int64_t n, int group, const void *codes, const float *scales, const float *zeros,
                       float *x, hipStream_t st);
}  // namespace tnc

struct tnc_ctx {
    int device = 0;
    uint8_t *ws = nullptr;
    size_t ws_bytes = 0;
    hipStream_t stream = nullptr;
    uint8_t *small = nullptr;          // 4 KiB of device scratch owned by the context
    tnc::Mlp *mlp = nullptr;
};

struct tnc_plan {
    tnc_ctx *ctx = nullptr;
    tnc::Analysis an;
    std::vector<int> plan_step_of;     // per step of the caller's path: device step, or -1 (run on the host)
    int host_steps = 0;                // steps pre-contracted on the host in FP64
    int S = 1;                         // slices in flight
    int64_t peak = 0;
    int nT = 0;                        // input tensors
    int n_qubits = 0;
    std::vector<int> output_labels;
    std::vector<int> closed_qubits;    // qubits whose output label is fixed per call
    std::vector<std::vector<int>> leaf_orig_labels;   // input labels as given
    // device buffers owned by the plan
    void *d_leafdata = nullptr;
    tnc::LeafDesc *d_desc = nullptr;   // invariant descriptors first, then dependent
    std::vector<tnc::LeafDesc> h_desc;
    int n_inv_leaves = 0, n_dep_leaves = 0;   // dependent = prefix leaves, then recomputed ones
    int n_inner_leaves = 0;                   // the recomputed (per-pass) leaves among the dependent ones
    std::vector<int> desc_of_leaf;
    uint32_t *d_maxw = nullptr;
    double *d_expw = nullptr;
    int *d_shift = nullptr;
    int *d_growth = nullptr;
    uint32_t *d_flags = nullptr;
    int64_t *d_params = nullptr;
    uint64_t *d_bits = nullptr;
    int64_t bits_cap = 0;
    double *d_acc = nullptr;
    int *d_qob = nullptr;
    float2 *d_part = nullptr;            // split-K partial sums (largest need over the steps)
    int64_t part_bytes = 0;              // size of d_part
    std::vector<int> h_growth;
    std::vector<int64_t> closed_state;  // closed_off per leaf last uploaded
    // graph cache: (slices, bitstrings, bits pointer) -> executable graph
    std::map<std::tuple<int64_t, int64_t, const void *>, hipGraphExec_t> graphs;
    bool use_graph = true;
    double tune_seconds = 0;
    bool timing = false;
    std::vector<double> step_ms, perm_ms;
    std::vector<int> step_launches;
    // sparse state: leaf block offsets, per-step block index arrays (one
    // buffer; offsets per step, -1 = none), the root block of each requested
    // bitstring, and the requested bitstrings themselves
    int64_t *d_spoff = nullptr;
    int nd_max = 1;
    int32_t *d_idx = nullptr;
    std::vector<int64_t> a_idx_off, b_idx_off, bp_idx_off, cp_idx_off;
    int32_t *d_map = nullptr;
    std::vector<uint64_t> sparse_bits;
    // exchange codec round trip applied to one step's result (complex64 plans)
    int codec_step = -1, codec_kind = 0, codec_group = 0;
    void *d_codes = nullptr;
    float *d_qscale = nullptr, *d_qzero = nullptr;
};
