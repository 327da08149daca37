/*
 * tnc -- sliced tensor-network amplitudes on one AMD Instinct MI355X (gfx950).
 *
 * The problem statement follows the paper (Fu et al., "Achieving Energetic
 * Superiority Through System-Level Quantum Circuit Simulation"):
 *   - a sub-network is a list of initial tensors plus a contraction path given
 *     as a sequence of pairwise einsums (Sec. 3.1, Alg. 1 "init");
 *   - slicing fixes the values of chosen labels; every assignment is an
 *     independent sub-network and the full result is the sum over all of them
 *     (Sec. 3.1, three-level scheme, global level);
 *   - the output is a set of bitstring amplitudes; bitstrings that share some
 *     qubit values form a correlated subspace whose open qubits are computed
 *     together (Sec. 1 and 2.3, correlated samples);
 *   - each pairwise contraction is an index permutation followed by a GEMM
 *     (Sec. 3.4.2), which is a pure GEMM exactly when the reduced labels are
 *     the intersection of the two operands' labels (Sec. 3.3, Eqs.
 *     contraction and remain_idx);
 *   - complex-half storage multiplies through one real GEMM whose small
 *     operand is padded to [B(re,-im), B(im,re)] (Sec. 3.3, Eq. eq_modified2).
 *
 * Conventions shared by every call:
 *   - Every label has dimension 2.  A tensor of rank r has 2^r complex entries.
 *   - Dense data is row-major with the first label slowest.
 *   - A bitstring is a uint64 whose bit q is the value of qubit q.
 *   - Return value: TNC_OK (0) or a negative TNC_E* code; tnc_last_error()
 *     then returns a message (thread-local, valid until the next call on the
 *     same thread).
 *   - Handles are owned by the caller and released with the matching
 *     *_destroy call.  A context and everything made from it is used from one
 *     host thread at a time.
 *   - Device pointers are HIP device addresses on the context's device; host
 *     pointers are ordinary host memory.  Every pointer argument marked "host"
 *     is read or written synchronously before the call returns.
 */
#ifndef TNC_H
#define TNC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    TNC_OK = 0,
    TNC_EINVAL = -1,       /* malformed argument (shape, label, path, range)      */
    TNC_ENOMEM = -2,       /* per-slice working set exceeds the workspace          */
    TNC_EDEVICE = -3,      /* a HIP runtime call failed                             */
    TNC_EOVERFLOW = -4,    /* FP16 range exceeded after the bounded rescale replays */
    TNC_EUNSUPPORTED = -5  /* valid input this engine does not handle               */
};

/* Arithmetic of the contraction steps.
 *   C64     : complex64 storage, FP32 matrix-core GEMM (4M as one real GEMM).
 *   F16_4M  : complex FP16 storage (re,im interleaved, 4 bytes per entry),
 *             one real FP16 GEMM with the padded small operand, FP32 accumulate.
 *   F16_3M  : complex FP16 storage, three real FP16 GEMMs (Gauss form:
 *             T1 = Ar Br, T2 = Ai Bi, T3 = (Ar+Ai)(Br+Bi); Cr = T1-T2,
 *             Ci = T3-T1-T2), FP32 accumulate.
 *   BF16_4M / BF16_3M : the same with bfloat16 storage.
 * The 16-bit forms keep a power-of-two exponent per tensor and slice (FP64 on
 * the device); the cross-slice amplitude sum is FP64 in every form. */
typedef enum {
    TNC_C64 = 0,
    TNC_F16_4M = 1,
    TNC_F16_3M = 2,
    TNC_BF16_4M = 3,
    TNC_BF16_3M = 4
} tnc_precision;

typedef struct tnc_ctx tnc_ctx;
typedef struct tnc_network tnc_network;
typedef struct tnc_plan tnc_plan;

/* Static description of a plan (filled by tnc_plan_info / tnc_plan_analyze). */
typedef struct {
    int32_t n_steps;               /* pairwise steps in the path                          */
    int32_t n_dep_steps;           /* steps that depend on the slice (run once per slice) */
    int32_t n_sliced;              /* sliced labels                                        */
    int32_t max_rank;              /* largest tensor rank of one slice                     */
    int32_t slices_in_flight;      /* slices batched through each step (0 before planning) */
    int32_t out_rank;              /* rank of the final open-qubit tensor                  */
    double flops_per_slice;        /* algorithmic real flops, 8*B*M*N*K per dependent step */
    double flops_invariant;        /* the same for slice-invariant steps (once per call)   */
    double bytes_per_slice;        /* algorithmic HBM bytes of the dependent steps         */
    double permute_bytes_per_slice;/* the part of bytes_per_slice spent in permutes        */
    double peak_bytes;             /* arena bytes needed at slices_in_flight               */
    double peak_elems_per_slice;   /* largest tensor of one slice, in complex entries      */
    double tune_seconds;           /* host time spent timing kernel variants at plan time  */
    int32_t n_host_steps;          /* steps of the given path contracted on the host in     */
                                   /* FP64 before the device path (not in n_steps)          */
    int32_t n_recompute;           /* recomputed labels (2^n_recompute passes per slice);   */
                                   /* flops and bytes per slice count every pass            */
    int32_t n_padded_steps;        /* sparse-state steps on the padded-index scheme         */
} tnc_plan_stats;

/* Results of one tnc_execute. */
typedef struct {
    double seconds;                /* device time of the slice block (HIP events)          */
    double flops;                  /* algorithmic real flops executed                      */
    int64_t slices;                /* slices summed                                        */
    int32_t replays;               /* rescale replays after an FP16 range flag             */
    int32_t graph_launches;        /* graph launches (1 when the block ran as one graph)   */
} tnc_report;

const char *tnc_last_error(void);
const char *tnc_version(void);

/* ------------------------------------------------------------------ context */

/* Make a context on HIP device `device`.
 * workspace / workspace_bytes: caller-owned device memory that holds every
 *   intermediate tensor (the arena); the library never frees it.  May be NULL
 *   with workspace_bytes = 0 for a context that only plans.
 * hip_stream: caller-owned hipStream_t (NULL = the null stream); all device
 *   work of this context is enqueued on it. */
int tnc_create(tnc_ctx **out, int device, void *workspace, size_t workspace_bytes, void *hip_stream);
int tnc_destroy(tnc_ctx *ctx);

/* ------------------------------------------------------------------ network */

/* Describe a network (host only; no device work).
 * ranks[n_tensors]; labels = the concatenation of every tensor's labels
 *   (first label slowest), each label id in [0, 2^30);
 * data_c128: the concatenation of every tensor's 2^rank complex entries as
 *   interleaved (re, im) doubles; copied.
 * output_labels[n_qubits]: the open leg of qubit q (its last wire); each
 *   occurs in at least one tensor, and no two qubits share one.
 * No label may repeat within a tensor (TNC_EINVAL).  A label held by one
 * tensor only that is not an output label is summed over here, in FP64 (the
 * reduction of Sec. 3.3, Eq. contraction, applied to a single operand).  A
 * label held by three or more tensors (a hyperedge) is accepted by the plan
 * calls, which keep it as a batch label until its last holder is contracted;
 * tnc_search and tnc_slice_path return TNC_EUNSUPPORTED for such networks. */
int tnc_network_create(int32_t n_tensors, const int32_t *ranks, const int32_t *labels,
                       const double *data_c128, int32_t n_qubits, const int32_t *output_labels,
                       tnc_network **out);
int tnc_network_destroy(tnc_network *net);

/* ------------------------------------------------------------------ search */

/* Find a contraction path and sliced labels for `net` with the qubits in
 * open_qubits[n_open] left open and every other qubit closed.
 * log2_cap: per-slice limit on the largest tensor, log2 of complex entries.
 * cost_model: 0 = FLOP/byte cost, 1 = the learned step-time model made
 *   active with tnc_costmodel_use (falls back to 0 when none is active).
 * restarts: randomized greedy trials (>= 1); seed makes the result
 *   deterministic.
 * ssa_out: host, capacity 2*(n_tensors-1) ints; receives the path as
 *   single-static-assignment pairs (ids >= n_tensors name step results).
 * sliced_out: host, capacity max_sliced; receives sliced label ids.
 * n_sliced: host out.  log2_cost_out (may be NULL): log2 of total real flops
 *   over all slices under the FLOP model. */
int tnc_search(const tnc_network *net, int32_t n_open, const int32_t *open_qubits, double log2_cap,
               int32_t cost_model, int32_t restarts, uint64_t seed, int32_t *ssa_out,
               int32_t max_sliced, int32_t *sliced_out, int32_t *n_sliced, double *log2_cost_out);

/* Slice an existing path further: starting from sliced_in[n_in], add sliced
 * labels (cheapest added work first) until no tensor of one slice exceeds
 * 2^log2_cap entries.  sliced_out (host, capacity max_sliced) receives the
 * whole set, the given labels first, in order; n_out the count. */
int tnc_slice_path(const tnc_network *net, int32_t n_steps, const int32_t *ssa_pairs, int32_t n_open,
                   const int32_t *open_qubits, double log2_cap, int32_t n_in, const int32_t *sliced_in,
                   int32_t max_sliced, int32_t *sliced_out, int32_t *n_out);

/* ------------------------------------------------------------------ plan */

/* Compile a path for execution on ctx's device (paper Sec. 3.1: a
 * sub-network and its pairwise contraction order, Alg. 1 "init"; slicing
 * fixes the chosen labels, Sec. 3.1 global level; each step a permutation
 * and a GEMM, Sec. 3.3 and 3.4.2).  Every step's GEMM kernel
 * variant is chosen by timing the candidates on the step's own operands
 * (environment: TNC_TUNE=0 keeps the shape-based default; TNC_TUNE_CACHE names
 * a file that persists the choices).
 * ssa_pairs[2*n_steps]: the path (a full binary tree over all tensors).
 * sliced_labels[n_sliced]: labels fixed per slice; slice s sets
 *   sliced_labels[j] to bit j of s.  Must not be output labels.
 * open_qubits[n_open]: qubits whose output labels stay open; the others are
 *   closed with the values the bitstrings give them at execute time.
 * max_slices_in_flight: upper bound on slices batched through each step
 *   (0 = as many as the workspace holds, at most 2^n_sliced).
 * Errors: TNC_EINVAL (path or labels), TNC_ENOMEM (one slice does not fit the
 *   workspace), TNC_EDEVICE. */
int tnc_plan_create(tnc_ctx *ctx, const tnc_network *net, int32_t n_steps, const int32_t *ssa_pairs,
                    int32_t n_sliced, const int32_t *sliced_labels, int32_t n_open,
                    const int32_t *open_qubits, tnc_precision prec, int32_t max_slices_in_flight,
                    tnc_plan **out);
/* Recomputation (paper Sec. 3.4.1): the large tensors of a slice are formed
 * in parts instead of at once.  As tnc_plan_create, plus recompute_labels
 * [n_recompute] (0..8 labels, neither sliced nor output labels), which are
 * fixed per pass instead of per slice.  The steps whose sub-tree holds no
 * recomputed label (the prefix) run once per slice and their results are kept;
 * the rest (the suffix from the steps that bring those labels in) run once per
 * pass, 2^n_recompute passes per slice, pass p setting recompute_labels[j] to
 * bit j of p, and the passes add up to the slice's value.  A slice's result is
 * the same sub-network sum as without recomputation (up to rounding order),
 * so ranges of slices compose as before; only the suffix's tensors shrink,
 * each by a factor 2 per recomputed label it holds.  tnc_plan_info then
 * reports flops and bytes per slice over all passes and n_recompute. */
int tnc_plan_create_recompute(tnc_ctx *ctx, const tnc_network *net, int32_t n_steps, const int32_t *ssa_pairs,
                              int32_t n_sliced, const int32_t *sliced_labels, int32_t n_recompute,
                              const int32_t *recompute_labels, int32_t n_open, const int32_t *open_qubits,
                              tnc_precision prec, int32_t max_slices_in_flight, tnc_plan **out);
/* Sparse-state contraction of uncorrelated bitstrings (paper Sec. 3.4.2,
 * "Tensor contraction during sparse state", Fig. sparse state): the
 * amplitudes of bitstrings[n_bitstrings] (host; any values, duplicates
 * allowed) in one contraction, whatever bits they share.  No output label is
 * closed or left open: a tensor holding the output labels of qubit set Q is
 * stored as one dense block per distinct value the bitstrings take on Q, and
 * each step forms every result block from the operand blocks with the
 * matching values (the multi-pair contraction of the figure), by one of its
 * two indexing schemes, chosen per step by the bytes it moves: (1) a batched
 * GEMM that reads its operand blocks through index arrays (no gathered copy
 * is made); (2) when many result blocks share an A block, the padded
 * two-dimensional index: each A block is multiplied once by B_P, the B
 * blocks of its result blocks side by side (index -1: zero blocks), and the
 * result blocks are taken out of that product; B_P and the product are built
 * a chunk of A blocks at a time in the arena, so they stay within the larger
 * of the result's size and 2^24 entries.  tnc_execute then takes exactly
 * these bitstrings (TNC_EINVAL otherwise) and returns their amplitudes summed
 * over the slice range.  Sliced labels as for tnc_plan_create.  Networks with
 * hyperedges: TNC_EUNSUPPORTED.  The arena holds every tensor's blocks, so
 * the path should bring the output labels in late (the sparse state of the
 * final stage). */
int tnc_plan_create_sparse(tnc_ctx *ctx, const tnc_network *net, int32_t n_steps, const int32_t *ssa_pairs,
                           int32_t n_sliced, const int32_t *sliced_labels, int64_t n_bitstrings,
                           const uint64_t *bitstrings, tnc_precision prec, int32_t max_slices_in_flight,
                           tnc_plan **out);
int tnc_plan_destroy(tnc_plan *plan);
int tnc_plan_info(const tnc_plan *plan, tnc_plan_stats *stats);

/* Host-only analysis of a path (no context, no device): fills `stats` for
 * one slice (slices_in_flight = 0, peak_bytes for one slice). */
int tnc_plan_analyze(const tnc_network *net, int32_t n_steps, const int32_t *ssa_pairs,
                     int32_t n_sliced, const int32_t *sliced_labels, int32_t n_open,
                     const int32_t *open_qubits, tnc_precision prec, tnc_plan_stats *stats);

/* tnc_plan_analyze with recomputed labels (as tnc_plan_create_recompute):
 * peak_bytes is one slice's arena with the suffix at one pass. */
int tnc_plan_analyze_recompute(const tnc_network *net, int32_t n_steps, const int32_t *ssa_pairs,
                               int32_t n_sliced, const int32_t *sliced_labels, int32_t n_recompute,
                               const int32_t *recompute_labels, int32_t n_open, const int32_t *open_qubits,
                               tnc_precision prec, tnc_plan_stats *stats);

/* tnc_plan_analyze for a sparse-state plan (as tnc_plan_create_sparse):
 * flops and bytes per slice over all blocks; peak_elems_per_slice is the
 * largest tensor's entries over all its blocks. */
int tnc_plan_analyze_sparse(const tnc_network *net, int32_t n_steps, const int32_t *ssa_pairs, int32_t n_sliced,
                            const int32_t *sliced_labels, int64_t n_bitstrings, const uint64_t *bitstrings,
                            tnc_precision prec, tnc_plan_stats *stats);

/* Choose recomputed labels for a sliced path (host only): while a tensor of
 * one pass holds more than 2^log2_cap entries, add the label of a largest
 * tensor (not an output label) whose recomputed suffix adds the least work
 * over all passes.  recompute_out: host, capacity max_recompute (<= 8);
 * n_out: host.  TNC_EINVAL when the cap needs more than max_recompute. */
int tnc_recompute_path(const tnc_network *net, int32_t n_steps, const int32_t *ssa_pairs, int32_t n_sliced,
                       const int32_t *sliced_labels, int32_t n_open, const int32_t *open_qubits, double log2_cap,
                       int32_t max_recompute, int32_t *recompute_out, int32_t *n_out);

/* Host-only per-step description of a path (arrays as in tnc_plan_steps,
 * capacity n_steps, each may be NULL). */
int tnc_plan_analyze_steps(const tnc_network *net, int32_t n_steps, const int32_t *ssa_pairs,
                           int32_t n_sliced, const int32_t *sliced_labels, int32_t n_open,
                           const int32_t *open_qubits, tnc_precision prec, int32_t *log2_mnkb,
                           int32_t *kernel, int32_t *dep, int32_t *perm_ab, double *flops,
                           double *bytes);

/* Sum the amplitudes of slices [slice_begin, slice_end) for each bitstring
 * (paper Sec. 3.1: the amplitude is the sum over the sliced sub-networks;
 * Sec. 1 and 2.3: the bitstrings of one correlated subspace share the
 * closed qubits and are read off the open-qubit tensor together).
 * bitstrings: host, n_bitstrings values; they must agree on every closed qubit
 *   (TNC_EINVAL otherwise); duplicates are allowed.
 * out_c128: 2*n_bitstrings doubles (re, im), host or device memory on the
 *   context's device; receives the FP64 partial sums, so disjoint ranges add.
 * rep: may be NULL.
 * Slices in [slice_begin, slice_end) run as one graph launch on the context's
 * stream; the call returns after the result is in out_c128. */
int tnc_execute(tnc_plan *plan, int64_t n_bitstrings, const uint64_t *bitstrings, int64_t slice_begin,
                int64_t slice_end, double *out_c128, tnc_report *rep);

/* Growth estimates of the scale epilogue (16-bit forms; not in the paper,
 * which computes in complex-half without per-tensor scaling).  Every 16-bit
 * step stores C * 2^-t with t = floor(log2 maxA) + floor(log2 maxB) + g - 13,
 * maxA / maxB its operands' largest stored components, so that the result's
 * largest stored component lands near 2^13; g is the step's growth estimate,
 * log2 of max|C| / (max|A| max|B|).  A stored maximum above 32752 (FP16: half
 * the range, so that a 3M consumer's re + im stays finite) or a non-finite
 * value flags the step; tnc_execute then raises the flagged steps' g by 4 and
 * runs the block again, at most 3 times (TNC_EOVERFLOW after that).  After
 * every successful call each g becomes ceil of the largest growth realized
 * by the slices of the last group, so estimates narrow as well as widen.
 * growth: host, one int per device step of the plan (tnc_plan_info n_steps),
 * values in [-64, 64].  TNC_EINVAL for complex64 plans (set) or a wrong count. */
int tnc_plan_get_growth(const tnc_plan *plan, int32_t n_steps, int32_t *growth);
int tnc_plan_set_growth(tnc_plan *plan, int32_t n_steps, const int32_t *growth);

/* Per-step device times of the last tnc_execute run with step timing on
 * (tnc_plan_set_timing; timed runs launch step by step, not as one graph).
 * Host arrays of capacity n_steps (each may be NULL): gemm_ms[t] and
 * permute_ms[t] are the summed HIP-event times of step t's GEMM launches and
 * operand permutes over the call, launches[t] the number of GEMM launches
 * (one per slice group for a slice-dependent step). */
int tnc_plan_set_timing(tnc_plan *plan, int32_t on);
int tnc_plan_step_times(const tnc_plan *plan, int32_t n_steps, double *gemm_ms, double *permute_ms,
                        int32_t *launches);

/* Per-step static description (host arrays of capacity n_steps, each may be
 * NULL): log2 of M, N, K and of the inner batch; the kernel variant id; 1 if
 * the step depends on the slice; the stride class of its A and B operands
 * (0 read in place as [free][k], 1 read in place as [k][free], 2 permuted first);
 * algorithmic real flops per slice (8 B M N K) and GEMM bytes per slice
 * (A + B + C at the storage size). */
int tnc_plan_steps(const tnc_plan *plan, int32_t n_steps, int32_t *log2_mnkb /* 4 per step */,
                   int32_t *kernel, int32_t *dep, int32_t *perm_ab /* 2 per step */, double *flops,
                   double *bytes);

/* ------------------------------------------------------------------ one contraction */

/* One pairwise contraction C = A . B on device-resident operands (paper
 * Eq. contraction), used by the step microbenchmark.
 * A, B, C: device, complex storage of `prec` (C64: 8-byte float pairs;
 *   16-bit forms: 4-byte (re, im) pairs), ranks a_rank/b_rank/c_rank with the
 *   given label lists (first label slowest).  Labels of C must be a subset of
 *   those of A and B; labels of A and B missing from C must occur in both.
 * scale_log2: 16-bit forms store C * 2^-scale_log2 (exact power of two).
 * times_ms: host, 4 doubles or NULL: permute(A), permute(B), GEMM, permute(C)
 *   device times of this call.
 * max_abs_out: host, 1 float or NULL: largest |re| or |im| stored in C. */
int tnc_contract(tnc_ctx *ctx, tnc_precision prec, const void *A, int32_t a_rank,
                 const int32_t *a_labels, const void *B, int32_t b_rank, const int32_t *b_labels,
                 void *C, int32_t c_rank, const int32_t *c_labels, int32_t scale_log2,
                 double *times_ms, float *max_abs_out);

/* ------------------------------------------------------------------ learned step-cost model */

/* Step-time MLP (3 Linear layers, in -> 128 -> 128 -> 1, ReLU, FP32), trained
 * on the device by the library's own forward, backward and Adam kernels.
 * Feature row layout (TNC_MLP_FEATURES floats): log2 M, log2 N, log2 K,
 * log2 batch, stride class of A, stride class of B, dtype (0 c64, 1 f16,
 * 2 bf16), algorithm (0 4M, 1 3M).  Target: log2 of the step time in
 * microseconds. */
#define TNC_MLP_FEATURES 8
#define TNC_MLP_HIDDEN 128

/* Train from scratch on n rows (host arrays x[n*TNC_MLP_FEATURES], y[n]) for
 * `epochs` epochs of minibatches of `batch` rows, Adam with learning rate lr,
 * initial weights from `seed`.  loss_out (host, may be NULL): final mean
 * squared error on the training rows.  The trained weights become the
 * context's cost model. */
int tnc_mlp_train(tnc_ctx *ctx, int64_t n, const float *x, const float *y, int32_t epochs,
                  int32_t batch, float lr, uint64_t seed, float *loss_out);
/* Continue from the current weights with `steps` full-batch Adam steps on
 * the n rows (host arrays as in tnc_mlp_train), from fresh moments (m = v = 0,
 * step count 0): beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected, as
 * tnc_mlp_train takes per minibatch.  loss_out (host, may be NULL): the mean
 * squared error after the last step.  The weights become the cost model. */
int tnc_mlp_adam(tnc_ctx *ctx, int64_t n, const float *x, const float *y, int32_t steps, float lr,
                 float *loss_out);
/* Predict n rows (host in, host out).  After tnc_mlp_train or tnc_mlp_adam
 * the network is not asked to extrapolate in the size features (log2 M, N,
 * K, batch): each is clamped to the range the training rows spanned, so the
 * output there is the value at the range's edge.  Weights loaded with
 * tnc_mlp_set_params carry no range and are evaluated as given. */
int tnc_mlp_predict(tnc_ctx *ctx, int64_t n, const float *x, float *y_out);
/* One forward + backward pass on n rows with the current weights: loss (MSE)
 * and the gradient of every parameter, concatenated in the order W1, b1, W2,
 * b2, W3, b3 (W row-major [out][in]); grads_out host, tnc_mlp_param_count()
 * floats.  Used to check gradients. */
int tnc_mlp_grad(tnc_ctx *ctx, int64_t n, const float *x, const float *y, float *loss_out,
                 float *grads_out);
int64_t tnc_mlp_param_count(void);
/* Copy weights out / in (host, tnc_mlp_param_count() floats, same order). */
int tnc_mlp_get_params(tnc_ctx *ctx, float *params_out);
int tnc_mlp_set_params(tnc_ctx *ctx, const float *params);
/* Make the context's MLP the cost model used by tnc_search(cost_model = 1)
 * on this thread.  The search prices a step at
 *     log2 t = tnc_costmodel_base(row) + MLP(row)   (microseconds),
 * so the network is trained on y = log2(measured t) - tnc_costmodel_base(row):
 * the learned part is the ratio of measured to roofline time, and a step
 * unlike the training rows keeps the baseline's scaling with its work. */
int tnc_costmodel_use(tnc_ctx *ctx);
/* Roofline baseline of n feature rows (host in, host out; layout as above):
 * log2 of 4 us plus the larger of the step's algorithmic flops (8 M N K per
 * batch entry) at the matrix-core peak of its dtype (complex64: FP32 157.3
 * TFLOP/s; FP16/BF16: 2516.6 TFLOP/s) and its bytes (A, B and C at the
 * storage size, 8 or 4 bytes an entry, plus a read and a write of each
 * operand of stride class 2) at 8 TB/s.  Host only; no context needed. */
int tnc_costmodel_base(int64_t n, const float *x, float *log2_us_out);

/* ------------------------------------------------------------------ low-precision exchange codec */

/* Quantization of the data a sub-network exchanges (paper Sec. 3.2, Eq.
 * quantcal with the parameters of Table quanttable).  A group of real values
 * y = sign(x)|x|^exp is mapped to q = y * scale + zero with
 *     scale = (q_max - q_min) / (max y - min y),
 *     zero  = (q_min max y - q_max min y) / (max y - min y),
 * rounded half-to-even and clamped for the integer kinds; decoding inverts
 * the map.  A complex tensor is coded as the real array of its interleaved
 * (re, im) float32 values (n = 2 x entries).  Kinds:
 *   TNC_Q_HALF  q in +-65504, exp 1, one group (the whole tensor), 2 bytes per value (FP16)
 *   TNC_Q_INT8  q in -128..127, exp 0.2, one group, 1 byte per value
 *   TNC_Q_INT4  q in 0..15, exp 1, groups of `group` values (a power of two,
 *               16..1024; 0 = 128), half a byte per value, value 2j in the low
 *               nibble of byte j; the last group may be short, and an unused
 *               high nibble is 0
 * The integer decision is taken in float32 with each operation rounded (no
 * fused multiply-add).  A group whose values are all equal gets scale 1 and
 * zero = q_min - value.  Values must be finite.
 * The compression rate of Eq. compress is (4 n_groups + 4 n_groups +
 * code_bytes) / (4 n). */
#define TNC_Q_HALF 0
#define TNC_Q_INT8 1
#define TNC_Q_INT4 2

/* Sizes for n values: bytes of codes and number of groups (host outputs,
 * either may be NULL).  TNC_EINVAL for an unknown kind or group size (half
 * and int8 take group 0). */
int tnc_quant_sizes(int32_t kind, int64_t n, int32_t group, int64_t *code_bytes, int64_t *n_groups);
/* Quantize n float32 values x (device, 16-byte aligned) into codes (device,
 * 16-byte aligned, tnc_quant_sizes bytes), scales and zeros (device float32,
 * one per group).  Runs on the context's stream and waits for it; ms_out
 * (host, may be NULL) receives the device time of the kernels. */
int tnc_quantize(tnc_ctx *ctx, int32_t kind, int64_t n, const float *x, int32_t group, void *codes,
                 float *scales, float *zeros, double *ms_out);
/* tnc_quantize for callers that cannot allocate: code under HIP graph
 * capture, tight serving loops, harnesses that forbid device allocation.  It
 * needs no context and makes no allocation of any kind (no hipMalloc, no
 * events): the min/max partials of the half and int8 kinds go to a
 * file-scope device array of 512 float2 (4 KB) that each GPU the library runs
 * on holds until the process ends; int4 uses none.  The array's address on a
 * device is looked up (hipGetSymbolAddress) on the first call made with that
 * device current.  Arguments as for tnc_quantize; the work is enqueued on
 * hip_stream (a hipStream_t, NULL = the null stream) of the current device,
 * and the call returns without waiting for it.  Results are bit-identical to
 * tnc_quantize's.  Every call on a GPU shares that GPU's array and every
 * partial is written before it is read, so nothing needs clearing; calls whose
 * work overlaps on one GPU (different streams, no ordering) race on it and
 * must be serialized by the caller.  TNC_EINVAL on a bad kind, group, length,
 * NULL or misaligned buffer; no length exceeds the array (the min/max pass
 * uses at most 512 blocks for any n). */
int tnc_quantize_noalloc(int32_t kind, int64_t n, const float *x, int32_t group, void *codes, float *scales,
                         float *zeros, void *hip_stream);
/* Decode n values from codes, scales and zeros (device) into x (device,
 * 16-byte aligned, float32).  Same stream and timing behaviour. */
int tnc_dequantize(tnc_ctx *ctx, int32_t kind, int64_t n, const void *codes, const float *scales,
                   const float *zeros, int32_t group, float *x, double *ms_out);
/* Pass the result of path step `step` of a complex64 plan through the codec
 * (quantize, then dequantize in place, each slice on its own) on every later
 * tnc_execute, as if that tensor were exchanged between devices (paper Sec.
 * 3.2; the single-step quantization study of Sec. 4.3.1).  step = -1 switches it off.
 * The plan allocates the code buffers.  TNC_EUNSUPPORTED for 16-bit plans. */
int tnc_plan_set_codec(tnc_plan *plan, int32_t step, int32_t kind, int32_t group);

/* ------------------------------------------------------------------ post-selection
 * Top-k post-selection in a correlated subspace (paper Sec. 1 and Sec. 2.3,
 * post-processing): of the n amplitudes of one subspace, the k bitstrings with
 * the largest probabilities.
 *
 * amps:     device, n complex128 amplitudes (interleaved re, im; the layout
 *           tnc_execute returns), 8-byte aligned, all finite.
 * k:        1..1024; min(k, n) entries are written.
 * idx_out:  device, int64 positions into amps, most probable first.
 * prob_out: device, float64 probabilities re*re + im*im (each operation
 *           rounded on its own) of those entries.
 * Order: probability descending, then position ascending, so the list is
 * unique even with ties.  The context's workspace holds the candidate rounds
 * (32 bytes x ceil(n / 2048) x k when n > 2048; TNC_ENOMEM if it is smaller).
 * Runs on the context's stream and waits for it; ms_out (optional) = device
 * time.  TNC_EINVAL on a NULL or misaligned buffer or k out of range. */
int tnc_topk(tnc_ctx *ctx, int64_t n, const double *amps, int32_t k, int64_t *idx_out, double *prob_out,
             double *ms_out);

#ifdef __cplusplus
}
#endif
#endif /* TNC_H */
