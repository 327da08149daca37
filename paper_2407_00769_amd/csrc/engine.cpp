// C-ABI entry points: context, network, plan, execution of a slice block,
// one-off contraction.  Every step of a slice runs in the library's HIP
// kernels; the host only validates, plans and enqueues.
#include "engine.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <set>

#include "planner.h"

using namespace tnc;

namespace tnc {
static thread_local std::string g_err;
void set_error(const std::string &msg) { g_err = msg; }
}  // namespace tnc

extern "C" const char *tnc_last_error(void) { return tnc::g_err.c_str(); }
extern "C" const char *tnc_version(void) { return "tnc 0.1 (gfx950)"; }

#define API_BEGIN try {
#define API_END                                            \
    }                                                      \
    catch (const tnc::Error &e) {                          \
        tnc::set_error(e.msg);                             \
        return e.code;                                     \
    }                                                      \
    catch (const std::bad_alloc &) {                       \
        tnc::set_error("host allocation failed");          \
        return TNC_ENOMEM;                                 \
    }                                                      \
    catch (const std::exception &e) {                      \
        tnc::set_error(e.what());                          \
        return TNC_EINVAL;                                 \
    }                                                      \
    return TNC_OK;

#define REQUIRE(cond, msg) \
    do {                   \
        if (!(cond)) TNC_THROW(TNC_EINVAL, msg); \
    } while (0)

// ------------------------------------------------------------------ context

extern "C" int tnc_create(tnc_ctx **out, int device, void *workspace, size_t workspace_bytes, void *hip_stream) {
    API_BEGIN
    REQUIRE(out, "out is NULL");
    *out = nullptr;
    int n = 0;
    HIP_CHECK(hipGetDeviceCount(&n));
    REQUIRE(device >= 0 && device < n, "device out of range");
    REQUIRE(workspace || workspace_bytes == 0, "workspace is NULL but workspace_bytes > 0");
    HIP_CHECK(hipSetDevice(device));
    auto *c = new tnc_ctx;
    c->device = device;
    c->ws = (uint8_t *)workspace;
    c->ws_bytes = workspace_bytes;
    c->stream = (hipStream_t)hip_stream;
    hipError_t e = hipMalloc((void **)&c->small, 4096);
    if (e != hipSuccess) {
        delete c;
        TNC_THROW(TNC_EDEVICE, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    *out = c;
    API_END
}

extern "C" int tnc_destroy(tnc_ctx *ctx) {
    API_BEGIN
    if (!ctx) return TNC_OK;
    hipSetDevice(ctx->device);
    if (ctx->small) hipFree(ctx->small);
    if (ctx->mlp) mlp_free(ctx->mlp);
    delete ctx;
    API_END
}

// ------------------------------------------------------------------ network

extern "C" int tnc_network_create(int32_t n_tensors, const int32_t *ranks, const int32_t *labels,
                                  const double *data_c128, int32_t n_qubits, const int32_t *output_labels,
                                  tnc_network **out) {
    API_BEGIN
    REQUIRE(out, "out is NULL");
    *out = nullptr;
    REQUIRE(n_tensors >= 1, "n_tensors < 1");
    REQUIRE(ranks && labels, "ranks or labels is NULL");
    REQUIRE(n_qubits >= 0 && n_qubits <= 64, "n_qubits must be in [0, 64]");
    REQUIRE(n_qubits == 0 || output_labels, "output_labels is NULL");
    auto *nw = new tnc_network;
    Network &net = nw->net;
    try {
        net.n_tensors = n_tensors;
        net.labels.resize(n_tensors);
        net.data.resize(n_tensors);
        int64_t lp = 0, dp = 0;
        int maxl = -1;
        for (int i = 0; i < n_tensors; i++) {
            REQUIRE(ranks[i] >= 0 && ranks[i] <= 30, "tensor rank out of [0, 30]");
            for (int j = 0; j < ranks[i]; j++) {
                int l = labels[lp++];
                REQUIRE(l >= 0 && l < (1 << 30), "label id out of range");
                net.labels[i].push_back(l);
                maxl = std::max(maxl, l);
            }
            std::vector<int> sorted = net.labels[i];
            std::sort(sorted.begin(), sorted.end());
            REQUIRE(std::adjacent_find(sorted.begin(), sorted.end()) == sorted.end(),
                    "tensor " + std::to_string(i) + " repeats a label");
            int64_t n = (int64_t)1 << ranks[i];
            if (data_c128) net.data[i].assign(data_c128 + 2 * dp, data_c128 + 2 * (dp + n));
            else net.data[i].assign(2 * n, 0.0);
            dp += n;
        }
        net.n_labels = maxl + 1;
        REQUIRE(net.n_labels <= (1 << 24), "label ids must be below 2^24 (dense ids expected)");
        std::vector<int> cnt(net.n_labels, 0), is_out(net.n_labels, 0);
        for (auto &v : net.labels)
            for (int l : v) cnt[l]++;
        net.n_qubits = n_qubits;
        for (int q = 0; q < n_qubits; q++) {
            int l = output_labels[q];
            REQUIRE(l >= 0 && l < net.n_labels && cnt[l] >= 1, "output label of qubit " + std::to_string(q) + " not in the network");
            REQUIRE(!is_out[l], "two qubits share an output label");
            is_out[l] = 1;
            net.output_labels.push_back(l);
        }
        // A label held by one tensor only, and not an output label, is summed
        // over here (paper Eq. contraction: a label that no other operand
        // holds and the result does not keep is reduced), in FP64.  A label
        // held by three or more tensors (a hyperedge) stays; the device path
        // keeps it as a batch label until its last holder is contracted.
        for (int i = 0; i < n_tensors; i++) {
            std::vector<int> &ls = net.labels[i];
            for (int j = (int)ls.size() - 1; j >= 0; j--) {
                const int l = ls[j];
                if (cnt[l] != 1 || is_out[l]) continue;
                const int r = (int)ls.size();
                const int64_t n_out = (int64_t)1 << (r - 1), lo = (int64_t)1 << (r - 1 - j);
                std::vector<double> d(2 * n_out, 0.0);
                for (int64_t o = 0; o < n_out; o++) {
                    const int64_t base = (o / lo) * 2 * lo + (o % lo);   // label bit 0
                    d[2 * o] = net.data[i][2 * base] + net.data[i][2 * (base + lo)];
                    d[2 * o + 1] = net.data[i][2 * base + 1] + net.data[i][2 * (base + lo) + 1];
                }
                net.data[i].swap(d);
                ls.erase(ls.begin() + j);
                cnt[l] = 0;
            }
        }
        for (int l = 0; l < net.n_labels; l++)
            if (cnt[l] > 2) net.hyperedges = true;
    } catch (...) {
        delete nw;
        throw;
    }
    *out = nw;
    API_END
}

extern "C" int tnc_network_destroy(tnc_network *net) {
    delete net;
    return TNC_OK;
}

// ------------------------------------------------------------------ plan

static void free_plan_device(tnc_plan *p) {
    for (auto &kv : p->graphs) hipGraphExecDestroy(kv.second);
    p->graphs.clear();
    void *ptrs[] = {p->d_leafdata, p->d_desc, p->d_maxw,  p->d_expw,  p->d_shift, p->d_growth, p->d_flags,
                    p->d_params,   p->d_bits, p->d_acc,   p->d_qob,   p->d_part,  p->d_codes,  p->d_qscale,
                    p->d_qzero,    p->d_spoff, p->d_idx,  p->d_map};
    for (void *q : ptrs)
        if (q) hipFree(q);
}

template <typename T> static T *dev_alloc(int64_t count) {
    T *p = nullptr;
    HIP_CHECK(hipMalloc((void **)&p, sizeof(T) * std::max<int64_t>(count, 1)));
    return p;
}

static void build_plan(tnc_plan *p, const Network &net, int max_sif) {
    Analysis &an = p->an;
    tnc_ctx *ctx = p->ctx;
    const int nT = net.n_tensors;
    p->nT = nT;
    p->n_qubits = net.n_qubits;
    p->output_labels = net.output_labels;
    p->leaf_orig_labels = net.labels;
    if (!an.sparse)
        for (int q = 0; q < net.n_qubits; q++)
            if (an.fixed[net.output_labels[q]] == 1) p->closed_qubits.push_back(q);
    // slices in flight: as many as fit, at most the slice count
    int64_t n_slices_total = (int64_t)1 << an.n_sliced;
    int64_t cap = n_slices_total;
    if (max_sif > 0) cap = std::min<int64_t>(cap, max_sif);
    cap = std::min<int64_t>(cap, 4096);
    int64_t peak1 = plan_memory(an, 1, false);
    if ((size_t)peak1 > ctx->ws_bytes)
        TNC_THROW(TNC_ENOMEM, "one slice needs " + std::to_string(peak1) + " workspace bytes, have " +
                                  std::to_string(ctx->ws_bytes));
    int S = 1;
    while (S * 2 <= cap && (size_t)plan_memory(an, S * 2, false) <= ctx->ws_bytes) S *= 2;
    p->S = S;
    p->peak = plan_memory(an, S, true);

    HIP_CHECK(hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    const Dtype dt = an.dt;
    const int es = elem_bytes(dt);
    // input tensors: upload complex128, convert on the device
    int64_t total = 0;
    std::vector<int64_t> leaf_off(nT);
    for (int i = 0; i < nT; i++) {
        leaf_off[i] = total;
        total += (int64_t)net.data[i].size() / 2;
    }
    p->d_leafdata = dev_alloc<uint8_t>(total * es);
    {
        double *tmp = dev_alloc<double>(2 * total);
        std::vector<double> h(2 * total);
        for (int i = 0; i < nT; i++) std::copy(net.data[i].begin(), net.data[i].end(), h.begin() + 2 * leaf_off[i]);
        HIP_CHECK(hipMemcpyAsync(tmp, h.data(), sizeof(double) * 2 * total, hipMemcpyHostToDevice, st));
        launch_convert_c128(tmp, total, dt, p->d_leafdata, st);
        HIP_CHECK(hipStreamSynchronize(st));
        hipFree(tmp);
    }
    // leaf descriptors: invariant first, then the slice prefix's, then the
    // recomputed ones (gathered once per pass)
    std::vector<int> inv, dep, inner;
    for (int i = 0; i < nT; i++) (!an.tensors[i].dep ? inv : (an.tensors[i].inner ? inner : dep)).push_back(i);
    p->n_inv_leaves = (int)inv.size();
    p->n_dep_leaves = (int)(dep.size() + inner.size());
    p->n_inner_leaves = (int)inner.size();
    p->desc_of_leaf.assign(nT, -1);
    std::vector<int> order = inv;
    order.insert(order.end(), dep.begin(), dep.end());
    order.insert(order.end(), inner.begin(), inner.end());
    std::vector<int64_t> spoff;   // sparse state: element offset of every leaf block
    for (int i : order) {
        const TensorRec &t = an.tensors[i];
        LeafDesc d{};
        d.src_off = leaf_off[i];
        d.dst_byte_off = t.off;
        d.dst_slice_stride = t.dep ? ((int64_t)1 << t.rank()) : 0;
        d.rank = t.rank();
        const auto &orig = net.labels[i];
        const int ro = (int)orig.size();
        for (int b = 0; b < d.rank; b++) {
            int l = t.labels[d.rank - 1 - b];
            int pos = ro - 1 - (int)(std::find(orig.begin(), orig.end(), l) - orig.begin());
            d.stride[b] = (int64_t)1 << pos;
        }
        for (int j = 0; j < ro; j++) {
            int l = orig[j];
            if (an.fixed[l] == 0) {
                d.slice_bit[d.n_sliced] = an.slice_bit[l];
                d.slice_stride[d.n_sliced] = (int64_t)1 << (ro - 1 - j);
                d.n_sliced++;
            }
        }
        d.n_slices = t.dep ? S : 1;
        d.max_slot = i * S;
        d.slot_stride = t.dep ? 1 : 0;
        d.nd = 1;
        d.sp_base = 0;
        if (an.sparse) {
            // block d of the leaf: its output labels at the qubit values of key d
            d.nd = (int)t.nd;
            d.sp_base = (int64_t)spoff.size();
            d.dst_slice_stride *= t.nd;
            for (uint64_t key : an.leaf_keys[i]) {
                int64_t o = 0;
                for (int j = 0; j < ro; j++) {
                    const int l = orig[j];
                    for (int q = 0; q < net.n_qubits; q++)
                        if (net.output_labels[q] == l && ((key >> q) & 1)) o += (int64_t)1 << (ro - 1 - j);
                }
                spoff.push_back(o);
            }
            p->nd_max = std::max<int>(p->nd_max, (int)t.nd);
        }
        p->desc_of_leaf[i] = (int)p->h_desc.size();
        p->h_desc.push_back(d);
    }
    if (an.sparse) {
        if (p->nd_max > 65535) TNC_THROW(TNC_EUNSUPPORTED, "an input tensor with more than 65535 sparse blocks");
        p->d_spoff = dev_alloc<int64_t>((int64_t)spoff.size());
        HIP_CHECK(hipMemcpyAsync(p->d_spoff, spoff.data(), sizeof(int64_t) * spoff.size(), hipMemcpyHostToDevice, st));
        // block index arrays of every step, one buffer
        std::vector<int32_t> idx;
        p->a_idx_off.assign(an.steps.size(), -1);
        p->b_idx_off.assign(an.steps.size(), -1);
        p->bp_idx_off.assign(an.steps.size(), -1);
        p->cp_idx_off.assign(an.steps.size(), -1);
        for (size_t k = 0; k < an.steps.size(); k++) {
            const StepRec &rec = an.steps[k];
            if (rec.scheme == 2) {
                p->bp_idx_off[k] = (int64_t)idx.size();
                idx.insert(idx.end(), rec.bp_idx.begin(), rec.bp_idx.end());
                p->cp_idx_off[k] = (int64_t)idx.size();
                idx.insert(idx.end(), rec.cp_idx.begin(), rec.cp_idx.end());
            }
            if (rec.a_mode == 2) {
                p->a_idx_off[k] = (int64_t)idx.size();
                idx.insert(idx.end(), rec.a_idx.begin(), rec.a_idx.end());
            }
            if (rec.b_mode == 2) {
                p->b_idx_off[k] = (int64_t)idx.size();
                idx.insert(idx.end(), rec.b_idx.begin(), rec.b_idx.end());
            }
        }
        p->d_idx = dev_alloc<int32_t>((int64_t)idx.size());
        if (!idx.empty())
            HIP_CHECK(hipMemcpyAsync(p->d_idx, idx.data(), sizeof(int32_t) * idx.size(), hipMemcpyHostToDevice, st));
        p->d_map = dev_alloc<int32_t>((int64_t)an.root_map.size());
        HIP_CHECK(hipMemcpyAsync(p->d_map, an.root_map.data(), sizeof(int32_t) * an.root_map.size(),
                                 hipMemcpyHostToDevice, st));
        HIP_CHECK(hipStreamSynchronize(st));
    }
    p->d_desc = dev_alloc<LeafDesc>((int64_t)p->h_desc.size());
    HIP_CHECK(hipMemcpyAsync(p->d_desc, p->h_desc.data(), sizeof(LeafDesc) * p->h_desc.size(),
                             hipMemcpyHostToDevice, st));
    p->closed_state.assign(nT, 0);
    const int64_t nslots = (int64_t)an.tensors.size() * S;
    p->d_maxw = dev_alloc<uint32_t>(nslots);
    p->d_expw = dev_alloc<double>(nslots);
    p->d_shift = dev_alloc<int>(nslots);
    const int ns = (int)an.steps.size();
    p->d_growth = dev_alloc<int>(ns);
    p->d_flags = dev_alloc<uint32_t>(ns);
    p->h_growth.resize(ns);
    for (int s = 0; s < ns; s++) {
        // expected log2 of max|C| / (max|A| max|B|): about half of log2 K for
        // random phases, plus one bit of margin
        int kb = (int)an.steps[s].k.size();
        p->h_growth[s] = (kb + 1) / 2 + 1;
    }
    HIP_CHECK(hipMemcpyAsync(p->d_growth, p->h_growth.data(), sizeof(int) * ns, hipMemcpyHostToDevice, st));
    launch_fill_u32(p->d_flags, 0, ns, st);
    launch_fill_f64(p->d_expw, 0.0, nslots, st);
    p->d_params = dev_alloc<int64_t>(4);
    const TensorRec &R = an.tensors[an.root];
    std::vector<int> qob(std::max(1, R.rank()));
    for (int b = 0; b < R.rank(); b++) qob[b] = an.open_qubit_of_label[R.labels[R.rank() - 1 - b]];
    p->d_qob = dev_alloc<int>((int64_t)qob.size());
    HIP_CHECK(hipMemcpyAsync(p->d_qob, qob.data(), sizeof(int) * qob.size(), hipMemcpyHostToDevice, st));
    HIP_CHECK(hipStreamSynchronize(st));
    // split-K partial sums: the largest need of any step under any kernel variant
    int64_t part_bytes = 0;
    for (const auto &rec : an.steps) {
        const TensorRec &A = an.tensors[rec.a], &B = an.tensors[rec.b], &Z = an.tensors[rec.z];
        GemmShape g = step_gemm_exec(rec);
        g.sA = A.dep ? 1 : 0;
        g.sB = B.dep ? 1 : 0;
        g.sC = 1;
        (void)Z;
        for (int k = K_MFMA_S; k < K_COUNT; k++)
            part_bytes = std::max(part_bytes, splitk_bytes(k, dt, an.al, g, rec.dep ? S : 1));
    }
    if (part_bytes > 0) p->d_part = (float2 *)dev_alloc<uint8_t>(part_bytes);
    p->part_bytes = part_bytes;
    p->step_ms.assign(ns, 0.0);
    p->perm_ms.assign(ns, 0.0);
    p->step_launches.assign(ns, 0);
    const char *ng = getenv("TNC_NO_GRAPH");
    // graphs are captured on the context's stream; the legacy null stream cannot be captured
    p->use_graph = !(ng && ng[0] == '1') && ctx->stream != nullptr;
}

// GEMM descriptor of step s as it runs in the arena: slice strides (per-slice
// size of a slice-dependent operand, 0 for a shared one), the split-K buffer,
// and, for sparse-state plans, which operand block every result block reads.
static GemmShape plan_step_shape(const tnc_plan *p, int s) {
    const Analysis &an = p->an;
    const StepRec &rec = an.steps[s];
    const TensorRec &A = an.tensors[rec.a], &B = an.tensors[rec.b], &Z = an.tensors[rec.z];
    const int64_t na = (int64_t)1 << A.rank(), nbb = (int64_t)1 << B.rank(), nz = (int64_t)1 << Z.rank();
    GemmShape g = step_gemm_exec(rec);
    g.sA = A.dep ? na * A.nd : 0;
    g.sB = B.dep ? nbb * B.nd : 0;
    g.sC = nz * Z.nd;
    g.part = p->d_part;
    g.part_cap = p->part_bytes;
    g.split_slices = rec.dep ? p->S : 1;   // the slice count d_part was sized for
    if (rec.scheme == 2) {
        // one chunk of A blocks against its B_P and C_P scratch (slice-major)
        g.sB = rec.chunk * rec.mr * nbb;
        g.sC = rec.chunk * rec.mr * nz;
        return g;
    }
    if (an.sparse) {
        if (rec.a_mode == 1) g.bA = 0;
        if (rec.b_mode == 1) g.bB = 0;
        if (rec.a_mode == 2) g.ia = p->d_idx + p->a_idx_off[s];
        if (rec.b_mode == 2) g.ib = p->d_idx + p->b_idx_off[s];
    }
    return g;
}

// Bit permutation of operand X (`from` -> its stored order) for n_slices
// slices: every slice's nd sparse blocks are permuted alike.
static void permute_operand(const tnc_plan *p, const TensorRec &X, const std::vector<int> &from, const void *src,
                            void *dst, int n_slices, hipStream_t st) {
    const Dtype dt = p->an.dt;
    const int64_t n = (int64_t)1 << X.rank();
    const int64_t total = (int64_t)n_slices * X.nd;
    const PermuteDesc d = make_permute(from, X.labels);
    const int64_t es = elem_bytes(dt);
    for (int64_t b0 = 0; b0 < total; b0 += 65535) {
        const int cnt = (int)std::min<int64_t>(65535, total - b0);
        launch_permute(dt, (const uint8_t *)src + b0 * n * es, (uint8_t *)dst + b0 * n * es, d, n, cnt, n, nullptr, n,
                       st);
    }
}

// ------------------------------------------------------------------ autotuner
// Each step's GEMM is timed with every kernel variant that supports its shape
// and operand orientation, on the step's real arena operands, and the fastest
// is kept.  Results are cached per (dtype, algorithm, log2 M, N, K, batch,
// orientation) for the process, and in the file named by TNC_TUNE_CACHE.
namespace {
using TuneKey = std::tuple<int, int, int, int, int, int, int, int, int>;
std::mutex g_tune_mu;
std::map<TuneKey, int> g_tune;
bool g_tune_loaded = false;

int ilog2(int64_t v) {
    int r = 0;
    while ((int64_t)1 << (r + 1) <= v) r++;
    return r;
}

void tune_cache_load() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char *f = getenv("TNC_TUNE_CACHE");
    if (!f) return;
    FILE *fp = fopen(f, "r");
    if (!fp) return;
    int a[10];
    while (fscanf(fp, "%d %d %d %d %d %d %d %d %d %d", &a[0], &a[1], &a[2], &a[3], &a[4], &a[5], &a[6], &a[7], &a[8],
                  &a[9]) == 10)
        g_tune[TuneKey(a[0], a[1], a[2], a[3], a[4], a[5], a[6], a[7], a[8])] = a[9];
    fclose(fp);
}

void tune_cache_append(const TuneKey &k, int kid) {
    const char *f = getenv("TNC_TUNE_CACHE");
    if (!f) return;
    FILE *fp = fopen(f, "a");
    if (!fp) return;
    fprintf(fp, "%d %d %d %d %d %d %d %d %d %d\n", std::get<0>(k), std::get<1>(k), std::get<2>(k), std::get<3>(k),
            std::get<4>(k), std::get<5>(k), std::get<6>(k), std::get<7>(k), std::get<8>(k), kid);
    fclose(fp);
}

double autotune_plan(tnc_plan *p) {
    // TNC_FORCE_KERNEL=<id>: every step that variant supports runs it, untimed
    // (tests of one variant over whole plans)
    if (const char *force = getenv("TNC_FORCE_KERNEL")) {
        const int f = atoi(force);
        for (size_t si = 0; si < p->an.steps.size(); si++)
            if (gemm_supported(f, p->an.dt, p->an.al, plan_step_shape(p, (int)si))) p->an.steps[si].kernel = f;
        return 0.0;
    }
    const char *env = getenv("TNC_TUNE");
    if (env && env[0] == '0') return 0.0;
    Analysis &an = p->an;
    const Dtype dt = an.dt;
    hipStream_t st = p->ctx->stream;
    uint8_t *ws = p->ctx->ws;
    std::lock_guard<std::mutex> lock(g_tune_mu);
    tune_cache_load();
    // Scale bookkeeping for the tuning launches: the producers' maxima and
    // exponents are one shared entry each (index stride 0), the per-slice
    // outputs (max |C|, exponent, shift) get S entries, since a launch covers
    // up to S slices.
    const int64_t S_t = p->S;
    const size_t off_maxc = 64, off_shift = off_maxc + 4 * S_t, off_expc = (off_shift + 4 * S_t + 7) & ~(size_t)7;
    const size_t tune_bytes = off_expc + 8 * S_t;
    uint8_t *tbuf = nullptr;
    HIP_CHECK(hipMalloc((void **)&tbuf, tune_bytes));
    struct FreeOnExit {
        uint8_t *ptr;
        hipStream_t st;
        ~FreeOnExit() {
            (void)hipStreamSynchronize(st);
            (void)hipFree(ptr);
        }
    } free_tbuf{tbuf, st};
    struct Head {
        uint32_t maxA, maxB, flag;
        int growth;
        double expA, expB;
    } h{0x3f800000u, 0x3f800000u, 0u, kTargetLog2Host, 0.0, 0.0};
    HIP_CHECK(hipMemsetAsync(tbuf, 0, tune_bytes, st));
    HIP_CHECK(hipMemcpyAsync(tbuf, &h, sizeof(h), hipMemcpyHostToDevice, st));
    HIP_CHECK(hipStreamSynchronize(st));
    Head *d = (Head *)tbuf;
    ScaleRefs sc{};
    sc.maxA = &d->maxA;
    sc.mA = 0;
    sc.maxB = &d->maxB;
    sc.mB = 0;
    sc.maxC = (uint32_t *)(tbuf + off_maxc);
    sc.flag = &d->flag;
    sc.growth = &d->growth;
    sc.shift = (int *)(tbuf + off_shift);
    sc.expA = &d->expA;
    sc.eA = 0;
    sc.expB = &d->expB;
    sc.eB = 0;
    sc.expC = (double *)(tbuf + off_expc);
    hipEvent_t e0, e1;
    HIP_CHECK(hipEventCreate(&e0));
    HIP_CHECK(hipEventCreate(&e1));
    auto t_start = std::chrono::steady_clock::now();
    for (size_t si = 0; si < an.steps.size(); si++) {
        auto &rec = an.steps[si];
        const TensorRec &A = an.tensors[rec.a], &B = an.tensors[rec.b], &Z = an.tensors[rec.z];
        const int64_t na = (int64_t)1 << A.rank(), nbb = (int64_t)1 << B.rank();
        GemmShape g = plan_step_shape(p, (int)si);
        const int Sl = rec.dep ? p->S : 1;
        // the per-slice bookkeeping of the tuning launches holds S_t slices
        if (Sl > S_t) TNC_THROW(TNC_EINVAL, "internal: tuning launch covers more slices than its scratch holds");
        std::vector<int> cands;
        // big steps: only the large matrix-core tiles are worth timing
        const bool big = rec.flops * (double)Sl > 1e13;
        static const int big_order[] = {K_DMA_8,   K_DMA_8W,   K_DMA_4,  K_DMA_2,   K_DMAP_2,  K_DMA_N64, K_DMA_N32,
                                        K_DMA3_N64, K_DMA3_2, K_MFMA_XL, K_MFMA_L2, K_MFMA_L};
        if (big) {
            for (int k : big_order)
                if (gemm_supported(k, dt, an.al, g)) cands.push_back(k);
        }
        if (cands.empty()) {
            for (int k = K_MFMA_S; k < K_COUNT; k++)
                if (gemm_supported(k, dt, an.al, g)) cands.push_back(k);
            // the VALU kernel where no matrix-core tile applies, the step is
            // tiny, or it is thin (N <= 16: HBM-bound, where either may win)
            if ((cands.empty() || rec.flops * (double)Sl < 1e9 || g.N <= 16) && gemm_supported(K_SKINNY_N, dt, an.al, g))
                cands.push_back(K_SKINNY_N);
        }
        if (cands.size() <= 1) continue;
        TuneKey key((int)dt, (int)an.al, ilog2(g.M), ilog2(g.N), ilog2(g.K), ilog2(g.nb), g.a_kc, g.b_kc, g.c_nc);
        auto it = g_tune.find(key);
        if (it != g_tune.end()) {
            if (gemm_supported(it->second, dt, an.al, g)) rec.kernel = it->second;
            continue;
        }
        const void *pa = ws + (rec.perm_a ? rec.scr_a : A.off);
        const void *pb = ws + (rec.perm_b ? rec.scr_b : B.off);
        void *pc = ws + Z.off;
        if (rec.scheme == 2) {   // the per-chunk GEMM reads B_P and writes C_P
            pb = ws + rec.scr_bp;
            pc = ws + rec.scr_cp;
        }
        {
            // the arena holds no data yet: give the operands random values
            const int64_t wa = (A.dep ? Sl : 1) * A.nd * na * elem_bytes(dt) / 4,
                          wb = rec.scheme == 2 ? (int64_t)Sl * rec.chunk * rec.mr * nbb * elem_bytes(dt) / 4
                                               : (B.dep ? Sl : 1) * B.nd * nbb * elem_bytes(dt) / 4;
            launch_fill_random(dt, (void *)pa, wa, 0x5eed0000u + (uint32_t)rec.a, st);
            launch_fill_random(dt, (void *)pb, wb, 0x5eed8000u + (uint32_t)rec.b, st);
        }
        // The clock of a loaded MI355X follows the power its matrix cores
        // draw, so a candidate timed after a cooler stretch looks faster.  A
        // big step first heats the chip (at least 100 ms of the first
        // candidate), then is timed in three rounds (forward, backward,
        // forward order over the candidates; after the first round only
        // those within 20% of the best), and each candidate is scored by the
        // median of its times.
        auto time_one = [&](int k, int reps) {
            HIP_CHECK(hipEventRecord(e0, st));
            for (int r = 0; r < reps; r++)
                launch_gemm(k, dt, an.al, pa, pb, pc, g, Sl, dt != Dtype::C64 ? &sc : nullptr, st);
            HIP_CHECK(hipEventRecord(e1, st));
            HIP_CHECK(hipEventSynchronize(e1));
            float ms = 0;
            HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
            return (double)ms / reps;
        };
        std::vector<std::vector<double>> t_ms(cands.size());
        double best = 1e30;
        const int rounds = big ? 3 : 1;
        const int reps = big ? 1 : 2;
        if (big) {
            double heat = 0;
            for (int w = 0; w < 8 && heat < 100.0; w++) heat += time_one(cands[0], 1);
        }
        for (int rd = 0; rd < rounds; rd++) {
            for (size_t i = 0; i < cands.size(); i++) {
                const size_t ci = (rd % 2 == 0) ? i : cands.size() - 1 - i;
                const int k = cands[ci];
                if (rd > 0 && *std::min_element(t_ms[ci].begin(), t_ms[ci].end()) > 1.2 * best) continue;
                if (rd == 0) launch_gemm(k, dt, an.al, pa, pb, pc, g, Sl, dt != Dtype::C64 ? &sc : nullptr, st);   // warm
                const double ms = time_one(k, reps);
                t_ms[ci].push_back(ms);
                best = std::min(best, ms);
            }
        }
        int best_k = rec.kernel;
        double best_score = 1e30;
        for (size_t ci = 0; ci < cands.size(); ci++) {
            std::vector<double> v = t_ms[ci];
            std::sort(v.begin(), v.end());
            const double med = v.size() % 2 ? v[v.size() / 2] : 0.5 * (v[v.size() / 2 - 1] + v[v.size() / 2]);
            if (med < best_score) {
                best_score = med;
                best_k = cands[ci];
            }
        }
        rec.kernel = best_k;
        g_tune[key] = best_k;
        tune_cache_append(key, best_k);
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
}
}  // namespace

static int create_plan(tnc_ctx *ctx, const tnc_network *net, int32_t n_steps, const int32_t *ssa_pairs,
                       int32_t n_sliced, const int32_t *sliced_labels, int32_t n_recompute,
                       const int32_t *recompute_labels, int32_t n_open, const int32_t *open_qubits,
                       int64_t n_sparse, const uint64_t *sparse_bits, tnc_precision prec, int32_t max_slices_in_flight,
                       tnc_plan **out) {
    API_BEGIN
    REQUIRE(out, "out is NULL");
    *out = nullptr;
    REQUIRE(ctx && net, "ctx or net is NULL");
    REQUIRE(n_steps == 0 || ssa_pairs, "ssa_pairs is NULL");
    REQUIRE(n_sliced == 0 || sliced_labels, "sliced_labels is NULL");
    REQUIRE(n_recompute == 0 || recompute_labels, "recompute_labels is NULL");
    REQUIRE(n_open == 0 || open_qubits, "open_qubits is NULL");
    auto *p = new tnc_plan;
    p->ctx = ctx;
    try {
        // a sparse-state plan keeps every output label (none is closed on the host)
        std::vector<int32_t> all_q;
        if (sparse_bits)
            for (int q = 0; q < net->net.n_qubits; q++) all_q.push_back(q);
        Simplified sp = presimplify(net->net, n_steps, ssa_pairs, n_sliced, sliced_labels,
                                    sparse_bits ? (int)all_q.size() : n_open, sparse_bits ? all_q.data() : open_qubits,
                                    host_rank_cap(), n_recompute, recompute_labels);
        p->plan_step_of = sp.plan_step_of;
        p->host_steps = sp.host_steps;
        p->an = analyze(sp.net, (int)sp.ssa.size() / 2, sp.ssa.data(), n_sliced, sliced_labels, n_open, open_qubits,
                        prec, n_recompute, recompute_labels, n_sparse, sparse_bits);
        if (sparse_bits) p->sparse_bits.assign(sparse_bits, sparse_bits + n_sparse);
        build_plan(p, sp.net, max_slices_in_flight);
        p->tune_seconds = autotune_plan(p);
    } catch (...) {
        free_plan_device(p);
        delete p;
        throw;
    }
    *out = p;
    API_END
}

extern "C" int tnc_plan_create_recompute(tnc_ctx *ctx, const tnc_network *net, int32_t n_steps,
                                         const int32_t *ssa_pairs, int32_t n_sliced, const int32_t *sliced_labels,
                                         int32_t n_recompute, const int32_t *recompute_labels, int32_t n_open,
                                         const int32_t *open_qubits, tnc_precision prec, int32_t max_slices_in_flight,
                                         tnc_plan **out) {
    return create_plan(ctx, net, n_steps, ssa_pairs, n_sliced, sliced_labels, n_recompute, recompute_labels, n_open,
                       open_qubits, 0, nullptr, prec, max_slices_in_flight, out);
}

extern "C" int tnc_plan_create_sparse(tnc_ctx *ctx, const tnc_network *net, int32_t n_steps, const int32_t *ssa_pairs,
                                      int32_t n_sliced, const int32_t *sliced_labels, int64_t n_bitstrings,
                                      const uint64_t *bitstrings, tnc_precision prec, int32_t max_slices_in_flight,
                                      tnc_plan **out) {
    if (n_bitstrings < 1 || !bitstrings) {
        set_error("a sparse-state plan needs at least one bitstring");
        return TNC_EINVAL;
    }
    return create_plan(ctx, net, n_steps, ssa_pairs, n_sliced, sliced_labels, 0, nullptr, 0, nullptr, n_bitstrings,
                       bitstrings, prec, max_slices_in_flight, out);
}

extern "C" int tnc_plan_create(tnc_ctx *ctx, const tnc_network *net, int32_t n_steps, const int32_t *ssa_pairs,
                               int32_t n_sliced, const int32_t *sliced_labels, int32_t n_open,
                               const int32_t *open_qubits, tnc_precision prec, int32_t max_slices_in_flight,
                               tnc_plan **out) {
    return tnc_plan_create_recompute(ctx, net, n_steps, ssa_pairs, n_sliced, sliced_labels, 0, nullptr, n_open,
                                     open_qubits, prec, max_slices_in_flight, out);
}

extern "C" int tnc_plan_destroy(tnc_plan *plan) {
    API_BEGIN
    if (!plan) return TNC_OK;
    hipSetDevice(plan->ctx->device);
    free_plan_device(plan);
    delete plan;
    API_END
}

extern "C" int tnc_plan_info(const tnc_plan *plan, tnc_plan_stats *stats) {
    API_BEGIN
    REQUIRE(plan && stats, "NULL argument");
    fill_stats(plan->an, *stats);
    stats->n_host_steps = plan->host_steps;
    stats->slices_in_flight = plan->S;
    stats->peak_bytes = (double)plan->peak;
    stats->tune_seconds = plan->tune_seconds;
    API_END
}

extern "C" int tnc_plan_analyze_recompute(const tnc_network *net, int32_t n_steps, const int32_t *ssa_pairs,
                                          int32_t n_sliced, const int32_t *sliced_labels, int32_t n_recompute,
                                          const int32_t *recompute_labels, int32_t n_open, const int32_t *open_qubits,
                                          tnc_precision prec, tnc_plan_stats *stats) {
    API_BEGIN
    REQUIRE(net && stats, "NULL argument");
    REQUIRE(n_steps == 0 || ssa_pairs, "ssa_pairs is NULL");
    REQUIRE(n_recompute == 0 || recompute_labels, "recompute_labels is NULL");
    Simplified sp = presimplify(net->net, n_steps, ssa_pairs, n_sliced, sliced_labels, n_open, open_qubits,
                                host_rank_cap(), n_recompute, recompute_labels);
    Analysis an = analyze(sp.net, (int)sp.ssa.size() / 2, sp.ssa.data(), n_sliced, sliced_labels, n_open, open_qubits,
                          prec, n_recompute, recompute_labels);
    fill_stats(an, *stats);
    stats->n_host_steps = sp.host_steps;
    stats->slices_in_flight = 0;
    stats->peak_bytes = (double)plan_memory(an, 1, false);
    API_END
}

extern "C" int tnc_plan_analyze_sparse(const tnc_network *net, int32_t n_steps, const int32_t *ssa_pairs,
                                       int32_t n_sliced, const int32_t *sliced_labels, int64_t n_bitstrings,
                                       const uint64_t *bitstrings, tnc_precision prec, tnc_plan_stats *stats) {
    API_BEGIN
    REQUIRE(net && stats, "NULL argument");
    REQUIRE(n_steps == 0 || ssa_pairs, "ssa_pairs is NULL");
    REQUIRE(n_bitstrings >= 1 && bitstrings, "a sparse-state plan needs at least one bitstring");
    std::vector<int32_t> all_q;
    for (int q = 0; q < net->net.n_qubits; q++) all_q.push_back(q);
    Simplified sp = presimplify(net->net, n_steps, ssa_pairs, n_sliced, sliced_labels, (int)all_q.size(), all_q.data(),
                                host_rank_cap());
    Analysis an = analyze(sp.net, (int)sp.ssa.size() / 2, sp.ssa.data(), n_sliced, sliced_labels, 0, nullptr, prec, 0,
                          nullptr, n_bitstrings, bitstrings);
    fill_stats(an, *stats);
    stats->n_host_steps = sp.host_steps;
    stats->slices_in_flight = 0;
    stats->peak_bytes = (double)plan_memory(an, 1, false);
    API_END
}

extern "C" int tnc_plan_analyze(const tnc_network *net, int32_t n_steps, const int32_t *ssa_pairs, int32_t n_sliced,
                                const int32_t *sliced_labels, int32_t n_open, const int32_t *open_qubits,
                                tnc_precision prec, tnc_plan_stats *stats) {
    return tnc_plan_analyze_recompute(net, n_steps, ssa_pairs, n_sliced, sliced_labels, 0, nullptr, n_open,
                                      open_qubits, prec, stats);
}

extern "C" int tnc_recompute_path(const tnc_network *net, int32_t n_steps, const int32_t *ssa_pairs,
                                  int32_t n_sliced, const int32_t *sliced_labels, int32_t n_open,
                                  const int32_t *open_qubits, double log2_cap, int32_t max_recompute,
                                  int32_t *recompute_out, int32_t *n_out) {
    API_BEGIN
    REQUIRE(net && n_out && (max_recompute == 0 || recompute_out), "NULL argument");
    REQUIRE(n_steps == 0 || ssa_pairs, "ssa_pairs is NULL");
    REQUIRE(max_recompute >= 0 && max_recompute <= 8, "max_recompute out of [0, 8]");
    // Greedy, as the slicer: while a tensor of one pass has more than 2^cap
    // entries, recompute the label of a largest tensor whose suffix adds the
    // least work over all passes.
    std::vector<int32_t> rec;
    auto eval = [&](const std::vector<int32_t> &r, Analysis *keep) {
        Simplified sp = presimplify(net->net, n_steps, ssa_pairs, n_sliced, sliced_labels, n_open, open_qubits,
                                    host_rank_cap(), (int)r.size(), r.data());
        Analysis an = analyze(sp.net, (int)sp.ssa.size() / 2, sp.ssa.data(), n_sliced, sliced_labels, n_open,
                              open_qubits, TNC_F16_4M, (int)r.size(), r.data());
        if (keep) *keep = std::move(an);
        else {
            tnc_plan_stats st;
            fill_stats(an, st);
            return st.flops_per_slice;
        }
        return 0.0;
    };
    std::vector<char> is_out(net->net.n_labels, 0);
    for (int l : net->net.output_labels) is_out[l] = 1;
    for (;;) {
        Analysis an;
        eval(rec, &an);
        int mr = 0;
        for (const auto &t : an.tensors) mr = std::max(mr, t.rank());
        if (mr <= log2_cap) break;
        if ((int)rec.size() >= max_recompute)
            TNC_THROW(TNC_EINVAL, "the cap needs more than max_recompute recomputed labels");
        std::vector<int> cand;
        for (const auto &t : an.tensors)
            if (t.rank() == mr)
                for (int l : t.labels)
                    if (!is_out[l] && std::find(cand.begin(), cand.end(), l) == cand.end()) cand.push_back(l);
        double best = 1e300;
        int bl = -1;
        for (int l : cand) {
            std::vector<int32_t> r = rec;
            r.push_back(l);
            const double f = eval(r, nullptr);
            if (f < best) {
                best = f;
                bl = l;
            }
        }
        if (bl < 0) TNC_THROW(TNC_EINVAL, "no label of the largest tensor can be recomputed");
        rec.push_back(bl);
    }
    std::copy(rec.begin(), rec.end(), recompute_out);
    *n_out = (int)rec.size();
    API_END
}

// ------------------------------------------------------------------ execution

namespace {

struct StepLaunch {
    const tnc_plan *p;
    hipStream_t st;
};

struct StepTimer {
    hipEvent_t e[3];
};

// Enqueue the permutes and the GEMM of step s for S slices; with a timer,
// events bracket the permutes and the GEMM.
void enqueue_step(tnc_plan *p, int s, int S_g, hipStream_t st, StepTimer *tm = nullptr) {
    const Analysis &an = p->an;
    const StepRec &rec = an.steps[s];
    const TensorRec &A = an.tensors[rec.a], &B = an.tensors[rec.b], &Z = an.tensors[rec.z];
    uint8_t *ws = p->ctx->ws;
    const Dtype dt = an.dt;
    const int es = elem_bytes(dt);
    const int Sl = rec.dep ? S_g : 1;
    const int64_t nz = (int64_t)1 << Z.rank();
    const void *pa = ws + A.off;
    const void *pb = ws + B.off;
    if (tm) HIP_CHECK(hipEventRecord(tm->e[0], st));
    if (rec.perm_a) {
        if (!rec.hoist_a) permute_operand(p, A, rec.a_from, ws + A.off, ws + rec.scr_a, A.dep ? S_g : 1, st);
        pa = ws + rec.scr_a;
    }
    if (rec.perm_b) {
        if (!rec.hoist_b) permute_operand(p, B, rec.b_from, ws + B.off, ws + rec.scr_b, B.dep ? S_g : 1, st);
        pb = ws + rec.scr_b;
    }
    GemmShape g = plan_step_shape(p, s);
    (void)es;
    ScaleRefs sc{};
    if (dt != Dtype::C64) {
        const int S = p->S;
        sc.maxA = p->d_maxw + (int64_t)rec.a * S;
        sc.mA = A.dep ? 1 : 0;
        sc.maxB = p->d_maxw + (int64_t)rec.b * S;
        sc.mB = B.dep ? 1 : 0;
        sc.maxC = p->d_maxw + (int64_t)rec.z * S;
        sc.expA = p->d_expw + (int64_t)rec.a * S;
        sc.eA = sc.mA;
        sc.expB = p->d_expw + (int64_t)rec.b * S;
        sc.eB = sc.mB;
        sc.expC = p->d_expw + (int64_t)rec.z * S;
        sc.shift = p->d_shift + (int64_t)rec.z * S;
        sc.growth = p->d_growth + s;
        sc.flag = p->d_flags + s;
    }
    if (tm) HIP_CHECK(hipEventRecord(tm->e[1], st));
    if (rec.scheme == 2) {
        // second sparse-state scheme, a chunk of A blocks at a time: B_P from
        // B's blocks (index -1: zeros), the GEMM into C_P, C's blocks out of C_P
        const int64_t nbb = (int64_t)1 << B.rank(), na = (int64_t)1 << A.rank();
        for (int64_t a0 = 0; a0 < A.nd; a0 += rec.chunk) {
            const int64_t nbc = std::min<int64_t>(rec.chunk, A.nd - a0);
            launch_block_copy(dt, pb, B.dep ? nbb * B.nd : 0, ws + rec.scr_bp, g.sB, p->d_idx + p->bp_idx_off[s] + a0 * rec.mr,
                              nbc * rec.mr, 0, B.nd, nbb, Sl, true, st);
            GemmShape gc = g;
            gc.nb = nbc;
            launch_gemm(rec.kernel, dt, an.al, (const uint8_t *)pa + a0 * na * es, ws + rec.scr_bp, ws + rec.scr_cp, gc,
                        Sl, dt != Dtype::C64 ? &sc : nullptr, st);
            launch_block_copy(dt, ws + rec.scr_cp, g.sC, ws + Z.off, nz * Z.nd, p->d_idx + p->cp_idx_off[s], Z.nd,
                              a0 * rec.mr, (a0 + nbc) * rec.mr, nz, Sl, false, st);
        }
    } else {
        launch_gemm(rec.kernel, dt, an.al, pa, pb, ws + Z.off, g, Sl, dt != Dtype::C64 ? &sc : nullptr, st);
    }
    if (s == p->codec_step) {
        // the result of this step passes through the exchange codec, one
        // slice at a time, as if it were sent to another device
        for (int q = 0; q < Sl; q++) {
            float *zr = (float *)(ws + Z.off) + (int64_t)q * 2 * nz;
            launch_quantize(p->codec_kind, 2 * nz, p->codec_group, zr, p->d_codes, p->d_qscale, p->d_qzero,
                            (float2 *)p->ctx->small, st);
            launch_dequantize(p->codec_kind, 2 * nz, p->codec_group, p->d_codes, p->d_qscale, p->d_qzero, zr, st);
        }
    }
    if (tm) HIP_CHECK(hipEventRecord(tm->e[2], st));
}

// The whole slice block: invariant phase, then every group of slices.
void enqueue_block(tnc_plan *p, int64_t nsl, int64_t nbits, hipStream_t st, bool timed) {
    const Analysis &an = p->an;
    const int S = p->S;
    const Dtype dt = an.dt;
    const int64_t nslots = (int64_t)an.tensors.size() * S;
    launch_fill_f64(p->d_acc, 0.0, 2 * nbits, st);
    if (dt != Dtype::C64) launch_fill_u32(p->d_maxw, 0u, nslots, st);
    launch_gather_leaves_impl(dt, p->n_inv_leaves, p->d_desc, p->d_params, p->d_leafdata, p->ctx->ws, p->d_maxw,
                              p->d_expw, 0, 1, st, p->d_spoff, p->nd_max);
    StepTimer tm{};
    if (timed)
        for (auto &e : tm.e) HIP_CHECK(hipEventCreate(&e));
    auto run = [&](int s, int S_g) {
        enqueue_step(p, s, S_g, st, timed ? &tm : nullptr);
        if (timed) {
            HIP_CHECK(hipEventSynchronize(tm.e[2]));
            float a = 0, b = 0;
            HIP_CHECK(hipEventElapsedTime(&a, tm.e[0], tm.e[1]));
            HIP_CHECK(hipEventElapsedTime(&b, tm.e[1], tm.e[2]));
            p->perm_ms[s] += a;
            p->step_ms[s] += b;
            p->step_launches[s] += 1;
        }
    };
    for (int s = 0; s < (int)an.steps.size(); s++)
        if (!an.steps[s].dep) run(s, 1);
    // permuted copies of invariant operands of dependent steps, once per call
    for (int s = 0; s < (int)an.steps.size(); s++) {
        const StepRec &rec = an.steps[s];
        uint8_t *ws = p->ctx->ws;
        if (rec.hoist_a) permute_operand(p, an.tensors[rec.a], rec.a_from, ws + an.tensors[rec.a].off, ws + rec.scr_a, 1, st);
        if (rec.hoist_b) permute_operand(p, an.tensors[rec.b], rec.b_from, ws + an.tensors[rec.b].off, ws + rec.scr_b, 1, st);
    }
    const TensorRec &R = an.tensors[an.root];
    const int n_outer_leaves = p->n_dep_leaves - p->n_inner_leaves;
    const int64_t passes = (int64_t)1 << an.n_recompute;
    for (int64_t g0 = 0; g0 < nsl; g0 += S) {
        const int S_g = (int)std::min<int64_t>(S, nsl - g0);
        if (dt != Dtype::C64 && g0 > 0) {
            // clear the dependent max words of the previous group
            for (size_t t = 0; t < an.tensors.size(); t++)
                if (an.tensors[t].dep) launch_fill_u32(p->d_maxw + (int64_t)t * S, 0u, S, st);
        }
        // the slice prefix: once per group
        launch_gather_leaves_impl(dt, n_outer_leaves, p->d_desc + p->n_inv_leaves, p->d_params, p->d_leafdata,
                                  p->ctx->ws, p->d_maxw, p->d_expw, g0, S_g, st, p->d_spoff, p->nd_max);
        for (int s = 0; s < (int)an.steps.size(); s++)
            if (an.steps[s].dep && !an.steps[s].inner) run(s, S_g);
        // the recomputed suffix: once per pass; a pass's recomputed label
        // values are the slice id bits above the sliced ones (the group's
        // slice ids stay below 2^n_sliced, so adding them carries nothing)
        for (int64_t pass = 0; pass < passes; pass++) {
            if (dt != Dtype::C64 && pass > 0)
                for (size_t t = 0; t < an.tensors.size(); t++)
                    if (an.tensors[t].inner) launch_fill_u32(p->d_maxw + (int64_t)t * S, 0u, S, st);
            launch_gather_leaves_impl(dt, p->n_inner_leaves, p->d_desc + p->n_inv_leaves + n_outer_leaves, p->d_params,
                                      p->d_leafdata, p->ctx->ws, p->d_maxw, p->d_expw,
                                      g0 + (pass << an.n_sliced), S_g, st, p->d_spoff, p->nd_max);
            for (int s = 0; s < (int)an.steps.size(); s++)
                if (an.steps[s].inner) run(s, S_g);
            launch_accumulate(dt, p->ctx->ws + R.off, R.rank(), S_g, ((int64_t)1 << R.rank()) * R.nd,
                              dt == Dtype::C64 ? nullptr : p->d_expw + (int64_t)an.root * S, 1, nbits, p->d_bits,
                              p->d_qob, p->d_acc, st, p->d_map);
        }
    }
    if (timed)
        for (auto &e : tm.e) hipEventDestroy(e);
}

}  // namespace

extern "C" int tnc_plan_set_codec(tnc_plan *plan, int32_t step, int32_t kind, int32_t group) {
    API_BEGIN
    REQUIRE(plan, "plan is NULL");
    REQUIRE(step >= -1 && step < (int)plan->plan_step_of.size(), "step out of range");
    if (step >= 0) {
        if (plan->plan_step_of[step] < 0)
            TNC_THROW(TNC_EUNSUPPORTED, "step " + std::to_string(step) + " is pre-contracted on the host");
        step = plan->plan_step_of[step];
    }
    if (step >= 0 && plan->an.dt != Dtype::C64)
        TNC_THROW(TNC_EUNSUPPORTED, "the codec round trip applies to complex64 plans (float32 values)");
    if (step >= 0 && plan->an.sparse) TNC_THROW(TNC_EUNSUPPORTED, "the codec round trip applies to dense plans");
    int64_t cb = 0, ng = 0;
    if (step >= 0) {
        // per-slice results sit nz complex values apart; the codec's vector
        // loads need each slice 16-byte aligned, so nz >= 2
        const int rz = plan->an.tensors[plan->an.steps[step].z].rank();
        if (rz < 1) TNC_THROW(TNC_EUNSUPPORTED, "the codec round trip needs a result of rank >= 1");
        const int64_t n = 2 * ((int64_t)1 << rz);
        int rc = tnc_quant_sizes(kind, n, group, &cb, &ng);
        if (rc != TNC_OK) return rc;
    }
    HIP_CHECK(hipSetDevice(plan->ctx->device));
    HIP_CHECK(hipStreamSynchronize(plan->ctx->stream));
    for (auto &kv : plan->graphs) hipGraphExecDestroy(kv.second);
    plan->graphs.clear();
    for (void *q : {(void *)plan->d_codes, (void *)plan->d_qscale, (void *)plan->d_qzero})
        if (q) HIP_CHECK(hipFree(q));
    plan->d_codes = nullptr;
    plan->d_qscale = plan->d_qzero = nullptr;
    plan->codec_step = step;
    plan->codec_kind = kind;
    plan->codec_group = kind == TNC_Q_INT4 && group == 0 ? 128 : group;
    if (step >= 0) {
        plan->d_codes = dev_alloc<uint8_t>(cb + 16);
        plan->d_qscale = dev_alloc<float>(ng);
        plan->d_qzero = dev_alloc<float>(ng);
    }
    API_END
}

extern "C" int tnc_plan_set_timing(tnc_plan *plan, int32_t on) {
    API_BEGIN
    REQUIRE(plan, "plan is NULL");
    plan->timing = on != 0;
    API_END
}

extern "C" int tnc_plan_step_times(const tnc_plan *plan, int32_t n_steps, double *gemm_ms, double *permute_ms,
                                   int32_t *launches) {
    API_BEGIN
    REQUIRE(plan, "plan is NULL");
    REQUIRE(n_steps >= (int)plan->step_ms.size(), "arrays too small");
    for (size_t i = 0; i < plan->step_ms.size(); i++) {
        if (gemm_ms) gemm_ms[i] = plan->step_ms[i];
        if (permute_ms) permute_ms[i] = plan->perm_ms[i];
        if (launches) launches[i] = plan->step_launches[i];
    }
    API_END
}

static void describe_steps(const Analysis &an, int32_t n_steps, int32_t *log2_mnkb, int32_t *kernel, int32_t *dep,
                           int32_t *perm_ab, double *flops, double *bytes) {
    const auto &st = an.steps;
    if (n_steps < (int)st.size()) TNC_THROW(TNC_EINVAL, "arrays too small");
    for (size_t i = 0; i < st.size(); i++) {
        const StepRec &r = st[i];
        if (log2_mnkb) {
            log2_mnkb[4 * i] = (int)r.m.size();
            log2_mnkb[4 * i + 1] = (int)r.n.size();
            log2_mnkb[4 * i + 2] = (int)r.k.size();
            log2_mnkb[4 * i + 3] = (int)r.beta.size();
        }
        if (kernel) kernel[i] = r.kernel;
        if (dep) dep[i] = r.dep ? 1 : 0;
        if (perm_ab) {   // operand stride class: 0 in place [m][k], 1 in place [k][m], 2 permuted
            perm_ab[2 * i] = r.perm_a ? 2 : (r.a_kc ? 0 : 1);
            perm_ab[2 * i + 1] = r.perm_b ? 2 : (r.b_kc ? 0 : 1);
        }
        if (flops) flops[i] = r.flops;
        if (bytes) bytes[i] = r.bytes;
    }
}

extern "C" int tnc_plan_steps(const tnc_plan *plan, int32_t n_steps, int32_t *log2_mnkb, int32_t *kernel, int32_t *dep,
                              int32_t *perm_ab, double *flops, double *bytes) {
    API_BEGIN
    REQUIRE(plan, "plan is NULL");
    describe_steps(plan->an, n_steps, log2_mnkb, kernel, dep, perm_ab, flops, bytes);
    API_END
}

extern "C" int tnc_plan_analyze_steps(const tnc_network *net, int32_t n_steps, const int32_t *ssa_pairs,
                                      int32_t n_sliced, const int32_t *sliced_labels, int32_t n_open,
                                      const int32_t *open_qubits, tnc_precision prec, int32_t *log2_mnkb,
                                      int32_t *kernel, int32_t *dep, int32_t *perm_ab, double *flops, double *bytes) {
    API_BEGIN
    REQUIRE(net, "net is NULL");
    REQUIRE(n_steps == 0 || ssa_pairs, "ssa_pairs is NULL");
    Simplified sp = presimplify(net->net, n_steps, ssa_pairs, n_sliced, sliced_labels, n_open, open_qubits,
                                host_rank_cap());
    Analysis an = analyze(sp.net, (int)sp.ssa.size() / 2, sp.ssa.data(), n_sliced, sliced_labels, n_open, open_qubits,
                          prec);
    describe_steps(an, n_steps, log2_mnkb, kernel, dep, perm_ab, flops, bytes);
    API_END
}

namespace {

// floor(log2 x) of a positive finite float, as the device takes it (frexp)
int floor_log2_host(float x) {
    int e = 0;
    std::frexp(x, &e);
    return e - 1;
}

// Growth estimates for the next call, from the slices of the last group.  A
// step stores C * 2^-t with t = floor(log2 mA) + floor(log2 mB) + g - target
// (mA, mB: its operands' stored maxima), so its stored maximum mC tells the
// realized growth
//     gamma = log2 mC + t - floor(log2 mA) - floor(log2 mB),
// the estimate that would have put mC at 2^target exactly.  Each step keeps
// ceil(max gamma) over the group's slices: the estimate narrows when a step
// grows less than planned, and widens again after a replay.
void adapt_growth(tnc_plan *p, int S_last) {
    const Analysis &an = p->an;
    const int S = p->S;
    const int64_t nslots = (int64_t)an.tensors.size() * S;
    std::vector<uint32_t> mw(nslots);
    std::vector<int> sh(nslots);
    HIP_CHECK(hipMemcpy(mw.data(), p->d_maxw, sizeof(uint32_t) * nslots, hipMemcpyDeviceToHost));
    HIP_CHECK(hipMemcpy(sh.data(), p->d_shift, sizeof(int) * nslots, hipMemcpyDeviceToHost));
    auto val = [&](int t, int q) {
        float f;
        std::memcpy(&f, &mw[(int64_t)t * S + q], 4);
        return f;
    };
    bool changed = false;
    for (size_t s = 0; s < an.steps.size(); s++) {
        const StepRec &rec = an.steps[s];
        const bool da = an.tensors[rec.a].dep, db = an.tensors[rec.b].dep;
        const int Sl = rec.dep ? S_last : 1;
        double gmax = -1e300;
        for (int q = 0; q < Sl; q++) {
            const float ma = val(rec.a, da ? q : 0), mb = val(rec.b, db ? q : 0), mc = val(rec.z, q);
            if (!(ma > 0.f && mb > 0.f && mc > 0.f) || !(ma <= 3.0e38f && mb <= 3.0e38f && mc <= 3.0e38f)) continue;
            const int t = sh[(int64_t)rec.z * S + q];
            const double gam = std::log2((double)mc) + t - floor_log2_host(ma) - floor_log2_host(mb);
            gmax = std::max(gmax, gam);
        }
        if (gmax < -1e299) continue;
        const int g = (int)std::max(-64.0, std::min(64.0, std::ceil(gmax - 1e-9)));
        if (g != p->h_growth[s]) {
            p->h_growth[s] = g;
            changed = true;
        }
    }
    if (changed)
        HIP_CHECK(hipMemcpyAsync(p->d_growth, p->h_growth.data(), sizeof(int) * p->h_growth.size(),
                                 hipMemcpyHostToDevice, p->ctx->stream));
}

}  // namespace

extern "C" int tnc_plan_get_growth(const tnc_plan *plan, int32_t n_steps, int32_t *growth) {
    API_BEGIN
    REQUIRE(plan && growth, "NULL argument");
    REQUIRE(n_steps >= (int)plan->h_growth.size(), "array too small");
    for (size_t s = 0; s < plan->h_growth.size(); s++) growth[s] = plan->h_growth[s];
    API_END
}

extern "C" int tnc_plan_set_growth(tnc_plan *plan, int32_t n_steps, const int32_t *growth) {
    API_BEGIN
    REQUIRE(plan && growth, "NULL argument");
    REQUIRE(n_steps == (int)plan->h_growth.size(), "n_steps must equal the plan's step count");
    for (int s = 0; s < n_steps; s++) REQUIRE(growth[s] >= -64 && growth[s] <= 64, "growth out of [-64, 64]");
    REQUIRE(plan->an.dt != Dtype::C64, "complex64 plans keep no scale exponents");
    HIP_CHECK(hipSetDevice(plan->ctx->device));
    for (int s = 0; s < n_steps; s++) plan->h_growth[s] = growth[s];
    HIP_CHECK(hipMemcpyAsync(plan->d_growth, plan->h_growth.data(), sizeof(int) * n_steps, hipMemcpyHostToDevice,
                             plan->ctx->stream));
    HIP_CHECK(hipStreamSynchronize(plan->ctx->stream));
    API_END
}

extern "C" int tnc_execute(tnc_plan *p, int64_t n_bitstrings, const uint64_t *bitstrings, int64_t slice_begin,
                           int64_t slice_end, double *out_c128, tnc_report *rep) {
    API_BEGIN
    REQUIRE(p, "plan is NULL");
    REQUIRE(n_bitstrings >= 0, "n_bitstrings < 0");
    REQUIRE(n_bitstrings == 0 || (bitstrings && out_c128), "bitstrings or out_c128 is NULL");
    const Analysis &an = p->an;
    const int64_t total = (int64_t)1 << an.n_sliced;
    REQUIRE(slice_begin >= 0 && slice_begin <= slice_end && slice_end <= total, "slice range out of [0, 2^n_sliced]");
    tnc_ctx *ctx = p->ctx;
    HIP_CHECK(hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    if (rep) *rep = tnc_report{};
    const int64_t nsl = slice_end - slice_begin;
    if (n_bitstrings == 0) return TNC_OK;
    if (an.sparse) {
        // a sparse-state plan computes the blocks of the bitstrings it was made for
        REQUIRE(n_bitstrings == (int64_t)p->sparse_bits.size() &&
                    std::equal(bitstrings, bitstrings + n_bitstrings, p->sparse_bits.begin()),
                "a sparse-state plan takes exactly the bitstrings it was created with");
    }
    // closed qubits: values must agree across the request
    std::vector<int> closed_val(p->n_qubits, 0);
    for (int q : p->closed_qubits) {
        int v = (int)((bitstrings[0] >> q) & 1ull);
        for (int64_t j = 1; j < n_bitstrings; j++)
            if ((int)((bitstrings[j] >> q) & 1ull) != v)
                TNC_THROW(TNC_EINVAL, "bitstrings disagree on closed qubit " + std::to_string(q));
        closed_val[q] = v;
    }
    bool desc_dirty = false;
    for (int i = 0; i < p->nT; i++) {
        const auto &orig = p->leaf_orig_labels[i];
        int64_t off = 0;
        const int ro = (int)orig.size();
        for (int j = 0; j < ro; j++) {
            int l = orig[j];
            if (an.fixed[l] == 1) {
                // a closed output label: the value of its qubit selects the half
                int q = -1;
                for (int qq : p->closed_qubits)
                    if (p->output_labels[qq] == l) q = qq;
                if (q >= 0 && closed_val[q]) off += (int64_t)1 << (ro - 1 - j);
            }
        }
        if (off != p->closed_state[i]) {
            p->closed_state[i] = off;
            p->h_desc[p->desc_of_leaf[i]].closed_off = off;
            desc_dirty = true;
        }
    }
    if (desc_dirty)
        HIP_CHECK(hipMemcpyAsync(p->d_desc, p->h_desc.data(), sizeof(LeafDesc) * p->h_desc.size(),
                                 hipMemcpyHostToDevice, st));
    if (n_bitstrings > p->bits_cap) {
        if (p->d_bits) hipFree(p->d_bits);
        if (p->d_acc) hipFree(p->d_acc);
        p->d_bits = nullptr;
        p->d_acc = nullptr;
        for (auto &kv : p->graphs) hipGraphExecDestroy(kv.second);
        p->graphs.clear();
        p->d_bits = dev_alloc<uint64_t>(n_bitstrings);
        p->d_acc = dev_alloc<double>(2 * n_bitstrings);
        p->bits_cap = n_bitstrings;
    }
    HIP_CHECK(hipMemcpyAsync(p->d_bits, bitstrings, sizeof(uint64_t) * n_bitstrings, hipMemcpyHostToDevice, st));
    int64_t params[4] = {slice_begin, 0, 0, 0};
    HIP_CHECK(hipMemcpyAsync(p->d_params, params, sizeof(params), hipMemcpyHostToDevice, st));

    const int ns = (int)an.steps.size();
    // overflow flags start clear (a call that ended in TNC_EOVERFLOW leaves them set)
    if (an.dt != Dtype::C64) launch_fill_u32(p->d_flags, 0u, ns, st);
    hipEvent_t ev0, ev1;
    HIP_CHECK(hipEventCreate(&ev0));
    HIP_CHECK(hipEventCreate(&ev1));
    int replays = 0, launches = 0;
    float ms = 0.f;
    for (;;) {
        if (p->timing) {
            std::fill(p->step_ms.begin(), p->step_ms.end(), 0.0);
            std::fill(p->perm_ms.begin(), p->perm_ms.end(), 0.0);
            std::fill(p->step_launches.begin(), p->step_launches.end(), 0);
        }
        bool graph = p->use_graph && !p->timing;
        if (graph) {
            auto key = std::make_tuple(nsl, n_bitstrings, (const void *)p->d_bits);
            auto it = p->graphs.find(key);
            if (it == p->graphs.end()) {
                hipGraph_t gr;
                HIP_CHECK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
                try {
                    enqueue_block(p, nsl, n_bitstrings, st, false);
                } catch (...) {
                    hipStreamEndCapture(st, &gr);
                    if (gr) hipGraphDestroy(gr);
                    throw;
                }
                HIP_CHECK(hipStreamEndCapture(st, &gr));
                hipGraphExec_t ex;
                HIP_CHECK(hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0));
                hipGraphDestroy(gr);
                it = p->graphs.emplace(key, ex).first;
            }
            HIP_CHECK(hipEventRecord(ev0, st));
            HIP_CHECK(hipGraphLaunch(it->second, st));
            HIP_CHECK(hipEventRecord(ev1, st));
            launches++;
        } else {
            HIP_CHECK(hipEventRecord(ev0, st));
            enqueue_block(p, nsl, n_bitstrings, st, p->timing);
            HIP_CHECK(hipEventRecord(ev1, st));
        }
        HIP_CHECK(hipEventSynchronize(ev1));
        float t = 0.f;
        HIP_CHECK(hipEventElapsedTime(&t, ev0, ev1));
        ms += t;
        if (an.dt == Dtype::C64) break;
        std::vector<uint32_t> flags(ns);
        HIP_CHECK(hipMemcpy(flags.data(), p->d_flags, sizeof(uint32_t) * ns, hipMemcpyDeviceToHost));
        bool any = false;
        for (int s = 0; s < ns; s++)
            if (flags[s]) {
                any = true;
                p->h_growth[s] += 4;
            }
        if (!any) {
            adapt_growth(p, nsl > 0 ? (int)(nsl - ((nsl - 1) / p->S) * p->S) : 0);
            break;
        }
        if (replays >= 3) {
            hipEventDestroy(ev0);
            hipEventDestroy(ev1);
            TNC_THROW(TNC_EOVERFLOW, "16-bit range exceeded after 3 rescale replays");
        }
        replays++;
        HIP_CHECK(hipMemcpyAsync(p->d_growth, p->h_growth.data(), sizeof(int) * ns, hipMemcpyHostToDevice, st));
        launch_fill_u32(p->d_flags, 0u, ns, st);
    }
    hipEventDestroy(ev0);
    hipEventDestroy(ev1);
    HIP_CHECK(hipMemcpyAsync(out_c128, p->d_acc, sizeof(double) * 2 * n_bitstrings, hipMemcpyDefault, st));
    HIP_CHECK(hipStreamSynchronize(st));
    if (rep) {
        double fl = 0;
        const double passes = std::ldexp(1.0, an.n_recompute);
        for (auto &s : an.steps) fl += s.dep ? s.flops * (double)nsl * (s.inner ? passes : 1.0) : s.flops;
        rep->seconds = ms * 1e-3;
        rep->flops = fl;
        rep->slices = nsl;
        rep->replays = replays;
        rep->graph_launches = launches;
    }
    API_END
}
