// Host planner.  For every pairwise step of the path it classifies labels
// (paper Sec. 3.3: a pairwise einsum is a pure GEMM when the reduced labels
// are exactly the labels both operands share and the result keeps the rest):
//   batch = in A, in B, kept;   m = A only, kept;   n = B only, kept;
//   k = in A and B, not kept (summed).
// It then picks storage orders so operands can be fed to the GEMM as
// [batch][m][k] and [batch][n][k] without a permute where possible, and
// lays out the arena.
#include <algorithm>
#include <cstdlib>
#include <cmath>
#include <numeric>

#include "planner.h"

namespace tnc {

static std::string lbl(int l) { return std::to_string(l); }

PermuteDesc make_permute(const std::vector<int> &from, const std::vector<int> &to) {
    PermuteDesc d{};
    const int r = (int)to.size();
    if (r > kMaxRank) TNC_THROW(TNC_EUNSUPPORTED, "tensor rank above 48");
    d.rank = r;
    const int rf = (int)from.size();
    for (int b = 0; b < r; b++) {
        int label = to[r - 1 - b];
        auto it = std::find(from.begin(), from.end(), label);
        if (it == from.end()) TNC_THROW(TNC_EINVAL, "internal: permute label missing");
        int pos = rf - 1 - (int)(it - from.begin());
        d.src_stride[b] = (int64_t)1 << pos;
    }
    return d;
}

bool plan_tile_bits(const PermuteDesc &d, int lw, int nt_max, TileBits &tb) {
    const int r = d.rank;
    if (r < lw + 1) return false;
    bool in_t[kMaxRank] = {false};
    for (int b = 0; b < lw; b++) in_t[b] = true;
    int nsrc = 0;
    for (int b = 0; b < r; b++)
        if (d.src_stride[b] < ((int64_t)1 << lw)) {
            in_t[b] = true;
            nsrc++;
        }
    if (nsrc != lw) return false;   // the lowest source bits are not all destination bits
    int nt = 0;
    for (int b = 0; b < r; b++) nt += in_t[b];
    if (nt > nt_max) return false;
    // grow T to nt_max bits, alternating the lowest destination bit and the
    // lowest source bit still outside it: every tile then keeps all threads
    // busy, and both HBM runs only get longer
    bool take_dst = true;
    while (nt < nt_max && nt < r) {
        int pick = -1;
        if (take_dst) {
            for (int b = 0; b < r && pick < 0; b++)
                if (!in_t[b]) pick = b;
        } else {
            for (int b = 0; b < r; b++)
                if (!in_t[b] && (pick < 0 || d.src_stride[b] < d.src_stride[pick])) pick = b;
        }
        in_t[pick] = true;
        nt++;
        take_dst = !take_dst;
    }
    tb.nt = 0;
    for (int b = 0; b < r; b++)
        if (in_t[b]) tb.dst_order[tb.nt++] = b;
    // source order of the tile bits: by source stride
    for (int i = 0; i < tb.nt; i++) tb.src_order[i] = tb.dst_order[i];
    std::sort(tb.src_order, tb.src_order + tb.nt, [&](int x, int y) { return d.src_stride[x] < d.src_stride[y]; });
    for (int i = 0; i < tb.nt; i++)
        for (int j = 0; j < tb.nt; j++)
            if (tb.dst_order[j] == tb.src_order[i]) tb.lds_bit[i] = j;
    tb.n_rest = 0;
    for (int b = 0; b < r; b++)
        if (!in_t[b]) tb.rest[tb.n_rest++] = b;
    return true;
}

static int ilog2_exact(int64_t v) {
    int b = 0;
    while (((int64_t)1 << b) < v) b++;
    if (((int64_t)1 << b) != v) TNC_THROW(TNC_EINVAL, "internal: GEMM extent is not a power of two");
    return b;
}

void set_plain_segs(GemmShape &g) {
    const int lm = ilog2_exact(g.M), ln = ilog2_exact(g.N), lk = ilog2_exact(g.K);
    g.am = g.a_kc ? Seg{62, lk, 0} : Seg{62, 0, 0};
    g.ak = g.a_kc ? Seg{62, 0, 0} : Seg{62, lm, 0};
    g.bn = g.b_kc ? Seg{62, lk, 0} : Seg{62, 0, 0};
    g.bk = g.b_kc ? Seg{62, 0, 0} : Seg{62, ln, 0};
    g.cm = g.c_nc ? Seg{62, ln, 0} : Seg{62, 0, 0};
    g.cn = g.c_nc ? Seg{62, 0, 0} : Seg{62, lm, 0};
}

// Segment of the index whose labels are `idx` (most significant first) in a
// tensor stored in `order` (most significant first); false if the labels are
// not in at most two runs of consecutive bits in index order.
bool derive_seg(const std::vector<int> &order, const std::vector<int> &idx, Seg &out) {
    const int r = (int)order.size(), n = (int)idx.size();
    out = Seg{};
    if (n == 0) return true;
    std::vector<int> bit(n);
    for (int j = 0; j < n; j++) {   // index bit j (0 = least significant) -> memory bit
        auto it = std::find(order.begin(), order.end(), idx[n - 1 - j]);
        if (it == order.end()) return false;
        bit[j] = r - 1 - (int)(it - order.begin());
    }
    int l = 1;
    while (l < n && bit[l] == bit[0] + l) l++;
    if (l == n) {
        out = Seg{62, bit[0], 0};
        return true;
    }
    for (int t = l + 1; t < n; t++)
        if (bit[t] != bit[l] + (t - l)) return false;
    out = Seg{l, bit[0], bit[l]};
    return true;
}

GemmShape step_gemm(const StepRec &st) {
    GemmShape g{st.M, st.N, st.K, st.nb, 0, 0, 0, st.M * st.K, st.N * st.K, st.M * st.N};
    g.a_kc = st.a_kc;
    g.b_kc = st.b_kc;
    g.c_nc = st.c_nc;
    g.am = st.am;
    g.ak = st.ak;
    g.bn = st.bn;
    g.bk = st.bk;
    g.cm = st.cm;
    g.cn = st.cn;
    return g;
}

GemmShape step_gemm_exec(const StepRec &st) {
    GemmShape g = step_gemm(st);
    if (st.scheme != 2) return g;
    // n' = r N + n: r is the top part of the column index in B_P and C_P,
    // whose blocks keep B's and C's own layouts
    const int ln = ilog2_exact(st.N);
    const int rb = ilog2_exact(st.N * st.K), rc = ilog2_exact(st.M * st.N);
    g.N = st.N * st.mr;
    g.nb = st.chunk;
    g.bA = st.M * st.K;
    g.bB = st.mr * st.N * st.K;
    g.bC = st.mr * st.M * st.N;
    g.bn = Seg{ln, st.bn.ls, rb};
    g.cn = Seg{ln, st.cn.ls, rc};
    return g;
}

// Does `order` read as [g0-block][g1-block][g2-block] (MSB first)?
static bool has_pattern(const std::vector<int> &order, const std::vector<int> &grp /* label -> group */,
                        const std::vector<int> &sizes) {
    int pos = 0;
    for (int gi = 0; gi < 3; gi++) {
        for (int c = 0; c < sizes[gi]; c++, pos++) {
            if (pos >= (int)order.size() || grp[order[pos]] != gi) return false;
        }
    }
    return pos == (int)order.size();
}

static std::vector<int> extract(const std::vector<int> &order, const std::vector<int> &grp, int gi) {
    std::vector<int> r;
    for (int l : order)
        if (grp[l] == gi) r.push_back(l);
    return r;
}

int choose_kernel(Dtype dt, Algo al, const GemmShape &g) {
    // largest matrix-core tile that divides the shape, once the step has
    // enough work for more than a handful of tiles; thin steps go to the VALU
    static const int order[] = {K_DMA_8, K_MFMA_XL, K_MFMA_L2, K_MFMA_L, K_MFMA_M, K_MFMA_W, K_MFMA_S};
    const double work = (double)g.M * (double)g.N * (double)g.K;
    if (work >= 1 << 18 && (g.N >= 16 || al == Algo::M3))
        for (int k : order)
            if (gemm_supported(k, dt, al, g)) return k;
    if (gemm_supported(K_SKINNY_N, dt, al, g)) return K_SKINNY_N;
    return K_NAIVE;
}

Analysis analyze(const Network &net, int n_steps, const int32_t *ssa, int n_sliced, const int32_t *sliced,
                 int n_open, const int32_t *open_q, tnc_precision prec, int n_recompute, const int32_t *recompute,
                 int64_t n_sparse, const uint64_t *sparse_bits) {
    Analysis an;
    an.dt = dtype_of(prec);
    an.al = algo_of(prec);
    if ((int)prec < 0 || (int)prec > 4) TNC_THROW(TNC_EINVAL, "unknown precision");
    if (an.dt == Dtype::C64 && an.al == Algo::M3) TNC_THROW(TNC_EINVAL, "3M needs 16-bit storage");
    const int nT = net.n_tensors;
    const int L = net.n_labels;
    if (n_steps != nT - 1) TNC_THROW(TNC_EINVAL, "path must have n_tensors - 1 steps");
    if (n_sliced < 0 || n_sliced > 62) TNC_THROW(TNC_EINVAL, "n_sliced out of range");
    if (n_recompute < 0 || n_recompute > 8 || n_sliced + n_recompute > 62)
        TNC_THROW(TNC_EINVAL, "n_recompute out of [0, 8] (or sliced + recomputed labels above 62)");
    if (n_recompute > 0 && !recompute) TNC_THROW(TNC_EINVAL, "recompute labels are NULL");
    if (n_open < 0 || n_open > net.n_qubits) TNC_THROW(TNC_EINVAL, "n_open out of range");

    an.fixed.assign(L, -1);
    an.slice_bit.assign(L, -1);
    an.open_qubit_of_label.assign(L, -1);
    std::vector<int> is_output(L, -1);
    for (int q = 0; q < net.n_qubits; q++) is_output[net.output_labels[q]] = q;
    std::vector<char> open(net.n_qubits, 0);
    for (int i = 0; i < n_open; i++) {
        int q = open_q[i];
        if (q < 0 || q >= net.n_qubits) TNC_THROW(TNC_EINVAL, "open qubit out of range");
        if (open[q]) TNC_THROW(TNC_EINVAL, "open qubit listed twice");
        open[q] = 1;
        an.open_qubit_of_label[net.output_labels[q]] = q;
    }
    for (int q = 0; q < net.n_qubits; q++)
        if (!open[q]) an.fixed[net.output_labels[q]] = 1;
    an.sparse = sparse_bits != nullptr;
    if (an.sparse) {
        if (n_open != 0) TNC_THROW(TNC_EINVAL, "a sparse-state plan takes no open qubits: every qubit follows the bitstrings");
        if (n_sparse < 1) TNC_THROW(TNC_EINVAL, "a sparse-state plan needs at least one bitstring");
        if (net.hyperedges) TNC_THROW(TNC_EUNSUPPORTED, "sparse-state plans take networks whose labels join two tensors");
    }
    for (int j = 0; j < n_sliced; j++) {
        int l = sliced[j];
        if (l < 0 || l >= L) TNC_THROW(TNC_EINVAL, "sliced label " + lbl(l) + " not in the network");
        if (is_output[l] >= 0) TNC_THROW(TNC_EINVAL, "sliced label " + lbl(l) + " is an output label");
        if (an.fixed[l] == 0) TNC_THROW(TNC_EINVAL, "sliced label " + lbl(l) + " listed twice");
        an.fixed[l] = 0;
        an.slice_bit[l] = j;
    }
    an.n_sliced = n_sliced;
    // recomputed labels: fixed per pass; a pass's values are the slice id
    // bits above the sliced ones
    std::vector<char> is_rec(L, 0);
    for (int j = 0; j < n_recompute; j++) {
        int l = recompute[j];
        if (l < 0 || l >= L) TNC_THROW(TNC_EINVAL, "recomputed label " + lbl(l) + " not in the network");
        if (is_output[l] >= 0) TNC_THROW(TNC_EINVAL, "recomputed label " + lbl(l) + " is an output label");
        if (an.fixed[l] == 0) TNC_THROW(TNC_EINVAL, "recomputed label " + lbl(l) + " is sliced or listed twice");
        an.fixed[l] = 0;
        an.slice_bit[l] = n_sliced + j;
        is_rec[l] = 1;
    }
    an.n_recompute = n_recompute;

    // input tensors with the fixed labels removed
    std::vector<int> needed(L, 0);
    an.tensors.resize(2 * nT - 1);
    for (int i = 0; i < nT; i++) {
        TensorRec &t = an.tensors[i];
        t.leaf = true;
        for (int l : net.labels[i]) {
            if (an.fixed[l] >= 0) {
                if (an.fixed[l] == 0) t.dep = true;
                if (is_rec[l]) t.inner = true;
                if (an.sparse && is_output[l] >= 0) t.sp_mask |= 1ull << is_output[l];
                continue;
            }
            t.labels.push_back(l);
            needed[l]++;
        }
        if (t.rank() > kMaxLeafRank) TNC_THROW(TNC_EUNSUPPORTED, "input tensor rank above 16 after slicing");
    }
    for (int q = 0; q < net.n_qubits; q++)
        if (open[q]) needed[net.output_labels[q]]++;
    if (n_sliced == 0)
        for (int i = 0; i < nT; i++) an.tensors[i].dep = true;

    // walk the path: label groups, dependence, consumers
    std::vector<char> alive(2 * nT - 1, 0);
    for (int i = 0; i < nT; i++) alive[i] = 1;
    std::vector<int> grp(L, -1);
    an.steps.resize(n_steps);
    for (int s = 0; s < n_steps; s++) {
        int x = ssa[2 * s], y = ssa[2 * s + 1];
        int z = nT + s;
        if (x < 0 || y < 0 || x >= z || y >= z || x == y) TNC_THROW(TNC_EINVAL, "path step " + lbl(s) + " has an invalid operand");
        if (!alive[x] || !alive[y]) TNC_THROW(TNC_EINVAL, "path step " + lbl(s) + " uses a tensor twice");
        alive[x] = alive[y] = 0;
        alive[z] = 1;
        StepRec &st = an.steps[s];
        st.x = x;
        st.y = y;
        st.z = z;
        TensorRec &X = an.tensors[x], &Y = an.tensors[y], &Z = an.tensors[z];
        X.consumer = s;
        Y.consumer = s;
        Z.producer = s;
        Z.dep = X.dep || Y.dep;
        Z.inner = X.inner || Y.inner;
        Z.sp_mask = X.sp_mask | Y.sp_mask;
        st.dep = Z.dep;
        st.inner = Z.inner;
        std::vector<char> inx(L, 0), iny(L, 0);
        for (int l : X.labels) inx[l] = 1;
        for (int l : Y.labels) iny[l] = 1;
        std::vector<int> uni;
        for (int l : X.labels) uni.push_back(l);
        for (int l : Y.labels)
            if (!inx[l]) uni.push_back(l);
        for (int l : uni) {
            int after = needed[l] - inx[l] - iny[l];
            bool keep = after > 0;
            needed[l] = after + (keep ? 1 : 0);
            if (keep) Z.labels.push_back(l);   // provisional order; fixed by the layout pass
            if (inx[l] && iny[l])
                (keep ? st.beta : st.k).push_back(l);
            else if (inx[l]) {
                if (!keep) TNC_THROW(TNC_EUNSUPPORTED, "label " + lbl(l) + " is summed inside one tensor");
                st.m.push_back(l);
            } else {
                if (!keep) TNC_THROW(TNC_EUNSUPPORTED, "label " + lbl(l) + " is summed inside one tensor");
                st.n.push_back(l);
            }
        }
        // A = operand with the larger free part (it becomes the GEMM rows)
        std::vector<int> fx = st.m, fy = st.n;
        bool swap = fy.size() > fx.size() || (fy.size() == fx.size() && Y.rank() > X.rank());
        st.a = swap ? y : x;
        st.b = swap ? x : y;
        if (swap) std::swap(st.m, st.n);
        if (Z.rank() > kMaxRank) TNC_THROW(TNC_EUNSUPPORTED, "intermediate rank above 48");
    }
    an.root = 2 * nT - 2;
    if (nT == 1) TNC_THROW(TNC_EUNSUPPORTED, "a network of one tensor has nothing to contract");
    // the root must hold exactly the open output labels
    {
        const TensorRec &R = an.tensors[an.root];
        int cnt = 0;
        for (int l : R.labels) {
            if (an.open_qubit_of_label[l] < 0) TNC_THROW(TNC_EINVAL, "label " + lbl(l) + " survives the path but is not open");
            cnt++;
        }
        if (cnt != n_open) TNC_THROW(TNC_EINVAL, "an open output label never reaches the root");
    }

    if (an.sparse) {
        // blocks of every tensor: the distinct values of the requested
        // bitstrings on its qubits (sorted), and for each step which operand
        // block every result block reads
        const size_t nT2 = an.tensors.size();
        std::vector<std::vector<uint64_t>> keys(nT2);
        auto keys_of = [&](uint64_t m) {
            std::vector<uint64_t> k(sparse_bits, sparse_bits + n_sparse);
            for (auto &v : k) v &= m;
            std::sort(k.begin(), k.end());
            k.erase(std::unique(k.begin(), k.end()), k.end());
            return k;
        };
        for (int i = 0; i < nT; i++) {
            keys[i] = keys_of(an.tensors[i].sp_mask);
            an.tensors[i].nd = (int64_t)keys[i].size();
        }
        an.leaf_keys.assign(keys.begin(), keys.begin() + nT);
        for (int s = 0; s < n_steps; s++) {
            StepRec &st = an.steps[s];
            TensorRec &Z = an.tensors[st.z];
            keys[st.z] = keys_of(Z.sp_mask);
            Z.nd = (int64_t)keys[st.z].size();
            if (Z.nd > (int64_t)1 << 31) TNC_THROW(TNC_EUNSUPPORTED, "more than 2^31 sparse blocks");
            auto side = [&](int x, int &mode, std::vector<int32_t> &idx) {
                const TensorRec &X = an.tensors[x];
                if (X.sp_mask == Z.sp_mask) mode = 0;
                else if (X.sp_mask == 0) mode = 1;
                else {
                    mode = 2;
                    idx.resize(Z.nd);
                    for (int64_t d = 0; d < Z.nd; d++) {
                        const uint64_t v = keys[st.z][d] & X.sp_mask;
                        idx[d] = (int32_t)(std::lower_bound(keys[x].begin(), keys[x].end(), v) - keys[x].begin());
                    }
                }
            };
            side(st.a, st.a_mode, st.a_idx);
            side(st.b, st.b_mode, st.b_idx);
            if (st.x >= nT) std::vector<uint64_t>().swap(keys[st.x]);
            if (st.y >= nT) std::vector<uint64_t>().swap(keys[st.y]);
        }
        const auto &rk = keys[an.root];
        const uint64_t rm = an.tensors[an.root].sp_mask;
        an.root_map.resize(n_sparse);
        for (int64_t i = 0; i < n_sparse; i++)
            an.root_map[i] = (int32_t)(std::lower_bound(rk.begin(), rk.end(), sparse_bits[i] & rm) - rk.begin());
    }

    // step at which each label is summed (open outputs: never)
    std::vector<int> kstep(L, n_steps + 1);
    for (int s = 0; s < n_steps; s++)
        for (int l : an.steps[s].k) kstep[l] = s;
    // layout pass: storage orders, operand orientations and permutes
    const int es = elem_bytes(an.dt);
    for (int s = 0; s < n_steps; s++) {
        StepRec &st = an.steps[s];
        TensorRec &A = an.tensors[st.a], &B = an.tensors[st.b], &Z = an.tensors[st.z];
        // consumer groups of Z's labels: 0 batch, 1 kept free, 2 contracted there
        std::vector<int> cg(L, 1);
        if (Z.consumer >= 0) {
            const StepRec &c = an.steps[Z.consumer];
            for (int l : c.beta) cg[l] = 0;
            for (int l : c.k) cg[l] = 2;
        }
        for (int l : st.beta) grp[l] = 0;
        for (int l : st.m) grp[l] = 1;
        for (int l : st.n) grp[l] = 1;
        for (int l : st.k) grp[l] = 2;
        std::vector<int> sa = {(int)st.beta.size(), (int)st.m.size(), (int)st.k.size()};
        std::vector<int> sb = {(int)st.beta.size(), (int)st.n.size(), (int)st.k.size()};
        // smallest run (bits) that a 16-byte chunk needs
        const int lq = an.dt == Dtype::C64 ? 1 : 2;
        // The thin matrix-core kernel reads A in 8-byte pairs of k, so where a
        // step is one it takes (N = 4..32, K = 2, 4 or 8..64, 64 rows or more)
        // a lowest reduced run of one bit will do.  That is a last resort:
        // where the 16-byte rule finds an in-place order it stands, since
        // accepting the looser orders everywhere leads later steps into worse
        // layouts (53-qubit path: 22 -> 36 GB of permutes per slice).
        int lq_k = lq;   // the run a lowest reduced group needs
        auto thin_ok = [&](const StepRec &t) {
            const int64_t N = (int64_t)1 << t.n.size(), K = (int64_t)1 << t.k.size();
            if (an.dt == Dtype::C64 || an.al != Algo::M4 || t.m.size() < 6) return false;
            if (!(N == 4 || N == 8 || N == 16 || N == 32)) return false;
            if (!(K == 2 || K == 4 || (K % 8 == 0 && K <= 64))) return false;
            return !(N == 32 && K > 16);
        };
        // Can a stored order be read in place by a GEMM whose groups are `g`
        // (0 batch, 1 free, 2 reduced)?  The batch labels must form the top
        // block; below it the free and the reduced labels may each lie in at
        // most two runs, and the lowest run must hold a whole chunk (lq_k bits
        // when it is reduced).  Returns the length of that lowest run (bits)
        // and its group, or 0.
        auto inplace = [&](const std::vector<int> &order, const std::vector<int> &g, int &low_group) -> int {
            const int r = (int)order.size();
            int pos = 0;
            while (pos < r && g[order[pos]] == 0) pos++;
            for (int t = pos; t < r; t++)
                if (g[order[t]] == 0 || g[order[t]] < 0) return 0;
            int runs[3] = {0, 0, 0};
            int last = -1, low_len = 0;
            for (int t = pos; t < r; t++) {
                int v = g[order[t]];
                if (v != last) {
                    runs[v]++;
                    low_len = 0;
                }
                low_len++;
                last = v;
            }
            if (runs[1] > 2 || runs[2] > 2) return 0;
            if (pos == r) {   // batch only: nothing to chunk
                low_group = 2;
                return 0;
            }
            low_group = last;
            return low_len >= (last == 2 ? lq_k : lq) ? low_len : 0;
        };
        auto orient = [&](const TensorRec &T) -> int {
            if (T.leaf) return -1;
            int lg = 0;
            if (!inplace(T.labels, grp, lg)) return -1;
            return lg == 2 ? 1 : 0;
        };
        int oa = orient(A), ob = orient(B);
        if (oa < 0 && !A.leaf && thin_ok(st)) {   // last resort: k pairs for the thin kernel
            lq_k = 1;
            oa = orient(A);
            lq_k = lq;
        }
        // A small operand (at most 2^8 entries beside one of 2^16 or more, or
        // at most 1/1024 of the large one) is permuted into the ranked order
        // below rather than read as stored: its free labels then enter the
        // large result grouped by the step that sums them, so the large
        // tensor's later consumers find their reduced labels in few runs
        // whatever order the small tensor's own producers left it in.  The
        // permute costs at most a thousandth of the large operand's bytes; on
        // the 53-qubit path it removes a quarter of the permute traffic.
        if (ob >= 0 && ((B.rank() <= 8 && A.rank() >= 16) || B.rank() + 10 <= A.rank())) ob = -1;
        // A kept operand at most 1/64 of the result is permuted into the
        // ranked order as well: the result's labels then follow the order in
        // which its consumers sum them rather than the operand's producers'
        // order, which can force a permute of the much larger result later
        // (on the 53-qubit path a 2^32-entry tensor, a third of that path's
        // permute traffic).  The permute costs at most 1/32 of the result's
        // bytes.
        if (oa >= 0 && A.rank() + 6 <= Z.rank()) oa = -1;
        if (ob >= 0 && B.rank() + 6 <= Z.rank()) ob = -1;
        // On a compute-bound 16-bit 4M step the k-chunked kernels (operands
        // streamed into LDS as whole k rows) are several times faster than
        // the ones that transpose in registers: permute an operand that is
        // stored [k][free] when the permute costs under a tenth of the GEMM
        // (at 5 TB/s for the permute and 1 PFLOP/s for the GEMM).
        if (an.dt != Dtype::C64 && an.al == Algo::M4) {
            const double fl = 8.0 * std::ldexp(1.0, sa[0] + sa[1] + sb[1] + sa[2]);
            auto cheap = [&](const TensorRec &T) { return 2.0 * es * std::ldexp(1.0, T.rank()) / 5e12 < 0.1 * fl / 1e15; };
            if (oa == 0 && cheap(A)) oa = -1;
            if (ob == 0 && cheap(B)) ob = -1;
        }
        const double szA = std::ldexp(1.0, A.rank()), szB = std::ldexp(1.0, B.rank());
        std::vector<int> beta_o, k_o, m_o, n_o, best_z;
        auto cat3 = [](const std::vector<int> &a, const std::vector<int> &b, const std::vector<int> &c) {
            std::vector<int> r = a;
            r.insert(r.end(), b.begin(), b.end());
            r.insert(r.end(), c.begin(), c.end());
            return r;
        };
        bool keepA = false, keepB = false;
        // A kept operand smaller than the result that leaves the result in no
        // order its consumer can read in place is permuted into the ranked
        // order instead, if that lets the result be read in place: the
        // operand's permute is cheaper than the consumer's permute of the
        // larger result.  Failing that, the first choice stands.
        bool dropA = false, dropB = false;
        // last resort for a thin consumer that reads this result as its A
        bool relax = false;
        const bool relax_ok = Z.consumer >= 0 && an.steps[Z.consumer].a == st.z && thin_ok(an.steps[Z.consumer]);
        for (int attempt = 0; attempt < 4; attempt++) {
            keepA = oa >= 0 && !dropA;
            keepB = ob >= 0 && !dropB;
            beta_o.clear();
            k_o.clear();
            // batch and k orders must agree between A and B; take them from a kept
            // operand, preferring the larger
            if (keepA && keepB) {
                if (extract(A.labels, grp, 0) != extract(B.labels, grp, 0) ||
                    extract(A.labels, grp, 2) != extract(B.labels, grp, 2)) {
                    if (szA >= szB) keepB = false;
                    else keepA = false;
                }
            }
            if (keepA) {
                beta_o = extract(A.labels, grp, 0);
                k_o = extract(A.labels, grp, 2);
            } else if (keepB) {
                beta_o = extract(B.labels, grp, 0);
                k_o = extract(B.labels, grp, 2);
            } else {
                const TensorRec &src = (!A.leaf || B.leaf) ? A : B;
                beta_o = extract(src.labels, grp, 0);
                k_o = extract(src.labels, grp, 2);
            }
            m_o = extract(A.labels, grp, 1);
            n_o = extract(B.labels, grp, 1);
            // Result order.  Free orders of operands that are permuted or gathered
            // follow the consumer's groups; within a group, labels summed later sit
            // higher, so the stem keeps its soon-summed labels at the low end.
            auto ranked = [&](std::vector<int> v, bool kfirst) {
                std::stable_sort(v.begin(), v.end(), [&](int p, int q) {
                    auto key = [&](int l) { return cg[l] == 0 ? 0 : (kfirst ? (cg[l] == 2 ? 1 : 2) : cg[l]); };
                    if (key(p) != key(q)) return key(p) < key(q);
                    return kstep[p] > kstep[q];
                });
                return v;
            };
            // score of a result order: -1 if the consumer must permute it, else the
            // shorter of the writer's and the reader's lowest runs (capped at 5
            // bits: 128-byte runs coalesce fully), minus a small cost per split
            std::vector<int> gw(L, -1);
            auto score = [&](const std::vector<int> &zo, const std::vector<int> &mm, int nsplit) -> double {
                for (int l : zo) gw[l] = 2;
                for (int l : mm) gw[l] = 1;
                for (int l : beta_o) gw[l] = 0;
                int lgw = 0;
                int wlow = inplace(zo, gw, lgw);
                for (int l : zo) gw[l] = -1;
                if (!wlow) return -1;
                int rlow = 5;
                if (Z.consumer >= 0) {
                    int lgr = 0;
                    if (relax) lq_k = 1;
                    rlow = inplace(zo, cg, lgr);
                    lq_k = lq;
                    if (!rlow) return -1;
                }
                return std::min({wlow, rlow, 5}) - 0.25 * nsplit;
            };
            std::vector<int> best_m = keepA ? m_o : ranked(m_o, false), best_n = keepB ? n_o : ranked(n_o, false);
            best_z.clear();
            double best_s = -2;
            for (int kfirst = 0; kfirst < 2; kfirst++) {
                std::vector<int> mm = keepA ? m_o : ranked(m_o, kfirst), nn = keepB ? n_o : ranked(n_o, kfirst);
                // plain [batch][X][Y] first; split layouts [batch][Xh][Yh][Xl][Yl]
                // only if no plain order fits with runs of at least 4 entries
                for (int pass = 0; pass < 2 && best_s < 2.5; pass++) {
                    for (int xm = 1; xm >= 0; xm--) {
                        const auto &X = xm ? mm : nn;
                        const auto &Y = xm ? nn : mm;
                        const int nx = (int)X.size(), ny = (int)Y.size();
                        for (int sx = pass ? 0 : nx; sx <= nx; sx++)
                            for (int sy = pass ? 0 : ny; sy <= ny; sy++) {
                                int nsplit = (sx > 0 && sx < nx) + (sy > 0 && sy < ny);
                                if (pass && !nsplit) continue;
                                std::vector<int> zo = beta_o;
                                zo.insert(zo.end(), X.begin(), X.begin() + sx);
                                zo.insert(zo.end(), Y.begin(), Y.begin() + sy);
                                zo.insert(zo.end(), X.begin() + sx, X.end());
                                zo.insert(zo.end(), Y.begin() + sy, Y.end());
                                double sc = score(zo, mm, nsplit);
                                if (sc > best_s) {
                                    best_s = sc;
                                    best_z = zo;
                                    best_m = mm;
                                    best_n = nn;
                                }
                            }
                    }
                }
                if (best_s >= 0) break;
            }
            if (best_s < 0) {   // nothing fits the consumer: plain order, the consumer permutes
                best_z = cat3(beta_o, best_m, best_n);
                std::vector<int> zt = cat3(beta_o, best_n, best_m);
                if (score(best_z, best_m, 0) < 0 && score(zt, best_m, 0) >= 0) best_z = zt;
            }
            m_o = best_m;
            n_o = best_n;
            if (attempt == 0 && best_s < 0 && Z.consumer >= 0) {
                dropA = keepA && A.rank() < Z.rank();
                dropB = keepB && B.rank() < Z.rank() && !dropA;
                if (dropA || dropB) continue;
            }
            if (attempt == 1 && best_s < 0) {
                dropA = dropB = false;
                continue;
            }
            if (best_s < 0 && !relax && relax_ok) {   // last resort: k pairs for a thin consumer
                relax = true;
                dropA = dropB = false;
                continue;
            }
            break;
        }
        // operand orders
        if (keepA) {
            st.a_kc = oa;
        } else {
            std::vector<int> want = cat3(beta_o, m_o, k_o);
            if (!A.leaf) {
                st.perm_a = true;
                st.a_from = A.labels;
            }
            A.labels = want;
            st.a_kc = 1;
        }
        if (keepB) {
            st.b_kc = ob;
        } else {
            std::vector<int> want = cat3(beta_o, n_o, k_o);
            if (!B.leaf) {
                st.perm_b = true;
                st.b_from = B.labels;
            }
            B.labels = want;
            st.b_kc = 1;
        }
        st.beta = beta_o;
        st.m = m_o;
        st.n = n_o;
        st.k = k_o;
        Z.labels = best_z;
        {
            // the result is written in chunks along the index of its lowest label
            int low = Z.labels.empty() ? -1 : Z.labels.back();
            st.c_nc = (low >= 0 && std::find(m_o.begin(), m_o.end(), low) != m_o.end()) ? 0 : 1;
        }
        // sparse state: the batch is the result's blocks (no batch labels there)
        st.nb = an.sparse ? Z.nd : (int64_t)1 << st.beta.size();
        st.M = (int64_t)1 << st.m.size();
        st.N = (int64_t)1 << st.n.size();
        st.K = (int64_t)1 << st.k.size();
        st.flops = 8.0 * (double)st.nb * (double)st.M * (double)st.N * (double)st.K;
        st.bytes = es * ((double)A.nd * std::ldexp(1.0, A.rank()) + (double)B.nd * std::ldexp(1.0, B.rank()) +
                         (double)Z.nd * std::ldexp(1.0, Z.rank()));
        st.perm_bytes = (st.perm_a ? 2.0 * es * (double)A.nd * szA : 0.0) + (st.perm_b ? 2.0 * es * (double)B.nd * szB : 0.0);
        st.hoist_a = st.perm_a && st.dep && !A.dep;
        st.hoist_b = st.perm_b && st.dep && !B.dep;
        if (!derive_seg(A.labels, st.m, st.am) || !derive_seg(A.labels, st.k, st.ak) ||
            !derive_seg(B.labels, st.n, st.bn) || !derive_seg(B.labels, st.k, st.bk) ||
            !derive_seg(Z.labels, st.m, st.cm) || !derive_seg(Z.labels, st.n, st.cn))
            TNC_THROW(TNC_EINVAL, "internal: operand layout has more than two runs per index");
        st.kernel = choose_kernel(an.dt, an.al, step_gemm(st));
        if (an.sparse && st.a_mode == 2 && st.bn.l == 62 && st.cn.l == 62) {
            // second scheme, when it moves fewer bytes: group the result
            // blocks by the A block they read
            const int64_t ndA = A.nd, ndZ = Z.nd;
            std::vector<int32_t> cnt(ndA, 0), rpos(ndZ);
            for (int64_t z = 0; z < ndZ; z++) rpos[z] = cnt[st.a_idx[z]]++;
            int64_t mr = 1;
            while (mr < *std::max_element(cnt.begin(), cnt.end())) mr *= 2;
            const double sA_ = std::ldexp(1.0, A.rank()), sB_ = std::ldexp(1.0, B.rank()), sZ_ = std::ldexp(1.0, Z.rank());
            const double bytes1 = (double)ndZ * (sA_ + sB_ + sZ_);
            const double bytes2 = (double)ndA * sA_ + (double)ndA * mr * (3.0 * sB_ + sZ_) + 2.0 * (double)ndZ * sZ_;
            const char *force = getenv("TNC_SPARSE_SCHEME");
            const int want = force ? atoi(force) : 0;
            if (mr >= 2 && (want == 2 || (want != 1 && bytes2 < 0.8 * bytes1))) {
                st.scheme = 2;
                st.mr = mr;
                st.bp_idx.assign(ndA * mr, -1);
                st.cp_idx.resize(ndZ);
                for (int64_t z = 0; z < ndZ; z++) {
                    const int64_t slot = (int64_t)st.a_idx[z] * mr + rpos[z];
                    st.bp_idx[slot] = st.b_mode == 2 ? st.b_idx[z] : (st.b_mode == 0 ? (int32_t)z : 0);
                    st.cp_idx[z] = (int32_t)slot;
                }
                // A blocks per chunk: B_P and C_P of one chunk within the
                // larger of the result's own size and 2^24 entries
                const double per_a = (double)mr * (sB_ + sZ_);
                const double budget = std::max((double)ndZ * sZ_, std::ldexp(1.0, 24));
                st.chunk = std::max<int64_t>(1, std::min<int64_t>(ndA, (int64_t)(budget / per_a)));
                const char *cap = getenv("TNC_SPARSE_CHUNK");   // smaller chunks (tests)
                if (cap && atoi(cap) > 0) st.chunk = std::min<int64_t>(st.chunk, atoi(cap));
                st.kernel = choose_kernel(an.dt, an.al, step_gemm_exec(st));
                st.bytes = es * bytes2;
            }
        }
        for (int l : st.beta) grp[l] = -1;
        for (int l : st.m) grp[l] = -1;
        for (int l : st.n) grp[l] = -1;
        for (int l : st.k) grp[l] = -1;
        an.max_rank = std::max({an.max_rank, A.rank(), B.rank(), Z.rank()});
    }
    return an;
}

// ------------------------------------------------------------------ arena

namespace {
struct Arena {
    std::map<int64_t, int64_t> free_;   // offset -> size
    int64_t top = 0, peak = 0;
    static int64_t align(int64_t v) { return (v + 255) & ~(int64_t)255; }
    int64_t alloc(int64_t bytes) {
        bytes = align(std::max<int64_t>(bytes, 1));
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                int64_t off = it->first, rem = it->second - bytes;
                free_.erase(it);
                if (rem > 0) free_[off + bytes] = rem;
                return off;
            }
        }
        int64_t off = top;
        top += bytes;
        peak = std::max(peak, top);
        return off;
    }
    void release(int64_t off, int64_t bytes) {
        bytes = align(std::max<int64_t>(bytes, 1));
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
                it = pv;
            }
        }
        if (it->first + it->second == top) {
            top = it->first;
            free_.erase(it);
        }
    }
};
}  // namespace

int64_t plan_memory(Analysis &an, int S, bool assign) {
    const int es = elem_bytes(an.dt);
    Arena ar;
    auto bytes_of = [&](const TensorRec &t) {
        return (int64_t)es * ((int64_t)1 << t.rank()) * t.nd * (t.dep ? S : 1);
    };
    std::vector<int64_t> off(an.tensors.size(), -1);
    const int nT = (int)(an.tensors.size() + 1) / 2;
    auto cls_t = [&](int t) { return exec_class(an.tensors[t].dep, an.tensors[t].inner); };
    // invariant phase
    for (int i = 0; i < nT; i++)
        if (cls_t(i) == 0) off[i] = ar.alloc(bytes_of(an.tensors[i]));
    std::vector<int64_t> scr_a(an.steps.size(), -1), scr_b(an.steps.size(), -1);
    std::vector<int64_t> scr_bp(an.steps.size(), -1), scr_cp(an.steps.size(), -1);
    auto run_step = [&](int s) {
        StepRec &st = an.steps[s];
        const TensorRec &A = an.tensors[st.a], &B = an.tensors[st.b], &Z = an.tensors[st.z];
        const bool pa = st.perm_a && !st.hoist_a, pb = st.perm_b && !st.hoist_b;
        if (pa) scr_a[s] = ar.alloc(bytes_of(A));
        if (pb) scr_b[s] = ar.alloc(bytes_of(B));
        off[st.z] = ar.alloc(bytes_of(Z));
        int64_t bp_bytes = 0, cp_bytes = 0;
        if (st.scheme == 2) {
            const int64_t Sl = st.dep ? S : 1;
            bp_bytes = (int64_t)es * st.chunk * st.mr * ((int64_t)1 << B.rank()) * Sl;
            cp_bytes = (int64_t)es * st.chunk * st.mr * ((int64_t)1 << Z.rank()) * Sl;
            scr_bp[s] = ar.alloc(bp_bytes);
            scr_cp[s] = ar.alloc(cp_bytes);
            ar.release(scr_cp[s], cp_bytes);
            ar.release(scr_bp[s], bp_bytes);
        }
        if (pa) ar.release(scr_a[s], bytes_of(A));
        if (pb) ar.release(scr_b[s], bytes_of(B));
        for (int t : {st.a, st.b}) {
            const TensorRec &T = an.tensors[t];
            // an operand of an earlier class (invariant for a slice step,
            // prefix for a recomputed one) is read again by every group or
            // pass: kept
            if (cls_t(t) == exec_class(st.dep, st.inner)) ar.release(off[t], bytes_of(T));
        }
    };
    for (int s = 0; s < (int)an.steps.size(); s++)
        if (!an.steps[s].dep) run_step(s);
    // permuted copies of invariant operands of dependent steps: made once, kept
    for (int s = 0; s < (int)an.steps.size(); s++) {
        StepRec &st = an.steps[s];
        if (st.hoist_a) {
            scr_a[s] = ar.alloc(bytes_of(an.tensors[st.a]));
            ar.release(off[st.a], bytes_of(an.tensors[st.a]));
        }
        if (st.hoist_b) {
            scr_b[s] = ar.alloc(bytes_of(an.tensors[st.b]));
            ar.release(off[st.b], bytes_of(an.tensors[st.b]));
        }
    }
    // dependent phase (one slice group): the prefix, then one recomputation pass
    for (int c = 1; c <= 2; c++) {
        for (int i = 0; i < nT; i++)
            if (cls_t(i) == c) off[i] = ar.alloc(bytes_of(an.tensors[i]));
        for (int s = 0; s < (int)an.steps.size(); s++)
            if (exec_class(an.steps[s].dep, an.steps[s].inner) == c) run_step(s);
    }
    if (assign) {
        for (size_t i = 0; i < an.tensors.size(); i++) an.tensors[i].off = off[i];
        for (size_t s = 0; s < an.steps.size(); s++) {
            an.steps[s].scr_a = scr_a[s];
            an.steps[s].scr_b = scr_b[s];
            an.steps[s].scr_bp = scr_bp[s];
            an.steps[s].scr_cp = scr_cp[s];
        }
    }
    return ar.peak;
}

void fill_stats(const Analysis &an, tnc_plan_stats &st) {
    st = tnc_plan_stats{};
    st.n_steps = (int)an.steps.size();
    st.n_sliced = an.n_sliced;
    st.max_rank = an.max_rank;
    st.out_rank = an.tensors[an.root].rank();
    double pe = 0;
    for (auto &t : an.tensors) pe = std::max(pe, (double)t.nd * std::ldexp(1.0, t.rank()));
    st.peak_elems_per_slice = pe;
    const double passes = std::ldexp(1.0, an.n_recompute);
    st.n_recompute = an.n_recompute;
    for (auto &s : an.steps) st.n_padded_steps += s.scheme == 2 ? 1 : 0;
    for (auto &s : an.steps) {
        if (s.dep) {
            const double w = s.inner ? passes : 1.0;
            st.n_dep_steps++;
            st.flops_per_slice += w * s.flops;
            st.bytes_per_slice += w * (s.bytes + s.perm_bytes);
            st.permute_bytes_per_slice += w * s.perm_bytes;
        } else {
            st.flops_invariant += s.flops;
        }
    }
}

}  // namespace tnc
