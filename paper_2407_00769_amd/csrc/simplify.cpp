// Host FP64 pre-contraction of the leaf-level sub-trees of a path.
//
// A random-circuit network holds many tiny tensors (initial wires, one-qubit
// gates, two-qubit gates).  Every step of the given path that absorbs a
// tensor of rank <= 2 into another input tensor (or into the result of such a
// step) without growing it is contracted here in complex128 before anything
// is converted to the device's storage type.  The device path then starts from those merged tensors: it
// runs fewer tiny steps, and the 16-bit forms round each merged tensor once
// instead of rounding every gate entry on its own (1/sqrt 2, for example,
// always rounds the same way in FP16).  The contraction tree is the given one;
// only where its leaf-level steps run changes.
//
// Labels that the plan fixes (sliced and recomputed labels, output labels of
// closed qubits) are never summed here: a merged tensor keeps them, and the slice gather
// selects their values per slice and per call as for any input tensor.  A
// label that both operands hold and no other tensor needs is summed (paper
// Eq. contraction); a label still held elsewhere stays, as a batch label.
#include <algorithm>
#include <cstdlib>

#include "planner.h"

namespace tnc {

namespace {

struct HostTensor {
    std::vector<int> labels;     // first label slowest
    std::vector<double> data;    // interleaved complex128
};

// Z[lz] = sum over the labels of X and Y not in lz of X[lx] * Y[ly].
HostTensor host_pair(const HostTensor &X, const HostTensor &Y, const std::vector<int> &lz) {
    std::vector<int> uni = X.labels;
    for (int l : Y.labels)
        if (std::find(uni.begin(), uni.end(), l) == uni.end()) uni.push_back(l);
    const int u = (int)uni.size();
    // stride of union bit j (bit 0 = last label of uni) in X, Y and Z
    std::vector<int64_t> sx(u, 0), sy(u, 0), sz(u, 0);
    auto stride_in = [](const std::vector<int> &ls, int l) -> int64_t {
        auto it = std::find(ls.begin(), ls.end(), l);
        if (it == ls.end()) return 0;
        return (int64_t)1 << (ls.size() - 1 - (it - ls.begin()));
    };
    for (int j = 0; j < u; j++) {
        const int l = uni[u - 1 - j];
        sx[j] = stride_in(X.labels, l);
        sy[j] = stride_in(Y.labels, l);
        sz[j] = stride_in(lz, l);
    }
    HostTensor Z;
    Z.labels = lz;
    Z.data.assign(2 * ((size_t)1 << lz.size()), 0.0);
    const int64_t n = (int64_t)1 << u;
    for (int64_t i = 0; i < n; i++) {
        int64_t ox = 0, oy = 0, oz = 0;
        for (int j = 0; j < u; j++)
            if ((i >> j) & 1) {
                ox += sx[j];
                oy += sy[j];
                oz += sz[j];
            }
        const double ar = X.data[2 * ox], ai = X.data[2 * ox + 1];
        const double br = Y.data[2 * oy], bi = Y.data[2 * oy + 1];
        Z.data[2 * oz] += ar * br - ai * bi;
        Z.data[2 * oz + 1] += ar * bi + ai * br;
    }
    return Z;
}

}  // namespace

int host_rank_cap() {
    const char *e = getenv("TNC_HOST_RANK");
    if (e && *e) {
        int v = atoi(e);
        return std::max(0, std::min(v, kMaxHostRank));
    }
    return kDefaultHostRank;
}

Simplified presimplify(const Network &net, int n_steps, const int32_t *ssa, int n_sliced, const int32_t *sliced,
                       int n_open, const int32_t *open_q, int max_rank, int n_recompute, const int32_t *recompute) {
    const int nT = net.n_tensors;
    const int L = net.n_labels;
    if (n_steps != nT - 1) TNC_THROW(TNC_EINVAL, "path must have n_tensors - 1 steps");
    Simplified out;
    out.plan_step_of.assign(n_steps, -1);
    if (n_steps == 0 || max_rank <= 0) {   // nothing to pre-contract
        out.net = net;
        out.ssa.assign(ssa, ssa + 2 * n_steps);
        for (int s = 0; s < n_steps; s++) out.plan_step_of[s] = s;
        return out;
    }
    // labels the plan fixes: never summed on the host
    std::vector<char> fixed(L, 0), open_out(L, 0);
    std::vector<char> is_open(net.n_qubits, 0);
    for (int i = 0; i < n_open; i++)
        if (open_q[i] >= 0 && open_q[i] < net.n_qubits) is_open[open_q[i]] = 1;
    for (int q = 0; q < net.n_qubits; q++) {
        const int l = net.output_labels[q];
        if (is_open[q]) open_out[l] = 1;
        else fixed[l] = 1;
    }
    for (int j = 0; j < n_sliced; j++)
        if (sliced[j] >= 0 && sliced[j] < L) fixed[sliced[j]] = 1;
    for (int j = 0; j < n_recompute; j++)
        if (recompute[j] >= 0 && recompute[j] < L) fixed[recompute[j]] = 1;
    // holders of each label among the live tensors
    std::vector<int> holders(L, 0);
    for (const auto &ls : net.labels)
        for (int l : ls) holders[l]++;

    const int nZ = nT + n_steps;
    std::vector<int> rank(nZ, 0), consumer(nZ, -1);
    std::vector<char> host(nZ, 0), alive(nZ, 0);
    std::vector<HostTensor> ht(nZ);
    for (int i = 0; i < nT; i++) {
        host[i] = 1;
        alive[i] = 1;
        rank[i] = (int)net.labels[i].size();
        ht[i].labels = net.labels[i];
        ht[i].data = net.data[i];
    }
    for (int s = 0; s < n_steps; s++) {
        const int x = ssa[2 * s], y = ssa[2 * s + 1], z = nT + s;
        if (x < 0 || y < 0 || x >= z || y >= z || x == y)
            TNC_THROW(TNC_EINVAL, "path step " + std::to_string(s) + " has an invalid operand");
        if (!alive[x] || !alive[y]) TNC_THROW(TNC_EINVAL, "path step " + std::to_string(s) + " uses a tensor twice");
        alive[x] = alive[y] = 0;
        alive[z] = 1;
        consumer[x] = consumer[y] = s;
        // labels of the result, in the order the device planner would keep them
        const std::vector<int> &lx = ht[x].labels, &ly = ht[y].labels;
        std::vector<int> lz;
        auto visit = [&](int l, bool inx, bool iny) {
            const int after = holders[l] - (inx ? 1 : 0) - (iny ? 1 : 0);
            if (after > 0 || fixed[l] || open_out[l]) lz.push_back(l);
        };
        for (int l : lx) visit(l, true, std::find(ly.begin(), ly.end(), l) != ly.end());
        for (int l : ly)
            if (std::find(lx.begin(), lx.end(), l) == lx.end()) visit(l, false, true);
        const bool last = s == n_steps - 1;
        // absorb a tensor of rank <= 2 (an initial wire, a one-qubit gate, or
        // a merge of those) into its partner when the result is no larger
        // than the larger operand
        const int rz = (int)lz.size();
        const bool on_host = host[x] && host[y] && !last && std::min(rank[x], rank[y]) <= 2 &&
                             rz <= std::max(rank[x], rank[y]) && rz <= max_rank;
        for (int l : lx) holders[l]--;
        for (int l : ly)
            if (std::find(lx.begin(), lx.end(), l) == lx.end()) holders[l]--;
        for (int l : lz) holders[l]++;
        rank[z] = (int)lz.size();
        if (on_host) {
            host[z] = 1;
            ht[z] = host_pair(ht[x], ht[y], lz);
            ht[x] = HostTensor{};
            ht[y] = HostTensor{};
            out.host_steps++;
        } else {
            ht[z].labels = lz;   // labels only; the device computes it
        }
    }
    // device leaves: host-side tensors read by device steps, by tensor id
    std::vector<int> new_id(nZ, -1);
    int nl = 0;
    for (int t = 0; t < nZ; t++)
        if (host[t] && consumer[t] >= 0 && !host[nT + consumer[t]]) new_id[t] = nl++;
    out.net.n_tensors = nl;
    out.net.n_qubits = net.n_qubits;
    out.net.output_labels = net.output_labels;
    out.net.n_labels = net.n_labels;
    out.net.labels.resize(nl);
    out.net.data.resize(nl);
    for (int t = 0; t < nZ; t++)
        if (new_id[t] >= 0) {
            out.net.labels[new_id[t]] = std::move(ht[t].labels);
            out.net.data[new_id[t]] = std::move(ht[t].data);
        }
    int ds = 0;
    for (int s = 0; s < n_steps; s++) {
        if (host[nT + s]) continue;
        out.plan_step_of[s] = ds;
        new_id[nT + s] = nl + ds;
        ds++;
    }
    out.ssa.reserve(2 * ds);
    for (int s = 0; s < n_steps; s++) {
        if (host[nT + s]) continue;
        out.ssa.push_back(new_id[ssa[2 * s]]);
        out.ssa.push_back(new_id[ssa[2 * s + 1]]);
    }
    return out;
}

}  // namespace tnc
