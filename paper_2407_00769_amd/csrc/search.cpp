// Contraction-path and slicing search (host).
//
// The paper takes its paths from prior work and states the trade-off they
// obey: slicing fixes the values of chosen labels, which caps the largest
// tensor of a sub-network while the total work grows (Sec. 3.1; Fig. 2,
// time complexity against the memory limit).  This search is:
//   1. randomized greedy pairwise merging: the pair whose result shrinks the
//      network most, score = |out| - alpha (|a| + |b|) on a log scale, with
//      Gumbel noise at temperature T (Boltzmann sampling); restart 0 is the
//      plain greedy order;
//   2. a slicer that, while the largest tensor of one slice exceeds the cap,
//      fixes the label of a largest tensor that adds the least total work;
//   3. a re-run of the greedy order on the network with those labels removed,
//      and slicing again, twice;
//   4. across restarts, the (path, sliced labels) with the least cost: total
//      FLOPs, or the learned step-time model's prediction when one is active.
#include <algorithm>
#include <cmath>
#include <functional>
#include <queue>
#include <random>

#include "engine.h"
#include "planner.h"

using namespace tnc;

namespace tnc {
// learned cost of a candidate (defined in mlp.hip); < 0 when no model is active
double mlp_path_cost(const Network &net, const std::vector<int> &ssa, const std::vector<int> &sliced,
                     const std::vector<int> &open_q);
}

namespace {

struct Tree {
    std::vector<int> ssa;                      // 2 per step
    std::vector<std::vector<int>> uni;         // per step: union of operand labels
    std::vector<std::vector<int>> labels;      // per tensor id (inputs, then steps)
};

// labels of each input after removing closed outputs and `removed`
std::vector<std::vector<int>> reduced_inputs(const Network &net, const std::vector<char> &gone) {
    std::vector<std::vector<int>> r(net.n_tensors);
    for (int i = 0; i < net.n_tensors; i++)
        for (int l : net.labels[i])
            if (!gone[l]) r[i].push_back(l);
    for (auto &v : r) std::sort(v.begin(), v.end());
    return r;
}

std::vector<int> symdiff(const std::vector<int> &a, const std::vector<int> &b, std::vector<int> *uni) {
    std::vector<int> out;
    uni->clear();
    size_t i = 0, j = 0;
    while (i < a.size() || j < b.size()) {
        if (j == b.size() || (i < a.size() && a[i] < b[j])) {
            out.push_back(a[i]);
            uni->push_back(a[i++]);
        } else if (i == a.size() || b[j] < a[i]) {
            out.push_back(b[j]);
            uni->push_back(b[j++]);
        } else {
            uni->push_back(a[i]);
            i++;
            j++;
        }
    }
    return out;
}

Tree greedy(const std::vector<std::vector<int>> &inputs, int n_labels, double alpha, double temp, std::mt19937_64 &rng) {
    const int n = (int)inputs.size();
    Tree t;
    t.labels = inputs;
    t.labels.resize(2 * n - 1);
    std::vector<char> alive(2 * n - 1, 0);
    for (int i = 0; i < n; i++) alive[i] = 1;
    std::vector<std::vector<int>> holders(n_labels);
    for (int i = 0; i < n; i++)
        for (int l : inputs[i]) holders[l].push_back(i);
    std::uniform_real_distribution<double> U(1e-12, 1.0);
    struct Cand {
        double score;
        int a, b;
        bool operator<(const Cand &o) const { return score > o.score; }   // min-heap
    };
    std::priority_queue<Cand> pq;
    std::vector<int> tmp;
    auto push = [&](int a, int b) {
        if (a > b) std::swap(a, b);
        std::vector<int> out = symdiff(t.labels[a], t.labels[b], &tmp);
        double so = std::ldexp(1.0, (int)out.size());
        double sa = std::ldexp(1.0, (int)t.labels[a].size()), sb = std::ldexp(1.0, (int)t.labels[b].size());
        double raw = so - alpha * (sa + sb);
        double sc = (raw >= 0 ? 1.0 : -1.0) * std::log2(1.0 + std::fabs(raw));
        if (temp > 0) sc -= temp * -std::log(-std::log(U(rng)));
        pq.push({sc, a, b});
    };
    for (int l = 0; l < n_labels; l++)
        if (holders[l].size() == 2) push(holders[l][0], holders[l][1]);
    int next = n;
    while (next < 2 * n - 1) {
        int a = -1, b = -1;
        while (!pq.empty()) {
            Cand c = pq.top();
            pq.pop();
            if (alive[c.a] && alive[c.b]) {
                a = c.a;
                b = c.b;
                break;
            }
        }
        if (a < 0) {   // disconnected parts: join the two smallest
            std::vector<int> live;
            for (int i = 0; i < next; i++)
                if (alive[i]) live.push_back(i);
            std::sort(live.begin(), live.end(), [&](int x, int y) {
                return t.labels[x].size() < t.labels[y].size() || (t.labels[x].size() == t.labels[y].size() && x < y);
            });
            a = live[0];
            b = live[1];
        }
        std::vector<int> uni;
        t.labels[next] = symdiff(t.labels[a], t.labels[b], &uni);
        t.uni.push_back(uni);
        t.ssa.push_back(a);
        t.ssa.push_back(b);
        alive[a] = alive[b] = 0;
        alive[next] = 1;
        for (int l : t.labels[next]) {
            auto &h = holders[l];
            for (auto &x : h)
                if (x == a || x == b) x = next;
            for (int x : h)
                if (x != next && alive[x]) push(x, next);
        }
        next++;
    }
    return t;
}

struct Sliced {
    std::vector<int> labels;
    double log2_total = 0;   // log2 of total real flops over all slices
    int max_rank = 0;
};

double log2_sum_flops(const Tree &t, const std::vector<char> &sl) {
    double tot = 0;
    for (auto &u : t.uni) {
        int r = 0;
        for (int l : u)
            if (!sl[l]) r++;
        tot += std::ldexp(8.0, r);
    }
    return std::log2(tot);
}

Sliced slice_tree(const Tree &t, int n_labels, const std::vector<char> &sliceable, double cap,
                  std::vector<char> sl /* initial */) {
    const int nt = (int)t.labels.size();
    std::vector<int> rank(nt);
    std::vector<std::vector<int>> tens_of(n_labels), steps_of(n_labels);
    for (int i = 0; i < nt; i++) {
        int r = 0;
        for (int l : t.labels[i]) {
            tens_of[l].push_back(i);
            if (!sl[l]) r++;
        }
        rank[i] = r;
    }
    std::vector<double> f(t.uni.size());
    double per = 0;
    for (size_t s = 0; s < t.uni.size(); s++) {
        int r = 0;
        for (int l : t.uni[s]) {
            steps_of[l].push_back((int)s);
            if (!sl[l]) r++;
        }
        f[s] = std::ldexp(8.0, r);
        per += f[s];
    }
    int ns = 0;
    for (int l = 0; l < n_labels; l++) ns += sl[l] ? 1 : 0;
    for (;;) {
        int mr = *std::max_element(rank.begin(), rank.end());
        if (mr <= cap) break;
        // candidates: labels of a largest tensor
        double best = 1e300;
        int bl = -1;
        for (int i = 0; i < nt; i++) {
            if (rank[i] != mr) continue;
            for (int l : t.labels[i]) {
                if (sl[l] || !sliceable[l]) continue;
                double d = 0;
                for (int s : steps_of[l]) d += f[s] * 0.5;
                double cost = (per - d) * 2.0;   // per-slice work halves on those steps, slices double
                if (cost < best) {
                    best = cost;
                    bl = l;
                }
            }
        }
        if (bl < 0) break;   // nothing left to slice
        sl[bl] = 1;
        ns++;
        for (int i : tens_of[bl]) rank[i]--;
        for (int s : steps_of[bl]) {
            per -= f[s] * 0.5;
            f[s] *= 0.5;
        }
    }
    Sliced r;
    for (int l = 0; l < n_labels; l++)
        if (sl[l]) r.labels.push_back(l);
    r.max_rank = *std::max_element(rank.begin(), rank.end());
    r.log2_total = std::log2(per) + ns;
    return r;
}

}  // namespace

extern "C" int tnc_search(const tnc_network *net_h, int32_t n_open, const int32_t *open_qubits, double log2_cap,
                          int32_t cost_model, int32_t restarts, uint64_t seed, int32_t *ssa_out, int32_t max_sliced,
                          int32_t *sliced_out, int32_t *n_sliced, double *log2_cost_out) {
    try {
        if (!net_h || !ssa_out || !n_sliced || (max_sliced > 0 && !sliced_out)) TNC_THROW(TNC_EINVAL, "NULL argument");
        const Network &net = net_h->net;
        if (restarts < 1) TNC_THROW(TNC_EINVAL, "restarts < 1");
        if (net.n_tensors < 2) TNC_THROW(TNC_EUNSUPPORTED, "a network of one tensor has nothing to contract");
        const int L = net.n_labels;
        std::vector<char> gone(L, 0), sliceable(L, 1), is_open(net.n_qubits, 0);
        std::vector<int> open_q;
        for (int i = 0; i < n_open; i++) {
            int q = open_qubits[i];
            if (q < 0 || q >= net.n_qubits || is_open[q]) TNC_THROW(TNC_EINVAL, "bad open qubit list");
            is_open[q] = 1;
            open_q.push_back(q);
        }
        for (int q = 0; q < net.n_qubits; q++) {
            sliceable[net.output_labels[q]] = 0;
            if (!is_open[q]) gone[net.output_labels[q]] = 1;   // closed: fixed per call
        }
        std::mt19937_64 rng(seed);
        std::uniform_real_distribution<double> ua(0.6, 1.6), ut(0.0, 1.0);
        double best_cost = 1e300;
        std::vector<int> best_ssa, best_sl;
        double best_flops = 0;
        for (int r = 0; r < restarts; r++) {
            double alpha = r == 0 ? 1.0 : ua(rng);
            double temp = r == 0 ? 0.0 : ut(rng) * ut(rng);
            std::vector<char> sl(L, 0);
            Tree t;
            Sliced s;
            for (int it = 0; it < 3; it++) {
                std::vector<char> g2 = gone;
                for (int l = 0; l < L; l++)
                    if (sl[l]) g2[l] = 1;
                Tree cand = greedy(reduced_inputs(net, g2), L, alpha, temp, rng);
                // the tree's labels must include the sliced ones for slice_tree's bookkeeping
                Tree full = cand;
                {
                    auto in = reduced_inputs(net, gone);
                    full.labels.assign(in.begin(), in.end());
                    full.labels.resize(2 * net.n_tensors - 1);
                    full.uni.clear();
                    std::vector<int> u;
                    for (size_t st = 0; st < cand.ssa.size() / 2; st++) {
                        full.labels[net.n_tensors + st] = symdiff(full.labels[cand.ssa[2 * st]], full.labels[cand.ssa[2 * st + 1]], &u);
                        full.uni.push_back(u);
                    }
                }
                Sliced sc = slice_tree(full, L, sliceable, log2_cap, sl);
                if (it == 0 || sc.log2_total < s.log2_total) {
                    t = full;
                    s = sc;
                }
                std::fill(sl.begin(), sl.end(), 0);
                for (int l : s.labels) sl[l] = 1;
            }
            if (s.max_rank > log2_cap) continue;
            double cost = s.log2_total;
            if (cost_model == 1) {
                double c = mlp_path_cost(net, t.ssa, s.labels, open_q);
                if (c > 0) cost = std::log2(c);
            }
            if (cost < best_cost) {
                best_cost = cost;
                best_ssa = t.ssa;
                best_sl = s.labels;
                best_flops = s.log2_total;
            }
        }
        if (best_ssa.empty()) TNC_THROW(TNC_EINVAL, "no path meets the memory cap");
        if ((int)best_sl.size() > max_sliced) TNC_THROW(TNC_EINVAL, "more sliced labels than max_sliced");
        std::copy(best_ssa.begin(), best_ssa.end(), ssa_out);
        std::copy(best_sl.begin(), best_sl.end(), sliced_out);
        *n_sliced = (int)best_sl.size();
        if (log2_cost_out) *log2_cost_out = best_flops;
        return TNC_OK;
    } catch (const Error &e) {
        set_error(e.msg);
        return e.code;
    } catch (const std::exception &e) {
        set_error(e.what());
        return TNC_EINVAL;
    }
}
