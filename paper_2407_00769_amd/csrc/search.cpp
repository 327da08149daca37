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
//      FLOPs, or the learned step-time model's prediction when one is active;
//      the same cost also picks between a restart's greedy variants and
//      decides whether a reconfigured tree is kept.  Under the learned model
//      the FLOP-cost search runs first and its choice stays unless the
//      model's own search finds a path it predicts to be faster.
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


// ------------------------------------------------------------------ subtree reconfiguration
// For a node v, take the frontier of at most kMaxFront sub-trees below it and
// find the cheapest way to contract them back into v by dynamic programming
// over subsets (cost = per-slice flops, sliced labels removed; no
// intermediate may exceed the cap).  Replace the old sub-tree when cheaper.

constexpr int kMaxFront = 8;

struct BTree {
    int n = 0;                                  // inputs
    std::vector<int> left, right;               // per node (-1 for inputs)
    std::vector<std::vector<int>> labels;       // per node, sorted, sliced labels removed
    int root = -1;
};

BTree to_btree(const Tree &t, int n_inputs, const std::vector<char> &sl) {
    BTree b;
    b.n = n_inputs;
    const int total = (int)t.labels.size();
    b.left.assign(total, -1);
    b.right.assign(total, -1);
    b.labels.resize(total);
    for (int i = 0; i < total; i++)
        for (int l : t.labels[i])
            if (!sl[l]) b.labels[i].push_back(l);
    for (size_t s = 0; s < t.ssa.size() / 2; s++) {
        b.left[n_inputs + s] = t.ssa[2 * s];
        b.right[n_inputs + s] = t.ssa[2 * s + 1];
    }
    b.root = total - 1;
    return b;
}

double node_cost(const BTree &b, int v) {
    if (b.left[v] < 0) return 0.0;
    std::vector<int> u;
    symdiff(b.labels[b.left[v]], b.labels[b.right[v]], &u);
    return std::ldexp(8.0, (int)u.size());
}

double subtree_cost(const BTree &b, int v, const std::vector<char> &stop) {
    if (b.left[v] < 0 || stop[v]) return 0.0;
    return node_cost(b, v) + subtree_cost(b, b.left[v], stop) + subtree_cost(b, b.right[v], stop);
}

// returns the number of improved nodes
int reconfigure_once(BTree &b, double cap, std::mt19937_64 &rng) {
    int improved = 0;
    const int total = (int)b.left.size();
    std::vector<int> order;
    for (int v = b.n; v < total; v++)
        if (b.left[v] >= 0) order.push_back(v);
    std::shuffle(order.begin(), order.end(), rng);
    std::vector<char> stop(total, 0);
    for (int v : order) {
        if (b.left[v] < 0) continue;
        // frontier: expand the largest internal frontier node until kMaxFront
        std::vector<int> front = {b.left[v], b.right[v]};
        std::vector<int> inner = {v};
        while ((int)front.size() < kMaxFront) {
            int best = -1;
            size_t bsz = 0;
            for (int i = 0; i < (int)front.size(); i++) {
                int f = front[i];
                if (b.left[f] >= 0 && (best < 0 || b.labels[f].size() > bsz)) {
                    best = i;
                    bsz = b.labels[f].size();
                }
            }
            if (best < 0) break;
            int f = front[best];
            inner.push_back(f);
            front[best] = b.left[f];
            front.push_back(b.right[f]);
        }
        const int m = (int)front.size();
        if (m < 3) continue;
        for (int f : front) stop[f] = 1;
        double old_cost = subtree_cost(b, v, stop);
        for (int f : front) stop[f] = 0;
        // local label bitsets
        std::vector<int> loc;
        for (int f : front) loc.insert(loc.end(), b.labels[f].begin(), b.labels[f].end());
        std::sort(loc.begin(), loc.end());
        loc.erase(std::unique(loc.begin(), loc.end()), loc.end());
        const int nw = ((int)loc.size() + 63) / 64;
        if (nw > 8) continue;
        const int NS = 1 << m;
        std::vector<uint64_t> bits((size_t)NS * nw, 0);
        for (int i = 0; i < m; i++)
            for (int l : b.labels[front[i]]) {
                int j = (int)(std::lower_bound(loc.begin(), loc.end(), l) - loc.begin());
                bits[(size_t)(1 << i) * nw + j / 64] |= 1ull << (j % 64);
            }
        std::vector<int> pc(NS, 0);
        for (int S = 1; S < NS; S++) {
            int low = S & -S;
            if (S != low)
                for (int w = 0; w < nw; w++) bits[(size_t)S * nw + w] = bits[(size_t)(S ^ low) * nw + w] ^ bits[(size_t)low * nw + w];
            int c = 0;
            for (int w = 0; w < nw; w++) c += __builtin_popcountll(bits[(size_t)S * nw + w]);
            pc[S] = c;
        }
        std::vector<double> cost(NS, 1e300);
        std::vector<int> split(NS, 0);
        for (int i = 0; i < m; i++) cost[1 << i] = 0.0;
        for (int S = 1; S < NS; S++) {
            if ((S & (S - 1)) == 0) continue;
            if (pc[S] > cap) continue;
            // enumerate splits S1 containing the lowest bit of S
            int low = S & -S;
            for (int S1 = (S - 1) & S; S1 > 0; S1 = (S1 - 1) & S) {
                if (!(S1 & low)) continue;
                int S2 = S ^ S1;
                if (cost[S1] >= 1e299 || cost[S2] >= 1e299) continue;
                int uni = 0;
                for (int w = 0; w < nw; w++)
                    uni += __builtin_popcountll(bits[(size_t)S1 * nw + w] | bits[(size_t)S2 * nw + w]);
                double c = cost[S1] + cost[S2] + std::ldexp(8.0, uni);
                if (c < cost[S]) {
                    cost[S] = c;
                    split[S] = S1;
                }
            }
        }
        if (!(cost[NS - 1] < old_cost * (1.0 - 1e-9))) continue;
        // rebuild: reuse the inner node ids (v keeps its id as the sub-tree root)
        std::vector<int> pool(inner.begin() + 1, inner.end());
        std::function<int(int, bool)> build = [&](int S, bool is_root) -> int {
            if ((S & (S - 1)) == 0) return front[__builtin_ctz(S)];
            int S1 = split[S], S2 = S ^ S1;
            int a = build(S1, false), c2 = build(S2, false);
            int id = is_root ? v : pool.back();
            if (!is_root) pool.pop_back();
            b.left[id] = a;
            b.right[id] = c2;
            std::vector<int> u;
            b.labels[id] = symdiff(b.labels[a], b.labels[c2], &u);
            return id;
        };
        build(NS - 1, true);
        improved++;
    }
    return improved;
}

// post-order SSA path of a BTree (inputs keep their ids)
std::vector<int> btree_ssa(const BTree &b) {
    std::vector<int> ssa;
    std::vector<int> newid(b.left.size(), -1);
    for (int i = 0; i < b.n; i++) newid[i] = i;
    int next = b.n;
    std::vector<std::pair<int, int>> st = {{b.root, 0}};
    while (!st.empty()) {
        auto &[v, state] = st.back();
        if (b.left[v] < 0) {
            st.pop_back();
            continue;
        }
        if (state == 0) {
            state = 1;
            int l = b.left[v], r = b.right[v];
            st.push_back({r, 0});
            st.push_back({l, 0});
            continue;
        }
        ssa.push_back(newid[b.left[v]]);
        ssa.push_back(newid[b.right[v]]);
        newid[v] = next++;
        st.pop_back();
    }
    return ssa;
}

Tree tree_from_ssa(const std::vector<std::vector<int>> &inputs, const std::vector<int> &ssa) {
    Tree t;
    t.labels = inputs;
    t.labels.resize(inputs.size() * 2 - 1);
    t.ssa = ssa;
    std::vector<int> u;
    for (size_t s = 0; s < ssa.size() / 2; s++) {
        t.labels[inputs.size() + s] = symdiff(t.labels[ssa[2 * s]], t.labels[ssa[2 * s + 1]], &u);
        t.uni.push_back(u);
    }
    return t;
}

}  // namespace

extern "C" int tnc_search(const tnc_network *net_h, int32_t n_open, const int32_t *open_qubits, double log2_cap,
                          int32_t cost_model, int32_t restarts, uint64_t seed, int32_t *ssa_out, int32_t max_sliced,
                          int32_t *sliced_out, int32_t *n_sliced, double *log2_cost_out) {
    try {
        if (!net_h || !ssa_out || !n_sliced || (max_sliced > 0 && !sliced_out)) TNC_THROW(TNC_EINVAL, "NULL argument");
        const Network &net = net_h->net;
        if (restarts < 1) TNC_THROW(TNC_EINVAL, "restarts < 1");
        if (net.hyperedges) TNC_THROW(TNC_EUNSUPPORTED, "the search takes networks whose labels join two tensors");
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
        const char *rc = getenv("TNC_SEARCH_RECONF");
        const int reconf_rounds = rc ? atoi(rc) : 8;
        struct Best {
            double cost = 1e300, flops = 0;
            std::vector<int> ssa, sl;
        };
        // One pass of restarts from the seed.  Cost of a candidate (log2): total
        // flops under the FLOP model, or the learned model's predicted device
        // time of the path the plan would run; it picks between the greedy
        // variants of a restart, decides whether a reconfigured tree replaces
        // the current one, and ranks the restarts.
        auto search_pass = [&](bool use_mlp) {
            std::mt19937_64 rng(seed);
            std::uniform_real_distribution<double> ua(0.6, 1.6), ut(0.0, 1.0);
            double best_cost = 1e300;
            std::vector<int> best_ssa, best_sl;
            double best_flops = 0;
            auto cost_of = [&](const Tree &tr, const Sliced &sv) -> double {
                if (use_mlp) {
                    double c = mlp_path_cost(net, tr.ssa, sv.labels, open_q);
                    if (c > 0) return std::log2(c);
                }
                return sv.log2_total;
            };
            for (int r = 0; r < restarts; r++) {
                double alpha = r == 0 ? 1.0 : ua(rng);
                double temp = r == 0 ? 0.0 : ut(rng) * ut(rng);
                std::vector<char> sl(L, 0);
                Tree t;
                Sliced s;
                double s_cost = 0;
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
                    const double c = cost_of(full, sc);
                    if (it == 0 || c < s_cost) {
                        t = full;
                        s = sc;
                        s_cost = c;
                    }
                    std::fill(sl.begin(), sl.end(), 0);
                    for (int l : s.labels) sl[l] = 1;
                }
                if (s.max_rank > log2_cap) continue;
                // local improvement: reconfigure sub-trees under the cap with the sliced
                // labels removed, then re-slice (the cap may now need fewer labels)
                if (reconf_rounds > 0) {
                    auto inputs = reduced_inputs(net, gone);
                    for (int rr = 0; rr < 2; rr++) {
                        std::vector<char> slv(L, 0);
                        for (int l : s.labels) slv[l] = 1;
                        BTree bt = to_btree(t, net.n_tensors, slv);
                        for (int q = 0; q < reconf_rounds; q++)
                            if (reconfigure_once(bt, log2_cap, rng) == 0) break;
                        Tree t2 = tree_from_ssa(inputs, btree_ssa(bt));
                        // drop sliced labels the new tree no longer needs, most expensive first
                        std::vector<char> sl2(L, 0);
                        Sliced s2 = slice_tree(t2, L, sliceable, log2_cap, sl2);
                        Sliced s3 = slice_tree(t2, L, sliceable, log2_cap, slv);
                        Sliced &pick = (s2.log2_total <= s3.log2_total) ? s2 : s3;
                        const double c2 = pick.max_rank <= log2_cap ? cost_of(t2, pick) : 1e300;
                        if (c2 < s_cost) {
                            t = t2;
                            s = pick;
                            s_cost = c2;
                        } else {
                            break;
                        }
                    }
                }
                const double cost = s_cost;
                if (cost < best_cost) {
                    best_cost = cost;
                    best_ssa = t.ssa;
                    best_sl = s.labels;
                    best_flops = s.log2_total;
                }
            }
            Best b;
            b.cost = best_cost;
            b.flops = best_flops;
            b.ssa = best_ssa;
            b.sl = best_sl;
            return b;
        };
        // Under the learned model the FLOP pass's choice is ranked beside the
        // model's own: the model leaves the FLOP path only for one it predicts
        // to be faster (the two passes search different candidate sets).
        Best pick = search_pass(false);
        if (cost_model == 1 && !pick.ssa.empty()) {
            const double cf = mlp_path_cost(net, pick.ssa, pick.sl, open_q);
            if (cf > 0) {
                Best m = search_pass(true);
                if (!m.ssa.empty() && m.cost < std::log2(cf)) pick = m;
            }
        }
        const std::vector<int> &best_ssa = pick.ssa, &best_sl = pick.sl;
        const double best_flops = pick.flops;
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

extern "C" int tnc_slice_path(const tnc_network *net_h, int32_t n_steps, const int32_t *ssa_pairs, int32_t n_open,
                              const int32_t *open_qubits, double log2_cap, int32_t n_in, const int32_t *sliced_in,
                              int32_t max_sliced, int32_t *sliced_out, int32_t *n_out) {
    try {
        if (!net_h || !ssa_pairs || !sliced_out || !n_out || (n_in > 0 && !sliced_in)) TNC_THROW(TNC_EINVAL, "NULL argument");
        const Network &net = net_h->net;
        if (n_steps != net.n_tensors - 1) TNC_THROW(TNC_EINVAL, "path must have n_tensors - 1 steps");
        if (net.hyperedges) TNC_THROW(TNC_EUNSUPPORTED, "the slicer takes networks whose labels join two tensors");
        const int L = net.n_labels;
        std::vector<char> gone(L, 0), sliceable(L, 1), is_open(net.n_qubits, 0);
        for (int i = 0; i < n_open; i++) {
            int q = open_qubits[i];
            if (q < 0 || q >= net.n_qubits || is_open[q]) TNC_THROW(TNC_EINVAL, "bad open qubit list");
            is_open[q] = 1;
        }
        for (int q = 0; q < net.n_qubits; q++) {
            sliceable[net.output_labels[q]] = 0;
            if (!is_open[q]) gone[net.output_labels[q]] = 1;
        }
        std::vector<int> ssa(ssa_pairs, ssa_pairs + 2 * n_steps);
        Tree t = tree_from_ssa(reduced_inputs(net, gone), ssa);
        std::vector<char> sl(L, 0);
        for (int j = 0; j < n_in; j++) {
            int l = sliced_in[j];
            if (l < 0 || l >= L || !sliceable[l]) TNC_THROW(TNC_EINVAL, "bad sliced label");
            sl[l] = 1;
        }
        Sliced s = slice_tree(t, L, sliceable, log2_cap, sl);
        if (s.max_rank > log2_cap) TNC_THROW(TNC_EINVAL, "the cap cannot be met by slicing");
        std::vector<int> out(sliced_in, sliced_in + n_in);
        for (int l : s.labels)
            if (std::find(out.begin(), out.end(), l) == out.end()) out.push_back(l);
        if ((int)out.size() > max_sliced) TNC_THROW(TNC_EINVAL, "more sliced labels than max_sliced");
        std::copy(out.begin(), out.end(), sliced_out);
        *n_out = (int)out.size();
        return TNC_OK;
    } catch (const Error &e) {
        set_error(e.msg);
        return e.code;
    } catch (const std::exception &e) {
        set_error(e.what());
        return TNC_EINVAL;
    }
}
