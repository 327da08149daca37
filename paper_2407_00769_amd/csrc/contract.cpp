// tnc_contract: one pairwise contraction on device-resident operands
// (paper Eq. contraction): permute the operands into GEMM form if needed, one
// batched complex GEMM, and a permute of the result if the requested output
// order is not the GEMM's.
#include <algorithm>
#include <cstring>

#include "engine.h"

using namespace tnc;

namespace {

std::vector<int> keep_order(const std::vector<int> &order, const std::vector<int> &set) {
    std::vector<int> r;
    for (int l : order)
        if (std::find(set.begin(), set.end(), l) != set.end()) r.push_back(l);
    return r;
}

std::vector<int> cat(std::initializer_list<const std::vector<int> *> parts) {
    std::vector<int> r;
    for (auto *p : parts) r.insert(r.end(), p->begin(), p->end());
    return r;
}

}  // namespace

extern "C" int tnc_contract(tnc_ctx *ctx, tnc_precision prec, const void *A, int32_t a_rank, const int32_t *a_labels,
                            const void *B, int32_t b_rank, const int32_t *b_labels, void *C, int32_t c_rank,
                            const int32_t *c_labels, int32_t scale_log2, double *times_ms, float *max_abs_out) {
    try {
        if (!ctx || !A || !B || !C) TNC_THROW(TNC_EINVAL, "NULL tensor or context");
        if ((int)prec < 0 || (int)prec > 4) TNC_THROW(TNC_EINVAL, "unknown precision");
        if (a_rank < 0 || b_rank < 0 || c_rank < 0 || a_rank > kMaxRank || b_rank > kMaxRank || c_rank > kMaxRank)
            TNC_THROW(TNC_EINVAL, "rank out of range");
        const Dtype dt = dtype_of(prec);
        const Algo al = algo_of(prec);
        std::vector<int> la(a_labels, a_labels + a_rank), lb(b_labels, b_labels + b_rank),
            lc(c_labels, c_labels + c_rank);
        auto has = [](const std::vector<int> &v, int l) { return std::find(v.begin(), v.end(), l) != v.end(); };
        for (const auto *v : {&la, &lb, &lc}) {
            std::vector<int> s = *v;
            std::sort(s.begin(), s.end());
            if (std::adjacent_find(s.begin(), s.end()) != s.end()) TNC_THROW(TNC_EINVAL, "a label repeats within a tensor");
        }
        std::vector<int> beta, m, n, k;
        for (int l : la) {
            bool inb = has(lb, l), inc = has(lc, l);
            if (inb && inc) beta.push_back(l);
            else if (inb) k.push_back(l);
            else if (inc) m.push_back(l);
            else TNC_THROW(TNC_EINVAL, "label of A is neither in B nor in C");
        }
        for (int l : lb) {
            bool ina = has(la, l), inc = has(lc, l);
            if (!ina && inc) n.push_back(l);
            else if (!ina) TNC_THROW(TNC_EINVAL, "label of B is neither in A nor in C");
        }
        for (int l : lc)
            if (!has(la, l) && !has(lb, l)) TNC_THROW(TNC_EINVAL, "label of C is in neither operand");
        if (dt == Dtype::C64 && al == Algo::M3) TNC_THROW(TNC_EINVAL, "3M needs 16-bit storage");

        // roles: rows operand R (the one with more free labels), cols operand Q
        const void *R = A, *Q = B;
        std::vector<int> lr = la, lq = lb, fr = m, fq = n;
        if (n.size() > m.size()) {
            std::swap(R, Q);
            std::swap(lr, lq);
            std::swap(fr, fq);
        }
        // Index orders.  A tensor is used in place when its batch labels form
        // the top block in the batch order and each of its two GEMM indices
        // lies in at most two runs, the lowest run holding a whole 16-byte
        // chunk; otherwise it is permuted to (or from) [batch][i1][i2].  Every
        // choice of orders taken from the tensors is tried; the one that
        // permutes the fewest bytes wins.
        const int lq_bits = dt == Dtype::C64 ? 1 : 2;
        struct Side {
            bool inplace = false;
            int kc = 1;
            Seg s1, s2;
        };
        auto check = [&](const std::vector<int> &order, const std::vector<int> &bo, const std::vector<int> &i1,
                         const std::vector<int> &i2, Side &sd) {
            sd = Side{};
            if (!std::equal(bo.begin(), bo.end(), order.begin())) return;
            Seg s1, s2;
            if (!derive_seg(order, i1, s1) || !derive_seg(order, i2, s2)) return;
            if (order.size() == bo.size()) {   // batch only
                sd = Side{true, 1, s1, s2};
                return;
            }
            const bool low2 = has(i2, order.back());
            const Seg &cs = low2 ? s2 : s1;
            const int64_t ext = (int64_t)1 << (low2 ? i2.size() : i1.size());
            if (cs.ls != 0 || seg_low_run(cs, ext) < lq_bits) return;
            sd = Side{true, low2 ? 1 : 0, s1, s2};
        };
        const int64_t nr = (int64_t)1 << lr.size(), nq = (int64_t)1 << lq.size(), nc = (int64_t)1 << lc.size();
        std::vector<int> bo, mo, no, ko;
        Side sr, sq, sc_;
        double best = -1;
        for (const auto *bsrc : {&lc, &lr, &lq})
            for (const auto *msrc : {&lr, &lc})
                for (const auto *nsrc : {&lq, &lc})
                    for (const auto *ksrc : {&lr, &lq}) {
                        std::vector<int> b1 = keep_order(*bsrc, beta), m1 = keep_order(*msrc, fr),
                                         n1 = keep_order(*nsrc, fq), k1 = keep_order(*ksrc, k);
                        Side x, y, z;
                        check(lr, b1, m1, k1, x);
                        check(lq, b1, n1, k1, y);
                        check(lc, b1, m1, n1, z);
                        double cost = (x.inplace ? 0.0 : (double)nr) + (y.inplace ? 0.0 : (double)nq) +
                                      (z.inplace ? 0.0 : (double)nc);
                        if (best < 0 || cost < best) {
                            best = cost;
                            bo = b1;
                            mo = m1;
                            no = n1;
                            ko = k1;
                            sr = x;
                            sq = y;
                            sc_ = z;
                        }
                    }
        std::vector<int> want_r = cat({&bo, &mo, &ko}), want_q = cat({&bo, &no, &ko}), gemm_c = cat({&bo, &mo, &no});
        const bool perm_r = !sr.inplace, perm_q = !sq.inplace, perm_c = !sc_.inplace;
        const int es = elem_bytes(dt);
        auto al256 = [](int64_t v) { return (v + 255) & ~(int64_t)255; };
        int64_t off = 0, off_r = 0, off_q = 0, off_c = 0;
        if (perm_r) { off_r = off; off += al256(nr * es); }
        if (perm_q) { off_q = off; off += al256(nq * es); }
        if (perm_c) { off_c = off; off += al256(nc * es); }
        if ((size_t)off > ctx->ws_bytes) TNC_THROW(TNC_ENOMEM, "workspace too small for the permuted operands");
        HIP_CHECK(hipSetDevice(ctx->device));
        hipStream_t st = ctx->stream;
        // scale bookkeeping in the context's small buffer: maxA = maxB = 1.0,
        // so shift = growth - target = scale_log2
        uint8_t *sm = ctx->small;
        ScaleRefs sc{};
        if (dt != Dtype::C64) {
            struct Small {
                uint32_t maxA, maxB, maxC, flag;
                int growth, shift, pad0, pad1;
                double expA, expB, expC;
            } h{0x3f800000u, 0x3f800000u, 0u, 0u, scale_log2 + 13, 0, 0, 0, 0.0, 0.0, 0.0};
            HIP_CHECK(hipMemcpyAsync(sm, &h, sizeof(h), hipMemcpyHostToDevice, st));
            HIP_CHECK(hipStreamSynchronize(st));   // h lives on this stack frame
            Small *d = (Small *)sm;
            sc.maxA = &d->maxA;
            sc.maxB = &d->maxB;
            sc.maxC = &d->maxC;
            sc.flag = &d->flag;
            sc.growth = &d->growth;
            sc.shift = &d->shift;
            sc.expA = &d->expA;
            sc.expB = &d->expB;
            sc.expC = &d->expC;
        }
        hipEvent_t ev[5];
        for (auto &e : ev) HIP_CHECK(hipEventCreate(&e));
        HIP_CHECK(hipEventRecord(ev[0], st));
        const void *pr = R, *pq = Q;
        if (perm_r) {
            launch_permute(dt, R, ctx->ws + off_r, make_permute(lr, want_r), nr, 1, 0, nullptr, 0, st);
            pr = ctx->ws + off_r;
        }
        HIP_CHECK(hipEventRecord(ev[1], st));
        if (perm_q) {
            launch_permute(dt, Q, ctx->ws + off_q, make_permute(lq, want_q), nq, 1, 0, nullptr, 0, st);
            pq = ctx->ws + off_q;
        }
        HIP_CHECK(hipEventRecord(ev[2], st));
        GemmShape g{};
        g.nb = (int64_t)1 << bo.size();
        g.M = (int64_t)1 << mo.size();
        g.N = (int64_t)1 << no.size();
        g.K = (int64_t)1 << ko.size();
        g.bA = g.M * g.K;
        g.bB = g.N * g.K;
        g.bC = g.M * g.N;
        g.a_kc = perm_r ? 1 : sr.kc;
        g.b_kc = perm_q ? 1 : sq.kc;
        g.c_nc = perm_c ? 1 : sc_.kc;
        set_plain_segs(g);
        if (!perm_r) {
            g.am = sr.s1;
            g.ak = sr.s2;
        }
        if (!perm_q) {
            g.bn = sq.s1;
            g.bk = sq.s2;
        }
        if (!perm_c) {
            g.cm = sc_.s1;
            g.cn = sc_.s2;
        }
        void *pc = perm_c ? (void *)(ctx->ws + off_c) : C;
        int kid = choose_kernel(dt, al, g);
        const char *force = getenv("TNC_FORCE_KERNEL");
        if (force) {
            int f = atoi(force);
            if (gemm_supported(f, dt, al, g)) kid = f;
        }
        // split-K partial sums go to the workspace after the permute scratch
        int64_t pb = splitk_bytes(kid, dt, al, g, 1);
        if (pb > 0 && (size_t)(off + pb) <= ctx->ws_bytes) {
            g.part = (float2 *)(ctx->ws + off);
            g.part_cap = pb;
        }
        launch_gemm(kid, dt, al, pr, pq, pc, g, 1, dt != Dtype::C64 ? &sc : nullptr, st);
        HIP_CHECK(hipEventRecord(ev[3], st));
        if (perm_c) launch_permute(dt, pc, C, make_permute(gemm_c, lc), nc, 1, 0, nullptr, 0, st);
        HIP_CHECK(hipEventRecord(ev[4], st));
        HIP_CHECK(hipEventSynchronize(ev[4]));
        if (times_ms) {
            float t;
            for (int i = 0; i < 4; i++) {
                HIP_CHECK(hipEventElapsedTime(&t, ev[i], ev[i + 1]));
                times_ms[i] = t;
            }
        }
        for (auto &e : ev) hipEventDestroy(e);
        if (max_abs_out) {
            if (dt == Dtype::C64) {
                *max_abs_out = 0.f;
            } else {
                uint32_t w = 0;
                HIP_CHECK(hipMemcpy(&w, sm + 8, 4, hipMemcpyDeviceToHost));
                float f;
                std::memcpy(&f, &w, 4);
                *max_abs_out = f;
            }
        }
        return TNC_OK;
    } catch (const Error &e) {
        set_error(e.msg);
        return e.code;
    } catch (const std::exception &e) {
        set_error(e.what());
        return TNC_EINVAL;
    }
}
