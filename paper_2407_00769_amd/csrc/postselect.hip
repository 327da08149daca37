// Top-k post-selection in a correlated subspace (paper Sec. 1 and Sec. 2.3,
// post-processing): the k most probable of N amplitudes.
//
// Probability p = re*re + im*im in FP64 with each operation rounded on its own;
// order: larger probability first, then smaller index (a total order, so the
// list is unique even with ties).  Each block sorts a tile of 2048 (p, index)
// pairs in LDS with a bitonic network and keeps its first k; rounds repeat on
// the kept candidates until one tile holds them all.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "common.h"

namespace tnc {

constexpr int kTopkTile = 2048;
constexpr int kTopkThreads = 512;

__device__ __forceinline__ bool topk_before(double pa, int64_t ia, double pb, int64_t ib) {
    return pa > pb || (pa == pb && ia < ib);
}

// FROM_AMPS: the input is n complex128 amplitudes (interleaved re, im) and the
// index of entry g is g; otherwise it is (probability, index) pairs kept by an
// earlier round.  Padding past n sorts last (probability -1).
template <bool FROM_AMPS>
__global__ void __launch_bounds__(kTopkThreads)
    topk_tile_kernel(const double *__restrict__ amps, const double *__restrict__ in_p,
                     const int64_t *__restrict__ in_i, int64_t n, int k, double *__restrict__ out_p,
                     int64_t *__restrict__ out_i) {
    __shared__ double sp[kTopkTile];
    __shared__ int64_t si[kTopkTile];
    const int64_t base = (int64_t)blockIdx.x * kTopkTile;
    for (int t = threadIdx.x; t < kTopkTile; t += kTopkThreads) {
        const int64_t g = base + t;
        double p = -1.0;
        int64_t id = INT64_MAX;
        if (g < n) {
            if constexpr (FROM_AMPS) {
                const double re = amps[2 * g], im = amps[2 * g + 1];
                p = __dadd_rn(__dmul_rn(re, re), __dmul_rn(im, im));
                id = g;
            } else {
                p = in_p[g];
                id = in_i[g];
            }
        }
        sp[t] = p;
        si[t] = id;
    }
    __syncthreads();
    for (int size = 2; size <= kTopkTile; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = threadIdx.x; t < kTopkTile / 2; t += kTopkThreads) {
                const int lo = 2 * t - (t & (stride - 1)), hi = lo + stride;
                const bool first_half = (lo & size) == 0;   // this run ends up in "before" order
                const double pl = sp[lo], ph = sp[hi];
                const int64_t il = si[lo], ih = si[hi];
                const bool swap = first_half ? topk_before(ph, ih, pl, il) : topk_before(pl, il, ph, ih);
                if (swap) {
                    sp[lo] = ph;
                    sp[hi] = pl;
                    si[lo] = ih;
                    si[hi] = il;
                }
            }
            __syncthreads();
        }
    }
    for (int t = threadIdx.x; t < k; t += kTopkThreads) {
        out_p[(int64_t)blockIdx.x * k + t] = sp[t];
        out_i[(int64_t)blockIdx.x * k + t] = si[t];
    }
}

int64_t topk_scratch_entries(int64_t n, int k) {
    if (n <= kTopkTile) return 0;
    return ((n + kTopkTile - 1) / kTopkTile) * (int64_t)k;
}

// scratch: two buffers of topk_scratch_entries(n, k) (p, index) pairs each
void launch_topk(int64_t n, const double *amps, int k, double *prob_out, int64_t *idx_out, double *scr_p0,
                 int64_t *scr_i0, double *scr_p1, int64_t *scr_i1, hipStream_t st) {
    if (n <= 0) return;
    const int kk = (int64_t)k < n ? k : (int)n;
    bool from_amps = true;
    const double *src_p = nullptr;
    const int64_t *src_i = nullptr;
    int64_t count = n;
    int cur = 0;
    while (true) {
        const int64_t nblk = (count + kTopkTile - 1) / kTopkTile;
        const bool last = nblk == 1;
        double *dp = last ? prob_out : (cur ? scr_p1 : scr_p0);
        int64_t *di = last ? idx_out : (cur ? scr_i1 : scr_i0);
        const int kout = last ? kk : k;
        if (from_amps)
            hipLaunchKernelGGL(topk_tile_kernel<true>, dim3((unsigned)nblk), dim3(kTopkThreads), 0, st, amps,
                               nullptr, nullptr, count, kout, dp, di);
        else
            hipLaunchKernelGGL(topk_tile_kernel<false>, dim3((unsigned)nblk), dim3(kTopkThreads), 0, st, nullptr,
                               src_p, src_i, count, kout, dp, di);
        HIP_CHECK(hipGetLastError());
        if (last) break;
        from_amps = false;
        src_p = dp;
        src_i = di;
        count = nblk * k;
        cur ^= 1;
    }
}

}  // namespace tnc
