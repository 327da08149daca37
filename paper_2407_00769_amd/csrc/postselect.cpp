// C ABI of the top-k post-selection (paper Sec. 1 and Sec. 2.3): argument
// checks, the workspace split for the candidate rounds, and timing.
#include "engine.h"

using namespace tnc;

namespace tnc {
int64_t topk_scratch_entries(int64_t n, int k);
void launch_topk(int64_t n, const double *amps, int k, double *prob_out, int64_t *idx_out, double *scr_p0,
                 int64_t *scr_i0, double *scr_p1, int64_t *scr_i1, hipStream_t st);
}  // namespace tnc

extern "C" int tnc_topk(tnc_ctx *ctx, int64_t n, const double *amps, int32_t k, int64_t *idx_out, double *prob_out,
                        double *ms_out) {
    try {
        if (!ctx) TNC_THROW(TNC_EINVAL, "NULL context");
        if (n < 0) TNC_THROW(TNC_EINVAL, "negative length");
        if (k < 1 || k > 1024) TNC_THROW(TNC_EINVAL, "k must be in 1..1024");
        if (ms_out) *ms_out = 0.0;
        if (n == 0) return TNC_OK;
        if (!amps || !idx_out || !prob_out) TNC_THROW(TNC_EINVAL, "NULL buffer");
        if (((uintptr_t)amps | (uintptr_t)idx_out | (uintptr_t)prob_out) & 7u)
            TNC_THROW(TNC_EINVAL, "buffers must be 8-byte aligned");
        const int64_t e = topk_scratch_entries(n, k);
        if ((uint64_t)(32 * e) > (uint64_t)ctx->ws_bytes)
            TNC_THROW(TNC_ENOMEM, "workspace too small for the candidate rounds");
        double *p0 = (double *)ctx->ws, *p1 = p0 + 2 * e;
        int64_t *i0 = (int64_t *)(p0 + e), *i1 = (int64_t *)(p1 + e);
        HIP_CHECK(hipSetDevice(ctx->device));
        hipStream_t st = ctx->stream;
        hipEvent_t e0, e1;
        HIP_CHECK(hipEventCreate(&e0));
        HIP_CHECK(hipEventCreate(&e1));
        HIP_CHECK(hipEventRecord(e0, st));
        launch_topk(n, amps, k, prob_out, idx_out, p0, i0, p1, i1, st);
        HIP_CHECK(hipEventRecord(e1, st));
        HIP_CHECK(hipEventSynchronize(e1));
        float ms = 0.f;
        HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
        if (ms_out) *ms_out = ms;
        hipEventDestroy(e0);
        hipEventDestroy(e1);
        return TNC_OK;
    } catch (const Error &err) {
        set_error(err.msg);
        return err.code;
    }
}
