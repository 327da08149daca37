// C ABI of the low-precision exchange codec (paper Sec. 3.2): argument
// checks, sizes and the launches of codec.hip on the context's stream.
#include <cstring>

#include "engine.h"

using namespace tnc;

namespace tnc {

int codec_group(int32_t kind, int32_t group) {
    if (kind < 0 || kind > 2) TNC_THROW(TNC_EINVAL, "unknown codec kind");
    if (kind != 2) {
        if (group != 0) TNC_THROW(TNC_EINVAL, "half and int8 use one group (the whole tensor): pass group 0");
        return 0;
    }
    if (group == 0) return 128;
    for (int g = 16; g <= 1024; g *= 2)
        if (group == g) return g;
    TNC_THROW(TNC_EINVAL, "int4 group size must be a power of two from 16 to 1024");
}

}  // namespace tnc

namespace {

bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

}  // namespace

extern "C" int tnc_quant_sizes(int32_t kind, int64_t n, int32_t group, int64_t *code_bytes, int64_t *n_groups) {
    try {
        if (n < 0) TNC_THROW(TNC_EINVAL, "negative length");
        const int g = codec_group(kind, group);
        const int64_t cb = kind == 0 ? 2 * n : (kind == 1 ? n : (n + 1) / 2);
        const int64_t ng = kind == 2 ? (n + g - 1) / g : (n > 0 ? 1 : 0);
        if (code_bytes) *code_bytes = cb;
        if (n_groups) *n_groups = ng;
        return TNC_OK;
    } catch (const Error &e) {
        set_error(e.msg);
        return e.code;
    }
}

extern "C" int tnc_quantize(tnc_ctx *ctx, int32_t kind, int64_t n, const float *x, int32_t group, void *codes,
                            float *scales, float *zeros, double *ms_out) {
    try {
        if (!ctx) TNC_THROW(TNC_EINVAL, "NULL context");
        if (n < 0) TNC_THROW(TNC_EINVAL, "negative length");
        const int g = codec_group(kind, group);
        if (n == 0) {
            if (ms_out) *ms_out = 0.0;
            return TNC_OK;
        }
        if (!x || !codes || !scales || !zeros) TNC_THROW(TNC_EINVAL, "NULL buffer");
        if (!aligned16(x) || !aligned16(codes)) TNC_THROW(TNC_EINVAL, "values and codes must be 16-byte aligned");
        HIP_CHECK(hipSetDevice(ctx->device));
        hipStream_t st = ctx->stream;
        hipEvent_t e0, e1;
        HIP_CHECK(hipEventCreate(&e0));
        HIP_CHECK(hipEventCreate(&e1));
        HIP_CHECK(hipEventRecord(e0, st));
        launch_quantize(kind, n, g, x, codes, scales, zeros, (float2 *)ctx->small, st);
        HIP_CHECK(hipEventRecord(e1, st));
        HIP_CHECK(hipEventSynchronize(e1));
        float ms = 0.f;
        HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
        if (ms_out) *ms_out = ms;
        hipEventDestroy(e0);
        hipEventDestroy(e1);
        return TNC_OK;
    } catch (const Error &e) {
        set_error(e.msg);
        return e.code;
    }
}

extern "C" int tnc_dequantize(tnc_ctx *ctx, int32_t kind, int64_t n, const void *codes, const float *scales,
                              const float *zeros, int32_t group, float *x, double *ms_out) {
    try {
        if (!ctx) TNC_THROW(TNC_EINVAL, "NULL context");
        if (n < 0) TNC_THROW(TNC_EINVAL, "negative length");
        const int g = codec_group(kind, group);
        if (n == 0) {
            if (ms_out) *ms_out = 0.0;
            return TNC_OK;
        }
        if (!x || !codes || !scales || !zeros) TNC_THROW(TNC_EINVAL, "NULL buffer");
        if (!aligned16(x) || !aligned16(codes)) TNC_THROW(TNC_EINVAL, "values and codes must be 16-byte aligned");
        HIP_CHECK(hipSetDevice(ctx->device));
        hipStream_t st = ctx->stream;
        hipEvent_t e0, e1;
        HIP_CHECK(hipEventCreate(&e0));
        HIP_CHECK(hipEventCreate(&e1));
        HIP_CHECK(hipEventRecord(e0, st));
        launch_dequantize(kind, n, g, codes, scales, zeros, x, st);
        HIP_CHECK(hipEventRecord(e1, st));
        HIP_CHECK(hipEventSynchronize(e1));
        float ms = 0.f;
        HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
        if (ms_out) *ms_out = ms;
        hipEventDestroy(e0);
        hipEventDestroy(e1);
        return TNC_OK;
    } catch (const Error &e) {
        set_error(e.msg);
        return e.code;
    }
}
