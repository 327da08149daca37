// Host-side launch guards of the GEMM dispatcher, exercised without a GPU:
// every check below throws before any HIP call, so the program needs no
// device.  Exit status 0 when every guard fires with TNC_EINVAL.
#include <cstdio>
#include <cstring>
#include <string>

#include "common.h"

using namespace tnc;

static int expect_einval(const char *what, const std::string &needle, void (*fn)()) {
    try {
        fn();
    } catch (const Error &e) {
        if (e.code == TNC_EINVAL && e.msg.find(needle) != std::string::npos) {
            std::printf("ok   %s: %s\n", what, e.msg.c_str());
            return 0;
        }
        std::printf("FAIL %s: code %d, message %s\n", what, e.code, e.msg.c_str());
        return 1;
    }
    std::printf("FAIL %s: no error\n", what);
    return 1;
}

// a long-k, one-tile shape on the 256 x 128 LDS-DMA tile: split-K applies
static GemmShape long_k() {
    GemmShape g{};
    g.M = 256;
    g.N = 128;
    g.K = 1 << 14;
    g.nb = 1;
    g.bA = g.M * g.K;
    g.bB = g.N * g.K;
    g.bC = g.M * g.N;
    set_plain_segs(g);
    return g;
}

static float2 g_dummy[4];

static void split_buffer_too_small() {
    GemmShape g = long_k();
    if (splitk_factor(K_DMA_8, Dtype::F16, Algo::M4, g, 1) < 2) throw Error{0, "shape does not split"};
    g.part = g_dummy;
    g.part_cap = sizeof(g_dummy);   // far below split x M x N x 8 bytes
    ScaleRefs sc{};
    launch_gemm(K_DMA_8, Dtype::F16, Algo::M4, g_dummy, g_dummy, g_dummy, g, 1, &sc, nullptr);
}

static void more_slices_than_sized() {
    GemmShape g = long_k();
    g.part = g_dummy;
    g.part_cap = 1ll << 40;
    g.split_slices = 2;   // the buffer was sized for 2 slices; the launch asks for 4
    ScaleRefs sc{};
    launch_gemm(K_DMA_8, Dtype::F16, Algo::M4, g_dummy, g_dummy, g_dummy, g, 4, &sc, nullptr);
}

static void unsupported_shape() {
    GemmShape g = long_k();
    g.M = 200;   // not a whole number of 256-row tiles
    ScaleRefs sc{};
    launch_gemm(K_DMA_8, Dtype::F16, Algo::M4, g_dummy, g_dummy, g_dummy, g, 1, &sc, nullptr);
}

static void missing_scale_bookkeeping() {
    GemmShape g = long_k();
    launch_gemm(K_DMA_8, Dtype::F16, Algo::M4, g_dummy, g_dummy, g_dummy, g, 1, nullptr, nullptr);
}

int main() {
    int bad = 0;
    bad += expect_einval("split-K buffer capacity", "split-K partial sums need", split_buffer_too_small);
    bad += expect_einval("split-K slice count", "more slices than its split-K buffer", more_slices_than_sized);
    bad += expect_einval("shape support", "cannot run this shape", unsupported_shape);
    bad += expect_einval("scale bookkeeping", "scale bookkeeping", missing_scale_bookkeeping);
    return bad ? 1 : 0;
}
