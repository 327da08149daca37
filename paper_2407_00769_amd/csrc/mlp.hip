// Learned step-cost model: a 3-layer MLP (in -> 128 -> 128 -> 1, ReLU, FP32)
// trained on the device by the kernels below (forward, backward, Adam) on
// timings the engine measures.  As the search's cost model it predicts a
// step's log2 device time in microseconds as a roofline baseline computed
// from the same features (step_base_log2_us) plus the network's output, the
// learned log2 ratio of measured to baseline time; it ranks the candidate
// paths of tnc_search (cost_model = 1).  A step unlike any training row then
// keeps the baseline's scaling with its work instead of an extrapolation of
// the network.
//
// Parameter layout (one float array): W1[128][F], b1[128], W2[128][128], b2[128],
// W3[1][128], b3[1].  Inputs are multiplied by a fixed per-feature scale
// (kInScale) before the first layer so every feature is O(1).
//
// Every reduction runs in a fixed order (one thread per output, loops over
// rows in index order), so training is deterministic for a given seed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <numeric>
#include <random>

#include "engine.h"
#include "planner.h"

namespace tnc {

constexpr int F = TNC_MLP_FEATURES;
constexpr int H = TNC_MLP_HIDDEN;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + H * F, OFF_W2 = OFF_B1 + H, OFF_B2 = OFF_W2 + H * H,
              OFF_W3 = OFF_B2 + H, OFF_B3 = OFF_W3 + H, NPARAM = OFF_B3 + 1;

// log2 M, N, K, batch (/16, /16, /16, /8); stride classes (/3); dtype (/2); algorithm
__constant__ float kInScale[F] = {1.f / 16, 1.f / 16, 1.f / 16, 1.f / 8, 1.f / 3, 1.f / 3, 1.f / 2, 1.f};

struct Mlp {
    float *params = nullptr, *grads = nullptr, *m = nullptr, *v = nullptr;   // device, NPARAM each
    int64_t cap = 0;                                                            // rows the buffers hold
    float *x = nullptr, *y = nullptr, *h1 = nullptr, *h2 = nullptr, *out = nullptr, *dout = nullptr,
          *dh1 = nullptr, *dh2 = nullptr, *loss = nullptr;
    int *idx = nullptr;
    int64_t step = 0;
    bool trained = false;
    // the range of the size features (log2 M, N, K, batch) in the rows the
    // weights were trained on; set by training, cleared by tnc_mlp_set_params
    bool support = false;
    float lo[4] = {0, 0, 0, 0}, hi[4] = {0, 0, 0, 0};
};

// Record the size-feature range of n training rows (host array, F per row).
static void set_support(Mlp *m, int64_t n, const float *x) {
    for (int f = 0; f < 4; f++) {
        m->lo[f] = x[f];
        m->hi[f] = x[f];
    }
    for (int64_t r = 1; r < n; r++)
        for (int f = 0; f < 4; f++) {
            m->lo[f] = std::min(m->lo[f], x[r * F + f]);
            m->hi[f] = std::max(m->hi[f], x[r * F + f]);
        }
    m->support = true;
}

static thread_local tnc_ctx *g_cost_ctx = nullptr;

// ------------------------------------------------------------------ kernels

// one block (H threads) per row: hidden layers and output
__global__ void __launch_bounds__(H) mlp_forward_kernel(const float *__restrict__ p, const float *__restrict__ x,
                                                        const int *__restrict__ idx, int64_t rows,
                                                        float *__restrict__ h1, float *__restrict__ h2,
                                                        float *__restrict__ out) {
    __shared__ float sh1[H], sx[F], red[H];
    const int j = threadIdx.x;
    for (int64_t r = blockIdx.x; r < rows; r += gridDim.x) {
        const int64_t src = idx ? idx[r] : r;
        if (j < F) sx[j] = x[src * F + j] * kInScale[j];
        __syncthreads();
        float a = p[OFF_B1 + j];
        for (int i = 0; i < F; i++) a = fmaf(p[OFF_W1 + j * F + i], sx[i], a);
        a = fmaxf(a, 0.f);
        sh1[j] = a;
        h1[r * H + j] = a;
        __syncthreads();
        float b = p[OFF_B2 + j];
        for (int i = 0; i < H; i++) b = fmaf(p[OFF_W2 + j * H + i], sh1[i], b);
        b = fmaxf(b, 0.f);
        h2[r * H + j] = b;
        red[j] = p[OFF_W3 + j] * b;
        __syncthreads();
        if (j == 0) {
            float s = p[OFF_B3];
            for (int i = 0; i < H; i++) s += red[i];
            out[r] = s;
        }
        __syncthreads();
    }
}

// dL/dout for L = mean (out - y)^2, then per row dh2 and dh1
__global__ void __launch_bounds__(H) mlp_backward_rows_kernel(const float *__restrict__ p, const float *__restrict__ y,
                                                              const int *__restrict__ idx, int64_t rows,
                                                              const float *__restrict__ h1, const float *__restrict__ h2,
                                                              const float *__restrict__ out, float *__restrict__ dout,
                                                              float *__restrict__ dh1, float *__restrict__ dh2) {
    __shared__ float sd2[H];
    const int j = threadIdx.x;
    for (int64_t r = blockIdx.x; r < rows; r += gridDim.x) {
        const int64_t src = idx ? idx[r] : r;
        const float g = 2.f * (out[r] - y[src]) / (float)rows;
        if (j == 0) dout[r] = g;
        float d2 = h2[r * H + j] > 0.f ? g * p[OFF_W3 + j] : 0.f;
        sd2[j] = d2;
        dh2[r * H + j] = d2;
        __syncthreads();
        float d1 = 0.f;
        for (int k = 0; k < H; k++) d1 = fmaf(sd2[k], p[OFF_W2 + k * H + j], d1);
        dh1[r * H + j] = h1[r * H + j] > 0.f ? d1 : 0.f;
        __syncthreads();
    }
}

// one thread per parameter, rows summed in index order
__global__ void mlp_grad_kernel(const float *__restrict__ x, const int *__restrict__ idx, int64_t rows,
                                const float *__restrict__ h1, const float *__restrict__ h2,
                                const float *__restrict__ dout, const float *__restrict__ dh1,
                                const float *__restrict__ dh2, float *__restrict__ grads) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= NPARAM) return;
    float s = 0.f;
    if (q < OFF_B1) {
        int j = q / F, i = q % F;
        for (int64_t r = 0; r < rows; r++) {
            int64_t src = idx ? idx[r] : r;
            s = fmaf(dh1[r * H + j], x[src * F + i] * kInScale[i], s);
        }
    } else if (q < OFF_W2) {
        int j = q - OFF_B1;
        for (int64_t r = 0; r < rows; r++) s += dh1[r * H + j];
    } else if (q < OFF_B2) {
        int j = (q - OFF_W2) / H, i = (q - OFF_W2) % H;
        for (int64_t r = 0; r < rows; r++) s = fmaf(dh2[r * H + j], h1[r * H + i], s);
    } else if (q < OFF_W3) {
        int j = q - OFF_B2;
        for (int64_t r = 0; r < rows; r++) s += dh2[r * H + j];
    } else if (q < OFF_B3) {
        int j = q - OFF_W3;
        for (int64_t r = 0; r < rows; r++) s = fmaf(dout[r], h2[r * H + j], s);
    } else {
        for (int64_t r = 0; r < rows; r++) s += dout[r];
    }
    grads[q] = s;
}

__global__ void mlp_adam_kernel(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                                float *__restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= NPARAM) return;
    float gg = g[q];
    float mm = b1 * m[q] + (1.f - b1) * gg;
    float vv = b2 * v[q] + (1.f - b2) * gg * gg;
    m[q] = mm;
    v[q] = vv;
    p[q] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

// mean squared error, one thread, rows in order
__global__ void mlp_loss_kernel(const float *__restrict__ y, const int *__restrict__ idx, int64_t rows,
                                const float *__restrict__ out, float *__restrict__ loss) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    double s = 0.0;
    for (int64_t r = 0; r < rows; r++) {
        int64_t src = idx ? idx[r] : r;
        double d = (double)out[r] - (double)y[src];
        s += d * d;
    }
    *loss = (float)(s / (double)(rows > 0 ? rows : 1));
}

// ------------------------------------------------------------------ host side

void mlp_free(Mlp *m) {
    if (!m) return;
    float *fs[] = {m->params, m->grads, m->m, m->v, m->x, m->y, m->h1, m->h2, m->out, m->dout, m->dh1, m->dh2, m->loss};
    for (float *f : fs)
        if (f) hipFree(f);
    if (m->idx) hipFree(m->idx);
    delete m;
}

static Mlp *mlp_of(tnc_ctx *ctx) {
    if (!ctx->mlp) {
        Mlp *m = new Mlp;
        ctx->mlp = m;
        HIP_CHECK(hipMalloc((void **)&m->params, NPARAM * sizeof(float)));
        HIP_CHECK(hipMalloc((void **)&m->grads, NPARAM * sizeof(float)));
        HIP_CHECK(hipMalloc((void **)&m->m, NPARAM * sizeof(float)));
        HIP_CHECK(hipMalloc((void **)&m->v, NPARAM * sizeof(float)));
        HIP_CHECK(hipMalloc((void **)&m->loss, sizeof(float)));
        HIP_CHECK(hipMemset(m->params, 0, NPARAM * sizeof(float)));
    }
    return ctx->mlp;
}

static void ensure_rows(Mlp *m, int64_t n) {
    if (n <= m->cap) return;
    float **bufs[] = {&m->x, &m->y, &m->h1, &m->h2, &m->out, &m->dout, &m->dh1, &m->dh2};
    for (float **b : bufs)
        if (*b) hipFree(*b), *b = nullptr;
    if (m->idx) hipFree(m->idx), m->idx = nullptr;
    HIP_CHECK(hipMalloc((void **)&m->x, n * F * sizeof(float)));
    HIP_CHECK(hipMalloc((void **)&m->y, n * sizeof(float)));
    HIP_CHECK(hipMalloc((void **)&m->h1, n * H * sizeof(float)));
    HIP_CHECK(hipMalloc((void **)&m->h2, n * H * sizeof(float)));
    HIP_CHECK(hipMalloc((void **)&m->out, n * sizeof(float)));
    HIP_CHECK(hipMalloc((void **)&m->dout, n * sizeof(float)));
    HIP_CHECK(hipMalloc((void **)&m->dh1, n * H * sizeof(float)));
    HIP_CHECK(hipMalloc((void **)&m->dh2, n * H * sizeof(float)));
    HIP_CHECK(hipMalloc((void **)&m->idx, n * sizeof(int)));
    m->cap = n;
}

static int grid_rows(int64_t rows) { return (int)std::max<int64_t>(1, std::min<int64_t>(rows, 4096)); }

static void forward(Mlp *m, const float *x, const int *idx, int64_t rows, hipStream_t st) {
    hipLaunchKernelGGL(mlp_forward_kernel, dim3(grid_rows(rows)), dim3(H), 0, st, m->params, x, idx, rows, m->h1,
                       m->h2, m->out);
    HIP_CHECK(hipGetLastError());
}

static void backward(Mlp *m, const float *x, const float *y, const int *idx, int64_t rows, hipStream_t st) {
    hipLaunchKernelGGL(mlp_backward_rows_kernel, dim3(grid_rows(rows)), dim3(H), 0, st, m->params, y, idx, rows, m->h1,
                       m->h2, m->out, m->dout, m->dh1, m->dh2);
    hipLaunchKernelGGL(mlp_grad_kernel, dim3((NPARAM + 255) / 256), dim3(256), 0, st, x, idx, rows, m->h1, m->h2,
                       m->dout, m->dh1, m->dh2, m->grads);
    HIP_CHECK(hipGetLastError());
}

static void init_params(Mlp *m, uint64_t seed, hipStream_t st) {
    std::vector<float> p(NPARAM, 0.f);
    std::mt19937_64 rng(seed);
    auto fill = [&](int off, int fan_out, int fan_in) {
        float b = std::sqrt(6.0f / (float)fan_in);   // He-uniform for ReLU layers
        std::uniform_real_distribution<float> u(-b, b);
        for (int i = 0; i < fan_out * fan_in; i++) p[off + i] = u(rng);
    };
    fill(OFF_W1, H, F);
    fill(OFF_W2, H, H);
    fill(OFF_W3, 1, H);
    HIP_CHECK(hipMemcpyAsync(m->params, p.data(), NPARAM * sizeof(float), hipMemcpyHostToDevice, st));
    HIP_CHECK(hipMemsetAsync(m->m, 0, NPARAM * sizeof(float), st));
    HIP_CHECK(hipMemsetAsync(m->v, 0, NPARAM * sizeof(float), st));
    HIP_CHECK(hipStreamSynchronize(st));
    m->step = 0;
}

// Host-side path cost for the search: sum of predicted step times.
// Roofline baseline of a step (log2 microseconds) from its feature row: a
// launch latency of 4 us plus the larger of its algorithmic flops (8 M N K
// per batch entry) at the matrix-core peak of its dtype (FP32 157.3 TFLOP/s
// for complex64, FP16/BF16 2516.6) and its bytes (A, B and C at the storage
// size, 8 or 4 bytes an entry, plus a read and a write of each permuted
// operand) at 8 TB/s.
double step_base_log2_us(const float *f) {
    const double m = f[0], n = f[1], k = f[2], b = f[3];
    const bool c64 = f[6] < 0.5f;
    const double s = c64 ? 8.0 : 4.0, peak = c64 ? 157.3e12 : 2516.6e12;
    const double flops = 8.0 * std::exp2(m + n + k + b);
    double bytes = s * (std::exp2(b + m + k) + std::exp2(b + n + k) + std::exp2(b + m + n));
    if (f[4] > 1.5f) bytes += 2.0 * s * std::exp2(b + m + k);
    if (f[5] > 1.5f) bytes += 2.0 * s * std::exp2(b + n + k);
    return std::log2(4.0 + 1e6 * std::max(flops / peak, bytes / 8e12));
}

double mlp_path_cost(const Network &net, const std::vector<int> &ssa, const std::vector<int> &sliced,
                     const std::vector<int> &open_q) {
    tnc_ctx *ctx = g_cost_ctx;
    if (!ctx || !ctx->mlp || !ctx->mlp->trained) return -1.0;
    // the device path the plan would run: host absorption first, as in tnc_plan_create
    Simplified sp = presimplify(net, (int)ssa.size() / 2, ssa.data(), (int)sliced.size(), sliced.data(),
                                (int)open_q.size(), open_q.data(), host_rank_cap());
    Analysis an = analyze(sp.net, (int)sp.ssa.size() / 2, sp.ssa.data(), (int)sliced.size(), sliced.data(),
                          (int)open_q.size(), open_q.data(), TNC_F16_4M);
    // slices per launch as the plan would hold them: the largest power of two
    // (at most 4096) whose arena fits the context's workspace
    const int64_t total = (int64_t)1 << an.n_sliced;
    const int64_t cap = std::min<int64_t>(total, 4096);
    if ((size_t)plan_memory(an, 1, false) > ctx->ws_bytes) return 1e30;   // does not fit: never chosen
    int64_t S = 1;
    while (S * 2 <= cap && (size_t)plan_memory(an, (int)(S * 2), false) <= ctx->ws_bytes) S *= 2;
    std::vector<float> x;
    std::vector<double> mult;
    for (const auto &s : an.steps) {
        double reps = s.dep ? (double)total / (double)S : 1.0;
        double batch = std::log2((double)s.nb * (s.dep ? (double)S : 1.0));
        float f[F] = {(float)s.m.size(), (float)s.n.size(), (float)s.k.size(), (float)batch,
                      (float)(s.perm_a ? 2 : (s.a_kc ? 0 : 1)), (float)(s.perm_b ? 2 : (s.b_kc ? 0 : 1)), 1.f, 0.f};
        x.insert(x.end(), f, f + F);
        mult.push_back(reps);
    }
    std::vector<float> y(mult.size());
    if (tnc_mlp_predict(ctx, (int64_t)mult.size(), x.data(), y.data()) != TNC_OK) return -1.0;
    double c = 0;
    for (size_t i = 0; i < y.size(); i++) c += mult[i] * std::exp2((double)y[i] + step_base_log2_us(&x[i * F]));
    return c;
}

}  // namespace tnc

using namespace tnc;

template <typename Fn> static int guard(Fn fn) {
    try {
        fn();
    } catch (const Error &e) {
        set_error(e.msg);
        return e.code;
    } catch (const std::exception &e) {
        set_error(e.what());
        return TNC_EINVAL;
    }
    return TNC_OK;
}

extern "C" int64_t tnc_mlp_param_count(void) { return NPARAM; }

extern "C" int tnc_costmodel_base(int64_t n, const float *x, float *log2_us_out) {
    return guard([&] {
        if (n < 0) TNC_THROW(TNC_EINVAL, "n < 0");
        if (n > 0 && (!x || !log2_us_out)) TNC_THROW(TNC_EINVAL, "NULL argument");
        for (int64_t r = 0; r < n; r++) log2_us_out[r] = (float)step_base_log2_us(x + r * F);
    });
}

extern "C" int tnc_mlp_train(tnc_ctx *ctx, int64_t n, const float *x, const float *y, int32_t epochs, int32_t batch,
                             float lr, uint64_t seed, float *loss_out) {
    return guard([&] {
        if (!ctx || !x || !y) TNC_THROW(TNC_EINVAL, "NULL argument");
        if (n < 1 || epochs < 1 || batch < 1) TNC_THROW(TNC_EINVAL, "n, epochs and batch must be positive");
        HIP_CHECK(hipSetDevice(ctx->device));
        hipStream_t st = ctx->stream;
        Mlp *m = mlp_of(ctx);
        ensure_rows(m, n);
        HIP_CHECK(hipMemcpyAsync(m->x, x, n * F * sizeof(float), hipMemcpyHostToDevice, st));
        HIP_CHECK(hipMemcpyAsync(m->y, y, n * sizeof(float), hipMemcpyHostToDevice, st));
        init_params(m, seed, st);
        std::mt19937_64 rng(seed ^ 0x9e3779b97f4a7c15ull);
        std::vector<int> perm(n);
        std::iota(perm.begin(), perm.end(), 0);
        const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
        // minibatch rows are laid out contiguously per epoch: idx[r] = shuffled row
        for (int e = 0; e < epochs; e++) {
            std::shuffle(perm.begin(), perm.end(), rng);
            HIP_CHECK(hipMemcpyAsync(m->idx, perm.data(), n * sizeof(int), hipMemcpyHostToDevice, st));
            HIP_CHECK(hipStreamSynchronize(st));   // perm is reshuffled next epoch
            for (int64_t r0 = 0; r0 < n; r0 += batch) {
                int64_t rows = std::min<int64_t>(batch, n - r0);
                forward(m, m->x, m->idx + r0, rows, st);
                backward(m, m->x, m->y, m->idx + r0, rows, st);
                m->step++;
                float c1 = 1.f - std::pow(b1, (float)m->step), c2 = 1.f - std::pow(b2, (float)m->step);
                hipLaunchKernelGGL(mlp_adam_kernel, dim3((NPARAM + 255) / 256), dim3(256), 0, st, m->params, m->grads,
                                   m->m, m->v, lr, b1, b2, eps, c1, c2);
                HIP_CHECK(hipGetLastError());
            }
        }
        forward(m, m->x, nullptr, n, st);
        hipLaunchKernelGGL(mlp_loss_kernel, dim3(1), dim3(1), 0, st, m->y, (const int *)nullptr, n, m->out, m->loss);
        float l = 0.f;
        HIP_CHECK(hipMemcpyAsync(&l, m->loss, sizeof(float), hipMemcpyDeviceToHost, st));
        HIP_CHECK(hipStreamSynchronize(st));
        if (loss_out) *loss_out = l;
        m->trained = true;
        set_support(m, n, x);
    });
}

extern "C" int tnc_mlp_adam(tnc_ctx *ctx, int64_t n, const float *x, const float *y, int32_t steps, float lr,
                            float *loss_out) {
    return guard([&] {
        if (!ctx || !x || !y) TNC_THROW(TNC_EINVAL, "NULL argument");
        if (n < 1 || steps < 1) TNC_THROW(TNC_EINVAL, "n and steps must be positive");
        HIP_CHECK(hipSetDevice(ctx->device));
        hipStream_t st = ctx->stream;
        Mlp *m = mlp_of(ctx);
        ensure_rows(m, n);
        HIP_CHECK(hipMemcpyAsync(m->x, x, n * F * sizeof(float), hipMemcpyHostToDevice, st));
        HIP_CHECK(hipMemcpyAsync(m->y, y, n * sizeof(float), hipMemcpyHostToDevice, st));
        HIP_CHECK(hipMemsetAsync(m->m, 0, NPARAM * sizeof(float), st));
        HIP_CHECK(hipMemsetAsync(m->v, 0, NPARAM * sizeof(float), st));
        const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
        for (int t = 1; t <= steps; t++) {
            forward(m, m->x, nullptr, n, st);
            backward(m, m->x, m->y, nullptr, n, st);
            const float c1 = 1.f - std::pow(b1, (float)t), c2 = 1.f - std::pow(b2, (float)t);
            hipLaunchKernelGGL(mlp_adam_kernel, dim3((NPARAM + 255) / 256), dim3(256), 0, st, m->params, m->grads,
                               m->m, m->v, lr, b1, b2, eps, c1, c2);
            HIP_CHECK(hipGetLastError());
        }
        forward(m, m->x, nullptr, n, st);
        hipLaunchKernelGGL(mlp_loss_kernel, dim3(1), dim3(1), 0, st, m->y, (const int *)nullptr, n, m->out, m->loss);
        float l = 0.f;
        HIP_CHECK(hipMemcpyAsync(&l, m->loss, sizeof(float), hipMemcpyDeviceToHost, st));
        HIP_CHECK(hipStreamSynchronize(st));
        if (loss_out) *loss_out = l;
        m->step = steps;
        m->trained = true;
        set_support(m, n, x);
    });
}

extern "C" int tnc_mlp_predict(tnc_ctx *ctx, int64_t n, const float *x, float *y_out) {
    return guard([&] {
        if (!ctx || !x || !y_out) TNC_THROW(TNC_EINVAL, "NULL argument");
        if (n < 0) TNC_THROW(TNC_EINVAL, "n < 0");
        if (n == 0) return;
        HIP_CHECK(hipSetDevice(ctx->device));
        hipStream_t st = ctx->stream;
        Mlp *m = mlp_of(ctx);
        ensure_rows(m, n);
        // Outside the trained size range the network is not asked to
        // extrapolate: a size feature is clamped to the range, so the learned
        // ratio to the roofline baseline is held at its edge value there.
        std::vector<float> xc;
        const float *xs = x;
        if (m->support) {
            xc.assign(x, x + n * F);
            for (int64_t r = 0; r < n; r++)
                for (int f = 0; f < 4; f++) {
                    float &v = xc[r * F + f];
                    v = std::min(std::max(v, m->lo[f]), m->hi[f]);
                }
            xs = xc.data();
        }
        HIP_CHECK(hipMemcpyAsync(m->x, xs, n * F * sizeof(float), hipMemcpyHostToDevice, st));
        forward(m, m->x, nullptr, n, st);
        HIP_CHECK(hipMemcpyAsync(y_out, m->out, n * sizeof(float), hipMemcpyDeviceToHost, st));
        HIP_CHECK(hipStreamSynchronize(st));
    });
}

extern "C" int tnc_mlp_grad(tnc_ctx *ctx, int64_t n, const float *x, const float *y, float *loss_out,
                            float *grads_out) {
    return guard([&] {
        if (!ctx || !x || !y) TNC_THROW(TNC_EINVAL, "NULL argument");
        if (n < 1) TNC_THROW(TNC_EINVAL, "n < 1");
        HIP_CHECK(hipSetDevice(ctx->device));
        hipStream_t st = ctx->stream;
        Mlp *m = mlp_of(ctx);
        ensure_rows(m, n);
        HIP_CHECK(hipMemcpyAsync(m->x, x, n * F * sizeof(float), hipMemcpyHostToDevice, st));
        HIP_CHECK(hipMemcpyAsync(m->y, y, n * sizeof(float), hipMemcpyHostToDevice, st));
        forward(m, m->x, nullptr, n, st);
        backward(m, m->x, m->y, nullptr, n, st);
        hipLaunchKernelGGL(mlp_loss_kernel, dim3(1), dim3(1), 0, st, m->y, (const int *)nullptr, n, m->out, m->loss);
        float l = 0.f;
        HIP_CHECK(hipMemcpyAsync(&l, m->loss, sizeof(float), hipMemcpyDeviceToHost, st));
        if (grads_out) HIP_CHECK(hipMemcpyAsync(grads_out, m->grads, NPARAM * sizeof(float), hipMemcpyDeviceToHost, st));
        HIP_CHECK(hipStreamSynchronize(st));
        if (loss_out) *loss_out = l;
    });
}

extern "C" int tnc_mlp_get_params(tnc_ctx *ctx, float *params_out) {
    return guard([&] {
        if (!ctx || !params_out) TNC_THROW(TNC_EINVAL, "NULL argument");
        HIP_CHECK(hipSetDevice(ctx->device));
        Mlp *m = mlp_of(ctx);
        HIP_CHECK(hipMemcpyAsync(params_out, m->params, NPARAM * sizeof(float), hipMemcpyDeviceToHost, ctx->stream));
        HIP_CHECK(hipStreamSynchronize(ctx->stream));
    });
}

extern "C" int tnc_mlp_set_params(tnc_ctx *ctx, const float *params) {
    return guard([&] {
        if (!ctx || !params) TNC_THROW(TNC_EINVAL, "NULL argument");
        HIP_CHECK(hipSetDevice(ctx->device));
        Mlp *m = mlp_of(ctx);
        HIP_CHECK(hipMemcpyAsync(m->params, params, NPARAM * sizeof(float), hipMemcpyHostToDevice, ctx->stream));
        HIP_CHECK(hipStreamSynchronize(ctx->stream));
        m->trained = true;
        m->support = false;   // weights from elsewhere: no known training range
    });
}

extern "C" int tnc_costmodel_use(tnc_ctx *ctx) {
    return guard([&] {
        if (ctx && (!ctx->mlp || !ctx->mlp->trained)) TNC_THROW(TNC_EINVAL, "the context has no trained model");
        g_cost_ctx = ctx;
    });
}
