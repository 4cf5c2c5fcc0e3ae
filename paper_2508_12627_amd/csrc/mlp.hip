// MLP cost model on the GPU: forward, mean-squared-error loss, backward and
// Adam, for the network F -> H1 -> H2 -> 1 with ReLU hidden layers.  The
// model maps features of a lowered elimination order to a log run time; it
// is trained on timings the engine itself measures and ranks candidate
// orders at plan time (costmodel.cpp holds the host inference used there).
//
// Parameters are one flat fp32 array, in this order:
//   mean[F] inv_std[F] W1[H1*F] b1[H1] W2[H2*H1] b2[H2] W3[H2] b3[1]
// (W row-major, output unit by input unit).  mean/inv_std standardise the
// inputs and are not trained.  Weight gradients are sums over samples taken
// in a fixed order (per-block strided sums, then a fixed LDS tree), so
// gradients and training runs are bitwise reproducible.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/ustat.h"
#include "costmodel.hpp"
#include "guard.hpp"

namespace ustat {
namespace {

struct Layout {
    int F, H1, H2;
    size_t mean, istd, W1, b1, W2, b2, W3, b3, total, first_trained;
    Layout(int f, int h1, int h2) : F(f), H1(h1), H2(h2) {
        size_t o = 0;
        mean = o; o += F;
        istd = o; o += F;
        W1 = o; o += (size_t)H1 * F;
        b1 = o; o += H1;
        W2 = o; o += (size_t)H2 * H1;
        b2 = o; o += H2;
        W3 = o; o += H2;
        b3 = o; o += 1;
        total = o;
        first_trained = W1;
    }
};

// One layer: out[i][j] = act(sum_k in[i][k] W[j][k] + b[j]), pre-activation
// kept for the backward pass.  Thread per (sample, unit).
__global__ void k_dense(const float *__restrict__ in, int K, const float *__restrict__ W,
                        const float *__restrict__ b, int J, int64_t N, float *__restrict__ pre,
                        float *__restrict__ out, int relu) {
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= N * J) return;
    int64_t i = idx / J;
    int j = (int)(idx % J);
    const float *x = in + i * K;
    const float *w = W + (size_t)j * K;
    float s = b[j];
    for (int k = 0; k < K; ++k) s = fmaf(x[k], w[k], s);
    if (pre) pre[idx] = s;
    out[idx] = relu ? (s > 0.f ? s : 0.f) : s;
}

// Standardised inputs: xn[i][f] = (x[i][f] - mean[f]) * inv_std[f].
__global__ void k_standardise(const float *__restrict__ x, const float *__restrict__ mean,
                              const float *__restrict__ istd, int F, int64_t N, float *__restrict__ xn) {
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= N * F) return;
    int f = (int)(idx % F);
    xn[idx] = (x[idx] - mean[f]) * istd[f];
}

// g[i] = 2 (yhat[i] - y[i]) / N and per-block partial sums of the squared
// residual (fixed order inside the block).
__global__ void k_residual(const float *__restrict__ yhat, const float *__restrict__ y, int64_t N,
                           float *__restrict__ g, double *__restrict__ part) {
    __shared__ double red[256];
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double r2 = 0;
    if (i < N) {
        float r = yhat[i] - y[i];
        g[i] = 2.f * r / (float)N;
        r2 = (double)r * r;
    }
    red[threadIdx.x] = r2;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < (unsigned)s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// Back through a layer: gin[i][k] = (sum_j gout[i][j] W[j][k]) * relu'(pre_in[i][k]).
__global__ void k_back_input(const float *__restrict__ gout, int J, const float *__restrict__ W, int K,
                             int64_t N, const float *__restrict__ pre_in, float *__restrict__ gin) {
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= N * K) return;
    int64_t i = idx / K;
    int k = (int)(idx % K);
    const float *go = gout + i * J;
    float s = 0.f;
    for (int j = 0; j < J; ++j) s = fmaf(go[j], W[(size_t)j * K + k], s);
    gin[idx] = pre_in[idx] > 0.f ? s : 0.f;
}

// Weight gradient: dW[j][k] = sum_i gout[i][j] in[i][k] and db[j] =
// sum_i gout[i][j]; one block per (j, k) entry (k == K is the bias), the
// 256 threads take samples i = t, t+256, ... and meet in a fixed tree.
__global__ void k_weight_grad(const float *__restrict__ gout, int J, const float *__restrict__ in,
                              int K, int64_t N, float *__restrict__ dW, float *__restrict__ db) {
    __shared__ double red[256];
    const int j = blockIdx.x / (K + 1), k = blockIdx.x % (K + 1);
    double s = 0;
    for (int64_t i = threadIdx.x; i < N; i += 256) {
        double a = (k < K) ? (double)in[i * K + k] : 1.0;
        s += (double)gout[i * J + j] * a;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < (unsigned)st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (k < K) dW[(size_t)j * K + k] = (float)red[0];
        else db[j] = (float)red[0];
    }
}

// Adam (Kingma & Ba) on params[first .. total), step t >= 1.
__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, size_t first, size_t total, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
    size_t i = first + (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    float gi = g[i];
    float mi = b1 * m[i] + (1.f - b1) * gi;
    float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

struct Dev {
    float *x = nullptr, *xn = nullptr, *y = nullptr, *params = nullptr, *grad = nullptr;
    float *m = nullptr, *v = nullptr, *pre1 = nullptr, *a1 = nullptr, *pre2 = nullptr, *a2 = nullptr;
    float *yhat = nullptr, *g3 = nullptr, *g2 = nullptr, *g1 = nullptr;
    double *part = nullptr;
    ~Dev() {
        float *fs[] = {x, xn, y, params, grad, m, v, pre1, a1, pre2, a2, yhat, g3, g2, g1};
        for (float *f : fs)
            if (f) (void)hipFree(f);
        if (part) (void)hipFree(part);
    }
};

#define MLPCHK(x)                                      \
    do {                                               \
        hipError_t e_ = (x);                           \
        if (e_ != hipSuccess) return hipGetErrorString(e_); \
    } while (0)

template <class T>
hipError_t dalloc(T **p, size_t n) {
    return hipMalloc((void **)p, std::max<size_t>(n, 1) * sizeof(T));
}

const char *setup(Dev &D, const Layout &L, const float *X, const float *y, int64_t N,
                  const float *params) {
    MLPCHK(dalloc(&D.x, (size_t)N * L.F));
    MLPCHK(dalloc(&D.xn, (size_t)N * L.F));
    MLPCHK(dalloc(&D.y, (size_t)N));
    MLPCHK(dalloc(&D.params, L.total));
    MLPCHK(dalloc(&D.grad, L.total));
    MLPCHK(dalloc(&D.m, L.total));
    MLPCHK(dalloc(&D.v, L.total));
    MLPCHK(dalloc(&D.pre1, (size_t)N * L.H1));
    MLPCHK(dalloc(&D.a1, (size_t)N * L.H1));
    MLPCHK(dalloc(&D.pre2, (size_t)N * L.H2));
    MLPCHK(dalloc(&D.a2, (size_t)N * L.H2));
    MLPCHK(dalloc(&D.yhat, (size_t)N));
    MLPCHK(dalloc(&D.g3, (size_t)N));
    MLPCHK(dalloc(&D.g2, (size_t)N * L.H2));
    MLPCHK(dalloc(&D.g1, (size_t)N * L.H1));
    MLPCHK(dalloc(&D.part, (size_t)(N + 255) / 256 + 1));
    MLPCHK(hipMemcpy(D.x, X, sizeof(float) * N * L.F, hipMemcpyHostToDevice));
    if (y) MLPCHK(hipMemcpy(D.y, y, sizeof(float) * N, hipMemcpyHostToDevice));
    MLPCHK(hipMemcpy(D.params, params, sizeof(float) * L.total, hipMemcpyHostToDevice));
    MLPCHK(hipMemset(D.m, 0, sizeof(float) * L.total));
    MLPCHK(hipMemset(D.v, 0, sizeof(float) * L.total));
    MLPCHK(hipMemset(D.grad, 0, sizeof(float) * L.total));
    return nullptr;
}

inline unsigned blocks(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

const char *forward(Dev &D, const Layout &L, int64_t N) {
    const float *P = D.params;
    hipLaunchKernelGGL(k_standardise, dim3(blocks(N * L.F)), dim3(256), 0, 0, D.x, P + L.mean,
                       P + L.istd, L.F, N, D.xn);
    hipLaunchKernelGGL(k_dense, dim3(blocks(N * L.H1)), dim3(256), 0, 0, D.xn, L.F, P + L.W1,
                       P + L.b1, L.H1, N, D.pre1, D.a1, 1);
    hipLaunchKernelGGL(k_dense, dim3(blocks(N * L.H2)), dim3(256), 0, 0, D.a1, L.H1, P + L.W2,
                       P + L.b2, L.H2, N, D.pre2, D.a2, 1);
    hipLaunchKernelGGL(k_dense, dim3(blocks(N)), dim3(256), 0, 0, D.a2, L.H2, P + L.W3, P + L.b3, 1,
                       N, (float *)nullptr, D.yhat, 0);
    MLPCHK(hipGetLastError());
    return nullptr;
}

// loss (mean squared residual) and the full parameter gradient in D.grad
const char *backward(Dev &D, const Layout &L, int64_t N, double *loss) {
    const float *P = D.params;
    const unsigned nb = blocks(N);
    hipLaunchKernelGGL(k_residual, dim3(nb), dim3(256), 0, 0, D.yhat, D.y, N, D.g3, D.part);
    // output layer
    hipLaunchKernelGGL(k_weight_grad, dim3(1 * (L.H2 + 1)), dim3(256), 0, 0, D.g3, 1, D.a2, L.H2, N,
                       D.grad + L.W3, D.grad + L.b3);
    hipLaunchKernelGGL(k_back_input, dim3(blocks(N * L.H2)), dim3(256), 0, 0, D.g3, 1, P + L.W3, L.H2,
                       N, D.pre2, D.g2);
    // second layer
    hipLaunchKernelGGL(k_weight_grad, dim3(L.H2 * (L.H1 + 1)), dim3(256), 0, 0, D.g2, L.H2, D.a1,
                       L.H1, N, D.grad + L.W2, D.grad + L.b2);
    hipLaunchKernelGGL(k_back_input, dim3(blocks(N * L.H1)), dim3(256), 0, 0, D.g2, L.H2, P + L.W2,
                       L.H1, N, D.pre1, D.g1);
    // first layer
    hipLaunchKernelGGL(k_weight_grad, dim3(L.H1 * (L.F + 1)), dim3(256), 0, 0, D.g1, L.H1, D.xn, L.F,
                       N, D.grad + L.W1, D.grad + L.b1);
    MLPCHK(hipGetLastError());
    if (loss) {
        std::vector<double> part(nb);
        MLPCHK(hipMemcpy(part.data(), D.part, sizeof(double) * nb, hipMemcpyDeviceToHost));
        double s = 0;
        for (double q : part) s += q;
        *loss = s / (double)N;
    }
    return nullptr;
}

ustat_status mlp_fail(const char *msg) {
    set_last_error(msg ? msg : "unknown");
    return USTAT_E_HIP;
}

bool bad_sizes(int32_t F, int32_t H1, int32_t H2, int64_t N) {
    return F < 1 || F > 256 || H1 < 1 || H1 > 1024 || H2 < 1 || H2 > 1024 || N < 1 || N > (1ll << 26);
}

}  // namespace
}  // namespace ustat

using namespace ustat;

extern "C" {

size_t ustat_mlp_num_params(int32_t F, int32_t H1, int32_t H2) {
    if (F < 1 || H1 < 1 || H2 < 1) return 0;
    return Layout(F, H1, H2).total;
}

ustat_status ustat_mlp_predict(int32_t F, int32_t H1, int32_t H2, const float *params,
                               const float *X, int64_t N, float *out) {
    USTAT_GUARD_BEGIN
    if (bad_sizes(F, H1, H2, N) || !params || !X || !out) {
        set_last_error("bad MLP arguments");
        return USTAT_E_INVALID;
    }
    Layout L(F, H1, H2);
    Dev D;
    if (const char *e = setup(D, L, X, nullptr, N, params)) return mlp_fail(e);
    if (const char *e = forward(D, L, N)) return mlp_fail(e);
    if (hipMemcpy(out, D.yhat, sizeof(float) * N, hipMemcpyDeviceToHost) != hipSuccess)
        return mlp_fail("copy failed");
    return USTAT_OK;
    USTAT_GUARD_END
}

ustat_status ustat_mlp_loss_grad(int32_t F, int32_t H1, int32_t H2, const float *params,
                                 const float *X, const float *y, int64_t N, double *loss,
                                 float *grad) {
    USTAT_GUARD_BEGIN
    if (bad_sizes(F, H1, H2, N) || !params || !X || !y || !loss || !grad) {
        set_last_error("bad MLP arguments");
        return USTAT_E_INVALID;
    }
    Layout L(F, H1, H2);
    Dev D;
    if (const char *e = setup(D, L, X, y, N, params)) return mlp_fail(e);
    if (const char *e = forward(D, L, N)) return mlp_fail(e);
    if (const char *e = backward(D, L, N, loss)) return mlp_fail(e);
    if (hipMemcpy(grad, D.grad, sizeof(float) * L.total, hipMemcpyDeviceToHost) != hipSuccess)
        return mlp_fail("copy failed");
    return USTAT_OK;
    USTAT_GUARD_END
}

ustat_status ustat_mlp_train(int32_t F, int32_t H1, int32_t H2, float *params, const float *X,
                             const float *y, int64_t N, int32_t steps, float lr, double *losses) {
    USTAT_GUARD_BEGIN
    if (bad_sizes(F, H1, H2, N) || !params || !X || !y || steps < 1 || !(lr > 0)) {
        set_last_error("bad MLP arguments");
        return USTAT_E_INVALID;
    }
    Layout L(F, H1, H2);
    Dev D;
    if (const char *e = setup(D, L, X, y, N, params)) return mlp_fail(e);
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    double c1 = 1, c2 = 1;
    const size_t ntr = L.total - L.first_trained;
    for (int t = 1; t <= steps; ++t) {
        double loss = 0;
        if (const char *e = forward(D, L, N)) return mlp_fail(e);
        if (const char *e = backward(D, L, N, losses ? &loss : nullptr)) return mlp_fail(e);
        if (losses) losses[t - 1] = loss;
        c1 *= b1;
        c2 *= b2;
        hipLaunchKernelGGL(k_adam, dim3(blocks((int64_t)ntr)), dim3(256), 0, 0, D.params, D.grad,
                           D.m, D.v, L.first_trained, L.total, lr, b1, b2, eps, (float)(1 - c1),
                           (float)(1 - c2));
        if (hipGetLastError() != hipSuccess) return mlp_fail("adam launch failed");
    }
    if (hipMemcpy(params, D.params, sizeof(float) * L.total, hipMemcpyDeviceToHost) != hipSuccess)
        return mlp_fail("copy failed");
    return USTAT_OK;
    USTAT_GUARD_END
}

ustat_status ustat_mlp_save(const char *path, int32_t F, int32_t H1, int32_t H2, const float *params) {
    USTAT_GUARD_BEGIN
    if (!path || !params || F < 1 || H1 < 1 || H2 < 1) return USTAT_E_INVALID;
    Layout L(F, H1, H2);
    MLPWeights w;
    w.F = F;
    w.H1 = H1;
    w.H2 = H2;
    auto take = [&](size_t off, size_t n) { return std::vector<float>(params + off, params + off + n); };
    w.mean = take(L.mean, F);
    w.inv_std = take(L.istd, F);
    w.W1 = take(L.W1, (size_t)H1 * F);
    w.b1 = take(L.b1, H1);
    w.W2 = take(L.W2, (size_t)H2 * H1);
    w.b2 = take(L.b2, H2);
    w.W3 = take(L.W3, H2);
    w.b3 = take(L.b3, 1);
    std::string err = save_mlp(path, w);
    if (!err.empty()) {
        set_last_error(err);
        return USTAT_E_INVALID;
    }
    return USTAT_OK;
    USTAT_GUARD_END
}

}  // extern "C"
