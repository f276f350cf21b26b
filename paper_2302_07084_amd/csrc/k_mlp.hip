// Surrogate network and downstream scorer for the hyperparameter search
// (section 4.4: the search over s_r, M, q, k, theta, mu is scored by the
// downstream task; here a small MLP learns that score and proposes trials, and
// the plain method scores every proposal).
//
// MLP: in -> hidden -> hidden -> 1, GELU, FP32, mean squared error, Adam.
// Parameters are one flat array: W1 (in x h), b1 (h), W2 (h x h), b2 (h),
// W3 (h), b3 (1).  Every reduction is a fixed-order loop in one thread, so
// results do not depend on scheduling.
//
// Scorer: one-vs-rest L2-regularised logistic regression on the embedding
// (standardised features, full-batch Adam), then each test vertex predicts its
// top-k labels with k its true label count; micro-F1 over the test set.
#include <cmath>
#include <cstring>

#include "common.hpp"
#include "philox.hpp"

namespace lne {

namespace {

constexpr uint32_t kTagInit = 4u << 24;

__device__ __forceinline__ float gelu(float z) {
    return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f));
}
__device__ __forceinline__ float gelu_d(float z) {
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) +
           z * 0.39894228040143268f * expf(-0.5f * z * z);
}

// Z = X W + b; A = gelu(Z) when A is given.  X: B x I, W: I x O.
__global__ void k_lin_fwd(const float *__restrict__ X, int I, const float *__restrict__ W,
                          const float *__restrict__ bias, int O, int64_t B,
                          float *__restrict__ Z, float *__restrict__ A) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= B * O) return;
    const int64_t b = t / O;
    const int o = (int)(t - b * O);
    float s = bias ? bias[o] : 0.0f;
    const float *x = X + b * I;
    for (int i = 0; i < I; ++i) s += x[i] * W[(int64_t)i * O + o];
    if (Z) Z[t] = s;
    if (A) A[t] = gelu(s);
}

// dW[i][o] = sum_b X[b][i] G[b][o] (+ l2 W[i][o]); db[o] = sum_b G[b][o].
__global__ void k_lin_wgrad(const float *__restrict__ X, int I, const float *__restrict__ G,
                            int O, int64_t B, const float *__restrict__ W, float l2,
                            float *__restrict__ dW, float *__restrict__ db) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < (int64_t)I * O) {
        const int i = (int)(t / O), o = (int)(t % O);
        float s = 0.0f;
        for (int64_t b = 0; b < B; ++b) s += X[b * I + i] * G[b * O + o];
        if (W) s += l2 * W[t];
        dW[t] = s;
    } else if (db && t < (int64_t)I * O + O) {
        const int o = (int)(t - (int64_t)I * O);
        float s = 0.0f;
        for (int64_t b = 0; b < B; ++b) s += G[b * O + o];
        db[o] = s;
    }
}

// dZ[b][i] = (sum_o G[b][o] W[i][o]) * gelu'(Zp[b][i]).
__global__ void k_lin_dgrad(const float *__restrict__ G, int O, const float *__restrict__ W, int I,
                            int64_t B, const float *__restrict__ Zp, float *__restrict__ dZ) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= B * I) return;
    const int64_t b = t / I;
    const int i = (int)(t - b * I);
    float s = 0.0f;
    for (int o = 0; o < O; ++o) s += G[b * O + o] * W[(int64_t)i * O + o];
    dZ[t] = Zp ? s * gelu_d(Zp[t]) : s;
}

// dy = 2 (y - t) / B and loss = mean (y - t)^2, one block, fixed order.
__global__ void k_mse(const float *__restrict__ y, const float *__restrict__ tgt, int64_t B,
                      float *__restrict__ dy, float *__restrict__ loss) {
    __shared__ float part[256];
    float s = 0.0f;
    for (int64_t b = threadIdx.x; b < B; b += 256) {
        const float e = y[b] - tgt[b];
        dy[b] = 2.0f * e / (float)B;
        s += e * e;
    }
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        float t = 0.0f;
        for (int i = 0; i < 256; ++i) t += part[i];
        if (loss) *loss = t / (float)B;
    }
}

__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, int64_t n, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Glorot-uniform weights from Philox words, zero biases.
__global__ void k_mlp_init(float *__restrict__ p, int in, int h, uint64_t seed) {
    const int64_t total = (int64_t)in * h + h + (int64_t)h * h + h + h + 1;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const int64_t o1 = (int64_t)in * h, o2 = o1 + h, o3 = o2 + (int64_t)h * h, o4 = o3 + h,
                  o5 = o4 + h;
    float a = 0.0f;
    if (i < o1) a = sqrtf(6.0f / (float)(in + h));
    else if (i >= o2 && i < o3) a = sqrtf(6.0f / (float)(2 * h));
    else if (i >= o4 && i < o5) a = sqrtf(6.0f / (float)(h + 1));
    if (a == 0.0f) { p[i] = 0.0f; return; }
    const uint4 z = philox4x32_10(make_uint4((uint32_t)i, (uint32_t)((uint64_t)i >> 32), 0, kTagInit),
                                  (uint32_t)seed, (uint32_t)(seed >> 32));
    const float u = ((float)(z.x >> 8) + 0.5f) * (1.0f / 16777216.0f);
    p[i] = a * (2.0f * u - 1.0f);
}

// ---- scorer ----------------------------------------------------------------
// Rows idx of X into Xs (n_sel x d) and labels into Ys (n_sel x L, 0/1).
// An index outside [0, n) is counted in *bad and its row left zero.
__global__ void k_gather_rows(const float *__restrict__ X, int64_t n, int d,
                             const uint8_t *__restrict__ lab, int L,
                             const int32_t *__restrict__ idx, int64_t n_sel,
                             float *__restrict__ Xs, float *__restrict__ Ys,
                             unsigned long long *__restrict__ bad) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_sel * (d + L)) return;
    const int64_t r = t / (d + L);
    const int c = (int)(t - r * (d + L));
    const int64_t src = idx[r];
    if (src < 0 || src >= n) {
        if (c == 0) atomicAdd(bad, 1ull);
        if (c < d) Xs[r * d + c] = 0.0f;
        else Ys[r * L + (c - d)] = 0.0f;
        return;
    }
    if (c < d) Xs[r * d + c] = X[src * d + c];
    else Ys[r * L + (c - d)] = (float)lab[src * L + (c - d)];
}

// Column mean and inverse standard deviation over the training rows.
__global__ void k_col_stats(const float *__restrict__ X, int64_t n, int d, float *__restrict__ mu,
                            float *__restrict__ isd) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= d) return;
    double s = 0.0, q = 0.0;
    for (int64_t r = 0; r < n; ++r) {
        const double x = X[r * d + c];
        s += x;
        q += x * x;
    }
    const double m = s / (double)n;
    const double var = q / (double)n - m * m;
    mu[c] = (float)m;
    isd[c] = var > 1e-30 ? (float)(1.0 / sqrt(var)) : 0.0f;
}

__global__ void k_standardize(float *__restrict__ X, int64_t n, int d, const float *__restrict__ mu,
                              const float *__restrict__ isd) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * d) return;
    const int c = (int)(t % d);
    X[t] = (X[t] - mu[c]) * isd[c];
}

// Gradient of the mean logistic loss: G = (sigmoid(Z) - Y) / n.
__global__ void k_bce_grad(const float *__restrict__ Z, const float *__restrict__ Y, int64_t cnt,
                           float inv_n, float *__restrict__ G) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= cnt) return;
    G[t] = (1.0f / (1.0f + expf(-Z[t])) - Y[t]) * inv_n;
}

// Per test row: predict the top-k labels (k = true label count, ties by
// label index) and accumulate true positives and the label count.
__global__ void k_topk_f1(const float *__restrict__ Z, const float *__restrict__ Y, int64_t n,
                          int L, unsigned long long *__restrict__ counts) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const float *z = Z + r * L;
    const float *y = Y + r * L;
    int k = 0;
    for (int l = 0; l < L; ++l) k += y[l] > 0.5f ? 1 : 0;
    int tp = 0;
    for (int l = 0; l < L; ++l) {
        int rank = 0;
        for (int j = 0; j < L; ++j) rank += (z[j] > z[l] || (z[j] == z[l] && j < l)) ? 1 : 0;
        if (rank < k && y[l] > 0.5f) ++tp;
    }
    atomicAdd(&counts[0], (unsigned long long)tp);
    atomicAdd(&counts[1], (unsigned long long)k);
}

struct MlpLayout {
    int64_t W1, b1, W2, b2, W3, b3, total;
    MlpLayout(int in, int h) {
        W1 = 0;
        b1 = (int64_t)in * h;
        W2 = b1 + h;
        b2 = W2 + (int64_t)h * h;
        W3 = b2 + h;
        b3 = W3 + h;
        total = b3 + 1;
    }
};

lne_status mlp_validate(lne_ctx *ctx, int in, int h, int64_t B) {
    if (in < 1 || in > 4096 || h < 1 || h > 4096 || B < 1)
        return fail(ctx, LNE_EINVAL, "mlp: dimensions in=%d hidden=%d batch=%lld", in, h, (long long)B);
    return LNE_OK;
}

// Forward pass keeping the pre-activations: Z1, A1, Z2, A2 (B x h each), y.
lne_status mlp_fwd(lne_ctx *ctx, int in, int h, const float *P, const float *X, int64_t B,
                   float *Z1, float *A1, float *Z2, float *A2, float *y) {
    const MlpLayout L(in, h);
    {
        Launch Lc(ctx, "mlp_forward");
        k_lin_fwd<<<grid_of(B * h, 256), 256, 0, ctx->stream>>>(X, in, P + L.W1, P + L.b1, h, B,
                                                                Z1, A1);
        k_lin_fwd<<<grid_of(B * h, 256), 256, 0, ctx->stream>>>(A1, h, P + L.W2, P + L.b2, h, B,
                                                                Z2, A2);
        k_lin_fwd<<<grid_of(B, 256), 256, 0, ctx->stream>>>(A2, h, P + L.W3, P + L.b3, 1, B, y,
                                                            nullptr);
    }
    return check_launch(ctx, "mlp_forward");
}

}  // namespace

}  // namespace lne

using namespace lne;

extern "C" {

int64_t lne_mlp_param_count(int32_t in_dim, int32_t hidden) {
    if (in_dim < 1 || hidden < 1) return 0;
    return MlpLayout(in_dim, hidden).total;
}

lne_status lne_mlp_init(lne_ctx *ctx, int32_t in_dim, int32_t hidden, uint64_t seed,
                        float *params) {
    if (!ctx) return LNE_EINVAL;
    LNE_TRY(mlp_validate(ctx, in_dim, hidden, 1));
    if (!params) return fail(ctx, LNE_EINVAL, "mlp_init: params is NULL");
    const int64_t n = MlpLayout(in_dim, hidden).total;
    {
        Launch L(ctx, "mlp_init");
        k_mlp_init<<<grid_of(n, 256), 256, 0, ctx->stream>>>(params, in_dim, hidden, seed);
    }
    return check_launch(ctx, "mlp_init");
}

lne_status lne_mlp_forward(lne_ctx *ctx, int32_t in_dim, int32_t hidden, const float *params,
                           const float *X, int64_t batch, float *y) {
    if (!ctx) return LNE_EINVAL;
    LNE_TRY(mlp_validate(ctx, in_dim, hidden, batch));
    if (!params || !X || !y) return fail(ctx, LNE_EINVAL, "mlp_forward: NULL argument");
    Buf act(ctx);
    LNE_TRY(alloc(ctx, act, sizeof(float) * (size_t)(2 * batch * hidden)));
    float *A1 = act.as<float>(), *A2 = A1 + batch * hidden;
    return mlp_fwd(ctx, in_dim, hidden, params, X, batch, nullptr, A1, nullptr, A2, y);
}

lne_status lne_mlp_grad(lne_ctx *ctx, int32_t in_dim, int32_t hidden, const float *params,
                        const float *X, const float *target, int64_t batch, float *grad,
                        float *loss) {
    if (!ctx) return LNE_EINVAL;
    LNE_TRY(mlp_validate(ctx, in_dim, hidden, batch));
    if (!params || !X || !target || !grad) return fail(ctx, LNE_EINVAL, "mlp_grad: NULL argument");
    const MlpLayout Ly(in_dim, hidden);
    const int64_t Bh = batch * hidden;
    Buf ws(ctx);
    LNE_TRY(alloc(ctx, ws, sizeof(float) * (size_t)(6 * Bh + 2 * batch)));
    float *Z1 = ws.as<float>(), *A1 = Z1 + Bh, *Z2 = A1 + Bh, *A2 = Z2 + Bh;
    float *dZ2 = A2 + Bh, *dZ1 = dZ2 + Bh, *y = dZ1 + Bh, *dy = y + batch;
    LNE_TRY(mlp_fwd(ctx, in_dim, hidden, params, X, batch, Z1, A1, Z2, A2, y));
    {
        Launch L(ctx, "mlp_backward");
        k_mse<<<1, 256, 0, ctx->stream>>>(y, target, batch, dy, loss);
        // output layer
        k_lin_wgrad<<<grid_of(hidden + 1, 256), 256, 0, ctx->stream>>>(
            A2, hidden, dy, 1, batch, nullptr, 0.0f, grad + Ly.W3, grad + Ly.b3);
        k_lin_dgrad<<<grid_of(Bh, 256), 256, 0, ctx->stream>>>(dy, 1, params + Ly.W3, hidden,
                                                               batch, Z2, dZ2);
        // second hidden layer
        k_lin_wgrad<<<grid_of((int64_t)hidden * hidden + hidden, 256), 256, 0, ctx->stream>>>(
            A1, hidden, dZ2, hidden, batch, nullptr, 0.0f, grad + Ly.W2, grad + Ly.b2);
        k_lin_dgrad<<<grid_of(Bh, 256), 256, 0, ctx->stream>>>(dZ2, hidden, params + Ly.W2,
                                                               hidden, batch, Z1, dZ1);
        // first layer
        k_lin_wgrad<<<grid_of((int64_t)in_dim * hidden + hidden, 256), 256, 0, ctx->stream>>>(
            X, in_dim, dZ1, hidden, batch, nullptr, 0.0f, grad + Ly.W1, grad + Ly.b1);
    }
    return check_launch(ctx, "mlp_backward");
}

lne_status lne_mlp_adam(lne_ctx *ctx, int64_t count, float *params, const float *grad, float *m,
                        float *v, int64_t step, float lr, float beta1, float beta2, float eps) {
    if (!ctx) return LNE_EINVAL;
    if (count < 1 || step < 1 || !params || !grad || !m || !v)
        return fail(ctx, LNE_EINVAL, "mlp_adam: bad arguments");
    const float c1 = 1.0f - powf(beta1, (float)step);
    const float c2 = 1.0f - powf(beta2, (float)step);
    {
        Launch L(ctx, "mlp_adam");
        k_adam<<<grid_of(count, 256), 256, 0, ctx->stream>>>(params, grad, m, v, count, lr, beta1,
                                                             beta2, eps, c1, c2);
    }
    return check_launch(ctx, "mlp_adam");
}

lne_status lne_score_micro_f1(lne_ctx *ctx, const float *X, int64_t n, int32_t d,
                              const uint8_t *labels, int32_t n_labels, const int32_t *train,
                              int64_t n_train, const int32_t *test, int64_t n_test,
                              int32_t epochs, float lr, float l2, double *f1) {
    if (!ctx) return LNE_EINVAL;
    if (!X || !labels || !train || !test || !f1 || n < 1 || d < 1 || n_labels < 1 ||
        n_labels > 1024 || n_train < 1 || n_test < 1 || epochs < 1)
        return fail(ctx, LNE_EINVAL, "score_micro_f1: bad arguments");
    const int L = n_labels;
    Buf ws(ctx), cnt(ctx);
    const int64_t wsz = n_train * (d + L) + n_test * (d + L) + 2 * d + 4 * ((int64_t)d * L + L) +
                        2 * n_train * L + n_test * L;
    LNE_TRY(alloc(ctx, ws, sizeof(float) * (size_t)wsz));
    LNE_TRY(alloc(ctx, cnt, 3 * sizeof(unsigned long long)));
    float *Xtr = ws.as<float>(), *Ytr = Xtr + n_train * d, *Xte = Ytr + n_train * L,
          *Yte = Xte + n_test * d, *mu = Yte + n_test * L, *isd = mu + d, *W = isd + d,
          *b = W + (int64_t)d * L, *gW = b + L, *gb = gW + (int64_t)d * L, *mW = gb + L,
          *vW = mW + ((int64_t)d * L + L), *Z = vW + ((int64_t)d * L + L), *G = Z + n_train * L,
          *Zte = G + n_train * L;
    // W and b are adjacent, as are their gradients: one Adam update covers both
    LNE_HIP(ctx, hipMemsetAsync(W, 0, sizeof(float) * (size_t)((int64_t)d * L + L), ctx->stream));
    LNE_HIP(ctx, hipMemsetAsync(mW, 0, sizeof(float) * (size_t)(2 * ((int64_t)d * L + L)),
                                ctx->stream));
    LNE_HIP(ctx, hipMemsetAsync(cnt.p, 0, 3 * sizeof(unsigned long long), ctx->stream));
    {
        Launch Lc(ctx, "score");
        unsigned long long *bad = cnt.as<unsigned long long>() + 2;
        k_gather_rows<<<grid_of(n_train * (d + L), 256), 256, 0, ctx->stream>>>(
            X, n, d, labels, L, train, n_train, Xtr, Ytr, bad);
        k_gather_rows<<<grid_of(n_test * (d + L), 256), 256, 0, ctx->stream>>>(
            X, n, d, labels, L, test, n_test, Xte, Yte, bad);
        k_col_stats<<<grid_of(d, 64), 64, 0, ctx->stream>>>(Xtr, n_train, d, mu, isd);
        k_standardize<<<grid_of(n_train * d, 256), 256, 0, ctx->stream>>>(Xtr, n_train, d, mu, isd);
        k_standardize<<<grid_of(n_test * d, 256), 256, 0, ctx->stream>>>(Xte, n_test, d, mu, isd);
        const float b1 = 0.9f, b2 = 0.999f;
        for (int e = 1; e <= epochs; ++e) {
            k_lin_fwd<<<grid_of(n_train * L, 256), 256, 0, ctx->stream>>>(Xtr, d, W, b, L, n_train,
                                                                          Z, nullptr);
            k_bce_grad<<<grid_of(n_train * L, 256), 256, 0, ctx->stream>>>(
                Z, Ytr, n_train * L, 1.0f / (float)n_train, G);
            k_lin_wgrad<<<grid_of((int64_t)d * L + L, 256), 256, 0, ctx->stream>>>(
                Xtr, d, G, L, n_train, W, l2, gW, gb);
            k_adam<<<grid_of((int64_t)d * L + L, 256), 256, 0, ctx->stream>>>(
                W, gW, mW, vW, (int64_t)d * L + L, lr, b1, b2, 1e-8f,
                1.0f - powf(b1, (float)e), 1.0f - powf(b2, (float)e));
        }
        k_lin_fwd<<<grid_of(n_test * L, 256), 256, 0, ctx->stream>>>(Xte, d, W, b, L, n_test, Zte,
                                                                     nullptr);
        k_topk_f1<<<grid_of(n_test, 256), 256, 0, ctx->stream>>>(Zte, Yte, n_test, L,
                                                                 cnt.as<unsigned long long>());
    }
    LNE_TRY(check_launch(ctx, "score"));
    unsigned long long h[3] = {0, 0, 0};
    LNE_HIP(ctx, hipMemcpyAsync(h, cnt.p, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
    LNE_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (h[2]) return fail(ctx, LNE_EINVAL, "score_micro_f1: %llu row indices outside [0, n)", h[2]);
    // top-k with k = true count: FP = FN = k - TP per row
    const double tp = (double)h[0], fp = (double)(h[1] - h[0]);
    *f1 = (2 * tp + 2 * fp) > 0 ? 2 * tp / (2 * tp + 2 * fp) : 0.0;
    return LNE_OK;
}

}  // extern "C"
