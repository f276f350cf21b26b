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

// ---- batched scorer ----------------------------------------------------------
// ntr embeddings scored at once: X is ntr x n x d (trial-major); the training
// rows of trial t are gathered into Xtr + t n_tr d and standardised with that
// trial's statistics; labels are shared.  Parameters of trial t: W (d x L)
// followed by b (L) at P + t (d + 1) L.

// Xs[t][r][c] = X[t][idx[r]][c]; out-of-range indices are counted in *bad.
__global__ void k_sc_gather(const float *__restrict__ X, int64_t n, int d, int ntr,
                            const int32_t *__restrict__ idx, int64_t n_sel,
                            float *__restrict__ Xs, unsigned long long *__restrict__ bad) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)ntr * n_sel * d) return;
    const int64_t tr = t / (n_sel * d);
    const int64_t rem = t - tr * n_sel * d;
    const int64_t r = rem / d;
    const int c = (int)(rem - r * d);
    const int64_t src = idx[r];
    if (src < 0 || src >= n) {
        if (c == 0 && tr == 0) atomicAdd(bad, 1ull);
        Xs[t] = 0.0f;
        return;
    }
    Xs[t] = X[(tr * n + src) * d + c];
}

__global__ void k_sc_labels(const uint8_t *__restrict__ lab, int64_t n, int L,
                            const int32_t *__restrict__ idx, int64_t n_sel,
                            float *__restrict__ Ys) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_sel * L) return;
    const int64_t r = t / L;
    const int64_t src = idx[r];
    Ys[t] = (src >= 0 && src < n) ? (float)lab[src * L + (t - r * L)] : 0.0f;
}

// Column mean and inverse standard deviation of each trial's training rows:
// one 256-thread block per (trial, column), FP64 partial sums.
__global__ void __launch_bounds__(256)
k_sc_stats(const float *__restrict__ Xs, int64_t n_sel, int d, float *__restrict__ mu,
           float *__restrict__ isd) {
    const int c = blockIdx.x, tr = blockIdx.y;
    const float *x = Xs + (int64_t)tr * n_sel * d + c;
    double s = 0.0, q = 0.0;
    for (int64_t r = threadIdx.x; r < n_sel; r += 256) {
        const double v = x[r * d];
        s += v;
        q += v * v;
    }
    __shared__ double S[256], Q[256];
    S[threadIdx.x] = s;
    Q[threadIdx.x] = q;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            S[threadIdx.x] += S[threadIdx.x + o];
            Q[threadIdx.x] += Q[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double m = S[0] / (double)n_sel;
        const double var = Q[0] / (double)n_sel - m * m;
        mu[(int64_t)tr * d + c] = (float)m;
        isd[(int64_t)tr * d + c] = var > 1e-30 ? (float)(1.0 / sqrt(var)) : 0.0f;
    }
}

__global__ void k_sc_standardize(float *__restrict__ Xs, int64_t n_sel, int d, int ntr,
                                 const float *__restrict__ mu, const float *__restrict__ isd) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)ntr * n_sel * d) return;
    const int64_t tr = t / (n_sel * d);
    const int c = (int)(t % d);
    Xs[t] = (Xs[t] - mu[tr * d + c]) * isd[tr * d + c];
}

// G[t][r][o] = (sigmoid(b_o + x_r . W[:, o]) - Y[r][o]) / n_sel
__global__ void k_sc_fwd_grad(const float *__restrict__ Xs, int64_t n_sel, int d, int L, int ntr,
                              const float *__restrict__ P, const float *__restrict__ Y,
                              float inv_n, float *__restrict__ G) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)ntr * n_sel * L) return;
    const int64_t tr = t / (n_sel * L);
    const int64_t rem = t - tr * n_sel * L;
    const int64_t r = rem / L;
    const int o = (int)(rem - r * L);
    const float *W = P + tr * (int64_t)(d + 1) * L;
    const float *x = Xs + (tr * n_sel + r) * d;
    float z = W[(int64_t)d * L + o];
    for (int i = 0; i < d; ++i) z += x[i] * W[(int64_t)i * L + o];
    G[t] = (1.0f / (1.0f + expf(-z)) - Y[rem]) * inv_n;
}

// part[t][p][i][o] = sum over rows r in chunk p of X[t][r][i] G[t][r][o]
// (row i = d: the bias, X = 1).
__global__ void k_sc_wgrad(const float *__restrict__ Xs, int64_t n_sel, int d, int L, int ntr,
                           const float *__restrict__ G, int nchunk, float *__restrict__ part) {
    const int64_t per = (int64_t)(d + 1) * L;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)ntr * nchunk * per) return;
    const int64_t tr = t / (nchunk * per);
    const int64_t rem = t - tr * nchunk * per;
    const int p = (int)(rem / per);
    const int64_t j = rem - (int64_t)p * per;
    const int i = (int)(j / L), o = (int)(j - (int64_t)i * L);
    const int64_t rows = (n_sel + nchunk - 1) / nchunk;
    const int64_t r0 = p * rows, r1 = min(n_sel, r0 + rows);
    const float *x = Xs + tr * n_sel * d;
    const float *g = G + tr * n_sel * L;
    float s = 0.0f;
    if (i < d)
        for (int64_t r = r0; r < r1; ++r) s += x[r * d + i] * g[r * L + o];
    else
        for (int64_t r = r0; r < r1; ++r) s += g[r * L + o];
    part[t] = s;
}

// Adam on every trial's (W, b): gradient = sum of the chunk partials + l2 W.
__global__ void k_sc_adam(float *__restrict__ P, const float *__restrict__ part, int nchunk,
                          int d, int L, int ntr, float l2, float *__restrict__ m,
                          float *__restrict__ v, float lr, float b1, float b2, float eps,
                          float c1, float c2) {
    const int64_t per = (int64_t)(d + 1) * L;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)ntr * per) return;
    const int64_t tr = t / per, j = t - tr * per;
    float g = 0.0f;
    for (int p = 0; p < nchunk; ++p) g += part[(tr * nchunk + p) * per + j];
    if (j < (int64_t)d * L) g += l2 * P[t];
    const float mm = b1 * m[t] + (1.0f - b1) * g;
    const float vv = b2 * v[t] + (1.0f - b2) * g * g;
    m[t] = mm;
    v[t] = vv;
    P[t] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

// Per (trial, test row): logits from the raw row X[t][idx[r]] standardised on
// the fly, top-k prediction with k the true label count (ties by label index)
// and the true positives; counts[2 t] += TP, counts[2 t + 1] += k.  LMAX > 0:
// the logits live in registers (L <= LMAX); LMAX == 0: in Z (L floats per row).
template <int LMAX>
__global__ void k_sc_test(const float *__restrict__ X, int64_t n, int d, int L, int ntr,
                          const int32_t *__restrict__ idx, int64_t n_sel,
                          const uint8_t *__restrict__ lab, const float *__restrict__ mu,
                          const float *__restrict__ isd, const float *__restrict__ P,
                          float *__restrict__ Z, unsigned long long *__restrict__ counts) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)ntr * n_sel) return;
    const int64_t tr = t / n_sel, r = t - tr * n_sel;
    const int64_t src = idx[r];
    if (src < 0 || src >= n) return;
    const float *x = X + (tr * n + src) * d;
    const float *W = P + tr * (int64_t)(d + 1) * L;
    const float *m = mu + tr * d, *s = isd + tr * d;
    const uint8_t *y = lab + src * L;
    int k = 0, tp = 0;
    if constexpr (LMAX > 0) {
        float z[LMAX];
#pragma unroll
        for (int o = 0; o < LMAX; ++o) z[o] = o < L ? W[(int64_t)d * L + o] : 0.0f;
        for (int i = 0; i < d; ++i) {
            const float xi = (x[i] - m[i]) * s[i];
            const float *w = W + (int64_t)i * L;
#pragma unroll
            for (int o = 0; o < LMAX; ++o)
                if (o < L) z[o] += xi * w[o];
        }
        bool pos[LMAX];
#pragma unroll
        for (int l = 0; l < LMAX; ++l) {
            pos[l] = l < L && y[l] != 0;
            k += pos[l] ? 1 : 0;
        }
#pragma unroll
        for (int l = 0; l < LMAX; ++l) {
            if (!pos[l]) continue;
            int rank = 0;
#pragma unroll
            for (int j = 0; j < LMAX; ++j)
                rank += (j < L && (z[j] > z[l] || (z[j] == z[l] && j < l))) ? 1 : 0;
            if (rank < k) ++tp;
        }
    } else {
        float *z = Z + t * L;
        for (int o = 0; o < L; ++o) z[o] = W[(int64_t)d * L + o];
        for (int i = 0; i < d; ++i) {
            const float xi = (x[i] - m[i]) * s[i];
            const float *w = W + (int64_t)i * L;
            for (int o = 0; o < L; ++o) z[o] += xi * w[o];
        }
        for (int l = 0; l < L; ++l) k += y[l] ? 1 : 0;
        for (int l = 0; l < L; ++l) {
            if (!y[l]) continue;
            int rank = 0;
            for (int j = 0; j < L; ++j) rank += (z[j] > z[l] || (z[j] == z[l] && j < l)) ? 1 : 0;
            if (rank < k) ++tp;
        }
    }
    atomicAdd(&counts[2 * tr], (unsigned long long)tp);
    atomicAdd(&counts[2 * tr + 1], (unsigned long long)k);
}

// *bad += number of indices outside [0, n)
__global__ void k_sc_check(const int32_t *__restrict__ idx, int64_t n_sel, int64_t n,
                           unsigned long long *__restrict__ bad) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n_sel && (idx[t] < 0 || idx[t] >= n)) atomicAdd(bad, 1ull);
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

lne_status lne_score_micro_f1_batch(lne_ctx *ctx, const float *X, int32_t n_trials, int64_t n,
                                    int32_t d, const uint8_t *labels, int32_t n_labels,
                                    const int32_t *train, int64_t n_train, const int32_t *test,
                                    int64_t n_test, int32_t epochs, float lr, float l2,
                                    double *f1) {
    if (!ctx) return LNE_EINVAL;
    if (!X || !labels || !train || !test || !f1 || n < 1 || d < 1 || d > 4096 || n_labels < 1 ||
        n_labels > 1024 || n_train < 1 || n_test < 1 || epochs < 1 || n_trials < 1 ||
        n_trials > 1024)
        return fail(ctx, LNE_EINVAL, "score_micro_f1: bad arguments");
    const int L = n_labels, ntr = n_trials;
    const int64_t per = (int64_t)(d + 1) * L;
    // row chunks of the weight gradient: enough threads to fill the device
    int nchunk = 1;
    while (nchunk < 64 && (int64_t)ntr * nchunk * per < (1 << 20) && n_train / (2 * nchunk) >= 64)
        nchunk *= 2;
    Buf xtr(ctx), ytr(ctx), st(ctx), prm(ctx), g(ctx), part(ctx), zte(ctx), cnt(ctx);
    LNE_TRY(alloc(ctx, xtr, sizeof(float) * (size_t)ntr * n_train * d));
    LNE_TRY(alloc(ctx, ytr, sizeof(float) * (size_t)n_train * L));
    LNE_TRY(alloc(ctx, st, sizeof(float) * (size_t)2 * ntr * d));
    LNE_TRY(alloc(ctx, prm, sizeof(float) * (size_t)3 * ntr * per));
    LNE_TRY(alloc(ctx, g, sizeof(float) * (size_t)ntr * n_train * L));
    LNE_TRY(alloc(ctx, part, sizeof(float) * (size_t)ntr * nchunk * per));
    LNE_TRY(alloc(ctx, zte, sizeof(float) * (size_t)(L <= 64 ? 1 : ntr * n_test * L)));
    LNE_TRY(alloc(ctx, cnt, sizeof(unsigned long long) * (size_t)(2 * ntr + 1)));
    float *mu = st.as<float>(), *isd = mu + (int64_t)ntr * d;
    float *P = prm.as<float>(), *m = P + (int64_t)ntr * per, *v = m + (int64_t)ntr * per;
    unsigned long long *counts = cnt.as<unsigned long long>(), *bad = counts + 2 * ntr;
    LNE_HIP(ctx, hipMemsetAsync(prm.p, 0, prm.bytes, ctx->stream));
    LNE_HIP(ctx, hipMemsetAsync(cnt.p, 0, cnt.bytes, ctx->stream));
    {
        Launch Lc(ctx, "score");
        const int64_t nx = (int64_t)ntr * n_train * d;
        k_sc_gather<<<grid_of(nx, 256), 256, 0, ctx->stream>>>(X, n, d, ntr, train, n_train,
                                                                xtr.as<float>(), bad);
        k_sc_labels<<<grid_of(n_train * L, 256), 256, 0, ctx->stream>>>(labels, n, L, train,
                                                                          n_train, ytr.as<float>());
        k_sc_stats<<<dim3((unsigned)d, (unsigned)ntr), 256, 0, ctx->stream>>>(
            xtr.as<float>(), n_train, d, mu, isd);
        k_sc_standardize<<<grid_of(nx, 256), 256, 0, ctx->stream>>>(xtr.as<float>(), n_train, d,
                                                                     ntr, mu, isd);
        const float b1 = 0.9f, b2 = 0.999f;
        const int64_t ng = (int64_t)ntr * n_train * L, nw = (int64_t)ntr * nchunk * per,
                      np = (int64_t)ntr * per;
        for (int e = 1; e <= epochs; ++e) {
            k_sc_fwd_grad<<<grid_of(ng, 256), 256, 0, ctx->stream>>>(
                xtr.as<float>(), n_train, d, L, ntr, P, ytr.as<float>(), 1.0f / (float)n_train,
                g.as<float>());
            k_sc_wgrad<<<grid_of(nw, 256), 256, 0, ctx->stream>>>(xtr.as<float>(), n_train, d, L,
                                                                   ntr, g.as<float>(), nchunk,
                                                                   part.as<float>());
            k_sc_adam<<<grid_of(np, 256), 256, 0, ctx->stream>>>(
                P, part.as<float>(), nchunk, d, L, ntr, l2, m, v, lr, b1, b2, 1e-8f,
                1.0f - powf(b1, (float)e), 1.0f - powf(b2, (float)e));
        }
        const unsigned gt = grid_of((int64_t)ntr * n_test, 128);
        if (L <= 64)
            k_sc_test<64><<<gt, 128, 0, ctx->stream>>>(X, n, d, L, ntr, test, n_test, labels, mu,
                                                       isd, P, nullptr, counts);
        else
            k_sc_test<0><<<gt, 128, 0, ctx->stream>>>(X, n, d, L, ntr, test, n_test, labels, mu,
                                                      isd, P, zte.as<float>(), counts);
        k_sc_check<<<grid_of(n_test, 256), 256, 0, ctx->stream>>>(test, n_test, n, bad);
    }
    LNE_TRY(check_launch(ctx, "score"));
    std::vector<unsigned long long> h((size_t)(2 * ntr + 1));
    LNE_HIP(ctx, hipMemcpyAsync(h.data(), cnt.p, sizeof(unsigned long long) * h.size(),
                                hipMemcpyDeviceToHost, ctx->stream));
    LNE_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (h[2 * ntr])
        return fail(ctx, LNE_EINVAL, "score_micro_f1: %llu row indices outside [0, n)", h[2 * ntr]);
    for (int t = 0; t < ntr; ++t) {
        // top-k with k = true count: FP = FN = k - TP per row
        const double tp = (double)h[2 * t], fp = (double)(h[2 * t + 1] - h[2 * t]);
        f1[t] = (2 * tp + 2 * fp) > 0 ? 2 * tp / (2 * tp + 2 * fp) : 0.0;
    }
    return LNE_OK;
}

lne_status lne_score_micro_f1(lne_ctx *ctx, const float *X, int64_t n, int32_t d,
                              const uint8_t *labels, int32_t n_labels, const int32_t *train,
                              int64_t n_train, const int32_t *test, int64_t n_test,
                              int32_t epochs, float lr, float l2, double *f1) {
    return lne_score_micro_f1_batch(ctx, X, 1, n, d, labels, n_labels, train, n_train, test,
                                    n_test, epochs, lr, l2, f1);
}

}  // extern "C"
