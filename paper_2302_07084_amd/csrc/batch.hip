// Batched hyperparameter trials on one graph (section 4.4 searches s_1..s_T,
// k, theta and mu per graph): one channel sampling pass shared by every
// trial, then the rest of the path for a whole batch of trials at once.
//
// A batch object keeps, per graph: the channel CSR (lengths kept in the
// columns), the shared Gaussian test matrix Omega, the trial-major dense
// workspace (n x k' and n x d blocks per trial), a device table of per-trial
// coefficients, and a scratch arena for the dense steps.  A run writes the
// coefficient table, then enqueues the batched steps; in graph mode that
// launch sequence is captured once per (trials, Chebyshev order) into a HIP
// graph and replayed, so a run costs one graph launch.  The launch shapes of
// the two SpMM kernels are picked by timing every variant on the batch's own
// matrix when the batch is created (optionally cached in a JSON-lines file
// named by LNE_TUNE_CACHE).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "common.hpp"

using namespace lne;

namespace {

constexpr int kMaxCheb = 64;

lne_status check_trial(lne_ctx *ctx, const lne_trial *t, int T) {
    double tot = 0.0;
    for (int r = 0; r < T; ++r) {
        if (!(t->s[r] >= 0.0) || !std::isfinite(t->s[r]))
            return fail(ctx, LNE_EINVAL, "trial: s must be finite and >= 0");
        tot += t->s[r];
    }
    if (!(tot > 0.0)) return fail(ctx, LNE_EINVAL, "trial: s must have a positive sum");
    if (t->cheb_k < 0 || t->cheb_k > kMaxCheb || !std::isfinite(t->theta) || t->theta < 0.0 ||
        !std::isfinite(t->mu))
        return fail(ctx, LNE_EINVAL, "trial: cheb_k in 0..64, theta >= 0, mu finite");
    return LNE_OK;
}

// Channel weights of each trial, 16 doubles per trial (zeros beyond T):
// s_t[r] / pi_r with s_t and the channel pass's length distribution pi
// (p->s) both normalised.
std::vector<double> trial_coef(const lne_trial *trials, int ntr, const lne_params *p) {
    const int T = p->T;
    double pt = 0.0;
    for (int r = 0; r < T; ++r) pt += p->s[r];
    std::vector<double> c(16 * (size_t)ntr, 0.0);
    for (int t = 0; t < ntr; ++t) {
        double tot = 0.0;
        for (int r = 0; r < T; ++r) tot += trials[t].s[r];
        for (int r = 0; r < T; ++r) {
            const double pi = p->s[r] / pt;
            c[16 * t + r] = pi > 0.0 ? (trials[t].s[r] / tot) / pi : 0.0;
        }
    }
    return c;
}

// A trial is estimable from the channels iff pi_r > 0 wherever s_r > 0.
lne_status check_support(lne_ctx *ctx, const lne_trial *t, const lne_params *p) {
    for (int r = 0; r < p->T; ++r)
        if (t->s[r] > 0.0 && !(p->s[r] > 0.0))
            return fail(ctx, LNE_EINVAL,
                        "trial: s_%d > 0 but the channel pass never draws length %d", r + 1, r + 1);
    return LNE_OK;
}

// vol^2 / (2 b M) / 2^16: Eq. (1)'s constant on fixed-point counts
double tl_scale(const Graph *g, const lne_params *p) {
    const double vol = (double)g->n_arcs;
    return vol * vol / (2.0 * (double)p->b * (double)p->M) / 65536.0;
}

int64_t round8(int64_t x) { return (x + 7) / 8 * 8; }
size_t round256(size_t x) { return (x + 255) / 256 * 256; }

bool trial_on(const lne_trial &t) { return t.cheb_k > 0 && t.theta >= 1e-12; }

// CholeskyQR2 of nb blocks (n x k, rows ld apart, blocks ys apart) in place;
// entry b's flags at fl + kFlagStride b: status, shifted count, third pass.
lne_status orth_batch(lne_ctx *ctx, float *Y, int64_t n, int k, int64_t ld, int64_t ys, int nb,
                      int32_t *fl) {
    Buf G(ctx), W(ctx);
    LNE_TRY(alloc(ctx, G, sizeof(double) * (size_t)nb * k * k));
    LNE_TRY(alloc(ctx, W, sizeof(double) * (size_t)nb * k * k));
    for (int pass = 0; pass < 3; ++pass) {
        const int32_t *skip = pass == 2 ? fl + 2 : nullptr;
        int32_t *next = pass == 0 ? fl + 2 : nullptr;
        LNE_TRY(gram(ctx, Y, LNE_F32, n, k, ld, G.as<double>(), skip, nb, ys));
        LNE_TRY(chol_inv(ctx, G.as<double>(), k, W.as<double>(), fl, fl + 1, n, skip, next, nb));
        LNE_TRY(project(ctx, Y, LNE_F32, ld, n, k, W.as<double>(), k, Y, LNE_F32, ld, skip, nb, ys,
                        (int64_t)k * k, ys));
    }
    return LNE_OK;
}

// eigSVD step of nb blocks: out_b = Y_b V_b Lambda_b^(-1/4) restricted to the
// top kout eigenpairs of Y_b^T Y_b (= U S^(1/2)); entries with on[b] == 0 are
// copied through (k == kout).
lne_status eig_project(lne_ctx *ctx, const float *Y, int64_t n, int k, int64_t ld, int64_t ys,
                       int nb, int kout, const int32_t *on, float *out, int64_t ldo, int64_t os) {
    Buf G(ctx), V(ctx), lam(ctx), W(ctx);
    LNE_TRY(alloc(ctx, G, sizeof(double) * (size_t)nb * k * k));
    LNE_TRY(alloc(ctx, V, sizeof(double) * (size_t)nb * k * k));
    LNE_TRY(alloc(ctx, lam, sizeof(double) * (size_t)nb * k));
    LNE_TRY(alloc(ctx, W, sizeof(double) * (size_t)nb * k * kout));
    LNE_TRY(gram(ctx, Y, LNE_F32, n, k, ld, G.as<double>(), nullptr, nb, ys));
    LNE_TRY(sym_eig(ctx, G.as<double>(), k, V.as<double>(), lam.as<double>(), nb));
    LNE_TRY(eig_weights(ctx, V.as<double>(), lam.as<double>(), k, kout, -0.25, W.as<double>(),
                        nullptr, nb, on));
    return project(ctx, Y, LNE_F32, ld, n, k, W.as<double>(), kout, out, LNE_F32, ldo, nullptr, nb,
                   ys, (int64_t)k * kout, os);
}

}  // namespace

struct lne_batch {
    lne_ctx *ctx = nullptr;
    Graph g{};
    Buf rp64;
    lne_params p{};
    int32_t max_trials = 0;
    int64_t n = 0;
    int32_t kp = 0, d = 0, dp = 0, d8 = 0;
    double scale = 0.0;
    lne_csr ext{};
    // device workspace
    Buf om, A, B, X0, P0, P1, P2, PZ, PC, XO, tab, flags, arena;
    size_t off_chan = 0, off_c0 = 0, off_one = 0, off_on = 0, off_pc = 0, tab_bytes = 0;
    int arena_for = 0;        // largest trial count the arena has been sized for
    int spmm_v = 0, gspmm_v = 0;
    // captured launch sequence
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int g_ntr = 0, g_K = -1, captures = 0;
    std::vector<char> host_tab;

    double *chan() const { return (double *)(tab.as<char>() + off_chan); }
    float *c0() const { return (float *)(tab.as<char>() + off_c0); }
    float *one() const { return (float *)(tab.as<char>() + off_one); }
    int32_t *on() const { return (int32_t *)(tab.as<char>() + off_on); }
    float *pc() const { return (float *)(tab.as<char>() + off_pc); }
};

namespace {

void drop_graph(lne_batch *b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->g_ntr = 0;
    b->g_K = -1;
}

// Every step after the sampling pass for trials 0..ntr-1 (coefficient table
// already on the device), highest Chebyshev order K; no host synchronisation,
// scratch only from the context allocator.
lne_status enqueue_trials(lne_batch *b, int ntr, int K) {
    lne_ctx *ctx = b->ctx;
    const int64_t n = b->n;
    const int kp = b->kp, d = b->d, dp = b->dp, d8 = b->d8;
    const int64_t ys = n * dp, xs = n * d8;
    int32_t *fl = b->flags.as<int32_t>();
    LNE_TRY(fill_u32(ctx, fl, (int64_t)ntr * kFlagStride, 0u));

    // fast randomized SVD (Algorithm "Fast Randomized SVD") of every trial
    float *Q = b->A.as<float>(), *Y = b->B.as<float>();
    LNE_TRY(spmm_chan(ctx, &b->ext, ntr, b->chan(), b->om.as<float>(), dp, 0, Y, dp, ys, dp,
                      b->spmm_v));
    LNE_TRY(orth_batch(ctx, Y, n, kp, dp, ys, ntr, fl));
    std::swap(Q, Y);
    for (int it = 1; it <= b->p.q; ++it) {
        LNE_TRY(spmm_chan(ctx, &b->ext, ntr, b->chan(), Q, dp, ys, Y, dp, ys, dp, b->spmm_v));
        if (it < b->p.q) {
            LNE_TRY(orth_batch(ctx, Y, n, kp, dp, ys, ntr, fl));
            std::swap(Q, Y);
        } else {
            LNE_TRY(eig_project(ctx, Y, n, kp, dp, ys, ntr, d, nullptr, b->X0.as<float>(), d8, xs));
        }
    }

    // Chebyshev propagation (section 4.3) of every trial, one graph SpMM per
    // recurrence step; trials that are off have all-zero recurrence
    // coefficients and a pass-through final step
    const float *F = b->X0.as<float>();
    if (K > 0) {
        float *T0 = b->P0.as<float>(), *T1 = b->P1.as<float>(), *T2 = b->P2.as<float>();
        float *Z = b->PZ.as<float>(), *conv = b->PC.as<float>();
        const int64_t tot = (int64_t)ntr * xs;
        const float *pc = b->pc();
        auto cc = [&](int call) { return pc + (size_t)call * ntr * 5; };
        LNE_TRY(scale_blocks(ctx, b->X0.as<float>(), T0, tot, xs, b->one()));
        LNE_TRY(scale_blocks(ctx, T0, conv, tot, xs, b->c0()));
        LNE_TRY(gspmm_batch(ctx, &b->g, ntr, d8, d8, xs, T0, Z, nullptr, nullptr, nullptr, cc(0),
                            b->gspmm_v));
        LNE_TRY(gspmm_batch(ctx, &b->g, ntr, d8, d8, xs, Z, T1, T0, nullptr, conv, cc(1),
                            b->gspmm_v));
        for (int i = 2; i <= K; ++i) {
            LNE_TRY(gspmm_batch(ctx, &b->g, ntr, d8, d8, xs, T1, Z, nullptr, nullptr, nullptr,
                                cc(2 * i - 2), b->gspmm_v));
            LNE_TRY(gspmm_batch(ctx, &b->g, ntr, d8, d8, xs, Z, T2, T1, T0, conv, cc(2 * i - 1),
                                b->gspmm_v));
            float *tmp = T0;
            T0 = T1;
            T1 = T2;
            T2 = tmp;
        }
        LNE_TRY(axpby(ctx, b->X0.p, conv, conv, (int64_t)ntr * n, d8, d8, LNE_F32, 1.0, -1.0));
        LNE_TRY(gspmm_batch(ctx, &b->g, ntr, d8, d8, xs, conv, Z, nullptr, nullptr, nullptr,
                            cc(2 * K), b->gspmm_v));
        F = Z;
    }
    // final eigSVD: X = U_p S_p^(1/2)
    return eig_project(ctx, F, n, d, d8, xs, ntr, d, b->on(), b->XO.as<float>(), d, n * d);
}

// Host side of the coefficient table for a run; returns the highest order K.
int fill_table(lne_batch *b, const lne_trial *tr, int ntr) {
    const int T = b->p.T;
    std::vector<char> &h = b->host_tab;
    std::fill(h.begin(), h.end(), 0);
    double *chan = (double *)(h.data() + b->off_chan);
    float *c0 = (float *)(h.data() + b->off_c0);
    float *one = (float *)(h.data() + b->off_one);
    int32_t *on = (int32_t *)(h.data() + b->off_on);
    float *pc = (float *)(h.data() + b->off_pc);
    const std::vector<double> cf = trial_coef(tr, ntr, &b->p);
    int K = 0;
    for (int t = 0; t < ntr; ++t) {
        for (int r = 0; r < T; ++r) chan[16 * t + r] = cf[16 * t + r];
        one[t] = 1.0f;
        on[t] = trial_on(tr[t]) ? 1 : 0;
        if (on[t]) K = std::max(K, (int)tr[t].cheb_k);
    }
    if (K == 0) return 0;
    auto set = [&](int call, int t, float a, float bb, float c1, float c2, float e) {
        float *q = pc + ((size_t)call * ntr + t) * 5;
        q[0] = a; q[1] = bb; q[2] = c1; q[3] = c2; q[4] = e;
    };
    for (int t = 0; t < ntr; ++t) {
        if (!on[t]) {
            set(2 * K, t, 1.f, 0.f, 0.f, 0.f, 0.f);       // X_sp = X0 - 0
            continue;
        }
        // g(lambda) = e^(-theta/2) [I0(theta) + 2 sum_i (-1)^i I_i(theta) T_i(x)],
        // x = (L - mu I)^2 / 2 - I; T_i by the three-term recurrence
        const double th = tr[t].theta;
        const float am = (float)(1.0 - tr[t].mu);
        auto cheb = [&](int i) {
            return (i == 0 ? 1.0 : 2.0 * ((i & 1) ? -1.0 : 1.0)) * std::exp(-th / 2.0) * bessel_i(i, th);
        };
        c0[t] = (float)cheb(0);
        set(0, t, am, -1.f, 0.f, 0.f, 0.f);
        set(1, t, 0.5f * am, -0.5f, -1.f, 0.f, (float)cheb(1));
        for (int i = 2; i <= K; ++i) {
            set(2 * i - 2, t, am, -1.f, 0.f, 0.f, 0.f);
            set(2 * i - 1, t, am, -1.f, -2.f, -1.f, i <= tr[t].cheb_k ? (float)cheb(i) : 0.f);
        }
        set(2 * K, t, 0.f, 1.f, 0.f, 0.f, 0.f);
    }
    return K;
}

// ---- launch-shape tuning -----------------------------------------------------
std::string tune_key(const char *op, const lne_batch *b, int k) {
    return shape_key(op, b->n, op[0] == 's' ? b->ext.nnz : b->g.n_arcs, k, LNE_F32);
}

lne_status tune(lne_batch *b) {
    lne_ctx *ctx = b->ctx;
    const int nt = std::min(2, b->max_trials);
    const int64_t ys = b->n * b->dp, xs = b->n * b->d8;
    // the batch's own distribution for timing: coef = 1
    std::vector<double> ch(16 * (size_t)nt, 0.0);
    for (int t = 0; t < nt; ++t)
        for (int r = 0; r < b->p.T; ++r) ch[16 * t + r] = 1.0;
    std::vector<float> pc(5 * (size_t)nt);
    for (int t = 0; t < nt; ++t) {
        pc[5 * t] = 0.8f; pc[5 * t + 1] = -1.f; pc[5 * t + 2] = 0.f; pc[5 * t + 3] = 0.f;
        pc[5 * t + 4] = 0.f;
    }
    LNE_HIP(ctx, hipMemcpyAsync(b->chan(), ch.data(), sizeof(double) * ch.size(),
                                hipMemcpyHostToDevice, ctx->stream));
    LNE_HIP(ctx, hipMemcpyAsync(b->pc(), pc.data(), sizeof(float) * pc.size(),
                                hipMemcpyHostToDevice, ctx->stream));
    LNE_TRY(pick_variant(ctx, tune_key("spmm_chan", b, b->dp), kSpmmChanVariants, [&](int var) {
        return spmm_chan(ctx, &b->ext, nt, b->chan(), b->om.as<float>(), b->dp, 0,
                         b->B.as<float>(), b->dp, ys, b->dp, var);
    }, &b->spmm_v));
    LNE_TRY(pick_variant(ctx, tune_key("graph_spmm_batch", b, b->d8), kGspmmBatchVariants,
                         [&](int var) {
        return gspmm_batch(ctx, &b->g, nt, b->d8, b->d8, xs, b->X0.as<float>(), b->P0.as<float>(),
                           nullptr, nullptr, nullptr, b->pc(), var);
    }, &b->gspmm_v));
    LNE_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return LNE_OK;
}

lne_status read_batch_flags(lne_batch *b, int ntr, lne_stats *st) {
    lne_ctx *ctx = b->ctx;
    std::vector<int32_t> h((size_t)ntr * kFlagStride);
    LNE_HIP(ctx, hipMemcpyAsync(h.data(), b->flags.p, sizeof(int32_t) * h.size(),
                                hipMemcpyDeviceToHost, ctx->stream));
    LNE_HIP(ctx, hipStreamSynchronize(ctx->stream));
    int bad = -1;
    for (int t = 0; t < ntr; ++t) {
        if (st) st->shifted += (uint32_t)h[(size_t)t * kFlagStride + 1];
        if (h[(size_t)t * kFlagStride] && bad < 0) bad = t;
    }
    if (bad >= 0) return fail(ctx, LNE_ENUMERIC, "Cholesky breakdown even after a shift (trial %d)", bad);
    return LNE_OK;
}

struct ArenaScope {
    lne_ctx *ctx;
    ArenaScope(lne_ctx *c, lne_batch *b) : ctx(c) {
        ctx->arena = b->arena.as<char>();
        ctx->arena_cap = b->arena.bytes;
        ctx->arena_used = 0;
        ctx->arena_on = true;
    }
    ~ArenaScope() {
        ctx->arena_on = false;
        ctx->arena = nullptr;
        ctx->arena_cap = 0;
        ctx->arena_used = 0;
    }
};

}  // namespace

extern "C" {

lne_status lne_sparsify_channels(lne_ctx *ctx, const lne_graph *gin, const lne_params *p,
                                 lne_csr *out, lne_stats *st) {
    if (ctx && gin && gin->weight)
        return fail(ctx, LNE_EUNSUPPORTED, "batched trials take unweighted graphs");
    if (!ctx) return LNE_EINVAL;
    if (!out) return fail(ctx, LNE_EINVAL, "sparsify_channels: out is NULL");
    LNE_TRY(validate_graph(ctx, gin));
    LNE_TRY(validate_params(ctx, p, gin->n, gin->n_arcs, false));
    std::memset(out, 0, sizeof(*out));
    GraphArg ga(ctx);
    LNE_TRY(bind_graph(ctx, gin, ga.rp, ga.g));
    const Graph *g = &ga.g;
    LNE_TRY(validate_graph_device(ctx, g));
    return channels_pass(ctx, g, p, out, st);
}

lne_status lne_trial_matrix(lne_ctx *ctx, const lne_graph *gin, const lne_params *p,
                            const lne_csr *channels, const lne_trial *trial, lne_csr *out) {
    if (ctx && gin && gin->weight)
        return fail(ctx, LNE_EUNSUPPORTED, "batched trials take unweighted graphs");
    if (!ctx) return LNE_EINVAL;
    LNE_TRY(validate_graph(ctx, gin));
    LNE_TRY(validate_params(ctx, p, gin->n, gin->n_arcs, false));
    if (!channels || !trial || !out || channels->val_type != LNE_U64 ||
        channels->n_rows != gin->n || channels->n_cols != (gin->n << 4))
        return fail(ctx, LNE_EINVAL, "trial_matrix: channels must come from lne_sparsify_channels");
    LNE_TRY(check_trial(ctx, trial, p->T));
    LNE_TRY(check_support(ctx, trial, p));
    std::memset(out, 0, sizeof(*out));
    GraphArg ga(ctx);
    LNE_TRY(bind_graph(ctx, gin, ga.rp, ga.g));
    const Graph *g = &ga.g;
    lne_csr st;
    std::memset(&st, 0, sizeof(st));
    Buf chan(ctx), sdev(ctx), vals(ctx);
    LNE_TRY(split_channels(ctx, channels, p->T, &st, chan));
    const std::vector<double> sh = trial_coef(trial, 1, p);
    lne_status s = alloc(ctx, sdev, sizeof(double) * 16);
    if (s == LNE_OK) s = alloc(ctx, vals, sizeof(float) * (size_t)(st.nnz ? st.nnz : 1));
    if (s == LNE_OK && hipMemcpyAsync(sdev.p, sh.data(), sizeof(double) * 16,
                                      hipMemcpyHostToDevice, ctx->stream) != hipSuccess)
        s = fail(ctx, LNE_EHIP, "trial_matrix: copy of s failed");
    if (s == LNE_OK)
        s = trial_values(ctx, g, &st, chan.as<uint64_t>(), p->T, sdev.as<double>(), 1,
                         tl_scale(g, p), vals.as<float>());
    if (s == LNE_OK) s = hipStreamSynchronize(ctx->stream) == hipSuccess ? LNE_OK : LNE_EHIP;
    if (s != LNE_OK) {
        lne_csr_free(ctx, &st);
        return s;
    }
    st.val = vals.detach();
    st.val_type = LNE_F32;
    *out = st;
    return LNE_OK;
}

lne_status lne_batch_create(lne_ctx *ctx, const lne_graph *gin, const lne_params *p,
                            int32_t max_trials, lne_batch **out, lne_stats *st) {
    if (ctx && gin && gin->weight)
        return fail(ctx, LNE_EUNSUPPORTED, "batched trials take unweighted graphs");
    if (!ctx) return LNE_EINVAL;
    if (!out) return fail(ctx, LNE_EINVAL, "batch_create: out is NULL");
    *out = nullptr;
    LNE_TRY(validate_graph(ctx, gin));
    LNE_TRY(validate_params(ctx, p, gin->n, gin->n_arcs, true));
    if (max_trials < 1 || max_trials > 256)
        return fail(ctx, LNE_EUNSUPPORTED, "batch_create: max_trials = %d outside 1..256", max_trials);
    if (p->precision != LNE_F32) return fail(ctx, LNE_EINVAL, "batch_create: precision must be LNE_F32");
    const int32_t kp = p->d + p->oversample;
    if (round8(kp) > 256 || round8(p->d) > 256)
        return fail(ctx, LNE_EUNSUPPORTED, "batch_create: d + oversample above 256");
    if (st) std::memset(st, 0, sizeof(*st));
    GraphArg ga(ctx);
    LNE_TRY(bind_graph(ctx, gin, ga.rp, ga.g));
    const Graph *g = &ga.g;
    LNE_TRY(validate_graph_device(ctx, g));

    lne_batch *b = new (std::nothrow) lne_batch();
    if (!b) return fail(ctx, LNE_ENOMEM, "batch_create: host allocation failed");
    struct Guard {
        lne_batch *b;
        ~Guard() { if (b) lne_batch_destroy(b); }
    } guard{b};
    b->ctx = ctx;
    b->g = *g;
    b->rp64.ctx = ctx;
    b->rp64.bytes = ga.rp.bytes;
    b->rp64.p = ga.rp.detach();   // widened offsets (if any) live with the batch
    b->p = *p;
    b->max_trials = max_trials;
    b->n = g->n;
    b->kp = kp;
    b->d = p->d;
    b->dp = (int32_t)round8(kp);
    b->d8 = (int32_t)round8(p->d);
    b->scale = tl_scale(g, p);
    for (Buf *x : {&b->om, &b->A, &b->B, &b->X0, &b->P0, &b->P1, &b->P2, &b->PZ, &b->PC, &b->XO,
                   &b->tab, &b->flags, &b->arena})
        x->ctx = ctx;

    LNE_TRY(channels_pass(ctx, g, p, &b->ext, st));
    if (st) st->nnz_counts = (uint64_t)b->ext.nnz;
    LNE_TRY(norm_channels(ctx, &b->ext, g, b->scale));

    const int64_t n = b->n, mt = max_trials;
    LNE_TRY(alloc(ctx, b->om, sizeof(float) * (size_t)n * b->dp));
    LNE_TRY(alloc(ctx, b->A, sizeof(float) * (size_t)(mt * n * b->dp)));
    LNE_TRY(alloc(ctx, b->B, sizeof(float) * (size_t)(mt * n * b->dp)));
    for (Buf *x : {&b->X0, &b->P0, &b->P1, &b->P2, &b->PZ, &b->PC})
        LNE_TRY(alloc(ctx, *x, sizeof(float) * (size_t)(mt * n * b->d8)));
    LNE_TRY(alloc(ctx, b->XO, sizeof(float) * (size_t)(mt * n * b->d)));
    LNE_TRY(alloc(ctx, b->flags, sizeof(int32_t) * (size_t)mt * kFlagStride));
    // padding columns stay zero for the life of the batch (no kernel writes them)
    for (Buf *x : {&b->om, &b->A, &b->B, &b->X0, &b->P0, &b->P1, &b->P2, &b->PZ, &b->PC})
        LNE_HIP(ctx, hipMemsetAsync(x->p, 0, x->bytes, ctx->stream));
    b->off_chan = 0;
    b->off_c0 = round256(b->off_chan + sizeof(double) * 16 * mt);
    b->off_one = round256(b->off_c0 + sizeof(float) * mt);
    b->off_on = round256(b->off_one + sizeof(float) * mt);
    b->off_pc = round256(b->off_on + sizeof(int32_t) * mt);
    b->tab_bytes = round256(b->off_pc + sizeof(float) * 5 * mt * (2 * kMaxCheb + 1));
    LNE_TRY(alloc(ctx, b->tab, b->tab_bytes));
    b->host_tab.assign(b->tab_bytes, 0);
    // the shared test matrix of Algorithm "Fast Randomized SVD" (same seed and
    // values as the single-trial path)
    LNE_TRY(launch_gaussian(ctx, n, kp, b->dp, p->seed, LNE_F32, b->om.p));
    LNE_TRY(tune(b));
    LNE_HIP(ctx, hipStreamSynchronize(ctx->stream));
    guard.b = nullptr;
    *out = b;
    return LNE_OK;
}

lne_status lne_batch_run(lne_batch *b, const lne_trial *trials, int32_t n_trials, int32_t mode,
                         float *X, lne_stats *st) {
    if (!b) return LNE_EINVAL;
    lne_ctx *ctx = b->ctx;
    if (!trials || !X) return fail(ctx, LNE_EINVAL, "batch_run: NULL trials or X");
    if (n_trials < 1 || n_trials > b->max_trials)
        return fail(ctx, LNE_EINVAL, "batch_run: n_trials = %d outside 1..%d", n_trials,
                    b->max_trials);
    if (mode != LNE_BATCH_EAGER && mode != LNE_BATCH_GRAPH)
        return fail(ctx, LNE_EINVAL, "batch_run: mode %d", mode);
    for (int t = 0; t < n_trials; ++t) {
        LNE_TRY(check_trial(ctx, &trials[t], b->p.T));
        LNE_TRY(check_support(ctx, &trials[t], &b->p));
    }
    if (st) std::memset(st, 0, sizeof(*st));
    const int ntr = n_trials;
    const int K = fill_table(b, trials, ntr);
    LNE_HIP(ctx, hipMemcpyAsync(b->tab.p, b->host_tab.data(), b->tab_bytes, hipMemcpyHostToDevice,
                                ctx->stream));
    if (b->arena_for < ntr) {
        // size the scratch arena on an eager run with real allocations
        drop_graph(b);
        b->arena.release();
        ctx->arena_need = 0;
        ctx->arena_measure = true;
        const lne_status s = enqueue_trials(b, ntr, K);
        ctx->arena_measure = false;
        LNE_TRY(s);
        LNE_HIP(ctx, hipStreamSynchronize(ctx->stream));
        LNE_TRY(alloc(ctx, b->arena, ctx->arena_need + 4096));
        b->arena_for = ntr;
    } else if (mode == LNE_BATCH_EAGER) {
        ArenaScope scope(ctx, b);
        LNE_TRY(enqueue_trials(b, ntr, K));
    } else {
        if (!b->exec || b->g_ntr != ntr || b->g_K != K) {
            drop_graph(b);
            if (!b->cap) LNE_HIP(ctx, hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
            hipStream_t user = ctx->stream;
            // the table upload above must land before the capture stream's
            // work is replayed; replays run on the user stream, so only the
            // captured launches go to the capture stream
            ctx->stream = b->cap;
            ctx->capturing = true;
            lne_status s;
            {
                ArenaScope scope(ctx, b);
                if (hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
                    s = fail(ctx, LNE_EHIP, "batch_run: stream capture could not start");
                } else {
                    s = enqueue_trials(b, ntr, K);
                    hipGraph_t gr = nullptr;
                    const hipError_t e = hipStreamEndCapture(b->cap, &gr);
                    if (s == LNE_OK && e != hipSuccess)
                        s = fail(ctx, LNE_EHIP, "batch_run: capture failed: %s", hipGetErrorString(e));
                    if (s == LNE_OK) {
                        b->graph = gr;
                        if (hipGraphInstantiate(&b->exec, gr, nullptr, nullptr, 0) != hipSuccess)
                            s = fail(ctx, LNE_EHIP, "batch_run: graph instantiation failed");
                    } else if (gr) {
                        (void)hipGraphDestroy(gr);
                    }
                }
            }
            ctx->capturing = false;
            ctx->stream = user;
            if (s != LNE_OK) {
                drop_graph(b);
                return s;
            }
            b->g_ntr = ntr;
            b->g_K = K;
            b->captures += 1;
        }
        LNE_HIP(ctx, hipGraphLaunch(b->exec, ctx->stream));
    }
    LNE_HIP(ctx, hipMemcpyAsync(X, b->XO.p, sizeof(float) * (size_t)ntr * b->n * b->d,
                                hipMemcpyDeviceToDevice, ctx->stream));
    if (st) {
        st->nnz_counts = (uint64_t)b->ext.nnz;
    }
    return read_batch_flags(b, ntr, st);
}

lne_status lne_batch_resample(lne_batch *b, const double *pi, lne_stats *st) {
    if (!b) return LNE_EINVAL;
    lne_ctx *ctx = b->ctx;
    if (!pi) return fail(ctx, LNE_EINVAL, "batch_resample: pi is NULL");
    lne_params p = b->p;
    for (int r = 0; r < p.T; ++r) p.s[r] = pi[r];
    LNE_TRY(validate_params(ctx, &p, b->g.n, b->g.n_arcs, true));
    if (st) std::memset(st, 0, sizeof(*st));
    LNE_HIP(ctx, hipStreamSynchronize(ctx->stream));
    drop_graph(b);
    lne_csr_free(ctx, &b->ext);
    std::memset(&b->ext, 0, sizeof(b->ext));
    b->p = p;
    LNE_TRY(channels_pass(ctx, &b->g, &b->p, &b->ext, st));
    if (st) st->nnz_counts = (uint64_t)b->ext.nnz;
    LNE_TRY(norm_channels(ctx, &b->ext, &b->g, b->scale));
    LNE_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return LNE_OK;
}

lne_status lne_batch_spmm(lne_batch *b, const lne_trial *trials, int32_t n_trials,
                          const float *X, int64_t ldx, int64_t xs, float *Y, int64_t ldy,
                          int64_t ys, int32_t k) {
    if (!b) return LNE_EINVAL;
    lne_ctx *ctx = b->ctx;
    if (!trials || !X || !Y) return fail(ctx, LNE_EINVAL, "batch_spmm: NULL argument");
    if (n_trials < 1 || n_trials > b->max_trials)
        return fail(ctx, LNE_EINVAL, "batch_spmm: n_trials = %d outside 1..%d", n_trials,
                    b->max_trials);
    if (k < 4 || ldx < k || ldy < k || xs < 0 || ys < (int64_t)b->n * ldy)
        return fail(ctx, LNE_EINVAL, "batch_spmm: bad dimensions");
    for (int t = 0; t < n_trials; ++t) {
        LNE_TRY(check_trial(ctx, &trials[t], b->p.T));
        LNE_TRY(check_support(ctx, &trials[t], &b->p));
    }
    (void)fill_table(b, trials, n_trials);
    LNE_HIP(ctx, hipMemcpyAsync(b->tab.p, b->host_tab.data(), b->tab_bytes, hipMemcpyHostToDevice,
                                ctx->stream));
    LNE_TRY(spmm_chan(ctx, &b->ext, n_trials, b->chan(), X, ldx, xs, Y, ldy, ys, k, b->spmm_v));
    LNE_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return LNE_OK;
}

lne_status lne_batch_info(const lne_batch *b, int32_t *spmm_variant, int32_t *gspmm_variant,
                          int64_t *channel_nnz, int32_t *captures) {
    if (!b) return LNE_EINVAL;
    if (spmm_variant) *spmm_variant = b->spmm_v;
    if (gspmm_variant) *gspmm_variant = b->gspmm_v;
    if (channel_nnz) *channel_nnz = b->ext.nnz;
    if (captures) *captures = b->captures;
    return LNE_OK;
}

void lne_batch_destroy(lne_batch *b) {
    if (!b) return;
    lne_ctx *ctx = b->ctx;
    if (ctx) (void)hipStreamSynchronize(ctx->stream);
    drop_graph(b);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    if (ctx) lne_csr_free(ctx, &b->ext);
    delete b;
}

lne_status lne_embed_batch(lne_ctx *ctx, const lne_graph *g, const lne_params *p,
                           const lne_trial *trials, int32_t n_trials, float *X, lne_stats *st) {
    if (ctx && g && g->weight)
        return fail(ctx, LNE_EUNSUPPORTED, "batched trials take unweighted graphs");
    if (!ctx) return LNE_EINVAL;
    if (!trials || !X) return fail(ctx, LNE_EINVAL, "embed_batch: NULL trials or X");
    if (n_trials < 1 || n_trials > 256)
        return fail(ctx, LNE_EUNSUPPORTED, "embed_batch: n_trials = %d outside 1..256", n_trials);
    LNE_TRY(validate_graph(ctx, g));
    LNE_TRY(validate_params(ctx, p, g->n, g->n_arcs, true));
    for (int t = 0; t < n_trials; ++t) {
        LNE_TRY(check_trial(ctx, &trials[t], p->T));
        LNE_TRY(check_support(ctx, &trials[t], p));
    }
    lne_batch *b = nullptr;
    lne_stats s0;
    LNE_TRY(lne_batch_create(ctx, g, p, n_trials, &b, &s0));
    const lne_status s = lne_batch_run(b, trials, n_trials, LNE_BATCH_EAGER, X, st);
    if (st) {
        st->attempted = s0.attempted;
        st->accepted = s0.accepted;
    }
    lne_batch_destroy(b);
    return s;
}

}  // extern "C"
