// Internal declarations shared by the library's translation units: the
// context, scratch buffers, launch bookkeeping, error propagation and the
// host-side entry points of every kernel family.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <functional>
#include <map>
#include <string>
#include <vector>

#include "../../include/lne.h"

struct lne_ctx {
    hipStream_t stream = nullptr;
    lne_alloc_fn alloc = nullptr;
    lne_free_fn free_fn = nullptr;
    void *user = nullptr;
    char err[512] = {0};
    bool prof = false;
    struct Mark { std::string name; hipEvent_t a, b; };
    std::vector<Mark> marks;
    std::map<std::string, std::pair<double, int64_t>> prof_acc;
    // Bump arena: while arena_on, scratch comes from [arena, arena + arena_cap)
    // and is never returned, so a sequence of launches can be captured into a
    // graph and replayed with the same addresses; while arena_measure, every
    // request's rounded size is added to arena_need (the memory is real).
    char *arena = nullptr;
    size_t arena_cap = 0, arena_used = 0, arena_need = 0;
    bool arena_on = false, arena_measure = false;
    bool capturing = false;   // no event bracketing while a graph is captured
    bool no_events = false;   // no event bracketing (allocation-free entry points)
    std::map<std::string, int> tuned;   // launch-shape choices (pick_variant)
};

namespace lne {

lne_status fail(lne_ctx *ctx, lne_status code, const char *fmt, ...);

#define LNE_TRY(expr)                         \
    do {                                      \
        lne_status _s = (expr);               \
        if (_s != LNE_OK) return _s;          \
    } while (0)

#define LNE_HIP(ctx, expr)                                                            \
    do {                                                                              \
        hipError_t _e = (expr);                                                       \
        if (_e != hipSuccess)                                                         \
            return ::lne::fail((ctx), LNE_EHIP, "%s failed: %s (%s:%d)", #expr,       \
                               hipGetErrorString(_e), __FILE__, __LINE__);            \
    } while (0)

// Device scratch from the context allocator, released at scope exit.
// The input graph as the kernels read it: 64-bit row offsets (lne_graph
// also accepts 32-bit ones; bind_graph widens them).
struct Graph {
    int64_t n = 0;
    int64_t n_arcs = 0;
    const int64_t *row_ptr = nullptr;
    const int32_t *col = nullptr;
    const uint32_t *weight = nullptr;
};

struct Buf {
    lne_ctx *ctx = nullptr;
    void *p = nullptr;
    size_t bytes = 0;
    Buf() = default;
    explicit Buf(lne_ctx *c) : ctx(c) {}
    Buf(const Buf &) = delete;
    Buf &operator=(const Buf &) = delete;
    Buf(Buf &&o) noexcept : ctx(o.ctx), p(o.p), bytes(o.bytes) { o.p = nullptr; }
    ~Buf() { release(); }
    void release();
    void *detach() { void *q = p; p = nullptr; return q; }
    template <class T> T *as() const { return static_cast<T *>(p); }
};

lne_status alloc(lne_ctx *ctx, Buf &b, size_t bytes);
void dev_free(lne_ctx *ctx, void *p);
void *dev_alloc(lne_ctx *ctx, size_t bytes);

// Launch bookkeeping: when profiling is on, brackets the launch with events.
struct Launch {
    lne_ctx *ctx;
    const char *name;
    hipEvent_t a = nullptr, b = nullptr;
    Launch(lne_ctx *c, const char *n);
    ~Launch();
};
lne_status check_launch(lne_ctx *ctx, const char *name);

// Launch-shape tuning (tune.hip).  `key` names the operation and its shape
// (a JSON fragment "op": ..., "n": ..., ...).  The first time a key is seen,
// every variant 0..nv-1 is run once (after one warm-up run) and timed with
// events; the fastest is kept in the context and, when LNE_TUNE_CACHE names
// a file, appended to it as one JSON line (later processes read it from
// there).  During graph capture nothing is timed: a known choice or 0.
// run(v) must leave the same result whatever v, and be repeatable.
lne_status pick_variant(lne_ctx *ctx, const std::string &key, int nv,
                        const std::function<lne_status(int)> &run, int *out);
// The choice made for key so far, or dflt.
int tuned_or(lne_ctx *ctx, const std::string &key, int dflt);
// Key of an SpMM-like shape: the operation, rows, a size class of the
// nonzero count (quarter octaves, so that matrices of one graph that differ a
// little in nnz share their choice), width and element type.
std::string shape_key(const char *op, int64_t n, int64_t nnz, int k, int dtype);

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline unsigned grid_of(int64_t work, int block) {
    int64_t g = ceil_div(work, block);
    return (unsigned)(g < 1 ? 1 : g);
}

// ---- scan (k_scan.hip) ---------------------------------------------------
// Exclusive prefix sum of n values (uint32 or uint64 input) into uint64
// out[0..n]; out[n] holds the total.  Synchronous only with respect to the
// stream.
lne_status scan_u32(lne_ctx *ctx, const uint32_t *in, uint64_t *out, int64_t n);
lne_status scan_u64(lne_ctx *ctx, const uint64_t *in, uint64_t *out, int64_t n);

// ---- sampler (k_sample.hip) -----------------------------------------------
struct SamplePlan {
    uint64_t seed;
    uint64_t base;        // floor(M/m)
    uint64_t frac_thr;    // Bernoulli threshold of frac(M/m)
    uint64_t theta[16];   // length thresholds
    int32_t T;
    int32_t no_ds;        // downsampling off
    double C;
    int64_t S;            // slots per edge
    int64_t J;            // slots per thread chunk
    int64_t chunks;       // chunks per edge
    int32_t colbits;      // bits of a column id in the packed key
    int32_t cbits;        // channel bits below the column (0, or 4 when the
                          // length r is kept: key column = col << 4 | r - 1)
    int32_t upper;        // emit one entry per sample, (min, max) of its two
                          // endpoints (the upper triangle; no row filter, no
                          // channels), instead of both orientations
    // weighted graphs (all null on an unweighted one)
    const uint32_t *wt;   // arc weights A
    const uint64_t *cw;   // cw[k] = sum of wt[0..k), n_arcs + 1 entries
    const uint32_t *ea;   // weight of edge e (u < v arcs in CSR order)
    const uint32_t *guide;  // guide table of each row (weight_guide)
};

lne_status make_plan(lne_ctx *ctx, const lne_params *p, int64_t n, int64_t n_arcs,
                     SamplePlan &pl);

// Device-side structural check of the input CSR; synchronises the stream.
lne_status validate_graph_device(lne_ctx *ctx, const Graph *g);
// Edge list (u < v arcs in CSR order): eu, ev of m entries; with ea, the
// edges' weights too (weighted graphs).
lne_status build_edges(lne_ctx *ctx, const Graph *g, Buf &eu, Buf &ev, int64_t m,
                       Buf *ea = nullptr);
// Weighted graph: cw (n_arcs + 1 prefix sums of the weights), vol = sum of
// weights; EINVAL on a zero weight, EUNSUPPORTED when a weighted degree or vol
// reaches 2^32.  Synchronises the stream.
lne_status weight_info(lne_ctx *ctx, const Graph *g, Buf &cw, uint64_t *vol);
// Guide table of the weighted walk step (one uint32 per arc): for row x with
// k arcs and weighted degree W, entry b (stored at rp[x] + b) is the local
// index of the arc whose cumulative-weight slice holds ceil(b W / k).  A step
// drawing t in [0, W) starts its scan at entry floor(t k / W), at or before
// the arc that holds t, and passes about one slice on average (the guide
// tables of Chen and Asau's cutpoint method).  cw from weight_info.
lne_status weight_guide(lne_ctx *ctx, const Graph *g, const uint64_t *cw, Buf &guide);

// Sparse-sign test matrix (LNE_FLAG_SPARSE_OMEGA): kSparseOmega signed
// column entries per row, int16 sign (column + 1), one 16-byte vector per row.
constexpr int kSparseOmega = 8;
lne_status launch_sparse_omega(lne_ctx *ctx, int64_t n, int32_t k, uint64_t seed, int16_t *out);
// Y = A Omega for a sparse-sign Omega (n x k logical): the row accumulator
// lives in LDS, each nonzero gathers one 16-byte row of Omega.
lne_status spmm_sparse_omega(lne_ctx *ctx, const lne_csr *A, const int16_t *om, void *Y,
                             int64_t ldy, int32_t k, int32_t dtype);
lne_status launch_sample_slots(lne_ctx *ctx, const Graph *g, const SamplePlan &pl,
                               const int32_t *eu, const int32_t *ev, int64_t e_begin,
                               int64_t e_end, int32_t *a, int32_t *b, uint64_t *w,
                               uint8_t *r);
// Per-wave pair-entry counts (count pass) and pair emission (emit pass) for
// the rows [row_lo, row_hi); keys are relative to row_lo.  A thread's
// accepted length-1 samples (all the pair (u, v) of its edge with one weight)
// are merged into as few entries as keep each sum below 2^32.  stats (may be
// NULL, device, 3 x uint64): [0] = attempted sample slots, [1] = the largest
// per-sample fixed-point weight of an edge with an accepted sample
// (saturated at 2^32 - 1), [2] = accepted samples.
lne_status launch_sample_count(lne_ctx *ctx, const Graph *g, const SamplePlan &pl,
                               const int32_t *eu, const int32_t *ev, int64_t m, int64_t row_lo,
                               int64_t row_hi, uint32_t *wave_cnt, int64_t n_waves,
                               unsigned long long *stats);
lne_status launch_sample_emit(lne_ctx *ctx, const Graph *g, const SamplePlan &pl,
                              const int32_t *eu, const int32_t *ev, int64_t m, int64_t row_lo,
                              int64_t row_hi, const uint64_t *wave_off, uint64_t *keys,
                              uint32_t *vals);
int64_t sample_threads(const SamplePlan &pl, int64_t m);
lne_status launch_philox(lne_ctx *ctx, uint64_t seed, const uint32_t *ctr, int64_t count,
                         uint32_t *out);
lne_status launch_gaussian(lne_ctx *ctx, int64_t n, int32_t k, int64_t ld, uint64_t seed,
                           int32_t dtype, void *out);

// ---- aggregation (k_sort.hip) ----------------------------------------------
// Sorts (key, val) by the low `bits` bits of key (stable LSD radix), ping-pong
// between the two buffer pairs; returns in *which (0 or 1) the sorted copy.
// With tag_deg (and bits <= kTagShift) the keys come out tagged: bits 48..63
// of each key hold deg[key & (2^colbits - 1)] of its column vertex, or
// kTagMax when that degree is kTagMax or more.  The tag is written by the
// first pass whose input is sorted by the column bits, so the degree reads of
// a tile stay within a short column range (cache hits instead of random
// gathers); equal keys stay equal and the sort bits are untouched.
constexpr int kTagShift = 48;
constexpr uint32_t kTagMax = 0xFFFFu;
// Shift of the tagging pass for a sort over `bits` key bits of which the low
// `colbits` are the column, or -1 when no pass qualifies (then no tags).
inline int radix_tag_shift(int bits, int colbits) {
    if (bits > kTagShift) return -1;
    for (int shift = 0; shift < bits; shift += 8)
        if (shift >= colbits) return shift;
    return -1;
}
// Stable LSD sort of (key, val) on key bits [lo_bit, bits); *which = the
// buffer pair holding the result.
lne_status radix_sort(lne_ctx *ctx, uint64_t *k0, uint32_t *v0, uint64_t *k1,
                      uint32_t *v1, int64_t n, int bits, int *which,
                      const uint32_t *tag_deg = nullptr, int colbits = 0, int lo_bit = 0);
// Sorted (key, val) -> count CSR (rows, cols from the packed key).
lne_status reduce_to_csr(lne_ctx *ctx, const uint64_t *keys, const uint32_t *vals,
                         int64_t n_items, int64_t n_rows, int colbits, lne_csr *out);

// ---- Eq. (1) constants ------------------------------------------------------
// x_ab = vol^2 / (2 b M) * (W_ab / 2^16) / (d_a d_b), kept iff x_ab > 1; the
// keep decision compares W vol^2 with (2 b M 2^16) d_a d_b as exact 128-bit
// products (vol < 2^32 and 2 b M < 2^40 are validated on the host).
// On a weighted graph (edges still sampled uniformly) the factor vol^2 is
// vol 2m: x_ab = vol 2m / (2 b M) (W_ab / 2^16) / (d_a d_b) with weighted
// degrees and vol; both factors are the arc count 2m on an unweighted graph.
struct TLConst {
    uint64_t vol2;     // vol 2m (vol^2 unweighted)
    uint64_t K;        // 2 b M 2^16
    double scale;      // vol 2m / (2 b M) / 2^16
};
inline TLConst tl_const(uint64_t vol, uint64_t arcs, const lne_params *p) {
    TLConst c;
    c.vol2 = vol * arcs;
    c.K = (2ull * (uint64_t)p->b * p->M) << 16;
    c.scale = ((double)vol * (double)arcs) / (2.0 * (double)p->b * (double)p->M) / 65536.0;
    return c;
}
__device__ __forceinline__ bool tl_keep(const TLConst &c, uint64_t W, uint64_t da, uint64_t db) {
    const uint64_t dd = da * db;
    const uint64_t lh = __umul64hi(W, c.vol2), ll = W * c.vol2;
    const uint64_t rh = __umul64hi(c.K, dd), rl = c.K * dd;
    return lh > rh || (lh == rh && ll > rl);
}

// Sorted (key, val) -> the truncated-log matrix directly (the count CSR is
// never stored): every distinct pair's weights are summed by the lane that
// holds its first item, its Eq. (1) entry is ln x if kept, else an explicit
// zero.  Rows are [row_lo, row_lo + n_rows) of the graph, deg its degrees
// (vertex_degrees).  *kept (host) = the
// number of nonzero entries.  val_type LNE_F64 or LNE_F32.  tagged: the keys
// carry radix_sort's degree tags (a tag below kTagMax is the column's degree;
// kTagMax means look it up in deg).
// sym (optional, F32 only): the keys hold one entry per sample, (min, max)
// of its endpoints (the upper triangle with the diagonal); a diagonal pair's
// sum counts twice, and every distinct pair is also written transposed into
// sym->keyT, sym->valT (max << colbits | min, the value's bits), allocated
// here with out->nnz entries, for sym_assemble.
struct SymOut {
    Buf keyT, valT;
    explicit SymOut(lne_ctx *ctx) : keyT(ctx), valT(ctx) {}
};
lne_status reduce_to_matrix(lne_ctx *ctx, const uint64_t *keys, const uint32_t *vals,
                            int64_t n_items, int64_t n_rows, int colbits, const Graph *g,
                            const uint32_t *deg, int64_t row_lo, const TLConst &c,
                            int32_t val_type, lne_csr *out, uint64_t *kept,
                            bool tagged = false, SymOut *sym = nullptr);
// The symmetric matrix from its upper triangle U (reduce_to_matrix with sym,
// all rows, F32) and the transposed pairs in sym: sorts them by (max, min)
// and merges each row's lower part (without the diagonal) with U's row.
// Frees U and sym's buffers; *out = the full n x n matrix, *kept = its
// nonzero entries (kept_u = U's).
lne_status sym_assemble(lne_ctx *ctx, lne_csr *U, SymOut &sym, int colbits, uint64_t kept_u,
                        lne_csr *out, uint64_t *kept);
// deg[i] = degree of vertex i (uint32, n entries): the compact degree table
// the fused reduction gathers from; with cw (weight_info) the weighted degree.
lne_status vertex_degrees(lne_ctx *ctx, const Graph *g, uint32_t *deg,
                          const uint64_t *cw = nullptr);
// Removes explicit zeros from an F32/F64 CSR (row block), in place of *m.
lne_status drop_zeros(lne_ctx *ctx, lne_csr *m);

// ---- trunc_log (k_trunclog.hip) ---------------------------------------------
// counts covers the rows [row_lo, row_lo + counts->n_rows) of the graph.
lne_status trunc_log_csr(lne_ctx *ctx, const Graph *g, const lne_params *p,
                         const lne_csr *counts, int64_t row_lo, int32_t val_type, lne_csr *out);
// Stacks row blocks (block b holds rows [lo_b, lo_b + n_rows_b), in order)
// into one CSR of n_rows rows; the blocks are released.
lne_status concat_rows(lne_ctx *ctx, std::vector<lne_csr> &blocks, int64_t n_rows,
                       lne_csr *out);

// ---- SpMM (k_spmm.hip) -------------------------------------------------------
lne_status spmm(lne_ctx *ctx, const lne_csr *A, const void *X, int64_t ldx, void *Y,
                int64_t ldy, int32_t k, int32_t dtype);
// out = a Z + b D^-1 A Z + c1 E1 + c2 E2 ; if acc: acc += cacc * out, or
// with acc_init acc = cinit * E1 + cacc * out (acc not read; E1 needed)
// (graph adjacency without values; E1/E2/acc may be null).
lne_status graph_spmm(lne_ctx *ctx, const Graph *g, const void *Z, void *out,
                      int64_t ld, int32_t k, int32_t dtype, double a, double b,
                      const void *E1, double c1, const void *E2, double c2, void *acc,
                      double cacc, bool acc_init = false, double cinit = 0.0);
// out = a x + b y over n rows of k columns (rows ld apart), dt F64 or F32.
lne_status axpby(lne_ctx *ctx, const void *x, const void *y, void *out, int64_t n, int32_t k,
                 int64_t ld, int32_t dt, double a, double b);
// Dense elementwise: y = alpha x (conversion between dtypes allowed).
lne_status dense_scale(lne_ctx *ctx, const void *x, int32_t xt, int64_t ldx, void *y,
                       int32_t yt, int64_t ldy, int64_t n, int32_t k, double alpha);

// ---- dense (k_dense.hip) -------------------------------------------------------
// Every dense step also runs on a batch of nb independent problems in one
// launch: operand b starts at its base pointer + b * (its stride), the k x k
// results of entry b at + b k k, and entry b's flags (skip, status, shifted,
// run_next) at + kFlagStride b.
constexpr int kFlagStride = 4;
// G (k x k, FP64, leading dimension k) = Y^T Y.
// part_ws (optional): caller workspace for the per-workgroup partial Grams
// (fewer workgroups when it is small; at least nb k'^2 doubles, k' = k
// rounded up to 16).
lne_status gram(lne_ctx *ctx, const void *Y, int32_t dtype, int64_t n, int32_t k,
                int64_t ld, double *G, const int32_t *skip, int32_t nb = 1, int64_t ys = 0,
                double *part_ws = nullptr, size_t part_ws_bytes = 0);
// out (n x kout, out_t) = Y (n x kin, y_t) W (kin x kout, FP64 device, ld kout).
lne_status project(lne_ctx *ctx, const void *Y, int32_t y_t, int64_t ldy, int64_t n,
                   int32_t kin, const double *W, int32_t kout, void *out, int32_t out_t,
                   int64_t ldo, const int32_t *skip, int32_t nb = 1, int64_t ys = 0,
                   int64_t ws = 0, int64_t os = 0, void *wt_ws = nullptr);
// Workspace of project's BF16 path (W transposed to BF16).
size_t project_bf16_ws_bytes(int32_t kin, int32_t kout, int32_t nb = 1);
// Upper Cholesky G = R^T R in place (R in upper triangle, lower zeroed) and
// W = R^-1; on breakdown retries with a shift and sets *shifted.  mode 0:
// plain; mode 1: the shift is always allowed.  status: 0 ok, 1 failed.
lne_status chol_inv(lne_ctx *ctx, double *G, int32_t k, double *W, int32_t *status,
                    int32_t *shifted, int64_t n_rows, const int32_t *skip,
                    int32_t *skip_next, int32_t nb = 1);
// Graph descriptors (k_stats.hip) behind lne_graph_stats; g validated.
lne_status graph_stats_impl(lne_ctx *ctx, const Graph *g, uint64_t seed, int32_t wedges,
                            int32_t iters, double *out);
// Symmetric eigen-decomposition of C (k x k, FP64): V (k x k, columns = vectors),
// lam (k), sorted by decreasing eigenvalue.  C is overwritten.  vw_ws: a
// workspace of sym_eig_ws_doubles(k, nb) doubles (allocated when NULL).
size_t sym_eig_ws_doubles(int32_t k, int32_t nb = 1);
lne_status sym_eig(lne_ctx *ctx, double *C, int32_t k, double *V, double *lam, int32_t nb = 1,
                   double *vw_ws = nullptr);
// W (k x kout) = V[:, :kout] diag(f(lam)) with f = lam^pow (0 for
// lam <= k eps lam_max); S (kout) = sqrt(lam) (optional).  Entries b with
// on[b] == 0 (on may be NULL) get W = I and S = 1 instead (k == kout).
lne_status eig_weights(lne_ctx *ctx, const double *V, const double *lam, int32_t k,
                       int32_t kout, double power, double *W, double *S, int32_t nb = 1,
                       const int32_t *on = nullptr);

// ---- batched trials (k_batch.hip) ------------------------------------------------
// Extended count CSR (columns col << 4 | r - 1) -> structure (val NULL) plus
// channels chan[entry * T + r - 1] (uint64).
lne_status split_channels(lne_ctx *ctx, const lne_csr *ext, int T, lne_csr *st, Buf &chan);
// vals[entry * ntr + t]: truncated log of trial t's mixed counts (0 if
// dropped); s_dev[16 t + r - 1] = s_t[r] / pi_r.
lne_status trial_values(lne_ctx *ctx, const Graph *g, const lne_csr *st, const uint64_t *chan,
                        int T, const double *s_dev, int ntr, double scale, float *vals);
// Channel CSR weights in place: counts W_r -> FP64 scale W_r / (d_a d_b)
// (val_type becomes LNE_F64).
lne_status norm_channels(lne_ctx *ctx, lne_csr *ext, const Graph *g, double scale);
// Y_t (rows ldy apart, trials ys apart) = M_t X_t (ldx, xs; xs = 0 shares one
// operand) for ntr trials, M_t generated from the normalised channel CSR
// `ext` with coef[16 t + r - 1] = s_t[r] / pi_r; k <= 256, k % 4 == 0, X's columns
// up to k zero-padded.  variant: launch shape 0..5.
lne_status spmm_chan(lne_ctx *ctx, const lne_csr *ext, int ntr, const double *coef,
                     const float *X, int64_t ldx, int64_t xs, float *Y, int64_t ldy, int64_t ys,
                     int k, int variant);
constexpr int kSpmmChanVariants = 6;
// Propagation step for ntr trials (blocks zs apart, rows ld apart, k columns):
// out = a Z + b D^-1 A Z + c1 E1 + c2 E2, acc += e out, coef[5 t + {a, b, c1,
// c2, e}]; E1, E2, acc may be NULL.  variant: launch shape 0..3.
lne_status gspmm_batch(lne_ctx *ctx, const Graph *g, int ntr, int k, int64_t ld, int64_t zs,
                       const float *Z, float *out, const float *E1, const float *E2, float *acc,
                       const float *coef, int variant);
constexpr int kGspmmBatchVariants = 4;
// y[i] = alpha[i / per] x[i], i < count.
lne_status scale_blocks(lne_ctx *ctx, const float *x, float *y, int64_t count, int64_t per,
                        const float *alpha);
// p[0..count) = v (32-bit words), a kernel so that it can sit in a captured graph.
lne_status fill_u32(lne_ctx *ctx, void *p, int64_t count, uint32_t v);
double bessel_i(int n, double x);
// The channel sampling pass (lengths kept in the columns) into one CSR.
lne_status channels_pass(lne_ctx *ctx, const Graph *g, const lne_params *p, lne_csr *out,
                         lne_stats *st);

// ---- validation (abi.hip) -------------------------------------------------------
lne_status validate_graph(lne_ctx *ctx, const lne_graph *g);
// g's 64-bit view (the one every kernel reads): 64-bit offsets are used in
// place; 32-bit ones are widened into `rp` (n + 1 int64 on the context's
// stream).  g must have passed validate_graph.
lne_status bind_graph(lne_ctx *ctx, const lne_graph *g, Buf &rp, Graph &out);
struct GraphArg {
    Buf rp;    // widened offsets, when the caller's are 32-bit
    Graph g;
    explicit GraphArg(lne_ctx *c) : rp(c) {}
};
lne_status validate_params(lne_ctx *ctx, const lne_params *p, int64_t n, int64_t n_arcs,
                           bool need_linalg);
size_t dtype_size(int32_t t);

}  // namespace lne
