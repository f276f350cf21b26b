/*
 * lne.h -- C ABI of the MI355X (gfx950) sparsified-NetMF embedding library.
 *
 * The library computes the network embedding of arXiv 2302.07084 (LightNE 2.0)
 * on one GPU:
 *   sparsifier  downsampled per-edge PathSampling (section 5.2, Algorithms
 *               "PathSampling" and "Downsampled Per-Edge PathSampling",
 *               degree sampling of section 4.1) aggregated into a CSR matrix
 *   trunc_log   the entry-wise truncated logarithm of Eq. (1)
 *   rSVD        the fast randomized SVD (section 4.2, Algorithms "eigSVD" and
 *               "Fast Randomized SVD"), embedding X0 = U S^(1/2)
 *   propagate   Chebyshev spectral propagation on the input graph (section
 *               4.3) followed by a final eigSVD
 *
 * Conventions shared by every entry point
 *   - Device pointers are HIP device addresses on the current device; host
 *     pointers are marked "host".  Dense matrices are row-major with a leading
 *     dimension (elements between consecutive rows) >= their width.
 *   - All work is enqueued on the context's HIP stream.  An entry point that
 *     must learn a data-dependent size (nnz) synchronises that stream and says
 *     so.  Outputs are valid once the stream has been synchronised.
 *   - The caller owns every buffer it passes in.  Buffers the library returns
 *     (lne_csr) are allocated through the context's allocator and released
 *     with lne_csr_free.  Scratch memory comes from the same allocator and is
 *     released before the call returns.
 *   - Every function returns an lne_status; nothing throws across the ABI.
 *     Arguments are validated on the host before any GPU work is enqueued; on
 *     an error no output is written and lne_last_error() describes it.
 *   - A context is used by one host thread at a time.
 */
#ifndef LNE_H
#define LNE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t lne_status;
#define LNE_OK 0
#define LNE_EINVAL (-1)        /* invalid argument or malformed input            */
#define LNE_ENOMEM (-2)        /* the allocator returned NULL                    */
#define LNE_EHIP (-3)          /* a HIP runtime call failed                      */
#define LNE_ENUMERIC (-4)      /* breakdown of a factorisation                   */
#define LNE_EUNSUPPORTED (-5)  /* valid request outside the supported range      */

/* element types of dense matrices and of CSR values */
#define LNE_F64 0
#define LNE_F32 1
#define LNE_BF16 2
#define LNE_U64 3

/* params.flags */
#define LNE_FLAG_NO_FINAL_EIGSVD 1u  /* lne_propagate: return the filtered matrix */
/* lne_rsvd / lne_embed: the vanilla randomized SVD the paper improves on
 * (section 4.2: Q spans M Omega, B = Q^T M, U = Q U_B) instead of the fast one
 * (U = the left singular vectors of M Q); same power steps and products. */
#define LNE_FLAG_VANILLA_RSVD 2u
/* lne_rsvd / lne_embed: a sparse-sign test matrix (lne_sparse_omega) instead
 * of the Gaussian one; the first product gathers 16 bytes per nonzero. */
#define LNE_FLAG_SPARSE_OMEGA 4u
/* lne_embed: keep the sparsifier's row blocks in pinned host memory (for
 * graphs whose sparsifier exceeds HBM); the products of the randomized SVD
 * stream them over PCIe in chunks of at most env LNE_HOST_CHUNK_NNZ entries
 * (default 2^28; a longer row is a chunk of its own), the copy of one chunk
 * overlapping the product with the previous one.  Results equal those of the
 * in-HBM path. */
#define LNE_FLAG_HOST_SPARSIFIER 8u

typedef void *(*lne_alloc_fn)(size_t bytes, void *user);
typedef void (*lne_free_fn)(void *ptr, void *user);

typedef struct lne_ctx lne_ctx;

/* Undirected, simple input graph in symmetric CSR form: row i lists the
 * neighbours of vertex i in ascending order, no self-loops, no duplicates,
 * and j is in row i iff i is in row j (checked only where cheap).  Isolated
 * vertices are allowed.  weight: NULL for an unweighted graph, else one
 * positive integer weight A_ij per arc (A_ij = A_ji); then degrees are
 * d_i = sum_j A_ij, vol = sum_i d_i, degree sampling uses
 * p_e = min(1, C A_uv (1/d_u + 1/d_v)), walk steps pick neighbour j of i
 * with probability A_ij / d_i, and an accepted sample weighs
 * (r / sum over its path's r edges of 1/A) / p_e (NetSMF's path estimator);
 * Eq. (1)'s factor vol^2 / (2 b M) becomes vol 2m / (2 b M), and propagation
 * uses the weighted D^-1 A.  Weighted degrees and vol must stay below 2^32.
 * The batched-trials entry points take unweighted graphs only. */
typedef struct {
    int64_t n;                 /* vertices                                   */
    int64_t n_arcs;            /* 2m, must be < 2^32 (= vol(G) unweighted)   */
    const void *row_ptr;       /* device, n + 1 offsets of index_bits bits,  *
                                * row_ptr[0] = 0                             */
    const int32_t *col;        /* device, n_arcs entries                     */
    const uint32_t *weight;    /* device, n_arcs entries, or NULL            */
    int32_t index_bits;        /* row_ptr element width: 64 (0 reads as 64)  *
                                * or 32 (int32 offsets, n_arcs < 2^31; the   *
                                * library widens them into its own buffer at *
                                * each call, after the host-side checks)     */
} lne_graph;

/* Hyperparameters (notation table of the paper; s_r of Eq. (1)). */
typedef struct {
    int32_t T;            /* window size, 1..16                                 */
    double s[16];         /* s_1..s_T >= 0, positive sum (normalised inside)    */
    uint64_t M;           /* number of edge samples                              */
    uint32_t b;           /* negative samples, >= 1; 2 b M < 2^40               */
    double C;             /* degree-sampling constant; <= 0: ln n; +inf: off    */
    int32_t d;            /* embedding dimension                                 */
    int32_t oversample;   /* rSVD oversampling s; d + oversample <= n, <= 288   */
    int32_t q;            /* power iterations, >= 1                              */
    int32_t cheb_k;       /* propagation order k; 0 switches propagation off     */
    double theta, mu;     /* propagation filter parameters; theta < 1e-12: off   */
    uint64_t seed;        /* Philox key                                          */
    int32_t precision;    /* LNE_F64, LNE_F32 or LNE_BF16 (see lne_rsvd)         */
    uint32_t flags;       /* LNE_FLAG_*                                          */
} lne_params;

/* CSR matrix owned by the library (release with lne_csr_free). */
typedef struct {
    int64_t n_rows, n_cols, nnz;
    int64_t *row_ptr;     /* device, n_rows + 1                                  */
    int32_t *col;         /* device, nnz, ascending inside each row              */
    void *val;            /* device, nnz values of type val_type                 */
    int32_t val_type;     /* LNE_U64 (count matrix), LNE_F64 or LNE_F32          */
} lne_csr;

typedef struct {
    uint64_t attempted;   /* sample slots drawn: sum over edges of n_e           */
    uint64_t accepted;    /* samples whose downsampling coin came up heads       */
    uint64_t nnz_counts;  /* nnz of the symmetric count matrix                   */
    uint64_t nnz_log;     /* nnz after the truncated logarithm                   */
    uint32_t shifted;     /* number of shifted Cholesky fallbacks taken          */
    uint32_t reserved;
    uint64_t entries;     /* pair entries the aggregation sorted: two per       *
                           * accepted sample, except that each sampler thread's  *
                           * length-1 samples of one edge (all the pair (u, v)) *
                           * are merged into one entry per orientation           */
} lne_stats;

/* ---- context ------------------------------------------------------------ */

/* Creates a context bound to `stream` (a hipStream_t; NULL = default stream).
 * alloc/free may be NULL together, in which case hipMalloc/hipFree are used.
 * Makes no HIP call.  Errors: EINVAL (out NULL, or only one of alloc/free). */
lne_status lne_ctx_create(lne_ctx **out, void *stream, lne_alloc_fn alloc,
                          lne_free_fn free_fn, void *user);
void lne_ctx_destroy(lne_ctx *ctx);
/* Message of the last failed call on ctx (static storage inside ctx). */
const char *lne_last_error(const lne_ctx *ctx);
/* Library version string. */
const char *lne_version(void);

/* Per-kernel timing with HIP events on the context stream.  While enabled,
 * every launch is bracketed by two events; lne_prof_get synchronises and
 * returns the summed duration and launch count of kernels named `name`. */
lne_status lne_prof_enable(lne_ctx *ctx, int32_t on);
lne_status lne_prof_get(lne_ctx *ctx, const char *name, double *total_ms,
                        int64_t *launches);
lne_status lne_prof_reset(lne_ctx *ctx);

/* ---- random numbers ----------------------------------------------------- */

/* Philox4x32-10 (Salmon et al., SC'11): out[4i..4i+3] = block of counter
 * ctr[4i..4i+3] under key (seed low word, seed high word).  ctr, out: device,
 * 4 * count uint32.  Errors: EINVAL (count < 0, NULL with count > 0). */
lne_status lne_philox(lne_ctx *ctx, uint64_t seed, const uint32_t *ctr,
                      int64_t count, uint32_t *out);

/* Gaussian test matrix Omega = randn(n, k) of the fast randomized SVD (first
 * step of Algorithm "Fast Randomized SVD").  Entry (i, c) is the Box-Muller
 * transform of the first two words of Philox(counter = (i_lo, i_hi, c / 2,
 * 3 << 24)): even c takes the cosine, odd c the sine.  out: device, n x k,
 * leading dimension ld, element type dtype (values computed in double and
 * rounded).  Errors: EINVAL. */
/* Sparse-sign test matrix, the alternative Omega of the randomized SVD
 * (LNE_FLAG_SPARSE_OMEGA): row i has 8 entries; word t (t < 8) of
 * Philox(counter = (i_lo, i_hi, t / 4, 5 << 24)) picks column (z >> 1) mod k
 * and sign -1 if z is odd, +1 otherwise; entries landing on one column add.
 * out: device n x 8 int16, entry sign * (column + 1), 16-byte aligned.
 * Errors: EINVAL (k outside 1..1024). */
lne_status lne_sparse_omega(lne_ctx *ctx, int64_t n, int32_t k, uint64_t seed, int16_t *out);
/* Y = A Omega for a library CSR A and a sparse-sign Omega (lne_sparse_omega,
 * n_cols x 8): Y device n_rows x k (ldy, dtype F64 / F32 / BF16 as in
 * lne_spmm, accumulated in F64 / F32).  Errors: EINVAL. */
lne_status lne_spmm_sparse_omega(lne_ctx *ctx, const lne_csr *A, const int16_t *om, void *Y,
                                 int64_t ldy, int32_t k, int32_t dtype);
lne_status lne_gaussian(lne_ctx *ctx, int64_t n, int32_t k, int64_t ld,
                        uint64_t seed, int32_t dtype, void *out);

/* ---- sparsifier ----------------------------------------------------------- */

/* Sample slots per edge: floor(M/m) + (frac(M/m) > 0), m = n_arcs / 2.
 * Host only, no GPU work.  Returns 0 on invalid input. */
int64_t lne_slots_per_edge(const lne_params *p, int64_t n_arcs);

/* Host-side constants of the sampler (for inspection): floor(M/m), the
 * Bernoulli threshold floor(frac(M/m) 2^32) and the length thresholds
 * theta_t = floor(2^32 cumsum(s)_t / sum(s)), theta_T = 2^32.  All host. */
lne_status lne_sampler_plan(const lne_params *p, int64_t n_arcs, uint64_t *base,
                            uint64_t *frac_thr, uint64_t *theta);

/* Every sample slot (e, j), e in [e_begin, e_end), j < slots per edge, of
 * Algorithm "Downsampled Per-Edge PathSampling"; edges are the arcs (u, v),
 * u < v, in CSR order.  Slot (e, j) is written at (e - e_begin) * S + j:
 *   r[.]  = 0 if j >= n_e (empty slot), else the drawn length r in 1..T
 *   w[.]  = fixed-point weight rint(2^16 / p_e) if accepted, 0 otherwise
 *   a[.], b[.] = (u', v') of PathSampling if accepted, -1 otherwise.
 * a, b: device int32; w: device uint64; r: device uint8.
 * Errors: EINVAL (bad graph/params/range). */
lne_status lne_sample_slots(lne_ctx *ctx, const lne_graph *g, const lne_params *p,
                            int64_t e_begin, int64_t e_end, int32_t *a, int32_t *b,
                            uint64_t *w, uint8_t *r);

/* Sparsifier construction (section 5.2): runs every sample of every edge and
 * sums the fixed-point weights of equal pairs, each sample counted in both
 * orientations.  out receives the symmetric count CSR (val_type LNE_U64, units
 * of 2^-16).  Synchronises the stream (twice: to size the pair buffer and the
 * CSR).  When the pair buffers (36 bytes per pair entry) would exceed the
 * budget (env LNE_HBM_BUDGET_GB, default 70% of device memory) the rows are
 * aggregated in ranges, each walking every sample again; the result is the
 * same.  st may be NULL.  Errors: EINVAL, ENOMEM, EHIP, EUNSUPPORTED (a
 * per-sample weight above 2^32 - 1 or more than 2^31 vertices). */
lne_status lne_sparsify(lne_ctx *ctx, const lne_graph *g, const lne_params *p,
                        lne_csr *out, lne_stats *st);

/* Rows [row_lo, row_hi) of the count matrix of lne_sparsify: every sample of
 * every edge is drawn and walked, and only the pair entries whose row falls in
 * the window are aggregated (the unit of work of the row-range passes, and of
 * a row-partitioned sparsifier).  out: (row_hi - row_lo) x n count CSR, row 0
 * = vertex row_lo.  Bit-identical to the same rows of lne_sparsify.
 * Synchronises the stream.  st: attempted and accepted over all edges,
 * nnz_counts of the window.  Errors: as lne_sparsify; EINVAL on an empty or
 * out-of-range window. */
lne_status lne_sparsify_rows(lne_ctx *ctx, const lne_graph *g, const lne_params *p,
                            int64_t row_lo, int64_t row_hi, lne_csr *out, lne_stats *st);

/* Truncated logarithm of Eq. (1) on the count matrix:
 *   x_ab = vol^2 / (2 b M) * (W_ab / 2^16) / (d_a d_b)
 * kept iff x_ab > 1 (decided exactly in 128-bit integers), value ln x_ab as
 * double (precision LNE_F64) or float (otherwise).  out is compacted.
 * Synchronises the stream once (nnz).  Errors: EINVAL, ENOMEM, EHIP. */
lne_status lne_trunc_log(lne_ctx *ctx, const lne_graph *g, const lne_params *p,
                         const lne_csr *counts, lne_csr *out);

/* The truncated-log matrix exactly as lne_embed builds it (section 5.2's
 * sparsifier with Eq. (1) applied while the pairs are aggregated; no count
 * matrix is stored).  Same entries and values as lne_trunc_log of
 * lne_sparsify, except that a row block keeps its dropped pairs as explicit
 * zeros unless they are more than 1/32 of its entries.  out: n x n, row
 * offsets from 0, columns ascending, values double (precision LNE_F64) or
 * float (LNE_F32, LNE_BF16); free with lne_csr_free.  stats: attempted,
 * accepted, nnz_log = the nonzero entries.  LNE_FLAG_HOST_SPARSIFIER is
 * ignored (the result is in device memory).  Errors: EINVAL, ENOMEM,
 * EUNSUPPORTED (weighted degrees or vol of 2^32 or more), EHIP. */
lne_status lne_sparsify_log(lne_ctx *ctx, const lne_graph *g, const lne_params *p,
                            lne_csr *out, lne_stats *st);

/* Copies a library CSR into caller device buffers (row_ptr: n_rows + 1,
 * col: nnz, val: nnz elements of val_type).  Errors: EINVAL. */
lne_status lne_csr_copy(lne_ctx *ctx, const lne_csr *m, int64_t *row_ptr,
                        int32_t *col, void *val);
void lne_csr_free(lne_ctx *ctx, lne_csr *m);

/* ---- linear algebra -------------------------------------------------------- */

/* Y = A X for a library CSR A (values F64 or F32) and a dense X of width k.
 * dtype is the element type of X and Y: F64 needs F64 values; F32 or BF16
 * need F32 values (BF16 operands are accumulated in FP32).
 * Errors: EINVAL. */
lne_status lne_spmm(lne_ctx *ctx, const lne_csr *A, const void *X, int64_t ldx,
                    void *Y, int64_t ldy, int32_t k, int32_t dtype);

/* eigSVD (Algorithm "eigSVD") of a dense Y (n x k, dtype): C = Y^T Y in FP64
 * (BF16 inputs: FP32 accumulation), C = V D V^T in FP64 on the device
 * (Householder tridiagonalization; the tridiagonal matrix torn in two halves
 * solved by implicit QL sweeps with Wilkinson's shift and merged through the
 * secular equation; the reflectors applied to the eigenvectors), S = sqrt(D) sorted descending, U = Y V S^-1 (columns with
 * S <= k eps S_1 are zero).  U: device n x k (ldu, dtype; BF16 input gives F32
 * U), S: device k doubles, V: device k x k doubles.  Any output may be NULL.
 * Errors: EINVAL, ENOMEM, EUNSUPPORTED (k > 288). */
lne_status lne_eigsvd(lne_ctx *ctx, const void *Y, int64_t n, int32_t k, int64_t ld,
                      int32_t dtype, void *U, int64_t ldu, double *S, double *V);

/* ---- graph descriptors ---------------------------------------------------- */

/* The eight descriptors of a graph that the hyperparameter search's surrogate
 * reads next to the trial's parameters (section 4.4 searches trials per
 * graph; the choice of descriptors is this library's): out[0] log n, out[1]
 * log max(m, 1), out[2] log of the mean degree, out[3] the degree coefficient
 * of variation (population standard deviation over mean), out[4] log of the
 * maximum degree, out[5] the Hill tail exponent 1 + |T| / sum_{d in T}
 * log(d / (x_min - 1/2)) with x_min = max(1, median degree) and T the degrees
 * >= x_min, out[6] the fraction of closed wedges among `wedges` sampled ones,
 * out[7] the spectral gap 1 - lambda_2 of D^-1/2 A D^-1/2.  Wedge t draws the
 * Philox block of counter (t_lo, t_hi, 0, 6 << 24) under key seed, words z0..z3:
 * its centre is candidate ((z1 << 32) | z0) mod C of the C vertices of degree
 * >= 2 in increasing order, its ends the neighbours at positions z2 mod d and
 * z3 mod (d - 1), the second moved past the first when not smaller.
 * lambda_2 = 2 S_2 - 1 after `iters` steps X <- U of [U, S] = eigSVD((X + D^-1/2
 * A D^-1/2 X) / 2), from X = the lne_gaussian block of n x min(16, n) under
 * key seed (isolated vertices: zero rows of D^-1/2 A D^-1/2).  g: unweighted,
 * with at least one edge.  out: host, 8 doubles.  Synchronous.
 * Errors: EINVAL (wedges < 1, iters < 1, invalid graph), EUNSUPPORTED
 * (weighted graph), ENOMEM, EHIP. */
lne_status lne_graph_stats(lne_ctx *ctx, const lne_graph *g, uint64_t seed, int32_t wedges,
                           int32_t iters, double *out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): lne_eigsvd
 * with no allocation.  Same arguments, results and errors as lne_eigsvd.
 * Every intermediate (the Gram's per-workgroup partial sums, the Gram, the
 * eigen-solver's working matrix, eigenvectors, eigenvalues and the projection
 * weights) lives in a fixed device array of LNE_EIGSVD_NOALLOC_SCRATCH bytes
 * that the library holds on each device it runs on until the process ends;
 * the call makes no hipMalloc, hipFree or allocator call and records no
 * profiling events.  The Gram uses as many workgroups as the array has room
 * for partial sums (fewer than lne_eigsvd for k > 160 or so), which changes
 * only its summation order.  Calls on one device share the array: calls that
 * overlap in time on one device (other streams, other threads) race; calls
 * ordered on one stream do not.  Errors: EINVAL, EUNSUPPORTED (k > 288), EHIP
 * (the array's device address could not be obtained). */
#define LNE_EIGSVD_NOALLOC_SCRATCH (64u << 20)
lne_status lne_eigsvd_noalloc(lne_ctx *ctx, const void *Y, int64_t n, int32_t k, int64_t ld,
                              int32_t dtype, void *U, int64_t ldu, double *S, double *V);

/* Orthonormal basis of range(Y) by CholeskyQR2 with a shifted first pass on
 * breakdown (Fukaya et al.), in place; the Cholesky factorisations are FP64.
 * This replaces eigSVD as the orthonormaliser of the power iteration: both
 * span range(Y), and the fast randomized SVD depends on the basis only
 * through that span.  Errors: EINVAL, ENOMEM, ENUMERIC. */
lne_status lne_orthonormalize(lne_ctx *ctx, void *Y, int64_t n, int32_t k, int64_t ld,
                              int32_t dtype);

/* Fast randomized SVD (Algorithm "Fast Randomized SVD") of the symmetric
 * sparsifier matrix M (values F64 for precision LNE_F64, F32 otherwise):
 * Omega (lne_gaussian, p->seed) -> Y = M Omega -> orthonormalise -> q times
 * {Y = M Q; T = Q; eigSVD(Y) or orthonormalise} -> U = Q[:, :d],
 * Sigma = S[:d], V = T V[:, :d], X0 = U Sigma^(1/2).
 * Dense n x (d + oversample) matrices are F64 (LNE_F64), F32 (LNE_F32) or
 * BF16 (LNE_BF16: the Gram products and projections run on BF16 MFMA with
 * FP32 accumulation, the Cholesky and the final eigen-solve stay FP64).
 * Outputs (any may be NULL): U, V, X0 device n x d (F64 for LNE_F64, else F32),
 * sigma device d doubles.  Errors: EINVAL, ENOMEM, EHIP, ENUMERIC. */
lne_status lne_rsvd(lne_ctx *ctx, const lne_csr *M, const lne_params *p, void *U,
                    double *sigma, void *V, void *X0);

/* Spectral propagation (section 4.3) on the input graph with L = I - D^-1 A:
 *   X_sp = D^-1 A (X0 - g_k(L) X0),  g_k = sum_{n<=k} c_n T_n((L - mu I)^2/2 - I),
 *   c_0 = e^(-theta/2) I_0(theta), c_n = 2 (-1)^n e^(-theta/2) I_n(theta),
 * the degree-k Chebyshev (Jacobi-Anger) expansion of the band-pass filter
 * exp(-theta/2 ((lambda - mu)^2 - 1)); then X = U_p S_p^(1/2) from eigSVD(X_sp)
 * unless LNE_FLAG_NO_FINAL_EIGSVD.  With k = 0 or theta < 1e-12 X = X0.
 * X0, X: device n x d, F64 if p->precision == LNE_F64 else F32.
 * Errors: EINVAL, ENOMEM, EHIP. */
lne_status lne_propagate(lne_ctx *ctx, const lne_graph *g, const lne_params *p,
                         const void *X0, void *X);

/* One product of the Chebyshev recurrence of lne_propagate (section 4.3):
 *   out = a Z + b D^-1 A Z
 * on the input graph (weighted: D^-1 A with the arc weights).  Z, out: device
 * n x k, row-major with leading dimension ld (elements), F64 or F32 (dtype),
 * 16-byte aligned, ld a multiple of the 16-byte vector (2 doubles, 4 floats);
 * out must not alias Z.  The launch shape is the one lne_propagate uses
 * (timed on the first call of a shape).  Errors: EINVAL (also a malformed
 * graph, found by a device check that synchronises the stream). */
lne_status lne_graph_spmm(lne_ctx *ctx, const lne_graph *g, const void *Z, int64_t ld,
                          int32_t k, int32_t dtype, double a, double b, void *out);

/* Whole path: sparsify -> trunc_log -> rSVD -> propagate.  X: device n x d
 * (F64 for LNE_F64, else F32).  Synchronises the stream (sizes).  st may be
 * NULL.  Errors: those of the stages. */
lne_status lne_embed(lne_ctx *ctx, const lne_graph *g, const lne_params *p, void *X,
                     lne_stats *st);

/* ---- batched trials sharing one sampling pass ------------------------------- */
/* One trial of the search space of section 4.4 (s_1..s_T of Eq. (1) and the
 * propagation parameters); M, q, d and the rest come from the base params. */
typedef struct {
    double s[16];       /* s_1..s_T >= 0, positive sum (normalised inside)    */
    int32_t cheb_k;     /* propagation order; 0 switches propagation off      */
    double theta, mu;   /* filter parameters; theta < 1e-12 switches it off   */
} lne_trial;

/* Sparsifier with per-length channels: lne_sparsify with the sampled length
 * r kept (p->s plays the role of the channel pass's length distribution pi):
 * the count CSR has n x 16n columns, column (b << 4) | (r - 1) holding the
 * weight of pairs (a, b) sampled at length r.  Synchronises the stream.
 * Errors: as lne_sparsify; EUNSUPPORTED if n > 2^30. */
lne_status lne_sparsify_channels(lne_ctx *ctx, const lne_graph *g, const lne_params *p,
                                 lne_csr *out, lne_stats *st);

/* Sparsifier matrix of one trial from the channel counts of a pass with
 * length distribution pi = p->s (normalised): the trial's weights are
 * sum_r (s_r / pi_r) W_r (an unbiased estimate of its own sampler's counts)
 * and the entries are ln x for x > 1 of Eq. (1), 0 for x <= 1 (the structure
 * is the union over lengths; zeros are kept).  out: F32 values.  Synchronises
 * the stream.  Errors: EINVAL (also when s_r > 0 where pi_r = 0), ENOMEM. */
lne_status lne_trial_matrix(lne_ctx *ctx, const lne_graph *g, const lne_params *p,
                            const lne_csr *channels, const lne_trial *trial, lne_csr *out);

/* A batch: the state that every trial on one graph shares.  Creating it runs
 * the channel sampling pass once (as lne_sparsify_channels), draws the
 * Gaussian test matrix of Algorithm "Fast Randomized SVD" (the same matrix
 * the single-trial path draws from p->seed) and allocates a trial-major FP32
 * workspace for max_trials trials (about (2 k'' + 7 d'') n 4 bytes per trial,
 * k'' and d'' = d + oversample and d rounded up to 8, plus the channel CSR).
 * It also picks the launch shapes of the batched SpMM kernels by timing each
 * shape on this matrix (with env LNE_TUNE_CACHE naming a JSON-lines file, the
 * choice is read from / appended to it).  The graph's device arrays must stay
 * valid until lne_batch_destroy.  p->s is the length distribution pi of the
 * channel pass (each trial brings its own s; a trial needs pi_r > 0 wherever
 * its s_r > 0, and its estimate has the least variance when pi is close to
 * its s); p->precision must be LNE_F32 and d + oversample <= 256.
 * Synchronises the stream.  st (may be NULL): attempted, accepted, nnz_counts
 * of the channel pass.  Errors: those of lne_sparsify_channels, EINVAL,
 * ENOMEM, EUNSUPPORTED (max_trials outside 1..256). */
typedef struct lne_batch lne_batch;
lne_status lne_batch_create(lne_ctx *ctx, const lne_graph *g, const lne_params *p,
                            int32_t max_trials, lne_batch **out, lne_stats *st);

/* Runs the channel sampling pass again with length distribution pi (T
 * doubles, normalised inside) in place of the batch's current one; the
 * workspace, tuned launch shapes and scratch arena are kept, a captured
 * graph is dropped.  Synchronises the stream.  st (may be NULL): as
 * lne_batch_create.  Errors: those of lne_batch_create. */
lne_status lne_batch_resample(lne_batch *b, const double *pi, lne_stats *st);

#define LNE_BATCH_EAGER 0   /* enqueue the launches of the run one by one          */
#define LNE_BATCH_GRAPH 1   /* replay them as one captured HIP graph               */
/* Embeddings of n_trials <= max_trials trials.  For every trial t, M_t (the
 * lne_trial_matrix of trial t) is regenerated on the fly inside each SpMM
 * from the channel CSR; the fast randomized SVD (CholeskyQR2 and eigSVD in
 * FP64 on MFMA, one launch per step for all trials), Chebyshev propagation
 * (one graph SpMM per recurrence step for all trials, per-trial k, theta, mu)
 * and the final eigSVD follow the single-trial path.  X: device n_trials x n x
 * d FP32 (trial-major).  The first run, and the first with more trials than
 * any run before, runs eagerly to size the scratch arena of the dense steps;
 * in mode LNE_BATCH_GRAPH later runs capture the launch sequence once per
 * (n_trials, largest k) and replay it.  Synchronises the stream.  st (may be
 * NULL): shifted Cholesky count, nnz_counts.  Errors: EINVAL, ENOMEM, EHIP,
 * ENUMERIC. */
lne_status lne_batch_run(lne_batch *b, const lne_trial *trials, int32_t n_trials, int32_t mode,
                         float *X, lne_stats *st);
/* Stage entry of the batched SpMM: Y_t = M_t X_t for t < n_trials with M_t
 * the trial matrix of trials[t] (as lne_trial_matrix), generated on the fly.
 * X_t = X + t xs (xs = 0: one operand for all trials), n x k with rows ldx
 * apart; Y_t = Y + t ys, rows ldy apart.  k % 4 == 0, k <= 256, X, Y,
 * ldx, ldy, xs, ys 16-byte aligned; columns of X beyond k are not read.
 * Synchronises the stream.  Errors: EINVAL. */
lne_status lne_batch_spmm(lne_batch *b, const lne_trial *trials, int32_t n_trials,
                          const float *X, int64_t ldx, int64_t xs, float *Y, int64_t ldy,
                          int64_t ys, int32_t k);
/* Launch shapes chosen by the tuner (0-based variant ids), nnz of the channel
 * CSR and the number of graph captures so far; any pointer may be NULL.
 * Host only.  Errors: EINVAL (b NULL). */
lne_status lne_batch_info(const lne_batch *b, int32_t *spmm_variant, int32_t *gspmm_variant,
                          int64_t *channel_nnz, int32_t *captures);
/* Waits for the context's stream and releases the batch (before the context
 * it was created on is destroyed). */
void lne_batch_destroy(lne_batch *b);

/* One-shot batch: lne_batch_create, one eager lne_batch_run, lne_batch_destroy.
 * st: attempted and accepted of the sampling pass, nnz_counts, shifted.
 * Errors: those of the two calls; EUNSUPPORTED (n_trials outside 1..256). */
lne_status lne_embed_batch(lne_ctx *ctx, const lne_graph *g, const lne_params *p,
                           const lne_trial *trials, int32_t n_trials, float *X, lne_stats *st);

/* ---- hyperparameter search: surrogate network and downstream scorer ------ */
/* Section 4.4 searches s_r, M, q, k, theta and mu against the downstream
 * score.  The surrogate is an MLP in_dim -> hidden -> hidden -> 1 with GELU
 * activations in FP32 that learns (hyperparameters, graph statistics) ->
 * score from trials of the plain method and ranks candidate trials; the plain
 * method (lne_embed + lne_score_micro_f1) scores every proposal.
 * Parameters are one flat FP32 device array: W1 (in_dim x hidden, row-major),
 * b1 (hidden), W2 (hidden x hidden), b2 (hidden), W3 (hidden), b3 (1). */

/* Number of parameters; 0 on invalid dimensions.  Host only. */
int64_t lne_mlp_param_count(int32_t in_dim, int32_t hidden);

/* Glorot-uniform weights (Philox words, key = seed), zero biases.
 * Errors: EINVAL. */
lne_status lne_mlp_init(lne_ctx *ctx, int32_t in_dim, int32_t hidden, uint64_t seed,
                        float *params);

/* y (batch) = MLP(X), X: device batch x in_dim row-major.  Errors: EINVAL, ENOMEM. */
lne_status lne_mlp_forward(lne_ctx *ctx, int32_t in_dim, int32_t hidden, const float *params,
                           const float *X, int64_t batch, float *y);

/* Gradient of the mean squared error mean_b (MLP(X)_b - target_b)^2 with
 * respect to every parameter (grad: device, same layout as params); loss:
 * device scalar or NULL.  Errors: EINVAL, ENOMEM. */
lne_status lne_mlp_grad(lne_ctx *ctx, int32_t in_dim, int32_t hidden, const float *params,
                        const float *X, const float *target, int64_t batch, float *grad,
                        float *loss);

/* One Adam step (Kingma & Ba) on count parameters with bias correction for
 * step >= 1: m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
 * p -= lr (m / (1-b1^step)) / (sqrt(v / (1-b2^step)) + eps).  Errors: EINVAL. */
lne_status lne_mlp_adam(lne_ctx *ctx, int64_t count, float *params, const float *grad, float *m,
                        float *v, int64_t step, float lr, float beta1, float beta2, float eps);

/* Downstream score of an embedding (the node-classification protocol of the
 * evaluation section): one-vs-rest L2-regularised logistic regression on the
 * standardised rows X[train] (full-batch Adam, `epochs` steps, rate lr, L2
 * weight l2), then each test vertex predicts its top-k labels with k its true
 * label count; *f1 (host) = micro-F1 over the test vertices.
 * X: device n x d FP32; labels: device n x n_labels uint8 (0/1); train, test:
 * device int32 row indices.  Synchronises the stream.  Errors: EINVAL, ENOMEM. */
lne_status lne_score_micro_f1(lne_ctx *ctx, const float *X, int64_t n, int32_t d,
                              const uint8_t *labels, int32_t n_labels, const int32_t *train,
                              int64_t n_train, const int32_t *test, int64_t n_test,
                              int32_t epochs, float lr, float l2, double *f1);
/* The same protocol for n_trials embeddings at once (X: device n_trials x n x
 * d, trial-major; same labels and split): every epoch is one launch sequence
 * over all trials.  f1: host array of n_trials.  Errors: as above. */
lne_status lne_score_micro_f1_batch(lne_ctx *ctx, const float *X, int32_t n_trials, int64_t n,
                                    int32_t d, const uint8_t *labels, int32_t n_labels,
                                    const int32_t *train, int64_t n_train, const int32_t *test,
                                    int64_t n_test, int32_t epochs, float lr, float l2,
                                    double *f1);

/* Link-prediction evaluation (the protocol of the very-large-graph runs in
 * the experiments section): each held-out edge i = (pos[2i], pos[2i+1]) =
 * (u, v) is ranked against its K corrupted edges (u, neg[i K + j]) by the
 * inner product of embedding rows, accumulated in FP64.  above[i] = number of
 * corrupted edges scoring strictly above (u, v), ties[i] = number scoring
 * equal; rank = 1 + above.  metrics (device, 4 doubles) = mean rank, mean
 * reciprocal rank, HITS@hits_k (share of ranks <= hits_k) and AUC (mean of
 * (K - above - ties / 2) / K).  X: device n x d rows (ldx, F32 or F64,
 * 16-byte aligned); pos: device h x 2 int32; neg: device h x K int32; above,
 * ties: device h uint32 each, or NULL.  Vertex ids outside [0, n) are not
 * read: EINVAL after the launch.  Synchronises the stream.
 * Errors: EINVAL, ENOMEM. */
lne_status lne_link_rank(lne_ctx *ctx, const void *X, int64_t n, int32_t d, int64_t ldx,
                         int32_t dtype, const int32_t *pos, int64_t h, const int32_t *neg,
                         int32_t K, int32_t hits_k, uint32_t *above, uint32_t *ties,
                         double *metrics);

#ifdef __cplusplus
}
#endif
#endif /* LNE_H */
