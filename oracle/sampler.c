/*
 * ORACLE -- test infrastructure only.  Plain, slow, single-purpose C that the
 * tests, the smoke check and the CPU baseline leg of the benchmark call to
 * decide what the GPU path must produce.  It shares no code with the GPU
 * library and must never be linked into it.
 *
 * What it computes (paper section 3, "NetMF" and "NetSMF"; section 4.1; section
 * 5.2, Algorithm "Downsampled Per-Edge PathSampling" and Algorithm
 * "PathSampling"; Eq. (1)):
 *
 * The sparsifier is a sum of path samples drawn edge by edge.  Each undirected
 * edge (u < v, numbered in CSR order) receives M/m samples on average: the
 * integer part always, the fractional part as one extra sample with that
 * probability.  A sample survives a degree-based coin whose success
 * probability p_e is C (1/d_u + 1/d_v) capped at one (section 4.1), and picks
 * a path length r from the normalised weights s.  A surviving sample places
 * the edge at a uniformly chosen position of a length-r path, extends the
 * path by uniform random-walk steps on both sides, and contributes the
 * inverse of its survival probability to the pair of path endpoints, in both
 * orientations.  Equal endpoint pairs are summed into counts W_ab, which Eq.
 * (1) turns into x_ab = vol 2m/(2 b M) W_ab/(d_a d_b) (vol = 2m without
 * weights); the matrix keeps ln x_ab wherever x_ab exceeds one.
 *
 * Weighted graphs (positive integer weights A_uv, symmetric): d_u = sum_v
 * A_uv, vol = sum_u d_u, p_e = min(1, C A_uv (1/d_u + 1/d_v)) (section 5.2,
 * degree sampling with A_uv), a walk step from x takes neighbour y with
 * probability A_xy / d_x, and a sample's weight is h / p_e with
 * h = r / sum_j (1 / A_j) over the r edges of its path (the centre edge, then
 * the steps from u, then the steps from v): NetSMF's path estimator for
 * weighted graphs, which is 1 for every path of an unweighted graph.  With
 * edges still drawn uniformly, E[W] = 2^F (M/m) sum_r s_r A (D^-1 A)^(r-1),
 * so Eq. (1)'s vol/b sum_r s_r (D^-1 A)^r D^-1 is vol m/(b M) W/(2^F d_a d_b).
 *
 * Readings of points the paper leaves open (each is restated in the design
 * notes):
 *   - randomness: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
 *     numbers: as easy as 1, 2, 3", SC'11) with key = seed and a counter that
 *     names the edge, the sample slot and a 4-word block;
 *   - every random decision is an integer comparison on a 32-bit word;
 *   - weights are fixed point with F = 16 fractional bits: w_e = rint(2^F/p_e);
 *   - each sample is added in both orientations so the sparsifier is exactly
 *     symmetric (a diagonal pair therefore receives 2 w_e);
 *   - the log is natural, the truncation keeps x > 1 strictly, and the keep
 *     decision is taken exactly in 128-bit integers.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORA_F 16
#define ORA_TAG_NE (1u << 24)
#define ORA_TAG_WALK (2u << 24)

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 as defined by Salmon et al. (SC'11): ten rounds of          */
/*   (c0,c1,c2,c3) -> (hi(R1*c2) ^ c1 ^ k0, lo(R1*c2), hi(R0*c0) ^ c3 ^ k1,   */
/*                     lo(R0*c0))                                            */
/* with the key bumped by the Weyl constants between rounds.                 */
/* ------------------------------------------------------------------------ */
static void philox(const uint32_t in[4], uint32_t k0, uint32_t k1, uint32_t out[4])
{
    const uint32_t R0 = 0xD2511F53u, R1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = in[0], c1 = in[1], c2 = in[2], c3 = in[3];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)R0 * c0;
        uint64_t p1 = (uint64_t)R1 * c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += W0; k1 += W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

void ora_philox(uint64_t seed, const uint32_t *ctr, int64_t count, uint32_t *out)
{
    for (int64_t i = 0; i < count; ++i)
        philox(ctr + 4 * i, (uint32_t)seed, (uint32_t)(seed >> 32), out + 4 * i);
}

/* ------------------------------------------------------------------------ */
/* Constants of the sampler that depend only on the hyperparameters.         */
/* ------------------------------------------------------------------------ */
typedef struct {
    uint64_t base;          /* floor(M / m) */
    uint64_t frac_thr;      /* floor(frac(M/m) * 2^32): Bernoulli(frac) iff word < frac_thr */
    uint64_t theta[16];     /* r = min{t : z < theta[t-1]}, theta[T-1] = 2^32 */
    int T;
} plan_t;

static void make_plan(int T, const double *s, uint64_t M, int64_t m, plan_t *pl)
{
    pl->T = T;
    /* a graph without edges has no sample slots */
    pl->base = m > 0 ? (uint64_t)(M / (uint64_t)m) : 0;
    uint64_t rem = m > 0 ? M % (uint64_t)m : 0;
    /* frac(M/m) * 2^32 floored, exactly, in integers */
    pl->frac_thr = m > 0 ? (uint64_t)(((unsigned __int128)rem << 32) / (uint64_t)m) : 0;
    double total = 0.0;
    for (int t = 0; t < T; ++t) total += s[t];
    double cum = 0.0;
    for (int t = 0; t < T; ++t) {
        cum += s[t];
        pl->theta[t] = (uint64_t)floor(cum / total * 4294967296.0);
        if (pl->theta[t] > 4294967296ull) pl->theta[t] = 4294967296ull;
    }
    pl->theta[T - 1] = 4294967296ull;
}

void ora_plan(int T, const double *s, uint64_t M, int64_t m, uint64_t *out_base,
              uint64_t *out_frac_thr, uint64_t *out_theta)
{
    plan_t pl;
    make_plan(T, s, M, m, &pl);
    *out_base = pl.base;
    *out_frac_thr = pl.frac_thr;
    for (int t = 0; t < T; ++t) out_theta[t] = pl.theta[t];
}

/* Degree-sampling probability p_e = C A_uv (1/d_u + 1/d_v) and its coin
 * threshold (section 4.1, 5.2).  no_ds != 0 switches downsampling off
 * (p_e = 1); so does p_e >= 1 (*all = 1). */
static void edge_coin(double C, int no_ds, uint32_t A, uint64_t du, uint64_t dv, int *all,
                      uint64_t *tau, double *p_out)
{
    *p_out = 1.0;
    if (no_ds) { *all = 1; *tau = 0; return; }
    double p = (C * (double)A) * (1.0 / (double)du + 1.0 / (double)dv);
    if (p >= 1.0) { *all = 1; *tau = 0; return; }
    *all = 0;
    *tau = (uint64_t)floor(p * 4294967296.0);
    *p_out = p;
}

/* Fixed-point weight of an accepted sample: rint(2^F h / p_e), h the path
 * factor (1 on unweighted graphs). */
static uint64_t sample_weight(double h, int all, double p)
{
    if (all) return (uint64_t)rint(65536.0 * h);
    return (uint64_t)rint(65536.0 * h / p);
}

typedef struct {
    int64_t n;
    const int64_t *rowptr;
    const int32_t *col;
    const uint32_t *wt;      /* arc weights, NULL: every weight 1 */
    const uint64_t *cw;      /* cw[k] = sum of wt[0..k) (weighted graphs) */
} graph_t;

static uint64_t degree(const graph_t *g, int64_t u)
{
    if (!g->wt) return (uint64_t)(g->rowptr[u + 1] - g->rowptr[u]);
    return g->cw[g->rowptr[u + 1]] - g->cw[g->rowptr[u]];
}

/* cw of a weighted graph; 0 on success, -4 if a weight is 0 or a weighted
 * degree reaches 2^32 (walk steps draw from 32-bit words). */
static int weight_prefix(const graph_t *g, uint64_t **out)
{
    *out = NULL;
    if (!g->wt) return 0;
    int64_t na = g->rowptr[g->n];
    uint64_t *cw = malloc(sizeof(uint64_t) * (size_t)(na + 1));
    if (!cw) return -1;
    cw[0] = 0;
    for (int64_t k = 0; k < na; ++k) {
        if (g->wt[k] == 0) { free(cw); return -4; }
        cw[k + 1] = cw[k] + g->wt[k];
    }
    for (int64_t u = 0; u < g->n; ++u)
        if (cw[g->rowptr[u + 1]] - cw[g->rowptr[u]] >= (1ull << 32)) { free(cw); return -4; }
    *out = cw;
    return 0;
}

/* Word stream of one sample slot: words z_0, z_1, ... come four at a time from
 * Philox(counter = (e_lo, e_hi, j, TAG_WALK | block)). */
typedef struct {
    uint32_t ctr[4];
    uint32_t buf[4];
    int used;
    uint32_t k0, k1;
} stream_t;

static void stream_init(stream_t *st, uint64_t seed, int64_t e, uint32_t j)
{
    st->ctr[0] = (uint32_t)e;
    st->ctr[1] = (uint32_t)((uint64_t)e >> 32);
    st->ctr[2] = j;
    st->ctr[3] = ORA_TAG_WALK;
    st->k0 = (uint32_t)seed;
    st->k1 = (uint32_t)(seed >> 32);
    st->used = 4;
}

static uint32_t stream_next(stream_t *st)
{
    if (st->used == 4) {
        philox(st->ctr, st->k0, st->k1, st->buf);
        st->ctr[3] += 1;
        st->used = 0;
    }
    return st->buf[st->used++];
}

static uint64_t draw_ne(uint64_t seed, int64_t e, const plan_t *pl)
{
    uint32_t c[4] = {(uint32_t)e, (uint32_t)((uint64_t)e >> 32), 0xFFFFFFFFu, ORA_TAG_NE};
    uint32_t o[4];
    philox(c, (uint32_t)seed, (uint32_t)(seed >> 32), o);
    return pl->base + ((uint64_t)o[0] < pl->frac_thr ? 1 : 0);
}

/* One step of a random walk: the next vertex is neighbour (z mod deg) of x;
 * on a weighted graph t = z mod d_x selects the neighbour whose slice of the
 * cumulative weights [sum of earlier weights, + A_xy) holds t.  *A = the
 * weight of the arc taken. */
static int32_t walk_step(const graph_t *g, int32_t x, uint32_t z, uint32_t *A)
{
    int64_t beg = g->rowptr[x];
    if (!g->wt) {
        int64_t deg = g->rowptr[x + 1] - beg;
        *A = 1;
        return g->col[beg + (int64_t)((uint64_t)z % (uint64_t)deg)];
    }
    uint64_t t = (uint64_t)z % degree(g, x);
    int64_t k = beg;
    while (g->cw[k + 1] - g->cw[beg] <= t) ++k;     /* first slice ending above t */
    *A = g->wt[k];
    return g->col[k];
}

/* One sample slot of edge e (weight A_uv): returns 1 if accepted and fills
 * (a, b, r) and the path factor h = r / sum_j (1 / A_j). */
static int sample_slot(const graph_t *g, const plan_t *pl, uint64_t seed, int64_t e,
                       int32_t u, int32_t v, uint32_t Auv, uint32_t j, int all, uint64_t tau,
                       int32_t *a, int32_t *b, int *r_out, double *h_out)
{
    stream_t st;
    stream_init(&st, seed, e, j);
    uint32_t z0 = stream_next(&st);   /* coin: p ~ U[0,1] (Downsampled Per-Edge PathSampling) */
    uint32_t z1 = stream_next(&st);   /* length: r ~ Multinomial(s) (same algorithm)          */
    if (!(all || (uint64_t)z0 < tau)) return 0;
    int r = 1;
    while ((uint64_t)z1 >= pl->theta[r - 1]) ++r;
    uint32_t z2 = stream_next(&st);   /* split: uniform in 0..r-1 (PathSampling)              */
    int split = (int)(z2 % (uint32_t)r);
    double inv = 1.0 / (double)Auv;
    uint32_t A;
    int32_t x = u;
    for (int i = 0; i < split; ++i) {
        x = walk_step(g, x, stream_next(&st), &A);
        inv += 1.0 / (double)A;
    }
    int32_t y = v;
    for (int i = 0; i < r - 1 - split; ++i) {
        y = walk_step(g, y, stream_next(&st), &A);
        inv += 1.0 / (double)A;
    }
    *a = x; *b = y; *r_out = r;
    *h_out = (double)r / inv;
    return 1;
}

/* Edge list: the arcs (u, v) with u < v, in CSR order; e is the position;
 * ea = the arc's weight. */
static int64_t edge_list(const graph_t *g, int32_t *eu, int32_t *ev, uint32_t *ea)
{
    int64_t e = 0;
    for (int64_t u = 0; u < g->n; ++u)
        for (int64_t k = g->rowptr[u]; k < g->rowptr[u + 1]; ++k)
            if (g->col[k] > u) {
                if (eu) {
                    eu[e] = (int32_t)u;
                    ev[e] = g->col[k];
                    ea[e] = g->wt ? g->wt[k] : 1u;
                }
                ++e;
            }
    return e;
}

/*
 * Every sample slot (e, j), j < n_e, of the edges e in [e_begin, e_end).
 * Per slot: edge id, slot j, accepted flag, r, (u', v'), weight.
 * Returns the number of slots, or -(needed) if cap is too small.
 */
int64_t ora_sample_slots(int64_t n, const int64_t *rowptr, const int32_t *col,
                         const uint32_t *wt, int T, const double *s, uint64_t M, double C,
                         int no_ds, uint64_t seed, int64_t e_begin, int64_t e_end, int64_t cap,
                         int64_t *o_e, uint32_t *o_j, uint8_t *o_acc, uint8_t *o_r,
                         int32_t *o_a, int32_t *o_b, uint64_t *o_w)
{
    graph_t g = {n, rowptr, col, wt, NULL};
    uint64_t *cw;
    int rc = weight_prefix(&g, &cw);
    if (rc) return INT64_MIN;
    g.cw = cw;
    int64_t m = edge_list(&g, NULL, NULL, NULL);
    int32_t *eu = malloc(sizeof(int32_t) * (size_t)(m ? m : 1));
    int32_t *ev = malloc(sizeof(int32_t) * (size_t)(m ? m : 1));
    uint32_t *ea = malloc(sizeof(uint32_t) * (size_t)(m ? m : 1));
    edge_list(&g, eu, ev, ea);
    plan_t pl;
    make_plan(T, s, M, m, &pl);
    int64_t k = 0;
    for (int64_t e = e_begin; e < e_end && e < m; ++e) {
        int32_t u = eu[e], v = ev[e];
        int all; uint64_t tau; double p;
        edge_coin(C, no_ds, ea[e], degree(&g, u), degree(&g, v), &all, &tau, &p);
        uint64_t ne = draw_ne(seed, e, &pl);
        for (uint64_t j = 0; j < ne; ++j) {
            int32_t a = -1, b = -1; int r = 0; double h = 0.0;
            int acc = sample_slot(&g, &pl, seed, e, u, v, ea[e], (uint32_t)j, all, tau, &a, &b,
                                  &r, &h);
            if (k < cap) {
                o_e[k] = e; o_j[k] = (uint32_t)j; o_acc[k] = (uint8_t)acc;
                o_r[k] = (uint8_t)r; o_a[k] = a; o_b[k] = b;
                o_w[k] = acc ? sample_weight(h, all, p) : 0;
            }
            ++k;
        }
    }
    free(eu); free(ev); free(ea); free(cw);
    return k <= cap ? k : -k;
}

/* ------------------------------------------------------------------------ */
/* Aggregation: W[a][b] += w and W[b][a] += w per accepted sample, restricted */
/* to rows in [row_lo, row_hi).  Threads split the edge range; the merge is a */
/* sort of (row, col, w) triples followed by summing equal keys.              */
/* ------------------------------------------------------------------------ */
typedef struct { int32_t a, b; uint64_t w; } trip_t;

typedef struct {
    const graph_t *g; const plan_t *pl; uint64_t seed; double C; int no_ds; int channels;
    const int32_t *eu, *ev;
    const uint32_t *ea;
    const int64_t *elist;      /* NULL: edges e0..e1-1; else elist[e0..e1-1] */
    int64_t e0, e1, row_lo, row_hi;
    trip_t *buf; int64_t len, cap;
    uint64_t accepted, attempted;
    int fail;
} job_t;

static void push(job_t *jb, int32_t a, int32_t b, uint64_t w)
{
    if (a < jb->row_lo || a >= jb->row_hi) return;
    if (jb->len == jb->cap) {
        int64_t nc = jb->cap ? jb->cap * 2 : 1 << 16;
        trip_t *nb = realloc(jb->buf, sizeof(trip_t) * (size_t)nc);
        if (!nb) { jb->fail = 1; return; }
        jb->buf = nb; jb->cap = nc;
    }
    jb->buf[jb->len].a = a; jb->buf[jb->len].b = b; jb->buf[jb->len].w = w;
    jb->len++;
}

static void *job_run(void *arg)
{
    job_t *jb = arg;
    const graph_t *g = jb->g;
    for (int64_t l = jb->e0; l < jb->e1 && !jb->fail; ++l) {
        const int64_t e = jb->elist ? jb->elist[l] : l;
        int32_t u = jb->eu[e], v = jb->ev[e];
        int all; uint64_t tau; double p;
        edge_coin(jb->C, jb->no_ds, jb->ea[e], degree(g, u), degree(g, v), &all, &tau, &p);
        uint64_t ne = draw_ne(jb->seed, e, jb->pl);
        jb->attempted += ne;
        for (uint64_t j = 0; j < ne; ++j) {
            int32_t a, b; int r; double h;
            if (!sample_slot(g, jb->pl, jb->seed, e, u, v, jb->ea[e], (uint32_t)j, all, tau, &a,
                             &b, &r, &h))
                continue;
            jb->accepted++;
            const uint64_t w = sample_weight(h, all, p);
            if (jb->channels) {
                /* per-length channels: column (b << 4) | (r - 1) */
                push(jb, a, (int32_t)(((uint32_t)b << 4) | (uint32_t)(r - 1)), w);
                push(jb, b, (int32_t)(((uint32_t)a << 4) | (uint32_t)(r - 1)), w);
            } else {
                push(jb, a, b, w);
                push(jb, b, a, w);
            }
        }
    }
    return NULL;
}

static int trip_cmp(const void *x, const void *y)
{
    const trip_t *p = x, *q = y;
    if (p->a != q->a) return p->a < q->a ? -1 : 1;
    if (p->b != q->b) return p->b < q->b ? -1 : 1;
    return 0;
}

/* Shared body of ora_count_rows and ora_count_rows_list (below). */
static int count_rows_impl(int64_t n, const int64_t *rowptr, const int32_t *col,
                           const uint32_t *wt, int T,
                           const double *s, uint64_t M, double C, int no_ds, uint64_t seed,
                           int64_t row_lo, int64_t row_hi, int64_t e_begin, int64_t e_end,
                           const int64_t *elist, int64_t n_list, int channels, int nthreads,
                           int64_t **o_rowptr, int32_t **o_col, uint64_t **o_w, int64_t *o_nnz,
                           uint64_t *o_attempted, uint64_t *o_accepted)
{
    graph_t g = {n, rowptr, col, wt, NULL};
    uint64_t *cw;
    int wrc = weight_prefix(&g, &cw);
    if (wrc) return wrc;
    g.cw = cw;
    int64_t m = edge_list(&g, NULL, NULL, NULL);
    int32_t *eu = malloc(sizeof(int32_t) * (size_t)(m ? m : 1));
    int32_t *ev = malloc(sizeof(int32_t) * (size_t)(m ? m : 1));
    uint32_t *ea = malloc(sizeof(uint32_t) * (size_t)(m ? m : 1));
    if (!eu || !ev || !ea) { free(eu); free(ev); free(ea); free(cw); return -1; }
    edge_list(&g, eu, ev, ea);
    plan_t pl;
    make_plan(T, s, M, m, &pl);
    if (nthreads < 1) nthreads = 1;
    if (e_end < 0 || e_end > m) e_end = m;
    if (e_begin < 0) e_begin = 0;
    if (e_begin > e_end) e_begin = e_end;
    if (elist) {
        for (int64_t l = 0; l < n_list; ++l)
            if (elist[l] < 0 || elist[l] >= m) { free(eu); free(ev); free(ea); free(cw); return -3; }
        e_begin = 0;
        e_end = n_list;
    }
    job_t *jobs = calloc((size_t)nthreads, sizeof(job_t));
    pthread_t *th = calloc((size_t)nthreads, sizeof(pthread_t));
    for (int t = 0; t < nthreads; ++t) {
        job_t *jb = &jobs[t];
        jb->g = &g; jb->pl = &pl; jb->seed = seed; jb->C = C; jb->no_ds = no_ds;
        jb->channels = channels;
        jb->eu = eu; jb->ev = ev; jb->ea = ea;
        jb->elist = elist;
        jb->e0 = e_begin + (e_end - e_begin) * t / nthreads;
        jb->e1 = e_begin + (e_end - e_begin) * (t + 1) / nthreads;
        jb->row_lo = row_lo; jb->row_hi = row_hi;
        pthread_create(&th[t], NULL, job_run, jb);
    }
    int64_t total = 0;
    int fail = 0;
    uint64_t att = 0, acc = 0;
    for (int t = 0; t < nthreads; ++t) {
        pthread_join(th[t], NULL);
        total += jobs[t].len;
        fail |= jobs[t].fail;
        att += jobs[t].attempted;
        acc += jobs[t].accepted;
    }
    free(th); free(eu); free(ev); free(ea); free(cw);
    *o_attempted = att; *o_accepted = acc;
    trip_t *all = fail ? NULL : malloc(sizeof(trip_t) * (size_t)(total ? total : 1));
    if (!all) {
        for (int t = 0; t < nthreads; ++t) free(jobs[t].buf);
        free(jobs);
        return -1;
    }
    int64_t off = 0;
    for (int t = 0; t < nthreads; ++t) {
        if (jobs[t].len) memcpy(all + off, jobs[t].buf, sizeof(trip_t) * (size_t)jobs[t].len);
        off += jobs[t].len;
        free(jobs[t].buf);
    }
    free(jobs);
    qsort(all, (size_t)total, sizeof(trip_t), trip_cmp);
    int64_t rows = row_hi - row_lo;
    int64_t *rp = calloc((size_t)rows + 1, sizeof(int64_t));
    int32_t *cc = malloc(sizeof(int32_t) * (size_t)(total ? total : 1));
    uint64_t *ww = malloc(sizeof(uint64_t) * (size_t)(total ? total : 1));
    if (!rp || !cc || !ww) { free(all); free(rp); free(cc); free(ww); return -1; }
    int64_t nnz = 0;
    int rc = 0;
    for (int64_t i = 0; i < total; ++i) {
        if (nnz > 0 && all[i].a == all[i - 1].a && all[i].b == all[i - 1].b) {
            uint64_t prev = ww[nnz - 1];
            ww[nnz - 1] = prev + all[i].w;
            if (ww[nnz - 1] < prev) rc = -2;
        } else {
            cc[nnz] = all[i].b;
            ww[nnz] = all[i].w;
            rp[all[i].a - row_lo + 1]++;
            ++nnz;
        }
    }
    for (int64_t r = 0; r < rows; ++r) rp[r + 1] += rp[r];
    free(all);
    *o_rowptr = rp; *o_col = cc; *o_w = ww; *o_nnz = nnz;
    return rc;
}

/*
 * Count CSR of the rows [row_lo, row_hi) from the samples of the edges
 * [e_begin, e_end) (e_end < 0: all edges): *o_rowptr has row_hi-row_lo+1
 * entries starting at 0, *o_col / *o_w have *o_nnz entries.  Buffers are
 * malloc'ed here and released with ora_free.  Also reports the number of
 * attempted and accepted samples of those edges.  With channels != 0 the
 * length r (drawn from s as always) is kept in the column: entry
 * (a, (b << 4) | (r - 1)).  wt: arc weights (NULL: unweighted).  Returns 0,
 * or -1 on allocation failure, -2 on a weight-sum overflow, -4 on a zero
 * weight or a weighted degree of 2^32 or more.
 */
int ora_count_rows(int64_t n, const int64_t *rowptr, const int32_t *col, const uint32_t *wt,
                   int T,
                   const double *s, uint64_t M, double C, int no_ds, uint64_t seed,
                   int64_t row_lo, int64_t row_hi, int64_t e_begin, int64_t e_end, int channels,
                   int nthreads,
                   int64_t **o_rowptr, int32_t **o_col, uint64_t **o_w, int64_t *o_nnz,
                   uint64_t *o_attempted, uint64_t *o_accepted)
{
    return count_rows_impl(n, rowptr, col, wt, T, s, M, C, no_ds, seed, row_lo, row_hi, e_begin,
                           e_end, NULL, 0, channels, nthreads, o_rowptr, o_col, o_w, o_nnz,
                           o_attempted, o_accepted);
}

/* The same from the samples of the listed edges elist[0..n_list) only (edge
 * ids as in the CSR order of u < v arcs; each listed once).  Returns -3 on an
 * id outside [0, m). */
int ora_count_rows_list(int64_t n, const int64_t *rowptr, const int32_t *col,
                        const uint32_t *wt, int T,
                        const double *s, uint64_t M, double C, int no_ds, uint64_t seed,
                        int64_t row_lo, int64_t row_hi, const int64_t *elist, int64_t n_list,
                        int nthreads, int64_t **o_rowptr, int32_t **o_col, uint64_t **o_w,
                        int64_t *o_nnz, uint64_t *o_attempted, uint64_t *o_accepted)
{
    return count_rows_impl(n, rowptr, col, wt, T, s, M, C, no_ds, seed, row_lo, row_hi, 0, -1,
                           elist, n_list, 0, nthreads, o_rowptr, o_col, o_w, o_nnz,
                           o_attempted, o_accepted);
}

void ora_free(void *p) { free(p); }

/* ------------------------------------------------------------------------ */
/* Truncated logarithm of Eq. (1) on the count matrix.                       */
/*   x_ab = vol 2m / (2 b M) * (W_ab / 2^F) / (d_a d_b)                       */
/* (2m = number of arcs; vol = 2m on an unweighted graph, so the factor is    */
/* vol^2 / (2 b M) there).  Keep iff x_ab > 1, decided exactly as             */
/* W_ab vol 2m > 2 b M 2^F d_a d_b in 128-bit unsigned integers; kept value   */
/* = log(x_ab) in double.  rows are [row_lo, row_lo + rows); deg is indexed   */
/* by global vertex id.                                                      */
/* ------------------------------------------------------------------------ */
void ora_trunc_log(int64_t rows, int64_t row_lo, const int64_t *deg,
                   const int64_t *rowptr, const int32_t *col, const uint64_t *w,
                   uint64_t vol, uint64_t arcs, uint64_t b, uint64_t M, uint8_t *keep, double *val)
{
    unsigned __int128 va = (unsigned __int128)vol * arcs;
    unsigned __int128 k = (unsigned __int128)(2 * b * M) << ORA_F;
    double scale = ((double)vol * (double)arcs) / (2.0 * (double)b * (double)M) / 65536.0;
    for (int64_t r = 0; r < rows; ++r) {
        int64_t a = row_lo + r;
        for (int64_t i = rowptr[r]; i < rowptr[r + 1]; ++i) {
            int64_t c = col[i];
            unsigned __int128 lhs = (unsigned __int128)w[i] * va;
            unsigned __int128 rhs = k * (unsigned __int128)((uint64_t)deg[a] * (uint64_t)deg[c]);
            keep[i] = lhs > rhs;
            double x = (double)w[i] * scale / ((double)deg[a] * (double)deg[c]);
            val[i] = keep[i] ? log(x) : 0.0;
        }
    }
}
