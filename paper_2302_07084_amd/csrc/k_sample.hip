// Sparsifier sampling on gfx950: the edge list, the per-edge downsampled
// PathSampling walkers, the Philox and Gaussian generators.
//
// Method (section 5.2 and its two sampling algorithms; degree sampling of
// section 4.1): every undirected edge e = (u, v), u < v, draws
// n_e = floor(M/m) + Bernoulli(frac(M/m)) sample slots; slot j flips a coin of
// probability p_e = min(1, C (1/d_u + 1/d_v)), draws a length r from
// Multinomial(s), a split uniform in {0..r-1}, walks u for split steps and v
// for r-1-split steps, and adds the pair with weight 1/p_e.
//
// GPU design.  One thread owns a chunk of J consecutive slots of one edge, so
// the edge's endpoints, degrees and coin threshold are loaded once per chunk
// and every random decision is an integer compare on a Philox word of a
// counter that names (edge, slot, block): results do not depend on the launch
// shape.  Pairs are emitted in two passes over the same streams: a count pass
// that only flips the coins (one Philox block per slot, no memory traffic
// besides the edge list) and an emit pass that walks and writes each wave's
// accepted pairs contiguously at an offset from the scanned per-wave counts,
// so the pair array is compact and in a fixed order without global atomics.
// Compiled with -ffp-contract=off: the coin thresholds and fixed-point
// weights are IEEE double operations taken one at a time.
//
// Weighted graphs (positive integer weights A): p_e = min(1, C A_uv (1/d_u +
// 1/d_v)) with weighted degrees; a walk step from x takes t = z mod d_x and
// the neighbour whose slice of the row's cumulative weights holds t (binary
// search in the prefix sums cw); an accepted sample weighs h / p_e with
// h = r / sum_j 1/A_j over its path's edges (the centre edge, the steps from
// u, then the steps from v), NetSMF's path estimator, 1 on unweighted graphs.
#include "common.hpp"
#include "philox.hpp"

namespace lne {

namespace {

constexpr int kBlock = 256;
constexpr int kWalkQ = 2;   // slots whose walks one lane advances together (emit pass)

struct Coin {
    bool all;        // p_e >= 1 (or downsampling off): every slot accepted
    uint64_t tau;    // accept iff word < tau
    double p;        // p_e (1 when all)
    uint64_t w;      // fixed-point weight rint(2^16 / p_e) of every sample on
                     // an unweighted graph
};

// Fixed-point weight of an accepted sample with path factor h.
__device__ __forceinline__ uint64_t sample_weight(double h, bool all, double p) {
    return all ? (uint64_t)rint(65536.0 * h) : (uint64_t)rint(65536.0 * h / p);
}

__device__ __forceinline__ Coin edge_coin(const SamplePlan &pl, uint32_t A, uint64_t du,
                                          uint64_t dv) {
    Coin c;
    c.p = 1.0;
    if (pl.no_ds) { c.all = true; c.tau = 0; c.w = sample_weight(1.0, true, 1.0); return c; }
    const double p = (pl.C * (double)A) * (1.0 / (double)du + 1.0 / (double)dv);
    if (p >= 1.0) { c.all = true; c.tau = 0; c.w = sample_weight(1.0, true, 1.0); return c; }
    c.all = false;
    c.tau = (uint64_t)floor(p * 4294967296.0);
    c.p = p;
    c.w = sample_weight(1.0, false, p);
    return c;
}

// degree of x: arcs, or the weight sum of its row
template <bool W>
__device__ __forceinline__ uint64_t vdeg(const SamplePlan &pl, const int64_t *__restrict__ rp,
                                         int64_t x) {
    if constexpr (W) return pl.cw[rp[x + 1]] - pl.cw[rp[x]];
    else return (uint64_t)(rp[x + 1] - rp[x]);
}

template <bool W>
__device__ __forceinline__ Coin coin_of(const SamplePlan &pl, const int64_t *__restrict__ rp,
                                        int64_t e, int32_t u, int32_t v) {
    return edge_coin(pl, W ? pl.ea[e] : 1u, vdeg<W>(pl, rp, u), vdeg<W>(pl, rp, v));
}

__device__ __forceinline__ uint64_t draw_ne(const SamplePlan &pl, int64_t e) {
    const uint4 o = philox4x32_10(
        make_uint4((uint32_t)e, (uint32_t)((uint64_t)e >> 32), 0xFFFFFFFFu, kTagEdgeCount),
        (uint32_t)pl.seed, (uint32_t)(pl.seed >> 32));
    return pl.base + ((uint64_t)o.x < pl.frac_thr ? 1u : 0u);
}

__device__ __forceinline__ uint4 slot_block(const SamplePlan &pl, int64_t e, uint32_t j,
                                            uint32_t blk) {
    return philox4x32_10(
        make_uint4((uint32_t)e, (uint32_t)((uint64_t)e >> 32), j, kTagWalk | blk),
        (uint32_t)pl.seed, (uint32_t)(pl.seed >> 32));
}

// r = min{t : z < theta_t}; theta is nondecreasing so this is one plus the
// number of thresholds at or below z.
__device__ __forceinline__ int draw_r(const SamplePlan &pl, uint32_t z) {
    int r = 1;
#pragma unroll
    for (int t = 0; t < 15; ++t) {
        if (t >= pl.T - 1) break;                   // uniform: T - 1 thresholds
        r += (uint64_t)z >= pl.theta[t] ? 1 : 0;
    }
    return r;
}

// One walk step from x with word z; on a weighted graph inv += 1 / A of the
// arc taken.
template <bool W>
__device__ __forceinline__ int32_t walk_step(const SamplePlan &pl, const int64_t *__restrict__ rp,
                                             const int32_t *__restrict__ col, int32_t x,
                                             uint32_t z, double &inv) {
    const int64_t beg = rp[x], end = rp[x + 1];
    if constexpr (!W) {
        const uint32_t deg = (uint32_t)(end - beg);
        return deg ? col[beg + (int64_t)(z % deg)] : x;   // a sink (asymmetric input) holds
    } else {
        const uint64_t base = pl.cw[beg];
        const uint32_t deg = (uint32_t)(pl.cw[end] - base);   // < 2^32 (validated)
        if (deg == 0) return x;
        const uint64_t t = base + (uint64_t)(z % deg);
        // the arc k of the row with cw[k] <= t < cw[k + 1]: from the guide
        // entry of t's bucket forward
        const uint64_t k = (uint64_t)(end - beg);
        const uint64_t bkt = (t - base) * k / deg;
        int64_t i = beg + (int64_t)min((uint64_t)pl.guide[beg + (int64_t)bkt], k - 1);
        while (i < end - 1 && pl.cw[i + 1] <= t) ++i;
        inv += 1.0 / (double)pl.wt[i];
        return col[i];
    }
}

// Walks of an accepted slot whose first Philox block is `blk0`; *h = the
// path factor r / sum 1/A (weighted graphs; 1 otherwise).
template <bool W>
__device__ __forceinline__ int walk_pair(const SamplePlan &pl, const int64_t *__restrict__ rp,
                                         const int32_t *__restrict__ col, int64_t e,
                                         uint32_t j, uint4 blk0, int32_t u, int32_t v,
                                         int32_t &a, int32_t &b, double *h = nullptr) {
    const int r = draw_r(pl, blk0.y);
    const int split = (int)(blk0.z % (uint32_t)r);
    uint4 buf = make_uint4(blk0.w, 0, 0, 0);
    int left = 1;
    uint32_t blk = 0;
    int32_t x = u, y = v;
    double inv = W ? 1.0 / (double)pl.ea[e] : 0.0;
    // words after the first three: split steps from u, then r-1-split from v
    for (int i = 0; i < r - 1; ++i) {
        if (left == 0) {
            buf = slot_block(pl, e, j, ++blk);
            left = 4;
        }
        const uint32_t z = buf.x;
        buf = make_uint4(buf.y, buf.z, buf.w, 0);
        --left;
        if (i < split) x = walk_step<W>(pl, rp, col, x, z, inv);
        else y = walk_step<W>(pl, rp, col, y, z, inv);
    }
    a = x;
    b = y;
    if (h) *h = W ? (double)r / inv : 1.0;
    return r;
}

// Every accepted length-1 sample of edge e is the pair (u, v) itself with the
// same weight (its path is the edge alone, h = 1 / (1 / A_uv)), so a thread
// merges its chunk's length-1 samples into entries of up to
// r1_group(w) samples each (the sum stays below 2^32); the walks of the
// longer samples are emitted one by one.  Count and emit passes use the same
// rule, so the pair stream is compact and its sums are those of the slots.
template <bool W>
__device__ __forceinline__ uint64_t weight_r1(const SamplePlan &pl, const Coin &cn, int64_t e) {
    if constexpr (!W) return cn.w;
    const double inv = 1.0 / (double)pl.ea[e];
    return sample_weight(1.0 / inv, cn.all, cn.p);
}

__device__ __forceinline__ uint64_t r1_group(uint64_t w) {
    const uint64_t g = w ? 0xFFFFFFFFull / w : 1;
    return g ? g : 1;
}

// Structural check of the input CSR (bit 1: offsets, 2: column range,
// 4: self-loop, 8: unsorted or duplicate column).  A group of 16 lanes walks
// one row's arcs in coalesced strides, so a hub row costs its degree / 16
// steps rather than its degree.
constexpr int kValLanes = 16;

__global__ void k_validate(const int64_t *__restrict__ rp, const int32_t *__restrict__ col,
                           int64_t n, int64_t n_arcs, uint32_t *__restrict__ flags) {
    const int64_t u = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kValLanes;
    const int sub = threadIdx.x % kValLanes;
    if (u >= n) return;
    uint32_t f = 0;
    if (sub == 0 && u == 0 && rp[0] != 0) f |= 1;
    if (sub == 0 && u == n - 1 && rp[n] != n_arcs) f |= 1;
    const int64_t b = rp[u], e = rp[u + 1];
    if (b < 0 || e < b || e > n_arcs) {
        if (sub == 0) atomicOr(flags, f | 1u);
        return;
    }
    for (int64_t k = b + sub; k < e; k += kValLanes) {
        const int32_t c = col[k];
        if (c < 0 || (int64_t)c >= n) f |= 2;
        if ((int64_t)c == u) f |= 4;
        if (k > b && c <= col[k - 1]) f |= 8;
    }
    if (f) atomicOr(flags, f);
}

__global__ void k_row_up(const int64_t *__restrict__ rp, const int32_t *__restrict__ col,
                         int64_t n, uint32_t *__restrict__ nup, int64_t *__restrict__ first) {
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n) return;
    int64_t lo = rp[u], hi = rp[u + 1];
    const int64_t end = hi;
    while (lo < hi) {                    // first arc with col > u
        const int64_t mid = (lo + hi) >> 1;
        if (col[mid] > (int32_t)u) hi = mid; else lo = mid + 1;
    }
    first[u] = lo;
    nup[u] = (uint32_t)(end - lo);
}

__global__ void k_fill_edges(const int64_t *__restrict__ rp, const int32_t *__restrict__ col,
                             int64_t n, const int64_t *__restrict__ first,
                             const uint64_t *__restrict__ eoff, int32_t *__restrict__ eu,
                             int32_t *__restrict__ ev, const uint32_t *__restrict__ wt,
                             uint32_t *__restrict__ ea) {
    const int64_t u = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (u >= n) return;
    const int64_t f = first[u], end = rp[u + 1];
    const int64_t base = (int64_t)eoff[u];
    for (int64_t k = f + lane; k < end; k += 64) {
        eu[base + (k - f)] = (int32_t)u;
        ev[base + (k - f)] = col[k];
        if (ea) ea[base + (k - f)] = wt[k];
    }
}

// Count pass: pair entries each wave will emit.  Without a row filter every
// accepted sample gives two entries and no walk is needed; with a filter
// [row_lo, row_hi) the walk decides which orientations fall inside.
template <bool FILTER, bool W>
__global__ void __launch_bounds__(kBlock)
k_sample_count(SamplePlan pl, const int64_t *__restrict__ rp, const int32_t *__restrict__ col,
               const int32_t *__restrict__ eu, const int32_t *__restrict__ ev, int64_t m,
               int64_t row_lo, int64_t row_hi, uint32_t *__restrict__ wave_cnt,
               unsigned long long *__restrict__ att_part, uint32_t *__restrict__ wmax_part,
               unsigned long long *__restrict__ acc_part) {
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t e = t / pl.chunks;
    const int64_t c = t - e * pl.chunks;
    uint32_t cnt = 0;
    uint64_t att = 0;
    uint64_t wmax = 0;
    uint32_t acc = 0;
    if (e < m) {
        const int32_t u = eu[e], v = ev[e];
        const Coin cn = coin_of<W>(pl, rp, e, u, v);
        const uint64_t ne = draw_ne(pl, e);
        const uint64_t j0 = (uint64_t)c * pl.J;
        const uint64_t j1 = min(j0 + (uint64_t)pl.J, ne);
        uint64_t c1 = 0;   // accepted length-1 samples (merged)
        for (uint64_t j = j0; j < j1; ++j) {
            const uint4 b0 = slot_block(pl, e, (uint32_t)j, 0);
            const bool ok = cn.all || (uint64_t)b0.x < cn.tau;
            if (!ok) continue;
            ++acc;
            if (draw_r(pl, b0.y) == 1) {
                ++c1;
            } else if (pl.upper) {
                cnt += 1;
            } else if (FILTER) {
                int32_t a = u, b = v;
                walk_pair<W>(pl, rp, col, e, (uint32_t)j, b0, u, v, a, b);
                cnt += (a >= row_lo && a < row_hi) ? 1u : 0u;
                cnt += (b >= row_lo && b < row_hi) ? 1u : 0u;
            } else {
                cnt += 2;
            }
        }
        if (c1) {
            const uint64_t g = r1_group(weight_r1<W>(pl, cn, e));
            const uint32_t nm = (uint32_t)((c1 + g - 1) / g);
            const uint32_t per = pl.upper ? 1u
                                 : FILTER ? ((u >= row_lo && u < row_hi) ? 1u : 0u) +
                                                ((v >= row_lo && v < row_hi) ? 1u : 0u)
                                          : 2u;
            cnt += nm * per;
        }
        att = j1 > j0 ? j1 - j0 : 0;
        // weighted: r / sum_j 1/A_j <= r A_uv (the centre edge's term alone),
        // so rint(2^16 T A_uv / p_e) bounds every sample weight of the edge
        wmax = acc ? (W ? sample_weight((double)pl.T * (double)pl.ea[e], cn.all, cn.p) : cn.w)
                   : 0;
    }
    uint64_t accw = acc;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        cnt += __shfl_xor(cnt, off, 64);
        att += __shfl_xor(att, off, 64);
        accw += __shfl_xor(accw, off, 64);
        const uint64_t o = __shfl_xor(wmax, off, 64);
        wmax = o > wmax ? o : wmax;
    }
    if ((threadIdx.x & 63) == 0) wave_cnt[t >> 6] = cnt;
    // per-block partial statistics (one writer per block, folded afterwards:
    // a device-wide atomic per wave would serialise millions of updates)
    if (att_part) {
        __shared__ unsigned long long s_att[kBlock / 64], s_acc[kBlock / 64];
        __shared__ uint64_t s_max[kBlock / 64];
        if ((threadIdx.x & 63) == 0) {
            s_att[threadIdx.x >> 6] = att;
            s_acc[threadIdx.x >> 6] = accw;
            s_max[threadIdx.x >> 6] = wmax;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned long long a = 0, ac = 0;
            uint64_t w = 0;
            for (int i = 0; i < kBlock / 64; ++i) {
                a += s_att[i];
                ac += s_acc[i];
                w = s_max[i] > w ? s_max[i] : w;
            }
            att_part[blockIdx.x] = a;
            acc_part[blockIdx.x] = ac;
            wmax_part[blockIdx.x] = w > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)w;
        }
    }
}

// out[0] = sum of att_part, out[1] (as uint32) = max of wmax_part, out[2] =
// sum of acc_part; one block.
__global__ void __launch_bounds__(1024)
k_fold_stats(const unsigned long long *__restrict__ att_part,
             const uint32_t *__restrict__ wmax_part,
             const unsigned long long *__restrict__ acc_part, int64_t n,
             unsigned long long *__restrict__ out) {
    __shared__ unsigned long long sa[1024], sc[1024];
    __shared__ uint32_t sm[1024];
    unsigned long long a = 0, ac = 0;
    uint32_t w = 0;
    for (int64_t i = threadIdx.x; i < n; i += 1024) {
        a += att_part[i];
        ac += acc_part[i];
        w = wmax_part[i] > w ? wmax_part[i] : w;
    }
    sa[threadIdx.x] = a;
    sc[threadIdx.x] = ac;
    sm[threadIdx.x] = w;
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            sa[threadIdx.x] += sa[threadIdx.x + o];
            sc[threadIdx.x] += sc[threadIdx.x + o];
            sm[threadIdx.x] = sm[threadIdx.x + o] > sm[threadIdx.x] ? sm[threadIdx.x + o]
                                                                    : sm[threadIdx.x];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = sa[0];
        out[1] = sm[0];
        out[2] = sc[0];
    }
}

// Emit pass: every wave writes its entries contiguously from the scanned
// per-wave count; the order inside a wave is (slot, lane, orientation).
// Keys are ((row - row_lo) << colbits) | col.
template <bool W>
__global__ void __launch_bounds__(kBlock)
k_sample_emit(SamplePlan pl, const int64_t *__restrict__ rp, const int32_t *__restrict__ col,
              const int32_t *__restrict__ eu, const int32_t *__restrict__ ev, int64_t m,
              int64_t row_lo, int64_t row_hi, const uint64_t *__restrict__ wave_off,
              uint64_t *__restrict__ keys, uint32_t *__restrict__ vals) {
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t e = t / pl.chunks;
    const int64_t c = t - e * pl.chunks;
    const int lane = threadIdx.x & 63;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    uint64_t pos = wave_off[t >> 6];
    int32_t u = 0, v = 0;
    Coin cn{true, 0, 1.0, 0};
    uint64_t ne = 0;
    const uint64_t j0 = (uint64_t)c * pl.J;
    if (e < m) {
        u = eu[e];
        v = ev[e];
        cn = coin_of<W>(pl, rp, e, u, v);
        ne = draw_ne(pl, e);
    }
    uint32_t w = (uint32_t)cn.w;
    const int kb = pl.colbits + pl.cbits;
    uint64_t c1 = 0;   // accepted length-1 samples, emitted merged below
    // writes the entries (a, b) and (b, a) that fall in the row range, at
    // this lane's place in the wave's contiguous output
    auto put = [&](bool ina, bool inb, int32_t a, int32_t b, uint64_t ch, uint32_t wv) {
        if (pl.upper) {
            // one entry (min, max) per sample (the rows cover all vertices)
            if (a > b) { const int32_t x = a; a = b; b = x; }
            inb = false;
        }
        const uint32_t cnt = (ina ? 1u : 0u) + (inb ? 1u : 0u);
        const uint64_t m0 = __ballot(cnt & 1u), m1 = __ballot(cnt & 2u);
        uint64_t idx = pos + (uint64_t)__popcll(m0 & lt) + 2ull * (uint64_t)__popcll(m1 & lt);
        if (ina) {
            keys[idx] = ((uint64_t)(uint32_t)(a - row_lo) << kb) |
                        ((uint64_t)(uint32_t)b << pl.cbits) | ch;
            vals[idx] = wv;
            ++idx;
        }
        if (inb) {
            keys[idx] = ((uint64_t)(uint32_t)(b - row_lo) << kb) |
                        ((uint64_t)(uint32_t)a << pl.cbits) | ch;
            vals[idx] = wv;
        }
        pos += (uint64_t)__popcll(m0) + 2ull * (uint64_t)__popcll(m1);
    };
    if constexpr (!W) {
        // kWalkQ slots at a time: their walks advance together, so each lane
        // has kWalkQ chains of dependent loads (row offsets, then the column)
        // in flight instead of one; the entries still go out in slot order.
        // A slot without a step to take loads from u (cached) and keeps its
        // vertex, so the loads carry no branch.
        for (int64_t jj = 0; jj < pl.J; jj += kWalkQ) {
            int32_t x[kWalkQ], y[kWalkQ];
            int r[kWalkQ], split[kWalkQ], steps[kWalkQ], left[kWalkQ];
            uint4 buf[kWalkQ];
            uint32_t blk[kWalkQ];
#pragma unroll
            for (int q = 0; q < kWalkQ; ++q) {
                x[q] = u; y[q] = v; r[q] = 1; split[q] = 0; steps[q] = 0; left[q] = 1;
                buf[q] = make_uint4(0, 0, 0, 0); blk[q] = 0;
            }
#pragma unroll
            for (int q = 0; q < kWalkQ; ++q) {
                const uint64_t j = j0 + (uint64_t)(jj + q);
                if (e < m && jj + q < pl.J && j < ne) {
                    const uint4 b0 = slot_block(pl, e, (uint32_t)j, 0);
                    if (cn.all || (uint64_t)b0.x < cn.tau) {
                        r[q] = draw_r(pl, b0.y);
                        if (r[q] == 1) {
                            ++c1;
                        } else {
                            split[q] = (int)(b0.z % (uint32_t)r[q]);
                            steps[q] = r[q] - 1;
                            buf[q] = make_uint4(b0.w, 0, 0, 0);
                        }
                    }
                }
            }
            int nsteps = 0;
#pragma unroll
            for (int q = 0; q < kWalkQ; ++q) nsteps = max(nsteps, steps[q]);
            for (int i = 0; i < nsteps; ++i) {
                int32_t cur[kWalkQ];
                uint32_t z[kWalkQ];
                bool act[kWalkQ];
#pragma unroll
                for (int q = 0; q < kWalkQ; ++q) {
                    act[q] = i < steps[q];
                    if (act[q] && left[q] == 0) {
                        buf[q] = slot_block(pl, e, (uint32_t)(j0 + (uint64_t)(jj + q)), ++blk[q]);
                        left[q] = 4;
                    }
                    z[q] = buf[q].x;
                    if (act[q]) {
                        buf[q] = make_uint4(buf[q].y, buf[q].z, buf[q].w, 0);
                        --left[q];
                    }
                    cur[q] = act[q] ? (i < split[q] ? x[q] : y[q]) : u;
                }
                int64_t beg[kWalkQ], end[kWalkQ];
#pragma unroll
                for (int q = 0; q < kWalkQ; ++q) { beg[q] = rp[cur[q]]; end[q] = rp[cur[q] + 1]; }
                int32_t nb[kWalkQ];
                uint32_t deg[kWalkQ];
#pragma unroll
                for (int q = 0; q < kWalkQ; ++q) {
                    deg[q] = (uint32_t)(end[q] - beg[q]);
                    const int64_t at = beg[q] + (int64_t)(deg[q] ? z[q] % deg[q] : 0u);
                    nb[q] = col[min(at, 2 * m - 1)];
                }
#pragma unroll
                for (int q = 0; q < kWalkQ; ++q) {
                    // a sink (asymmetric input) holds
                    const int32_t nx = deg[q] ? nb[q] : cur[q];
                    if (act[q]) {
                        if (i < split[q]) x[q] = nx;
                        else y[q] = nx;
                    }
                }
            }
#pragma unroll
            for (int q = 0; q < kWalkQ; ++q) {
                if (jj + q >= pl.J) break;                              // uniform
                const bool walked = steps[q] > 0;
                const bool ina = walked && x[q] >= row_lo && x[q] < row_hi;
                const bool inb = walked && y[q] >= row_lo && y[q] < row_hi;
                const uint64_t ch = pl.cbits && walked ? (uint64_t)(r[q] - 1) : 0;
                put(ina, inb, walked ? x[q] : u, walked ? y[q] : v, ch, w);
            }
        }
    } else {
        // the weighted walk, kWalkQ slots at a time as above: each level of a
        // step's dependent loads (row bounds, cumulative weights at them, the
        // guide entry, the arc's weight and column) is requested for every
        // slot before the next level; each slot keeps its own path factor
        const double inv0 = e < m ? 1.0 / (double)pl.ea[e] : 1.0;
        for (int64_t jj = 0; jj < pl.J; jj += kWalkQ) {
            int32_t x[kWalkQ], y[kWalkQ];
            int r[kWalkQ], split[kWalkQ], steps[kWalkQ], left[kWalkQ];
            uint4 buf[kWalkQ];
            uint32_t blk[kWalkQ];
            double inv[kWalkQ];
#pragma unroll
            for (int q = 0; q < kWalkQ; ++q) {
                x[q] = u; y[q] = v; r[q] = 1; split[q] = 0; steps[q] = 0; left[q] = 1;
                buf[q] = make_uint4(0, 0, 0, 0); blk[q] = 0; inv[q] = inv0;
            }
#pragma unroll
            for (int q = 0; q < kWalkQ; ++q) {
                const uint64_t j = j0 + (uint64_t)(jj + q);
                if (e < m && jj + q < pl.J && j < ne) {
                    const uint4 b0 = slot_block(pl, e, (uint32_t)j, 0);
                    if (cn.all || (uint64_t)b0.x < cn.tau) {
                        r[q] = draw_r(pl, b0.y);
                        if (r[q] == 1) {
                            ++c1;
                        } else {
                            split[q] = (int)(b0.z % (uint32_t)r[q]);
                            steps[q] = r[q] - 1;
                            buf[q] = make_uint4(b0.w, 0, 0, 0);
                        }
                    }
                }
            }
            int nsteps = 0;
#pragma unroll
            for (int q = 0; q < kWalkQ; ++q) nsteps = max(nsteps, steps[q]);
            for (int i = 0; i < nsteps; ++i) {
                int32_t cur[kWalkQ];
                uint32_t z[kWalkQ];
                bool act[kWalkQ];
#pragma unroll
                for (int q = 0; q < kWalkQ; ++q) {
                    act[q] = i < steps[q];
                    if (act[q] && left[q] == 0) {
                        buf[q] = slot_block(pl, e, (uint32_t)(j0 + (uint64_t)(jj + q)), ++blk[q]);
                        left[q] = 4;
                    }
                    z[q] = buf[q].x;
                    if (act[q]) {
                        buf[q] = make_uint4(buf[q].y, buf[q].z, buf[q].w, 0);
                        --left[q];
                    }
                    cur[q] = act[q] ? (i < split[q] ? x[q] : y[q]) : u;
                }
                int64_t beg[kWalkQ], end[kWalkQ];
#pragma unroll
                for (int q = 0; q < kWalkQ; ++q) { beg[q] = rp[cur[q]]; end[q] = rp[cur[q] + 1]; }
                uint64_t base[kWalkQ], top[kWalkQ];
#pragma unroll
                for (int q = 0; q < kWalkQ; ++q) { base[q] = pl.cw[beg[q]]; top[q] = pl.cw[end[q]]; }
                // the arc k of the row with cw[k] <= t < cw[k + 1]: from the
                // guide entry of t's bucket forward (as in walk_step)
                uint32_t deg[kWalkQ];
                uint64_t tt[kWalkQ];
                int64_t ai[kWalkQ];
#pragma unroll
                for (int q = 0; q < kWalkQ; ++q) {
                    deg[q] = (uint32_t)(top[q] - base[q]);   // < 2^32 (validated)
                    const uint64_t k = (uint64_t)(end[q] - beg[q]);
                    tt[q] = base[q] + (uint64_t)(deg[q] ? z[q] % deg[q] : 0u);
                    const uint64_t bkt = deg[q] ? (tt[q] - base[q]) * k / deg[q] : 0;
                    ai[q] = deg[q] ? beg[q] + (int64_t)min((uint64_t)pl.guide[beg[q] + (int64_t)bkt],
                                                           k - 1)
                                   : beg[q];
                }
#pragma unroll
                for (int q = 0; q < kWalkQ; ++q)
                    if (act[q] && deg[q])
                        while (ai[q] < end[q] - 1 && pl.cw[ai[q] + 1] <= tt[q]) ++ai[q];
                uint32_t wa[kWalkQ];
                int32_t nb[kWalkQ];
#pragma unroll
                for (int q = 0; q < kWalkQ; ++q) {
                    const int64_t at = min(ai[q], 2 * m - 1);
                    wa[q] = pl.wt[at];
                    nb[q] = col[at];
                }
#pragma unroll
                for (int q = 0; q < kWalkQ; ++q) {
                    if (act[q] && deg[q]) {
                        inv[q] += 1.0 / (double)wa[q];
                        if (i < split[q]) x[q] = nb[q];
                        else y[q] = nb[q];
                    }
                    // a sink (asymmetric input) holds
                }
            }
#pragma unroll
            for (int q = 0; q < kWalkQ; ++q) {
                if (jj + q >= pl.J) break;                              // uniform
                const bool walked = steps[q] > 0;
                const bool ina = walked && x[q] >= row_lo && x[q] < row_hi;
                const bool inb = walked && y[q] >= row_lo && y[q] < row_hi;
                const uint64_t ch = pl.cbits && walked ? (uint64_t)(r[q] - 1) : 0;
                // the path factor r / sum 1/A; the count pass bounded the
                // weight below 2^32
                const uint32_t wq =
                    walked ? (uint32_t)sample_weight((double)r[q] / inv[q], cn.all, cn.p) : w;
                put(ina, inb, walked ? x[q] : u, walked ? y[q] : v, ch, wq);
            }
        }
    }
    // the merged length-1 samples: ceil(c1 / g) entries of up to g samples
    uint64_t g = 1, w1 = 0;
    uint32_t nm = 0;
    if (c1) {
        w1 = weight_r1<W>(pl, cn, e);
        g = r1_group(w1);
        nm = (uint32_t)((c1 + g - 1) / g);
    }
    uint32_t nmax = nm;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const uint32_t o = __shfl_xor(nmax, off, 64);
        nmax = o > nmax ? o : nmax;
    }
    for (uint32_t q = 0; q < nmax; ++q) {
        const bool has = q < nm;
        const uint64_t cq = has ? min(g, c1 - (uint64_t)q * g) : 0;
        put(has && u >= row_lo && u < row_hi, has && v >= row_lo && v < row_hi, u, v, 0,
            (uint32_t)(cq * w1));
    }
}

template <bool W>
__global__ void k_sample_slots(SamplePlan pl, const int64_t *__restrict__ rp,
                               const int32_t *__restrict__ col, const int32_t *__restrict__ eu,
                               const int32_t *__restrict__ ev, int64_t e_begin, int64_t count,
                               int32_t *__restrict__ oa, int32_t *__restrict__ ob,
                               uint64_t *__restrict__ ow, uint8_t *__restrict__ orr) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= count) return;
    const int64_t e = e_begin + s / pl.S;
    const uint64_t j = (uint64_t)(s % pl.S);
    const int32_t u = eu[e], v = ev[e];
    int32_t a = -1, b = -1;
    uint64_t w = 0;
    uint8_t r = 0;
    if (j < draw_ne(pl, e)) {
        const Coin cn = coin_of<W>(pl, rp, e, u, v);
        const uint4 b0 = slot_block(pl, e, (uint32_t)j, 0);
        if (cn.all || (uint64_t)b0.x < cn.tau) {
            a = u;
            b = v;
            double h;
            walk_pair<W>(pl, rp, col, e, (uint32_t)j, b0, u, v, a, b, &h);
            r = (uint8_t)draw_r(pl, b0.y);
            w = W ? sample_weight(h, cn.all, cn.p) : cn.w;
        }
    }
    oa[s] = a;
    ob[s] = b;
    ow[s] = w;
    orr[s] = r;
}

__global__ void k_philox(uint64_t seed, const uint4 *__restrict__ ctr, int64_t count,
                         uint4 *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    out[i] = philox4x32_10(ctr[i], (uint32_t)seed, (uint32_t)(seed >> 32));
}

template <class T> __device__ __forceinline__ T from_double(double x);
template <> __device__ __forceinline__ double from_double<double>(double x) { return x; }
template <> __device__ __forceinline__ float from_double<float>(double x) { return (float)x; }
template <> __device__ __forceinline__ __bf16 from_double<__bf16>(double x) {
    return (__bf16)(float)x;
}

template <class T>
__global__ void k_gaussian(int64_t n, int32_t k, int64_t ld, uint64_t seed, T *__restrict__ out) {
    const int32_t half = (k + 1) >> 1;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * half) return;
    const int64_t i = t / half;
    const uint32_t h = (uint32_t)(t - i * half);
    const uint4 z = philox4x32_10(
        make_uint4((uint32_t)i, (uint32_t)((uint64_t)i >> 32), h, kTagOmega),
        (uint32_t)seed, (uint32_t)(seed >> 32));
    const double u1 = ((double)z.x + 0.5) * 2.3283064365386963e-10;   // 2^-32
    const double u2 = ((double)z.y + 0.5) * 2.3283064365386963e-10;
    const double rad = sqrt(-2.0 * log(u1));
    const double ang = 2.0 * 3.141592653589793 * u2;
    double sn, cs;
    sincos(ang, &sn, &cs);   // one argument reduction for both
    const int64_t c = 2 * (int64_t)h;
    out[i * ld + c] = from_double<T>(rad * cs);
    if (c + 1 < k) out[i * ld + c + 1] = from_double<T>(rad * sn);
}

// Sparse-sign test matrix: row i holds kSparseOmega entries; word t of
// Philox(counter = (i_lo, i_hi, t / 4, 5 << 24)) gives column (z >> 1) mod k
// and sign (z & 1 ? -1 : +1), stored as sign (column + 1) in int16.
__global__ void k_sparse_omega(int64_t n, int32_t k, uint64_t seed, int16_t *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int16_t e[kSparseOmega];
#pragma unroll
    for (int b = 0; b < kSparseOmega / 4; ++b) {
        const uint4 z = philox4x32_10(
            make_uint4((uint32_t)i, (uint32_t)((uint64_t)i >> 32), (uint32_t)b, kTagSparseOmega),
            (uint32_t)seed, (uint32_t)(seed >> 32));
        const uint32_t w[4] = {z.x, z.y, z.z, z.w};
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int c = (int)((w[t] >> 1) % (uint32_t)k) + 1;
            e[4 * b + t] = (int16_t)((w[t] & 1u) ? -c : c);
        }
    }
    *reinterpret_cast<uint4 *>(out + i * kSparseOmega) = *reinterpret_cast<const uint4 *>(e);
}

}  // namespace

lne_status launch_sparse_omega(lne_ctx *ctx, int64_t n, int32_t k, uint64_t seed, int16_t *out) {
    if (n <= 0) return LNE_OK;
    {
        Launch L(ctx, "sparse_omega");
        k_sparse_omega<<<grid_of(n, 256), 256, 0, ctx->stream>>>(n, k, seed, out);
    }
    return check_launch(ctx, "sparse_omega");
}

int64_t sample_threads(const SamplePlan &pl, int64_t m) {
    return ceil_div(m * pl.chunks, kBlock) * kBlock;
}

lne_status validate_graph_device(lne_ctx *ctx, const Graph *g) {
    Buf fl(ctx);
    LNE_TRY(alloc(ctx, fl, sizeof(uint32_t)));
    LNE_HIP(ctx, hipMemsetAsync(fl.p, 0, sizeof(uint32_t), ctx->stream));
    {
        Launch L(ctx, "validate_graph");
        k_validate<<<grid_of(g->n * kValLanes, 256), 256, 0, ctx->stream>>>(
            g->row_ptr, g->col, g->n, g->n_arcs, fl.as<uint32_t>());
    }
    LNE_TRY(check_launch(ctx, "validate_graph"));
    uint32_t f = 0;
    LNE_HIP(ctx, hipMemcpyAsync(&f, fl.p, sizeof(f), hipMemcpyDeviceToHost, ctx->stream));
    LNE_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (f)
        return fail(ctx, LNE_EINVAL,
                    "graph CSR is malformed (%s%s%s%s)", (f & 1) ? "offsets " : "",
                    (f & 2) ? "column-range " : "", (f & 4) ? "self-loop " : "",
                    (f & 8) ? "unsorted-or-duplicate" : "");
    return LNE_OK;
}

lne_status build_edges(lne_ctx *ctx, const Graph *g, Buf &eu, Buf &ev, int64_t m,
                       Buf *ea) {
    Buf nup(ctx), first(ctx), eoff(ctx);
    if (ea) LNE_TRY(alloc(ctx, *ea, sizeof(uint32_t) * (size_t)(m > 0 ? m : 1)));
    LNE_TRY(alloc(ctx, nup, sizeof(uint32_t) * (size_t)(g->n + 1)));
    LNE_TRY(alloc(ctx, first, sizeof(int64_t) * (size_t)(g->n + 1)));
    LNE_TRY(alloc(ctx, eoff, sizeof(uint64_t) * (size_t)(g->n + 1)));
    LNE_TRY(alloc(ctx, eu, sizeof(int32_t) * (size_t)(m > 0 ? m : 1)));
    LNE_TRY(alloc(ctx, ev, sizeof(int32_t) * (size_t)(m > 0 ? m : 1)));
    {
        Launch L(ctx, "row_up");
        k_row_up<<<grid_of(g->n, 256), 256, 0, ctx->stream>>>(g->row_ptr, g->col, g->n,
                                                              nup.as<uint32_t>(),
                                                              first.as<int64_t>());
    }
    LNE_TRY(check_launch(ctx, "row_up"));
    LNE_TRY(scan_u32(ctx, nup.as<uint32_t>(), eoff.as<uint64_t>(), g->n));
    {
        Launch L(ctx, "fill_edges");
        k_fill_edges<<<grid_of(g->n * 64, 256), 256, 0, ctx->stream>>>(
            g->row_ptr, g->col, g->n, first.as<int64_t>(), eoff.as<uint64_t>(),
            eu.as<int32_t>(), ev.as<int32_t>(), g->weight, ea ? ea->as<uint32_t>() : nullptr);
    }
    return check_launch(ctx, "fill_edges");
}

// Weighted rows: flag 1 = a zero weight, 2 = a weighted degree of 2^32 or
// more.  16 lanes per row.
__global__ void k_weight_check(const int64_t *__restrict__ rp, const uint32_t *__restrict__ wt,
                               const uint64_t *__restrict__ cw, int64_t n,
                               uint32_t *__restrict__ flags) {
    const int64_t u = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kValLanes;
    const int sub = threadIdx.x % kValLanes;
    if (u >= n) return;
    const int64_t b = rp[u], e = rp[u + 1];
    uint32_t f = 0;
    for (int64_t k = b + sub; k < e; k += kValLanes) f |= wt[k] == 0 ? 1u : 0u;
    if (sub == 0 && cw[e] - cw[b] >= (1ull << 32)) f |= 2;
    if (f) atomicOr(flags, f);
}

// 16 lanes per row, each lane the buckets of every 16th arc.  Bucket b's
// value ceil(b W / k) lies in the slice [s, e) of the arcs with
// B(s) <= b < B(e), B(s) = number of buckets whose value is below s =
// floor((s - 1) k / W) + 1 (0 for s = 0); B(W) = k as weights are >= 1.
__global__ void k_guide(const int64_t *__restrict__ rp, const uint64_t *__restrict__ cw,
                        int64_t n, uint32_t *__restrict__ guide) {
    const int64_t u = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kValLanes;
    const int sub = threadIdx.x % kValLanes;
    if (u >= n) return;
    const int64_t b0 = rp[u], e0 = rp[u + 1];
    const uint64_t k = (uint64_t)(e0 - b0);
    if (k == 0) return;
    const uint64_t base = cw[b0], W = cw[e0] - base;
    for (int64_t i = sub; i < (int64_t)k; i += kValLanes) {
        const uint64_t s = cw[b0 + i] - base, e = cw[b0 + i + 1] - base;
        const uint64_t lo = s == 0 ? 0 : (s - 1) * k / W + 1;
        const uint64_t hi = min((e - 1) * k / W + 1, k);
        for (uint64_t b = lo; b < hi; ++b) guide[b0 + (int64_t)b] = (uint32_t)i;
    }
}

lne_status weight_guide(lne_ctx *ctx, const Graph *g, const uint64_t *cw, Buf &guide) {
    LNE_TRY(alloc(ctx, guide, sizeof(uint32_t) * (size_t)(g->n_arcs > 0 ? g->n_arcs : 1)));
    if (g->n > 0) {
        Launch L(ctx, "weight_guide");
        k_guide<<<grid_of(g->n * kValLanes, 256), 256, 0, ctx->stream>>>(
            g->row_ptr, cw, g->n, guide.as<uint32_t>());
    }
    return check_launch(ctx, "weight_guide");
}

lne_status weight_info(lne_ctx *ctx, const Graph *g, Buf &cw, uint64_t *vol) {
    LNE_TRY(alloc(ctx, cw, sizeof(uint64_t) * (size_t)(g->n_arcs + 1)));
    LNE_TRY(scan_u32(ctx, g->weight, cw.as<uint64_t>(), g->n_arcs));
    Buf fl(ctx);
    LNE_TRY(alloc(ctx, fl, sizeof(uint32_t)));
    LNE_HIP(ctx, hipMemsetAsync(fl.p, 0, sizeof(uint32_t), ctx->stream));
    if (g->n > 0) {
        Launch L(ctx, "weight_check");
        k_weight_check<<<grid_of(g->n * kValLanes, 256), 256, 0, ctx->stream>>>(
            g->row_ptr, g->weight, cw.as<uint64_t>(), g->n, fl.as<uint32_t>());
    }
    LNE_TRY(check_launch(ctx, "weight_check"));
    uint32_t h[1] = {0};
    uint64_t total = 0;
    LNE_HIP(ctx, hipMemcpyAsync(h, fl.p, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
    LNE_HIP(ctx, hipMemcpyAsync(&total, cw.as<uint64_t>() + g->n_arcs, sizeof(total),
                                hipMemcpyDeviceToHost, ctx->stream));
    LNE_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (h[0] & 1) return fail(ctx, LNE_EINVAL, "graph weights must be positive");
    if ((h[0] & 2) || total >= (1ull << 32))
        return fail(ctx, LNE_EUNSUPPORTED, "weighted degrees and vol must be below 2^32");
    *vol = total;
    return LNE_OK;
}

lne_status launch_sample_slots(lne_ctx *ctx, const Graph *g, const SamplePlan &pl,
                               const int32_t *eu, const int32_t *ev, int64_t e_begin,
                               int64_t e_end, int32_t *a, int32_t *b, uint64_t *w,
                               uint8_t *r) {
    const int64_t count = (e_end - e_begin) * pl.S;
    if (count <= 0) return LNE_OK;
    {
        Launch L(ctx, "sample_slots");
        if (pl.wt)
            k_sample_slots<true><<<grid_of(count, 256), 256, 0, ctx->stream>>>(
                pl, g->row_ptr, g->col, eu, ev, e_begin, count, a, b, w, r);
        else
            k_sample_slots<false><<<grid_of(count, 256), 256, 0, ctx->stream>>>(
                pl, g->row_ptr, g->col, eu, ev, e_begin, count, a, b, w, r);
    }
    return check_launch(ctx, "sample_slots");
}

lne_status launch_sample_count(lne_ctx *ctx, const Graph *g, const SamplePlan &pl,
                               const int32_t *eu, const int32_t *ev, int64_t m, int64_t row_lo,
                               int64_t row_hi, uint32_t *wave_cnt, int64_t n_waves,
                               unsigned long long *stats) {
    const int64_t threads = sample_threads(pl, m);
    if (threads / 64 != n_waves) return fail(ctx, LNE_EINVAL, "sampler wave count mismatch");
    const bool filter = !(row_lo <= 0 && row_hi >= g->n);
    const int64_t nblocks = threads / kBlock;
    Buf ap(ctx), wp(ctx), cp(ctx);
    if (stats) {
        LNE_TRY(alloc(ctx, ap, sizeof(unsigned long long) * (size_t)(nblocks > 0 ? nblocks : 1)));
        LNE_TRY(alloc(ctx, wp, sizeof(uint32_t) * (size_t)(nblocks > 0 ? nblocks : 1)));
        LNE_TRY(alloc(ctx, cp, sizeof(unsigned long long) * (size_t)(nblocks > 0 ? nblocks : 1)));
    }
    unsigned long long *att_part = stats ? ap.as<unsigned long long>() : nullptr;
    uint32_t *wmax_part = stats ? wp.as<uint32_t>() : nullptr;
    unsigned long long *acc_part = stats ? cp.as<unsigned long long>() : nullptr;
    {
        Launch L(ctx, filter ? "sample_count_range" : "sample_count");
#define LNE_CNT(FF, WW)                                                                    \
    k_sample_count<FF, WW><<<(unsigned)nblocks, kBlock, 0, ctx->stream>>>(                 \
        pl, g->row_ptr, g->col, eu, ev, m, row_lo, row_hi, wave_cnt, att_part, wmax_part,  \
        acc_part)
        if (filter) {
            if (pl.wt) LNE_CNT(true, true);
            else LNE_CNT(true, false);
        } else {
            if (pl.wt) LNE_CNT(false, true);
            else LNE_CNT(false, false);
        }
#undef LNE_CNT
    }
    LNE_TRY(check_launch(ctx, "sample_count"));
    if (stats) {
        Launch L(ctx, "fold_stats");
        k_fold_stats<<<1, 1024, 0, ctx->stream>>>(att_part, wmax_part, acc_part, nblocks,
                                                   stats);
    }
    return check_launch(ctx, "fold_stats");
}

lne_status launch_sample_emit(lne_ctx *ctx, const Graph *g, const SamplePlan &pl,
                              const int32_t *eu, const int32_t *ev, int64_t m, int64_t row_lo,
                              int64_t row_hi, const uint64_t *wave_off, uint64_t *keys,
                              uint32_t *vals) {
    const int64_t threads = sample_threads(pl, m);
    {
        Launch L(ctx, "sample_emit");
        if (pl.wt)
            k_sample_emit<true><<<(unsigned)(threads / kBlock), kBlock, 0, ctx->stream>>>(
                pl, g->row_ptr, g->col, eu, ev, m, row_lo, row_hi, wave_off, keys, vals);
        else
            k_sample_emit<false><<<(unsigned)(threads / kBlock), kBlock, 0, ctx->stream>>>(
                pl, g->row_ptr, g->col, eu, ev, m, row_lo, row_hi, wave_off, keys, vals);
    }
    return check_launch(ctx, "sample_emit");
}

lne_status launch_philox(lne_ctx *ctx, uint64_t seed, const uint32_t *ctr, int64_t count,
                         uint32_t *out) {
    if (count <= 0) return LNE_OK;
    {
        Launch L(ctx, "philox");
        k_philox<<<grid_of(count, 256), 256, 0, ctx->stream>>>(
            seed, reinterpret_cast<const uint4 *>(ctr), count, reinterpret_cast<uint4 *>(out));
    }
    return check_launch(ctx, "philox");
}

lne_status launch_gaussian(lne_ctx *ctx, int64_t n, int32_t k, int64_t ld, uint64_t seed,
                           int32_t dtype, void *out) {
    const int64_t work = n * ((k + 1) / 2);
    if (work <= 0) return LNE_OK;
    {
        Launch L(ctx, "gaussian");
        const unsigned gr = grid_of(work, 256);
        if (dtype == LNE_F64)
            k_gaussian<double><<<gr, 256, 0, ctx->stream>>>(n, k, ld, seed, (double *)out);
        else if (dtype == LNE_F32)
            k_gaussian<float><<<gr, 256, 0, ctx->stream>>>(n, k, ld, seed, (float *)out);
        else
            k_gaussian<__bf16><<<gr, 256, 0, ctx->stream>>>(n, k, ld, seed, (__bf16 *)out);
    }
    return check_launch(ctx, "gaussian");
}

}  // namespace lne
