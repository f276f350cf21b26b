// Pair aggregation: stable LSD radix sort of packed (row, col) keys with
// their fixed-point weights, then a segmented sum of equal keys that writes
// the count CSR directly (section 5.2: each distinct sampled pair with the
// exact sum of its weights; here order-independent integer sums instead of a
// lock-free hash, so the result is bit-identical for any launch shape).
//
// Radix pass (8-bit digit, 8192-item tiles): per-tile digit histograms
// (digit-major table, full tiles read as 16-byte vectors), one device-wide
// scan of the table, then a scatter in which every tile ranks its items
// stably (each of its 8 waves ranks a contiguous eighth of the tile with
// ballots per digit bit and its own digit counters in LDS; a block-wide
// prefix then orders the waves), stages them in LDS in digit order (keys,
// then values, through one buffer) and writes each digit run contiguously.
// For the embedding's fused reduction, the first pass whose input is in
// column order also writes each column's degree into the keys' spare bits.
#include "common.hpp"

namespace lne {

namespace {

constexpr int kT = 256;              // threads per block (heads, reductions)
constexpr int kIt = 16;              // items per thread
constexpr int kTile = kT * kIt;      // items per tile
constexpr int kWaves = kT / 64;
// Radix tiles are twice as large: a tile's run of one digit averages 32
// items, so fewer of its cache lines are written in part.
constexpr int kST = 512;             // threads per radix block
constexpr int kSTile = kST * kIt;    // items per radix tile
constexpr int kSWaves = kST / 64;

// Tile of a histogram or scatter block.  Workgroups are dispatched to the 8
// XCDs round robin, so block b runs on XCD b % 8; giving each XCD a
// contiguous range of tiles puts neighbouring tiles, whose runs of one digit
// (and whose entries of the digit-major count table) meet inside a cache
// line, in the same L2, where their partial lines merge before write-back.
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t ntiles) {
    const int64_t q = ntiles >> 3, r = ntiles & 7, x = b & 7, i = b >> 3;
    return x * q + min(x, r) + i;
}

__global__ void __launch_bounds__(kST) k_hist(const uint64_t *__restrict__ keys, int64_t n,
                                              int shift, int64_t ntiles,
                                              uint32_t *__restrict__ hist) {
    __shared__ uint32_t cnt[kSWaves][256];   // per-wave counters, summed at the end
    const int tid = threadIdx.x, wv = tid >> 6;
    for (int i = tid; i < kSWaves * 256; i += kST) cnt[i >> 8][i & 255] = 0;
    __syncthreads();
    const int64_t tile = xcd_tile(blockIdx.x, ntiles);
    const int64_t base = tile * kSTile;
    if (base + kSTile <= n) {
        // a full tile: two keys per 16-byte load, all loads issued first
        const uint4 *p = reinterpret_cast<const uint4 *>(keys + base);
        uint4 v[kIt / 2];
#pragma unroll
        for (int j = 0; j < kIt / 2; ++j) v[j] = p[j * kST + tid];
#pragma unroll
        for (int j = 0; j < kIt / 2; ++j) {
            const uint64_t k0 = (uint64_t)v[j].x | ((uint64_t)v[j].y << 32);
            const uint64_t k1 = (uint64_t)v[j].z | ((uint64_t)v[j].w << 32);
            atomicAdd(&cnt[wv][(k0 >> shift) & 255u], 1u);
            atomicAdd(&cnt[wv][(k1 >> shift) & 255u], 1u);
        }
    } else {
        for (int64_t i = base + tid; i < n; i += kST)
            atomicAdd(&cnt[wv][(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    if (tid < 256) {
        uint32_t c = 0;
#pragma unroll
        for (int w = 0; w < kSWaves; ++w) c += cnt[w][tid];
        hist[(int64_t)tid * ntiles + tile] = c;
    }
}

constexpr int kWaveItems = kIt * 64;   // contiguous items ranked by one wave

template <bool TAG>
__global__ void __launch_bounds__(kST) __attribute__((amdgpu_waves_per_eu(4)))
k_scatter(const uint64_t *__restrict__ kin, const uint32_t *__restrict__ vin, int64_t n,
          int shift, int64_t ntiles, const uint64_t *__restrict__ offs,
          uint64_t *__restrict__ kout, uint32_t *__restrict__ vout,
          const uint32_t *__restrict__ tag_deg, uint64_t colmask) {
    // one staging buffer, used for the keys and then for the values (75 KB of
    // LDS with the counters: two blocks, sixteen waves per CU)
    __shared__ uint64_t stage[kSTile];
    __shared__ uint32_t wcnt[kSWaves][256];   // per-wave digit counts, then offsets
    __shared__ uint32_t tpre[256];
    __shared__ uint64_t gbase[256];
    __shared__ uint32_t wtot[4];               // digit totals of the 4 digit waves

    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t tile = xcd_tile(blockIdx.x, ntiles);
    const int64_t base = tile * kSTile;
    const int64_t wbase = base + (int64_t)wv * kWaveItems;
    for (int i = tid; i < kSWaves * 256; i += kST) wcnt[i >> 8][i & 255] = 0;
    if (tid < 256) gbase[tid] = offs[(int64_t)tid * ntiles + tile];

    // all of this thread's items are loaded before the ranking starts, so
    // the tile's loads are in flight together
    uint64_t keys_r[kIt];
    uint32_t vals_r[kIt];
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
        const int64_t i = wbase + it * 64 + lane;
        keys_r[it] = i < n ? kin[i] : 0ull;
        vals_r[it] = i < n ? vin[i] : 0u;
    }
    if constexpr (TAG) {
        // this pass's input is sorted by column: the tile's degree reads
        // fall in a short range of the table
#pragma unroll
        for (int it = 0; it < kIt; ++it)
            if (wbase + it * 64 + lane < n) {
                const uint32_t d = tag_deg[keys_r[it] & colmask];
                keys_r[it] |= (uint64_t)min(d, kTagMax) << kTagShift;
            }
    }
    __syncthreads();

    // stable rank of each item among the wave's items of its digit: lanes
    // with equal digits are found by one ballot per digit bit; the lowest
    // such lane advances the wave's running count of that digit (one writer
    // per digit and step, read back by the whole wave at the next step)
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    uint32_t pos_r[kIt];
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
        const bool valid = wbase + it * 64 + lane < n;
        const uint32_t d = (uint32_t)(keys_r[it] >> shift) & 255u;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const uint64_t bal = __ballot((d >> b) & 1u);
            peers &= ((d >> b) & 1u) ? bal : ~bal;
        }
        const uint32_t rank = (uint32_t)__popcll(peers & lt);
        const uint32_t before = wcnt[wv][d];
        pos_r[it] = before + rank;
        __builtin_amdgcn_wave_barrier();
        if (valid && rank == 0) wcnt[wv][d] = before + (uint32_t)__popcll(peers);
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();

    // waves 0-3, thread tid = digit: the tile's exclusive digit prefix and
    // each wave's offset inside the digit's run
    uint32_t c = 0, inc = 0;
    if (tid < 256) {
#pragma unroll
        for (int w = 0; w < kSWaves; ++w) c += wcnt[w][tid];
        inc = c;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(inc, off, 64);
            if (lane >= off) inc += y;
        }
        if (lane == 63) wtot[wv] = inc;
    }
    __syncthreads();
    if (tid < 256) {
        uint32_t run = inc - c;
        for (int i = 0; i < wv; ++i) run += wtot[i];
        tpre[tid] = run;
#pragma unroll
        for (int w = 0; w < kSWaves; ++w) {
            const uint32_t t = wcnt[w][tid];
            wcnt[w][tid] = run;
            run += t;
        }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
        if (wbase + it * 64 + lane < n) {
            const uint32_t d = (uint32_t)(keys_r[it] >> shift) & 255u;
            pos_r[it] += wcnt[wv][d];           // the item's place in the tile
            stage[pos_r[it]] = keys_r[it];
        }
    }
    __syncthreads();

    // keys out in digit runs; each thread keeps the destinations of its
    // places for the values
    const int cnt = (int)min((int64_t)kSTile, n - base);
    uint64_t dst_r[kIt];
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
        const int p = it * kST + tid;
        if (p < cnt) {
            const uint64_t key = stage[p];
            const uint32_t d = (uint32_t)(key >> shift) & 255u;
            dst_r[it] = gbase[d] + (uint64_t)(p - (int)tpre[d]);
            kout[dst_r[it]] = key;
        }
    }
    __syncthreads();
    uint32_t *sval = reinterpret_cast<uint32_t *>(stage);
#pragma unroll
    for (int it = 0; it < kIt; ++it)
        if (wbase + it * 64 + lane < n) sval[pos_r[it]] = vals_r[it];
    __syncthreads();
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
        const int p = it * kST + tid;
        if (p < cnt) vout[dst_r[it]] = sval[p];
    }
}

__global__ void __launch_bounds__(kT) k_heads(const uint64_t *__restrict__ keys, int64_t n,
                                              uint32_t *__restrict__ tile_heads) {
    const int64_t base = (int64_t)blockIdx.x * kTile;
    uint32_t c = 0;
    for (int it = 0; it < kIt; ++it) {
        const int64_t i = base + it * kT + threadIdx.x;
        if (i < n && (i == 0 || keys[i] != keys[i - 1])) ++c;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
    __shared__ uint32_t ws[kWaves];
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int i = 0; i < kWaves; ++i) t += ws[i];
        tile_heads[blockIdx.x] = t;
    }
}

// Segmented sums of equal keys.  Items are visited 256 at a time in order, so
// a wave holds 64 consecutive items.  Segments strictly inside a wave are
// stored; the first and last segment of a wave may continue into a
// neighbour and are added atomically (integer, so order-independent).
__global__ void __launch_bounds__(kT) k_reduce(const uint64_t *__restrict__ keys,
                                               const uint32_t *__restrict__ vals, int64_t n,
                                               const uint64_t *__restrict__ head_off,
                                               int colbits, int32_t *__restrict__ col,
                                               unsigned long long *__restrict__ W,
                                               int64_t *__restrict__ rowptr) {
    __shared__ uint32_t wh[kWaves];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t base = (int64_t)blockIdx.x * kTile;
    const uint64_t colmask = (1ull << colbits) - 1;
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    uint64_t running = head_off[blockIdx.x];   // heads before this iteration
    for (int it = 0; it < kIt; ++it) {
        const int64_t i = base + it * kT + tid;
        const bool valid = i < n;
        uint64_t key = 0, prev = 0;
        uint64_t v = 0;
        bool head = false;
        if (valid) {
            key = keys[i];
            v = vals[i];
            prev = i > 0 ? keys[i - 1] : ~0ull;
            head = (i == 0) || key != prev;
        }
        const uint64_t hm = __ballot(head);
        if (lane == 0) wh[wv] = (uint32_t)__popcll(hm);
        __syncthreads();
        uint64_t before = running;
        uint64_t itot = 0;
        for (int w = 0; w < kWaves; ++w) {
            if (w < wv) before += wh[w];
            itot += wh[w];
        }
        __syncthreads();
        running += itot;
        // unique index: heads up to and including this item, minus one
        const uint64_t u = before + (uint64_t)__popcll(hm & (lt | (1ull << lane))) - 1;
        // inclusive segmented sum within the wave
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint64_t ov = __shfl_up(v, off, 64);
            const uint64_t ou = __shfl_up(u, off, 64);
            if (lane >= off && ou == u) v += ov;
        }
        const uint64_t nu = __shfl_down(u, 1, 64);
        const bool next_valid = i + 1 < n;
        if (!valid) continue;
        if (head) {
            col[u] = (int32_t)(key & colmask);
            const int64_t row = (int64_t)(key >> colbits);
            const int64_t prow = i == 0 ? -1 : (int64_t)(prev >> colbits);
            for (int64_t r = prow + 1; r <= row; ++r) rowptr[r] = (int64_t)u;
        }
        const bool last_in_wave = lane == 63 || !next_valid || nu != u;
        if (last_in_wave) {
            // A head at or below this lane means the segment started in this
            // wave; below lane 63 it also ends here.  Only such segments are
            // touched by one wave alone.
            const bool started_here = (hm & (lt | (1ull << lane))) != 0;
            if (started_here && lane < 63)
                W[u] = v;
            else
                atomicAdd(&W[u], (unsigned long long)v);
        }
    }
}

// Segmented sum fused with Eq. (1).  Each wave owns a contiguous chunk of
// kRChunk items and walks it 64 at a time with no block barrier, the loads of
// the next kPF groups of 64 in flight while the current one is reduced.  The
// unique index of a run comes from the chunk's head offset (k_chunk_heads +
// scan) and the wave's running head count.  A wave sums each run of equal
// keys with a segmented scan and carries the open run's partial sum from one
// group to the next; the lane holding a run's last item owns it and writes
// the column and ln x (kept) or 0 (dropped).  A run that goes on past the
// chunk is finished by the same wave, which reads on 64 keys at a time and
// finds the run's end with a ballot (a lane adding a long run item by item
// waits one memory latency per item, and a few pairs of hubs have runs of
// thousands); the next chunk's wave skips that run.  Row offsets as in
// k_reduce.  Each distinct pair is written by exactly one lane with an
// integer sum, so the result does not depend on the launch shape.  The
// cross-lane steps are DPP moves and lane reads (no LDS round trips), the
// keys at uniform places scalar loads, and the row degrees come from an LDS
// window filled once per chunk: a vector load whose value is needed at once
// would make the wave wait for every load issued before it, the prefetched
// groups included.
constexpr int kRChunk = 1024;
constexpr int kPF = 4;   // groups of 64 items a reducing wave has in flight
// Rows whose degrees a reducing wave keeps in LDS: those from its chunk's
// first row on (a chunk spans more only across empty rows; the rest are read
// from memory).
constexpr int kDegWin = 1024;

// Cross-lane moves without the LDS crossbar (gfx9 DPP): a lane with no
// source lane under the control keeps `old`.
template <int CTRL, int ROWS = 0xf>
__device__ __forceinline__ uint32_t dpp32(uint32_t old, uint32_t src) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)src, CTRL, ROWS, 0xf, false);
}
template <int CTRL>
__device__ __forceinline__ uint64_t dpp64(uint64_t old, uint64_t src) {
    return (uint64_t)dpp32<CTRL>((uint32_t)old, (uint32_t)src) |
           ((uint64_t)dpp32<CTRL>((uint32_t)(old >> 32), (uint32_t)(src >> 32)) << 32);
}
constexpr int kDppWaveShr1 = 0x138, kDppWaveShl1 = 0x130;   // whole-wave shift by one lane
constexpr int kDppRowShr = 0x110;                           // + n: shift by n in a row of 16
constexpr int kDppRowBcast15 = 0x142, kDppRowBcast31 = 0x143;

__device__ __forceinline__ uint64_t readlane64(uint64_t x, int l) {
    return (uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, l) |
           ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), l) << 32);
}

// One step of a segmented inclusive sum: add the partial sum of the source
// lane when it belongs to the same segment (seg ids rise along the lanes, so
// equal ids mean every lane between is in the segment too).
template <int CTRL, int ROWS>
__device__ __forceinline__ void seg_step(uint64_t &v, uint32_t seg) {
    const uint32_t s2 = dpp32<CTRL, ROWS>(~0u, seg);
    const uint64_t v2 = (uint64_t)dpp32<CTRL, ROWS>(0u, (uint32_t)v) |
                        ((uint64_t)dpp32<CTRL, ROWS>(0u, (uint32_t)(v >> 32)) << 32);
    if (s2 == seg) v += v2;
}

// Segmented inclusive sum over the wave: shifts by 1, 2, 4, 8 inside each row
// of 16 lanes, then lane 15 of rows 0 and 2 into rows 1 and 3, then lane 31
// into rows 2 and 3.
__device__ __forceinline__ uint64_t seg_scan64(uint64_t v, uint32_t seg) {
    seg_step<kDppRowShr + 1, 0xf>(v, seg);
    seg_step<kDppRowShr + 2, 0xf>(v, seg);
    seg_step<kDppRowShr + 4, 0xf>(v, seg);
    seg_step<kDppRowShr + 8, 0xf>(v, seg);
    seg_step<kDppRowBcast15, 0xa>(v, seg);
    seg_step<kDppRowBcast31, 0xc>(v, seg);
    return v;
}

__global__ void __launch_bounds__(kT) k_chunk_heads(const uint64_t *__restrict__ keys, int64_t n,
                                                    int64_t nchunks,
                                                    uint32_t *__restrict__ chunk_heads) {
    const int lane = threadIdx.x & 63;
    const int64_t w = ((int64_t)blockIdx.x * kT + threadIdx.x) >> 6;
    if (w >= nchunks) return;
    const int64_t base = w * kRChunk;
    uint32_t c = 0;
    // kPF groups of 64 keys loaded at a time; the key before a group's lane 0
    // is the previous group's lane 63 key
    uint64_t prev_last = base > 0 ? keys[base - 1] : ~0ull;
    for (int it0 = 0; it0 < kRChunk / 64; it0 += kPF) {
        uint64_t kq[kPF];
#pragma unroll
        for (int g = 0; g < kPF; ++g) {
            const int64_t i = base + (it0 + g) * 64 + lane;
            kq[g] = i < n ? keys[i] : ~0ull;
        }
#pragma unroll
        for (int g = 0; g < kPF; ++g) {
            const int64_t i = base + (it0 + g) * 64 + lane;
            const uint64_t prev = dpp64<kDppWaveShr1>(prev_last, kq[g]);   // lane 0: prev_last
            prev_last = readlane64(kq[g], 63);
            if (i < n && (i == 0 || kq[g] != prev)) ++c;
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
    if (lane == 0) chunk_heads[w] = c;
}

template <class VT>
__global__ void __launch_bounds__(kT) k_reduce_tl(const uint64_t *__restrict__ keys,
                                                  const uint32_t *__restrict__ vals, int64_t n,
                                                  int64_t nchunks,
                                                  const uint64_t *__restrict__ head_off,
                                                  int colbits, const uint32_t *__restrict__ deg,
                                                  int64_t row_lo, TLConst c,
                                                  int32_t *__restrict__ col, VT *__restrict__ val,
                                                  int64_t *__restrict__ rowptr,
                                                  uint32_t *__restrict__ chunk_kept,
                                                  bool tagged, uint64_t *__restrict__ keyT,
                                                  uint32_t *__restrict__ valT) {
    __shared__ uint32_t dwin[kT / 64][kDegWin];   // per wave: deg of rows rfirst, rfirst + 1, ...
    __shared__ uint32_t dmiss[kT / 64][2][64];      // per lane: a row's, a column's degree
    const int lane = threadIdx.x & 63;
    // the wave's chunk as scalars: the keys at uniform places are then scalar
    // loads, waited for apart from the vector loads in flight
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t w = (int64_t)blockIdx.x * (kT / 64) + wv;
    if (w >= nchunks) return;
    const int64_t base = w * kRChunk;
    const int64_t cend = min(n, base + kRChunk);          // end of this chunk
    const uint64_t colmask = (1ull << colbits) - 1;
    const uint64_t keymask = tagged ? (1ull << kTagShift) - 1 : ~0ull;
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    uint64_t running = head_off[w];   // heads before the current 64 items
    uint32_t my_kept = 0;
    int64_t rfirst = 0;               // first row of the chunk (of the degree window)
    // Eq. (1) for the run of `key` with weight sum W and unique index u.
    // With keyT (the upper triangle: one entry per sample, (min, max)), a
    // diagonal pair counts twice (its sample lands in both orientations of
    // the symmetric matrix) and the pair is also written transposed,
    // (max << colbits | min, value bits), for the lower triangle's sort.
    auto finish = [&](uint64_t key, uint64_t W, uint64_t u) {
        const int32_t b = (int32_t)(key & colmask);
        const int64_t row = (int64_t)((key & keymask) >> colbits);
        if (keyT && (int64_t)b == row_lo + row) W *= 2;
        // degrees from LDS: a row past the window, or a column whose tag
        // is saturated, is read from memory into the lane's LDS slot first,
        // inside the branch, so that the usual path waits for no vector load
        const int64_t rr = row - rfirst;
        const uint32_t tag = tagged ? (uint32_t)(key >> kTagShift) : kTagMax;
        if (rr >= kDegWin) dmiss[wv][0][lane] = deg[row_lo + row];
        if (tag >= kTagMax) dmiss[wv][1][lane] = deg[b];
        const uint64_t da = rr < kDegWin ? dwin[wv][rr] : dmiss[wv][0][lane];
        const uint64_t db = tag < kTagMax ? tag : dmiss[wv][1][lane];
        const bool k = tl_keep(c, W, da, db);
        const VT x = k ? (VT)log((double)W * c.scale / ((double)da * (double)db)) : (VT)0;
        col[u] = b;
        val[u] = x;
        if constexpr (sizeof(VT) == 4) {
            if (keyT) {
                keyT[u] = ((uint64_t)(uint32_t)b << colbits) | (uint64_t)(row_lo + row);
                valT[u] = __float_as_uint((float)x);
            }
        }
        my_kept += k ? 1u : 0u;
    };
    // kPF groups of 64 items in flight: group it lives in ring slot it % kPF
    // until group it + kPF replaces it.  The slots are loaded unconditionally
    // (indices past the chunk clamped to its last item) and masked where a
    // group is used: a conditional load would be merged into its slot by a
    // register copy that waits for it, and the loads would not overlap.
    // the key before the chunk and the first key after it, loaded first and
    // kept in scalar registers (waiting for them leaves the ring in flight)
    uint64_t kq[kPF];
    uint32_t vq[kPF];
#pragma unroll
    for (int g = 0; g < kPF; ++g) {
        const int64_t i = min(base + g * 64 + lane, cend - 1);
        kq[g] = keys[i];
        vq[g] = vals[i];
    }
    // scalar loads: the key before the chunk, its first and last keys and the
    // first key after it
    const uint64_t before0 = keys[max(base - 1, (int64_t)0)];
    const uint64_t first0 = keys[base];
    const uint64_t last0 = keys[cend - 1];
    const uint64_t after0 = keys[min(cend, n - 1)];
    // the degrees of the chunk's rows into the wave's LDS window (a run
    // going on past the chunk keeps the last key's row); the vector loads
    // in flight are the ones the first groups need first anyway
    rfirst = (int64_t)((first0 & keymask) >> colbits);
    {
        const int64_t span = (int64_t)((last0 & keymask) >> colbits) - rfirst + 1;
        const int nwin = (int)min(span, (int64_t)kDegWin);
        for (int j = lane; j < nwin; j += 64) dwin[wv][j] = deg[row_lo + rfirst + j];
    }
    // the key before each group's lane 0 (the last key of the group before),
    // and the first key of the next chunk
    uint64_t prev_last = base > 0 ? before0 : ~0ull;
    const uint64_t next_first = cend < n ? after0 : ~0ull;
    // the chunk's first run continues the previous chunk's last run: that
    // wave sums it, this one skips it (until its first head)
    bool skipping = base > 0 && first0 == prev_last;
    uint64_t carry = 0;               // the open run's sum in earlier groups
    uint64_t last_key = 0;
    bool open_end = false;            // the last group's last run goes on
    for (int it0 = 0; it0 < kRChunk / 64; it0 += kPF) {
#pragma unroll
        for (int g = 0; g < kPF; ++g) {
            const int it = it0 + g;
            const int64_t i = base + it * 64 + lane;
            if (base + it * 64 >= cend) break;                 // wave-uniform
            const bool valid = i < cend;
            const uint64_t key = valid ? kq[g] : ~0ull;
            uint64_t v = valid ? vq[g] : 0;
            const bool more = it + 1 < kRChunk / 64 && base + (it + 1) * 64 < cend;
            // the key after lane 63's item (a scalar load)
            const uint64_t after = more ? keys[base + (it + 1) * 64] : next_first;
            // the loads of group it + kPF go out before this reduction (past
            // the chunk they re-read its last item: no branch around them)
            {
                const int64_t j = min(i + 64 * kPF, cend - 1);
                kq[g] = keys[j];
                vq[g] = vals[j];
            }
            const uint64_t prev = dpp64<kDppWaveShr1>(prev_last, key);   // lane 0: prev_last
            prev_last = readlane64(key, 63);
            const bool head = valid && (i == 0 || key != prev);
            const uint64_t hm = __ballot(head);
            // the lane's run within the group: heads up to and including it
            const uint32_t seg = (uint32_t)__popcll(hm & (lt | (1ull << lane)));
            const uint64_t u = running + (uint64_t)seg - 1;
            running += (uint64_t)__popcll(hm);
            v = seg_scan64(v, seg);
            // lanes before the group's first head continue the open run
            const bool first_seg = seg == 0;
            if (first_seg) v += carry;
            const uint64_t nxt = dpp64<kDppWaveShl1>(after, key);         // lane 63: after
            const bool ends = valid && (i + 1 >= n || nxt != key);
            // the sum so far of a run still open after lane 63's item
            const int last = (int)min((int64_t)63, cend - 1 - (base + it * 64));
            const uint64_t vl = readlane64(v, last);
            const bool open = __builtin_amdgcn_readlane((int)(valid && !ends), last) != 0;
            carry = open ? vl : 0;
            last_key = readlane64(key, last);
            open_end = open;
            const bool skip = skipping && first_seg;
            if (hm) skipping = false;
            if (head) {
                const int64_t row = (int64_t)((key & keymask) >> colbits);
                const int64_t prow = i == 0 ? -1 : (int64_t)((prev & keymask) >> colbits);
                for (int64_t r = prow + 1; r <= row; ++r) rowptr[r] = (int64_t)u;
            }
            if (!valid || !ends || skip) continue;
            finish(key, v, u);
        }
    }
    // The run still open at the chunk's end, unless the chunk had no head
    // (then all of it continues the previous chunk's run, which that wave
    // finishes): read on, 64 keys at a time, until it ends.
    if (open_end && !skipping) {
        uint64_t W = carry;
        for (int64_t j0 = cend; j0 < n; j0 += 64) {
            const int64_t j = j0 + lane;
            const uint64_t kj = j < n ? keys[j] : ~0ull;
            const bool same = j < n && kj == last_key;
            const uint64_t m = __ballot(same);
            const int cnt = m == ~0ull ? 64 : __builtin_ctzll(~m);   // leading matches
            uint64_t s2 = lane < cnt ? (uint64_t)vals[j] : 0;
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) s2 += __shfl_xor(s2, off, 64);
            W += s2;
            if (cnt < 64) break;
        }
        if (lane == 0) finish(last_key, W, running - 1);
    }
    // the chunk's count of kept entries (summed by a scan afterwards: one
    // counter hit by every wave serialises the whole grid on it)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) my_kept += __shfl_xor(my_kept, off, 64);
    if (lane == 0) chunk_kept[w] = my_kept;
}

// Row offsets of a stream sorted by row (key >> shift): rp[r] = the first
// item whose row is at least r, for r up to the last row present (the rest
// are set by k_row_bounds_tail).
__global__ void k_row_bounds(const uint64_t *__restrict__ keys, int64_t n, int shift,
                             int64_t *__restrict__ rp) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t row = (int64_t)(keys[i] >> shift);
    const int64_t prow = i == 0 ? -1 : (int64_t)(keys[i - 1] >> shift);
    for (int64_t r = prow + 1; r <= row; ++r) rp[r] = i;
}

__global__ void k_row_bounds_tail(const uint64_t *__restrict__ keys, int64_t n, int shift,
                                  int64_t n_rows, int64_t *__restrict__ rp) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r > n_rows) return;
    const int64_t last = n > 0 ? (int64_t)(keys[n - 1] >> shift) : -1;
    if (r > last) rp[r] = n;
}

// Symmetric matrix from its upper triangle U (rows = min, with the diagonal)
// and the transposed stream L (U's pairs sorted by (max, min)): row a is L's
// segment of a without its last entry when that is the diagonal (a, a), then
// U's row a.  len[a] = row a's length; dk[block] = kept diagonal entries.
template <class VT>
__global__ void k_sym_rowlen(const int64_t *__restrict__ rpU, const int32_t *__restrict__ colU,
                             const VT *__restrict__ valU, const int64_t *__restrict__ rpL,
                             int64_t n_rows, uint32_t *__restrict__ len,
                             uint32_t *__restrict__ dk) {
    const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t kd = 0;
    if (a < n_rows) {
        const int64_t u0 = rpU[a], u1 = rpU[a + 1];
        const bool diag = u1 > u0 && colU[u0] == (int32_t)a;
        len[a] = (uint32_t)((u1 - u0) + (rpL[a + 1] - rpL[a]) - (diag ? 1 : 0));
        kd = diag && valU[u0] != (VT)0 ? 1u : 0u;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) kd += __shfl_xor(kd, off, 64);
    __shared__ uint32_t ws[4];
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = kd;
    __syncthreads();
    if (threadIdx.x == 0) dk[blockIdx.x] = ws[0] + ws[1] + ws[2] + ws[3];
}

// One wave per row: L's entries (cols below a), then U's (cols from a).
template <class VT>
__global__ void k_sym_merge(const int64_t *__restrict__ rpU, const int32_t *__restrict__ colU,
                            const VT *__restrict__ valU, const int64_t *__restrict__ rpL,
                            const uint64_t *__restrict__ keyL, const uint32_t *__restrict__ valL,
                            int64_t n_rows, uint64_t colmask, const uint64_t *__restrict__ rpF,
                            int32_t *__restrict__ colF, VT *__restrict__ valF) {
    const int64_t a = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (a >= n_rows) return;
    const int64_t u0 = rpU[a], u1 = rpU[a + 1];
    const int64_t l0 = rpL[a], l1r = rpL[a + 1];
    const int64_t o = (int64_t)rpF[a];
    // four entries per lane and step, their loads issued before any store
    constexpr int Q = 4;
    if (l1r - l0 <= 64 * Q && u1 - u0 <= 64 * Q) {
        // a short row (the usual case): both parts' loads go out together
        // (clamped to the part, so that none is predicated), then the diagonal
        // test reads U's first column from them, then every store
        uint64_t kq[Q];
        uint32_t vq[Q];
        int32_t cq[Q];
        VT wq[Q];
        if (l1r > l0) {
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const int64_t j = min(l0 + q * 64 + lane, l1r - 1);
                kq[q] = keyL[j];
                vq[q] = valL[j];
            }
        }
        if (u1 > u0) {
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const int64_t j = min(u0 + q * 64 + lane, u1 - 1);
                cq[q] = colU[j];
                wq[q] = valU[j];
            }
        }
        // keep the loads above every store (the compiler would otherwise sink
        // each part's loads to the stores that use them)
        __asm__ volatile("" ::: "memory");
        const bool diag = u1 > u0 && __builtin_amdgcn_readfirstlane(cq[0]) == (int32_t)a;
        const int64_t l1 = l1r - (diag ? 1 : 0);
        if (l1r > l0) {
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const int64_t j = l0 + q * 64 + lane;
                if (j < l1) {
                    colF[o + (j - l0)] = (int32_t)(kq[q] & colmask);
                    valF[o + (j - l0)] = (VT)__uint_as_float(vq[q]);
                }
            }
        }
        if (u1 > u0) {
            const int64_t o2 = o + (l1 - l0);
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const int64_t j = u0 + q * 64 + lane;
                if (j < u1) {
                    colF[o2 + (j - u0)] = cq[q];
                    valF[o2 + (j - u0)] = wq[q];
                }
            }
        }
        return;
    }
    const bool diag = u1 > u0 && colU[u0] == (int32_t)a;
    const int64_t l1 = l1r - (diag ? 1 : 0);
    for (int64_t j0 = l0; j0 < l1; j0 += 64 * Q) {
        uint64_t kq[Q];
        uint32_t vq[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int64_t j = j0 + q * 64 + lane;
            if (j < l1) { kq[q] = keyL[j]; vq[q] = valL[j]; }
        }
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int64_t j = j0 + q * 64 + lane;
            if (j < l1) {
                colF[o + (j - l0)] = (int32_t)(kq[q] & colmask);
                valF[o + (j - l0)] = (VT)__uint_as_float(vq[q]);
            }
        }
    }
    const int64_t o2 = o + (l1 - l0);
    for (int64_t j0 = u0; j0 < u1; j0 += 64 * Q) {
        int32_t cq[Q];
        VT wq[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int64_t j = j0 + q * 64 + lane;
            if (j < u1) { cq[q] = colU[j]; wq[q] = valU[j]; }
        }
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int64_t j = j0 + q * 64 + lane;
            if (j < u1) {
                colF[o2 + (j - u0)] = cq[q];
                valF[o2 + (j - u0)] = wq[q];
            }
        }
    }
}

__global__ void k_degrees(const int64_t *__restrict__ rp, const uint64_t *__restrict__ cw,
                          int64_t n, uint32_t *__restrict__ deg) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) deg[i] = cw ? (uint32_t)(cw[rp[i + 1]] - cw[rp[i]]) : (uint32_t)(rp[i + 1] - rp[i]);
}

__global__ void k_rowptr_tail(const uint64_t *__restrict__ keys, int64_t n_items,
                              int colbits, const uint64_t *__restrict__ nnz_p,
                              int64_t n_rows, int64_t *__restrict__ rowptr,
                              uint64_t keymask) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r > n_rows) return;
    const int64_t last =
        n_items > 0 ? (int64_t)((keys[n_items - 1] & keymask) >> colbits) : -1;
    if (r > last) rowptr[r] = (int64_t)*nnz_p;
}

}  // namespace

lne_status radix_sort(lne_ctx *ctx, uint64_t *k0, uint32_t *v0, uint64_t *k1, uint32_t *v1,
                      int64_t n, int bits, int *which, const uint32_t *tag_deg, int colbits,
                      int lo_bit) {
    *which = 0;
    if (n <= 1) return LNE_OK;
    if ((uintptr_t)k0 % 16 || (uintptr_t)k1 % 16)
        return fail(ctx, LNE_EINVAL, "radix_sort: key buffers must be 16-byte aligned");
    const int64_t ntiles = ceil_div(n, kSTile);
    Buf hist(ctx), offs(ctx);
    LNE_TRY(alloc(ctx, hist, sizeof(uint32_t) * (size_t)(256 * ntiles)));
    LNE_TRY(alloc(ctx, offs, sizeof(uint64_t) * (size_t)(256 * ntiles + 1)));
    uint64_t *ks[2] = {k0, k1};
    uint32_t *vs[2] = {v0, v1};
    int cur = 0;
    // the tagging pass: the first whose input is sorted by the column bits
    const int tag_shift = tag_deg ? radix_tag_shift(bits, colbits) : -1;
    const uint64_t colmask = (1ull << colbits) - 1;
    for (int shift = lo_bit; shift < bits; shift += 8) {
        {
            Launch L(ctx, "radix_hist");
            k_hist<<<(unsigned)ntiles, kST, 0, ctx->stream>>>(ks[cur], n, shift, ntiles,
                                                              hist.as<uint32_t>());
        }
        LNE_TRY(check_launch(ctx, "radix_hist"));
        LNE_TRY(scan_u32(ctx, hist.as<uint32_t>(), offs.as<uint64_t>(), 256 * ntiles));
        {
            Launch L(ctx, "radix_scatter");
            if (shift == tag_shift)
                k_scatter<true><<<(unsigned)ntiles, kST, 0, ctx->stream>>>(
                    ks[cur], vs[cur], n, shift, ntiles, offs.as<uint64_t>(), ks[cur ^ 1],
                    vs[cur ^ 1], tag_deg, colmask);
            else
                k_scatter<false><<<(unsigned)ntiles, kST, 0, ctx->stream>>>(
                    ks[cur], vs[cur], n, shift, ntiles, offs.as<uint64_t>(), ks[cur ^ 1],
                    vs[cur ^ 1], nullptr, colmask);
        }
        LNE_TRY(check_launch(ctx, "radix_scatter"));
        cur ^= 1;
    }
    *which = cur;
    return LNE_OK;
}

lne_status reduce_to_csr(lne_ctx *ctx, const uint64_t *keys, const uint32_t *vals,
                         int64_t n_items, int64_t n_rows, int colbits, lne_csr *out) {
    const int64_t ntiles = ceil_div(n_items > 0 ? n_items : 1, kTile);
    Buf th(ctx), hoff(ctx);
    LNE_TRY(alloc(ctx, th, sizeof(uint32_t) * (size_t)ntiles));
    LNE_TRY(alloc(ctx, hoff, sizeof(uint64_t) * (size_t)(ntiles + 1)));
    {
        Launch L(ctx, "heads");
        k_heads<<<(unsigned)ntiles, kT, 0, ctx->stream>>>(keys, n_items, th.as<uint32_t>());
    }
    LNE_TRY(check_launch(ctx, "heads"));
    LNE_TRY(scan_u32(ctx, th.as<uint32_t>(), hoff.as<uint64_t>(), ntiles));
    uint64_t nnz = 0;
    LNE_HIP(ctx, hipMemcpyAsync(&nnz, hoff.as<uint64_t>() + ntiles, sizeof(uint64_t),
                                hipMemcpyDeviceToHost, ctx->stream));
    LNE_HIP(ctx, hipStreamSynchronize(ctx->stream));

    Buf rp(ctx), cc(ctx), ww(ctx);
    LNE_TRY(alloc(ctx, rp, sizeof(int64_t) * (size_t)(n_rows + 1)));
    LNE_TRY(alloc(ctx, cc, sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1)));
    LNE_TRY(alloc(ctx, ww, sizeof(uint64_t) * (size_t)(nnz > 0 ? nnz : 1)));
    LNE_HIP(ctx, hipMemsetAsync(ww.p, 0, sizeof(uint64_t) * (size_t)(nnz > 0 ? nnz : 1),
                                ctx->stream));
    if (n_items > 0) {
        Launch L(ctx, "reduce");
        k_reduce<<<(unsigned)ntiles, kT, 0, ctx->stream>>>(
            keys, vals, n_items, hoff.as<uint64_t>(), colbits, cc.as<int32_t>(),
            ww.as<unsigned long long>(), rp.as<int64_t>());
    }
    LNE_TRY(check_launch(ctx, "reduce"));
    {
        Launch L(ctx, "rowptr_tail");
        k_rowptr_tail<<<grid_of(n_rows + 1, 256), 256, 0, ctx->stream>>>(
            keys, n_items, colbits, hoff.as<uint64_t>() + ntiles, n_rows, rp.as<int64_t>(),
            ~0ull);
    }
    LNE_TRY(check_launch(ctx, "rowptr_tail"));
    out->n_rows = n_rows;
    out->n_cols = n_rows;
    out->nnz = (int64_t)nnz;
    out->row_ptr = (int64_t *)rp.detach();
    out->col = (int32_t *)cc.detach();
    out->val = ww.detach();
    out->val_type = LNE_U64;
    return LNE_OK;
}

lne_status vertex_degrees(lne_ctx *ctx, const Graph *g, uint32_t *deg, const uint64_t *cw) {
    if (g->n > 0) {
        Launch L(ctx, "degrees");
        k_degrees<<<grid_of(g->n, 256), 256, 0, ctx->stream>>>(g->row_ptr, cw, g->n, deg);
    }
    return check_launch(ctx, "degrees");
}

lne_status reduce_to_matrix(lne_ctx *ctx, const uint64_t *keys, const uint32_t *vals,
                            int64_t n_items, int64_t n_rows, int colbits, const Graph *g,
                            const uint32_t *deg, int64_t row_lo, const TLConst &c,
                            int32_t val_type, lne_csr *out, uint64_t *kept, bool tagged,
                            SymOut *sym) {
    if (val_type != LNE_F32 && val_type != LNE_F64)
        return fail(ctx, LNE_EINVAL, "reduce_to_matrix: F32 or F64 values");
    if (sym && val_type != LNE_F32)
        return fail(ctx, LNE_EINVAL, "reduce_to_matrix: the upper-triangle path takes F32");
    const int64_t nchunks = ceil_div(n_items > 0 ? n_items : 1, kRChunk);
    const unsigned nblocks = (unsigned)ceil_div(nchunks, kT / 64);
    Buf th(ctx), hoff(ctx), bk(ctx), bko(ctx);
    LNE_TRY(alloc(ctx, th, sizeof(uint32_t) * (size_t)nchunks));
    LNE_TRY(alloc(ctx, hoff, sizeof(uint64_t) * (size_t)(nchunks + 1)));
    LNE_TRY(alloc(ctx, bk, sizeof(uint32_t) * (size_t)nchunks));
    LNE_TRY(alloc(ctx, bko, sizeof(uint64_t) * (size_t)(nchunks + 1)));
    {
        Launch L(ctx, "heads");
        k_chunk_heads<<<nblocks, kT, 0, ctx->stream>>>(keys, n_items, nchunks, th.as<uint32_t>());
    }
    LNE_TRY(check_launch(ctx, "heads"));
    LNE_TRY(scan_u32(ctx, th.as<uint32_t>(), hoff.as<uint64_t>(), nchunks));
    uint64_t nnz = 0;
    LNE_HIP(ctx, hipMemcpyAsync(&nnz, hoff.as<uint64_t>() + nchunks, sizeof(uint64_t),
                                hipMemcpyDeviceToHost, ctx->stream));
    LNE_HIP(ctx, hipStreamSynchronize(ctx->stream));
    Buf rp(ctx), cc(ctx), vv(ctx);
    LNE_TRY(alloc(ctx, rp, sizeof(int64_t) * (size_t)(n_rows + 1)));
    LNE_TRY(alloc(ctx, cc, sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1)));
    LNE_TRY(alloc(ctx, vv, dtype_size(val_type) * (size_t)(nnz > 0 ? nnz : 1)));
    if (sym) {
        LNE_TRY(alloc(ctx, sym->keyT, sizeof(uint64_t) * (size_t)(nnz > 0 ? nnz : 1)));
        LNE_TRY(alloc(ctx, sym->valT, sizeof(uint32_t) * (size_t)(nnz > 0 ? nnz : 1)));
    }
    uint64_t *kT_ = sym ? sym->keyT.as<uint64_t>() : nullptr;
    uint32_t *vT_ = sym ? sym->valT.as<uint32_t>() : nullptr;
    if (n_items > 0) {
        Launch L(ctx, "reduce_trunc_log");
        if (val_type == LNE_F64)
            k_reduce_tl<double><<<nblocks, kT, 0, ctx->stream>>>(
                keys, vals, n_items, nchunks, hoff.as<uint64_t>(), colbits, deg, row_lo, c,
                cc.as<int32_t>(), vv.as<double>(), rp.as<int64_t>(), bk.as<uint32_t>(), tagged,
                nullptr, nullptr);
        else
            k_reduce_tl<float><<<nblocks, kT, 0, ctx->stream>>>(
                keys, vals, n_items, nchunks, hoff.as<uint64_t>(), colbits, deg, row_lo, c,
                cc.as<int32_t>(), vv.as<float>(), rp.as<int64_t>(), bk.as<uint32_t>(), tagged,
                kT_, vT_);
    }
    LNE_TRY(check_launch(ctx, "reduce_trunc_log"));
    {
        Launch L(ctx, "rowptr_tail");
        k_rowptr_tail<<<grid_of(n_rows + 1, 256), 256, 0, ctx->stream>>>(
            keys, n_items, colbits, hoff.as<uint64_t>() + nchunks, n_rows, rp.as<int64_t>(),
            tagged ? (1ull << kTagShift) - 1 : ~0ull);
    }
    LNE_TRY(check_launch(ctx, "rowptr_tail"));
    uint64_t k = 0;
    if (n_items > 0) {
        LNE_TRY(scan_u32(ctx, bk.as<uint32_t>(), bko.as<uint64_t>(), nchunks));
        LNE_HIP(ctx, hipMemcpyAsync(&k, bko.as<uint64_t>() + nchunks, sizeof(k),
                                    hipMemcpyDeviceToHost, ctx->stream));
        LNE_HIP(ctx, hipStreamSynchronize(ctx->stream));
    }
    *kept = k;
    out->n_rows = n_rows;
    out->n_cols = g->n;
    out->nnz = (int64_t)nnz;
    out->row_ptr = (int64_t *)rp.detach();
    out->col = (int32_t *)cc.detach();
    out->val = vv.detach();
    out->val_type = val_type;
    return LNE_OK;
}

lne_status sym_assemble(lne_ctx *ctx, lne_csr *U, SymOut &sym, int colbits, uint64_t kept_u,
                        lne_csr *out, uint64_t *kept) {
    const int64_t n = U->n_rows, nu = U->nnz;
    // the transposed pairs, in U's (min, max) order, sorted stably by max
    Buf k1(ctx), v1(ctx);
    int which = 0;
    if (nu > 1) {
        LNE_TRY(alloc(ctx, k1, sizeof(uint64_t) * (size_t)nu));
        LNE_TRY(alloc(ctx, v1, sizeof(uint32_t) * (size_t)nu));
        LNE_TRY(radix_sort(ctx, sym.keyT.as<uint64_t>(), sym.valT.as<uint32_t>(),
                           k1.as<uint64_t>(), v1.as<uint32_t>(), nu, 2 * colbits, &which,
                           nullptr, 0, colbits));
    }
    if (which) { sym.keyT.release(); sym.valT.release(); } else { k1.release(); v1.release(); }
    const uint64_t *keyL = which ? k1.as<uint64_t>() : sym.keyT.as<uint64_t>();
    const uint32_t *valL = which ? v1.as<uint32_t>() : sym.valT.as<uint32_t>();
    Buf rpL(ctx), len(ctx), rpF(ctx), dk(ctx), dko(ctx);
    LNE_TRY(alloc(ctx, rpL, sizeof(int64_t) * (size_t)(n + 1)));
    if (nu > 0) {
        Launch L(ctx, "sym_bounds");
        k_row_bounds<<<grid_of(nu, 256), 256, 0, ctx->stream>>>(keyL, nu, colbits,
                                                                 rpL.as<int64_t>());
    }
    LNE_TRY(check_launch(ctx, "sym_bounds"));
    {
        Launch L(ctx, "sym_bounds");
        k_row_bounds_tail<<<grid_of(n + 1, 256), 256, 0, ctx->stream>>>(keyL, nu, colbits, n,
                                                                          rpL.as<int64_t>());
    }
    LNE_TRY(check_launch(ctx, "sym_bounds"));
    const int64_t nb = ceil_div(n > 0 ? n : 1, 256);
    LNE_TRY(alloc(ctx, len, sizeof(uint32_t) * (size_t)(n > 0 ? n : 1)));
    LNE_TRY(alloc(ctx, rpF, sizeof(uint64_t) * (size_t)(n + 1)));
    LNE_TRY(alloc(ctx, dk, sizeof(uint32_t) * (size_t)nb));
    LNE_TRY(alloc(ctx, dko, sizeof(uint64_t) * (size_t)(nb + 1)));
    {
        Launch L(ctx, "sym_rowlen");
        k_sym_rowlen<float><<<(unsigned)nb, 256, 0, ctx->stream>>>(
            U->row_ptr, U->col, (const float *)U->val, rpL.as<int64_t>(), n,
            len.as<uint32_t>(), dk.as<uint32_t>());
    }
    LNE_TRY(check_launch(ctx, "sym_rowlen"));
    LNE_TRY(scan_u32(ctx, len.as<uint32_t>(), rpF.as<uint64_t>(), n));
    LNE_TRY(scan_u32(ctx, dk.as<uint32_t>(), dko.as<uint64_t>(), nb));
    uint64_t host[2] = {0, 0};
    LNE_HIP(ctx, hipMemcpyAsync(&host[0], rpF.as<uint64_t>() + n, 8, hipMemcpyDeviceToHost,
                                ctx->stream));
    LNE_HIP(ctx, hipMemcpyAsync(&host[1], dko.as<uint64_t>() + nb, 8, hipMemcpyDeviceToHost,
                                ctx->stream));
    LNE_HIP(ctx, hipStreamSynchronize(ctx->stream));
    const int64_t nnz = (int64_t)host[0];
    Buf cF(ctx), vF(ctx);
    LNE_TRY(alloc(ctx, cF, sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1)));
    LNE_TRY(alloc(ctx, vF, sizeof(float) * (size_t)(nnz > 0 ? nnz : 1)));
    if (n > 0) {
        Launch L(ctx, "sym_merge");
        k_sym_merge<float><<<grid_of(n * 64, 256), 256, 0, ctx->stream>>>(
            U->row_ptr, U->col, (const float *)U->val, rpL.as<int64_t>(), keyL, valL, n,
            (1ull << colbits) - 1, rpF.as<uint64_t>(), cF.as<int32_t>(), vF.as<float>());
    }
    LNE_TRY(check_launch(ctx, "sym_merge"));
    // row offsets as int64 (the scan's uint64 offsets have the same bits)
    out->n_rows = n;
    out->n_cols = U->n_cols;
    out->nnz = nnz;
    out->row_ptr = (int64_t *)rpF.detach();
    out->col = (int32_t *)cF.detach();
    out->val = vF.detach();
    out->val_type = LNE_F32;
    *kept = 2 * kept_u - host[1];
    lne_csr_free(ctx, U);
    return LNE_OK;
}

}  // namespace lne
