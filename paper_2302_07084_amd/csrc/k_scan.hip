// Device-wide exclusive prefix sums (uint32 or uint64 in, uint64 out).
// Reduce-then-scan: per-tile totals, a recursive scan of the totals, then a
// tile-local scan offset by its total.  A tile is 4096 items, 16 contiguous
// per thread of a 256-thread block.
#include "common.hpp"

namespace lne {

namespace {

constexpr int kT = 256;
constexpr int kPer = 16;
constexpr int kTile = kT * kPer;

// A thread's kPer items; a full run is read with 16-byte loads when the
// buffers are 16-byte aligned (vec; base is a multiple of kPer).
template <class TI>
__device__ __forceinline__ uint64_t thread_load(const TI *__restrict__ in, int64_t base,
                                                int64_t n, uint64_t v[kPer], bool vec) {
    constexpr int E = 16 / sizeof(TI);   // items per 16-byte load
    uint64_t s = 0;
    if (vec && base + kPer <= n) {
#pragma unroll
        for (int q = 0; q < kPer / E; ++q) {
            const uint4 w = *reinterpret_cast<const uint4 *>(in + base + q * E);
            if constexpr (E == 4) {
                v[4 * q] = w.x; v[4 * q + 1] = w.y; v[4 * q + 2] = w.z; v[4 * q + 3] = w.w;
            } else {
                v[2 * q] = (uint64_t)w.x | ((uint64_t)w.y << 32);
                v[2 * q + 1] = (uint64_t)w.z | ((uint64_t)w.w << 32);
            }
        }
    } else {
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const int64_t idx = base + i;
            v[i] = idx < n ? (uint64_t)in[idx] : 0;
        }
    }
#pragma unroll
    for (int i = 0; i < kPer; ++i) s += v[i];
    return s;
}

// Exclusive scan of one value per thread across the block; returns the
// block total through *total.
__device__ __forceinline__ uint64_t block_exclusive(uint64_t x, uint64_t *total) {
    __shared__ uint64_t wsum[kT / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint64_t inc = x;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint64_t y = __shfl_up(inc, off, 64);
        if (lane >= off) inc += y;
    }
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    uint64_t before = 0, all = 0;
#pragma unroll
    for (int i = 0; i < kT / 64; ++i) {
        if (i < w) before += wsum[i];
        all += wsum[i];
    }
    __syncthreads();
    *total = all;
    return before + inc - x;
}

template <class TI>
__global__ void __launch_bounds__(kT) k_tile_sum(const TI *__restrict__ in, int64_t n,
                                                  uint64_t *__restrict__ sums, int vec) {
    uint64_t v[kPer];
    const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kPer;
    uint64_t s = thread_load(in, base, n, v, vec != 0);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    __shared__ uint64_t ws[kT / 64];
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t t = 0;
        for (int i = 0; i < kT / 64; ++i) t += ws[i];
        sums[blockIdx.x] = t;
    }
}

template <class TI>
__global__ void __launch_bounds__(kT) k_tile_scan(const TI *__restrict__ in, int64_t n,
                                                   const uint64_t *__restrict__ tile_off,
                                                   uint64_t *__restrict__ out, int vec) {
    uint64_t v[kPer];
    const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kPer;
    const uint64_t s = thread_load(in, base, n, v, vec != 0);
    uint64_t total;
    uint64_t run = block_exclusive(s, &total) + (tile_off ? tile_off[blockIdx.x] : 0);
    if (vec && base + kPer <= n) {
        // a full run: two outputs per 16-byte store
#pragma unroll
        for (int q = 0; q < kPer / 2; ++q) {
            const uint64_t a = run;
            run += v[2 * q];
            const uint64_t b = run;
            run += v[2 * q + 1];
            *reinterpret_cast<uint4 *>(out + base + 2 * q) =
                make_uint4((uint32_t)a, (uint32_t)(a >> 32), (uint32_t)b, (uint32_t)(b >> 32));
        }
    } else {
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const int64_t idx = base + i;
            if (idx <= n) out[idx] = run;   // out[n] receives the grand total
            run += v[i];
        }
    }
}

template <class TI>
lne_status scan_impl(lne_ctx *ctx, const TI *in, uint64_t *out, int64_t n) {
    if (n < 0) return fail(ctx, LNE_EINVAL, "scan of negative length");
    // tiles cover items 0..n inclusive so that out[n] is written
    const int64_t tiles = ceil_div(n + 1, kTile);
    const int vec = ((uintptr_t)in % 16 == 0 && (uintptr_t)out % 16 == 0) ? 1 : 0;
    if (tiles == 1) {
        {
            Launch L(ctx, "scan");
            k_tile_scan<TI><<<1, kT, 0, ctx->stream>>>(in, n, nullptr, out, vec);
        }
        return check_launch(ctx, "scan");
    }
    Buf sums(ctx), offs(ctx);
    LNE_TRY(alloc(ctx, sums, sizeof(uint64_t) * (size_t)tiles));
    LNE_TRY(alloc(ctx, offs, sizeof(uint64_t) * (size_t)(tiles + 1)));
    {
        Launch L(ctx, "scan");
        k_tile_sum<TI><<<(unsigned)tiles, kT, 0, ctx->stream>>>(in, n, sums.as<uint64_t>(), vec);
    }
    LNE_TRY(check_launch(ctx, "scan"));
    LNE_TRY(scan_impl<uint64_t>(ctx, sums.as<uint64_t>(), offs.as<uint64_t>(), tiles));
    {
        Launch L(ctx, "scan");
        k_tile_scan<TI><<<(unsigned)tiles, kT, 0, ctx->stream>>>(in, n, offs.as<uint64_t>(),
                                                                 out, vec);
    }
    return check_launch(ctx, "scan");
}

}  // namespace

lne_status scan_u32(lne_ctx *ctx, const uint32_t *in, uint64_t *out, int64_t n) {
    return scan_impl<uint32_t>(ctx, in, out, n);
}
lne_status scan_u64(lne_ctx *ctx, const uint64_t *in, uint64_t *out, int64_t n) {
    return scan_impl<uint64_t>(ctx, in, out, n);
}

}  // namespace lne
