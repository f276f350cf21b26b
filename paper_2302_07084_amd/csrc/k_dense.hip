// Dense steps of the fast randomized SVD (section 4.2): tall-skinny Gram
// products C = Y^T Y and projections Y W on MFMA, and the small FP64 solves
// (Cholesky with inverse, symmetric eigen-decomposition) of eigSVD and
// CholeskyQR2, each in one workgroup so the whole chain stays on the device.
//
// MFMA use (gfx950, 64-lane waves, 16 x 16 output tiles):
//   FP64 / FP32 data: v_mfma_f64_16x16x4f64 (FP32 inputs widened to FP64)
//   BF16 data:        v_mfma_f32_16x16x32_bf16 with FP32 accumulation
// Operand lane layout of a 16 x 16 x K step: lane l supplies A[l % 16][k-block
// l / 16] and B[k-block l / 16][l % 16].  Accumulator value i of lane l is
// column l % 16 of the output tile, row 4 (l / 16) + i for the FP32/BF16
// forms but row l / 16 + 4 i for the FP64 form (checked by a lane probe).
#include <mutex>

#include "common.hpp"

namespace lne {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

template <class T> __device__ __forceinline__ double to_d(T x) { return (double)x; }
template <> __device__ __forceinline__ double to_d<__bf16>(__bf16 x) { return (double)(float)x; }

__device__ __forceinline__ void upper_tile(int t, int nt, int &I, int &J) {
    I = 0;
    while (t >= nt - I) { t -= nt - I; ++I; }
    J = I + t;
}

// ---------------------------------------------------------------- Gram FP64
constexpr int kGramRows = 16;
constexpr int kGramThreads = 512;

// Widest padded k whose upper 16 x 16 tiles fit SPLIT blocks of 8 waves x
// MAXT tiles.
constexpr int gram_kp_max(int maxt, int split) {
    int nt = 1;
    while ((nt + 1) * (nt + 2) / 2 <= 8 * maxt * split) ++nt;
    return 16 * nt;
}

// Two LDS tiles of kGramRows rows: the next tile's loads are issued into
// registers before the matrix-core steps of the current one and stored to
// the other buffer after them, so one block barrier per tile separates them.
// Small tiles (16 rows) keep a block's LDS small enough for three blocks per
// CU at k' <= 144 and two at k' <= 272, so that other blocks' matrix-core
// steps cover each block's barrier and tile turnaround.  SPLIT blocks
// (blockIdx.z) share a row range and split its upper output tiles, so that a
// wide k keeps its accumulators in registers.
template <class YT, int MAXT, int SPLIT>
__global__ void __launch_bounds__(kGramThreads, MAXT <= 6 ? 6 : 2)
k_gram64(const YT *__restrict__ Y, int64_t n, int k, int64_t ld, int KP, int64_t rows_per_wg,
         double *__restrict__ part, const int32_t *__restrict__ skip, int64_t ys) {
    Y += (int64_t)blockIdx.y * ys;
    part += (int64_t)blockIdx.y * gridDim.x * KP * KP;
    if (skip) skip += kFlagStride * blockIdx.y;
    if (skip && *skip == 0) return;
    constexpr int KPM = gram_kp_max(MAXT, SPLIT);
    __shared__ double tile[2][kGramRows * KPM];       // kGramRows x KP each
    // the wave index as a scalar, so that the tile indices below are too
    const int tid = threadIdx.x, lane = tid & 63, w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int nt = KP / 16, ntu = nt * (nt + 1) / 2;
    // a block takes a contiguous run of the upper tiles in row order and each
    // wave a contiguous part of it, so that a wave's tiles mostly share their
    // tile row and its A fragment is read from LDS once per step
    const int cb = (ntu + SPLIT - 1) / SPLIT, cw = (cb + 7) / 8;
    const int t0 = (int)blockIdx.z * cb + w * cw, t1 = min(min(ntu, ((int)blockIdx.z + 1) * cb),
                                                           t0 + cw);
    int TI[MAXT], TJ[MAXT];
    v4d acc[MAXT];
#pragma unroll
    for (int s = 0; s < MAXT; ++s) {
        acc[s] = (v4d){0, 0, 0, 0};
        const int t = t0 + s;
        if (t < t1) upper_tile(t, nt, TI[s], TJ[s]); else { TI[s] = TJ[s] = -1; }
    }
    const int64_t r_begin = (int64_t)blockIdx.x * rows_per_wg;
    const int64_t r_end = min(n, r_begin + rows_per_wg);
    const int kr = lane >> 4, kc = lane & 15;
    // a tile is loaded by whole rows: wave w takes rows w, w + 8, ... and its
    // lanes the row's columns 64 apart (no index division per element)
    constexpr int RPW = kGramRows / 8, CPR = (KPM + 63) / 64, NLD = RPW * CPR;
    auto gload = [&](int64_t r0, YT v[NLD]) {
#pragma unroll
        for (int i = 0; i < RPW; ++i) {
            const int64_t row = r0 + w + 8 * i;
#pragma unroll
            for (int j = 0; j < CPR; ++j) {
                const int c = lane + 64 * j;
                v[i * CPR + j] = (row < r_end && c < k) ? Y[row * ld + c] : (YT)0;
            }
        }
    };
    auto lstore = [&](int buf, const YT v[NLD]) {
#pragma unroll
        for (int i = 0; i < RPW; ++i)
#pragma unroll
            for (int j = 0; j < CPR; ++j) {
                const int c = lane + 64 * j;
                if (c < KP) tile[buf][(w + 8 * i) * KP + c] = to_d(v[i * CPR + j]);
            }
    };
auto mfma_tile = [&](int cur) {
#pragma unroll
        for (int kk = 0; kk < kGramRows; kk += 4) {
            const double *trow = tile[cur] + (kk + kr) * KP + kc;
            double a = 0.0;
#pragma unroll
            for (int s = 0; s < MAXT; ++s) {
                if (TI[s] >= 0) {
                    if (s == 0 || TI[s] != TI[s - 1]) a = trow[16 * TI[s]];
                    const double b = trow[16 * TJ[s]];
                    acc[s] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[s], 0, 0, 0);
                }
            }
        }
    };
    YT v[NLD];
    if (r_begin < r_end) {
        gload(r_begin, v);
        lstore(0, v);
    }
    __syncthreads();
    int cur = 0;
    for (int64_t r0 = r_begin; r0 < r_end; r0 += kGramRows, cur ^= 1) {
        const bool more = r0 + kGramRows < r_end;
        if (more) gload(r0 + kGramRows, v);
        mfma_tile(cur);
        if (more) lstore(cur ^ 1, v);
        __syncthreads();
    }
    double *P = part + (int64_t)blockIdx.x * KP * KP;
#pragma unroll
    for (int s = 0; s < MAXT; ++s) {
        if (TI[s] < 0) continue;
#pragma unroll
        for (int i = 0; i < 4; ++i)
            P[(int64_t)(16 * TI[s] + kr + 4 * i) * KP + 16 * TJ[s] + kc] = acc[s][i];
    }
}

// ---------------------------------------------------------------- Gram BF16
constexpr int kTS = 40;   // LDS row stride (bf16) of the transposed tile: 80 B

constexpr int kBR = 128;           // rows per BF16 Gram tile (four MFMA k-steps)
constexpr int kTS2 = kBR + 8;      // LDS row stride (bf16) of the transposed tile: 272 B
constexpr int kGBThreads = 1024;   // BF16 Gram block: sixteen waves
constexpr int kGBWaves = kGBThreads / 64;

// Loads 8 consecutive bf16 of row `row` from column c (zero beyond k or r_end).
__device__ __forceinline__ v8bf load8(const __bf16 *__restrict__ Y, int64_t ld, int64_t row,
                                      int64_t r_end, int c, int k, bool vec) {
    v8bf v;
    if (row < r_end && vec && c + 8 <= k) {
        v = *reinterpret_cast<const v8bf *>(Y + row * ld + c);
    } else {
#pragma unroll
        for (int i = 0; i < 8; ++i)
            v[i] = (row < r_end && c + i < k) ? Y[row * ld + c + i] : (__bf16)0.0f;
    }
    return v;
}

// BF16 Gram: 128-row tiles read with 16-byte loads (consecutive lanes take
// consecutive rows of one 8-column chunk, so the transposed LDS writes do not
// conflict), four 16 x 16 x 32 MFMA steps per tile and output tile.  Sixteen
// waves share a block, so each holds few output tiles and one block per CU
// has a whole 128-row tile (68 KB at k' = 266) of loads in flight; the
// transposed tile lives in dynamic LDS (KP x kTS2 bf16).  The per-block sums
// are FP32 (the accumulators' own type).  vec: rows are 16-byte aligned
// (ld % 8 == 0, aligned base).
template <int MAXT>
__global__ void __launch_bounds__(kGBThreads)
k_gram_bf16(const __bf16 *__restrict__ Y, int64_t n, int k, int64_t ld, int KP,
            int64_t rows_per_wg, float *__restrict__ part, const int32_t *__restrict__ skip,
            int64_t ys, int vec) {
    Y += (int64_t)blockIdx.y * ys;
    part += (int64_t)blockIdx.y * gridDim.x * KP * KP;
    if (skip) skip += kFlagStride * blockIdx.y;
    if (skip && *skip == 0) return;
    extern __shared__ __attribute__((aligned(16))) __bf16 tt[];   // KP x kTS2, transposed
    // the wave index as a scalar, so that the tile indices below are too
    const int tid = threadIdx.x, lane = tid & 63, w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int nt = KP / 16, ntu = nt * (nt + 1) / 2;
    int TI[MAXT], TJ[MAXT];
    v4f acc[MAXT];
#pragma unroll
    for (int s = 0; s < MAXT; ++s) {
        acc[s] = (v4f){0, 0, 0, 0};
        const int t = w + kGBWaves * s;
        if (t < ntu) upper_tile(t, nt, TI[s], TJ[s]); else { TI[s] = TJ[s] = -1; }
    }
    const int64_t r_begin = (int64_t)blockIdx.x * rows_per_wg;
    const int64_t r_end = min(n, r_begin + rows_per_wg);
    const int kr = lane >> 4, kc = lane & 15;
    const int nch = KP / 8;
    // the next tile's 16-byte chunks are requested into registers before the
    // matrix-core steps of the current one and written to LDS after them
    constexpr int NP = (288 / 8 * kBR + kGBThreads - 1) / kGBThreads;
    v8bf pv[NP];
    auto fetch = [&](int64_t r0) {
#pragma unroll
        for (int u = 0; u < NP; ++u) {
            const int idx = tid + u * kGBThreads;
            if (idx < nch * kBR) pv[u] = load8(Y, ld, r0 + idx % kBR, r_end, (idx / kBR) * 8, k, vec != 0);
        }
    };
    if (r_begin < r_end) fetch(r_begin);
    for (int64_t r0 = r_begin; r0 < r_end; r0 += kBR) {
#pragma unroll
        for (int u = 0; u < NP; ++u) {
            const int idx = tid + u * kGBThreads;
            if (idx < nch * kBR) {
                const int rr = idx % kBR, c = (idx / kBR) * 8;
#pragma unroll
                for (int i = 0; i < 8; ++i) tt[(c + i) * kTS2 + rr] = pv[u][i];
            }
        }
        __syncthreads();
        if (r0 + kBR < r_end) fetch(r0 + kBR);
#pragma unroll
        for (int ks = 0; ks < kBR; ks += 32) {
#pragma unroll
            for (int s = 0; s < MAXT; ++s) {
                if (TI[s] >= 0) {
                    const v8bf a =
                        *reinterpret_cast<const v8bf *>(tt + (16 * TI[s] + kc) * kTS2 + ks + 8 * kr);
                    const v8bf b =
                        *reinterpret_cast<const v8bf *>(tt + (16 * TJ[s] + kc) * kTS2 + ks + 8 * kr);
                    acc[s] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[s], 0, 0, 0);
                }
            }
        }
        __syncthreads();
    }
    float *P = part + (int64_t)blockIdx.x * KP * KP;
#pragma unroll
    for (int s = 0; s < MAXT; ++s) {
        if (TI[s] < 0) continue;
#pragma unroll
        for (int i = 0; i < 4; ++i)
            P[(int64_t)(16 * TI[s] + 4 * kr + i) * KP + 16 * TJ[s] + kc] = acc[s][i];
    }
}

// G = sum of the per-workgroup upper partial Grams, mirrored.  A block sums
// 64 consecutive entries (a, b), b >= a, of one row a: its four waves take
// the workgroups w = q mod 4, two running sums each, combined in a fixed
// order (the result does not depend on the launch).
constexpr int kRedThreads = 256;
template <class PT>
__global__ void __launch_bounds__(kRedThreads)
k_gram_reduce(const PT *__restrict__ part, int nwg, int KP, int k, double *__restrict__ G,
              const int32_t *__restrict__ skip) {
    part += (int64_t)blockIdx.y * nwg * KP * KP;
    G += (int64_t)blockIdx.y * k * k;
    if (skip) skip += kFlagStride * blockIdx.y;
    if (skip && *skip == 0) return;
    const int nbc = (k + 63) / 64;
    const int a = (int)blockIdx.x / nbc, b = ((int)blockIdx.x % nbc) * 64 + (threadIdx.x & 63);
    const int q = threadIdx.x >> 6;
    __shared__ double sums[4][64];
    double s0 = 0.0, s1 = 0.0;
    if (b >= a && b < k) {
        const PT *pa = part + (int64_t)a * KP + b;
        const int64_t step = (int64_t)KP * KP;
        int w = q;
        for (; w + 4 < nwg; w += 8) {
            s0 += (double)pa[w * step];
            s1 += (double)pa[(w + 4) * step];
        }
        if (w < nwg) s0 += (double)pa[w * step];
    }
    sums[q][threadIdx.x & 63] = s0 + s1;
    __syncthreads();
    if (q == 0 && b >= a && b < k) {
        const int l = threadIdx.x;
        const double g = (sums[0][l] + sums[1][l]) + (sums[2][l] + sums[3][l]);
        G[(int64_t)a * k + b] = g;
        G[(int64_t)b * k + a] = g;
    }
}

// ---------------------------------------------------------------- projection
constexpr int kProjRows = 128;
constexpr int kProjThreads = 512;
constexpr int kKC = 16;           // K chunk (FP64 path)
constexpr int kAS = kKC + 1;      // padded LDS row stride (doubles)

// Four consecutive elements of row `row` from column c as doubles (zero
// beyond k or n); vec: 16-byte (FP32) or 2 x 16-byte (FP64) loads allowed.
template <class YT>
__device__ __forceinline__ void load4d(const YT *__restrict__ Y, int64_t ld, int64_t row,
                                       int64_t n, int c, int k, bool vec, double out[4]) {
    if (row < n && vec && c + 4 <= k) {
        if constexpr (sizeof(YT) == 4) {
            const float4 v = *reinterpret_cast<const float4 *>(Y + row * ld + c);
            out[0] = v.x; out[1] = v.y; out[2] = v.z; out[3] = v.w;
        } else {
            const double2 v0 = *reinterpret_cast<const double2 *>(Y + row * ld + c);
            const double2 v1 = *reinterpret_cast<const double2 *>(Y + row * ld + c + 2);
            out[0] = v0.x; out[1] = v0.y; out[2] = v1.x; out[3] = v1.y;
        }
    } else {
#pragma unroll
        for (int i = 0; i < 4; ++i)
            out[i] = (row < n && c + i < k) ? to_d(Y[row * ld + c + i]) : 0.0;
    }
}

// FP64-MFMA projection out = Y W.  Each 16 x 16 x 4 step sums over four k;
// lane group kr takes k = k0 + 4 kr + t in step t, so a lane's A operands for
// a 16-wide k chunk are four consecutive elements of its row, read with one
// vector load; the chunk of W is staged in LDS.
template <class YT, class OT, int MAXJ>
__global__ void __launch_bounds__(kProjThreads, MAXJ <= 3 ? 6 : 2)
k_proj64(const YT *__restrict__ Y, int64_t ldy, int64_t n, int kin,
         const double *__restrict__ W, int kout, OT *__restrict__ out, int64_t ldo,
         const int32_t *__restrict__ skip, int64_t ys, int64_t ws, int64_t os, int vec) {
    Y += (int64_t)blockIdx.y * ys;
    W += (int64_t)blockIdx.y * ws;
    out += (int64_t)blockIdx.y * os;
    if (skip) skip += kFlagStride * blockIdx.y;
    if (skip && *skip == 0) return;
    // two W chunks in LDS: chunk i + 1 is loaded into registers before the
    // matrix-core steps of chunk i and stored to the other buffer after them,
    // so one block barrier per chunk separates the two
    constexpr int KPo = 16 * MAXJ;
    constexpr int kWn = (kKC * KPo + kProjThreads - 1) / kProjThreads;
    __shared__ double Ws[2][kKC * KPo];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    // blockIdx.z takes output column tiles jz .. jz + MAXJ - 1
    const int jz = (int)blockIdx.z * MAXJ, cz = 16 * jz;
    const int ntout = min(MAXJ, (kout + 15) / 16 - jz);
    const int64_t r0 = (int64_t)blockIdx.x * kProjRows;
    const int kr = lane >> 4, kc = lane & 15;
    const int64_t arow = r0 + 16 * w + kc;
    auto wload = [&](int k0, double wr[kWn]) {
#pragma unroll
        for (int u = 0; u < kWn; ++u) {
            const int idx = tid + u * kProjThreads;
            const int rr = idx / KPo, c = idx - rr * KPo;
            const int krow = k0 + rr;
            wr[u] = (idx < kKC * KPo && krow < kin && cz + c < kout)
                        ? W[(int64_t)krow * kout + cz + c]
                        : 0.0;
        }
    };
    auto wstore = [&](int buf, const double wr[kWn]) {
#pragma unroll
        for (int u = 0; u < kWn; ++u) {
            const int idx = tid + u * kProjThreads;
            if (idx < kKC * KPo) Ws[buf][idx] = wr[u];
        }
    };
    v4d acc[MAXJ];
#pragma unroll
    for (int J = 0; J < MAXJ; ++J) acc[J] = (v4d){0, 0, 0, 0};
    double wr[kWn], a4[4];
    wload(0, wr);
    load4d<YT>(Y, ldy, arow, n, 4 * kr, kin, vec != 0, a4);
    wstore(0, wr);
    __syncthreads();
    for (int k0 = 0, cur = 0; k0 < kin; k0 += kKC, cur ^= 1) {
        const bool more = k0 + kKC < kin;
        double a4n[4];
        if (more) {
            wload(k0 + kKC, wr);
            load4d<YT>(Y, ldy, arow, n, k0 + kKC + 4 * kr, kin, vec != 0, a4n);
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
#pragma unroll
            for (int J = 0; J < MAXJ; ++J) {
                if (J < ntout) {
                    const double b = Ws[cur][(4 * kr + t) * KPo + 16 * J + kc];
                    acc[J] = __builtin_amdgcn_mfma_f64_16x16x4f64(a4[t], b, acc[J], 0, 0, 0);
                }
            }
        }
        if (more) {
            wstore(cur ^ 1, wr);
#pragma unroll
            for (int i = 0; i < 4; ++i) a4[i] = a4n[i];
        }
        __syncthreads();
    }
#pragma unroll
    for (int J = 0; J < MAXJ; ++J) {
        if (J >= ntout) continue;
        const int c = cz + 16 * J + kc;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t row = r0 + 16 * w + kr + 4 * i;
            if (row < n && c < kout) out[row * ldo + c] = (OT)acc[J][i];
        }
    }
}

// BF16 projection: each lane reads its A operand (8 consecutive k of one
// row) straight from memory with one 16-byte load; the 32-k slice of W^T is
// staged in LDS, double-buffered: the next step's operand and W slice are
// requested into registers before the current step's matrix-core steps and
// the slice is stored to the other buffer after them, one barrier per step.
template <class OT, int MAXJ>
__global__ void __launch_bounds__(kProjThreads)
k_proj_bf16(const __bf16 *__restrict__ Y, int64_t ldy, int64_t n, int kin,
            const __bf16 *__restrict__ Wt, int ldw, int kout, OT *__restrict__ out,
            int64_t ldo, const int32_t *__restrict__ skip, int64_t ys, int64_t os, int vec) {
    Y += (int64_t)blockIdx.y * ys;
    Wt += (int64_t)blockIdx.y * kout * ldw;
    out += (int64_t)blockIdx.y * os;
    if (skip) skip += kFlagStride * blockIdx.y;
    if (skip && *skip == 0) return;
    __shared__ __attribute__((aligned(16))) __bf16 Ws[2][16 * MAXJ * kTS];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int ntout = (kout + 15) / 16;
    const int64_t r0 = (int64_t)blockIdx.x * kProjRows;
    const int kr = lane >> 4, kc = lane & 15;
    const int64_t arow = r0 + 16 * w + kc;
    // a thread's share of one W slice: 16 MAXJ columns x 4 chunks of 8 k
    constexpr int NW = (16 * MAXJ * 4 + kProjThreads - 1) / kProjThreads;
    auto wload = [&](int k0, v8bf v[NW]) {
#pragma unroll
        for (int u = 0; u < NW; ++u) {
            const int idx = tid + u * kProjThreads;
            const int c = idx >> 2, kcol = k0 + (idx & 3) * 8;
            if (idx >= 16 * MAXJ * 4) continue;
            if (c < kout && kcol + 8 <= kin) {
                v[u] = *reinterpret_cast<const v8bf *>(Wt + (int64_t)c * ldw + kcol);
            } else {
#pragma unroll
                for (int i = 0; i < 8; ++i)
                    v[u][i] = (c < kout && kcol + i < kin) ? Wt[(int64_t)c * ldw + kcol + i]
                                                           : (__bf16)0.0f;
            }
        }
    };
    auto wstore = [&](int buf, const v8bf v[NW]) {
#pragma unroll
        for (int u = 0; u < NW; ++u) {
            const int idx = tid + u * kProjThreads;
            if (idx < 16 * MAXJ * 4)
                *reinterpret_cast<v8bf *>(Ws[buf] + (idx >> 2) * kTS + (idx & 3) * 8) = v[u];
        }
    };
    v4f acc[MAXJ];
#pragma unroll
    for (int J = 0; J < MAXJ; ++J) acc[J] = (v4f){0, 0, 0, 0};
    v8bf wv[NW];
    wload(0, wv);
    wstore(0, wv);
    v8bf a = load8(Y, ldy, arow, n, 8 * kr, kin, vec != 0);
    __syncthreads();
    int cur = 0;
    for (int k0 = 0; k0 < kin; k0 += 32, cur ^= 1) {
        const bool more = k0 + 32 < kin;
        v8bf an = a;
        if (more) {
            an = load8(Y, ldy, arow, n, k0 + 32 + 8 * kr, kin, vec != 0);
            wload(k0 + 32, wv);
        }
#pragma unroll
        for (int J = 0; J < MAXJ; ++J) {
            if (J < ntout) {
                const v8bf b =
                    *reinterpret_cast<const v8bf *>(Ws[cur] + (16 * J + kc) * kTS + 8 * kr);
                acc[J] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[J], 0, 0, 0);
            }
        }
        if (more) wstore(cur ^ 1, wv);
        __syncthreads();
        a = an;
    }
#pragma unroll
    for (int J = 0; J < MAXJ; ++J) {
        if (J >= ntout) continue;
        const int c = 16 * J + kc;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t row = r0 + 16 * w + 4 * kr + i;
            if (row < n && c < kout) out[row * ldo + c] = (OT)acc[J][i];
        }
    }
}

__global__ void k_w_to_bf16t(const double *__restrict__ W, int kin, int kout,
                             __bf16 *__restrict__ Wt, int ldw, int64_t ws) {
    W += (int64_t)blockIdx.y * ws;
    Wt += (int64_t)blockIdx.y * kout * ldw;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)kin * kout) return;
    const int i = (int)(t / kout), c = (int)(t % kout);
    Wt[(int64_t)c * ldw + i] = (__bf16)(float)W[t];
}

// ---------------------------------------------------------------- Cholesky
constexpr int kSolveThreads = 1024;
constexpr int kEigMaxK = 288;   // widest k of the Cholesky and eigen-solver kernels

// Right-looking upper Cholesky of A (k x k, in place; LDS or global).
// Returns false on a pivot that is not positive relative to the original
// diagonal.  The trailing update takes rows by wave and columns by lane.
__device__ bool chol_upper(double *A, int k, const double *diag0) {
    __shared__ int bad;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    constexpr int NW = kSolveThreads / 64;
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    for (int j = 0; j < k; ++j) {
        const double piv = A[(int64_t)j * k + j];
        const bool ok = piv > 1e-14 * diag0[j] && piv > 0.0 && isfinite(piv);
        if (!ok) {
            if (threadIdx.x == 0) bad = 1;
            __syncthreads();
            return false;
        }
        const double r = sqrt(piv);
        __syncthreads();
        for (int c = j + 1 + threadIdx.x; c < k; c += kSolveThreads) A[(int64_t)j * k + c] /= r;
        if (threadIdx.x == 0) A[(int64_t)j * k + j] = r;
        __syncthreads();
        for (int i = j + 1 + wv; i < k; i += NW) {
            const double aji = A[(int64_t)j * k + i];
            for (int c = i + lane; c < k; c += 64)
                A[(int64_t)i * k + c] -= aji * A[(int64_t)j * k + c];
        }
        __syncthreads();
    }
    return bad == 0;
}

// Cholesky of the Gram G = R^T R (a shifted retry if a pivot fails) and W =
// R^-1.  IN_LDS: the k x k matrix is factored in LDS (k <= kCholMaxLds), then
// W is formed there row by row while R is read from G.  The inverse takes
// the rows from the bottom up, all columns of a row at once; each entry is
// the sum over j ascending of R[i][j] W[j][c], as a column-by-column
// back-substitution forms it.
constexpr int kCholMaxLds = 140;
template <bool IN_LDS>
__global__ void __launch_bounds__(kSolveThreads)
k_chol_inv(double *__restrict__ G, int k, double *__restrict__ W, double *__restrict__ diag0,
           int32_t *__restrict__ status, int32_t *__restrict__ shifted, int64_t n_rows,
           const int32_t *__restrict__ skip, int32_t *__restrict__ run_next) {
    extern __shared__ double lds_m[];
    {
        const int64_t b = blockIdx.x;
        G += b * k * k;
        W += b * k * k;
        diag0 += b * k;
        status += kFlagStride * b;
        shifted += kFlagStride * b;
        if (skip) skip += kFlagStride * b;
        if (run_next) run_next += kFlagStride * b;
    }
    if (skip && *skip == 0) {
        if (run_next && threadIdx.x == 0) *run_next = 0;
        return;
    }
    const int64_t kk = (int64_t)k * k;
    __shared__ double trace;
    double *A = IN_LDS ? lds_m : G;
    for (int64_t i = threadIdx.x; i < kk; i += kSolveThreads) {
        W[i] = G[i];
        if (IN_LDS) A[i] = G[i];
    }
    for (int i = threadIdx.x; i < k; i += kSolveThreads) diag0[i] = G[(int64_t)i * k + i];
    __syncthreads();
    bool ok = chol_upper(A, k, diag0);
    bool sh = false;
    if (!ok) {
        // shifted retry: G + sigma I, sigma = 11 (n k + k (k + 1)) u trace(G)
        if (threadIdx.x == 0) {
            double t = 0.0;
            for (int i = 0; i < k; ++i) t += diag0[i];
            trace = t;
        }
        __syncthreads();
        const double sigma = 11.0 * ((double)n_rows * k + (double)k * (k + 1)) *
                             1.1102230246251565e-16 * trace;
        for (int64_t i = threadIdx.x; i < kk; i += kSolveThreads)
            A[i] = W[i] + ((i / k == i % k) ? sigma : 0.0);
        __syncthreads();
        for (int i = threadIdx.x; i < k; i += kSolveThreads) diag0[i] = 0.0;
        __syncthreads();
        ok = chol_upper(A, k, diag0);
        sh = true;
    }
    if (threadIdx.x == 0) {
        if (!ok) *status = 1;
        if (sh) atomicAdd(shifted, 1);
        if (run_next) *run_next = sh ? 1 : 0;
    }
    // R (upper; its lower triangle zero) to G
    for (int64_t i = threadIdx.x; i < kk; i += kSolveThreads)
        G[i] = (i / k > i % k) ? 0.0 : A[i];
    __syncthreads();
    // W = R^-1 (upper), in LDS for the LDS variant (A is free now); row i of
    // R is staged in LDS for its step
    __shared__ double rrow[kEigMaxK];   // the widest k accepted
    double *Wm = IN_LDS ? lds_m : W;
    for (int i = k - 1; i >= 0; --i) {
        for (int j = i + threadIdx.x; j < k; j += kSolveThreads) rrow[j] = G[(int64_t)i * k + j];
        __syncthreads();
        const double rii = rrow[i];
        for (int c = threadIdx.x; c < k; c += kSolveThreads) {
            double x;
            if (c < i) {
                x = 0.0;
            } else if (c == i) {
                x = ok ? 1.0 / rii : 0.0;
            } else {
                // the products' operands four at a time (loads ahead of the
                // still sequential sum)
                double s = 0.0;
                int j = i + 1;
                for (; j + 3 <= c; j += 4) {
                    const double r0 = rrow[j], r1 = rrow[j + 1], r2 = rrow[j + 2], r3 = rrow[j + 3];
                    const double w0 = Wm[(int64_t)j * k + c], w1 = Wm[(int64_t)(j + 1) * k + c];
                    const double w2 = Wm[(int64_t)(j + 2) * k + c], w3 = Wm[(int64_t)(j + 3) * k + c];
                    s += r0 * w0;
                    s += r1 * w1;
                    s += r2 * w2;
                    s += r3 * w3;
                }
                for (; j <= c; ++j) s += rrow[j] * Wm[(int64_t)j * k + c];
                x = ok ? -s / rii : 0.0;
            }
            Wm[(int64_t)i * k + c] = x;
        }
        __syncthreads();
    }
    if constexpr (IN_LDS)
        for (int64_t i = threadIdx.x; i < kk; i += kSolveThreads) W[i] = Wm[i];
}

// ---------------------------------------------------------------- eigen-solver
// Symmetric eigen-decomposition of a k x k matrix by one workgroup, in three
// phases (Householder reduction to tridiagonal form, the tridiagonal
// eigen-problem, the reflectors applied to its eigenvectors):
//  1. k - 2 Householder steps.  Step j reflects the entries of column j below
//     the subdiagonal to zero: with x = A[j+1.., j], beta = -sign(x0) |x|,
//     v = (1, x1 / (x0 - beta), ...), tau = (beta - x0) / beta, the trailing
//     block becomes A - v w^T - w v^T with p = tau A v, w = p - (tau/2)(p.v) v.
//     v is written into row j (which later steps never touch).  The two
//     products of the rank-2 update are rounded separately, so the block
//     stays exactly symmetric.
//  2. The tridiagonal matrix (d, e): implicit QL sweeps (Wilkinson's shift)
//     chase the shifted bulge from the bottom of an unreduced block to its
//     top with plane rotations.  One wave computes a sweep's rotations while
//     other waves apply the previous sweep's rotations to the eigenvector
//     rows (two rotation buffers, one block barrier per sweep); each of their
//     lanes owns one component of every eigenvector.  From kEigSplit on, the
//     matrix is first torn in two halves plus a rank-one term (Cuppen), the
//     halves are swept side by side by two waves, and a merge solves the
//     rank-one problem (its comment gives the steps).
//  3. Every wave takes whole eigenvectors (in registers) and applies the
//     reflectors k-3 .. 0 to them without block barriers, then writes them to
//     V in order of decreasing eigenvalue.
// IN_LDS: A (and then the reflectors) lives in LDS (k^2 doubles of dynamic
// shared memory); otherwise it is worked on in place in global memory.  The
// eigenvectors of the tridiagonal matrix are kept transposed in Zt (row i =
// eigenvector i), so a rotation of eigenvectors (i, i+1) reads two rows; the
// workspace Zt holds 2 k^2 doubles (the merge writes its rows to the second
// half) and V serves as the merge's scratch before it receives the result.
constexpr int kEigMaxLds = 144;   // largest k of the LDS variant
constexpr int kEigSplit = 32;   // tear the tridiagonal matrix from this size on

// A double moved between lanes by a DPP pattern (both halves).
template <int CTRL>
__device__ inline double dpp_d(double x) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}

__device__ inline double readlane_d(double x, int l) {
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(x), l),
                            __builtin_amdgcn_readlane(__double2loint(x), l));
}

// Sum over a fully active wave, the same bits in every lane: pairs, quads,
// half rows and rows by DPP (each step adds two equal sums in either order),
// then the four row sums read from lanes 0, 16, 32 and 48.
__device__ inline double wave_sum(double x) {
    x += dpp_d<0xB1>(x);    // quad_perm [1, 0, 3, 2]
    x += dpp_d<0x4E>(x);    // quad_perm [2, 3, 0, 1]
    x += dpp_d<0x141>(x);   // row_half_mirror
    x += dpp_d<0x140>(x);   // row_mirror
    return (readlane_d(x, 0) + readlane_d(x, 16)) + (readlane_d(x, 32) + readlane_d(x, 48));
}

// Serial QL state of the producing wave.
struct QlState {
    int l = 0;      // eigenvalues 0 .. l-1 have converged
    int iter = 0;   // sweeps spent on eigenvalue l
};

// The rotations of one QL sweep, rows m-1 up to l, from the values (d, e)
// held when the sweep started: lane j keeps entries 64 q + j in D[q], E[q]
// and the serial chain reads them by lane index; lane 0 stores the new d, e
// and the rotations (rc, rs at the index of their upper row).  The matrix is
// scaled to unit size, so f^2 + g^2 is a normal number unless both are
// negligible (below 2^-500), which is where the sweep must deflate instead.
// CHECK = false runs the chain with no branch on that test and returns -2 if
// it failed anywhere (the stored values are then void); CHECK = true returns
// the row at which it deflated, or -1 when the sweep completed.
template <int R, bool CHECK>
__device__ int ql_chain(const double (&D)[R], const double (&E)[R], int l, int m, double g,
                        double dn, double dl, double *d, double *e, double *rc, double *rs,
                        bool w0) {
    double s = 1.0, c = 1.0, p = 0.0;
    bool bad = false;
    // segments of 64 rows from the bottom, each reading its own registers
    // (q is a constant in each unrolled copy)
#pragma unroll
    for (int q = R - 1; q >= 0; --q) {
        if (q > ((m - 1) >> 6) || q < (l >> 6)) continue;
        const double Dq = D[q], Eq = E[q];
        const int ilo = l > 64 * q ? l : 64 * q;
        for (int i = (m - 1 < 64 * q + 63 ? m - 1 : 64 * q + 63); i >= ilo; --i) {
            const double di = readlane_d(Dq, i - 64 * q), ei = readlane_d(Eq, i - 64 * q);
            const double f = s * ei, b = c * ei;
            const double x = fma(f, f, g * g);
            if constexpr (CHECK) {
                if (!(x >= 0x1p-1000)) {   // both vanished: deflate at i + 1
                    if (w0) {
                        e[i + 1] = 0.0;
                        d[i + 1] = dn - p;
                        e[m] = 0.0;
                    }
                    return i;
                }
            } else {
                bad |= !(x >= 0x1p-1000);
            }
            // 1/sqrt(x) by the hardware estimate and two Newton steps, the
            // last step's product folded into c, s and r
            const double h = 0.5 * x, y0 = __builtin_amdgcn_rsq(x);
            const double y1 = y0 * fma(-h * y0, y0, 1.5);
            const double u2 = fma(-h * y1, y1, 1.5);
            c = (g * y1) * u2;
            s = (f * y1) * u2;
            const double gp = dn - p;
            const double r2 = fma(di - gp, s, (2.0 * b) * c);
            p = s * r2;
            g = fma(c, r2, -b);
            if (w0) {
                e[i + 1] = (x * y1) * u2;
                d[i + 1] = gp + p;
                rc[i] = c;
                rs[i] = s;
            }
            dn = di;
        }
    }
    if (!CHECK && bad) return -2;
    if (w0) {
        d[l] = dl - p;
        e[l] = g;
        e[m] = 0.0;
    }
    return -1;
}

// One QL sweep on (d, e) (length-k diagonal and coupling e[i] between i and
// i+1, e[k-1] = 0), run by a whole wave computing the same values.  Returns
// false once every eigenvalue has converged; else the sweep's rotations are
// in rc, rs over [*lo, *hi).
template <int R>
__device__ bool ql_sweep(double *d, double *e, int k, QlState &st, double *rc, double *rs,
                         int *lo, int *hi, int lane) {
    const double eps = 2.220446049250313e-16;
    const bool w0 = lane == 0;
    while (st.l < k) {
        const int l = st.l;
        double D[R], E[R];
        int m = k - 1;
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int j = 64 * q + lane;
            D[q] = j < k ? d[j] : 0.0;
            E[q] = j < k ? e[j] : 0.0;
            const double dn = j + 1 < k ? d[j + 1] : 0.0;
            // the first coupling at or after l that is negligible
            const bool split = j >= l && j < k - 1 && fabs(E[q]) <= eps * (fabs(D[q]) + fabs(dn));
            const uint64_t bal = __ballot(split);
            if (bal && m == k - 1) m = 64 * q + __builtin_ctzll(bal);
        }
        if (m == l) {
            st.l = l + 1;
            st.iter = 0;
            continue;
        }
        if (st.iter++ >= 64) {   // not expected: give up on this coupling
            if (w0) e[l] = 0.0;
            __builtin_amdgcn_wave_barrier();
            continue;
        }
        const double dl = d[l], dl1 = d[l + 1], el = e[l], dm = d[m];
        // shift: the eigenvalue of the leading 2 x 2 block nearer d[l]
        double g = (dl1 - dl) / (2.0 * el);
        const double r = hypot(g, 1.0);
        g = dm - dl + el / (g + (g >= 0.0 ? r : -r));
        int at = ql_chain<R, false>(D, E, l, m, g, dm, dl, d, e, rc, rs, w0);
        if (at == -2) {
            // put the sweep's starting values back, then take the checked path
#pragma unroll
            for (int q = 0; q < R; ++q) {
                const int j = 64 * q + lane;
                if (j < k) { d[j] = D[q]; e[j] = E[q]; }
            }
            __builtin_amdgcn_wave_barrier();
            at = ql_chain<R, true>(D, E, l, m, g, dm, dl, d, e, rc, rs, w0);
        }
        __builtin_amdgcn_wave_barrier();
        *lo = at >= 0 ? at + 1 : l;
        *hi = m;
        if (*lo < *hi) return true;
    }
    return false;
}

template <bool IN_LDS>
__global__ void __launch_bounds__(kSolveThreads)
k_sym_eig(double *__restrict__ Ag, int k, double *__restrict__ Zt, double *__restrict__ V,
          double *__restrict__ lam) {
    constexpr int MK = IN_LDS ? kEigMaxLds : kEigMaxK;
    extern __shared__ double lds_a[];
    __shared__ double dg[MK], eg[MK], taus[MK];
    __shared__ double buf[4 * MK];   // p of a Householder step, then the rotation buffers
    __shared__ int s_lo[2][2], s_hi[2][2], s_more[2][2];   // [problem][buffer]
    __shared__ int idx[2 * MK];                             // merge: order, kept and deflated rows
    __shared__ double s_rho, s_unit, s_tol;
    __shared__ int s_K, s_flip;
    {
        const int64_t b = blockIdx.x;
        Ag += b * k * k;
        Zt += b * 2 * k * k;
        V += b * k * k;
        lam += b * k;
    }
    // the wave index as a scalar, so that code under `w == 0` branches as a
    // uniform wave
    const int tid = threadIdx.x, lane = tid & 63, w = __builtin_amdgcn_readfirstlane(tid >> 6);
    constexpr int NW = kSolveThreads / 64;
    double *__restrict__ A = Ag;
    if constexpr (IN_LDS) {
        for (int64_t i = tid; i < (int64_t)k * k; i += kSolveThreads) lds_a[i] = Ag[i];
        A = lds_a;
    }
    for (int64_t i = tid; i < (int64_t)k * k; i += kSolveThreads)
        Zt[i] = (i / k == i % k) ? 1.0 : 0.0;
    __syncthreads();

    // ---- 1. Householder reduction.  Per step: every wave forms the
    // reflector from row j; threads (row i, part q) sum parts of p = tau A v;
    // thread i < m finishes p_i and writes v_i into row j (where phase 3
    // reads it back, first entry 1); threads (column l, row group g) apply
    // the rank-2 update.  Three block barriers per step.
    constexpr int P = kSolveThreads / MK < 4 ? kSolveThreads / MK : 4;   // parts per row sum
    constexpr int G = kSolveThreads / MK;                                 // row groups
    double *pq = buf;   // P x MK partial sums, then p (row 0) and v (row 1)
    for (int j = 0; j + 2 < k; ++j) {
        const int m = k - j - 1;   // trailing indices j+1 .. k-1
        double *x = A + (int64_t)j * k + j + 1;
        double sg = 0.0;
        for (int l = 1 + lane; l < m; l += 64) sg += x[l] * x[l];
        sg = wave_sum(sg);
        const double x0 = x[0];
        if (tid == 0) dg[j] = A[(int64_t)j * k + j];
        if (sg == 0.0) {   // already reduced: H = I
            if (tid == 0) { eg[j] = x0; taus[j] = 0.0; }
            continue;
        }
        const double beta = -copysign(sqrt(x0 * x0 + sg), x0);
        const double tau = (beta - x0) / beta, sc = 1.0 / (x0 - beta);
        if (tid == 0) { eg[j] = beta; taus[j] = tau; }
        {
            const int i = tid % MK, q = tid / MK, L = (m + P - 1) / P;
            if (q < P && i < m) {
                // A[j+1+l][j+1+i] = A[j+1+i][j+1+l]: lanes read along a row
                const double *col = A + (int64_t)(j + 1) * k + j + 1 + i;
                const int l1 = m < (q + 1) * L ? m : (q + 1) * L;
                double acc0 = 0.0, acc1 = 0.0;
                int l = q * L;
                if (l == 0) { acc0 = col[0]; l = 1; }
                for (; l + 1 < l1; l += 2) {
                    acc0 += col[(int64_t)l * k] * (x[l] * sc);
                    acc1 += col[(int64_t)(l + 1) * k] * (x[l + 1] * sc);
                }
                if (l < l1) acc0 += col[(int64_t)l * k] * (x[l] * sc);
                pq[q * MK + i] = acc0 + acc1;
            }
        }
        __syncthreads();
        if (tid < m) {
            double ps = 0.0;
            for (int q = 0; q < P; ++q) ps += pq[q * MK + tid];
            const double v = tid == 0 ? 1.0 : x[tid] * sc;
            pq[tid] = tau * ps;
            pq[MK + tid] = v;
            x[tid] = v;
        }
        __syncthreads();
        double pd = 0.0;
        for (int l = lane; l < m; l += 64) pd += pq[l] * pq[MK + l];
        const double K = 0.5 * tau * wave_sum(pd);
        {
            const int l = tid % MK, g = tid / MK;
            if (g < G && l < m) {
                const double vl = pq[MK + l], wl = pq[l] - K * vl;
                double *colp = A + (int64_t)(j + 1) * k + j + 1 + l;
#pragma unroll 4
                for (int i = g; i < m; i += G) {
                    const double vi = pq[MK + i], wi = pq[i] - K * vi;
                    colp[(int64_t)i * k] -= __dadd_rn(__dmul_rn(vi, wl), __dmul_rn(wi, vl));
                }
            }
        }
        __syncthreads();
    }
    if (tid == 0) {
        for (int j = (k >= 2 ? k - 2 : 0); j < k; ++j) dg[j] = A[(int64_t)j * k + j];
        if (k >= 2) eg[k - 2] = A[(int64_t)(k - 2) * k + k - 1];
        eg[k - 1] = 0.0;
        s_more[0][0] = s_more[0][1] = s_more[1][0] = s_more[1][1] = 0;
    }
    __syncthreads();

    // ---- 2. eigen-decomposition of the tridiagonal matrix T = (d, e).
    // Wave 0 scales (d, e) by a power of two to unit size (exact).  For
    // k >= kEigSplit, T is torn at h = k/2 into blockdiag(T1, T2) + rho w w^T
    // (w = e_{h-1} + e_h, rho the coupling, taken off d[h-1] and d[h]); waves
    // 0 and 1 run the QL sweeps of T1 and T2 side by side while waves 2..
    // apply each problem's previous sweep to its block of eigenvector rows
    // (component c by thread c; rotation buffer b: cosines at buf + 2 MK b,
    // sines MK further, indexed by global row).  The merge below then solves
    // the rank-one problem.  Smaller k: one problem, waves 1.. apply.
    const int h = k >= kEigSplit ? k / 2 : k;
    const int np = h < k ? 2 : 1;
    if (w == 0) {
        double amax = 0.0;
        for (int i = lane; i < k; i += 64) amax = fmax(amax, fmax(fabs(dg[i]), fabs(eg[i])));
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) amax = fmax(amax, __shfl_xor(amax, o, 64));
        double unit = 1.0;
        if (amax > 0.0 && isfinite(amax)) {
            unit = ldexp(1.0, -ilogb(amax));
            for (int i = lane; i < k; i += 64) { dg[i] *= unit; eg[i] *= unit; }
        }
        __builtin_amdgcn_wave_barrier();
        if (lane == 0) {
            s_unit = unit;
            s_rho = 0.0;
            if (np == 2) {
                const double rho = eg[h - 1];
                dg[h - 1] -= rho;
                dg[h] -= rho;
                eg[h - 1] = 0.0;
                s_rho = rho;
            }
        }
    }
    __syncthreads();
    {
        QlState st;
        for (int t = 0;; ++t) {
            const int b = t & 1;
            if (w < np) {
                const int base = w == 0 ? 0 : h, n = w == 0 ? h : k - h;
                int lo = 0, hi = 0;
                double *cb = buf + 2 * MK * b + base;
                const bool more = ql_sweep<(MK + 63) / 64>(dg + base, eg + base, n, st, cb,
                                                          cb + MK, &lo, &hi, lane);
                if (lane == 0) {
                    s_more[w][b] = more ? 1 : 0;
                    s_lo[w][b] = base + lo;
                    s_hi[w][b] = base + hi;
                }
            }
            const int pb = b ^ 1;
            const int kk = tid - 64 * np;
            const int pr = kk >= h ? 1 : 0;
            if (t > 0 && kk >= 0 && kk < k && s_more[pr][pb]) {
                const int lo = s_lo[pr][pb], hi = s_hi[pr][pb];
                const double *c = buf + 2 * MK * pb, *s = c + MK;
                double carry = Zt[(int64_t)hi * k + kk];
                // rotations hi-1 .. lo, loads of up to 16 rows issued ahead
                for (int i0 = hi - 1; i0 >= lo; i0 -= 16) {
                    double z[16];
                    const int cnt = i0 - lo + 1 < 16 ? i0 - lo + 1 : 16;
#pragma unroll
                    for (int u = 0; u < 16; ++u)
                        if (u < cnt) z[u] = Zt[(int64_t)(i0 - u) * k + kk];
#pragma unroll
                    for (int u = 0; u < 16; ++u)
                        if (u < cnt) {
                            const int i = i0 - u;
                            Zt[(int64_t)(i + 1) * k + kk] = s[i] * z[u] + c[i] * carry;
                            carry = c[i] * z[u] - s[i] * carry;
                        }
                }
                Zt[(int64_t)lo * k + kk] = carry;
            }
            __syncthreads();
            if (!s_more[0][b] && !s_more[1][b]) break;
        }
    }
    const double *Zv = Zt;   // the eigenvector rows phase 3 starts from
    if (np == 1) {
        for (int i = tid; i < k; i += kSolveThreads) dg[i] /= s_unit;
    } else {
        // ---- merge: eigenvalues and eigenvectors of D + rho z z^T, D the
        // eigenvalues of T1 and T2, z the rows h-1 / h of their eigenvectors.
        // Deflation (a negligible weight, or two poles whose rotation
        // leaves a negligible coupling), then per root a bisection of the
        // secular equation 1 + rho sum z_i^2 / (d_i - lambda) = 0 in its
        // interval between poles (its distance to the nearer pole kept as
        // (origin, tau) so that differences stay accurate), weights
        // recomputed from the roots (Gu and Eisenstat) so that the
        // eigenvectors z_i / (d_i - lambda_j) come out orthogonal, and the
        // new rows Zt2 = U Zt[kept] (U in V as scratch).
        double *Zt2 = Zt + (int64_t)k * k;
        double *Ut = V;
        int *ord = idx, *kept = idx + MK;
        double *dk = buf, *zk = buf + MK, *tau = buf + 2 * MK, *zh = buf + 3 * MK;
        for (int i = tid; i < k; i += kSolveThreads)
            eg[i] = i < h ? Zt[(int64_t)i * k + h - 1] : Zt[(int64_t)i * k + h];
        __syncthreads();
        if (w == 0) {
            double zz = 0.0, dmax = 0.0;
            for (int i = lane; i < k; i += 64) {
                zz += eg[i] * eg[i];
                dmax = fmax(dmax, fabs(dg[i]));
            }
            zz = wave_sum(zz);
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) dmax = fmax(dmax, __shfl_xor(dmax, o, 64));
            if (lane == 0) {
                const double rt = s_rho * zz;
                s_flip = rt < 0.0 ? 1 : 0;
                s_rho = fabs(rt);
                s_tol = 8.0 * 2.220446049250313e-16 * fmax(dmax, fabs(rt));
                zh[0] = zz > 0.0 ? 1.0 / sqrt(zz) : 0.0;
            }
        }
        __syncthreads();
        {
            const double sz = zh[0];
            const bool flip = s_flip != 0;
            for (int i = tid; i < k; i += kSolveThreads) {
                eg[i] *= sz;
                if (flip) dg[i] = -dg[i];
            }
        }
        __syncthreads();
        // ascending order of the poles (ties by index)
        for (int i = tid; i < k; i += kSolveThreads) {
            const double di = dg[i];
            int r = 0;
            for (int j = 0; j < k; ++j) r += (dg[j] < di || (dg[j] == di && j < i)) ? 1 : 0;
            ord[r] = i;
        }
        __syncthreads();
        // deflation, in pole order, by wave 0
        if (w == 0) {
            const double rho = s_rho, tol = s_tol;
            int K = 0, nd = 0, prev = -1;
            for (int sidx = 0; sidx < k; ++sidx) {
                const int i = ord[sidx];
                const double zi = eg[i];
                if (rho * fabs(zi) <= tol) {
                    if (lane == 0) kept[k - 1 - nd] = i;
                    ++nd;
                    continue;
                }
                if (prev >= 0) {
                    const double zp = eg[prev], dp = dg[prev], di = dg[i];
                    const double r = hypot(zp, zi);
                    const double c = zi / r, sn = zp / r;
                    if (fabs(c * sn * (di - dp)) <= tol) {
                        // rotate rows prev, i so that prev's weight vanishes
                        for (int cc = lane; cc < k; cc += 64) {
                            const double a = Zt[(int64_t)prev * k + cc], bb = Zt[(int64_t)i * k + cc];
                            Zt[(int64_t)prev * k + cc] = c * a - sn * bb;
                            Zt[(int64_t)i * k + cc] = sn * a + c * bb;
                        }
                        if (lane == 0) {
                            dg[prev] = c * c * dp + sn * sn * di;
                            dg[i] = sn * sn * dp + c * c * di;
                            eg[i] = r;
                            eg[prev] = 0.0;
                            kept[k - 1 - nd] = prev;
                        }
                        __builtin_amdgcn_wave_barrier();
                        ++nd;
                        prev = i;
                        continue;
                    }
                    if (lane == 0) kept[K] = prev;
                    ++K;
                }
                prev = i;
            }
            if (prev >= 0) {
                if (lane == 0) kept[K] = prev;
                ++K;
            }
            if (lane == 0) s_K = K;
        }
        __syncthreads();
        const int K = s_K;
        const double rho = s_rho;
        for (int j = tid; j < K; j += kSolveThreads) {
            dk[j] = dg[kept[j]];
            zk[j] = eg[kept[j]];
        }
        __syncthreads();
        // roots: lambda_j in (dk_j, dk_j+1), the last in (dk_K-1, dk_K-1 +
        // rho |z|^2].  Four lanes per root (partial sums over every fourth
        // pole, quad sums by DPP); Newton steps on the secular function
        // inside its bracket, a bisection step whenever Newton leaves it.
        for (int j0 = 0; j0 < K; j0 += kSolveThreads / 4) {
            const int j = j0 + (tid >> 2), sub = tid & 3;
            if (j < K) {
                // 1 + rho sum z^2 / delta and its derivative, delta_i =
                // (dk_i - dk_o) - t
                auto secular = [&](int oo, double tt, double &der) {
                    double f = 0.0, g = 0.0;
                    for (int i = sub; i < K; i += 4) {
                        const double r = 1.0 / ((dk[i] - dk[oo]) - tt);
                        const double a2 = zk[i] * zk[i] * r;
                        f += a2;
                        g += a2 * r;
                    }
                    f += dpp_d<0xB1>(f);
                    f += dpp_d<0x4E>(f);
                    g += dpp_d<0xB1>(g);
                    g += dpp_d<0x4E>(g);
                    der = rho * g;
                    return 1.0 + rho * f;
                };
                int o;
                double lo, hi, der;
                if (j < K - 1) {
                    const double gap = dk[j + 1] - dk[j];
                    if (secular(j, 0.5 * gap, der) >= 0.0) { o = j; lo = 0.0; hi = 0.5 * gap; }
                    else { o = j + 1; lo = -0.5 * gap; hi = 0.0; }
                } else {
                    double zz = 0.0;
                    for (int i = 0; i < K; ++i) zz += zk[i] * zk[i];
                    o = j; lo = 0.0; hi = rho * zz;
                }
                double t = 0.5 * (lo + hi);
                for (int it = 0; it < 200; ++it) {
                    const double f = secular(o, t, der);
                    if (f == 0.0) break;
                    if (f < 0.0) lo = t; else hi = t;
                    double tn = t - f / der;
                    if (!(tn > lo && tn < hi)) tn = 0.5 * (lo + hi);
                    const bool done = !(tn > lo && tn < hi) ||
                                      fabs(tn - t) <= 4.440892098500626e-16 * fabs(tn);
                    if (!(tn > lo && tn < hi)) break;
                    t = tn;
                    if (done) break;
                }
                if (sub == 0) {
                    ord[j] = o;
                    tau[j] = t;
                }
            }
        }
        __syncthreads();
        // recomputed weights: zh_i^2 = prod_j (lambda_j - dk_i) / (rho prod_l!=i (dk_l - dk_i))
        for (int i = tid; i < K; i += kSolveThreads) {
            auto lmd = [&](int j) { return (dk[ord[j]] - dk[i]) + tau[j]; };   // lambda_j - dk_i
            double P = lmd(K - 1) / rho;
            for (int j = 0; j < i; ++j) P *= lmd(j) / (dk[j] - dk[i]);
            for (int j = i; j < K - 1; ++j) P *= lmd(j) / (dk[j + 1] - dk[i]);
            zh[i] = copysign(sqrt(fmax(P, 0.0)), zk[i]);
        }
        __syncthreads();
        // eigenvectors of the rank-one problem (rows of Ut), and the new
        // eigenvalues (unscaled, sign restored) next to the deflated ones
        {
            const double sgn = s_flip ? -1.0 : 1.0, un = s_unit;
            for (int j = tid; j < K; j += kSolveThreads) {
                const double dj = dk[ord[j]], tj = tau[j];
                double nrm = 0.0;
                for (int i = 0; i < K; ++i) {
                    const double u = zh[i] / ((dk[i] - dj) - tj);
                    nrm += u * u;
                }
                const double inv = 1.0 / sqrt(nrm);
                for (int i = 0; i < K; ++i) Ut[(int64_t)j * K + i] = zh[i] / ((dk[i] - dj) - tj) * inv;
            }
            __syncthreads();
            // zk is free now: the final eigenvalues
            for (int j = tid; j < k; j += kSolveThreads)
                zk[j] = sgn * (j < K ? dk[ord[j]] + tau[j] : dg[kept[j]]) / un;
        }
        __syncthreads();
        for (int j = tid; j < k; j += kSolveThreads) dg[j] = zk[j];
        // new rows: Zt2[j] = sum_i Ut[j][i] Zt[kept_i] (j < K); the deflated
        // rows are copied.  4 x 4 output tiles per thread.
        {
            const int nt4 = (k + 3) / 4;
            for (int tt = tid; tt < nt4 * nt4; tt += kSolveThreads) {
                const int j0 = (tt / nt4) * 4, c0 = (tt % nt4) * 4;
                double acc[4][4];
#pragma unroll
                for (int a4 = 0; a4 < 4; ++a4)
#pragma unroll
                    for (int b4 = 0; b4 < 4; ++b4) acc[a4][b4] = 0.0;
                const int jn = K - j0;   // rows of this tile that are sums
                if (jn > 0) {
                    for (int i = 0; i < K; ++i) {
                        const double *zr = Zt + (int64_t)kept[i] * k + c0;
                        double zv[4], uv[4];
#pragma unroll
                        for (int b4 = 0; b4 < 4; ++b4) zv[b4] = c0 + b4 < k ? zr[b4] : 0.0;
#pragma unroll
                        for (int a4 = 0; a4 < 4; ++a4)
                            uv[a4] = a4 < jn ? Ut[(int64_t)(j0 + a4) * K + i] : 0.0;
#pragma unroll
                        for (int a4 = 0; a4 < 4; ++a4)
#pragma unroll
                            for (int b4 = 0; b4 < 4; ++b4) acc[a4][b4] += uv[a4] * zv[b4];
                    }
                }
#pragma unroll
                for (int a4 = 0; a4 < 4; ++a4) {
                    const int j = j0 + a4;
                    if (j >= k) break;
#pragma unroll
                    for (int b4 = 0; b4 < 4; ++b4) {
                        const int c = c0 + b4;
                        if (c >= k) break;
                        Zt2[(int64_t)j * k + c] = j < K ? acc[a4][b4] : Zt[(int64_t)kept[j] * k + c];
                    }
                }
            }
        }
        __syncthreads();
        Zv = Zt2;
    }

    // ---- 3. reflectors applied to each eigenvector, then sorted output.  A
    // wave takes three eigenvectors at a time (three independent sums per
    // reflector); reflector j is row j of A from column j + 1 on.
    constexpr int R = (MK + 63) / 64;
    for (int c0 = w; c0 < k; c0 += 3 * NW) {
        double z[3][R];
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            const int c = c0 + r * NW;
#pragma unroll
            for (int q = 0; q < R; ++q) {
                const int i = lane + 64 * q;
                z[r][q] = c < k && i < k ? Zv[(int64_t)c * k + i] : 0.0;
            }
        }
        for (int j = k - 3; j >= 0; --j) {
            const double tau = taus[j];
            if (tau == 0.0) continue;
            double v[R];
#pragma unroll
            for (int q = 0; q < R; ++q) {
                const int i = lane + 64 * q;
                v[q] = i > j && i < k ? A[(int64_t)j * k + i] : 0.0;
            }
            double f[3];
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                double dot = 0.0;
#pragma unroll
                for (int q = 0; q < R; ++q) dot += v[q] * z[r][q];
                f[r] = dot;
            }
#pragma unroll
            for (int r = 0; r < 3; ++r) f[r] = tau * wave_sum(f[r]);
#pragma unroll
            for (int r = 0; r < 3; ++r)
#pragma unroll
                for (int q = 0; q < R; ++q) z[r][q] -= f[r] * v[q];
        }
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            const int c = c0 + r * NW;
            if (c >= k) break;
            // rank by decreasing eigenvalue, ties by index
            const double lc = dg[c];
            int rank = 0;
            for (int j0 = 0; j0 < k; j0 += 64) {
                const int j = j0 + lane;
                const bool before = j < k && (dg[j] > lc || (dg[j] == lc && j < c));
                rank += __popcll(__ballot(before));
            }
            if (lane == 0) lam[rank] = lc;
#pragma unroll
            for (int q = 0; q < R; ++q) {
                const int i = lane + 64 * q;
                if (i < k) V[(int64_t)i * k + rank] = z[r][q];
            }
        }
    }
}

__global__ void k_eig_weights(const double *__restrict__ V, const double *__restrict__ lam,
                              int k, int kout, double power, double *__restrict__ W,
                              double *__restrict__ S, const int32_t *__restrict__ on) {
    const int64_t b = blockIdx.y;
    V += b * k * k;
    lam += b * k;
    if (W) W += b * k * kout;
    if (S) S += b * kout;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (on && on[b] == 0) {
        // pass-through entry: identity weights
        if (W && t < (int64_t)k * kout) W[t] = (t / kout == t % kout) ? 1.0 : 0.0;
        if (S && t < kout) S[t] = 1.0;
        return;
    }
    const double lmax = lam[0] > 0.0 ? lam[0] : 0.0;
    const double floor_ = (double)k * 2.220446049250313e-16 * lmax;
    if (S && t < kout) {
        const double l = lam[t];
        S[t] = l > floor_ ? sqrt(l) : 0.0;
    }
    if (W && t < (int64_t)k * kout) {
        const int i = (int)(t / kout), c = (int)(t % kout);
        const double l = lam[c];
        W[t] = l > floor_ ? V[(int64_t)i * k + c] * pow(l, power) : 0.0;
    }
}

}  // namespace

// ---------------------------------------------------------------- host side
// Lets `fn` use `bytes` of dynamic LDS (above the default 64 KB), once per
// kernel; fails when the device offers less.
static lne_status lds_opt_in(lne_ctx *ctx, const void *fn, size_t bytes) {
    static std::mutex mu;
    static std::map<const void *, size_t> done;
    std::lock_guard<std::mutex> lock(mu);
    auto it = done.find(fn);
    if (it != done.end() && it->second >= bytes) return LNE_OK;
    if (bytes > 64 * 1024 &&
        hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) !=
            hipSuccess) {
        (void)hipGetLastError();
        return fail(ctx, LNE_EUNSUPPORTED, "%zu bytes of LDS per block are not available", bytes);
    }
    done[fn] = bytes;
    return LNE_OK;
}

size_t project_bf16_ws_bytes(int32_t kin, int32_t kout, int32_t nb) {
    return sizeof(__bf16) * (size_t)nb * kout * (((kin + 31) / 32) * 32);
}

lne_status gram(lne_ctx *ctx, const void *Y, int32_t dtype, int64_t n, int32_t k, int64_t ld,
                double *G, const int32_t *skip, int32_t nb, int64_t ys, double *part_ws,
                size_t part_ws_bytes) {
    if (k < 1) return fail(ctx, LNE_EINVAL, "gram: k = %d", k);
    const int KP = ((k + 15) / 16) * 16;
    const int nt = KP / 16, ntu = nt * (nt + 1) / 2;
    const int per_wave = (ntu + 7) / 8;
    if (per_wave > 22) return fail(ctx, LNE_EUNSUPPORTED, "gram: k = %d above 288", k);
    if (nb < 1 || nb > 65535) return fail(ctx, LNE_EINVAL, "gram: batch of %d", nb);
    // BF16: row ranges in whole 128-row tiles, one sixteen-wave block per CU
    const bool bf = dtype == LNE_BF16;
    const int rows_unit = bf ? kBR : kGramRows;
    const int64_t blocks_rows = ceil_div(n > 0 ? n : 1, rows_unit);
    // about 768 (512 for wide k, 256 for BF16) workgroups over the whole
    // batch, one round of three (two, one) blocks per CU, or as many
    // per-workgroup partial sums as a caller's workspace holds
    int64_t target = std::max<int64_t>(1, (bf ? 256 : KP > 160 ? 512 : 768) / nb);
    // per-workgroup sums: FP32 for BF16 data (its accumulators), else FP64
    const size_t part_es = dtype == LNE_BF16 ? sizeof(float) : sizeof(double);
    const size_t part_one = part_es * (size_t)nb * KP * KP;
    if (part_ws) {
        if (part_ws_bytes < part_one)
            return fail(ctx, LNE_EUNSUPPORTED, "gram: workspace of %zu bytes below %zu",
                        part_ws_bytes, part_one);
        target = std::min<int64_t>(target, (int64_t)(part_ws_bytes / part_one));
    }
    const int nwg = (int)std::min<int64_t>(blocks_rows, target);
    const int64_t rows_per_wg = ceil_div(blocks_rows, nwg) * rows_unit;
    Buf part(ctx);
    if (part_ws) part.p = part_ws, part.ctx = nullptr;   // borrowed: never released
    else LNE_TRY(alloc(ctx, part, part_one * nwg));
    const dim3 grid((unsigned)nwg, (unsigned)nb);
    const int vec = ((uintptr_t)Y % 16 == 0 && ld % 8 == 0 && ys % 8 == 0) ? 1 : 0;
    {
        Launch L(ctx, "gram");
        if (bf) {
            const int bpw = (ntu + kGBWaves - 1) / kGBWaves;
            const size_t lds = sizeof(__bf16) * (size_t)KP * kTS2;
#define LNE_GB(MT)                                                                         \
    do {                                                                                   \
        LNE_TRY(lds_opt_in(ctx, (const void *)k_gram_bf16<MT>, lds));                      \
        k_gram_bf16<MT><<<grid, kGBThreads, lds, ctx->stream>>>(                           \
            (const __bf16 *)Y, n, k, ld, KP, rows_per_wg, part.as<float>(), skip, ys, vec); \
    } while (0)
            if (bpw <= 1) LNE_GB(1);
            else if (bpw <= 6) LNE_GB(6);
            else if (bpw <= 10) LNE_GB(10);
            else LNE_GB(12);
#undef LNE_GB
        } else {
#define LNE_G64(T, MT, SP)                                                               \
    k_gram64<T, MT, SP><<<dim3(grid.x, grid.y, SP), kGramThreads, 0, ctx->stream>>>(   \
        (const T *)Y, n, k, ld, KP, rows_per_wg, part.as<double>(), skip, ys)
            if (dtype == LNE_F64) {
                if (per_wave <= 1) LNE_G64(double, 1, 1);
                else if (per_wave <= 6) LNE_G64(double, 6, 1);
                else if (per_wave <= 12) LNE_G64(double, 12, 1);
                else LNE_G64(double, 11, 2);
            } else {
                if (per_wave <= 1) LNE_G64(float, 1, 1);
                else if (per_wave <= 6) LNE_G64(float, 6, 1);
                else if (per_wave <= 12) LNE_G64(float, 12, 1);
                else LNE_G64(float, 11, 2);
            }
#undef LNE_G64
        }
    }
    LNE_TRY(check_launch(ctx, "gram"));
    {
        Launch L(ctx, "gram_reduce");
        const dim3 rgrid((unsigned)(k * ((k + 63) / 64)), (unsigned)nb);
        if (dtype == LNE_BF16)
            k_gram_reduce<float><<<rgrid, kRedThreads, 0, ctx->stream>>>(part.as<float>(), nwg, KP,
                                                                         k, G, skip);
        else
            k_gram_reduce<double><<<rgrid, kRedThreads, 0, ctx->stream>>>(part.as<double>(), nwg,
                                                                          KP, k, G, skip);
    }
    return check_launch(ctx, "gram_reduce");
}

lne_status project(lne_ctx *ctx, const void *Y, int32_t y_t, int64_t ldy, int64_t n,
                   int32_t kin, const double *W, int32_t kout, void *out, int32_t out_t,
                   int64_t ldo, const int32_t *skip, int32_t nb, int64_t ys, int64_t ws,
                   int64_t os, void *wt_ws) {
    if (kout > 288 || kin > 288) return fail(ctx, LNE_EUNSUPPORTED, "project: width above 288");
    if (nb < 1 || nb > 65535) return fail(ctx, LNE_EINVAL, "project: batch of %d", nb);
    const dim3 grid(grid_of(n > 0 ? n : 1, kProjRows), (unsigned)nb);
    const int ntout = (kout + 15) / 16;
    if (y_t == LNE_BF16) {
        const int ldw = ((kin + 31) / 32) * 32;
        const int vec = ((uintptr_t)Y % 16 == 0 && ldy % 8 == 0 && ys % 8 == 0) ? 1 : 0;
        Buf wt(ctx);
        // wt_ws (if given) holds project_bf16_ws_bytes(kin, kout, nb)
        if (wt_ws) wt.p = wt_ws, wt.ctx = nullptr;
        else LNE_TRY(alloc(ctx, wt, project_bf16_ws_bytes(kin, kout, nb)));
        {
            Launch L(ctx, "w_to_bf16");
            k_w_to_bf16t<<<dim3(grid_of((int64_t)kin * kout, 256), (unsigned)nb), 256, 0,
                           ctx->stream>>>(W, kin, kout, wt.as<__bf16>(), ldw, ws);
        }
        LNE_TRY(check_launch(ctx, "w_to_bf16"));
        Launch L(ctx, "project");
#define LNE_PB(OT, MJ)                                                                     \
    k_proj_bf16<OT, MJ><<<grid, kProjThreads, 0, ctx->stream>>>(                           \
        (const __bf16 *)Y, ldy, n, kin, wt.as<__bf16>(), ldw, kout, (OT *)out, ldo, skip, ys, os, \
        vec)
        if (out_t == LNE_BF16) {
            if (ntout <= 3) LNE_PB(__bf16, 3);
            else if (ntout <= 9) LNE_PB(__bf16, 9);
            else LNE_PB(__bf16, 18);
        } else if (out_t == LNE_F32) {
            if (ntout <= 3) LNE_PB(float, 3);
            else if (ntout <= 9) LNE_PB(float, 9);
            else LNE_PB(float, 18);
        } else {
            return fail(ctx, LNE_EINVAL, "project: bf16 input needs bf16/f32 output");
        }
#undef LNE_PB
    } else {
        const int vmul = y_t == LNE_F64 ? 2 : 4;
        const int vec = ((uintptr_t)Y % 16 == 0 && ldy % vmul == 0 && ys % vmul == 0) ? 1 : 0;
        Launch L(ctx, "project");
        // at most 9 output column tiles per block: a wider output is split
        // over blockIdx.z (fewer accumulators per wave, so that two blocks
        // share a CU and cover each other's barriers; at k' <= 144 a split
        // costs more in repeated Y reads and spills than it gains)
#define LNE_P64(YT, OT, MJ)                                                                \
    k_proj64<YT, OT, MJ><<<dim3(grid.x, grid.y, (unsigned)((ntout + (MJ) - 1) / (MJ))),  \
                           kProjThreads, 0, ctx->stream>>>(                                \
        (const YT *)Y, ldy, n, kin, W, kout, (OT *)out, ldo, skip, ys, ws, os, vec)
#define LNE_P64J(YT, OT)                                                                   \
    do {                                                                                   \
        if (ntout <= 3) LNE_P64(YT, OT, 3);                                                \
        else LNE_P64(YT, OT, 9);                                                           \
    } while (0)
        if (y_t == LNE_F64 && out_t == LNE_F64) LNE_P64J(double, double);
        else if (y_t == LNE_F32 && out_t == LNE_F32) LNE_P64J(float, float);
        else if (y_t == LNE_F32 && out_t == LNE_F64) LNE_P64J(float, double);
        else if (y_t == LNE_F64 && out_t == LNE_F32) LNE_P64J(double, float);
        else return fail(ctx, LNE_EINVAL, "project: unsupported types");
#undef LNE_P64J
#undef LNE_P64
    }
    return check_launch(ctx, "project");
}

lne_status chol_inv(lne_ctx *ctx, double *G, int32_t k, double *W, int32_t *status,
                    int32_t *shifted, int64_t n_rows, const int32_t *skip, int32_t *skip_next,
                    int32_t nb) {
    if (k < 1 || k > kEigMaxK) return fail(ctx, LNE_EUNSUPPORTED, "chol_inv: k = %d", k);
    Buf diag(ctx);
    LNE_TRY(alloc(ctx, diag, sizeof(double) * (size_t)nb * k));
    // the LDS variant when k^2 doubles fit beside the kernel's static arrays
    static int lds_limit = -1;
    if (lds_limit < 0) {
        int dev = 0, bytes = 0, base = 0;
        lds_limit = 0;
        hipFuncAttributes fa;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&base, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) ==
                hipSuccess &&
            hipDeviceGetAttribute(&bytes, hipDeviceAttributeSharedMemPerBlockOptin, dev) ==
                hipSuccess &&
            hipFuncGetAttributes(&fa, (const void *)k_chol_inv<true>) == hipSuccess &&
            (bytes = bytes > base ? bytes : base) > (int)fa.sharedSizeBytes &&
            hipFuncSetAttribute((const void *)k_chol_inv<true>,
                                hipFuncAttributeMaxDynamicSharedMemorySize,
                                bytes - (int)fa.sharedSizeBytes) == hipSuccess)
            lds_limit = bytes - (int)fa.sharedSizeBytes;
        (void)hipGetLastError();
    }
    const size_t need = sizeof(double) * (size_t)k * k;
    {
        Launch L(ctx, "chol_inv");
        if (k <= kCholMaxLds && need <= (size_t)lds_limit)
            k_chol_inv<true><<<nb, kSolveThreads, need, ctx->stream>>>(
                G, k, W, diag.as<double>(), status, shifted, n_rows, skip, skip_next);
        else
            k_chol_inv<false><<<nb, kSolveThreads, 0, ctx->stream>>>(
                G, k, W, diag.as<double>(), status, shifted, n_rows, skip, skip_next);
    }
    return check_launch(ctx, "chol_inv");
}

size_t sym_eig_ws_doubles(int32_t k, int32_t nb) { return (size_t)nb * 2 * k * k; }

lne_status sym_eig(lne_ctx *ctx, double *C, int32_t k, double *V, double *lam, int32_t nb,
                   double *vw_ws) {
    if (k > kEigMaxK) return fail(ctx, LNE_EUNSUPPORTED, "sym_eig: k = %d above %d", k, kEigMaxK);
    Buf vw(ctx);
    // vw_ws (if given) holds sym_eig_ws_doubles(k, nb) doubles
    if (vw_ws) vw.p = vw_ws, vw.ctx = nullptr;
    else LNE_TRY(alloc(ctx, vw, sizeof(double) * sym_eig_ws_doubles(k, nb)));
    // the LDS variant when k^2 doubles fit next to the kernel's static arrays
    static int lds_limit = -1;
    if (lds_limit < 0) {
        int dev = 0, bytes = 0;
        lds_limit = 0;
        int base = 0;
        hipFuncAttributes fa;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&base, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) ==
                hipSuccess &&
            hipDeviceGetAttribute(&bytes, hipDeviceAttributeSharedMemPerBlockOptin, dev) ==
                hipSuccess &&
            hipFuncGetAttributes(&fa, (const void *)k_sym_eig<true>) == hipSuccess &&
            (bytes = bytes > base ? bytes : base) > (int)fa.sharedSizeBytes &&
            hipFuncSetAttribute((const void *)k_sym_eig<true>,
                                hipFuncAttributeMaxDynamicSharedMemorySize,
                                bytes - (int)fa.sharedSizeBytes) == hipSuccess)
            lds_limit = bytes - (int)fa.sharedSizeBytes;
        (void)hipGetLastError();
    }
    const size_t need = sizeof(double) * (size_t)k * k;
    if (k <= kEigMaxLds && need <= (size_t)lds_limit) {
        Launch L(ctx, "sym_eig");
        k_sym_eig<true><<<nb, kSolveThreads, need, ctx->stream>>>(C, k, vw.as<double>(), V, lam);
    } else {
        Launch L(ctx, "sym_eig");
        k_sym_eig<false><<<nb, kSolveThreads, 0, ctx->stream>>>(C, k, vw.as<double>(), V, lam);
    }
    return check_launch(ctx, "sym_eig");
}

lne_status eig_weights(lne_ctx *ctx, const double *V, const double *lam, int32_t k,
                       int32_t kout, double power, double *W, double *S, int32_t nb,
                       const int32_t *on) {
    if (on && k != kout) return fail(ctx, LNE_EINVAL, "eig_weights: pass-through needs k == kout");
    {
        Launch L(ctx, "eig_weights");
        k_eig_weights<<<dim3(grid_of((int64_t)k * kout, 256), (unsigned)nb), 256, 0,
                        ctx->stream>>>(V, lam, k, kout, power, W, S, on);
    }
    return check_launch(ctx, "eig_weights");
}

}  // namespace lne
