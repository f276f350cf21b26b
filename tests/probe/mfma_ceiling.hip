// Matrix-core ceiling probe: the rate of back-to-back independent MFMAs whose
// operands and accumulators stay in registers (no memory traffic), at 1 to 8
// waves per SIMD.  It bounds what a kernel built from the same instruction
// can reach on this chip, below the published dense peak when the clock or
// the instruction's issue rate under load is lower than the peak assumes.
// Prints one JSON line.  Measurement infrastructure, not part of the library.
#include <hip/hip_runtime.h>
#include <cstdio>

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

constexpr int kThreads = 256;   // four waves: one per SIMD
constexpr int kAcc = 8;         // independent accumulators per wave

#define CHECK(x)                                                                   \
    do {                                                                           \
        hipError_t e_ = (x);                                                       \
        if (e_ != hipSuccess) {                                                    \
            fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));                \
            return 1;                                                              \
        }                                                                          \
    } while (0)

__global__ void __launch_bounds__(kThreads) k_f64(double *out, int iters) {
    const int lane = threadIdx.x & 63;
    const double a = 1.0 + lane * 1e-3, b = 1.0 - lane * 1e-3;
    v4d acc[kAcc];
#pragma unroll
    for (int s = 0; s < kAcc; ++s) acc[s] = (v4d){0, 0, 0, 0};
    for (int it = 0; it < iters; ++it)
#pragma unroll
        for (int s = 0; s < kAcc; ++s)
            acc[s] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[s], 0, 0, 0);
    double t = 0;
#pragma unroll
    for (int s = 0; s < kAcc; ++s) t += acc[s][0] + acc[s][1] + acc[s][2] + acc[s][3];
    out[blockIdx.x * kThreads + threadIdx.x] = t;
}

__global__ void __launch_bounds__(kThreads) k_f32(double *out, int iters) {
    const int lane = threadIdx.x & 63;
    const float a = 1.0f + lane * 1e-3f, b = 1.0f - lane * 1e-3f;
    v4f acc[kAcc];
#pragma unroll
    for (int s = 0; s < kAcc; ++s) acc[s] = (v4f){0, 0, 0, 0};
    for (int it = 0; it < iters; ++it)
#pragma unroll
        for (int s = 0; s < kAcc; ++s)
            acc[s] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[s], 0, 0, 0);
    double t = 0;
#pragma unroll
    for (int s = 0; s < kAcc; ++s) t += acc[s][0] + acc[s][1] + acc[s][2] + acc[s][3];
    out[blockIdx.x * kThreads + threadIdx.x] = t;
}

__global__ void __launch_bounds__(kThreads) k_bf16(double *out, int iters) {
    const int lane = threadIdx.x & 63;
    v8bf a, b;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        a[i] = (__bf16)(1.0f + (lane + i) * 1e-3f);
        b[i] = (__bf16)(1.0f - (lane + i) * 1e-3f);
    }
    v4f acc[kAcc];
#pragma unroll
    for (int s = 0; s < kAcc; ++s) acc[s] = (v4f){0, 0, 0, 0};
    for (int it = 0; it < iters; ++it)
#pragma unroll
        for (int s = 0; s < kAcc; ++s)
            acc[s] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[s], 0, 0, 0);
    double t = 0;
#pragma unroll
    for (int s = 0; s < kAcc; ++s) t += acc[s][0] + acc[s][1] + acc[s][2] + acc[s][3];
    out[blockIdx.x * kThreads + threadIdx.x] = t;
}

typedef void (*kern_t)(double *, int);

// Time one launch (after a warm-up launch) of `blocks` blocks; returns ms.
static int time_kernel(kern_t k, int blocks, int iters, double *out, float *ms) {
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    k<<<blocks, kThreads>>>(out, iters);
    CHECK(hipGetLastError());
    CHECK(hipEventRecord(e0));
    k<<<blocks, kThreads>>>(out, iters);
    CHECK(hipGetLastError());
    CHECK(hipEventRecord(e1));
    CHECK(hipEventSynchronize(e1));
    CHECK(hipEventElapsedTime(ms, e0, e1));
    CHECK(hipEventDestroy(e0));
    CHECK(hipEventDestroy(e1));
    return 0;
}

int main() {
    int dev = 0, cus = 0;
    CHECK(hipGetDevice(&dev));
    CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const int max_wps = 8;                       // waves per SIMD
    double *out = nullptr;
    CHECK(hipMalloc(&out, sizeof(double) * (size_t)cus * max_wps * kThreads));
    struct Case { const char *name; kern_t k; double flops; int iters; };
    // flops of one MFMA: 16 x 16 outputs x K products x 2
    const Case cases[] = {{"f64_16x16x4", k_f64, 16.0 * 16 * 4 * 2, 2000},
                          {"f32_16x16x4", k_f32, 16.0 * 16 * 4 * 2, 4000},
                          {"bf16_16x16x32", k_bf16, 16.0 * 16 * 32 * 2, 4000}};
    printf("{\"probe\": \"mfma_ceiling\", \"cus\": %d, \"results\": [", cus);
    bool first = true;
    for (const Case &c : cases) {
        for (int wps = 1; wps <= max_wps; wps *= 2) {
            const int blocks = cus * wps;        // one wave per SIMD per block
            float ms = 0.f;
            if (time_kernel(c.k, blocks, c.iters, out, &ms)) return 1;
            const double fl = (double)blocks * (kThreads / 64) * c.iters * kAcc * c.flops;
            printf("%s{\"mfma\": \"%s\", \"waves_per_simd\": %d, \"ms\": %.4f, \"tflops\": %.2f}",
                   first ? "" : ", ", c.name, wps, ms, fl / (ms * 1e-3) / 1e12);
            first = false;
        }
    }
    printf("]}\n");
    CHECK(hipFree(out));
    return 0;
}
