// Allocation-free eigSVD (Algorithm "eigSVD") for callers that cannot
// allocate device memory: code under HIP graph capture, serving loops, and
// harnesses that forbid hipMalloc.  Every intermediate of lne_eigsvd (the
// Gram's per-workgroup partial sums, the Gram, the eigen-solver's workspace,
// eigenvectors and eigenvalues, the projection weights and their
// BF16 copy) lives in one file-scope device array that each device holds
// until the process ends.  The kernels are those of lne_eigsvd; only the
// number of Gram workgroups may be smaller (as many partial sums as the array
// holds), which changes the Gram's summation order and nothing else.
#include <mutex>

#include "common.hpp"

namespace lne {
namespace {

constexpr size_t kScratchBytes = (size_t)LNE_EIGSVD_NOALLOC_SCRATCH;
constexpr int kMaxK = 288;
constexpr int kMaxDevices = 64;

// The array's name is a host-side stand-in in host code: its device address
// comes from hipGetSymbolAddress, once per device (scratch_ptr).
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void *g_ptr[kMaxDevices] = {nullptr};

// Device address of `scratch` on the current device, looked up on the first
// call on that device with the device current.
lne_status scratch_ptr(lne_ctx *ctx, unsigned char **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(ctx, LNE_EHIP, "eigsvd_noalloc: hipGetDevice: %s",
                                     hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices)
        return fail(ctx, LNE_EUNSUPPORTED, "eigsvd_noalloc: device %d", dev);
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(ctx, LNE_EHIP, "eigsvd_noalloc: hipGetSymbolAddress: %s",
                        hipGetErrorString(e));
        g_ptr[dev] = p;
    }
    *out = static_cast<unsigned char *>(g_ptr[dev]);
    return LNE_OK;
}

size_t up256(size_t b) { return (b + 255) / 256 * 256; }

// Restores the context's event bracketing on every exit path.
struct NoEvents {
    lne_ctx *ctx;
    bool saved;
    explicit NoEvents(lne_ctx *c) : ctx(c), saved(c->no_events) { c->no_events = true; }
    ~NoEvents() { ctx->no_events = saved; }
};

}  // namespace
}  // namespace lne

using namespace lne;

extern "C" {

lne_status lne_eigsvd_noalloc(lne_ctx *ctx, const void *Y, int64_t n, int32_t k, int64_t ld,
                              int32_t dtype, void *U, int64_t ldu, double *S, double *V) {
    if (!ctx) return LNE_EINVAL;
    if (!Y || n < 1 || k < 1 || ld < k || (U && ldu < k) || dtype < LNE_F64 || dtype > LNE_BF16)
        return fail(ctx, LNE_EINVAL, "eigsvd_noalloc: bad arguments");
    if (k > kMaxK) return fail(ctx, LNE_EUNSUPPORTED, "eigsvd_noalloc: k = %d above %d", k, kMaxK);
    // layout: G, eigenvectors, weights (k x k doubles each), the
    // eigen-solver's workspace, eigenvalues, BF16 weights, then the partial
    // Grams
    const size_t kk = up256(sizeof(double) * (size_t)k * k);
    const size_t ws = up256(sizeof(double) * sym_eig_ws_doubles(k));
    const size_t fixed = 3 * kk + ws + up256(sizeof(double) * (size_t)k) +
                         up256(project_bf16_ws_bytes(k, k));
    const int KP = (k + 15) / 16 * 16;
    const size_t one_part = sizeof(double) * (size_t)KP * KP;
    if (fixed + one_part > kScratchBytes)
        return fail(ctx, LNE_EUNSUPPORTED, "eigsvd_noalloc: k = %d needs more than %zu bytes",
                    k, kScratchBytes);
    unsigned char *base = nullptr;
    LNE_TRY(scratch_ptr(ctx, &base));
    NoEvents guard(ctx);
    double *G = reinterpret_cast<double *>(base);
    double *Vk = reinterpret_cast<double *>(base + kk);
    double *W = reinterpret_cast<double *>(base + 2 * kk);
    double *vw = reinterpret_cast<double *>(base + 3 * kk);
    double *lam = reinterpret_cast<double *>(base + 3 * kk + ws);
    void *wt = base + 3 * kk + ws + up256(sizeof(double) * (size_t)k);
    double *part = reinterpret_cast<double *>(base + fixed);
    // every entry these kernels read is written first in the same call, so
    // nothing needs clearing between calls
    LNE_TRY(gram(ctx, Y, dtype, n, k, ld, G, nullptr, 1, 0, part, kScratchBytes - fixed));
    LNE_TRY(sym_eig(ctx, G, k, Vk, lam, 1, vw));
    if (U) {
        LNE_TRY(eig_weights(ctx, Vk, lam, k, k, -0.5, W, nullptr));
        const int32_t ut = dtype == LNE_BF16 ? LNE_F32 : dtype;
        LNE_TRY(project(ctx, Y, dtype, ld, n, k, W, k, U, ut, ldu, nullptr, 1, 0, 0, 0, wt));
    }
    if (S) LNE_TRY(eig_weights(ctx, Vk, lam, k, k, 0.0, nullptr, S));
    if (V) {
        const hipError_t e = hipMemcpyAsync(V, Vk, sizeof(double) * (size_t)k * k,
                                            hipMemcpyDeviceToDevice, ctx->stream);
        if (e != hipSuccess)
            return fail(ctx, LNE_EHIP, "eigsvd_noalloc: copy of V: %s", hipGetErrorString(e));
    }
    return LNE_OK;
}

}  // extern "C"
