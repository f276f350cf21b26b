// Launch-shape tuning: time each variant of a kernel on the caller's own data
// the first time a shape is seen, keep the fastest per context, optionally in
// a JSON-lines file shared between processes (LNE_TUNE_CACHE).
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "common.hpp"

namespace lne {

namespace {

int file_variant(const std::string &key) {
    const char *path = std::getenv("LNE_TUNE_CACHE");
    if (!path || !*path) return -1;
    FILE *f = std::fopen(path, "r");
    if (!f) return -1;
    char line[1024];
    int v = -1;
    const std::string probe = key + ",";
    while (std::fgets(line, sizeof(line), f)) {
        if (!std::strstr(line, probe.c_str())) continue;
        const char *q = std::strstr(line, "\"variant\": ");
        if (q) v = std::atoi(q + 11);
    }
    std::fclose(f);
    return v;
}

void file_store(const std::string &key, int v, const std::vector<float> &ms) {
    const char *path = std::getenv("LNE_TUNE_CACHE");
    if (!path || !*path) return;
    FILE *f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "{%s, \"variant\": %d, \"ms\": [", key.c_str(), v);
    for (size_t i = 0; i < ms.size(); ++i) std::fprintf(f, "%s%.4f", i ? ", " : "", ms[i]);
    std::fprintf(f, "]}\n");
    std::fclose(f);
}

}  // namespace

std::string shape_key(const char *op, int64_t n, int64_t nnz, int k, int dtype) {
    const int cls = nnz > 0 ? (int)std::floor(4.0 * std::log2((double)nnz)) : -1;
    char buf[192];
    snprintf(buf, sizeof(buf), "\"op\": \"%s\", \"n\": %lld, \"nnz_class\": %d, \"k\": %d, "
             "\"dtype\": %d", op, (long long)n, cls, k, dtype);
    return buf;
}

int tuned_or(lne_ctx *ctx, const std::string &key, int dflt) {
    auto it = ctx->tuned.find(key);
    return it == ctx->tuned.end() ? dflt : it->second;
}

lne_status pick_variant(lne_ctx *ctx, const std::string &key, int nv,
                        const std::function<lne_status(int)> &run, int *out) {
    auto it = ctx->tuned.find(key);
    if (it != ctx->tuned.end()) {
        *out = it->second;
        return LNE_OK;
    }
    int v = file_variant(key);
    if (v >= 0 && v < nv) {
        ctx->tuned[key] = v;
        *out = v;
        return LNE_OK;
    }
    if (ctx->capturing || nv <= 1) {
        *out = 0;
        return LNE_OK;
    }
    hipEvent_t e0, e1;
    LNE_HIP(ctx, hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(ctx, LNE_EHIP, "pick_variant: event creation failed");
    }
    std::vector<float> ms(nv, 0.f);
    lne_status s = run(0);   // warm-up
    for (int i = 0; i < nv && s == LNE_OK; ++i) {
        (void)hipEventRecord(e0, ctx->stream);
        s = run(i);
        (void)hipEventRecord(e1, ctx->stream);
        if (s == LNE_OK && hipEventSynchronize(e1) != hipSuccess)
            s = fail(ctx, LNE_EHIP, "pick_variant: event wait failed");
        if (s == LNE_OK) (void)hipEventElapsedTime(&ms[i], e0, e1);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    LNE_TRY(s);
    v = (int)(std::min_element(ms.begin(), ms.end()) - ms.begin());
    ctx->tuned[key] = v;
    file_store(key, v, ms);
    *out = v;
    return LNE_OK;
}

}  // namespace lne
