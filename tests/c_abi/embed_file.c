/* A plain C caller of the library (include/lne.h and the HIP runtime only,
 * no Python, no torch): the whole embedding of a graph read from a file.
 *
 *   embed_file IN OUT   reads IN, runs lne_embed on the default stream with
 *                       hipMalloc'd buffers, writes X (n x d, row-major, F32
 *                       or F64 by the parameters' precision) to OUT
 *   embed_file --check  argument checks that make no GPU call
 *
 * IN (little-endian): int64 n, int64 n_arcs, int32 index_bits, int32 zero,
 * the lne_params struct as laid out by include/lne.h, the n + 1 row offsets
 * (index_bits / 8 bytes each) and the n_arcs int32 columns.
 * Test infrastructure: tests/test_gpu_c_abi.py compares its X bit for bit
 * with the same embedding through the Python binding. */
#include <hip/hip_runtime_api.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "lne.h"

static int fail(const char *what) {
    fprintf(stderr, "embed_file: %s\n", what);
    return 1;
}

static int check(void) {
    lne_ctx *ctx = NULL;
    int bad = 0;
    /* only one of alloc / free */
    if (lne_ctx_create(&ctx, NULL, (lne_alloc_fn)(uintptr_t)1, NULL, NULL) != LNE_EINVAL) bad |= 1;
    if (lne_ctx_create(NULL, NULL, NULL, NULL, NULL) != LNE_EINVAL) bad |= 2;
    if (lne_ctx_create(&ctx, NULL, NULL, NULL, NULL) != LNE_OK || !ctx) return fail("ctx_create");
    lne_params p;
    memset(&p, 0, sizeof(p));
    p.T = 2; p.s[0] = p.s[1] = 0.5; p.M = 100; p.b = 1; p.d = 2; p.oversample = 2; p.q = 1;
    p.precision = LNE_F32;
    lne_graph g;
    memset(&g, 0, sizeof(g));
    g.n = 10; g.n_arcs = 20;
    g.row_ptr = (const void *)(uintptr_t)0x1000; g.col = (const int32_t *)(uintptr_t)0x2000;
    if (lne_embed(ctx, NULL, &p, (void *)(uintptr_t)0x3000, NULL) != LNE_EINVAL) bad |= 4;
    g.index_bits = 16;   /* neither 32 nor 64 */
    if (lne_embed(ctx, &g, &p, (void *)(uintptr_t)0x3000, NULL) != LNE_EINVAL) bad |= 8;
    g.index_bits = 32; g.n_arcs = (int64_t)1 << 31;   /* 32-bit offsets cannot reach */
    if (lne_embed(ctx, &g, &p, (void *)(uintptr_t)0x3000, NULL) != LNE_EINVAL) bad |= 16;
    g.index_bits = 64; g.n_arcs = 20; p.T = 0;        /* bad window */
    if (lne_embed(ctx, &g, &p, (void *)(uintptr_t)0x3000, NULL) != LNE_EINVAL) bad |= 32;
    const char *msg = lne_last_error(ctx);
    if (!msg || !msg[0]) bad |= 64;
    lne_ctx_destroy(ctx);
    if (bad) {
        fprintf(stderr, "embed_file: checks failed (mask %d)\n", bad);
        return 1;
    }
    printf("checks ok\n");
    return 0;
}

int main(int argc, char **argv) {
    if (argc == 2 && strcmp(argv[1], "--check") == 0) return check();
    if (argc != 3) return fail("usage: embed_file IN OUT | embed_file --check");
    FILE *f = fopen(argv[1], "rb");
    if (!f) return fail("cannot open IN");
    int64_t n = 0, n_arcs = 0;
    int32_t bits = 0, zero = 0;
    lne_params p;
    if (fread(&n, 8, 1, f) != 1 || fread(&n_arcs, 8, 1, f) != 1 || fread(&bits, 4, 1, f) != 1 ||
        fread(&zero, 4, 1, f) != 1 || fread(&p, sizeof(p), 1, f) != 1)
        return fail("short header");
    if (n < 1 || n_arcs < 0 || (bits != 32 && bits != 64)) return fail("bad header");
    const size_t ob = (size_t)bits / 8, rp_bytes = ob * (size_t)(n + 1);
    const size_t col_bytes = 4 * (size_t)n_arcs;
    void *h_rp = malloc(rp_bytes), *h_col = malloc(col_bytes ? col_bytes : 1);
    if (!h_rp || !h_col) return fail("host allocation");
    if (fread(h_rp, 1, rp_bytes, f) != rp_bytes || fread(h_col, 1, col_bytes, f) != col_bytes)
        return fail("short body");
    fclose(f);

    const size_t es = p.precision == LNE_F64 ? 8 : 4, x_bytes = es * (size_t)n * p.d;
    void *d_rp = NULL, *d_col = NULL, *d_x = NULL;
    if (hipMalloc(&d_rp, rp_bytes) != hipSuccess || hipMalloc(&d_col, col_bytes ? col_bytes : 4) != hipSuccess ||
        hipMalloc(&d_x, x_bytes) != hipSuccess)
        return fail("hipMalloc");
    if (hipMemcpy(d_rp, h_rp, rp_bytes, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(d_col, h_col, col_bytes, hipMemcpyHostToDevice) != hipSuccess)
        return fail("hipMemcpy to device");

    lne_ctx *ctx = NULL;
    if (lne_ctx_create(&ctx, NULL, NULL, NULL, NULL) != LNE_OK) return fail("ctx_create");
    lne_graph g;
    memset(&g, 0, sizeof(g));
    g.n = n; g.n_arcs = n_arcs; g.row_ptr = d_rp; g.col = (const int32_t *)d_col;
    g.weight = NULL; g.index_bits = bits;
    lne_stats st;
    const lne_status rc = lne_embed(ctx, &g, &p, d_x, &st);
    if (rc != LNE_OK) {
        fprintf(stderr, "embed_file: lne_embed: %d %s\n", (int)rc, lne_last_error(ctx));
        return 1;
    }
    if (hipDeviceSynchronize() != hipSuccess) return fail("synchronize");
    void *h_x = malloc(x_bytes);
    if (!h_x || hipMemcpy(h_x, d_x, x_bytes, hipMemcpyDeviceToHost) != hipSuccess)
        return fail("hipMemcpy to host");
    FILE *o = fopen(argv[2], "wb");
    if (!o || fwrite(h_x, 1, x_bytes, o) != x_bytes) return fail("cannot write OUT");
    fclose(o);
    printf("attempted %llu accepted %llu nnz_log %llu\n", (unsigned long long)st.attempted,
           (unsigned long long)st.accepted, (unsigned long long)st.nnz_log);
    lne_ctx_destroy(ctx);
    hipFree(d_rp); hipFree(d_col); hipFree(d_x);
    free(h_rp); free(h_col); free(h_x);
    return 0;
}
