/*
 * Driver for a sanitizer build of the library's host code (ASan + UBSan on the
 * host side of every .hip file; device code unchanged): exercises every entry
 * point path that finishes before any GPU work -- planning under each
 * selector, workspace sizing of every variant over a sweep of sizes and knobs,
 * the argument checks of the join, statistics, scratch-free and batch calls,
 * selector features / class plans / model installation -- with no GPU
 * present. Exit status 0 when every call returns the documented status.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "eiger.h"

#define EXPECT(cond)                                                     \
    do {                                                                 \
        if (!(cond)) {                                                   \
            printf("FAILED %s:%d: %s (%s)\n", __FILE__, __LINE__, #cond, \
                   eiger_last_error());                                  \
            return 1;                                                    \
        }                                                                \
    } while (0)

static eiger_stats_t st(int64_t n, int64_t lo, int64_t hi, double ndv, int32_t dt) {
    eiger_stats_t s;
    memset(&s, 0, sizeof(s));
    s.n = n;
    s.min = lo;
    s.max = hi;
    s.ndv = ndv;
    s.dtype = dt;
    s.hll_p = EIGER_HLL_P;
    return s;
}

static eiger_column col(uintptr_t p, int64_t n, int32_t dt) {
    eiger_column c;
    c.data = (const void *)p;
    c.n = n;
    c.dtype = dt;
    c.reserved = 0;
    return c;
}

int main(void) {
    const int32_t dts[2] = {EIGER_INT32, EIGER_INT64};
    const int64_t sizes[] = {0, 1, 63, 4096, 65536, 1000003, 16777216, 536870912, EIGER_MAX_ROWS};
    const float lfs[] = {0.1f, 0.25f, 0.5f, 0.75f, 0.9f};
    size_t bytes = 0;
    for (int d = 0; d < 2; ++d)
        for (unsigned a = 0; a < sizeof(sizes) / sizeof(sizes[0]); ++a)
            for (unsigned b = 0; b < sizeof(sizes) / sizeof(sizes[0]); b += 2) {
                const int64_t nR = sizes[a], nS = sizes[b];
                eiger_stats_t sb = st(nR, -1000, nR > 0 ? 4 * nR : 0, (double)nR, dts[d]);
                eiger_stats_t sp = st(nS, -1000, nS + 10, (double)nS / 2, dts[d]);
                eiger_plan_t p;
                for (int sel = EIGER_SEL_RULE; sel <= EIGER_SEL_FIXED_HASH; ++sel) {
                    if (sel == EIGER_SEL_LEARNED) continue;
                    EXPECT(eiger_join_plan(&sb, &sp, sel, NULL, &p) == EIGER_OK);
                    eiger_column k = col(4096, nR, dts[d]), s = col(4096, nS, dts[d]);
                    int rc = eiger_join_workspace_size(&p, k, k, s, s, &bytes);
                    EXPECT(rc == EIGER_OK || rc == EIGER_ERR_TOO_LARGE || rc == EIGER_ERR_UNSUPPORTED);
                }
                for (int v = EIGER_GLOBAL_HASH; v <= EIGER_RADIX_CACHE; ++v)
                    for (unsigned l = 0; l < sizeof(lfs) / sizeof(lfs[0]); ++l)
                        for (int bits = 1; bits <= 18; bits += 3) {
                            eiger_plan_t f, q;
                            memset(&f, 0, sizeof(f));
                            f.variant = v;
                            f.radix_bits = bits;
                            f.radix_passes = bits > 9 ? 2 : 1;
                            f.load_factor = lfs[l];
                            EXPECT(eiger_join_plan(&sb, &sp, EIGER_SEL_FORCED, &f, &q) == EIGER_OK);
                            eiger_column k = col(4096, nR, dts[d]), s = col(4096, nS, dts[d]);
                            int rc = eiger_join_workspace_size(&q, k, k, s, s, &bytes);
                            EXPECT(rc == EIGER_OK || rc == EIGER_ERR_TOO_LARGE || rc == EIGER_ERR_INVALID_ARG);
                        }
            }
    /* argument checks of the join (all before any GPU work) */
    eiger_stats_t s10 = st(10, 0, 9, 10.0, EIGER_INT32);
    eiger_plan_t p;
    EXPECT(eiger_join_plan(&s10, &s10, EIGER_SEL_RULE, NULL, &p) == EIGER_OK);
    int64_t cnt = 0, cs = 0;
    eiger_column g = col(4096, 10, EIGER_INT32);
    EXPECT(eiger_join(g, g, col(4096, 10, EIGER_INT64), col(4096, 10, EIGER_INT64), &p, NULL, NULL, 0, &cnt, &cs,
                      NULL, 0, NULL) == EIGER_ERR_DTYPE);
    EXPECT(eiger_join(col(4098, 10, EIGER_INT32), g, g, g, &p, NULL, NULL, 0, &cnt, &cs, NULL, 0, NULL) ==
           EIGER_ERR_INVALID_ARG);
    EXPECT(eiger_join(col(4096, EIGER_MAX_ROWS + 1, EIGER_INT32), col(4096, EIGER_MAX_ROWS + 1, EIGER_INT32), g, g,
                      &p, NULL, NULL, 0, &cnt, &cs, NULL, 0, NULL) == EIGER_ERR_TOO_LARGE);
    EXPECT(eiger_join(g, g, g, g, &p, NULL, NULL, 0, &cnt, &cs, NULL, 0, NULL) == EIGER_ERR_WORKSPACE);
    EXPECT(eiger_join(g, g, g, g, NULL, NULL, NULL, 0, &cnt, &cs, NULL, 0, NULL) == EIGER_ERR_INVALID_ARG);
    EXPECT(eiger_join_noalloc(g, g, g, g, &p, (uint32_t *)4096, NULL, 5, &cnt, &cs, NULL) == EIGER_ERR_INVALID_ARG);
    {
        eiger_stats_t big = st(10000000, -(1ll << 40), 1ll << 40, 1e7, EIGER_INT64);
        eiger_plan_t h;
        EXPECT(eiger_join_plan(&big, &big, EIGER_SEL_FIXED_HASH, NULL, &h) == EIGER_OK);
        eiger_column b = col(4096, 10000000, EIGER_INT64);
        EXPECT(eiger_join_noalloc(b, b, b, b, &h, NULL, NULL, 0, &cnt, &cs, NULL) == EIGER_ERR_TOO_LARGE);
    }
    /* statistics of an empty column need no GPU */
    eiger_stats_t out;
    uint8_t regs[EIGER_HLL_REGISTERS];
    EXPECT(eiger_stats(col(0, 0, EIGER_INT64), &out, regs, NULL, 0, NULL) == EIGER_OK && out.n == 0);
    EXPECT(eiger_stats(col(0, 0, 9), &out, NULL, NULL, 0, NULL) == EIGER_ERR_DTYPE);
    /* selector: features, class plans, model installation, learned planning */
    float f[EIGER_SEL_FEATURES];
    eiger_stats_t b64 = st(1 << 20, -(1ll << 40), 1ll << 40, (double)(1 << 20), EIGER_INT64);
    eiger_stats_t p64 = st(1 << 22, -(1ll << 40), 1ll << 40, (double)(1 << 20), EIGER_INT64);
    EXPECT(eiger_selector_features(&b64, &p64, f) == EIGER_OK);
    for (int c = 0; c < EIGER_SEL_CLASSES; ++c) {
        eiger_plan_t q;
        int rc = eiger_selector_class_plan(c, &b64, &p64, &q);
        EXPECT(rc == EIGER_OK || rc == EIGER_ERR_UNSUPPORTED);
    }
    const int64_t np = eiger_mlp_param_count();
    float *params = calloc((size_t)np, sizeof(float));
    float mean[EIGER_SEL_FEATURES], sd[EIGER_SEL_FEATURES], lo[EIGER_SEL_FEATURES], hi[EIGER_SEL_FEATURES];
    for (int i = 0; i < EIGER_SEL_FEATURES; ++i) {
        mean[i] = 0.f;
        sd[i] = 1.f;
        lo[i] = f[i] - 0.5f;
        hi[i] = f[i] + 0.5f;
    }
    for (int64_t i = 0; i < np; ++i) params[i] = (float)((i * 2654435761u) % 1000) / 1000.f - 0.5f;
    EXPECT(eiger_selector_load(params, mean, sd, lo, hi) == EIGER_OK && eiger_selector_loaded());
    EXPECT(eiger_join_plan(&b64, &p64, EIGER_SEL_LEARNED, NULL, &p) == EIGER_OK);
    EXPECT(eiger_selector_load(params, mean, sd, hi, lo) == EIGER_ERR_MODEL);
    free(params);
    /* batch sizing and checks */
    eiger_batch_join bj[2];
    memset(bj, 0, sizeof(bj));
    bj[0].build_keys = bj[0].build_payload = bj[0].probe_keys = bj[0].probe_payload = (const void *)4096;
    bj[0].n_build = 1000;
    bj[0].n_probe = 8000;
    bj[1] = bj[0];
    bj[1].n_build = 0;
    EXPECT(eiger_join_batch_workspace_size(bj, 2, EIGER_INT32, EIGER_INT32, NULL, &bytes) == EIGER_OK && bytes > 0);
    EXPECT(eiger_join_batch_workspace_size(bj, 0, EIGER_INT32, EIGER_INT32, NULL, &bytes) == EIGER_ERR_INVALID_ARG);
    void *h = NULL;
    EXPECT(eiger_join_batch_create(bj, 2, EIGER_INT32, EIGER_INT32, NULL, NULL, NULL, NULL, 0, NULL, &h) ==
           EIGER_ERR_INVALID_ARG);
    EXPECT(eiger_join_batch_launch(NULL, NULL) == EIGER_ERR_INVALID_ARG);
    EXPECT(eiger_profile_enable(0) == EIGER_OK);
    printf("host selftest ok (version %d)\n", eiger_version());
    return 0;
}
