/*
 * Driver for a sanitizer build of the join oracle (ASan + UBSan): runs every
 * oracle entry point on small seeded inputs (duplicates, negative keys, empty
 * sides, more than one thread for the sorts) and checks that the three join
 * functions agree with each other: sort-merge count/checksum == per-key totals,
 * and the per-probe-row match lists add up to the same count. Exit status 0
 * when everything agrees; the sanitizers abort on any memory or UB error.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_join_sortmerge(int64_t nR, const int64_t *kR, const int64_t *pR, int64_t nS, const int64_t *kS,
                          const int64_t *pS, uint64_t *pairs, int64_t cap, int threads, int64_t *count_out,
                          int64_t *checksum_out);
int oracle_join_totals(int64_t nR, const int64_t *kR, const int64_t *pR, int64_t nS, const int64_t *kS,
                       const int64_t *pS, int threads, int64_t *count_out, int64_t *checksum_out);
int oracle_probe_matches(int64_t nR, const int64_t *kR, const int64_t *kS, int64_t nq, const int64_t *q,
                         int64_t *offs, uint32_t *ids, int64_t cap, int threads);
uint64_t oracle_fmix64(uint64_t k);
void oracle_hll_registers(int64_t n, const int64_t *keys, int p, uint8_t *regs);

static uint64_t state = 0x9E3779B97F4A7C15ull;
static uint64_t next(void) {  /* SplitMix64 step (Steele et al.) */
    uint64_t z = (state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static int run_case(int64_t nR, int64_t nS, int64_t lo, int64_t span, int threads) {
    int64_t *kR = malloc(sizeof(int64_t) * (nR ? nR : 1)), *pR = malloc(sizeof(int64_t) * (nR ? nR : 1));
    int64_t *kS = malloc(sizeof(int64_t) * (nS ? nS : 1)), *pS = malloc(sizeof(int64_t) * (nS ? nS : 1));
    for (int64_t i = 0; i < nR; ++i) { kR[i] = lo + (int64_t)(next() % (uint64_t)span); pR[i] = (int64_t)next(); }
    for (int64_t j = 0; j < nS; ++j) { kS[j] = lo + (int64_t)(next() % (uint64_t)span); pS[j] = (int64_t)next(); }
    int64_t c1, s1, c2, s2, c3, s3;
    if (oracle_join_sortmerge(nR, kR, pR, nS, kS, pS, NULL, 0, threads, &c1, &s1) < 0) return 1;
    uint64_t *pairs = malloc(sizeof(uint64_t) * (c1 ? c1 : 1));
    if (oracle_join_sortmerge(nR, kR, pR, nS, kS, pS, pairs, c1, threads, &c2, &s2) != 0) return 2;
    for (int64_t t = 1; t < c2; ++t)
        if (pairs[t - 1] >= pairs[t]) return 3;  /* canonical: strictly ascending */
    if (oracle_join_totals(nR, kR, pR, nS, kS, pS, threads, &c3, &s3) != 0) return 4;
    if (c1 != c2 || c1 != c3 || s1 != s2 || s1 != s3) return 5;
    int64_t nq = nS < 500 ? nS : 500;
    int64_t *q = malloc(sizeof(int64_t) * (nq ? nq : 1)), *offs = malloc(sizeof(int64_t) * (nq + 1));
    for (int64_t t = 0; t < nq; ++t) q[t] = (int64_t)(next() % (uint64_t)nS);
    if (oracle_probe_matches(nR, kR, kS, nq, q, offs, NULL, 0, threads) < 0) return 6;
    uint32_t *ids = malloc(sizeof(uint32_t) * (offs[nq] ? offs[nq] : 1));
    if (oracle_probe_matches(nR, kR, kS, nq, q, offs, ids, offs[nq], threads) != 0) return 7;
    for (int64_t t = 0; t < nq; ++t)
        for (int64_t u = offs[t]; u < offs[t + 1]; ++u)
            if (ids[u] >= (uint64_t)nR || kR[ids[u]] != kS[q[t]]) return 8;
    uint8_t regs[1 << 14];
    oracle_hll_registers(nR, kR, 14, regs);
    (void)oracle_fmix64((uint64_t)kR[0 < nR ? 0 : 0]);
    free(kR); free(pR); free(kS); free(pS); free(pairs); free(q); free(offs); free(ids);
    return 0;
}

int main(void) {
    const struct { int64_t nR, nS, lo, span; } cases[] = {
        {0, 10, 0, 5}, {10, 0, 0, 5}, {1, 1, 7, 1}, {1000, 5000, -500, 1000}, {3000, 70000, -100, 40},
        {70000, 150000, INT64_MIN / 2, INT64_MAX}, {100000, 100000, 0, 1 << 20},
    };
    for (unsigned c = 0; c < sizeof(cases) / sizeof(cases[0]); ++c)
        for (int threads = 1; threads <= 4; threads += 3) {
            int rc = run_case(cases[c].nR, cases[c].nS, cases[c].lo, cases[c].span, threads);
            if (rc) {
                printf("case %u threads %d failed: %d\n", c, threads, rc);
                return 1;
            }
        }
    printf("oracle selftest ok\n");
    return 0;
}
