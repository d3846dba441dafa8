/*
 * eiger_oracle.c -- CPU reference for the single-GPU equi-join path.
 *
 * TEST INFRASTRUCTURE ONLY. Only tests, the smoke check and the benchmark's
 * CPU-baseline leg may load this library. It shares no code with the GPU
 * library: no headers, no helpers, no tables.
 *
 * Every function is a plain, slow, obviously correct statement of what the
 * path computes. Keys and payloads arrive sign-extended to int64 (the Python
 * wrapper widens int32 columns), so key equality and the payload products are
 * the same for 4- and 8-byte columns.
 *
 * Result of an inner equi-join of R (build) and S (probe), following the
 * paper's join definition (Section 5.2: R the smaller side, S the larger;
 * Section 2.2: tuple ids as the late-materialization delegate):
 *   P        = { (i, j) : kR[i] == kS[j] }
 *   count    = |P|
 *   checksum = sum over P of pR[i] * pS[j], multiply and add mod 2^64,
 *              reinterpreted as int64
 * Canonical form of P: ascending by (i, j), i.e. ascending u64 (i << 32) | j.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int64_t key;
    uint32_t id;
} keyed_row;

static int cmp_keyed_row(const void *a, const void *b)
{
    const keyed_row *x = (const keyed_row *)a, *y = (const keyed_row *)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    if (x->id != y->id) return x->id < y->id ? -1 : 1;
    return 0;
}

static int cmp_u64(const void *a, const void *b)
{
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

/*
 * Sort n elements of `size` bytes ascending by `cmp` with up to `threads`
 * threads: each thread sorts one contiguous slice with qsort, then neighbouring
 * sorted runs are merged pairwise (ties taken from the left run first) until
 * one run remains. The result is the same ascending order qsort gives (the
 * comparators below are total orders, so the sorted array is unique); only the
 * time differs. Returns -1 if the merge buffer cannot be allocated.
 */
static void merge_runs(const char *src, size_t lo, size_t mid, size_t hi, char *dst, size_t size,
                       int (*cmp)(const void *, const void *))
{
    size_t a = lo, b = mid, o = lo;
    while (a < mid && b < hi) {
        if (cmp(src + b * size, src + a * size) < 0) {
            memcpy(dst + o * size, src + b * size, size);
            ++b;
        } else {
            memcpy(dst + o * size, src + a * size, size);
            ++a;
        }
        ++o;
    }
    if (a < mid) memcpy(dst + o * size, src + a * size, (mid - a) * size);
    if (b < hi) memcpy(dst + o * size + (mid - a) * size, src + b * size, (hi - b) * size);
}

static int par_sort(void *base, size_t n, size_t size, int (*cmp)(const void *, const void *), int threads)
{
    if (threads < 2 || n < ((size_t)1 << 16)) {
        qsort(base, n, size, cmp);
        return 0;
    }
    const int t = threads;
    size_t *bounds = (size_t *)malloc((size_t)(t + 1) * sizeof(size_t));
    char *tmp = (char *)malloc(n * size);
    if (!bounds || !tmp) {
        free(bounds);
        free(tmp);
        return -1;
    }
    for (int i = 0; i <= t; ++i) bounds[i] = n * (size_t)i / (size_t)t;
#ifdef _OPENMP
#pragma omp parallel for num_threads(t) schedule(static, 1)
#endif
    for (int i = 0; i < t; ++i)
        qsort((char *)base + bounds[i] * size, bounds[i + 1] - bounds[i], size, cmp);
    char *src = (char *)base, *dst = tmp;
    int runs = t;
    while (runs > 1) {
        const int pairs = runs / 2;
#ifdef _OPENMP
#pragma omp parallel for num_threads(t) schedule(static, 1)
#endif
        for (int r = 0; r < pairs; ++r)
            merge_runs(src, bounds[2 * r], bounds[2 * r + 1], bounds[2 * r + 2], dst, size, cmp);
        if (runs % 2)
            memcpy(dst + bounds[runs - 1] * size, src + bounds[runs - 1] * size,
                   (bounds[runs] - bounds[runs - 1]) * size);
        const int next = (runs + 1) / 2;
        for (int i = 0; i < next; ++i) bounds[i] = bounds[2 * i];
        bounds[next] = n;
        runs = next;
        char *sw = src;
        src = dst;
        dst = sw;
    }
    if (src != (char *)base) memcpy(base, src, n * size);
    free(tmp);
    free(bounds);
    return 0;
}

static keyed_row *sorted_rows(int64_t n, const int64_t *keys, int threads)
{
    keyed_row *r = (keyed_row *)malloc((size_t)(n > 0 ? n : 1) * sizeof(keyed_row));
    if (!r) return NULL;
    for (int64_t i = 0; i < n; ++i) {
        r[i].key = keys[i];
        r[i].id = (uint32_t)i;
    }
    if (par_sort(r, (size_t)n, sizeof(keyed_row), cmp_keyed_row, threads) != 0) {
        free(r);
        return NULL;
    }
    return r;
}

/*
 * Sort-merge join (the textbook form of the paper's SMJ, Section 3.2 and
 * Table 1): sort both sides by (key, row id), walk them with two cursors, and
 * on a run of equal keys emit the cross product of the two runs.
 *
 * pairs: NULL (count and checksum only) or room for `cap` u64 packed pairs.
 * threads: threads for the sorts (par_sort); the merge walk is sequential.
 * Returns 0 on success, 1 if pairs was given and count > cap (the first cap
 * pairs found are written, not canonically), -1 on allocation failure.
 */
int oracle_join_sortmerge(int64_t nR, const int64_t *kR, const int64_t *pR,
                          int64_t nS, const int64_t *kS, const int64_t *pS,
                          uint64_t *pairs, int64_t cap, int threads,
                          int64_t *count_out, int64_t *checksum_out)
{
    keyed_row *A = sorted_rows(nR, kR, threads);
    keyed_row *B = sorted_rows(nS, kS, threads);
    if (!A || !B) {
        free(A);
        free(B);
        return -1;
    }
    int64_t a = 0, b = 0, count = 0;
    uint64_t checksum = 0;
    while (a < nR && b < nS) {
        if (A[a].key < B[b].key) {
            ++a;
        } else if (A[a].key > B[b].key) {
            ++b;
        } else {
            const int64_t k = A[a].key;
            int64_t a_end = a, b_end = b;
            while (a_end < nR && A[a_end].key == k) ++a_end;
            while (b_end < nS && B[b_end].key == k) ++b_end;
            for (int64_t x = a; x < a_end; ++x) {
                for (int64_t y = b; y < b_end; ++y) {
                    if (pairs && count < cap)
                        pairs[count] = ((uint64_t)A[x].id << 32) | (uint64_t)B[y].id;
                    ++count;
                    checksum += (uint64_t)pR[A[x].id] * (uint64_t)pS[B[y].id];
                }
            }
            a = a_end;
            b = b_end;
        }
    }
    free(A);
    free(B);
    if (pairs && par_sort(pairs, (size_t)(count < cap ? count : cap), sizeof(uint64_t), cmp_u64, threads) != 0)
        return -1;
    *count_out = count;
    *checksum_out = (int64_t)checksum;
    return (pairs && count > cap) ? 1 : 0;
}

/*
 * Count and checksum from per-key aggregates of R, an independent route to
 * the same two numbers:
 *   count    = sum_j cR(kS[j])             with cR(k) = #{i : kR[i] == k}
 *   checksum = sum_j sR(kS[j]) * pS[j]     with sR(k) = sum of pR[i] over kR[i] == k
 * which equals the pair sums because multiplication distributes over addition
 * in the ring of integers mod 2^64. Distinct R keys are found by sorting; each
 * probe row finds its key by binary search. The probe loop is split over
 * `threads` OpenMP threads; the sums are wrapping integer sums, so the result
 * does not depend on the thread count.
 */
int oracle_join_totals(int64_t nR, const int64_t *kR, const int64_t *pR,
                       int64_t nS, const int64_t *kS, const int64_t *pS,
                       int threads, int64_t *count_out, int64_t *checksum_out)
{
    keyed_row *A = sorted_rows(nR, kR, threads);
    if (!A) return -1;
    int64_t nd = 0;
    int64_t *dkey = (int64_t *)malloc((size_t)(nR > 0 ? nR : 1) * sizeof(int64_t));
    int64_t *dcnt = (int64_t *)malloc((size_t)(nR > 0 ? nR : 1) * sizeof(int64_t));
    uint64_t *dsum = (uint64_t *)malloc((size_t)(nR > 0 ? nR : 1) * sizeof(uint64_t));
    if (!dkey || !dcnt || !dsum) {
        free(A); free(dkey); free(dcnt); free(dsum);
        return -1;
    }
    for (int64_t a = 0; a < nR; ++a) {
        if (nd == 0 || dkey[nd - 1] != A[a].key) {
            dkey[nd] = A[a].key;
            dcnt[nd] = 0;
            dsum[nd] = 0;
            ++nd;
        }
        dcnt[nd - 1] += 1;
        dsum[nd - 1] += (uint64_t)pR[A[a].id];
    }
    free(A);
    int64_t count = 0;
    uint64_t checksum = 0;
    (void)threads;
#ifdef _OPENMP
#pragma omp parallel for num_threads(threads > 0 ? threads : 1) reduction(+ : count, checksum) schedule(static)
#endif
    for (int64_t j = 0; j < nS; ++j) {
        int64_t lo = 0, hi = nd; /* first index with dkey >= kS[j] */
        while (lo < hi) {
            int64_t mid = lo + (hi - lo) / 2;
            if (dkey[mid] < kS[j]) lo = mid + 1; else hi = mid;
        }
        if (lo < nd && dkey[lo] == kS[j]) {
            count += dcnt[lo];
            checksum += dsum[lo] * (uint64_t)pS[j];
        }
    }
    free(dkey); free(dcnt); free(dsum);
    *count_out = count;
    *checksum_out = (int64_t)checksum;
    return 0;
}

/*
 * The build rows matching each of `nq` queried probe rows q[0..nq), for
 * checking a full-size result one probe row at a time. Writes, for query t,
 * the matching build row ids ascending into ids[offs[t] .. offs[t+1]).
 * With ids == NULL only offs is filled (sizing call). Returns -1 on
 * allocation failure, 1 if offs[nq] > cap, else 0.
 */
int oracle_probe_matches(int64_t nR, const int64_t *kR, const int64_t *kS,
                         int64_t nq, const int64_t *q, int64_t *offs,
                         uint32_t *ids, int64_t cap, int threads)
{
    keyed_row *A = sorted_rows(nR, kR, threads);
    if (!A) return -1;
    int64_t total = 0;
    offs[0] = 0;
    for (int64_t t = 0; t < nq; ++t) {
        const int64_t k = kS[q[t]];
        int64_t lo = 0, hi = nR;
        while (lo < hi) {
            int64_t mid = lo + (hi - lo) / 2;
            if (A[mid].key < k) lo = mid + 1; else hi = mid;
        }
        for (int64_t a = lo; a < nR && A[a].key == k; ++a) {
            if (ids && total < cap) ids[total] = A[a].id; /* ascending: rows sort by (key, id) */
            ++total;
        }
        offs[t + 1] = total;
    }
    free(A);
    return (ids && total > cap) ? 1 : 0;
}

/*
 * 64-bit finalizer of MurmurHash3 (fmix64, Austin Appleby, public domain):
 * xor-shift by 33, multiply, xor-shift by 33, multiply, xor-shift by 33.
 * Each step is invertible, so the function is a bijection of 64-bit words.
 */
uint64_t oracle_fmix64(uint64_t k)
{
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdULL;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ULL;
    k ^= k >> 33;
    return k;
}

/*
 * HyperLogLog registers (dense form; the sketch the paper uses for distinct
 * counts, Section 4.1, citing HLL++). With m = 2^p registers and h the 64-bit
 * hash of the sign-extended key:
 *   bucket = top p bits of h
 *   w      = the remaining 64 - p bits, left-aligned
 *   rank   = position of the first 1 bit of w, counting from 1
 *            (64 - p + 1 when w is all zero)
 *   M[bucket] = max(M[bucket], rank)
 */
void oracle_hll_registers(int64_t n, const int64_t *keys, int p, uint8_t *regs)
{
    memset(regs, 0, (size_t)1 << p);
    for (int64_t i = 0; i < n; ++i) {
        const uint64_t h = oracle_fmix64((uint64_t)keys[i]);
        const uint64_t bucket = h >> (64 - p);
        const uint64_t w = h << p;
        const uint8_t rank = w == 0 ? (uint8_t)(64 - p + 1) : (uint8_t)(__builtin_clzll(w) + 1);
        if (rank > regs[bucket]) regs[bucket] = rank;
    }
}
