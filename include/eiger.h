/*
 * eiger.h -- C ABI of the MI355X (gfx950) equi-join library.
 *
 * The library implements the runtime-adaptive equi-join of "Eiger: An
 * Efficient Library for GPU-based Data Analytics": lightweight statistics of
 * a key column (min, max and an HLL++-style distinct-count sketch, Section 4
 * and Section 4.1), a choice of join variant and knobs from those statistics
 * (Section 4, "algorithm selection"; join factors in Table 1), and an inner
 * equi-join that returns matched row-id pairs (late materialization through
 * tuple ids, Section 2.2) plus a payload aggregate, the "narrow join" of
 * Section 5.2.1 whose materialization is inlined into the join.
 *
 * Conventions shared by every entry point:
 *  - Data pointers marked DEVICE point to GPU memory owned by the caller; the
 *    library never allocates, frees or keeps them. HOST pointers are ordinary
 *    host memory owned by the caller.
 *  - Scratch memory is the caller's: size it with the *_workspace_size call
 *    and pass it as (ws, ws_bytes). Its contents on entry do not matter and
 *    are unspecified on return.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Work is ordered on that stream. Calls that return host values
 *    synchronize the stream before returning.
 *  - Every call returns an eiger_status; on failure eiger_last_error() holds
 *    a message for the calling thread. No C++ exception crosses the ABI.
 *  - Row ids are uint32: a column may hold at most EIGER_MAX_ROWS =
 *    2^32 - 2^16 rows (EIGER_ERR_TOO_LARGE beyond that; the margin keeps the
 *    kernels' 32-bit tile bounds from wrapping). Counts and sizes are int64.
 *  - Calls on different streams may run concurrently when each has its own
 *    workspace and outputs.
 */
#ifndef EIGER_H
#define EIGER_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    EIGER_OK = 0,
    EIGER_ERR_INVALID_ARG = -1, /* null pointer, negative size, bad enum value */
    EIGER_ERR_DTYPE = -2,       /* unsupported dtype or key dtypes that differ */
    EIGER_ERR_TOO_LARGE = -3,   /* more than EIGER_MAX_ROWS rows, or a table beyond its limit */
    EIGER_ERR_CAPACITY = -4,    /* output capacity below the result size; count is set */
    EIGER_ERR_WORKSPACE = -5,   /* ws_bytes below the size the *_workspace_size call gives */
    EIGER_ERR_HIP = -6,         /* a HIP runtime call failed (message has the HIP error) */
    EIGER_ERR_UNSUPPORTED = -7, /* a plan the library cannot run (e.g. DIRECT over a huge range) */
    EIGER_ERR_MODEL = -8        /* learned selector: no model loaded, or a malformed model */
} eiger_status;

typedef enum { EIGER_INT32 = 0, EIGER_INT64 = 1 } eiger_dtype;

/* Most rows a column (or one side of a batched join) may hold: 2^32 - 2^16. */
#define EIGER_MAX_ROWS 4294901760LL

/* A column: `n` values of `dtype` at DEVICE address `data` (may be NULL when n == 0). */
typedef struct {
    const void *data;
    int64_t n;
    int32_t dtype;
    int32_t reserved;
} eiger_column;

#define EIGER_HLL_P 14                 /* 2^14 one-byte registers */
#define EIGER_HLL_REGISTERS (1 << EIGER_HLL_P)
#define EIGER_STATS_EMPTY 1u           /* flag: the column has no rows */

/*
 * Statistics of one key column (Section 4: min and max of intermediate data;
 * Section 4.1: an HLL++ sketch for the number of distinct values).
 * min/max are the sign-extended key values (0 and 0 for an empty column).
 * ndv is the distinct-count estimate from the 2^14 dense registers.
 */
typedef struct {
    int64_t n;
    int64_t min;
    int64_t max;
    double ndv;
    int32_t dtype;
    int32_t hll_p;
    uint32_t flags;
    uint32_t reserved;
} eiger_stats_t;

/* Join variants (Table 1 lists the paper's join algorithms; DIRECT is this
 * library's addition for dense key ranges). */
typedef enum {
    EIGER_DIRECT = 0,      /* table indexed by key - min; needs a dense build key range */
    EIGER_GLOBAL_HASH = 1, /* one open-addressing table in HBM (non-partitioned hash join) */
    EIGER_RADIX = 2,       /* hash-radix partitioning, then LDS-resident tables per partition */
    EIGER_RADIX_CACHE = 3, /* one partitioning pass of the probe side; one partition-major table in
                              HBM whose per-partition regions are read from one XCD's L2 at a time */
    EIGER_SORT_MERGE = 4   /* both sides radix-sorted on key - build_min, then merged (Section 3.2,
                              Table 1); needs the plan's build_min/build_max to cover the build keys */
} eiger_variant;

typedef enum {
    EIGER_SEL_RULE = 0,       /* rule from the statistics (cardinalities, range, distinct count) */
    EIGER_SEL_LEARNED = 1,    /* the loaded MLP selector (eiger_selector_load) */
    EIGER_SEL_FIXED_HASH = 2, /* always GLOBAL_HASH at load factor 0.5 (a fixed-choice baseline) */
    EIGER_SEL_FORCED = 3      /* take variant and knobs from `forced`, fill the rest */
} eiger_selector;

/*
 * A join plan. eiger_join_plan fills it; callers may also build one by hand
 * through EIGER_SEL_FORCED. Fields:
 *  variant      eiger_variant
 *  radix_bits   RADIX: total partition bits (fan-out 2^radix_bits), 1..18;
 *               RADIX_CACHE: partition bits of its single pass, 1..10
 *  radix_passes RADIX: 1 or 2 partitioning passes over each side (ignored by RADIX_CACHE)
 *  load_factor  GLOBAL_HASH / RADIX / RADIX_CACHE: target occupancy of a table, (0, 0.9]
 *  key_dtype    dtype of both key columns
 *  build_min/max  DIRECT: range of the build keys (from the build statistics)
 *  predicted_out  estimated result size |R||S| / max(ndv_R, ndv_S) (informational)
 *  flags        EIGER_PLAN_* bits set by eiger_join_plan (informational)
 */
/* plan.flags: EIGER_SEL_LEARNED met statistics outside its model's training
 * domain and returned the rule plan instead. */
#define EIGER_PLAN_RULE_FALLBACK 1u

typedef struct {
    int32_t variant;
    int32_t radix_bits;
    int32_t radix_passes;
    int32_t key_dtype;
    float load_factor;
    uint32_t flags;
    int64_t build_min;
    int64_t build_max;
    int64_t predicted_out;
    int64_t reserved[4];
} eiger_plan_t;

/* ---- statistics ------------------------------------------------------------ */

/* Workspace bytes eiger_stats needs for a column of n rows of dtype. */
size_t eiger_stats_workspace_size(int64_t n, int32_t dtype);

/*
 * Count, min, max and distinct estimate of a key column in one pass over it
 * (Section 4 / Section 4.1). Each key is sign-extended to 64 bits and hashed
 * with MurmurHash3's fmix64; the top 14 bits pick a register, which keeps the
 * largest rank (1 + leading zeros of the remaining 50 bits, 51 if all zero).
 *  keys          DEVICE column, int32 or int64
 *  out           HOST, filled on success
 *  hll_regs_host HOST, 2^14 bytes receiving the registers, or NULL
 *  ws, ws_bytes  DEVICE workspace of eiger_stats_workspace_size(keys.n, dtype)
 * Synchronizes `stream`.
 */
int eiger_stats(eiger_column keys, eiger_stats_t *out, uint8_t *hll_regs_host,
                void *ws, size_t ws_bytes, void *stream);

/* ---- planning (host only, no GPU work) -------------------------------------- */

/*
 * Choose a variant and its knobs from the two sides' statistics (Section 4:
 * runtime statistics drive algorithm selection; Table 1 names cardinalities,
 * key distribution and match ratio as the join's runtime factors).
 *  selector  eiger_selector
 *  forced    HOST, used with EIGER_SEL_FORCED (variant, radix_bits,
 *            radix_passes, load_factor taken from it), else may be NULL
 *  out       HOST, the plan
 */
int eiger_join_plan(const eiger_stats_t *build, const eiger_stats_t *probe, int32_t selector,
                    const eiger_plan_t *forced, eiger_plan_t *out);

/* ---- join ------------------------------------------------------------------- */

/* Workspace bytes eiger_join needs for this plan and these columns (data
 * pointers are not read). Writes the size to *bytes. */
int eiger_join_workspace_size(const eiger_plan_t *plan, eiger_column build_keys,
                              eiger_column build_payload, eiger_column probe_keys,
                              eiger_column probe_payload, size_t *bytes);

/*
 * Inner equi-join of build side R and probe side S (Section 3.2 / Section 5.2).
 * Result: every (i, j) with build_keys[i] == probe_keys[j], written as
 * out_build_rowid[t] = i, out_probe_rowid[t] = j for t < count, in no
 * particular order; *out_count = number of pairs; *out_checksum = sum over the
 * pairs of build_payload[i] * probe_payload[j], payloads sign-extended to 64
 * bits, products and sum mod 2^64, as int64.
 *  build_*, probe_*  DEVICE columns; keys share a dtype; payload dtypes free;
 *                    each payload column has as many rows as its key column
 *  plan              HOST, from eiger_join_plan (or EIGER_SEL_FORCED)
 *  out_*_rowid       DEVICE uint32 arrays of out_capacity entries, or both
 *                    NULL with out_capacity == 0 (count-only mode)
 *  out_count, out_checksum  HOST
 * If the result has more than out_capacity pairs, returns EIGER_ERR_CAPACITY
 * with *out_count = the exact pair count and *out_checksum set; the output
 * arrays then hold an unspecified subset. Synchronizes `stream`.
 */
int eiger_join(eiger_column build_keys, eiger_column build_payload, eiger_column probe_keys,
               eiger_column probe_payload, const eiger_plan_t *plan, uint32_t *out_build_rowid,
               uint32_t *out_probe_rowid, int64_t out_capacity, int64_t *out_count,
               int64_t *out_checksum, void *ws, size_t ws_bytes, void *stream);

/* ---- wide joins (payload columns materialized) ------------------------------
 * The "wide join" of Section 5.2.1: every result pair also carries the payload
 * columns of both relations. Two ways to produce them (Section 3.2):
 *  EIGER_MAT_GFUR  gather from the untransformed relations: join the keys with
 *                  any variant, then gather each payload column from the
 *                  caller's columns by row id (random reads).
 *  EIGER_MAT_GFTR  gather from the transformed relations (RADIX plans only):
 *                  the payload columns are carried through the partitioning
 *                  passes with the keys, and each result block gathers its
 *                  payloads from one partition's contiguous range.
 *  EIGER_MAT_AUTO  GFTR for RADIX plans whose estimated match ratio
 *                  (predicted_out / probe rows) is at least 0.25, else GFUR
 *                  (Section 5.2.3: GFUR wins at low match ratios).
 * With no payload column on either side the two coincide (GFUR is reported). */
typedef enum { EIGER_MAT_GFUR = 0, EIGER_MAT_GFTR = 1, EIGER_MAT_AUTO = 2 } eiger_materialize;

/* Workspace bytes of eiger_join_wide for these columns (data not read). */
int eiger_join_wide_workspace_size(const eiger_plan_t *plan, int32_t materialize, eiger_column build_keys,
                                   const eiger_column *build_cols, int32_t n_build_cols,
                                   eiger_column probe_keys, const eiger_column *probe_cols,
                                   int32_t n_probe_cols, size_t *bytes);

/*
 * Inner equi-join of R and S with materialized payloads. Result row t is a
 * pair (i, j) with build_keys[i] == probe_keys[j]:
 *   out_build_rowid[t] = i, out_probe_rowid[t] = j,
 *   out_build_cols[c][t] = build_cols[c][i]   (c < n_build_cols),
 *   out_probe_cols[c][t] = probe_cols[c][j]   (c < n_probe_cols),
 * rows in no particular order, each output column in its input column's dtype.
 *  build_cols, probe_cols  HOST arrays of 0..4 DEVICE columns (int32 or int64,
 *                 as many rows as their side's keys)
 *  plan           from eiger_join_plan; its variant joins the keys
 *  materialize    eiger_materialize; *out_materialized (HOST, may be NULL)
 *                 receives the strategy used
 *  out_*          DEVICE arrays of out_capacity entries (out_*_cols: HOST arrays
 *                 of DEVICE pointers); out_capacity == 0 with NULL row-id
 *                 outputs counts only
 *  out_count      HOST: number of result rows
 * EIGER_ERR_CAPACITY when the result exceeds out_capacity (*out_count set,
 * outputs hold an unspecified subset); EIGER_ERR_UNSUPPORTED for GFTR with a
 * plan other than RADIX. Synchronizes `stream`.
 */
int eiger_join_wide(eiger_column build_keys, const eiger_column *build_cols, int32_t n_build_cols,
                    eiger_column probe_keys, const eiger_column *probe_cols, int32_t n_probe_cols,
                    const eiger_plan_t *plan, int32_t materialize, uint32_t *out_build_rowid,
                    uint32_t *out_probe_rowid, void *const *out_build_cols, void *const *out_probe_cols,
                    int64_t out_capacity, int64_t *out_count, int32_t *out_materialized, void *ws,
                    size_t ws_bytes, void *stream);

/* ---- group-by ---------------------------------------------------------------
 * Groups of a key column with a row count and the sum (mod 2^64, values
 * sign-extended) of up to two value columns per group (Section 3.3: group-by
 * algorithms). The algorithm is picked from the HLL++ distinct-count estimate
 * of the keys (Section 4.1: the number of groups decides, and sizes the hash
 * table; Section 5.3.2: "Auto"):
 *  EIGER_GB_HASH       one NDV-sized open-addressing table of groups in HBM;
 *                      each workgroup pre-aggregates its rows in LDS first
 *  EIGER_GB_PARTITION  rows partitioned on the key hash (values carried), then
 *                      one LDS table per partition, written out directly
 */
typedef enum { EIGER_GB_HASH = 0, EIGER_GB_PARTITION = 1 } eiger_groupby_variant;
#define EIGER_GB_NO_SENTINEL 1u /* plan.flags: int64 keys cover both ends of the domain (unsupported) */

typedef struct {
    int32_t variant;          /* eiger_groupby_variant */
    int32_t radix_bits;       /* PARTITION: 2^radix_bits partitions (1..18), made by stable radix
                                 passes of at most 8 bits (narrower for wide rows) */
    int32_t key_dtype;
    uint32_t flags;           /* EIGER_GB_* */
    int64_t slots;            /* slots of the global group table (power of two >= 1024) */
    int64_t predicted_groups; /* the distinct-count estimate the plan used */
    int64_t sentinel;         /* a value no key takes: marks empty slots */
    int64_t reserved[2];
} eiger_groupby_plan_t;

/* Plan a group-by from the key column's statistics. selector: EIGER_SEL_RULE
 * (HASH up to 1024 estimated groups, what one LDS table holds, else PARTITION
 * with about 512 groups per partition; the global table gets twice the
 * estimate in slots) or
 * EIGER_SEL_FORCED (variant and radix_bits from `forced`). Host only. */
int eiger_groupby_plan(const eiger_stats_t *keys, int32_t selector, const eiger_groupby_plan_t *forced,
                       eiger_groupby_plan_t *out);

int eiger_groupby_workspace_size(const eiger_groupby_plan_t *plan, eiger_column keys, const eiger_column *vals,
                                 int32_t n_vals, size_t *bytes);

/*
 * Group-by of `keys` (DEVICE, int32/int64) with 0..2 value columns (HOST array
 * of DEVICE int32/int64 columns of the same length). Group t (in no particular
 * order): out_keys[t] (key dtype), out_counts[t] = its rows, out_sums[c][t] =
 * the sum of vals[c] over its rows (int64, mod 2^64). out_* are DEVICE arrays
 * of out_capacity entries (out_sums: HOST array of DEVICE pointers);
 * out_capacity == 0 counts the groups only. *out_groups (HOST) = number of
 * groups. EIGER_ERR_CAPACITY when the groups exceed out_capacity;
 * EIGER_ERR_TOO_LARGE when they exceed plan.slots (the estimate was too low:
 * plan again with more slots); EIGER_ERR_UNSUPPORTED for int64 keys that take
 * both INT64_MIN and INT64_MAX. Synchronizes `stream`.
 */
int eiger_groupby(eiger_column keys, const eiger_column *vals, int32_t n_vals, const eiger_groupby_plan_t *plan,
                  void *out_keys, int64_t *out_counts, int64_t *const *out_sums, int64_t out_capacity,
                  int64_t *out_groups, void *ws, size_t ws_bytes, void *stream);

/* ---- sorting and smart key fusion (Sections 3.6 and 4.3, Algorithm 1) ----------
 * A sort on one numeric key is a radix sort; several numeric keys are first
 * fused into one 4- or 8-byte key (smart key fusion) and then radix-sorted. The
 * same fused key turns a join on several key columns into a single-key join.
 */

/* Workspace bytes for eiger_sort_pairs with these arguments. */
int eiger_sort_pairs_workspace_size(int32_t key_bytes, int64_t n, int32_t key_bits, size_t *bytes);

/*
 * Stable LSD radix sort of n (key, value) pairs, ascending by the unsigned value
 * of the key's low key_bits bits (bits above are ignored, so pass keys below
 * 2^key_bits). key_bytes 4 or 8 (uint32 / uint64 keys); key_bits 0..8*key_bytes
 * sets the number of passes (ceil(key_bits / 8)). keys_in, vals_in, keys_out,
 * vals_out: DEVICE arrays of n entries; vals_in == NULL sorts the row ids
 * 0..n-1 along (vals_out is then the stable sorting permutation). Outputs must
 * not alias inputs. Does not synchronize `stream`.
 */
int eiger_sort_pairs(int32_t key_bytes, const void *keys_in, const uint32_t *vals_in, int64_t n, int32_t key_bits,
                     void *keys_out, uint32_t *vals_out, void *ws, size_t ws_bytes, void *stream);

#define EIGER_SKF_MAX_KEYS 8
#define EIGER_SKF_FOR_MAX_BITS 16        /* default: keys whose range fits 16 bits take frame of reference */
#define EIGER_SKF_DICT_MAX_NDV (1 << 20) /* default: keys of up to 2^20 distinct values take the dictionary */
typedef enum { EIGER_SKF_FOR = 0, EIGER_SKF_DICT = 1 } eiger_skf_code;

typedef struct {
    int32_t code;       /* eiger_skf_code */
    int32_t bits;       /* width of the key's code inside the fused key */
    int32_t shift;      /* position of the code's lowest bit in the fused key */
    int32_t descending; /* 1: the key sorts descending (its code is complemented within its width) */
    int64_t base;       /* FOR: the minimum subtracted from every key */
    int64_t ndv;        /* DICT: distinct estimate in a plan, exact count after eiger_skf_fuse */
    int64_t slots;      /* DICT: slots of the encoding's hash table (power of two) */
    int32_t dtype;      /* EIGER_INT32 / EIGER_INT64 */
    int32_t range_bits; /* bit width of max - min (DICT: the sort width of the distinct values) */
} eiger_skf_key_t;

typedef struct {
    int32_t n_keys;
    int32_t total_bits;  /* sum of the key widths */
    int32_t fused_bytes; /* 4 or 8; 0: the codes need more than 64 bits and cannot be fused */
    int32_t reserved;
    eiger_skf_key_t key[EIGER_SKF_MAX_KEYS];
} eiger_skf_plan_t;

/*
 * Smart key fusion plan (Section 4.3) from per-key statistics (HOST arrays of
 * n_keys entries; stats from eiger_stats). Per key, in order: a range max - min
 * of at most for_max_bits bits takes frame-of-reference encoding at that width;
 * otherwise an HLL distinct estimate of at most dict_max_ndv takes the
 * order-preserving dictionary (its width is set from the exact count when
 * eiger_skf_fuse encodes it; the plan holds the estimate's width); otherwise the
 * key keeps its full frame-of-reference width. The first key takes the most
 * significant bits. descending may be NULL (all ascending). Host only.
 */
int eiger_skf_plan(const eiger_stats_t *stats, const int32_t *descending, int32_t n_keys, int32_t for_max_bits,
                   int64_t dict_max_ndv, eiger_skf_plan_t *out);

/* The same plan for a join on n_keys columns of two relations: each key's
 * frame of reference spans both sides' range, its dictionary covers both
 * sides' values (the estimate is the sum of the two estimates), all ascending. */
int eiger_skf_plan_join(const eiger_stats_t *build_stats, const eiger_stats_t *probe_stats, int32_t n_keys,
                        int32_t for_max_bits, int64_t dict_max_ndv, eiger_skf_plan_t *out);

/* Workspace bytes for eiger_skf_fuse / eiger_sort_multikey with this plan and these row counts. */
int eiger_skf_workspace_size(const eiger_skf_plan_t *plan, int64_t n_a, int64_t n_b, int32_t sort, size_t *bytes);

/*
 * Fuse the key columns of one relation (keys_a, n_keys DEVICE columns of equal
 * length) or of two (keys_b, same key dtypes; NULL for one) into one key per row:
 * dictionary keys are encoded over all rows of both relations together
 * (Algorithm 1: hash-table group ids with a leader per value, the distinct values
 * retrieved, sorted, and their positions scattered to the groups and gathered
 * by every row), then each row's codes are shifted into place (Section 4.3).
 * out_a / out_b: DEVICE, 8 bytes per row of capacity; they receive uint32 keys
 * when out_plan->fused_bytes == 4, uint64 keys when 8. *out_plan (HOST) is the
 * plan with each dictionary key's exact count and width. Comparing fused keys as
 * unsigned integers orders rows lexicographically by the keys (ascending or
 * descending per key); equal fused keys mean equal key tuples.
 * EIGER_ERR_UNSUPPORTED when the exact widths need more than 64 bits (*out_plan
 * is still set); EIGER_ERR_TOO_LARGE when a key has more distinct values than
 * half its table's slots (plan again with more slots). Synchronizes `stream`.
 */
int eiger_skf_fuse(const eiger_column *keys_a, const eiger_column *keys_b, int32_t n_keys,
                   const eiger_skf_plan_t *plan, void *out_a, void *out_b, eiger_skf_plan_t *out_plan, void *ws,
                   size_t ws_bytes, void *stream);

/*
 * Multi-key sort (Section 3.6, case 2): eiger_skf_fuse on one relation, then
 * eiger_sort_pairs of the fused keys with the row ids. out_perm (DEVICE, n
 * uint32): rows in sorted order (stable: equal key tuples keep their row order).
 * out_sorted (DEVICE, 8 bytes per row of capacity, may be NULL): the sorted
 * fused keys, 4 or 8 bytes each as out_plan->fused_bytes says. Synchronizes
 * `stream`; errors as eiger_skf_fuse.
 */
int eiger_sort_multikey(const eiger_column *keys, int32_t n_keys, const eiger_skf_plan_t *plan, uint32_t *out_perm,
                        void *out_sorted, eiger_skf_plan_t *out_plan, void *ws, size_t ws_bytes, void *stream);

/*
 * Order-preserving dictionary encoding of one column (Algorithm 1): out_codes
 * (DEVICE, n uint32) = the rank of each row's value among the column's distinct
 * values; out_dict (DEVICE, key dtype, dict_capacity entries, may be NULL) = the
 * distinct values ascending; *out_ndv (HOST) = their number. slots: hash-table
 * slots (power of two >= 2); EIGER_ERR_TOO_LARGE when the column has more than
 * slots / 2 distinct values, EIGER_ERR_CAPACITY when more than dict_capacity
 * (with out_dict given). Synchronizes `stream`.
 */
int eiger_dict_encode_workspace_size(eiger_column col, int64_t slots, size_t *bytes);
int eiger_dict_encode(eiger_column col, int64_t slots, uint32_t *out_codes, void *out_dict, int64_t dict_capacity,
                      int64_t *out_ndv, void *ws, size_t ws_bytes, void *stream);

/* Bytes of the fixed device scratch array behind eiger_join_noalloc (64 MiB). */
#define EIGER_NOALLOC_SCRATCH_BYTES (64u * 1024u * 1024u)

/*
 * eiger_join for callers that cannot allocate device memory (code under HIP
 * graph capture setup, tight serving loops, hosts that forbid hipMalloc): the
 * same join, arguments and results, but its scratch memory is a fixed array of
 * EIGER_NOALLOC_SCRATCH_BYTES inside the library (one per GPU, held until the
 * process ends) instead of a caller workspace. The library allocates nothing.
 * The caller still passes inputs and DEVICE outputs.
 *  - Returns EIGER_ERR_TOO_LARGE, before any GPU work, when the plan's
 *    workspace (eiger_join_workspace_size) exceeds EIGER_NOALLOC_SCRATCH_BYTES.
 *  - `stream` must belong to the current device (EIGER_ERR_INVALID_ARG otherwise).
 *  - All calls on one GPU share its array: calls that overlap in time on one GPU
 *    (different streams or threads) race and must be serialized by the caller.
 * Synchronizes `stream`.
 */
int eiger_join_noalloc(eiger_column build_keys, eiger_column build_payload, eiger_column probe_keys,
                       eiger_column probe_payload, const eiger_plan_t *plan, uint32_t *out_build_rowid,
                       uint32_t *out_probe_rowid, int64_t out_capacity, int64_t *out_count,
                       int64_t *out_checksum, void *stream);

/* ---- batched joins: many independent joins in one graph launch -----------------
 * Every join of a batch runs the same path (statistics of the build keys ->
 * per-join variant choice on the device -> build -> probe -> materialize) with
 * no host round trip: the work of all joins is captured once into a hipGraph
 * whose kernels walk flat lists of (join, tile) work items; each launch replays
 * it. Build keys must be distinct within a join (the usual primary-key side of
 * a star join); a join whose build keys repeat is flagged and its result is
 * not valid (run it through eiger_join instead). Keys share one dtype and
 * payloads one dtype across the batch.
 */
typedef struct {
    const void *build_keys;    /* DEVICE */
    const void *build_payload; /* DEVICE */
    const void *probe_keys;    /* DEVICE */
    const void *probe_payload; /* DEVICE */
    int64_t n_build;
    int64_t n_probe;
} eiger_batch_join;

/* Knobs for the joins whose build side has 2^b .. 2^(b+1)-1 rows (bucket b). */
typedef struct {
    float load_factor;   /* hash-table occupancy, (0, 0.9]; default 0.5 (RADIX: its LDS tables') */
    int32_t probe_tile;  /* probe rows per work item, 256..2^20; default 16384 */
    int32_t radix_bits;  /* 0: the per-join table choice on the device (DIRECT or GLOBAL_HASH);
                            1..16: the bucket's joins run the partitioned RADIX join inside the
                            graph with 2^radix_bits partitions (two passes above 8 bits) */
} eiger_batch_tune;
#define EIGER_BATCH_BUCKETS 33
#define EIGER_BATCH_DUPLICATE_BUILD 1u /* result flag: the join's build keys repeat */
#define EIGER_BATCH_CAPACITY 2u        /* result flag: a RADIX join found more pairs than its
                                          n_probe output slots (its pairs are incomplete) */

/* Workspace bytes for a batch (tune: EIGER_BATCH_BUCKETS entries or NULL for defaults). */
int eiger_join_batch_workspace_size(const eiger_batch_join *joins, int32_t n_joins, int32_t key_dtype,
                                    int32_t payload_dtype, const eiger_batch_tune *tune, size_t *bytes);

/*
 * Capture the batch into a graph (nothing runs yet). The pairs of join j go to
 * out_*_rowid[off_j .. off_j + count_j) with off_j = sum of n_probe over the
 * joins before j (so each array needs sum(n_probe) entries, DEVICE). The
 * handle keeps pointers to the caller's descriptors' data, outputs and
 * workspace; they must stay valid until eiger_join_batch_destroy.
 */
int eiger_join_batch_create(const eiger_batch_join *joins, int32_t n_joins, int32_t key_dtype,
                            int32_t payload_dtype, const eiger_batch_tune *tune, uint32_t *out_build_rowid,
                            uint32_t *out_probe_rowid, void *ws, size_t ws_bytes, void *stream,
                            void **handle);

/* Launch the captured graph on `stream` (asynchronous). */
int eiger_join_batch_launch(void *handle, void *stream);

/* Wait for `stream` and copy per-join results to HOST arrays of n_joins entries
 * (any may be NULL): pair counts, checksums, variant used, EIGER_BATCH_* flags. */
int eiger_join_batch_results(void *handle, int64_t *counts, int64_t *checksums, int32_t *variants,
                             uint32_t *flags, void *stream);

int eiger_join_batch_destroy(void *handle);

/* ---- learned variant selector ---------------------------------------------------
 * A small MLP (EIGER_SEL_FEATURES -> 64 -> 64 -> EIGER_SEL_CLASSES, ReLU) predicts
 * log2(join time in ms) of every plan class from 16 features of the two sides'
 * statistics; EIGER_SEL_LEARNED picks the feasible class with the smallest
 * prediction, except that when that class is GLOBAL_HASH, a GLOBAL_HASH class of
 * larger load factor (smaller table) predicted within 1% of it is taken instead
 * (the largest such load factor). This selector is this library's addition: the paper selects
 * algorithms from runtime statistics (Section 4) but gives no selection model.
 * Parameters are one fp32 array: W1[16][64], b1[64], W2[64][64], b2[64],
 * W3[64][16], b3[16] (row-major, input index first). Training runs on the GPU
 * with the kernels below (fp32, fixed summation order, no float atomics, so two
 * runs on the same data give bit-identical parameters).
 */
#define EIGER_SEL_FEATURES 16
#define EIGER_SEL_CLASSES 16
#define EIGER_MLP_HIDDEN 64

/* Number of fp32 parameters of the selector MLP (6288). */
int64_t eiger_mlp_param_count(void);

/* Features of a (build, probe) pair of statistics, un-normalized (HOST out[16]),
 * in this order (R = build, S = probe, d = distinct estimate, r = max - min + 1):
 * log2(1+|R|), log2(1+|S|), log2(1+d_R), log2(1+d_S), log2(1+r_R), log2(1+r_S),
 * 1 for int64 keys else 0, min(1, d_R/|R|), min(1, d_S/|S|), log2(|R|/d_R) (>= 0),
 * log2(d_R/r_R) clamped to [-64, 0], overlap of the key ranges as a share of r_S,
 * log2(|S|/|R|), log2(1 + |R||S|/max(d_R, d_S) * overlap), log2(1 + |S|/d_R),
 * log2(1 + d_S/d_R). All are finite for any valid statistics. */
int eiger_selector_features(const eiger_stats_t *build, const eiger_stats_t *probe, float *out);

/* The plan of class `cls` (0..EIGER_SEL_CLASSES-1) for these statistics.
 * Returns EIGER_ERR_UNSUPPORTED when the class cannot run them (DIRECT over a
 * key range above 2^30). */
int eiger_selector_class_plan(int32_t cls, const eiger_stats_t *build, const eiger_stats_t *probe,
                              eiger_plan_t *out);

/* Forward pass on the GPU: y[batch][16] = MLP(x[batch][16]). All DEVICE
 * pointers; x is already normalized. */
int eiger_mlp_forward(const float *params, const float *x, int32_t batch, float *y, void *stream);

/* Workspace bytes of eiger_mlp_train_step for a batch. */
size_t eiger_mlp_train_workspace_size(int32_t batch);

/*
 * One full-batch training step on the GPU: forward, masked mean squared error
 * L = sum(mask * (y - target)^2) / sum(mask), backward, and an Adam update
 * (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected with step number `step` >= 1).
 *  params, adam_m, adam_v  DEVICE, eiger_mlp_param_count() floats each, updated in place
 *  grads                   DEVICE, eiger_mlp_param_count() floats (gradients on return)
 *  x, target, mask         DEVICE, batch x 16 floats (mask entries 0 or 1)
 *  loss                    DEVICE, 1 float: the loss before the update
 */
int eiger_mlp_train_step(float *params, float *adam_m, float *adam_v, float *grads, const float *x,
                         const float *target, const float *mask, int32_t batch, float lr, int32_t step,
                         float *loss, void *ws, size_t ws_bytes, void *stream);

/* Install the model used by EIGER_SEL_LEARNED (HOST arrays, copied):
 * params (eiger_mlp_param_count floats) and the feature normalization
 * x_norm = (x - mean) / std (16 floats each, std > 0). Process-wide.
 * feat_lo / feat_hi (16 floats each, lo <= hi, or both NULL) give the box of
 * raw features the model was trained on: for statistics whose features fall
 * outside it, EIGER_SEL_LEARNED returns the rule plan (EIGER_SEL_RULE) and sets
 * EIGER_PLAN_RULE_FALLBACK in plan.flags, since the model's predictions there are
 * extrapolations. Both NULL: no domain check. One of them NULL:
 * EIGER_ERR_INVALID_ARG. */
int eiger_selector_load(const float *params, const float *feat_mean, const float *feat_std,
                        const float *feat_lo, const float *feat_hi);

/* 1 when a model is installed, else 0. */
int eiger_selector_loaded(void);

/* ---- diagnostics -------------------------------------------------------------- */

/* Message of the calling thread's last failure ("" if none). */
const char *eiger_last_error(void);

/* Library version as major * 10000 + minor * 100 + patch. */
int eiger_version(void);

/* Per-kernel timing with HIP events recorded on the launch stream around each
 * kernel the library launches. Off by default; enabling it clears the table. */
typedef struct {
    char name[48];
    int64_t launches;
    double total_ms;
} eiger_kernel_time_t;

int eiger_profile_enable(int on);
/* Copies up to max_entries rows into HOST `out`, sets *n_out to the number of
 * distinct kernels seen. Resolves pending events (synchronizes them). */
int eiger_profile_read(eiger_kernel_time_t *out, int max_entries, int *n_out);

/* Bandwidth ceilings for measurement reports (not part of the join path),
 * timed with HIP events on `stream`; *ms (HOST) receives the kernel time.
 *  kind 0  copy n_bytes (a multiple of 16) from DEVICE a to DEVICE b with
 *          16-byte loads and stores (read + write bytes = 2 n_bytes)
 *  kind 1  `reads` random 32-byte reads (8 in flight per thread) from the
 *          DEVICE table a of n_bytes (the largest power-of-two number of
 *          32-byte slots that fits is used); DEVICE b receives one 4-byte word
 *          per 64 reads
 * Synchronizes `stream`. */
int eiger_calibrate(int32_t kind, void *a, void *b, int64_t n_bytes, int64_t reads, double *ms, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* EIGER_H */
