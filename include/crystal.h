/*
 * crystal.h -- C ABI of a tile-based fused query library for AMD MI355X (gfx950).
 *
 * The library implements the tile-based execution model of Shanbhag, Madden
 * and Yu, "A Study of the Fundamental Performance Characteristics of GPUs and
 * CPUs for Database Analytics" (SIGMOD 2020), section 3.2: a workgroup is the
 * unit of execution and processes a tile of BLOCK x IPT items held in
 * registers, so one kernel per query runs selection, projection, hash-join
 * probes and aggregation with no intermediate result written to memory.
 *
 * Conventions shared by every call:
 *  - Column, table and output pointers are DEVICE pointers owned by the caller.
 *    The library never allocates or frees device memory.
 *  - Column pointers must be 16-byte aligned (the kernels issue 128-bit loads);
 *    a misaligned pointer is rejected with CRYSTAL_EINVAL.
 *  - Every call is asynchronous on `stream` (a hipStream_t passed as void*;
 *    NULL means the default stream).  Host-detectable argument errors are
 *    returned synchronously and nothing is launched.
 *  - Outputs are overwritten: the library clears them on the stream first.
 *  - Device-detectable errors (duplicate key, full table, key or group index
 *    out of range) are recorded in a caller-provided device int32 `status`
 *    word with a compare-and-swap from 0, so the first error sticks.  The
 *    library never clears `status`; the caller zeroes it and reads it after
 *    synchronising the stream.
 *  - Functions are reentrant.  The only global state is the tile-size tuning
 *    table (crystal_tune_*), which calls read and tuning calls write; do not
 *    tune while other threads launch.
 */
#ifndef CRYSTAL_H
#define CRYSTAL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum crystal_status {
    CRYSTAL_OK = 0,
    CRYSTAL_EINVAL = 1,   /* bad argument (null, negative size, misaligned, bad plan)   */
    CRYSTAL_ESCRATCH = 2, /* caller-provided scratch or slot memory too small           */
    CRYSTAL_EFULL = 3,    /* hash table has no free slot (device status)                */
    CRYSTAL_EDUPKEY = 4,  /* duplicate build key (device status)                        */
    CRYSTAL_EHIP = 5,     /* HIP runtime or launch error                                */
    CRYSTAL_EBUSY = 6,    /* shared-scan batch or server has no free slot               */
    CRYSTAL_ERANGE = 7,   /* key outside a direct table, or group index outside the
                             dense group array (device status); the row is skipped     */
    CRYSTAL_ETIMEDOUT = 8 /* served query dropped at its deadline                       */
} crystal_status;

/* Inclusive int32 range lo <= x <= hi.  lo > hi is the empty range. */
typedef struct crystal_range {
    int32_t lo;
    int32_t hi;
} crystal_range;

/* Human-readable name of a status code.  Never NULL. */
const char *crystal_status_string(int32_t status);

/* ABI version of this header (incremented on any layout change). */
#define CRYSTAL_ABI_VERSION 10
int32_t crystal_abi_version(void);

/* sizeof of the ABI structs as compiled into the library, so a binding can
 * check its own layout: 0 crystal_range, 1 crystal_ht, 2 crystal_pred,
 * 3 crystal_join, 4 crystal_star_query, 5 crystal_qmask_table,
 * 6 crystal_batch_query, 7 crystal_batch, 8 crystal_server_template,
 * 9 crystal_server_config, 10 crystal_server_stats, 11 crystal_ht_build_item,
 * 12 crystal_col_format, 13 crystal_qmask_build_item.  0 for any other value. */
size_t crystal_struct_size(int32_t which);

/* ------------------------------------------------------------------------ */
/* Selection -- section 4.2, query Q3 (and section 3.2, query Q0):           */
/*   SELECT y FROM R WHERE pred.lo <= y <= pred.hi                           */
/* One kernel: BlockLoad, BlockPred, BlockScan of the match counts,         */
/* BlockShuffle of the matches into an LDS buffer of two tiles; when the     */
/* buffer could not take another tile, thread 0 reserves its output range    */
/* with one 64-bit atomic on *out_count and the buffer is stored coalesced.  */
/*   in        device, n int32 values                                        */
/*   out       device, capacity for every match (n values always suffice)    */
/*   out_count device int64; cleared, then the number of matches             */
/* Output order: the matches of a tile are contiguous, in a fixed order      */
/* within the tile (wave by wave; within a wave, item slot by item slot,     */
/* lane by lane); tiles follow the order in which their reservations         */
/* completed, which varies between runs.  The multiset of values and the     */
/* count are exact.                                                          */
/* ------------------------------------------------------------------------ */
crystal_status crystal_select(const int32_t *in, int64_t n, crystal_range pred,
                              int32_t *out, int64_t *out_count, void *stream);

/* The same selection with the qualifying values in input order (a stable    */
/* compaction, identical on every run).  Each tile publishes its match count */
/* in its own status word and finds its output offset by decoupled look-back */
/* over its predecessors' words instead of an atomic reservation; slower on  */
/* MI355X, whose eight XCD caches are not coherent, so every look-back round */
/* is a memory round trip.                                                   */
/*   scratch   device, >= crystal_select_stable_scratch_bytes(n) bytes,      */
/*             16-byte aligned (tile status words); calls sharing it must be */
/*             ordered on one stream                                         */
/*   out_count the number of matches, or -1 if a tile's wait for its         */
/*             predecessors gave up (ruled out by in-order dispatch)          */
size_t crystal_select_stable_scratch_bytes(int64_t n);
crystal_status crystal_select_stable(const int32_t *in, int64_t n, crystal_range pred,
                                     int32_t *out, int64_t *out_count, void *scratch,
                                     size_t scratch_bytes, void *stream);

/* ------------------------------------------------------------------------ */
/* Projection -- section 4.1, query Q1:  SELECT a*x1 + b*x2 FROM R          */
/* fp32, each product and the sum rounded to nearest-even, no fused          */
/* multiply-add.  x1, x2, out: device, n floats.                             */
/* ------------------------------------------------------------------------ */
crystal_status crystal_project(const float *x1, const float *x2, int64_t n,
                               float a, float b, float *out, void *stream);

/* Section 4.1, query Q2:  SELECT sigmoid(a*x1 + b*x2) FROM R, with
 * sigmoid(t) = 1 / (1 + e^-t) evaluated in fp32 with the device expf. */
crystal_status crystal_project_sigmoid(const float *x1, const float *x2, int64_t n,
                                       float a, float b, float *out, void *stream);

/* ------------------------------------------------------------------------ */
/* Hash tables -- section 4.3 (build and probe phases, linear probing) and   */
/* section 5.3 (perfect hashing of dense dimension keys).                    */
/*                                                                          */
/* CRYSTAL_HT_LINEAR: open addressing with linear probing.  capacity is the  */
/*   smallest power of two >= max(64, 2 * n_keys) (at most 50% fill); each   */
/*   slot is 8 bytes {int32 key, int32 payload}; the empty key is INT32_MIN, */
/*   which therefore cannot be inserted.  Slot of key k: multiplicative      */
/*   hashing, (k * 2654435761 mod 2^32) >> (32 - log2 capacity), then the    */
/*   following slots in order.                                               */
/* CRYSTAL_HT_DIRECT: one entry per key in [key_min, key_max] (perfect       */
/*   hashing): a presence bitmap of ceil(span/32) 32-bit words padded to a   */
/*   multiple of 64 words, followed by span int32 payloads if has_payload.   */
/* ------------------------------------------------------------------------ */
enum { CRYSTAL_HT_LINEAR = 0, CRYSTAL_HT_DIRECT = 1 };

typedef struct crystal_ht {
    void *mem;             /* device memory of crystal_ht_bytes() bytes (caller-owned) */
    int64_t capacity;      /* LINEAR: number of slots; DIRECT: key span                 */
    int32_t kind;          /* CRYSTAL_HT_LINEAR or CRYSTAL_HT_DIRECT                    */
    int32_t key_min;       /* DIRECT: key stored in entry 0                             */
    int32_t has_payload;   /* 0: keys only (a probe sums 0 per match)                   */
    int32_t log2_capacity; /* LINEAR: log2(capacity)                                    */
} crystal_ht;

/* Host only: fill the descriptor for a table that will hold up to n_keys keys
 * (LINEAR) or every key of [key_min, key_max] (DIRECT); sets mem = NULL. */
crystal_status crystal_ht_init(crystal_ht *ht, int32_t kind, int64_t n_keys,
                               int32_t key_min, int32_t key_max, int32_t has_payload);
/* Device bytes the described table needs (0 for an invalid descriptor). */
size_t crystal_ht_bytes(const crystal_ht *ht);

/* Build phase: clear the table, then insert (keys[i], payload[i]) for every
 * row i < n whose filter_col[i] lies in `filter` (all rows when filter_col is
 * NULL).  payload may be NULL only for a table without payload.  Duplicate
 * keys set CRYSTAL_EDUPKEY, a full LINEAR table CRYSTAL_EFULL, a key outside a
 * DIRECT table's span CRYSTAL_ERANGE, the empty key CRYSTAL_EINVAL, in
 * *status.  One thread per row; a 64-bit compare-and-swap claims a slot. */
crystal_status crystal_ht_build(const crystal_ht *ht, const int32_t *keys,
                                const int32_t *payload, const int32_t *filter_col,
                                crystal_range filter, int64_t n, int32_t *status,
                                void *stream);

/* Probe phase of query Q4 (section 4.3):
 *   SELECT SUM(A.v + B.v) FROM A, B WHERE A.k = B.k
 * with A the built table and B the probe rows (fk[i], probe_payload[i]).
 *   *out_sum     device int64: sum of the table payload of every match, plus
 *                probe_payload[i] when probe_payload is not NULL (wraps mod 2^64)
 *   *out_matches device int64: number of probe rows that found their key
 * Tables that fit the workgroup's LDS are staged there once per workgroup. */
/* Build several tables in one call (section 5.3: the build phase of a star
 * query builds one table per dimension before the single probe kernel).
 * Same result, per item, as crystal_ht_build on it; the tables are cleared
 * by one kernel and built by a second one whose workgroups are split among
 * them, instead of two launches per table.  Items must use distinct table
 * memory; n_items <= CRYSTAL_MAX_BUILD_BATCH.  `ht` points to a host
 * descriptor; the other pointers are device memory as in crystal_ht_build. */
#define CRYSTAL_MAX_BUILD_BATCH 8
typedef struct {
    const crystal_ht *ht;
    const int32_t *keys;
    const int32_t *payload;    /* NULL unless ht->has_payload */
    const int32_t *filter_col; /* NULL: no build filter */
    crystal_range filter;
    int64_t n;
} crystal_ht_build_item;
crystal_status crystal_ht_build_batch(const crystal_ht_build_item *items, int32_t n_items, int32_t *status,
                                      void *stream);

/* The build phase of a repeated star query in one launch (section 5.3: the
 * dimension builds before the probe kernel), for a caller that alternates
 * between two sets of tables: the items' tables must already be clear (an
 * earlier call listed them in `clear`), and the same launch
 *   - builds every item, with the same result as crystal_ht_build_batch,
 *   - clears the n_clear tables in `clear` (the other set, for the next call),
 *   - sets the zero_n int64 at `zero` to 0 (e.g. the group array that a
 *     following crystal_run_star_query_accumulate adds into; NULL when
 *     zero_n is 0).
 * So one step of a repeated query is two launches (this and the fused
 * kernel) instead of four (clear, build, output clear, kernel).
 * To start, clear both sets with a call that has no items.
 * Errors (CRYSTAL_EINVAL, nothing launched): n_items or n_clear outside
 * 0..CRYSTAL_MAX_BUILD_BATCH, an invalid descriptor, zero_n < 0, zero NULL
 * or not 8-byte aligned with zero_n > 0, or any two of the items' tables,
 * the cleared tables and the zeroed range sharing memory.  `clear` and the
 * descriptors are host memory; table memory, columns, `zero` and `status`
 * are device memory; device errors of the builds go to *status as in
 * crystal_ht_build. */
crystal_status crystal_ht_build_batch_fused(const crystal_ht_build_item *items, int32_t n_items,
                                            const crystal_ht *const *clear, int32_t n_clear, int64_t *zero,
                                            int64_t zero_n, int32_t *status, void *stream);

crystal_status crystal_ht_probe(const crystal_ht *ht, const int32_t *fk,
                                const int32_t *probe_payload, int64_t n,
                                int64_t *out_sum, int64_t *out_matches, void *stream);

/* ------------------------------------------------------------------------ */
/* Dense group-by aggregate (the aggregation table of section 5.3 in the     */
/* dense form small group keys allow):  sums[group[i]] += value[i]  (int64). */
/* Rows whose group lies outside [0, n_groups) are skipped and set           */
/* CRYSTAL_ERANGE in *status.  sums: device, n_groups int64, overwritten.     */
/* ------------------------------------------------------------------------ */
crystal_status crystal_groupby_agg(const int32_t *group, const int32_t *value, int64_t n,
                                   int64_t n_groups, int64_t *sums, int32_t *status,
                                   void *stream);

/* ------------------------------------------------------------------------ */
/* Fused star query -- section 3.1 (SSB Q1.1) and section 5.3 (SSB Q2.1):   */
/*   SELECT agg FROM fact, dim_1..dim_J                                      */
/*   WHERE fact predicates AND fact.fk_j = dim_j.key AND dimension filters  */
/*   GROUP BY dense index                                                    */
/* One persistent kernel.  Per tile: BlockLoad of the first step's column,  */
/* then BlockLoadSel (only items still alive) of the second step's column,  */
/* each step probing (BlockProbeHT) or testing its predicate and clearing   */
/* the items that fail; rows still alive are compacted into an LDS queue    */
/* (BlockScan + BlockShuffle) and finished in batches: remaining steps, the */
/* group index and the measure, added with 64-bit atomics per survivor      */
/* (grouped) or reduced per workgroup (BlockAggregate) and summed by a      */
/* finalize kernel (single group).  Steps run in plan order: predicates,    */
/* then joins.                                                               */
/*                                                                          */
/* Payload fields: a join may read two fields from the 32-bit payload of    */
/* the matched entry, field = (uint32(payload) >> shift) & (2^bits - 1), or */
/* the whole payload as a signed int32 when bits == 32.                     */
/*   filter_bits > 0: keep the row only if the field lies in `filter`       */
/*                    (dimension predicate evaluated at probe time);        */
/*   group_bits  > 0: group += (field - group_base) * group_stride.          */
/* A table built with a filter (crystal_ht_build) needs no filter field.     */
/* ------------------------------------------------------------------------ */
#define CRYSTAL_MAX_COLS 16
#define CRYSTAL_MAX_PREDS 4
#define CRYSTAL_MAX_JOINS 4

typedef enum crystal_agg {
    CRYSTAL_AGG_SUM = 0,         /* SUM(col0)                                  */
    CRYSTAL_AGG_SUM_PRODUCT = 1, /* SUM(col0 * col1), product in int64         */
    CRYSTAL_AGG_SUM_DIFF = 2,    /* SUM(col0 - col1)                           */
    CRYSTAL_AGG_COUNT = 3        /* COUNT(*)                                   */
} crystal_agg;

typedef struct crystal_pred {
    int32_t col;          /* fact column index                              */
    crystal_range range;  /* keep lo <= fact[col] <= hi                     */
} crystal_pred;

typedef struct crystal_join {
    crystal_ht ht;        /* built dimension table                          */
    int32_t fk_col;       /* fact column holding the foreign key            */
    int32_t filter_bits;  /* 0: no dimension predicate on the payload       */
    int32_t filter_shift;
    crystal_range filter;
    int32_t group_bits;   /* 0: no contribution to the group index          */
    int32_t group_shift;
    int32_t group_base;
    int32_t reserved;
    int64_t group_stride;
} crystal_join;

/* Storage of one fact column (compressed columns, section 5.5's outlook:
 * fewer HBM bytes for a little ALU).  bits == 0: width 0 or 4 means int32
 * values; width 2 or 1 means uint16 or uint8 offsets from `base` (frame of
 * reference), value = base + stored; crystal_pack_column writes such a
 * column.  bits in 1..16 (width 0): a bit-packed column, written by
 * crystal_pack_column_bits: value = base + the `bits`-bit field of the row
 * (layout below). */
typedef struct crystal_col_format {
    int32_t width;
    int32_t base;
    int32_t bits;
    int32_t reserved;
} crystal_col_format;

typedef struct crystal_star_query {
    const int32_t *cols[CRYSTAL_MAX_COLS]; /* fact columns (device; a narrow
                                              column's pointer is cast)     */
    int64_t n_rows;
    int32_t n_cols;
    int32_t n_preds;
    crystal_pred preds[CRYSTAL_MAX_PREDS]; /* evaluated first, in order      */
    int32_t n_joins;
    int32_t agg;                           /* crystal_agg                    */
    int32_t agg_col0;
    int32_t agg_col1;
    int64_t n_groups;                      /* >= 1; 1 means a scalar result  */
    crystal_join joins[CRYSTAL_MAX_JOINS]; /* evaluated after the predicates */
    crystal_col_format formats[CRYSTAL_MAX_COLS]; /* all zero: int32 columns */
} crystal_star_query;

/* Device scratch bytes a call needs: per-workgroup partial sums when the
 * result is a single group (0 for grouped plans or an invalid plan). */
size_t crystal_star_query_scratch_bytes(const crystal_star_query *q);

/* Run one query.  out: device, n_groups int64, overwritten.  scratch: device
 * memory of at least crystal_star_query_scratch_bytes(q) bytes, 16-byte
 * aligned, owned by the caller (may be NULL when that size is 0); too small
 * a buffer returns CRYSTAL_ESCRATCH.  Calls that share a scratch buffer must
 * be ordered on one stream.  A plan with no step aggregates every row. */
crystal_status crystal_run_star_query(const crystal_star_query *q, int64_t *out,
                                      int32_t *status, void *scratch, size_t scratch_bytes,
                                      void *stream);

/* Same as crystal_run_star_query, but adds the query's result into out
 * instead of overwriting it (wrapping modulo 2^64), so one query can be
 * answered over successive row ranges (plans whose cols point at each range
 * in turn) or a caller can clear out itself.  Nothing else is launched
 * besides the query kernel and, for a scalar result, its finalize kernel. */
crystal_status crystal_run_star_query_accumulate(const crystal_star_query *q, int64_t *out,
                                                 int32_t *status, void *scratch, size_t scratch_bytes,
                                                 void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * query and result as crystal_run_star_query, with no caller scratch.  The
 * per-workgroup partials of a scalar result go to a fixed array of
 * CRYSTAL_STAR_NOALLOC_PARTIALS int64 words (64 KiB) that the library holds
 * in each device's memory until the process ends; its address is looked up
 * once per device, on the first call made with that device current.
 * Nothing is allocated, here or later.  Limit: a scalar plan whose
 * crystal_star_query_scratch_bytes exceeds 64 KiB (more than
 * CRYSTAL_STAR_NOALLOC_PARTIALS workgroups, i.e. above about 1.3e11 rows on a
 * 256-CU device) returns CRYSTAL_ESCRATCH and launches nothing.  Grouped
 * plans use no scratch.  Every call on one device shares that device's
 * array: scalar-result calls that overlap on one device (other streams, other
 * threads) race and must be ordered by the caller.  Each workgroup writes its
 * own partial before the finalize kernel reads it, so no clearing is needed
 * between calls. */
#define CRYSTAL_STAR_NOALLOC_PARTIALS 8192
crystal_status crystal_run_star_query_noalloc(const crystal_star_query *q, int64_t *out, int32_t *status,
                                              void *stream);

/* Write a narrow column: out[i] = in[i] - base as a `width`-byte unsigned
 * value (width 1 or 2).  in: device int32[n], 16-byte aligned; out: device,
 * n * width bytes, 16-byte aligned.  A value outside [base, base + 2^(8 width)
 * - 1] is stored truncated and sets *status (device) to CRYSTAL_ERANGE.
 * Narrow columns are read by crystal_run_star_query(_accumulate); the
 * shared-scan batch and the server take int32 columns only (CRYSTAL_EINVAL). */
crystal_status crystal_pack_column(const int32_t *in, int64_t n, int32_t base, int32_t width, void *out,
                                   int32_t *status, void *stream);

/* Bit-packed frame-of-reference column.  The packed form is a stream of
 * 32-bit words, least significant bit first: row i's field in[i] - base
 * occupies stream bits [i * bits, (i + 1) * bits), and stream bit j is bit
 * (j mod 32) of word floor(j / 32).  The buffer holds
 * ceil(n * bits / 32) words and four zero words of padding (readers load
 * whole words past a row's last bit):
 * crystal_packed_column_bytes(n, bits) bytes, 0 when bits is outside 1..16
 * or n < 0.  in: device int32[n], 16-byte aligned; out: device, 16-byte
 * aligned, that many bytes, fully written.  A value outside
 * [base, base + 2^bits - 1] is stored truncated to its low bits and sets
 * *status (device) to CRYSTAL_ERANGE.  Read by
 * crystal_run_star_query(_accumulate) through crystal_col_format.bits. */
size_t crystal_packed_column_bytes(int64_t n, int32_t bits);
crystal_status crystal_pack_column_bits(const int32_t *in, int64_t n, int32_t base, int32_t bits, void *out,
                                        int32_t *status, void *stream);

/* ------------------------------------------------------------------------ */
/* Shared-scan batches: up to CRYSTAL_MAX_BATCH queries of one star-query    */
/* template (same columns, predicate columns, joins, group spec, aggregate;  */
/* each query with its own predicate constants and dimension filters) are    */
/* answered in one pass over a range of fact rows.  Each fact column is read */
/* once per pass and each join costs one 2-byte lookup per row, in the       */
/* batch's query-mask table of that dimension (bit q of entry k: the         */
/* dimension row with key k passes query q's dimension filter).  This is an  */
/* extension of the paper's single-query kernels for serving many queries.   */
/* ------------------------------------------------------------------------ */
#define CRYSTAL_MAX_BATCH 16

typedef struct crystal_qmask_table {
    void *mem;         /* device, 16-byte aligned, caller-owned: crystal_qmask_bytes(span)
                          bytes, or crystal_qmask_ranked_bytes(span, ranked) when ranked > 0 */
    int64_t span;      /* keys key_min .. key_min + span - 1                          */
    int32_t key_min;
    int32_t ranked;    /* 0: one 16-bit entry per key of the span.  > 0: rank-compressed
                          (for a sparse key domain): a directory of the keys present,
                          built once by crystal_qmask_rank, and one entry per present
                          key, at most `ranked` of them                                */
} crystal_qmask_table;

size_t crystal_qmask_bytes(int64_t span);

/* Rank-compressed layout, for a dimension whose keys fill a small part of
 * their span (dates stored as yyyymmdd: 2,556 keys over a span of 61,130):
 *   dir[w], w = 0 .. ceil(span / 32): two 32-bit words, the presence bits of
 *     keys key_min + 32 w .. + 31 and the number of present keys before them;
 *     the last entry has no presence bits (keys past the span read it);
 *   then ranked + 1 16-bit entries, entry r for the present key of rank r,
 *     entry `ranked` always 0 (absent keys read it).
 * A key's entry is found with one directory read and a population count.
 * 0 when ranked <= 0, span <= 0 or span > 2^26. */
size_t crystal_qmask_ranked_bytes(int64_t span, int32_t ranked);

/* Build a ranked table's directory from the dimension's key column keys[n]
 * (device; duplicates count once) and clear its entries.  A key outside the
 * span sets CRYSTAL_ERANGE in *status, more than t->ranked distinct keys
 * CRYSTAL_EFULL (the table is then unusable).  Run once per dimension; the
 * directory stays valid for every later crystal_qmask_build of the table. */
crystal_status crystal_qmask_rank(const crystal_qmask_table *t, const int32_t *keys, int64_t n,
                                  int32_t *status, void *stream);

/* Clear the table's entries, then for every dimension row i < n with key
 * keys[i] set bit q of the key's entry when filter_col[i] lies in ranges[q]
 * (q < n_queries; every row passes when filter_col is NULL).  ranges: HOST
 * array.  A key outside the span, or (ranked table) absent from its
 * directory, sets CRYSTAL_ERANGE in *status. */
crystal_status crystal_qmask_build(const crystal_qmask_table *t, const int32_t *keys,
                                   const int32_t *filter_col, int64_t n,
                                   const crystal_range *ranges, int32_t n_queries,
                                   int32_t *status, void *stream);

/* Build the query-mask tables of several joins in one call: the same
 * result, per item, as crystal_qmask_build on it, from two launches (one
 * clears every table, one builds them all) instead of two per table.  Items
 * must use distinct table memory; n_items <= CRYSTAL_MAX_JOINS.  `t` and
 * `ranges` point to host memory; the other pointers are device memory as in
 * crystal_qmask_build.  This is the call the server makes when a template's
 * set of queries changes. */
typedef struct {
    const crystal_qmask_table *t;
    const int32_t *keys;
    const int32_t *filter_col;    /* NULL: every row passes */
    int64_t n;
    const crystal_range *ranges;  /* n_queries ranges */
    int32_t n_queries;
    int32_t reserved;
} crystal_qmask_build_item;
crystal_status crystal_qmask_build_batch(const crystal_qmask_build_item *items, int32_t n_items,
                                         int32_t *status, void *stream);

typedef struct crystal_batch_query {
    crystal_range preds[CRYSTAL_MAX_PREDS]; /* this query's fact-predicate ranges, plan order */
    int64_t *out;                           /* device, n_groups int64, ACCUMULATED (not cleared) */
} crystal_batch_query;

typedef struct crystal_batch {
    crystal_star_query plan;                    /* template; its predicate ranges are ignored and
                                                   its joins' tables are used for group payloads */
    crystal_qmask_table masks[CRYSTAL_MAX_JOINS]; /* per join, built for this batch's queries */
    int32_t n_queries;                          /* 1 .. CRYSTAL_MAX_BATCH (0: nothing to do) */
    int32_t reserved;
    crystal_batch_query queries[CRYSTAL_MAX_BATCH];
    int64_t row_begin;                          /* fact rows [row_begin, row_end); row_begin % 4 == 0 */
    int64_t row_end;
} crystal_batch;

/* One pass over rows [row_begin, row_end) for every query of the batch,
 * adding into each query's output.  Query q's answer over a row range is the
 * plain star query's answer restricted to those rows, so launches over a
 * partition of the fact table accumulate the full answer. */
crystal_status crystal_run_shared_scan(const crystal_batch *b, int32_t *status, void *stream);

/* ------------------------------------------------------------------------ */
/* Serving: continuous batching of star queries over shared-scan passes.     */
/* The fact table is cut into segments of segment_rows rows; a server       */
/* thread runs a clock whose every step scans the next segment once per     */
/* template for all queries in that template's slots (crystal_run_shared_   */
/* scan, outputs accumulated per slot).  A query admitted at step p is done */
/* after one full cycle of segments; its slot output is copied to pinned    */
/* host memory and the slot is reused.  Requests that arrive while others   */
/* run wait in a FIFO per template (at most max_queue; beyond that submit   */
/* returns CRYSTAL_EBUSY) and are admitted into free slots at the next      */
/* step.  Slot memory is the admission budget: the workspace holds          */
/* slots_per_template outputs per template.                                  */
/* ------------------------------------------------------------------------ */
#define CRYSTAL_SERVER_MAX_TEMPLATES 4

typedef struct crystal_server_template {
    crystal_star_query plan;                      /* template plan over the one fact table      */
    const int32_t *dim_keys[CRYSTAL_MAX_JOINS];   /* per join: dimension key column (device)    */
    const int32_t *dim_filter[CRYSTAL_MAX_JOINS]; /* per join: dimension filter column (device) */
    int64_t dim_rows[CRYSTAL_MAX_JOINS];
    crystal_qmask_table masks[CRYSTAL_MAX_JOINS]; /* per join: its own mask table (caller-owned; a
                                                     ranked one's directory built beforehand) */
} crystal_server_template;

typedef struct crystal_server_config {
    int32_t n_templates;          /* 1 .. CRYSTAL_SERVER_MAX_TEMPLATES                         */
    int32_t slots_per_template;   /* 1 .. CRYSTAL_MAX_BATCH concurrent queries per template     */
    int64_t segment_rows;         /* rows per clock step, a multiple of 4                       */
    int32_t max_queue;            /* waiting requests per template                              */
    int32_t inflight_steps;       /* steps issued ahead of the oldest unfinished one (1 .. 64)  */
    void *workspace;              /* device, >= crystal_server_workspace_bytes(), 16-byte aligned */
    size_t workspace_bytes;
    void *stream;                 /* hipStream_t to launch on; NULL: the server creates one     */
    int32_t fake_executor;        /* 1: no GPU work, every step takes fake_step_ns (tests)      */
    int32_t reserved;
    int64_t fake_step_ns;
    crystal_server_template templates[CRYSTAL_SERVER_MAX_TEMPLATES];
} crystal_server_config;

typedef struct crystal_server_stats {
    int64_t admitted, completed, rejected, queued, steps, busy_slot_steps, n_segments, cancelled, timed_out;
} crystal_server_stats;

typedef struct crystal_server crystal_server;

size_t crystal_server_workspace_bytes(const crystal_server_config *cfg);
/* Validates the configuration, starts the server thread. */
crystal_status crystal_server_create(const crystal_server_config *cfg, crystal_server **out);
/* Queue one query of template_id with its constants: preds[i] for the
 * template's fact predicates, dim_filters[j] for its joins' dimension filter
 * columns (host arrays).  Returns a ticket.  deadline_ns > 0: a query not
 * complete that many nanoseconds after submission is dropped (from the
 * queue, or from its slot if its last segment has not been issued yet) and
 * polls as CRYSTAL_ETIMEDOUT; 0: no deadline. */
crystal_status crystal_server_submit(crystal_server *s, int32_t template_id, const crystal_range *preds,
                                     const crystal_range *dim_filters, int64_t deadline_ns, int64_t *ticket);
/* Withdraw a query: a queued one leaves its queue, a running one frees its
 * slot at the next clock step (unless its last segment is already on the
 * GPU; the slot is then freed when that step completes), a finished one's
 * result is discarded.  The ticket is released: polling it returns
 * CRYSTAL_EINVAL.  Unknown ticket: CRYSTAL_EINVAL. */
crystal_status crystal_server_cancel(crystal_server *s, int64_t ticket);
/* *done = 1 once the query has finished; then its n_groups int64 result is
 * copied into `result` (host, may be NULL), *latency_ns is the time from
 * submit to completion, and the ticket is released.  A query dropped at its
 * deadline returns CRYSTAL_ETIMEDOUT with *done = 1 (no result; the ticket
 * is released).  result_capacity: the
 * number of int64 values `result` holds; less than the n_groups of the
 * ticket's template returns CRYSTAL_EINVAL and copies nothing.
 * Device errors: the kernels' status word is copied back with every step
 * that completes a query and checked before that step's results are
 * released; a nonzero code (CRYSTAL_ERANGE for a dimension key outside its
 * mask table or a group index outside the group array, CRYSTAL_EFULL for a
 * full ranked table) stops the server, and this call, crystal_server_submit
 * and crystal_server_get_stats return that code from then on. */
crystal_status crystal_server_poll(crystal_server *s, int64_t ticket, int64_t *result, int64_t result_capacity,
                                   int32_t *done, int64_t *latency_ns);
crystal_status crystal_server_get_stats(crystal_server *s, crystal_server_stats *out);
/* Stops the thread after the work on the GPU has drained; frees the server. */
crystal_status crystal_server_destroy(crystal_server *s);

/* ------------------------------------------------------------------------ */
/* HIP graphs: record every crystal_* call made on `stream` between begin and */
/* end (stream capture), then replay the whole launch sequence with one call. */
/* The library clears outputs and tables with fill kernels, never memset     */
/* nodes, so each replay recomputes every result from its inputs.  Pointers  */
/* and plan constants are frozen at capture; make one eager call of each     */
/* entry point on the device before capturing (it caches device attributes). */
/* ------------------------------------------------------------------------ */
typedef struct crystal_graph crystal_graph;
crystal_status crystal_graph_begin(void *stream);
crystal_status crystal_graph_end(void *stream, crystal_graph **out);
crystal_status crystal_graph_launch(crystal_graph *g, void *stream);
crystal_status crystal_graph_destroy(crystal_graph *g);

/* ------------------------------------------------------------------------ */
/* Radix partitioning and sort (section 4.4).                               */
/*                                                                          */
/* Keys and values are 32-bit words in device memory; keys are ordered as   */
/* unsigned integers (flip bit 31 of a signed key to sort it as signed).    */
/* A pass with radix `bits` (1..8) and start bit `shift` (shift + bits <=   */
/* 32) uses the digit (key >> shift) & (2^bits - 1).  n must be below 2^32. */
/* Inputs are never modified; outputs must not overlap the inputs.          */
/* ------------------------------------------------------------------------ */

/* Histogram phase: hist[d] (device, 2^bits words, overwritten) = number of  */
/* keys whose digit is d.                                                    */
crystal_status crystal_radix_histogram(const uint32_t *keys, int64_t n, int32_t shift, int32_t bits,
                                       uint32_t *hist, void *stream);

/* Scratch (device, 256-byte aligned) of one partition pass over n keys     */
/* with the current tuning: the per-workgroup digit counts and their        */
/* prefix sums.                                                             */
size_t crystal_radix_partition_scratch_bytes(int64_t n);

/* One partition pass: histogram + shuffle.  Writes the pairs into 2^bits   */
/* contiguous partitions in digit order, stably (pairs with equal digits    */
/* keep their input order).  vals / out_vals: both null (keys only) or both */
/* device arrays of n words.  part_offsets: null, or device array of        */
/* 2^bits + 1 words that receives the start of each partition and n.        */
/* Scratch too small: CRYSTAL_ESCRATCH.  Calls sharing scratch race.        */
crystal_status crystal_radix_partition(const uint32_t *keys, const uint32_t *vals, int64_t n, int32_t shift,
                                       int32_t bits, uint32_t *out_keys, uint32_t *out_vals,
                                       uint32_t *part_offsets, void *scratch, size_t scratch_bytes,
                                       void *stream);

/* The same pass with the unstable shuffle of section 4.4: the partitions,
 * their bounds and the pairs in each partition are those of
 * crystal_radix_partition, but pairs with equal digits may appear in any
 * order within their partition.  Cheaper per item (no ballot ranking). */
crystal_status crystal_radix_partition_unstable(const uint32_t *keys, const uint32_t *vals, int64_t n,
                                                int32_t shift, int32_t bits, uint32_t *out_keys,
                                                uint32_t *out_vals, uint32_t *part_offsets, void *scratch,
                                                size_t scratch_bytes, void *stream);

/* Scratch (device, 256-byte aligned) of crystal_sort_pairs: one ping-pong  */
/* copy of the keys (and of the values when with_values) plus one pass's    */
/* scratch.                                                                 */
size_t crystal_sort_pairs_scratch_bytes(int64_t n, int32_t with_values);

/* Stable sort of n (key, value) pairs by unsigned key: four stable 8-bit   */
/* partition passes from the low byte up.  vals / out_vals as above.        */
crystal_status crystal_sort_pairs(const uint32_t *keys, const uint32_t *vals, int64_t n, uint32_t *out_keys,
                                  uint32_t *out_vals, void *scratch, size_t scratch_bytes, void *stream);

/* MSB radix sort (section 4.4: the GPU sort takes the most significant     */
/* 8-bit digit first).  Same result as crystal_sort_pairs: the stable       */
/* ascending order of the pairs by unsigned key.  Levels of stable 8-bit    */
/* partitions split every segment longer than 8,192 pairs by its next digit */
/* (the first level splits the whole input by the top byte); every shorter  */
/* segment is then sorted in LDS by its remaining low bits by one           */
/* workgroup.  Uniform keys take two partition levels and the local pass.   */
/* Arguments, ownership and errors as crystal_sort_pairs; scratch (device,  */
/* 256-byte aligned) of crystal_sort_pairs_msb_scratch_bytes(n, with_values) */
/* bytes holds one copy of the pairs and the work lists.                    */
size_t crystal_sort_pairs_msb_scratch_bytes(int64_t n, int32_t with_values);
crystal_status crystal_sort_pairs_msb(const uint32_t *keys, const uint32_t *vals, int64_t n, uint32_t *out_keys,
                                      uint32_t *out_vals, void *scratch, size_t scratch_bytes, void *stream);

/* ------------------------------------------------------------------------ */
/* Tile-size tuning (section 3.3: the tile is BLOCK threads x IPT items per */
/* thread; the best shape depends on the kernel and the input).  The table  */
/* maps (kernel, size bucket = floor(log2 n)) to a compiled variant.  A     */
/* grid_per_cu of 0 launches one workgroup per tile; k > 0 launches k       */
/* workgroups per compute unit that stride over the tiles.                  */
/* ------------------------------------------------------------------------ */
enum {
    CRYSTAL_K_SELECT = 0,
    CRYSTAL_K_PROJECT = 1,
    CRYSTAL_K_HT_PROBE = 2,
    CRYSTAL_K_GROUPBY = 3,
    CRYSTAL_K_STAR = 4,
    CRYSTAL_K_SHARED_SCAN = 5,        /* shared-scan batches of grouped templates */
    CRYSTAL_K_RADIX = 6,
    CRYSTAL_K_SHARED_SCAN_SCALAR = 7, /* shared-scan batches of scalar templates  */
    CRYSTAL_K_COUNT = 8
};

/* Number of compiled (block, ipt) variants of `kernel`; fills up to `max`. */
int32_t crystal_tune_variants(int32_t kernel, int32_t *blocks, int32_t *ipts, int32_t max);
/* Set the variant for sizes in bucket [bucket_lo, bucket_hi] (-1, -1: all). */
crystal_status crystal_tune_set(int32_t kernel, int32_t bucket_lo, int32_t bucket_hi,
                                int32_t block, int32_t ipt, int32_t grid_per_cu);
/* Variant that a call of `kernel` on n items would use. */
crystal_status crystal_tune_get(int32_t kernel, int64_t n, int32_t *block, int32_t *ipt,
                                int32_t *grid_per_cu);
/* Restore the built-in defaults. */
void crystal_tune_reset(void);
/* Text cache: one line "kernel bucket_lo bucket_hi block ipt grid_per_cu". */
crystal_status crystal_tune_load(const char *path);
crystal_status crystal_tune_save(const char *path);

#ifdef __cplusplus
}
#endif

#endif /* CRYSTAL_H */
