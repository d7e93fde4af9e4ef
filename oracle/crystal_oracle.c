/*
 * Crystal CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, row-at-a-time C definitions of what the tile-based GPU query
 * path computes (Shanbhag, Madden, Yu, "A Study of the Fundamental Performance
 * Characteristics of GPUs and CPUs for Database Analytics", SIGMOD 2020).
 * Only the test suite, the smoke entry point and the benchmark's CPU-baseline
 * leg may load this library.  It shares no code, header or constant with the
 * HIP path, and the HIP path never calls it.
 *
 * Every function evaluates the SQL statement the paper states, one row at a
 * time, in the order that statement reads.  Integer aggregates are kept in
 * unsigned 64-bit arithmetic (two's-complement wrap modulo 2^64), which is
 * associative and commutative: any summation order gives the same bits.
 * Floating point is evaluated in double precision and rounded once to the
 * 4-byte float the paper fixes for its columns.
 *
 * Return codes: 0 ok, 1 bad argument, 4 duplicate dimension key,
 * 7 group index outside the dense group array.
 */
#define _GNU_SOURCE /* qsort_r: the comparison gets the key column as an argument */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define ORACLE_OK 0
#define ORACLE_EINVAL 1
#define ORACLE_EDUPKEY 4
#define ORACLE_ERANGE 7

/* ------------------------------------------------------------------------ */
/* Selection (section 4.2, query Q3; section 3.2, query Q0).                 */
/* SELECT y FROM R WHERE lo <= y <= hi.  The branching loop of the paper's   */
/* selection-scan figure: a value is copied to the cursor and the cursor     */
/* advances only when the predicate holds.  Output is in input order.        */
/* Returns the count.                                                        */
/* ------------------------------------------------------------------------ */
int64_t oracle_select(const int32_t *y, int64_t n, int32_t lo, int32_t hi,
                      int32_t *out)
{
    int64_t count = 0;
    for (int64_t i = 0; i < n; ++i) {
        int32_t v = y[i];
        if (v >= lo && v <= hi) {
            if (out) out[count] = v;
            count += 1;
        }
    }
    return count;
}

/* ------------------------------------------------------------------------ */
/* Projection (section 4.1, query Q1): SELECT a*x1 + b*x2 FROM R.           */
/* Evaluated in double and rounded once to float.                            */
/* ------------------------------------------------------------------------ */
void oracle_project(const float *x1, const float *x2, int64_t n, double a,
                    double b, float *out)
{
    for (int64_t i = 0; i < n; ++i) {
        double v = a * (double)x1[i] + b * (double)x2[i];
        out[i] = (float)v;
    }
}

/* Projection with a user-defined function (section 4.1, query Q2):
 * SELECT sigmoid(a*x1 + b*x2) FROM R, sigmoid(x) = 1 / (1 + e^-x). */
void oracle_project_sigmoid(const float *x1, const float *x2, int64_t n,
                            double a, double b, float *out)
{
    for (int64_t i = 0; i < n; ++i) {
        double v = a * (double)x1[i] + b * (double)x2[i];
        out[i] = (float)(1.0 / (1.0 + exp(-v)));
    }
}

/* ------------------------------------------------------------------------ */
/* Key -> row index of a dimension table (the build side of a join).         */
/* Two plain structures, neither of them the GPU's linear-probing table:     */
/*  - a direct array over [min_key, max_key] when the keys are dense;        */
/*  - otherwise the rows sorted by key, searched by bisection.               */
/* A duplicate key makes the join ill-defined for a primary key and is       */
/* reported.                                                                  */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t n;
    int32_t min_key, max_key;
    int64_t *direct;    /* direct[k - min_key] = row or -1 (dense case) */
    int64_t *order;     /* row indices sorted by key (sparse case)      */
    const int32_t *key;
} key_index;

static int cmp_rows_by_key(const void *pa, const void *pb, void *keys)
{
    const int32_t *key = (const int32_t *)keys;
    int32_t ka = key[*(const int64_t *)pa];
    int32_t kb = key[*(const int64_t *)pb];
    return (ka > kb) - (ka < kb);
}

static void key_index_free(key_index *ix)
{
    free(ix->direct);
    free(ix->order);
    ix->direct = NULL;
    ix->order = NULL;
}

static int key_index_build(key_index *ix, const int32_t *key, int64_t n)
{
    memset(ix, 0, sizeof(*ix));
    ix->n = n;
    ix->key = key;
    if (n == 0) return ORACLE_OK;
    int32_t lo = key[0], hi = key[0];
    for (int64_t r = 1; r < n; ++r) {
        if (key[r] < lo) lo = key[r];
        if (key[r] > hi) hi = key[r];
    }
    ix->min_key = lo;
    ix->max_key = hi;
    int64_t span = (int64_t)hi - (int64_t)lo + 1;
    if (span <= 4 * n + 1024) {
        ix->direct = (int64_t *)malloc((size_t)span * sizeof(int64_t));
        if (!ix->direct) return ORACLE_EINVAL;
        for (int64_t s = 0; s < span; ++s) ix->direct[s] = -1;
        for (int64_t r = 0; r < n; ++r) {
            int64_t s = (int64_t)key[r] - lo;
            if (ix->direct[s] >= 0) { key_index_free(ix); return ORACLE_EDUPKEY; }
            ix->direct[s] = r;
        }
        return ORACLE_OK;
    }
    ix->order = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    if (!ix->order) return ORACLE_EINVAL;
    for (int64_t r = 0; r < n; ++r) ix->order[r] = r;
    qsort_r(ix->order, (size_t)n, sizeof(int64_t), cmp_rows_by_key, (void *)key);
    for (int64_t r = 1; r < n; ++r)
        if (key[ix->order[r]] == key[ix->order[r - 1]]) {
            key_index_free(ix);
            return ORACLE_EDUPKEY;
        }
    return ORACLE_OK;
}

/* Row of the dimension whose key equals k, or -1 when there is none. */
static int64_t key_index_find(const key_index *ix, int32_t k)
{
    if (ix->n == 0 || k < ix->min_key || k > ix->max_key) return -1;
    if (ix->direct) return ix->direct[(int64_t)k - ix->min_key];
    int64_t a = 0, b = ix->n - 1;
    while (a <= b) {
        int64_t m = a + (b - a) / 2;
        int32_t km = ix->key[ix->order[m]];
        if (km == k) return ix->order[m];
        if (km < k) a = m + 1; else b = m - 1;
    }
    return -1;
}

/* ------------------------------------------------------------------------ */
/* Hash join with sum (section 4.3, query Q4):                               */
/*   SELECT SUM(A.v + B.v) FROM A, B WHERE A.k = B.k                         */
/* A is the build side (dimension rows), optionally restricted to the rows   */
/* whose filter attribute lies in [flo, fhi]; B is the probe side.  The sum  */
/* adds the build payload of every matching probe row, plus the probe        */
/* payload when one is given; a build side without payload contributes 0.    */
/* *matches counts the probe rows that found a partner.                      */
/* ------------------------------------------------------------------------ */
int oracle_join_sum(const int32_t *bkey, const int32_t *bval,
                    const int32_t *bfilter, int32_t flo, int32_t fhi,
                    int64_t nb, const int32_t *pkey, const int32_t *pval,
                    int64_t np, int64_t *sum, int64_t *matches)
{
    if (nb < 0 || np < 0 || (nb > 0 && !bkey) || (np > 0 && !pkey))
        return ORACLE_EINVAL;
    key_index ix;
    int rc = key_index_build(&ix, bkey, nb);
    if (rc) return rc;
    uint64_t s = 0;
    int64_t m = 0;
    for (int64_t i = 0; i < np; ++i) {
        int64_t r = key_index_find(&ix, pkey[i]);
        if (r < 0) continue;
        if (bfilter && (bfilter[r] < flo || bfilter[r] > fhi)) continue;
        if (bval) s += (uint64_t)(int64_t)bval[r];
        if (pval) s += (uint64_t)(int64_t)pval[i];
        m += 1;
    }
    key_index_free(&ix);
    *sum = (int64_t)s;
    *matches = m;
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------ */
/* Dense group-by aggregate: sums[g[i]] += v[i] over int64.                  */
/* The global aggregation table of the section 5.3 case study, in the dense  */
/* form its small group keys allow.                                          */
/* ------------------------------------------------------------------------ */
int oracle_groupby(const int32_t *g, const int32_t *v, int64_t n,
                   int64_t n_groups, int64_t *sums)
{
    if (n < 0 || n_groups <= 0) return ORACLE_EINVAL;
    uint64_t *acc = (uint64_t *)calloc((size_t)n_groups, sizeof(uint64_t));
    if (!acc) return ORACLE_EINVAL;
    int rc = ORACLE_OK;
    for (int64_t i = 0; i < n; ++i) {
        if (g[i] < 0 || (int64_t)g[i] >= n_groups) { rc = ORACLE_ERANGE; continue; }
        acc[g[i]] += (uint64_t)(int64_t)v[i];
    }
    for (int64_t k = 0; k < n_groups; ++k) sums[k] = (int64_t)acc[k];
    free(acc);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Star query (section 3.1, SSB Q1.1; section 5.3, SSB Q2.1):                */
/*   SELECT agg(...) FROM fact, dim_1 ... dim_J                              */
/*   WHERE fact.fk_j = dim_j.key  (j = 1..J)                                 */
/*     AND lo_p <= fact.col_p <= hi_p          (fact predicates)            */
/*     AND flo_j <= dim_j.filter <= fhi_j       (dimension predicates)       */
/*   GROUP BY dense index  sum_j (dim_j.group - base_j) * stride_j           */
/* For each fact row: test the fact predicates, find each dimension row by   */
/* key (dropping the fact row when there is none or its predicate fails),    */
/* form the group index from the dimension attributes, add the aggregate.   */
/* agg: 0 SUM(c0), 1 SUM(c0*c1), 2 SUM(c0-c1), 3 COUNT(*).                   */
/* ------------------------------------------------------------------------ */
#define ORACLE_MAX_JOINS 8

typedef struct {
    int64_t n_rows;
    int32_t n_cols;
    const int32_t *const *cols;
    int32_t n_preds;
    const int32_t *pred_col;
    const int32_t *pred_lo;
    const int32_t *pred_hi;
    int32_t n_joins;
    const int32_t *join_fk_col;
    const int32_t *const *dim_key;
    const int64_t *dim_rows;
    const int32_t *const *dim_filter; /* entries may be NULL */
    const int32_t *dim_flo;
    const int32_t *dim_fhi;
    const int32_t *const *dim_group;  /* entries may be NULL */
    const int64_t *group_base;
    const int64_t *group_stride;
    int32_t agg_kind;
    int32_t agg_col0;
    int32_t agg_col1;
    int64_t n_groups;
} oracle_star_plan;

int oracle_star(const oracle_star_plan *p, int64_t *out, int64_t *survivors)
{
    if (!p || p->n_rows < 0 || p->n_groups <= 0 || p->n_joins < 0 ||
        p->n_joins > ORACLE_MAX_JOINS || p->agg_kind < 0 || p->agg_kind > 3)
        return ORACLE_EINVAL;
    for (int32_t q = 0; q < p->n_preds; ++q)
        if (p->pred_col[q] < 0 || p->pred_col[q] >= p->n_cols) return ORACLE_EINVAL;
    for (int32_t j = 0; j < p->n_joins; ++j)
        if (p->join_fk_col[j] < 0 || p->join_fk_col[j] >= p->n_cols) return ORACLE_EINVAL;
    if (p->agg_kind != 3 && (p->agg_col0 < 0 || p->agg_col0 >= p->n_cols)) return ORACLE_EINVAL;
    if ((p->agg_kind == 1 || p->agg_kind == 2) && (p->agg_col1 < 0 || p->agg_col1 >= p->n_cols))
        return ORACLE_EINVAL;

    key_index ix[ORACLE_MAX_JOINS];
    for (int32_t j = 0; j < p->n_joins; ++j) {
        int rc = key_index_build(&ix[j], p->dim_key[j], p->dim_rows[j]);
        if (rc) {
            for (int32_t k = 0; k < j; ++k) key_index_free(&ix[k]);
            return rc;
        }
    }
    uint64_t *acc = (uint64_t *)calloc((size_t)p->n_groups, sizeof(uint64_t));
    if (!acc) return ORACLE_EINVAL;
    int rc = ORACLE_OK;
    int64_t kept = 0;
    for (int64_t i = 0; i < p->n_rows; ++i) {
        int pass = 1;
        for (int32_t q = 0; q < p->n_preds && pass; ++q) {
            int32_t v = p->cols[p->pred_col[q]][i];
            if (v < p->pred_lo[q] || v > p->pred_hi[q]) pass = 0;
        }
        int64_t group = 0;
        for (int32_t j = 0; j < p->n_joins && pass; ++j) {
            int64_t r = key_index_find(&ix[j], p->cols[p->join_fk_col[j]][i]);
            if (r < 0) { pass = 0; break; }
            if (p->dim_filter[j]) {
                int32_t f = p->dim_filter[j][r];
                if (f < p->dim_flo[j] || f > p->dim_fhi[j]) { pass = 0; break; }
            }
            if (p->dim_group[j])
                group += ((int64_t)p->dim_group[j][r] - p->group_base[j]) * p->group_stride[j];
        }
        if (!pass) continue;
        if (group < 0 || group >= p->n_groups) { rc = ORACLE_ERANGE; continue; }
        uint64_t val;
        switch (p->agg_kind) {
        case 0: val = (uint64_t)(int64_t)p->cols[p->agg_col0][i]; break;
        case 1: val = (uint64_t)((int64_t)p->cols[p->agg_col0][i] *
                                 (int64_t)p->cols[p->agg_col1][i]); break;
        case 2: val = (uint64_t)((int64_t)p->cols[p->agg_col0][i] -
                                 (int64_t)p->cols[p->agg_col1][i]); break;
        default: val = 1; break;
        }
        acc[group] += val;
        kept += 1;
    }
    for (int64_t g = 0; g < p->n_groups; ++g) out[g] = (int64_t)acc[g];
    if (survivors) *survivors = kept;
    free(acc);
    for (int32_t j = 0; j < p->n_joins; ++j) key_index_free(&ix[j]);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Radix partitioning (section 4.4): with radix r and start bit a, the digit */
/* of key e is bits a .. a+r-1 of e (unsigned); a partition pass places the */
/* elements into 2^r contiguous partitions by digit.  The histogram counts   */
/* each digit; the partition is stable (within a partition, input order).   */
/* ------------------------------------------------------------------------ */
static uint32_t digit_of(uint32_t key, int32_t shift, int32_t bits)
{
    return (key >> shift) & ((1u << bits) - 1u);
}

int oracle_radix_histogram(const uint32_t *keys, int64_t n, int32_t shift, int32_t bits, int64_t *hist)
{
    if (n < 0 || bits < 1 || bits > 16 || shift < 0 || shift + bits > 32) return ORACLE_EINVAL;
    for (int64_t d = 0; d < ((int64_t)1 << bits); ++d) hist[d] = 0;
    for (int64_t i = 0; i < n; ++i) hist[digit_of(keys[i], shift, bits)] += 1;
    return ORACLE_OK;
}

int oracle_radix_partition(const uint32_t *keys, const uint32_t *vals, int64_t n, int32_t shift, int32_t bits,
                           uint32_t *out_keys, uint32_t *out_vals)
{
    if (n < 0 || bits < 1 || bits > 16 || shift < 0 || shift + bits > 32) return ORACLE_EINVAL;
    const int64_t nd = (int64_t)1 << bits;
    int64_t *next = (int64_t *)calloc((size_t)nd, sizeof(int64_t));
    if (!next) return ORACLE_EINVAL;
    /* counting sort: count, exclusive prefix, then place in input order */
    for (int64_t i = 0; i < n; ++i) next[digit_of(keys[i], shift, bits)] += 1;
    int64_t run = 0;
    for (int64_t d = 0; d < nd; ++d) {
        int64_t c = next[d];
        next[d] = run;
        run += c;
    }
    for (int64_t i = 0; i < n; ++i) {
        int64_t pos = next[digit_of(keys[i], shift, bits)]++;
        out_keys[pos] = keys[i];
        if (vals) out_vals[pos] = vals[i];
    }
    free(next);
    return ORACLE_OK;
}

/* Sort of 32-bit (key, value) pairs by unsigned key, stable (section 4.4,
 * the sort the radix passes build up to). */
static int cmp_pairs(const void *pa, const void *pb, void *keys)
{
    const uint32_t *ukey = (const uint32_t *)keys;
    int64_t a = *(const int64_t *)pa, b = *(const int64_t *)pb;
    uint32_t ka = ukey[a], kb = ukey[b];
    if (ka != kb) return ka < kb ? -1 : 1;
    return (a > b) - (a < b); /* equal keys keep input order */
}

int oracle_sort_pairs(const uint32_t *keys, const uint32_t *vals, int64_t n, uint32_t *out_keys,
                      uint32_t *out_vals)
{
    if (n < 0) return ORACLE_EINVAL;
    int64_t *idx = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    if (!idx) return ORACLE_EINVAL;
    for (int64_t i = 0; i < n; ++i) idx[i] = i;
    qsort_r(idx, (size_t)n, sizeof(int64_t), cmp_pairs, (void *)keys);
    for (int64_t i = 0; i < n; ++i) {
        out_keys[i] = keys[idx[i]];
        if (vals) out_vals[i] = vals[idx[i]];
    }
    free(idx);
    return ORACLE_OK;
}
