// C ABI entry points: argument validation, plan translation, tuning table.
// Every compute step runs in the kernels of scan_ops.hip, hash_ops.hip and
// star.hip; this file only checks arguments and launches them.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "block.hpp"
#include "internal.hpp"
#include "variants.hpp"

namespace crystal {

// ------------------------------------------------------------ device info --
static int g_cu[64];
static int64_t g_lds[64];

static int cur_device() {
    int d = 0;
    if (hipGetDevice(&d) != hipSuccess || d < 0 || d >= 64) d = 0;
    return d;
}

int device_cu_count() {
    const int d = cur_device();
    if (!g_cu[d]) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, d) != hipSuccess || v <= 0)
            v = 256;
        g_cu[d] = v;
    }
    return g_cu[d];
}

int64_t device_lds_per_cu() {
    static int64_t cache[64];
    const int d = cur_device();
    if (!cache[d]) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, d) != hipSuccess ||
            v <= 0)
            v = 65536;
        cache[d] = v;
    }
    return cache[d];
}

hipError_t resident_per_cu(const void *fn, int block, int64_t lds_bytes, int64_t &out) {
    static std::mutex mu;
    static std::map<std::tuple<int, const void *, int, int64_t>, int64_t> cache;
    const auto key = std::make_tuple(cur_device(), fn, block, lds_bytes);
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(key);
    if (it == cache.end()) {
        int n = 0;
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fn, block, (size_t)lds_bytes);
        if (e != hipSuccess) return e;
        it = cache.emplace(key, (int64_t)n).first;
    }
    out = it->second;
    return hipSuccess;
}

int64_t device_lds_per_block() {
    const int d = cur_device();
    if (!g_lds[d]) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, d) != hipSuccess || v <= 0)
            v = 65536;
        g_lds[d] = v;
    }
    return g_lds[d];
}

// ----------------------------------------------------------------- tuning --
struct TuneEntry {
    int kernel, blo, bhi;
    LaunchCfg cfg;
};

static std::mutex g_tune_mu;
static std::vector<TuneEntry> g_tune;

static LaunchCfg default_cfg(int kernel) {
    switch (kernel) {
    case CRYSTAL_K_SELECT: return {1024, 16, 0};
    case CRYSTAL_K_PROJECT: return {256, 16, 0};
    case CRYSTAL_K_HT_PROBE: return {256, 16, 8};
    case CRYSTAL_K_GROUPBY: return {256, 16, 0};
    case CRYSTAL_K_STAR: return {256, 16, 0};
    case CRYSTAL_K_SHARED_SCAN: return {1024, 16, 0};
    case CRYSTAL_K_SHARED_SCAN_SCALAR: return {1024, 8, 0};
    case CRYSTAL_K_RADIX: return {1024, 16, 0};
    default: return {256, 16, 0};
    }
}

static int size_bucket(int64_t n) {
    int b = 0;
    while (b < 62 && (int64_t(1) << (b + 1)) <= n) ++b;
    return b;
}

LaunchCfg tune_lookup(int kernel, int64_t n) {
    const int b = size_bucket(n);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (auto it = g_tune.rbegin(); it != g_tune.rend(); ++it)
        if (it->kernel == kernel && b >= it->blo && b <= it->bhi) return it->cfg;
    return default_cfg(kernel);
}

static bool variant_exists(int kernel, int block, int ipt) {
    const int key = CRYSTAL_VARIANT_KEY(block, ipt);
    if (kernel == CRYSTAL_K_RADIX) {
        switch (key) {
#define X(B, I) case CRYSTAL_VARIANT_KEY(B, I): return true;
            CRYSTAL_VARIANTS_RADIX(X)
#undef X
        default: return false;
        }
    }
    if (kernel == CRYSTAL_K_SELECT) {
        switch (key) {
#define X(B, I) case CRYSTAL_VARIANT_KEY(B, I): return true;
            CRYSTAL_VARIANTS_ALL(X)
#undef X
        default: return false;
        }
    }
    switch (key) {
#define X(B, I) case CRYSTAL_VARIANT_KEY(B, I): return true;
        CRYSTAL_VARIANTS_VEC(X)
#undef X
    default: return false;
    }
}

static hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

// ------------------------------------------------------- plan translation --
static uint32_t field_mask(int bits) { return bits >= 32 ? 0xffffffffu : ((1u << bits) - 1u); }

static bool ht_valid(const crystal_ht &ht) {
    if (!ht.mem || !aligned16(ht.mem) || ht.capacity <= 0) return false;
    if (ht.kind == CRYSTAL_HT_LINEAR)
        return ht.log2_capacity >= 6 && ht.log2_capacity <= 31 &&
               ht.capacity == (int64_t(1) << ht.log2_capacity);
    if (ht.kind == CRYSTAL_HT_DIRECT) return ht.capacity <= (int64_t(1) << 32);
    return false;
}

static int64_t bitmap_words(int64_t span) { return ((span + 31) / 32 + 63) / 64 * 64; }

crystal_status star_plan_to_dev(const crystal_star_query &q, StarPlanDev &d) {
    memset(&d, 0, sizeof(d));
    if (q.n_rows < 0 || q.n_cols < 0 || q.n_cols > CRYSTAL_MAX_COLS || q.n_preds < 0 ||
        q.n_preds > CRYSTAL_MAX_PREDS || q.n_joins < 0 || q.n_joins > CRYSTAL_MAX_JOINS ||
        q.n_groups < 1 || q.n_groups > INT32_MAX || q.agg < 0 || q.agg > CRYSTAL_AGG_COUNT)
        return CRYSTAL_EINVAL;
    // a plan over zero rows may carry null column pointers (nothing is read)
    auto col_ok = [&](int c) {
        return c >= 0 && c < q.n_cols && (q.n_rows == 0 || (q.cols[c] && aligned16(q.cols[c])));
    };
    for (int c = 0; c < q.n_cols; ++c) {
        if (q.cols[c] && !aligned16(q.cols[c])) return CRYSTAL_EINVAL;
        d.col[c].p = q.cols[c];
        const int32_t w = q.formats[c].width, nb = q.formats[c].bits;
        if (w != 0 && w != 1 && w != 2 && w != 4) return CRYSTAL_EINVAL;
        if (nb < 0 || nb > 16 || (nb > 0 && w != 0)) return CRYSTAL_EINVAL;
        d.col[c].width = nb > 0 ? 0 : w == 0 ? 4 : w;
        d.col[c].bits = nb;
        d.col[c].base = nb > 0 || w == 1 || w == 2 ? q.formats[c].base : 0;
    }
    for (int c = q.n_cols; c < CRYSTAL_MAX_COLS; ++c) d.col[c].width = 4;
    d.n_rows = q.n_rows;
    d.n_groups = q.n_groups;
    d.n_preds = q.n_preds;
    d.n_joins = q.n_joins;
    for (int i = 0; i < q.n_preds; ++i) {
        if (!col_ok(q.preds[i].col)) return CRYSTAL_EINVAL;
        d.pred_col[i] = q.preds[i].col;
        d.pred_lo[i] = q.preds[i].range.lo;
        d.pred_hi[i] = q.preds[i].range.hi;
    }
    d.agg = q.agg;
    d.agg_col0 = q.agg_col0;
    d.agg_col1 = q.agg_col1;
    if (q.agg != CRYSTAL_AGG_COUNT && !col_ok(q.agg_col0)) return CRYSTAL_EINVAL;
    if ((q.agg == CRYSTAL_AGG_SUM_PRODUCT || q.agg == CRYSTAL_AGG_SUM_DIFF) && !col_ok(q.agg_col1))
        return CRYSTAL_EINVAL;
    bool any_group = false;
    for (int i = 0; i < q.n_joins; ++i) {
        const crystal_join &j = q.joins[i];
        StarJoinDev &o = d.joins[i];
        if (!ht_valid(j.ht) || !col_ok(j.fk_col)) return CRYSTAL_EINVAL;
        if (j.filter_bits < 0 || j.filter_bits > 32 || j.group_bits < 0 || j.group_bits > 32)
            return CRYSTAL_EINVAL;
        if (j.filter_shift < 0 || j.filter_shift > 31 || j.group_shift < 0 || j.group_shift > 31)
            return CRYSTAL_EINVAL;
        if ((j.filter_bits > 0 || j.group_bits > 0) && !j.ht.has_payload) return CRYSTAL_EINVAL;
        o.kind = j.ht.kind;
        o.has_payload = j.ht.has_payload;
        if (j.ht.kind == CRYSTAL_HT_DIRECT) {
            o.bitmap = (const uint32_t *)j.ht.mem;
            o.payload = j.ht.has_payload ? (const int32_t *)j.ht.mem + bitmap_words(j.ht.capacity) : nullptr;
            o.span = j.ht.capacity;
            o.key_min = j.ht.key_min;
        } else {
            o.slots = j.ht.mem;
            o.mask = (uint32_t)(j.ht.capacity - 1);
            o.shift = 32 - j.ht.log2_capacity;
        }
        o.fk_col = j.fk_col;
        o.f_bits = j.filter_bits;
        o.f_shift = j.filter_shift;
        o.f_mask = field_mask(j.filter_bits);
        o.f_lo = j.filter.lo;
        o.f_hi = j.filter.hi;
        o.g_bits = j.group_bits;
        o.g_shift = j.group_shift;
        o.g_mask = field_mask(j.group_bits);
        o.g_base = j.group_base;
        o.g_stride = j.group_stride;
        if (j.group_bits > 0) any_group = true;
    }
    d.scalar = (q.n_groups == 1 && !any_group) ? 1 : 0;
    return CRYSTAL_OK;
}

}  // namespace crystal

using namespace crystal;

extern "C" {

const char *crystal_status_string(int32_t s) {
    switch (s) {
    case CRYSTAL_OK: return "ok";
    case CRYSTAL_EINVAL: return "invalid argument";
    case CRYSTAL_ESCRATCH: return "scratch or slot memory too small";
    case CRYSTAL_EFULL: return "hash table full";
    case CRYSTAL_EDUPKEY: return "duplicate build key";
    case CRYSTAL_EHIP: return "HIP runtime error";
    case CRYSTAL_EBUSY: return "no free slot";
    case CRYSTAL_ERANGE: return "key or group index out of range";
    case CRYSTAL_ETIMEDOUT: return "query dropped at its deadline";
    default: return "unknown status";
    }
}

int32_t crystal_abi_version(void) { return CRYSTAL_ABI_VERSION; }

size_t crystal_struct_size(int32_t which) {
    switch (which) {
    case 0: return sizeof(crystal_range);
    case 1: return sizeof(crystal_ht);
    case 2: return sizeof(crystal_pred);
    case 3: return sizeof(crystal_join);
    case 4: return sizeof(crystal_star_query);
    case 5: return sizeof(crystal_qmask_table);
    case 6: return sizeof(crystal_batch_query);
    case 7: return sizeof(crystal_batch);
    case 8: return sizeof(crystal_server_template);
    case 9: return sizeof(crystal_server_config);
    case 10: return sizeof(crystal_server_stats);
    case 11: return sizeof(crystal_ht_build_item);
    case 12: return sizeof(crystal_col_format);
    case 13: return sizeof(crystal_qmask_build_item);
    default: return 0;
    }
}

crystal_status crystal_select(const int32_t *in, int64_t n, crystal_range pred, int32_t *out,
                              int64_t *out_count, void *stream) {
    if (n < 0 || !out_count || (n > 0 && (!in || !out || !aligned16(in)))) return CRYSTAL_EINVAL;
    return from_hip(launch_select(tune_lookup(CRYSTAL_K_SELECT, n), in, n, pred.lo, pred.hi, out, out_count,
                                  nullptr, false, as_stream(stream)));
}

size_t crystal_select_stable_scratch_bytes(int64_t n) {
    if (n <= 0) return 16;
    const int64_t items = select_tile_items(tune_lookup(CRYSTAL_K_SELECT, n));
    return (size_t)((n + items - 1) / items) * 8 + 16;
}

crystal_status crystal_select_stable(const int32_t *in, int64_t n, crystal_range pred, int32_t *out,
                                     int64_t *out_count, void *scratch, size_t scratch_bytes, void *stream) {
    if (n < 0 || !out_count || (n > 0 && (!in || !out || !aligned16(in)))) return CRYSTAL_EINVAL;
    if (n > 0 && pred.lo <= pred.hi) {
        if (!scratch || !aligned16(scratch)) return scratch ? CRYSTAL_EINVAL : CRYSTAL_ESCRATCH;
        if (scratch_bytes < crystal_select_stable_scratch_bytes(n)) return CRYSTAL_ESCRATCH;
    }
    return from_hip(launch_select(tune_lookup(CRYSTAL_K_SELECT, n), in, n, pred.lo, pred.hi, out, out_count,
                                  (uint64_t *)scratch, true, as_stream(stream)));
}

static crystal_status project_common(const float *x1, const float *x2, int64_t n, float a, float b,
                                     float *out, void *stream, bool sigmoid) {
    if (n < 0 || (n > 0 && (!x1 || !x2 || !out || !aligned16(x1) || !aligned16(x2) || !aligned16(out))))
        return CRYSTAL_EINVAL;
    if (n == 0) return CRYSTAL_OK;
    return from_hip(launch_project(tune_lookup(CRYSTAL_K_PROJECT, n), x1, x2, n, a, b, out, sigmoid,
                                   as_stream(stream)));
}

crystal_status crystal_project(const float *x1, const float *x2, int64_t n, float a, float b,
                               float *out, void *stream) {
    return project_common(x1, x2, n, a, b, out, stream, false);
}

crystal_status crystal_project_sigmoid(const float *x1, const float *x2, int64_t n, float a, float b,
                                       float *out, void *stream) {
    return project_common(x1, x2, n, a, b, out, stream, true);
}

crystal_status crystal_ht_init(crystal_ht *ht, int32_t kind, int64_t n_keys, int32_t key_min,
                               int32_t key_max, int32_t has_payload) {
    if (!ht || n_keys < 0) return CRYSTAL_EINVAL;
    memset(ht, 0, sizeof(*ht));
    ht->kind = kind;
    ht->has_payload = has_payload ? 1 : 0;
    if (kind == CRYSTAL_HT_LINEAR) {
        int l = 6;
        while ((int64_t(1) << l) < 2 * n_keys) ++l;
        if (l > 31) return CRYSTAL_EINVAL;
        ht->log2_capacity = l;
        ht->capacity = int64_t(1) << l;
        return CRYSTAL_OK;
    }
    if (kind == CRYSTAL_HT_DIRECT) {
        if (key_max < key_min) return CRYSTAL_EINVAL;
        ht->key_min = key_min;
        ht->capacity = (int64_t)key_max - (int64_t)key_min + 1;
        return CRYSTAL_OK;
    }
    return CRYSTAL_EINVAL;
}

size_t crystal_ht_bytes(const crystal_ht *ht) {
    if (!ht || ht->capacity <= 0) return 0;
    if (ht->kind == CRYSTAL_HT_LINEAR) return (size_t)ht->capacity * 8;
    if (ht->kind == CRYSTAL_HT_DIRECT)
        return (size_t)bitmap_words(ht->capacity) * 4 + (ht->has_payload ? (size_t)ht->capacity * 4 : 0);
    return 0;
}

crystal_status crystal_ht_build(const crystal_ht *ht, const int32_t *keys, const int32_t *payload,
                                const int32_t *filter_col, crystal_range filter, int64_t n,
                                int32_t *status, void *stream) {
    if (!ht || !ht_valid(*ht) || n < 0 || !status || (n > 0 && !keys) ||
        (ht->has_payload && n > 0 && !payload))
        return CRYSTAL_EINVAL;
    return from_hip(launch_ht_build(*ht, keys, ht->has_payload ? payload : nullptr, filter_col,
                                    filter.lo, filter.hi, n, status, as_stream(stream)));
}

crystal_status crystal_ht_build_batch(const crystal_ht_build_item *items, int32_t n_items, int32_t *status,
                                      void *stream) {
    if (!items || !status || n_items < 0 || n_items > CRYSTAL_MAX_BUILD_BATCH) return CRYSTAL_EINVAL;
    for (int i = 0; i < n_items; ++i) {
        const crystal_ht_build_item &it = items[i];
        if (!it.ht || !ht_valid(*it.ht) || it.n < 0 || (it.n > 0 && !it.keys) ||
            (it.ht->has_payload && it.n > 0 && !it.payload))
            return CRYSTAL_EINVAL;
        for (int j = 0; j < i; ++j)
            if (items[j].ht->mem == it.ht->mem) return CRYSTAL_EINVAL;
    }
    if (n_items == 0) return CRYSTAL_OK;
    return from_hip(launch_ht_build_batch(items, n_items, status, as_stream(stream)));
}

crystal_status crystal_ht_build_batch_fused(const crystal_ht_build_item *items, int32_t n_items,
                                            const crystal_ht *const *clear, int32_t n_clear, int64_t *zero,
                                            int64_t zero_n, int32_t *status, void *stream) {
    if (!status || n_items < 0 || n_items > CRYSTAL_MAX_BUILD_BATCH || n_clear < 0 ||
        n_clear > CRYSTAL_MAX_BUILD_BATCH || (n_items > 0 && !items) || (n_clear > 0 && !clear) || zero_n < 0 ||
        (zero_n > 0 && (!zero || ((uintptr_t)zero & 7u))))
        return CRYSTAL_EINVAL;
    // every memory range the launch writes: the items' tables, the cleared tables, the zeroed words
    struct Span {
        uintptr_t lo, hi;
    };
    Span spans[2 * CRYSTAL_MAX_BUILD_BATCH + 1];
    int n_spans = 0;
    for (int i = 0; i < n_items; ++i) {
        const crystal_ht_build_item &it = items[i];
        if (!it.ht || !ht_valid(*it.ht) || it.n < 0 || (it.n > 0 && !it.keys) ||
            (it.ht->has_payload && it.n > 0 && !it.payload))
            return CRYSTAL_EINVAL;
        spans[n_spans++] = {(uintptr_t)it.ht->mem, (uintptr_t)it.ht->mem + crystal_ht_bytes(it.ht)};
    }
    for (int i = 0; i < n_clear; ++i) {
        if (!clear[i] || !ht_valid(*clear[i])) return CRYSTAL_EINVAL;
        spans[n_spans++] = {(uintptr_t)clear[i]->mem, (uintptr_t)clear[i]->mem + crystal_ht_bytes(clear[i])};
    }
    if (zero_n > 0) spans[n_spans++] = {(uintptr_t)zero, (uintptr_t)zero + (uintptr_t)zero_n * 8};
    for (int i = 0; i < n_spans; ++i)
        for (int j = 0; j < i; ++j)
            if (spans[i].lo < spans[j].hi && spans[j].lo < spans[i].hi) return CRYSTAL_EINVAL;
    return from_hip(launch_ht_build_batch_fused(items, n_items, clear, n_clear, zero, zero_n, status,
                                                as_stream(stream)));
}

crystal_status crystal_ht_probe(const crystal_ht *ht, const int32_t *fk, const int32_t *probe_payload,
                                int64_t n, int64_t *out_sum, int64_t *out_matches, void *stream) {
    if (!ht || !ht_valid(*ht) || n < 0 || !out_sum || !out_matches || (n > 0 && (!fk || !aligned16(fk))) ||
        (probe_payload && !aligned16(probe_payload)))
        return CRYSTAL_EINVAL;
    return from_hip(launch_ht_probe(tune_lookup(CRYSTAL_K_HT_PROBE, n), *ht, fk, probe_payload, n,
                                    (uint64_t *)out_sum, (uint64_t *)out_matches, as_stream(stream)));
}

crystal_status crystal_groupby_agg(const int32_t *group, const int32_t *value, int64_t n,
                                   int64_t n_groups, int64_t *sums, int32_t *status, void *stream) {
    if (n < 0 || n_groups < 1 || !sums || !status ||
        (n > 0 && (!group || !value || !aligned16(group) || !aligned16(value))))
        return CRYSTAL_EINVAL;
    return from_hip(launch_groupby(tune_lookup(CRYSTAL_K_GROUPBY, n), group, value, n, n_groups,
                                   (uint64_t *)sums, status, as_stream(stream)));
}

size_t crystal_star_query_scratch_bytes(const crystal_star_query *q) {
    if (!q) return 0;
    StarPlanDev d;
    if (star_plan_to_dev(*q, d) != CRYSTAL_OK || !d.scalar) return 0;
    return (size_t)star_max_grid(q->n_rows) * 8;
}

static crystal_status run_star(const crystal_star_query *q, int64_t *out, int32_t *status, void *scratch,
                               size_t scratch_bytes, void *stream, bool accumulate) {
    if (!q || !out || !status) return CRYSTAL_EINVAL;
    StarPlanDev d;
    crystal_status st = star_plan_to_dev(*q, d);
    if (st != CRYSTAL_OK) return st;
    if (d.scalar) {
        if (!scratch || !aligned16(scratch)) return scratch ? CRYSTAL_EINVAL : CRYSTAL_ESCRATCH;
        if (scratch_bytes < (size_t)star_max_grid(q->n_rows) * 8) return CRYSTAL_ESCRATCH;
    }
    return from_hip(launch_star(tune_lookup(CRYSTAL_K_STAR, q->n_rows), d, (uint64_t *)out, status,
                                (uint64_t *)scratch, accumulate, as_stream(stream)));
}

crystal_status crystal_run_star_query(const crystal_star_query *q, int64_t *out, int32_t *status,
                                      void *scratch, size_t scratch_bytes, void *stream) {
    return run_star(q, out, status, scratch, scratch_bytes, stream, false);
}

crystal_status crystal_run_star_query_accumulate(const crystal_star_query *q, int64_t *out, int32_t *status,
                                                 void *scratch, size_t scratch_bytes, void *stream) {
    return run_star(q, out, status, scratch, scratch_bytes, stream, true);
}

crystal_status crystal_run_star_query_noalloc(const crystal_star_query *q, int64_t *out, int32_t *status,
                                              void *stream) {
    if (!q || !out || !status) return CRYSTAL_EINVAL;
    StarPlanDev d;
    crystal_status st = star_plan_to_dev(*q, d);
    if (st != CRYSTAL_OK) return st;
    uint64_t *partials = nullptr;
    if (d.scalar) {
        if (star_max_grid(q->n_rows) > kStarNoallocPartials) return CRYSTAL_ESCRATCH;
        const hipError_t e = star_noalloc_partials(&partials);
        if (e != hipSuccess) return from_hip(e);
    }
    return from_hip(launch_star(tune_lookup(CRYSTAL_K_STAR, q->n_rows), d, (uint64_t *)out, status, partials,
                                false, as_stream(stream)));
}

size_t crystal_packed_column_bytes(int64_t n, int32_t bits) {
    if (n < 0 || bits < 1 || bits > 16) return 0;
    return (size_t)(((n * bits + 31) / 32 + 4) * 4);
}

crystal_status crystal_pack_column_bits(const int32_t *in, int64_t n, int32_t base, int32_t bits, void *out,
                                        int32_t *status, void *stream) {
    if (n < 0 || bits < 1 || bits > 16 || !status || !out || !aligned16(out) || (n > 0 && (!in || !aligned16(in))))
        return CRYSTAL_EINVAL;
    const int64_t words = (int64_t)crystal_packed_column_bytes(n, bits) / 4;
    return from_hip(launch_pack_column_bits(in, n, base, bits, (uint32_t *)out, words, status, as_stream(stream)));
}

crystal_status crystal_pack_column(const int32_t *in, int64_t n, int32_t base, int32_t width, void *out,
                                   int32_t *status, void *stream) {
    if (n < 0 || (width != 1 && width != 2) || !status || (n > 0 && (!in || !out || !aligned16(in) || !aligned16(out))))
        return CRYSTAL_EINVAL;
    if (n == 0) return CRYSTAL_OK;
    return from_hip(launch_pack_column(in, n, base, width, out, status, as_stream(stream)));
}

// ------------------------------------------------------------ shared scan --
size_t crystal_qmask_bytes(int64_t span) {
    if (span <= 0) return 0;
    return (size_t)((span + 1) / 2) * 4;
}

static constexpr int64_t kMaxRankedSpan = int64_t(1) << 26;

size_t crystal_qmask_ranked_bytes(int64_t span, int32_t ranked) {
    if (ranked <= 0 || span <= 0 || span > kMaxRankedSpan) return 0;
    return (size_t)((qmask_ranked_words(span, ranked) * 4 + 15) / 16 * 16);
}

// A table descriptor the kernels can use: plain, or ranked with a span the
// directory scan handles.
static bool qmask_table_ok(const crystal_qmask_table *t) {
    if (!t || !t->mem || !aligned16(t->mem) || t->span <= 0 || t->span > (int64_t(1) << 32) || t->ranked < 0)
        return false;
    return t->ranked == 0 || t->span <= kMaxRankedSpan;
}

crystal_status crystal_qmask_rank(const crystal_qmask_table *t, const int32_t *keys, int64_t n, int32_t *status,
                                  void *stream) {
    if (!qmask_table_ok(t) || t->ranked == 0 || n < 0 || (n > 0 && !keys) || !status) return CRYSTAL_EINVAL;
    return from_hip(launch_qmask_rank((uint32_t *)t->mem, t->span, t->key_min, t->ranked, keys, n, status,
                                      as_stream(stream)));
}

crystal_status crystal_qmask_build(const crystal_qmask_table *t, const int32_t *keys, const int32_t *filter_col,
                                   int64_t n, const crystal_range *ranges, int32_t n_queries, int32_t *status,
                                   void *stream) {
    if (!qmask_table_ok(t) || n < 0 || (n > 0 && !keys) || n_queries < 0 || n_queries > CRYSTAL_MAX_BATCH ||
        (n_queries > 0 && !ranges) || !status)
        return CRYSTAL_EINVAL;
    QmaskRanges r = {};
    r.n = n_queries;
    for (int q = 0; q < n_queries; ++q) {
        r.lo[q] = ranges[q].lo;
        r.hi[q] = ranges[q].hi;
    }
    return from_hip(launch_qmask_build((uint16_t *)t->mem, t->span, t->key_min, t->ranked, keys, filter_col, n, r,
                                       status, as_stream(stream)));
}

crystal_status crystal_qmask_build_batch(const crystal_qmask_build_item *items, int32_t n_items, int32_t *status,
                                         void *stream) {
    if (!items || !status || n_items < 0 || n_items > CRYSTAL_MAX_JOINS) return CRYSTAL_EINVAL;
    QmaskItem it[CRYSTAL_MAX_JOINS];
    for (int i = 0; i < n_items; ++i) {
        const crystal_qmask_build_item &x = items[i];
        if (!qmask_table_ok(x.t) || x.n < 0 || (x.n > 0 && !x.keys) || x.n_queries < 0 ||
            x.n_queries > CRYSTAL_MAX_BATCH || (x.n_queries > 0 && !x.ranges))
            return CRYSTAL_EINVAL;
        for (int j = 0; j < i; ++j)
            if (items[j].t->mem == x.t->mem) return CRYSTAL_EINVAL;
        QmaskItem &d = it[i];
        d.words = (uint32_t *)x.t->mem;
        d.span = x.t->span;
        d.key_min = x.t->key_min;
        d.ranked = x.t->ranked;
        d.keys = x.keys;
        d.filter_col = x.filter_col;
        d.n = x.n;
        d.r = QmaskRanges{};
        d.r.n = x.n_queries;
        for (int q = 0; q < x.n_queries; ++q) {
            d.r.lo[q] = x.ranges[q].lo;
            d.r.hi[q] = x.ranges[q].hi;
        }
    }
    return from_hip(launch_qmask_build_batch(it, n_items, status, as_stream(stream)));
}

crystal_status crystal_run_shared_scan(const crystal_batch *b, int32_t *status, void *stream) {
    if (!b || !status || b->n_queries < 0 || b->n_queries > CRYSTAL_MAX_BATCH) return CRYSTAL_EINVAL;
    BatchDev d;
    memset(&d, 0, sizeof(d));
    crystal_status st = star_plan_to_dev(b->plan, d.plan);
    if (st != CRYSTAL_OK) return st;
    for (int c = 0; c < CRYSTAL_MAX_COLS; ++c)
        if (d.plan.col[c].width != 4) return CRYSTAL_EINVAL;  // the batch kernel reads int32 columns
    if (b->row_begin < 0 || b->row_end > b->plan.n_rows || (b->row_begin & 3)) return CRYSTAL_EINVAL;
    for (int j = 0; j < b->plan.n_joins; ++j) {
        const crystal_qmask_table &m = b->masks[j];
        if (!qmask_table_ok(&m)) return CRYSTAL_EINVAL;
        d.mask[j].mem = (const uint16_t *)m.mem;
        d.mask[j].span = m.span;
        d.mask[j].key_min = m.key_min;
        d.mask[j].ranked = m.ranked;
    }
    d.n_queries = b->n_queries;
    d.all_queries = b->n_queries >= 32 ? 0xffffffffu : ((1u << b->n_queries) - 1u);
    for (int q = 0; q < b->n_queries; ++q) {
        if (!b->queries[q].out) return CRYSTAL_EINVAL;
        d.out[q] = (uint64_t *)b->queries[q].out;
        for (int i = 0; i < b->plan.n_preds; ++i) {
            d.pred_lo[q][i] = b->queries[q].preds[i].lo;
            d.pred_hi[q][i] = b->queries[q].preds[i].hi;
        }
    }
    d.row_begin = b->row_begin;
    d.row_end = b->row_end;
    const int kernel = d.plan.scalar ? CRYSTAL_K_SHARED_SCAN_SCALAR : CRYSTAL_K_SHARED_SCAN;
    return from_hip(launch_shared_scan(tune_lookup(kernel, b->row_end - b->row_begin), d, status,
                                       as_stream(stream)));
}

// ----------------------------------------------------------------- graphs --
struct crystal_graph {
    hipGraph_t graph;
    hipGraphExec_t exec;
};

crystal_status crystal_graph_begin(void *stream) {
    if (!stream) return CRYSTAL_EINVAL;  // the legacy default stream cannot be captured
    return from_hip(hipStreamBeginCapture(as_stream(stream), hipStreamCaptureModeThreadLocal));
}

crystal_status crystal_graph_end(void *stream, crystal_graph **out) {
    if (!stream || !out) return CRYSTAL_EINVAL;
    *out = nullptr;
    hipGraph_t g = nullptr;
    if (hipStreamEndCapture(as_stream(stream), &g) != hipSuccess || !g) return CRYSTAL_EHIP;
    hipGraphExec_t e = nullptr;
    if (hipGraphInstantiate(&e, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(g);
        return CRYSTAL_EHIP;
    }
    *out = new crystal_graph{g, e};
    return CRYSTAL_OK;
}

crystal_status crystal_graph_launch(crystal_graph *g, void *stream) {
    if (!g) return CRYSTAL_EINVAL;
    return from_hip(hipGraphLaunch(g->exec, as_stream(stream)));
}

crystal_status crystal_graph_destroy(crystal_graph *g) {
    if (!g) return CRYSTAL_EINVAL;
    hipError_t e1 = hipGraphExecDestroy(g->exec);
    hipError_t e2 = hipGraphDestroy(g->graph);
    delete g;
    return (e1 == hipSuccess && e2 == hipSuccess) ? CRYSTAL_OK : CRYSTAL_EHIP;
}

// ------------------------------------------------------------------ radix --
static bool radix_args_ok(const uint32_t *keys, const uint32_t *vals, int64_t n, const uint32_t *ok,
                          const uint32_t *ov) {
    if (n < 0 || n > (int64_t)UINT32_MAX - 1) return false;
    if (n == 0) return true;  // nothing is read or written
    if ((vals == nullptr) != (ov == nullptr)) return false;
    if (!keys || !ok || ((uintptr_t)keys & 3u) || ((uintptr_t)ok & 3u)) return false;
    if (vals && (((uintptr_t)vals & 3u) || ((uintptr_t)ov & 3u))) return false;
    // outputs must not overlap inputs
    auto overlap = [n](const void *a, const void *b) {
        const char *x = (const char *)a, *y = (const char *)b;
        return x < y + n * 4 && y < x + n * 4;
    };
    if (overlap(keys, ok) || (vals && (overlap(vals, ov) || overlap(keys, ov) || overlap(vals, ok) ||
                                      overlap(ok, ov))))
        return false;
    return true;
}

crystal_status crystal_radix_histogram(const uint32_t *keys, int64_t n, int32_t shift, int32_t bits,
                                       uint32_t *hist, void *stream) {
    if (bits < 1 || bits > 8 || shift < 0 || shift + bits > 32 || !hist || n < 0 || n > (int64_t)UINT32_MAX - 1 ||
        (n > 0 && (!keys || ((uintptr_t)keys & 3u))))
        return CRYSTAL_EINVAL;
    const LaunchCfg cfg = tune_lookup(CRYSTAL_K_RADIX, n);
    return from_hip(launch_radix_histogram(cfg, keys, n, shift, bits, hist, as_stream(stream)));
}

size_t crystal_radix_partition_scratch_bytes(int64_t n) {
    return (size_t)radix_pass_scratch_bytes(tune_lookup(CRYSTAL_K_RADIX, n), n);
}

static crystal_status radix_partition_common(const uint32_t *keys, const uint32_t *vals, int64_t n, int32_t shift,
                                             int32_t bits, uint32_t *out_keys, uint32_t *out_vals,
                                             uint32_t *part_offsets, void *scratch, size_t scratch_bytes,
                                             void *stream, bool stable) {
    if (bits < 1 || bits > 8 || shift < 0 || shift + bits > 32 || !radix_args_ok(keys, vals, n, out_keys, out_vals))
        return CRYSTAL_EINVAL;
    const LaunchCfg cfg = tune_lookup(CRYSTAL_K_RADIX, n);
    if (!radix_variant_fits(cfg.block, cfg.ipt)) return CRYSTAL_EINVAL;
    if (n > 0) {
        if (!scratch || ((uintptr_t)scratch & 255u)) return scratch ? CRYSTAL_EINVAL : CRYSTAL_ESCRATCH;
        if (scratch_bytes < (size_t)radix_pass_scratch_bytes(cfg, n)) return CRYSTAL_ESCRATCH;
    }
    return from_hip(launch_radix_partition(cfg, keys, vals, n, shift, bits, out_keys, out_vals, part_offsets,
                                           scratch, stable, as_stream(stream)));
}

crystal_status crystal_radix_partition(const uint32_t *keys, const uint32_t *vals, int64_t n, int32_t shift,
                                       int32_t bits, uint32_t *out_keys, uint32_t *out_vals,
                                       uint32_t *part_offsets, void *scratch, size_t scratch_bytes,
                                       void *stream) {
    return radix_partition_common(keys, vals, n, shift, bits, out_keys, out_vals, part_offsets, scratch,
                                  scratch_bytes, stream, true);
}

crystal_status crystal_radix_partition_unstable(const uint32_t *keys, const uint32_t *vals, int64_t n,
                                                int32_t shift, int32_t bits, uint32_t *out_keys,
                                                uint32_t *out_vals, uint32_t *part_offsets, void *scratch,
                                                size_t scratch_bytes, void *stream) {
    return radix_partition_common(keys, vals, n, shift, bits, out_keys, out_vals, part_offsets, scratch,
                                  scratch_bytes, stream, false);
}

static int64_t round256(int64_t b) { return (b + 255) / 256 * 256; }

size_t crystal_sort_pairs_scratch_bytes(int64_t n, int32_t with_values) {
    if (n <= 0) return 256;
    const int64_t copy = round256(n * 4);
    return (size_t)(copy * (with_values ? 2 : 1) +
                    radix_pass_scratch_bytes(tune_lookup(CRYSTAL_K_RADIX, n), n));
}

crystal_status crystal_sort_pairs(const uint32_t *keys, const uint32_t *vals, int64_t n, uint32_t *out_keys,
                                  uint32_t *out_vals, void *scratch, size_t scratch_bytes, void *stream) {
    if (!radix_args_ok(keys, vals, n, out_keys, out_vals)) return CRYSTAL_EINVAL;
    if (n == 0) return CRYSTAL_OK;
    const LaunchCfg cfg = tune_lookup(CRYSTAL_K_RADIX, n);
    if (!radix_variant_fits(cfg.block, cfg.ipt)) return CRYSTAL_EINVAL;
    if (!scratch || ((uintptr_t)scratch & 255u)) return scratch ? CRYSTAL_EINVAL : CRYSTAL_ESCRATCH;
    if (scratch_bytes < crystal_sort_pairs_scratch_bytes(n, vals != nullptr)) return CRYSTAL_ESCRATCH;
    const int64_t copy = round256(n * 4);
    uint32_t *tk = (uint32_t *)scratch;
    uint32_t *tv = vals ? (uint32_t *)((char *)scratch + copy) : nullptr;
    void *pass = (char *)scratch + copy * (vals ? 2 : 1);
    // in -> tmp -> out -> tmp -> out, 8 bits per pass from the low byte up
    const uint32_t *ik[4] = {keys, tk, out_keys, tk};
    const uint32_t *iv[4] = {vals, tv, out_vals, tv};
    uint32_t *ok[4] = {tk, out_keys, tk, out_keys};
    uint32_t *ov[4] = {tv, out_vals, tv, out_vals};
    for (int p = 0; p < 4; ++p) {
        hipError_t e = launch_radix_partition(cfg, ik[p], iv[p], n, 8 * p, 8, ok[p], ov[p], nullptr, pass, true,
                                              as_stream(stream));
        if (e != hipSuccess) return CRYSTAL_EHIP;
    }
    return CRYSTAL_OK;
}

size_t crystal_sort_pairs_msb_scratch_bytes(int64_t n, int32_t with_values) {
    if (n <= 0) return 256;
    return (size_t)msb_sort_scratch_bytes(n, with_values != 0);
}

crystal_status crystal_sort_pairs_msb(const uint32_t *keys, const uint32_t *vals, int64_t n, uint32_t *out_keys,
                                      uint32_t *out_vals, void *scratch, size_t scratch_bytes, void *stream) {
    if (!radix_args_ok(keys, vals, n, out_keys, out_vals)) return CRYSTAL_EINVAL;
    if (n == 0) return CRYSTAL_OK;
    if (!scratch || ((uintptr_t)scratch & 255u)) return scratch ? CRYSTAL_EINVAL : CRYSTAL_ESCRATCH;
    if (scratch_bytes < crystal_sort_pairs_msb_scratch_bytes(n, vals != nullptr)) return CRYSTAL_ESCRATCH;
    const LaunchCfg cfg = tune_lookup(CRYSTAL_K_RADIX, n);  // the first level's partition pass
    if (!radix_variant_fits(cfg.block, cfg.ipt)) return CRYSTAL_EINVAL;
    return from_hip(launch_msb_sort(keys, vals, n, out_keys, out_vals, scratch, as_stream(stream)));
}

// ----------------------------------------------------------------- tuning --
int32_t crystal_tune_variants(int32_t kernel, int32_t *blocks, int32_t *ipts, int32_t max) {
    if (kernel < 0 || kernel >= CRYSTAL_K_COUNT) return 0;
    int32_t n = 0;
    auto add = [&](int b, int i) {
        if (blocks && ipts && n < max) {
            blocks[n] = b;
            ipts[n] = i;
        }
        ++n;
    };
    if (kernel == CRYSTAL_K_SELECT) {
#define X(B, I) add(B, I);
        CRYSTAL_VARIANTS_ALL(X)
#undef X
    } else if (kernel == CRYSTAL_K_RADIX) {
#define X(B, I) add(B, I);
        CRYSTAL_VARIANTS_RADIX(X)
#undef X
    } else {
#define X(B, I) add(B, I);
        CRYSTAL_VARIANTS_VEC(X)
#undef X
    }
    return n;
}

crystal_status crystal_tune_set(int32_t kernel, int32_t bucket_lo, int32_t bucket_hi, int32_t block,
                                int32_t ipt, int32_t grid_per_cu) {
    if (kernel < 0 || kernel >= CRYSTAL_K_COUNT || !variant_exists(kernel, block, ipt) || grid_per_cu < 0 ||
        grid_per_cu > 64)
        return CRYSTAL_EINVAL;
    if (bucket_lo < 0 && bucket_hi < 0) {
        bucket_lo = 0;
        bucket_hi = 63;
    }
    if (bucket_lo < 0 || bucket_hi < bucket_lo) return CRYSTAL_EINVAL;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.push_back({kernel, bucket_lo, bucket_hi, {block, ipt, grid_per_cu}});
    return CRYSTAL_OK;
}

crystal_status crystal_tune_get(int32_t kernel, int64_t n, int32_t *block, int32_t *ipt,
                                int32_t *grid_per_cu) {
    if (kernel < 0 || kernel >= CRYSTAL_K_COUNT || !block || !ipt || !grid_per_cu) return CRYSTAL_EINVAL;
    LaunchCfg c = tune_lookup(kernel, n);
    *block = c.block;
    *ipt = c.ipt;
    *grid_per_cu = c.grid_per_cu;
    return CRYSTAL_OK;
}

void crystal_tune_reset(void) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.clear();
}

crystal_status crystal_tune_load(const char *path) {
    if (!path) return CRYSTAL_EINVAL;
    FILE *f = fopen(path, "r");
    if (!f) return CRYSTAL_EINVAL;
    char line[256];
    crystal_status st = CRYSTAL_OK;
    while (fgets(line, sizeof line, f)) {
        if (line[0] == '#' || line[0] == '\n') continue;
        int k, lo, hi, b, i, g;
        if (sscanf(line, "%d %d %d %d %d %d", &k, &lo, &hi, &b, &i, &g) != 6) {
            st = CRYSTAL_EINVAL;
            continue;
        }
        if (crystal_tune_set(k, lo, hi, b, i, g) != CRYSTAL_OK) st = CRYSTAL_EINVAL;
    }
    fclose(f);
    return st;
}

crystal_status crystal_tune_save(const char *path) {
    if (!path) return CRYSTAL_EINVAL;
    FILE *f = fopen(path, "w");
    if (!f) return CRYSTAL_EINVAL;
    fprintf(f, "# kernel bucket_lo bucket_hi block ipt grid_per_cu\n");
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (const auto &t : g_tune)
        fprintf(f, "%d %d %d %d %d %d\n", t.kernel, t.blo, t.bhi, t.cfg.block, t.cfg.ipt, t.cfg.grid_per_cu);
    fclose(f);
    return CRYSTAL_OK;
}

}  // extern "C"
