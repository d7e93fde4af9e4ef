// Host-side internals shared by the C ABI and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "crystal.h"

namespace crystal {

struct LaunchCfg {
    int block;
    int ipt;
    int grid_per_cu;  // 0: one workgroup per tile
};

// Compute units of the current device (cached per device).
int device_cu_count();
// Largest dynamic LDS a workgroup may allocate on the current device.
int64_t device_lds_per_block();
// LDS of one compute unit of the current device.
int64_t device_lds_per_cu();
// Workgroups of kernel `fn` resident on one CU of the current device at
// once, for `block` threads and `lds_bytes` of dynamic LDS (the occupancy
// query, cached per device, kernel and LDS size).  A persistent grid larger
// than this per CU would start its extra workgroups late.
hipError_t resident_per_cu(const void *fn, int block, int64_t lds_bytes, int64_t &out);

// Workgroups to launch for n_tiles tiles under cfg.
inline int64_t grid_for(int64_t n_tiles, const LaunchCfg &cfg) {
    if (n_tiles <= 0) return 0;
    if (cfg.grid_per_cu <= 0) return n_tiles;
    int64_t g = (int64_t)cfg.grid_per_cu * device_cu_count();
    return g < n_tiles ? g : n_tiles;
}

LaunchCfg tune_lookup(int kernel, int64_t n);

inline crystal_status from_hip(hipError_t e) {
    return e == hipSuccess ? CRYSTAL_OK : CRYSTAL_EHIP;
}

inline bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

// ------------------------------------------------------------- launchers ----
// Every launcher returns hipSuccess or the launch error; argument checking has
// been done by the C ABI layer.
hipError_t fill_u64(uint64_t *p, int64_t n, uint64_t value, hipStream_t s);
// zero the slots slots[0..count) (each len words) of base in one launch; count <= kMaxSlots
constexpr int kMaxSlots = 64;
hipError_t zero_slots(uint64_t *base, int64_t len, const int32_t *slots, int count, hipStream_t s);
hipError_t fill_u32(uint32_t *p, int64_t n, uint32_t value, hipStream_t s);
// Zero two separate 64-bit words with one launch.
hipError_t zero_pair(uint64_t *a, uint64_t *b, hipStream_t s);

hipError_t launch_pack_column_bits(const int32_t *in, int64_t n, int32_t base, int32_t bits, uint32_t *out,
                                   int64_t words, int32_t *status, hipStream_t s);
hipError_t launch_pack_column(const int32_t *in, int64_t n, int32_t base, int32_t width, void *out,
                              int32_t *status, hipStream_t s);
hipError_t launch_select(const LaunchCfg &cfg, const int32_t *in, int64_t n, int32_t lo, int32_t hi,
                         int32_t *out, int64_t *count, uint64_t *status_words, bool stable, hipStream_t s);
// Items per selection tile under cfg (status words needed: ceil(n / items)).
int64_t select_tile_items(const LaunchCfg &cfg);
hipError_t launch_project(const LaunchCfg &cfg, const float *x1, const float *x2, int64_t n,
                          float a, float b, float *out, bool sigmoid, hipStream_t s);

struct DevTable;
hipError_t launch_ht_clear(const crystal_ht &ht, hipStream_t s);
hipError_t launch_ht_build(const crystal_ht &ht, const int32_t *keys, const int32_t *payload,
                           const int32_t *filter_col, int32_t flo, int32_t fhi, int64_t n,
                           int32_t *status, hipStream_t s);
// Clear and build up to kMaxBuildBatch tables in two launches (arguments checked).
constexpr int kMaxBuildBatch = CRYSTAL_MAX_BUILD_BATCH;
hipError_t launch_ht_build_batch(const crystal_ht_build_item *items, int n_items, int32_t *status,
                                 hipStream_t s);
// MSB radix sort of key/value pairs (vals, out_vals may be null together).
int64_t msb_sort_scratch_bytes(int64_t n, bool with_values);
hipError_t launch_msb_sort(const uint32_t *keys, const uint32_t *vals, int64_t n, uint32_t *out_keys,
                           uint32_t *out_vals, void *scratch, hipStream_t s);

// The builds of a batch into tables that are already clear, the clears of
// other tables and the zeroing of zero_n int64 words, in one launch.
hipError_t launch_ht_build_batch_fused(const crystal_ht_build_item *items, int n_items, const crystal_ht *const *clear,
                                       int n_clear, int64_t *zero, int64_t zero_n, int32_t *status, hipStream_t s);
hipError_t launch_ht_probe(const LaunchCfg &cfg, const crystal_ht &ht, const int32_t *fk,
                           const int32_t *probe_payload, int64_t n, uint64_t *sum, uint64_t *count,
                           hipStream_t s);
hipError_t launch_groupby(const LaunchCfg &cfg, const int32_t *group, const int32_t *value,
                          int64_t n, int64_t n_groups, uint64_t *sums, int32_t *status,
                          hipStream_t s);

// Device form of a star query (validated, table descriptors resolved).
struct StarJoinDev {
    // table
    const uint32_t *bitmap;
    const int32_t *payload;
    const void *slots;
    int64_t span;
    uint32_t mask;
    int32_t key_min;
    int32_t kind;
    int32_t shift;
    int32_t has_payload;
    // plan
    int32_t fk_col;
    int32_t f_bits, f_shift;
    uint32_t f_mask;
    int32_t f_lo, f_hi;
    int32_t g_bits, g_shift;
    uint32_t g_mask;
    int32_t g_base;
    int64_t g_stride;
};

// One fact column: its storage, its width (4, 2 or 1 bytes per stored value)
// and, for widths 2 and 1, the base the stored offsets add to.  (One array of
// these, rather than parallel arrays, keeps dynamically indexed accesses to
// the kernel argument in the kernel-argument segment.)
struct ColDev {
    const int32_t *p;
    int32_t width;  // bytes per stored value (4, 2 or 1); 0 for a bit-packed column
    int32_t base;
    int32_t bits;   // bit-packed: bits per value (1..16); 0 otherwise
    int32_t reserved;
};

struct StarPlanDev {
    ColDev col[CRYSTAL_MAX_COLS];
    int64_t n_rows;
    int64_t n_groups;
    int32_t n_preds;
    int32_t n_joins;
    int32_t pred_col[CRYSTAL_MAX_PREDS];
    int32_t pred_lo[CRYSTAL_MAX_PREDS];
    int32_t pred_hi[CRYSTAL_MAX_PREDS];
    int32_t agg, agg_col0, agg_col1;
    int32_t scalar;  // single group and no group fields: BlockAggregate path
    // set by the launcher: LDS word offsets of the staged bitmaps of the two
    // dense steps (-1: not staged) and of the survivor queue
    int32_t stage_off[2];
    int32_t queue_off;
    int32_t queue_cap;
    StarJoinDev joins[CRYSTAL_MAX_JOINS];
};

// Persistent star-kernel workgroups per CU never exceed this.
constexpr int kStarMaxGridPerCu = 32;
// Largest grid the star kernel launches for n rows (sizes the scalar partials).
int64_t star_max_grid(int64_t n_rows);
// Capacity of the per-device partials array used by
// crystal_run_star_query_noalloc: star_max_grid() on a 256-CU device.
constexpr int64_t kStarNoallocPartials = CRYSTAL_STAR_NOALLOC_PARTIALS;
// Device address of that array on the current device (looked up once per
// device with hipGetSymbolAddress).
hipError_t star_noalloc_partials(uint64_t **ptr);

crystal_status star_plan_to_dev(const crystal_star_query &q, StarPlanDev &d);

// ----------------------------------------------------------- shared scan --
constexpr int kMaxBatch = CRYSTAL_MAX_BATCH;

struct QmaskRanges {
    int32_t n;
    int32_t lo[kMaxBatch];
    int32_t hi[kMaxBatch];
};

// Rank-compressed query-mask table: ceil(span / 32) + 1 directory entries of
// two 32-bit words (presence bits, keys present before them; the last entry
// all zero), then ranked + 1 16-bit entries (the last one zero).
__host__ __device__ inline int64_t qmask_dir_entries(int64_t span) { return (span + 31) / 32 + 1; }
__host__ __device__ inline int64_t qmask_ranked_words(int64_t span, int32_t ranked) {
    return 2 * qmask_dir_entries(span) + ((int64_t)ranked + 2) / 2;
}

// One join's query-mask table as the batch kernel reads it.  (One struct per
// join rather than parallel arrays: a dynamic index into a kernel argument's
// arrays can make the compiler copy the whole argument into scratch.)
struct MaskDev {
    const uint16_t *mem;   // the batch's query-mask table
    int64_t span;
    int32_t key_min;
    int32_t ranked;        // 0: plain table; else rank-compressed with this many entries
    // set by the launcher: the table is copied into the dynamic LDS at 32-bit
    // word stage_off (stage_words words, then one zero word) when
    // stage_words > 0
    int64_t stage_off;
    int64_t stage_words;
};

struct BatchDev {
    StarPlanDev plan;                          // the template
    MaskDev mask[CRYSTAL_MAX_JOINS];           // per join
    int32_t n_queries;
    uint32_t all_queries;                      // (1 << n_queries) - 1
    int32_t pred_lo[kMaxBatch][CRYSTAL_MAX_PREDS];
    int32_t pred_hi[kMaxBatch][CRYSTAL_MAX_PREDS];
    uint64_t *out[kMaxBatch];
    int64_t row_begin;
    int64_t row_end;
    // set by the launcher: 32-bit word of the dynamic LDS where the per-wave
    // queues of sparse rows start (kQueueCap rows and masks per wave), or -1
    int64_t queue_off;
};

hipError_t launch_qmask_build(uint16_t *table, int64_t span, int32_t key_min, int32_t ranked, const int32_t *keys,
                              const int32_t *filter_col, int64_t n, const QmaskRanges &r, int32_t *status,
                              hipStream_t s);
// One table of a batched query-mask build.
struct QmaskItem {
    uint32_t *words;
    int64_t span;
    int32_t key_min;
    int32_t ranked;
    const int32_t *keys;
    const int32_t *filter_col;
    int64_t n;
    QmaskRanges r;
};
hipError_t launch_qmask_build_batch(const QmaskItem *items, int n_items, int32_t *status, hipStream_t s);
hipError_t launch_qmask_rank(uint32_t *table, int64_t span, int32_t key_min, int32_t ranked, const int32_t *keys,
                             int64_t n, int32_t *status, hipStream_t s);
hipError_t launch_shared_scan(const LaunchCfg &cfg, const BatchDev &b, int32_t *status, hipStream_t s);
// accumulate: add into out instead of overwriting it
hipError_t launch_star(const LaunchCfg &cfg, const StarPlanDev &plan, uint64_t *out,
                       int32_t *status, uint64_t *partials, bool accumulate, hipStream_t s);

// ----------------------------------------------------------------- radix --
// Scratch of one partition pass (count matrix + digit totals) under cfg.
int64_t radix_pass_scratch_bytes(const LaunchCfg &cfg, int64_t n);
// Whether the (block, ipt) shuffle variant exists and its LDS fits a workgroup.
bool radix_variant_fits(int block, int ipt);
hipError_t launch_radix_histogram(const LaunchCfg &cfg, const uint32_t *keys, int64_t n, int shift, int bits,
                                  uint32_t *hist, hipStream_t s);
hipError_t launch_radix_partition(const LaunchCfg &cfg, const uint32_t *keys, const uint32_t *vals, int64_t n,
                                  int shift, int bits, uint32_t *out_keys, uint32_t *out_vals,
                                  uint32_t *part_offsets, void *scratch, bool stable, hipStream_t s);

}  // namespace crystal
