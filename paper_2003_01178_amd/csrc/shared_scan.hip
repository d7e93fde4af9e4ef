// Shared-scan batch kernel: up to 16 queries of one star-query template
// (same columns, joins, group spec and aggregate; their own constants) are
// answered in one pass over a range of fact rows.
//
// Every row carries a 16-bit query mask (bit q: still alive for query q).  A
// predicate step loads its column once (BlockLoad / BlockLoadSel on rows alive
// for any query) and clears the bits of the queries whose range the value
// misses.  A join step loads its foreign-key column once and ANDs the row's
// mask with the dimension's query-mask table: for every key, the set of
// batch queries whose dimension filter that row passes (built per batch by
// qmask_build_kernel).  So a join costs one 2-byte lookup per row (a
// directory read and an entry read for a rank-compressed table) however many
// queries share the pass.  Tables that fit are copied into LDS once per
// workgroup and read there.  The first steps run over whole tiles; once few
// rows of a wave's tile are still alive, they go to a per-wave queue and are
// finished 64 at a time, one row per lane.  Survivors form their group index from the
// template's dimension payloads once, then add the measure to every query
// whose bit is set: grouped results with 64-bit atomics into the query's own
// output, scalar results through per-workgroup LDS accumulators.
//
// Outputs are accumulated, never cleared here: a query admitted into a batch
// can be answered over several launches that cover successive row ranges.
#include "block.hpp"
#include "internal.hpp"
#include "variants.hpp"

namespace crystal {

// ------------------------------------------------------------ mask tables --
// Entry of a key (offset off from key_min) in a rank-compressed table, from
// its directory entry d = (presence bits, keys present before them): the
// key's rank among the present keys, or `ranked` (the zero entry) when the
// key is absent.
__device__ __forceinline__ uint32_t ranked_entry(uint32_t bits, uint32_t before, uint32_t off, uint32_t ranked) {
    const uint32_t bit = off & 31u;
    return ((bits >> bit) & 1u) ? before + (uint32_t)__builtin_popcount(bits & ((1u << bit) - 1u)) : ranked;
}

// entry[key - key_min] |= bit q for every query q whose range holds the row's
// filter attribute (entry[rank of the key] for a ranked table).  Two 16-bit
// entries share a 32-bit word, set with atomicOr.
__device__ __forceinline__ void qmask_row(uint32_t *__restrict__ words, int64_t span, int32_t key_min,
                                          int32_t ranked, const int32_t *__restrict__ keys,
                                          const int32_t *__restrict__ filter_col, int64_t i, const QmaskRanges &r,
                                          int32_t *status) {
    const uint32_t *dir = words;
    uint32_t *entries = ranked ? words + 2 * qmask_dir_entries(span) : words;
    const uint32_t off = (uint32_t)keys[i] - (uint32_t)key_min;
    if ((int64_t)off >= span) {
        set_status(status, CRYSTAL_ERANGE);
        return;
    }
    uint32_t e = off;
    if (ranked) {
        e = ranked_entry(dir[2 * (off >> 5)], dir[2 * (off >> 5) + 1], off, (uint32_t)ranked);
        if (e >= (uint32_t)ranked) {  // not in the directory
            set_status(status, CRYSTAL_ERANGE);
            return;
        }
    }
    const int32_t f = filter_col ? filter_col[i] : 0;
    uint32_t m = 0;
    for (int q = 0; q < r.n; ++q) m |= (uint32_t)(filter_col ? in_range(f, r.lo[q], r.hi[q]) : true) << q;
    if (m) atomicOr(entries + (e >> 1), m << ((e & 1u) * 16u));
}

// words of a table's entries, cleared before every build
__host__ __device__ inline int64_t qmask_entry_words(int64_t span, int32_t ranked) {
    return ranked ? ((int64_t)ranked + 2) / 2 : (span + 1) / 2;
}
__host__ __device__ inline int64_t qmask_entry_offset(int64_t span, int32_t ranked) {
    return ranked ? 2 * qmask_dir_entries(span) : 0;
}

__global__ __launch_bounds__(256) void qmask_build_kernel(uint32_t *__restrict__ words, int64_t span,
                                                          int32_t key_min, int32_t ranked,
                                                          const int32_t *__restrict__ keys,
                                                          const int32_t *__restrict__ filter_col, int64_t n,
                                                          QmaskRanges r, int32_t *status) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        qmask_row(words, span, key_min, ranked, keys, filter_col, i, r, status);
}

hipError_t launch_qmask_build(uint16_t *table, int64_t span, int32_t key_min, int32_t ranked, const int32_t *keys,
                              const int32_t *filter_col, int64_t n, const QmaskRanges &r, int32_t *status,
                              hipStream_t s) {
    uint32_t *words = (uint32_t *)table;
    hipError_t e = fill_u32(words + qmask_entry_offset(span, ranked), qmask_entry_words(span, ranked), 0u, s);
    if (e != hipSuccess || n == 0) return e;
    int64_t grid = (n + 255) / 256;
    const int64_t cap = (int64_t)device_cu_count() * 16;
    if (grid > cap) grid = cap;
    hipLaunchKernelGGL(qmask_build_kernel, dim3((unsigned)grid), dim3(256), 0, s, words, span, key_min, ranked, keys,
                       filter_col, n, r, status);
    return hipGetLastError();
}

// Batched build: one kernel clears every table's entries, a second builds
// them all, its workgroups split among the tables in proportion to their rows.
struct QmaskBatchDev {
    int32_t count;
    QmaskItem it[CRYSTAL_MAX_JOINS];
    int64_t block0[CRYSTAL_MAX_JOINS + 1];  // first workgroup of each table; block0[count] = grid
};

__global__ __launch_bounds__(256) void qmask_clear_batch_kernel(QmaskBatchDev b) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t g0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int t = 0; t < b.count; ++t) {
        const QmaskItem &it = b.it[t];
        uint32_t *w = it.words + qmask_entry_offset(it.span, it.ranked);
        const int64_t n = qmask_entry_words(it.span, it.ranked);
        for (int64_t i = g0; i < n; i += stride) w[i] = 0u;
    }
}

__global__ __launch_bounds__(256) void qmask_build_batch_kernel(QmaskBatchDev b, int32_t *status) {
    int t = 0;
    while (t + 1 < b.count && (int64_t)blockIdx.x >= b.block0[t + 1]) ++t;
    const QmaskItem &it = b.it[t];
    const int64_t stride = (b.block0[t + 1] - b.block0[t]) * blockDim.x;
    for (int64_t i = ((int64_t)blockIdx.x - b.block0[t]) * blockDim.x + threadIdx.x; i < it.n; i += stride)
        qmask_row(it.words, it.span, it.key_min, it.ranked, it.keys, it.filter_col, i, it.r, status);
}

hipError_t launch_qmask_build_batch(const QmaskItem *items, int n_items, int32_t *status, hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    QmaskBatchDev b = {};
    b.count = n_items;
    int64_t clear_words = 0, blocks = 0;
    const int64_t cap = (int64_t)device_cu_count() * 16;
    for (int t = 0; t < n_items; ++t) {
        b.it[t] = items[t];
        const int64_t w = qmask_entry_words(items[t].span, items[t].ranked);
        clear_words = w > clear_words ? w : clear_words;
        b.block0[t] = blocks;
        int64_t nb = (items[t].n + 255) / 256;
        if (nb > cap) nb = cap;
        if (nb < 1) nb = 1;  // a table with no rows still owns one (idle) workgroup
        blocks += nb;
    }
    b.block0[n_items] = blocks;
    int64_t cgrid = (clear_words + 255) / 256;
    if (cgrid > cap) cgrid = cap;
    if (cgrid < 1) cgrid = 1;
    hipLaunchKernelGGL(qmask_clear_batch_kernel, dim3((unsigned)cgrid), dim3(256), 0, s, b);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(qmask_build_batch_kernel, dim3((unsigned)blocks), dim3(256), 0, s, b, status);
    return hipGetLastError();
}

// Directory of a ranked table: presence bits first, then one workgroup turns
// them into the number of keys present before each entry.
__global__ __launch_bounds__(256) void qmask_rank_bits_kernel(uint32_t *__restrict__ dir, int64_t span,
                                                              int32_t key_min, const int32_t *__restrict__ keys,
                                                              int64_t n, int32_t *status) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint32_t off = (uint32_t)keys[i] - (uint32_t)key_min;
        if ((int64_t)off >= span) {
            set_status(status, CRYSTAL_ERANGE);
            continue;
        }
        atomicOr(dir + 2 * (off >> 5), 1u << (off & 31u));
    }
}

constexpr int kRankScanBlock = 1024;

__global__ __launch_bounds__(kRankScanBlock) void qmask_rank_scan_kernel(uint32_t *__restrict__ dir, int64_t n_dir,
                                                                         int32_t ranked, int32_t *status) {
    __shared__ uint32_t wave_sums[kRankScanBlock / kWave];
    // thread t owns the entries [t * seg, (t + 1) * seg)
    const int64_t seg = (n_dir + kRankScanBlock - 1) / kRankScanBlock;
    const int64_t lo = (int64_t)threadIdx.x * seg;
    const int64_t hi = lo + seg < n_dir ? lo + seg : n_dir;
    uint32_t local = 0;
    for (int64_t i = lo; i < hi; ++i) local += (uint32_t)__builtin_popcount(dir[2 * i]);
    uint32_t total;
    uint32_t run = block_exclusive_scan<kRankScanBlock, 27>(local, wave_sums, total);
    for (int64_t i = lo; i < hi; ++i) {
        dir[2 * i + 1] = run;
        run += (uint32_t)__builtin_popcount(dir[2 * i]);
    }
    if (threadIdx.x == 0 && total > (uint32_t)ranked) set_status(status, CRYSTAL_EFULL);
}

hipError_t launch_qmask_rank(uint32_t *table, int64_t span, int32_t key_min, int32_t ranked, const int32_t *keys,
                             int64_t n, int32_t *status, hipStream_t s) {
    const int64_t n_dir = qmask_dir_entries(span);
    hipError_t e = fill_u32(table, qmask_ranked_words(span, ranked), 0u, s);
    if (e != hipSuccess) return e;
    if (n > 0) {
        int64_t grid = (n + 255) / 256;
        const int64_t cap = (int64_t)device_cu_count() * 16;
        if (grid > cap) grid = cap;
        hipLaunchKernelGGL(qmask_rank_bits_kernel, dim3((unsigned)grid), dim3(256), 0, s, table, span, key_min, keys,
                           n, status);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(qmask_rank_scan_kernel, dim3(1), dim3(kRankScanBlock), 0, s, table, n_dir, ranked, status);
    return hipGetLastError();
}

// ---------------------------------------------------------- shared scan ----
// The VEC rows from row0 of a column, read as one vector when one of them is
// flagged in `sel` (items past row_end are never read).
template <int VEC>
__device__ __forceinline__ void load_vec_sel(const int32_t *__restrict__ col, int64_t row0, int64_t row_end,
                                             uint32_t sel, int32_t (&dst)[VEC]) {
    if (!sel) return;
    if (row0 + VEC <= row_end) {
        load_vec<VEC, true>(col + row0, dst);
    } else {
#pragma unroll
        for (int e = 0; e < VEC; ++e)
            if ((sel >> e) & 1u) dst[e] = col[row0 + e];
    }
}

// Column of plan step s (predicates first, then joins).  Both candidates are
// loaded (indices clamped into range) and the value is selected: a select
// between two addresses inside the kernel argument would make the compiler
// copy the whole argument into scratch memory.
__device__ __forceinline__ int shared_step_col(const StarPlanDev &p, int s) {
    const int i = s < CRYSTAL_MAX_PREDS ? s : CRYSTAL_MAX_PREDS - 1;
    const int j = s - p.n_preds;
    const int pc = p.pred_col[i < 0 ? 0 : i];
    const int jc = p.joins[j < 0 ? 0 : (j < CRYSTAL_MAX_JOINS ? j : CRYSTAL_MAX_JOINS - 1)].fk_col;
    return s < p.n_preds ? pc : jc;
}

// Queue of sparse rows per wave: once a tile's rows still alive after the
// dense steps are few, they are appended (row, query mask, next step) to the
// wave's queue and finished 64 at a time, one row per lane, instead of
// running every later step over the whole tile.
constexpr int kQueueCap = 128;  // entries per wave (a power of two, at least 2 x 64)

// One plan step for one queued row: its value x and query mask m.
__device__ __forceinline__ uint32_t step_one(const BatchDev &b, const uint32_t *lds_words, int s, int32_t x,
                                             uint32_t m) {
    const StarPlanDev &p = b.plan;
    if (s < p.n_preds) {
        uint32_t r = 0;
        for (int q = 0; q < b.n_queries; ++q) {
            const uint32_t bit = 1u << q;
            if (ballot((m & bit) != 0u) == 0) continue;
            r |= in_range(x, b.pred_lo[q][s], b.pred_hi[q][s]) ? bit : 0u;
        }
        return m & r;
    }
    const MaskDev &md = b.mask[s - p.n_preds];
    const uint32_t off = (uint32_t)x - (uint32_t)md.key_min;
    const uint32_t rk = (uint32_t)md.ranked;
    if (md.stage_words > 0) {
        const uint32_t *sw = lds_words + md.stage_off;
        if (rk) {
            const uint32_t dlast = (uint32_t)(qmask_dir_entries(md.span) - 1);
            const uint32_t wi = (off >> 5) < dlast ? (off >> 5) : dlast;
            const uint2 d = *reinterpret_cast<const uint2 *>(sw + 2 * wi);
            const uint16_t *ent = reinterpret_cast<const uint16_t *>(sw + 2 * (dlast + 1u));
            return m & (uint32_t)ent[ranked_entry(d.x, d.y, off, rk)];
        }
        const uint16_t *stage = reinterpret_cast<const uint16_t *>(sw);
        const uint32_t span = (uint32_t)md.span;
        return m & (uint32_t)stage[off < span ? off : span];
    }
    if (m == 0u || (int64_t)off >= md.span) return 0u;
    if (rk) {
        const uint32_t *gw = reinterpret_cast<const uint32_t *>(md.mem);
        const uint2 d = *reinterpret_cast<const uint2 *>(gw + 2 * (off >> 5));
        const uint16_t *ent = reinterpret_cast<const uint16_t *>(gw + 2 * qmask_dir_entries(md.span));
        return m & (uint32_t)ent[ranked_entry(d.x, d.y, off, rk)];
    }
    return m & (uint32_t)md.mem[off];
}

template <int BLOCK, int IPT>
__global__ __launch_bounds__(BLOCK) void shared_scan_kernel(const BatchDev batch, int32_t *status, int64_t n_tiles) {
    using T = TileShape<BLOCK, IPT>;
    // The batch is read in place from the kernel-argument segment, where it
    // is the first argument (offset 0).  Used as a by-value parameter, its
    // many dynamically indexed fields made the compiler copy all 1.6 KB of it
    // into scratch memory.
#if __HIP_DEVICE_COMPILE__
    const BatchDev &b = *reinterpret_cast<const BatchDev *>(__builtin_amdgcn_kernarg_segment_ptr());
#else  // the host pass only parses the body
    const BatchDev &b = batch;
#endif
    // scalar results: one LDS accumulator per (query, lane), shared by the
    // workgroup's waves.  The lanes of a wave add to distinct slots, and the
    // adds are LDS atomics without return, so no wave waits on another's;
    // reduced once per workgroup at the end.
    // dynamic LDS: b.n_queries * 64 64-bit slots for a scalar plan, then the
    // staged mask tables (see MaskDev::stage_off)
    extern __shared__ uint64_t dyn[];
    uint64_t(*acc)[kWave] = reinterpret_cast<uint64_t(*)[kWave]>(dyn);
    uint32_t *lds_words = reinterpret_cast<uint32_t *>(dyn);
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const StarPlanDev &p = b.plan;
    const int n_steps = p.n_preds + p.n_joins;
    if (p.scalar) {
        for (int i = threadIdx.x; i < b.n_queries * kWave; i += BLOCK) dyn[i] = 0;
    }
    bool any_staged = false;
    for (int j = 0; j < p.n_joins; ++j) {
        const MaskDev &md = b.mask[j];
        if (md.stage_words == 0) continue;
        any_staged = true;
        const uint32_t *src = reinterpret_cast<const uint32_t *>(md.mem);
        uint32_t *dst = lds_words + md.stage_off;
        for (int64_t i = threadIdx.x; i < md.stage_words; i += BLOCK) dst[i] = src[i];
        if (threadIdx.x == 0) dst[md.stage_words] = 0u;  // entries past the table read 0
    }
    if (any_staged || p.scalar) __syncthreads();
    bool bad_group = false;
    uint32_t qm[IPT];

    // One plan step over the tile's values x: range predicates per query, or a
    // lookup of the join's query-mask table.
    auto apply_step = [&](int s, const int32_t(&x)[IPT]) {
        if (s < p.n_preds) {
            // queries outer, items inner: each query's bounds are uniform, and
            // a query no row of the wave is still alive for is skipped
            uint32_t lane_live = 0, m[IPT];
#pragma unroll
            for (int k = 0; k < IPT; ++k) {
                lane_live |= qm[k];
                m[k] = 0;
            }
            for (int q = 0; q < b.n_queries; ++q) {
                const uint32_t bit = 1u << q;
                if (ballot((lane_live & bit) != 0u) == 0) continue;
                const int32_t lo = b.pred_lo[q][s], hi = b.pred_hi[q][s];
#pragma unroll
                for (int k = 0; k < IPT; ++k) m[k] |= in_range(x[k], lo, hi) ? bit : 0u;
            }
#pragma unroll
            for (int k = 0; k < IPT; ++k) qm[k] &= m[k];
        } else {
            const MaskDev &md = b.mask[s - p.n_preds];
            const uint32_t last = (uint32_t)(md.span - 1);
            const int32_t kmin = md.key_min;
            const uint32_t rk = (uint32_t)md.ranked;
            if (md.stage_words > 0 && rk) {
                // ranked table in LDS: keys past the span read the directory's
                // last entry, which has no presence bits
                const uint32_t *sw = lds_words + md.stage_off;
                const uint32_t dlast = (uint32_t)(qmask_dir_entries(md.span) - 1);
                const uint16_t *ent = reinterpret_cast<const uint16_t *>(sw + 2 * (dlast + 1u));
                // a vector of VEC items at a time: its directory reads issued
                // together, then its entry reads, so the two dependent LDS
                // latencies are paid once per vector rather than per item
#pragma unroll
                for (int c = 0; c < IPT; c += T::VEC) {
                    uint32_t off[T::VEC], e[T::VEC];
                    uint2 d[T::VEC];
#pragma unroll
                    for (int i = 0; i < T::VEC; ++i) {
                        off[i] = (uint32_t)x[c + i] - (uint32_t)kmin;
                        const uint32_t wi = (off[i] >> 5) < dlast ? (off[i] >> 5) : dlast;
                        d[i] = *reinterpret_cast<const uint2 *>(sw + 2 * wi);
                    }
#pragma unroll
                    for (int i = 0; i < T::VEC; ++i) e[i] = ranked_entry(d[i].x, d[i].y, off[i], rk);
#pragma unroll
                    for (int i = 0; i < T::VEC; ++i) qm[c + i] &= (uint32_t)ent[e[i]];
                }
            } else if (md.stage_words > 0) {
                // LDS-typed path (a pointer that may also address global
                // memory would compile to flat loads).  Keys outside the
                // table are clamped to the zero entry after it, so no range
                // test is needed.
                const uint16_t *stage = reinterpret_cast<const uint16_t *>(lds_words + md.stage_off);
                const uint32_t span = last + 1u;
#pragma unroll
                for (int k = 0; k < IPT; ++k) {
                    const uint32_t off = (uint32_t)x[k] - (uint32_t)kmin;
                    qm[k] &= (uint32_t)stage[off < span ? off : span];
                }
            } else if (rk) {
                const uint32_t *gw = reinterpret_cast<const uint32_t *>(md.mem);
                const uint16_t *ent = reinterpret_cast<const uint16_t *>(gw + 2 * qmask_dir_entries(md.span));
#pragma unroll
                for (int k = 0; k < IPT; ++k) {
                    const uint32_t off = (uint32_t)x[k] - (uint32_t)kmin;
                    uint32_t m = 0;
                    if (qm[k] != 0u && off <= last) {
                        const uint2 d = *reinterpret_cast<const uint2 *>(gw + 2 * (off >> 5));
                        m = ent[ranked_entry(d.x, d.y, off, rk)];
                    }
                    qm[k] &= m;
                }
            } else {
                const uint16_t *mt = md.mem;
#pragma unroll
                for (int k = 0; k < IPT; ++k) {
                    const uint32_t off = (uint32_t)x[k] - (uint32_t)kmin;
                    const bool in = qm[k] != 0u && off <= last;
                    qm[k] &= in ? (uint32_t)mt[off] : 0u;
                }
            }
        }
    };

    // queue of sparse rows (see kQueueCap): absolute row, then query mask |
    // (next step << 16); head and tail are the same in every lane of the wave
    uint32_t *q_row = lds_words + (b.queue_off >= 0 ? b.queue_off : 0) + (threadIdx.x / kWave) * (2 * kQueueCap);
    uint32_t *q_msk = q_row + kQueueCap;
    uint32_t head = 0, tail = 0;

    // The remaining plan steps of one queued row from step s0, then its
    // aggregate for every query still set in m.
    auto finish_row = [&](int64_t row, uint32_t m, int s0) {
        for (int s = 2; s < n_steps; ++s) {
            if (ballot(m != 0u) == 0) return;
            if (s < s0) continue;
            const int32_t x = m ? p.col[shared_step_col(p, s)].p[row] : 0;
            m = step_one(b, lds_words, s, x, m);
        }
        if (m == 0u) return;
        uint64_t val = 1;
        if (p.agg != CRYSTAL_AGG_COUNT) {
            const int64_t a = p.col[p.agg_col0].p[row];
            const int64_t c = (p.agg == CRYSTAL_AGG_SUM_PRODUCT || p.agg == CRYSTAL_AGG_SUM_DIFF)
                                  ? (int64_t)p.col[p.agg_col1].p[row] : 0;
            val = (uint64_t)(p.agg == CRYSTAL_AGG_SUM ? a : p.agg == CRYSTAL_AGG_SUM_PRODUCT ? a * c : a - c);
        }
        int64_t g = 0;
        if (!p.scalar) {
            for (int jj = 0; jj < p.n_joins; ++jj) {
                const StarJoinDev &j = p.joins[jj];
                if (j.g_bits == 0) continue;
                const int32_t fk = p.col[j.fk_col].p[row];
                int32_t pay = 0;
                if (j.kind == CRYSTAL_HT_DIRECT) {
                    const uint32_t off = (uint32_t)fk - (uint32_t)j.key_min;
                    if ((int64_t)off < j.span && j.payload) pay = j.payload[off];
                } else if (fk != kEmptyKey) {
                    probe_linear((const v2i *)j.slots, j.mask, j.shift, fk, pay);
                }
                g += ((int64_t)payload_field(pay, j.g_shift, j.g_mask, j.g_bits) - (int64_t)j.g_base) * j.g_stride;
            }
            if ((uint64_t)g >= (uint64_t)p.n_groups) {
                bad_group = true;
                return;
            }
        }
        while (m) {
            const int q = __builtin_ctz(m);
            m &= m - 1u;
            if (p.scalar)
                __hip_atomic_fetch_add((__attribute__((address_space(3))) uint64_t *)&acc[q][lane], val,
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            else
                atomic_add_u64(b.out[q] + g, val);
        }
    };
    auto finish_entry = [&](uint32_t slot) {
        const uint32_t mw = q_msk[slot];
        finish_row((int64_t)q_row[slot], mw & 0xffffu, (int)(mw >> 16));
    };

    // Step 2's column is loaded in full at the start of a tile while the
    // wave's selective loads of it touched at least 3/4 of their cache lines
    // (measured on the wave's previous tile): then the full load costs little
    // more and saves one dependent memory round trip.
    bool dense2 = true;

    // One tile.  `cur` holds the first step's column of this tile (loaded one
    // tile ahead); the same column of the workgroup's next tile is loaded into
    // `nxt` before this tile's steps run, so that load overlaps them.
    const int col0 = n_steps > 0 ? shared_step_col(p, 0) : 0;
    auto run_tile = [&](int64_t tile, int32_t(&cur)[IPT], int32_t(&nxt)[IPT]) {
        const int64_t base = b.row_begin + tile * T::ITEMS;
        const uint32_t valid = valid_mask<BLOCK, IPT>(base, b.row_end);
#pragma unroll
        for (int k = 0; k < IPT; ++k) qm[k] = ((valid >> k) & 1u) ? b.all_queries : 0u;
        // the second step's column is read in full together with the first
        // (with up to 16 queries most of its vectors hold a live row anyway),
        // so the two loads share one memory round trip
        int32_t w[IPT], w2[IPT];
        int w_col = n_steps > 1 ? shared_step_col(p, 1) : -1;  // the column w holds for the live rows
        if (n_steps > 1) block_load<BLOCK, IPT, true>(p.col[w_col].p, base, b.row_end, w);
        const bool pre2 = n_steps > 2 && dense2;
        if (pre2) block_load<BLOCK, IPT, true>(p.col[shared_step_col(p, 2)].p, base, b.row_end, w2);
        const int64_t tn = tile + gridDim.x;
        if (n_steps > 0 && tn < n_tiles)
            block_load<BLOCK, IPT, true>(p.col[col0].p, b.row_begin + tn * T::ITEMS, b.row_end, nxt);
        if (n_steps > 0) apply_step(0, cur);
        if (n_steps > 1) apply_step(1, w);
        for (int s = 2; s < n_steps; ++s) {
            uint32_t any = 0;
#pragma unroll
            for (int k = 0; k < IPT; ++k) any |= (uint32_t)(qm[k] != 0u) << k;
            if (ballot(any != 0u) == 0) return;
            if (s == 2) {
                // cache lines a selective load would touch: eight lanes'
                // 16-byte vectors per 128-byte line
                int touched = 0;
#pragma unroll
                for (int ch = 0; ch < T::CHUNKS; ++ch) {
                    uint64_t m = ballot(((any >> (ch * T::VEC)) & T::VMASK) != 0u);
                    m |= m >> 4;
                    m |= m >> 2;
                    m |= m >> 1;
                    touched += __builtin_popcountll(m & 0x0101010101010101ull);
                }
                dense2 = 4 * touched >= 3 * 8 * T::CHUNKS;
                if (pre2) {
                    apply_step(2, w2);
                    continue;
                }
            }
            if (b.queue_off >= 0) {
                // few live rows left in the wave: queue them (the queue holds
                // fewer than 64 before, so at most 127 after) and finish the
                // queue 64 rows at a time
                uint32_t total;
                const uint32_t before = wave_exclusive_scan_small<T::CBITS>((uint32_t)__builtin_popcount(any), total);
                if (total <= (uint32_t)kWave) {
                    uint32_t pos = tail + before;
#pragma unroll
                    for (int k = 0; k < IPT; ++k) {
                        if ((any >> k) & 1u) {
                            const uint32_t slot = pos & (uint32_t)(kQueueCap - 1);
                            q_row[slot] = (uint32_t)T::index(base, k / T::VEC, k % T::VEC);
                            q_msk[slot] = qm[k] | ((uint32_t)s << 16);
                            ++pos;
                        }
                    }
                    tail += total;
                    __builtin_amdgcn_wave_barrier();
                    while (tail - head >= (uint32_t)kWave) {
                        finish_entry((head + lane) & (uint32_t)(kQueueCap - 1));
                        head += kWave;
                    }
                    __builtin_amdgcn_wave_barrier();
                    return;
                }
            }
            w_col = shared_step_col(p, s);
            block_load_sel<BLOCK, IPT, true>(p.col[w_col].p, base, b.row_end, any, w);
            apply_step(s, w);
        }
        // survivors.  Their measures are read for the whole tile at once (one
        // memory round trip); the group index is formed a vector of VEC rows
        // at a time, skipping vectors without a survivor.
        uint32_t surv = 0;
#pragma unroll
        for (int k = 0; k < IPT; ++k) surv |= (uint32_t)(qm[k] != 0u) << k;
        if (ballot(surv != 0u) == 0) return;
        // A measure that is also the column still held in w (the last step
        // column read for these rows; the Q1.1 template's discount) is taken
        // from the registers.  Only up to 8 items per thread: at 16 keeping w
        // live this long spills.
        int32_t a[IPT], c[IPT];
        const bool a_in_w = IPT <= 8 && p.agg_col0 == w_col, c_in_w = IPT <= 8 && p.agg_col1 == w_col;
        if (p.agg != CRYSTAL_AGG_COUNT) {
            if (a_in_w) {
#pragma unroll
                for (int k = 0; k < IPT; ++k) a[k] = w[k];
            } else {
                block_load_sel<BLOCK, IPT, true>(p.col[p.agg_col0].p, base, b.row_end, surv, a);
            }
        }
        if (p.agg == CRYSTAL_AGG_SUM_PRODUCT || p.agg == CRYSTAL_AGG_SUM_DIFF) {
            if (c_in_w) {
#pragma unroll
                for (int k = 0; k < IPT; ++k) c[k] = w[k];
            } else {
                block_load_sel<BLOCK, IPT, true>(p.col[p.agg_col1].p, base, b.row_end, surv, c);
            }
        }
#pragma unroll
        for (int ch = 0; ch < T::CHUNKS; ++ch) {
            const uint32_t sc = (surv >> (ch * T::VEC)) & T::VMASK;
            if (ballot(sc != 0u) == 0) continue;
            const int64_t row0 = T::index(base, ch, 0);
            int64_t g[T::VEC];
#pragma unroll
            for (int e = 0; e < T::VEC; ++e) g[e] = 0;
            if (!p.scalar) {
                for (int jj = 0; jj < p.n_joins; ++jj) {
                    const StarJoinDev &j = p.joins[jj];
                    if (j.g_bits == 0) continue;
                    int32_t fk[T::VEC], pay[T::VEC];
                    load_vec_sel<T::VEC>(p.col[j.fk_col].p, row0, b.row_end, sc, fk);
#pragma unroll
                    for (int e = 0; e < T::VEC; ++e) {
                        pay[e] = 0;
                        if (!((sc >> e) & 1u)) continue;
                        if (j.kind == CRYSTAL_HT_DIRECT) {
                            const uint32_t off = (uint32_t)fk[e] - (uint32_t)j.key_min;
                            if ((int64_t)off < j.span && j.payload) pay[e] = j.payload[off];
                        } else if (fk[e] != kEmptyKey) {
                            probe_linear((const v2i *)j.slots, j.mask, j.shift, fk[e], pay[e]);
                        }
                    }
#pragma unroll
                    for (int e = 0; e < T::VEC; ++e)
                        g[e] += ((int64_t)payload_field(pay[e], j.g_shift, j.g_mask, j.g_bits) - (int64_t)j.g_base) *
                                j.g_stride;
                }
            }
            if (p.scalar) {
                // The (row, query) pairs of each two rows of the chunk as one
                // 32-bit mask, 16 bits per row: the lanes walk their own pairs
                // together, so the wave loops as often as its busiest lane has
                // pairs in the two rows, not once per row for each row's busiest
                // lane, and each trip picks its row's value with one compare.
                constexpr int HALVES = (T::VEC + 1) / 2;
                uint64_t vals[T::VEC];
                uint32_t pend[HALVES];
#pragma unroll
                for (int h = 0; h < HALVES; ++h) pend[h] = 0;
#pragma unroll
                for (int e = 0; e < T::VEC; ++e) {
                    const int k = ch * T::VEC + e;
                    const uint32_t mk = qm[k] & 0xffffu;
                    uint64_t val = 0;
                    if (mk) {  // only survivors' measures were loaded
                        val = 1;
                        if (p.agg == CRYSTAL_AGG_SUM)
                            val = (uint64_t)(int64_t)a[k];
                        else if (p.agg == CRYSTAL_AGG_SUM_PRODUCT)
                            val = (uint64_t)((int64_t)a[k] * (int64_t)c[k]);
                        else if (p.agg == CRYSTAL_AGG_SUM_DIFF)
                            val = (uint64_t)((int64_t)a[k] - (int64_t)c[k]);
                    }
                    vals[e] = val;
                    pend[e / 2] |= mk << (16 * (e & 1));
                }
#pragma unroll
                for (int h = 0; h < HALVES; ++h) {
                    uint32_t pm = pend[h];
                    const uint64_t v0 = vals[2 * h], v1 = vals[2 * h + 1 < T::VEC ? 2 * h + 1 : 2 * h];  // no bit of a missing row is set
                    while (pm) {
                        const uint32_t bit = (uint32_t)__builtin_ctz(pm);
                        pm &= pm - 1u;
                        const uint64_t val = bit >= 16u ? v1 : v0;
                        __hip_atomic_fetch_add((__attribute__((address_space(3))) uint64_t *)&acc[bit & 15u][lane], val,
                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    }
                }
                __builtin_amdgcn_sched_barrier(0);
                continue;
            }
#pragma unroll
            for (int e = 0; e < T::VEC; ++e) {
                const int k = ch * T::VEC + e;
                uint32_t m = qm[k];
                if (!m) continue;
                uint64_t val = 1;
                if (p.agg == CRYSTAL_AGG_SUM)
                    val = (uint64_t)(int64_t)a[k];
                else if (p.agg == CRYSTAL_AGG_SUM_PRODUCT)
                    val = (uint64_t)((int64_t)a[k] * (int64_t)c[k]);
                else if (p.agg == CRYSTAL_AGG_SUM_DIFF)
                    val = (uint64_t)((int64_t)a[k] - (int64_t)c[k]);
                if (!p.scalar && (uint64_t)g[e] >= (uint64_t)p.n_groups) {
                    bad_group = true;
                    continue;
                }
                while (m) {
                    const int q = __builtin_ctz(m);
                    m &= m - 1u;
                    if (p.scalar)  // the lane's slot: an LDS add without return
                        __hip_atomic_fetch_add((__attribute__((address_space(3))) uint64_t *)&acc[q][lane], val,
                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    else
                        atomic_add_u64(b.out[q] + g[e], val);
                }
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    };

    int32_t va[IPT], vb[IPT];
    int64_t tile = blockIdx.x;
    if (n_steps > 0 && tile < n_tiles)
        block_load<BLOCK, IPT, true>(p.col[col0].p, b.row_begin + tile * T::ITEMS, b.row_end, va);
    // unrolled by two so that the buffer receiving loads is never copied
    while (tile < n_tiles) {
        run_tile(tile, va, vb);
        tile += gridDim.x;
        if (tile >= n_tiles) break;
        run_tile(tile, vb, va);
        tile += gridDim.x;
    }
    if (lane < tail - head) finish_entry((head + lane) & (uint32_t)(kQueueCap - 1));
    if (bad_group) set_status(status, CRYSTAL_ERANGE);
    if (p.scalar) {
        __syncthreads();  // every wave's adds are done
        if (threadIdx.x < kWave) {
            for (int q = 0; q < b.n_queries; ++q) {
                const uint64_t t = wave_sum_u64(acc[q][lane]);
                if (lane == 0 && t) atomic_add_u64(b.out[q], t);
            }
        }
    }
}

template <int BLOCK, int IPT>
static hipError_t shared_t(const LaunchCfg &cfg_in, const BatchDev &b_in, int32_t *status, hipStream_t s) {
    using T = TileShape<BLOCK, IPT>;
    BatchDev b = b_in;
    const int64_t rows = b.row_end - b.row_begin;
    const int64_t n_tiles = (rows + T::ITEMS - 1) / T::ITEMS;
    LaunchCfg cfg = cfg_in;
    if (cfg.grid_per_cu <= 0) cfg.grid_per_cu = (2048 / BLOCK) > 0 ? (2048 / BLOCK) : 1;
    // LDS: the scalar accumulators, then, in join order, every join's mask
    // table (plus one zero word) that still fits without dropping below 8
    // waves per CU
    const int64_t acc_words32 = b.plan.scalar ? (int64_t)b.n_queries * kWave * 2 : 0;
    const int64_t min_blocks = (8 * kWave + BLOCK - 1) / BLOCK;
    int64_t words32 = acc_words32;
    for (int j = 0; j < CRYSTAL_MAX_JOINS; ++j) {
        MaskDev &md = b.mask[j];
        md.stage_off = 0;
        md.stage_words = 0;
        if (j >= b.plan.n_joins) continue;
        // a ranked table starts at an even word (its directory is read 64
        // bits at a time) and carries its own zero entries; a plain one is
        // followed by one zero word
        const bool ranked = md.ranked > 0;
        const int64_t w = ranked ? qmask_ranked_words(md.span, md.ranked) : (md.span + 1) / 2;
        const int64_t at = ranked ? (words32 + 1) & ~int64_t(1) : words32;
        const int64_t bytes = (at + w + 1) * 4;
        if (bytes + 1024 > device_lds_per_block() || device_lds_per_cu() / (bytes + 1024) < min_blocks) continue;
        md.stage_off = at;
        md.stage_words = w;
        words32 = at + w + 1;
    }
    // the per-wave queues of sparse rows, when the plan has steps after the
    // two dense ones, rows fit in 32 bits and the LDS has room
    b.queue_off = -1;
    const int64_t qwords = (int64_t)T::WAVES * 2 * kQueueCap;
    if (b.plan.n_preds + b.plan.n_joins > 2 && b.plan.n_rows <= (int64_t)UINT32_MAX &&
        (words32 + qwords) * 4 + 1024 <= device_lds_per_block()) {
        b.queue_off = words32;
        words32 += qwords;
    }
    const int64_t lds_bytes = words32 * 4;
    const size_t lds = (size_t)lds_bytes;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void *)shared_scan_kernel<BLOCK, IPT>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    // persistent workgroups: no more per CU than are resident at once
    // (registers and LDS permitting)
    int64_t fit = 0;
    hipError_t e = resident_per_cu((const void *)shared_scan_kernel<BLOCK, IPT>, BLOCK, lds_bytes, fit);
    if (e != hipSuccess) return e;
    if (fit < 1) fit = 1;
    if (cfg.grid_per_cu > fit) cfg.grid_per_cu = (int)fit;
    const int64_t grid = grid_for(n_tiles, cfg);
    if (grid == 0) return hipSuccess;
    hipLaunchKernelGGL((shared_scan_kernel<BLOCK, IPT>), dim3((unsigned)grid), dim3(BLOCK), lds, s, b, status,
                       n_tiles);
    return hipGetLastError();
}

hipError_t launch_shared_scan(const LaunchCfg &cfg, const BatchDev &b, int32_t *status, hipStream_t s) {
    if (b.row_end <= b.row_begin || b.n_queries == 0) return hipSuccess;
    switch (CRYSTAL_VARIANT_KEY(cfg.block, cfg.ipt)) {
#define X(B, I) case CRYSTAL_VARIANT_KEY(B, I): return shared_t<B, I>(cfg, b, status, s);
        CRYSTAL_VARIANTS_VEC(X)
#undef X
    default: return hipErrorInvalidValue;
    }
}

}  // namespace crystal
