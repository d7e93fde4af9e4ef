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
// qmask_build_kernel).  So a join costs one 2-byte lookup per row however many
// queries share the pass.  Survivors form their group index from the
// template's dimension payloads once, then add the measure to every query
// whose bit is set: grouped results with 64-bit atomics into the query's own
// output, scalar results through per-workgroup LDS partials.
//
// Outputs are accumulated, never cleared here: a query admitted into a batch
// can be answered over several launches that cover successive row ranges.
#include "block.hpp"
#include "internal.hpp"
#include "variants.hpp"

namespace crystal {

// ------------------------------------------------------------ mask tables --
// mask[key - key_min] |= bit q for every query q whose range holds the row's
// filter attribute.  Two 16-bit entries share a 32-bit word, set with atomicOr.
__global__ __launch_bounds__(256) void qmask_build_kernel(uint32_t *__restrict__ words, int64_t span,
                                                          int32_t key_min, const int32_t *__restrict__ keys,
                                                          const int32_t *__restrict__ filter_col, int64_t n,
                                                          QmaskRanges r, int32_t *status) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint32_t off = (uint32_t)keys[i] - (uint32_t)key_min;
        if ((int64_t)off >= span) {
            set_status(status, CRYSTAL_ERANGE);
            continue;
        }
        const int32_t f = filter_col ? filter_col[i] : 0;
        uint32_t m = 0;
        for (int q = 0; q < r.n; ++q)
            m |= (uint32_t)(filter_col ? in_range(f, r.lo[q], r.hi[q]) : true) << q;
        if (m) atomicOr(words + (off >> 1), m << ((off & 1u) * 16u));
    }
}

hipError_t launch_qmask_build(uint16_t *table, int64_t span, int32_t key_min, const int32_t *keys,
                              const int32_t *filter_col, int64_t n, const QmaskRanges &r, int32_t *status,
                              hipStream_t s) {
    hipError_t e = fill_u32((uint32_t *)table, (span + 1) / 2, 0u, s);
    if (e != hipSuccess || n == 0) return e;
    int64_t grid = (n + 255) / 256;
    const int64_t cap = (int64_t)device_cu_count() * 16;
    if (grid > cap) grid = cap;
    hipLaunchKernelGGL(qmask_build_kernel, dim3((unsigned)grid), dim3(256), 0, s, (uint32_t *)table, span, key_min,
                       keys, filter_col, n, r, status);
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

__device__ __forceinline__ int shared_step_col(const StarPlanDev &p, int s) {
    return s < p.n_preds ? p.pred_col[s] : p.joins[s - p.n_preds].fk_col;
}

template <int BLOCK, int IPT>
__global__ __launch_bounds__(BLOCK) void shared_scan_kernel(const BatchDev b, int32_t *status, int64_t n_tiles) {
    using T = TileShape<BLOCK, IPT>;
    // scalar results: one private LDS accumulator per (query, thread), so that
    // adds never contend; reduced once per workgroup at the end
    // dynamic LDS: b.n_queries * BLOCK words for a scalar plan, then the
    // staged mask tables (see BatchDev::stage_off)
    extern __shared__ uint64_t dyn[];
    uint64_t(*acc)[BLOCK] = reinterpret_cast<uint64_t(*)[BLOCK]>(dyn);
    uint32_t *lds_words = reinterpret_cast<uint32_t *>(dyn);
    __shared__ uint64_t red[BLOCK / kWave];
    const StarPlanDev &p = b.plan;
    const int n_steps = p.n_preds + p.n_joins;
    if (p.scalar) {
        for (int q = 0; q < b.n_queries; ++q) acc[q][threadIdx.x] = 0;
    }
    bool any_staged = false;
    for (int j = 0; j < p.n_joins; ++j) {
        if (b.stage_words[j] == 0) continue;
        any_staged = true;
        const uint32_t *src = reinterpret_cast<const uint32_t *>(b.mask[j]);
        uint32_t *dst = lds_words + b.stage_off[j];
        for (int64_t i = threadIdx.x; i < b.stage_words[j]; i += BLOCK) dst[i] = src[i];
        if (threadIdx.x == 0) dst[b.stage_words[j]] = 0u;  // entries past the table read 0
    }
    if (any_staged) __syncthreads();
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
            const int j = s - p.n_preds;
            const uint32_t last = (uint32_t)(b.mask_span[j] - 1);
            const int32_t kmin = b.mask_kmin[j];
            if (b.stage_words[j] > 0) {
                // LDS-typed path (a pointer that may also address global
                // memory would compile to flat loads).  Keys outside the
                // table are clamped to the zero entry after it, so no range
                // test is needed.
                const uint16_t *stage = reinterpret_cast<const uint16_t *>(lds_words + b.stage_off[j]);
                const uint32_t span = last + 1u;
#pragma unroll
                for (int k = 0; k < IPT; ++k) {
                    const uint32_t off = (uint32_t)x[k] - (uint32_t)kmin;
                    qm[k] &= (uint32_t)stage[off < span ? off : span];
                }
            } else {
                const uint16_t *mt = b.mask[j];
#pragma unroll
                for (int k = 0; k < IPT; ++k) {
                    const uint32_t off = (uint32_t)x[k] - (uint32_t)kmin;
                    const bool in = qm[k] != 0u && off <= last;
                    qm[k] &= in ? (uint32_t)mt[off] : 0u;
                }
            }
        }
    };

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
        int32_t w[IPT];
        if (n_steps > 1) block_load<BLOCK, IPT, true>(p.col[shared_step_col(p, 1)].p, base, b.row_end, w);
        const int64_t tn = tile + gridDim.x;
        if (n_steps > 0 && tn < n_tiles)
            block_load<BLOCK, IPT, true>(p.col[col0].p, b.row_begin + tn * T::ITEMS, b.row_end, nxt);
        if (n_steps > 0) apply_step(0, cur);
        if (n_steps > 1) apply_step(1, w);
        for (int s = 2; s < n_steps; ++s) {
            uint32_t any = 0;
#pragma unroll
            for (int k = 0; k < IPT; ++k) any |= (uint32_t)(qm[k] != 0u) << k;
            if (ballot(any != 0u) == 0) break;
            block_load_sel<BLOCK, IPT, true>(p.col[shared_step_col(p, s)].p, base, b.row_end, any, w);
            apply_step(s, w);
        }
        // survivors: the measure and group index once per row, then every query
        // that kept the row.  A vector of VEC rows is handled at a time: its
        // loads (measures, then group keys, then their payloads) are issued
        // together whenever one of its rows survives, so a vector pays one
        // memory round trip per load step instead of one per surviving row,
        // and only one vector's values are live at a time.
        uint32_t surv = 0;
#pragma unroll
        for (int k = 0; k < IPT; ++k) surv |= (uint32_t)(qm[k] != 0u) << k;
        if (ballot(surv != 0u) == 0) return;
#pragma unroll
        for (int ch = 0; ch < T::CHUNKS; ++ch) {
            const uint32_t sc = (surv >> (ch * T::VEC)) & T::VMASK;
            if (ballot(sc != 0u) == 0) continue;
            const int64_t row0 = T::index(base, ch, 0);
            int32_t a[T::VEC], c[T::VEC];
            int64_t g[T::VEC];
#pragma unroll
            for (int e = 0; e < T::VEC; ++e) g[e] = 0;
            if (p.agg != CRYSTAL_AGG_COUNT) load_vec_sel<T::VEC>(p.col[p.agg_col0].p, row0, b.row_end, sc, a);
            if (p.agg == CRYSTAL_AGG_SUM_PRODUCT || p.agg == CRYSTAL_AGG_SUM_DIFF)
                load_vec_sel<T::VEC>(p.col[p.agg_col1].p, row0, b.row_end, sc, c);
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
#pragma unroll
            for (int e = 0; e < T::VEC; ++e) {
                uint32_t m = qm[ch * T::VEC + e];
                if (!m) continue;
                uint64_t val = 1;
                if (p.agg == CRYSTAL_AGG_SUM)
                    val = (uint64_t)(int64_t)a[e];
                else if (p.agg == CRYSTAL_AGG_SUM_PRODUCT)
                    val = (uint64_t)((int64_t)a[e] * (int64_t)c[e]);
                else if (p.agg == CRYSTAL_AGG_SUM_DIFF)
                    val = (uint64_t)((int64_t)a[e] - (int64_t)c[e]);
                if (!p.scalar && (uint64_t)g[e] >= (uint64_t)p.n_groups) {
                    bad_group = true;
                    continue;
                }
                while (m) {
                    const int q = __builtin_ctz(m);
                    m &= m - 1u;
                    if (p.scalar)  // private slot: an LDS add without return, no read-modify-write wait
                        __hip_atomic_fetch_add((__attribute__((address_space(3))) uint64_t *)&acc[q][threadIdx.x],
                                               val, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
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
    if (bad_group) set_status(status, CRYSTAL_ERANGE);
    if (p.scalar) {
        for (int q = 0; q < b.n_queries; ++q) {
            const uint64_t t = block_sum_u64<BLOCK>(acc[q][threadIdx.x], red);
            if (threadIdx.x == 0 && t) atomic_add_u64(b.out[q], t);
            __syncthreads();  // red is reused by the next query's sum
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
    const int64_t acc_words32 = b.plan.scalar ? (int64_t)b.n_queries * BLOCK * 2 : 0;
    const int64_t min_blocks = (8 * kWave + BLOCK - 1) / BLOCK;
    int64_t words32 = acc_words32;
    for (int j = 0; j < CRYSTAL_MAX_JOINS; ++j) {
        b.stage_off[j] = 0;
        b.stage_words[j] = 0;
        if (j >= b.plan.n_joins) continue;
        const int64_t w = (b.mask_span[j] + 1) / 2;
        const int64_t bytes = (words32 + w + 1) * 4;
        if (bytes + 1024 > device_lds_per_block() || device_lds_per_cu() / (bytes + 1024) < min_blocks) continue;
        b.stage_off[j] = words32;
        b.stage_words[j] = w;
        words32 += w + 1;
    }
    const int64_t lds_bytes = words32 * 4;
    if (words32 > acc_words32) {
        const int64_t fit = device_lds_per_cu() / (lds_bytes + 1024);
        if (cfg.grid_per_cu > fit) cfg.grid_per_cu = (int)fit;
    }
    const int64_t grid = grid_for(n_tiles, cfg);
    if (grid == 0) return hipSuccess;
    const size_t lds = (size_t)lds_bytes;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void *)shared_scan_kernel<BLOCK, IPT>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
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
