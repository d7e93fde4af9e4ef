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
__device__ __forceinline__ int shared_step_col(const StarPlanDev &p, int s) {
    return s < p.n_preds ? p.pred_col[s] : p.joins[s - p.n_preds].fk_col;
}

// Group index of one surviving row from the template's dimension payloads.
__device__ __forceinline__ int64_t shared_group(const StarPlanDev &p, int64_t row) {
    int64_t g = 0;
    for (int jj = 0; jj < p.n_joins; ++jj) {
        const StarJoinDev &j = p.joins[jj];
        if (j.g_bits == 0) continue;
        const int32_t key = p.cols[j.fk_col][row];
        int32_t pay = 0;
        if (j.kind == CRYSTAL_HT_DIRECT) {
            const uint32_t off = (uint32_t)key - (uint32_t)j.key_min;
            if ((int64_t)off < j.span && j.payload) pay = j.payload[off];
        } else if (key != kEmptyKey) {
            probe_linear((const v2i *)j.slots, j.mask, j.shift, key, pay);
        }
        g += ((int64_t)payload_field(pay, j.g_shift, j.g_mask, j.g_bits) - (int64_t)j.g_base) * j.g_stride;
    }
    return g;
}

template <int BLOCK, int IPT>
__global__ __launch_bounds__(BLOCK) void shared_scan_kernel(const BatchDev b, int32_t *status, int64_t n_tiles) {
    using T = TileShape<BLOCK, IPT>;
    __shared__ uint64_t acc[kMaxBatch];
    const StarPlanDev &p = b.plan;
    const int n_steps = p.n_preds + p.n_joins;
    if (p.scalar) {
        if (threadIdx.x < kMaxBatch) acc[threadIdx.x] = 0;
        __syncthreads();
    }
    bool bad_group = false;
    for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const int64_t base = b.row_begin + tile * T::ITEMS;
        const uint32_t valid = valid_mask<BLOCK, IPT>(base, b.row_end);
        uint32_t qm[IPT];
#pragma unroll
        for (int k = 0; k < IPT; ++k) qm[k] = ((valid >> k) & 1u) ? b.all_queries : 0u;
        int32_t v[IPT];
        for (int s = 0; s < n_steps; ++s) {
            uint32_t any = 0;
#pragma unroll
            for (int k = 0; k < IPT; ++k) any |= (uint32_t)(qm[k] != 0u) << k;
            const int col = shared_step_col(p, s);
            if (s == 0) {
                block_load<BLOCK, IPT, true>(p.cols[col], base, b.row_end, v);
            } else {
                if (ballot(any != 0u) == 0) break;
                block_load_sel<BLOCK, IPT, true>(p.cols[col], base, b.row_end, any, v);
            }
            if (s < p.n_preds) {
#pragma unroll
                for (int k = 0; k < IPT; ++k) {
                    uint32_t m = 0;
                    for (int q = 0; q < b.n_queries; ++q)
                        m |= (uint32_t)in_range(v[k], b.pred_lo[q][s], b.pred_hi[q][s]) << q;
                    qm[k] &= m;
                }
            } else {
                const int j = s - p.n_preds;
                const uint16_t *mt = b.mask[j];
                const uint32_t last = (uint32_t)(b.mask_span[j] - 1);
                const int32_t kmin = b.mask_kmin[j];
#pragma unroll
                for (int k = 0; k < IPT; ++k) {
                    const uint32_t off = (uint32_t)v[k] - (uint32_t)kmin;
                    const bool in = qm[k] != 0u && off <= last;
                    qm[k] &= in ? (uint32_t)mt[off] : 0u;
                }
            }
        }
        // survivors: group index and measure once, then every query that kept the row
#pragma unroll
        for (int k = 0; k < IPT; ++k) {
            uint32_t m = qm[k];
            if (!m) continue;
            const int64_t row = T::index(base, k / T::VEC, k % T::VEC);
            const int64_t g = p.scalar ? 0 : shared_group(p, row);
            uint64_t val = 1;
            if (p.agg != CRYSTAL_AGG_COUNT) {
                const int64_t a = p.cols[p.agg_col0][row];
                if (p.agg == CRYSTAL_AGG_SUM) {
                    val = (uint64_t)a;
                } else {
                    const int64_t c = p.cols[p.agg_col1][row];
                    val = p.agg == CRYSTAL_AGG_SUM_PRODUCT ? (uint64_t)(a * c) : (uint64_t)(a - c);
                }
            }
            if (!p.scalar && (uint64_t)g >= (uint64_t)p.n_groups) {
                bad_group = true;
                continue;
            }
            while (m) {
                const int q = __builtin_ctz(m);
                m &= m - 1u;
                if (p.scalar)
                    atomicAdd((unsigned long long *)&acc[q], (unsigned long long)val);
                else
                    atomic_add_u64(b.out[q] + g, val);
            }
        }
    }
    if (bad_group) set_status(status, CRYSTAL_ERANGE);
    if (p.scalar) {
        __syncthreads();
        if (threadIdx.x < b.n_queries && acc[threadIdx.x]) atomic_add_u64(b.out[threadIdx.x], acc[threadIdx.x]);
    }
}

template <int BLOCK, int IPT>
static hipError_t shared_t(const LaunchCfg &cfg_in, const BatchDev &b, int32_t *status, hipStream_t s) {
    using T = TileShape<BLOCK, IPT>;
    const int64_t rows = b.row_end - b.row_begin;
    const int64_t n_tiles = (rows + T::ITEMS - 1) / T::ITEMS;
    LaunchCfg cfg = cfg_in;
    if (cfg.grid_per_cu <= 0) cfg.grid_per_cu = (2048 / BLOCK) > 0 ? (2048 / BLOCK) : 1;
    const int64_t grid = grid_for(n_tiles, cfg);
    if (grid == 0) return hipSuccess;
    hipLaunchKernelGGL((shared_scan_kernel<BLOCK, IPT>), dim3((unsigned)grid), dim3(BLOCK), 0, s, b, status,
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
