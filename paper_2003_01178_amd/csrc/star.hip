// Fused star-query kernel: the pipelined multi-join probe of the section 5.3
// case study, and the fact-side selection of SSB Q1.1 (section 3.1), in one
// launch with nothing materialised between operators.
#include "block.hpp"
#include "internal.hpp"
#include "variants.hpp"

namespace crystal {

__device__ __forceinline__ bool star_probe(const StarJoinDev &j, int32_t key, int32_t &payload,
                                           bool want_payload) {
    if (j.kind == CRYSTAL_HT_DIRECT) {
        const uint32_t off = (uint32_t)key - (uint32_t)j.key_min;
        if ((int64_t)off >= j.span) return false;
        const bool hit = (j.bitmap[off >> 5] >> (off & 31u)) & 1u;
        if (hit && want_payload) payload = j.payload[off];
        return hit;
    }
    if (key == kEmptyKey) return false;
    return probe_linear((const v2i *)j.slots, j.mask, j.shift, key, payload);
}

// One join step over the tile: BlockProbeHT on every live item, then the
// dimension predicate on the payload field when the plan has one.
template <int IPT>
__device__ __forceinline__ uint32_t star_join_step(const StarJoinDev &j, const int32_t (&key)[IPT],
                                                   uint32_t alive) {
    if (j.kind == CRYSTAL_HT_DIRECT && j.f_bits == 0) {
        // presence only: issue every bitmap load before testing any bit
        uint32_t word[IPT];
        uint32_t inspan = 0;
#pragma unroll
        for (int k = 0; k < IPT; ++k) {
            const uint32_t off = (uint32_t)key[k] - (uint32_t)j.key_min;
            const bool ok = ((alive >> k) & 1u) && (int64_t)off < j.span;
            inspan |= (uint32_t)ok << k;
            word[k] = ok ? j.bitmap[off >> 5] : 0u;
        }
        uint32_t hit = 0;
#pragma unroll
        for (int k = 0; k < IPT; ++k) {
            const uint32_t off = (uint32_t)key[k] - (uint32_t)j.key_min;
            hit |= ((word[k] >> (off & 31u)) & 1u) << k;
        }
        return alive & inspan & hit;
    }
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
        if (!((alive >> k) & 1u)) continue;
        int32_t pay = 0;
        bool hit = star_probe(j, key[k], pay, j.f_bits > 0);
        if (hit && j.f_bits > 0)
            hit = in_range(payload_field(pay, j.f_shift, j.f_mask, j.f_bits), j.f_lo, j.f_hi);
        if (!hit) alive &= ~(1u << k);
    }
    return alive;
}

template <int BLOCK, int IPT>
__global__ __launch_bounds__(BLOCK) void star_kernel(const StarPlanDev p, uint64_t *__restrict__ out,
                                                     int32_t *status, int64_t n_tiles) {
    using T = TileShape<BLOCK, IPT>;
    __shared__ uint64_t red[T::WAVES];
    const int n_steps = p.n_preds + p.n_joins;
    uint64_t scalar_acc = 0;
    bool bad_group = false;

    for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const int64_t base = tile * T::ITEMS;
        uint32_t alive = valid_mask<BLOCK, IPT>(base, p.n_rows);
        int32_t v[IPT];

        // select / probe pipeline: the first column in full, the rest selectively
        for (int s = 0; s < n_steps; ++s) {
            const bool is_pred = s < p.n_preds;
            const int col = is_pred ? p.pred_col[s] : p.joins[s - p.n_preds].fk_col;
            if (s == 0)
                block_load<BLOCK, IPT, true>(p.cols[col], base, p.n_rows, v);
            else
                block_load_sel<BLOCK, IPT, true>(p.cols[col], base, p.n_rows, alive, v);
            if (is_pred)
                alive = block_pred_range<IPT>(v, alive, p.pred_lo[s], p.pred_hi[s]);
            else
                alive = star_join_step<IPT>(p.joins[s - p.n_preds], v, alive);
        }
        if (!alive) continue;

        // survivors: group index from the dimension payloads, then the measure
        int64_t grp[IPT];
#pragma unroll
        for (int k = 0; k < IPT; ++k) grp[k] = 0;
        if (!p.scalar) {
            for (int jj = 0; jj < p.n_joins; ++jj) {
                const StarJoinDev &j = p.joins[jj];
                if (j.g_bits == 0) continue;
                block_load_sel<BLOCK, IPT, false>(p.cols[j.fk_col], base, p.n_rows, alive, v);
#pragma unroll
                for (int k = 0; k < IPT; ++k) {
                    if (!((alive >> k) & 1u)) continue;
                    int32_t pay = 0;
                    star_probe(j, v[k], pay, true);
                    const int32_t f = payload_field(pay, j.g_shift, j.g_mask, j.g_bits);
                    grp[k] += ((int64_t)f - (int64_t)j.g_base) * j.g_stride;
                }
            }
        }
        int32_t a[IPT], b[IPT];
        if (p.agg != CRYSTAL_AGG_COUNT)
            block_load_sel<BLOCK, IPT, false>(p.cols[p.agg_col0], base, p.n_rows, alive, a);
        if (p.agg == CRYSTAL_AGG_SUM_PRODUCT || p.agg == CRYSTAL_AGG_SUM_DIFF)
            block_load_sel<BLOCK, IPT, false>(p.cols[p.agg_col1], base, p.n_rows, alive, b);
#pragma unroll
        for (int k = 0; k < IPT; ++k) {
            if (!((alive >> k) & 1u)) continue;
            uint64_t val;
            switch (p.agg) {
            case CRYSTAL_AGG_SUM: val = (uint64_t)(int64_t)a[k]; break;
            case CRYSTAL_AGG_SUM_PRODUCT: val = (uint64_t)((int64_t)a[k] * (int64_t)b[k]); break;
            case CRYSTAL_AGG_SUM_DIFF: val = (uint64_t)((int64_t)a[k] - (int64_t)b[k]); break;
            default: val = 1; break;
            }
            if (p.scalar) {
                scalar_acc += val;
            } else if ((uint64_t)grp[k] < (uint64_t)p.n_groups) {
                atomic_add_u64(out + grp[k], val);
            } else {
                bad_group = true;
            }
        }
    }
    if (bad_group) set_status(status, CRYSTAL_ERANGE);
    if (p.scalar) {
        const uint64_t t = block_sum_u64<BLOCK>(scalar_acc, red);
        if (threadIdx.x == 0 && t) atomic_add_u64(out, t);
    }
}

template <int BLOCK, int IPT>
static hipError_t star_t(const LaunchCfg &cfg, const StarPlanDev &p, uint64_t *out,
                         int32_t *status, hipStream_t s) {
    using T = TileShape<BLOCK, IPT>;
    const int64_t n_tiles = (p.n_rows + T::ITEMS - 1) / T::ITEMS;
    const int64_t grid = grid_for(n_tiles, cfg);
    if (grid == 0) return hipSuccess;
    hipLaunchKernelGGL((star_kernel<BLOCK, IPT>), dim3((unsigned)grid), dim3(BLOCK), 0, s, p, out,
                       status, n_tiles);
    return hipGetLastError();
}

hipError_t launch_star(const LaunchCfg &cfg, const StarPlanDev &plan, uint64_t *out,
                       int32_t *status, hipStream_t s) {
    hipError_t e = fill_u64(out, plan.n_groups, 0ull, s);
    if (e != hipSuccess || plan.n_rows == 0) return e;
    switch (CRYSTAL_VARIANT_KEY(cfg.block, cfg.ipt)) {
#define X(B, I) case CRYSTAL_VARIANT_KEY(B, I): return star_t<B, I>(cfg, plan, out, status, s);
        CRYSTAL_VARIANTS_VEC(X)
#undef X
    default: return hipErrorInvalidValue;
    }
}

}  // namespace crystal
