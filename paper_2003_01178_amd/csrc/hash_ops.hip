// Hash-join build and probe (section 4.3; perfect hashing of section 5.3)
// and the dense group-by aggregate.
#include "block.hpp"
#include "internal.hpp"
#include "variants.hpp"

namespace crystal {

static constexpr uint64_t kEmptySlot = (uint64_t)(uint32_t)kEmptyKey;  // {EMPTY, 0}

static inline int64_t direct_bitmap_words(int64_t span) {
    int64_t w = (span + 31) / 32;
    return (w + 63) / 64 * 64;
}

static DevTable to_dev(const crystal_ht &ht) {
    DevTable t = {};
    t.kind = ht.kind;
    t.has_payload = ht.has_payload;
    if (ht.kind == CRYSTAL_HT_DIRECT) {
        t.bitmap = (const uint32_t *)ht.mem;
        t.payload = ht.has_payload ? (const int32_t *)ht.mem + direct_bitmap_words(ht.capacity)
                                   : nullptr;
        t.span = ht.capacity;
        t.key_min = ht.key_min;
    } else {
        t.slots = (const v2i *)ht.mem;
        t.mask = (uint32_t)(ht.capacity - 1);
        t.shift = 32 - ht.log2_capacity;
    }
    return t;
}

hipError_t launch_ht_clear(const crystal_ht &ht, hipStream_t s) {
    if (ht.kind == CRYSTAL_HT_DIRECT)
        return fill_u32((uint32_t *)ht.mem, direct_bitmap_words(ht.capacity), 0u, s);
    return fill_u64((uint64_t *)ht.mem, ht.capacity, kEmptySlot, s);
}

// --------------------------------------------------------------- build ----
// One thread per build row: a 64-bit compare-and-swap claims an empty slot
// {EMPTY, 0} -> {key, payload} (linear probing), or an atomic OR sets the
// key's presence bit and the payload is stored (direct table).
template <int KIND>
__device__ __forceinline__ void build_row(const DevTable &t, const int32_t *__restrict__ keys,
                                          const int32_t *__restrict__ payload,
                                          const int32_t *__restrict__ filter_col, int32_t flo, int32_t fhi,
                                          int64_t i, int32_t *status) {
    if (filter_col && !in_range(filter_col[i], flo, fhi)) return;
    const int32_t k = keys[i];
    const int32_t v = payload ? payload[i] : 0;
    if constexpr (KIND == CRYSTAL_HT_DIRECT) {
        const uint32_t off = (uint32_t)k - (uint32_t)t.key_min;
        if ((int64_t)off >= t.span) {
            set_status(status, CRYSTAL_ERANGE);
            return;
        }
        const uint32_t bit = 1u << (off & 31u);
        const uint32_t old = atomicOr(const_cast<uint32_t *>(t.bitmap) + (off >> 5), bit);
        if (old & bit) {
            set_status(status, CRYSTAL_EDUPKEY);
            return;
        }
        if (t.payload) const_cast<int32_t *>(t.payload)[off] = v;
    } else {
        if (k == kEmptyKey) {
            set_status(status, CRYSTAL_EINVAL);
            return;
        }
        unsigned long long *slots = (unsigned long long *)const_cast<v2i *>(t.slots);
        const unsigned long long want = (unsigned long long)(uint32_t)k | ((unsigned long long)(uint32_t)v << 32);
        uint32_t sl = hash_slot(k, t.shift);
        for (uint32_t step = 0; step <= t.mask; ++step) {
            const unsigned long long old = atomicCAS(slots + sl, (unsigned long long)kEmptySlot, want);
            if (old == kEmptySlot) return;
            if ((int32_t)(uint32_t)old == k) {
                set_status(status, CRYSTAL_EDUPKEY);
                return;
            }
            sl = (sl + 1u) & t.mask;
        }
        set_status(status, CRYSTAL_EFULL);
    }
}

template <int KIND>
__global__ __launch_bounds__(256) void ht_build_kernel(DevTable t, const int32_t *__restrict__ keys,
                                                       const int32_t *__restrict__ payload,
                                                       const int32_t *__restrict__ filter_col,
                                                       int32_t flo, int32_t fhi, int64_t n,
                                                       int32_t *status) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        build_row<KIND>(t, keys, payload, filter_col, flo, fhi, i, status);
}

// ------------------------------------------------------------ batch build --
// Several tables in two launches: one clear of every table's memory, then
// one build kernel whose workgroups are split between the tables (a range of
// workgroups per table, each striding over that table's rows).
struct ClearRange {
    uint64_t *p;
    int64_t n;        // 64-bit words
    uint64_t value;
};

// up to kMaxBuildBatch tables, and one more range (an output to zero)
struct ClearBatch {
    int32_t count;
    ClearRange r[kMaxBuildBatch + 1];
};

// the clears, spread over `blocks` workgroups of which this is `block`
__device__ __forceinline__ void clear_part(const ClearBatch &b, int64_t block, int64_t blocks) {
    const int64_t stride = blocks * blockDim.x;
    const int64_t g0 = block * blockDim.x + threadIdx.x;
    for (int r = 0; r < b.count; ++r)
        for (int64_t i = g0; i < b.r[r].n; i += stride) b.r[r].p[i] = b.r[r].value;
}

__global__ __launch_bounds__(256) void clear_batch_kernel(ClearBatch b) {
    clear_part(b, blockIdx.x, gridDim.x);
}

// clear memory of a table, as crystal_ht_clear would leave it
ClearRange table_clear_range(const crystal_ht &ht) {
    ClearRange c;
    c.p = (uint64_t *)ht.mem;
    if (ht.kind == CRYSTAL_HT_DIRECT) {
        c.n = direct_bitmap_words(ht.capacity) / 2;  // an even number of 32-bit words
        c.value = 0;
    } else {
        c.n = ht.capacity;
        c.value = kEmptySlot;
    }
    return c;
}

struct BuildItemDev {
    DevTable t;
    const int32_t *keys;
    const int32_t *payload;
    const int32_t *filter;
    int32_t flo, fhi;
    int64_t n;
    int64_t block0, blocks;
};

struct BuildBatch {
    int32_t count;
    BuildItemDev it[kMaxBuildBatch];
};

// workgroup `block` of the build part: its item's range of workgroups strides over that item's rows
__device__ __forceinline__ void build_part(const BuildBatch &b, int64_t block, int32_t *status) {
    int r = 0;
    while (r + 1 < b.count && block >= b.it[r + 1].block0) ++r;
    const BuildItemDev &it = b.it[r];
    const int64_t stride = it.blocks * blockDim.x;
    for (int64_t i = (block - it.block0) * blockDim.x + threadIdx.x; i < it.n; i += stride) {
        if (it.t.kind == CRYSTAL_HT_DIRECT)
            build_row<CRYSTAL_HT_DIRECT>(it.t, it.keys, it.payload, it.filter, it.flo, it.fhi, i, status);
        else
            build_row<CRYSTAL_HT_LINEAR>(it.t, it.keys, it.payload, it.filter, it.flo, it.fhi, i, status);
    }
}

__global__ __launch_bounds__(256) void build_batch_kernel(BuildBatch b, int32_t *status) {
    build_part(b, blockIdx.x, status);
}

// Builds into tables that are already clear, and, in other workgroups of the
// same launch, clears of memory no build touches: the first build_blocks
// workgroups build, the rest clear.
__global__ __launch_bounds__(256) void build_clear_kernel(BuildBatch b, ClearBatch c, int64_t build_blocks,
                                                          int32_t *status) {
    const int64_t block = blockIdx.x;
    if (block < build_blocks)
        build_part(b, block, status);
    else
        clear_part(c, block - build_blocks, (int64_t)gridDim.x - build_blocks);
}

// build items of a batch with their workgroup ranges; returns the workgroups used
static int64_t fill_build_batch(const crystal_ht_build_item *items, int n_items, BuildBatch &bb) {
    int64_t blocks = 0;
    const int64_t cap = (int64_t)device_cu_count() * 32;
    for (int i = 0; i < n_items; ++i) {
        if (items[i].n == 0) continue;
        const crystal_ht &ht = *items[i].ht;
        BuildItemDev &d = bb.it[bb.count++];
        d.t = to_dev(ht);
        d.keys = items[i].keys;
        d.payload = ht.has_payload ? items[i].payload : nullptr;
        d.filter = items[i].filter_col;
        d.flo = items[i].filter.lo;
        d.fhi = items[i].filter.hi;
        d.n = items[i].n;
        int64_t nb = (items[i].n + 255) / 256;
        if (nb > cap) nb = cap;
        d.block0 = blocks;
        d.blocks = nb;
        blocks += nb;
    }
    return blocks;
}

// workgroups for clearing `words` 64-bit words at most per range
static int64_t clear_grid(int64_t words) {
    const int64_t cap = (int64_t)device_cu_count() * 32;
    int64_t g = (words + 255) / 256;
    if (g > cap) g = cap;
    return g < 1 ? 1 : g;
}

hipError_t launch_ht_build_batch(const crystal_ht_build_item *items, int n_items, int32_t *status,
                                 hipStream_t s) {
    ClearBatch cb = {};
    BuildBatch bb = {};
    int64_t clear_words = 0;
    for (int i = 0; i < n_items; ++i) {
        ClearRange &c = cb.r[cb.count++];
        c = table_clear_range(*items[i].ht);
        clear_words = c.n > clear_words ? c.n : clear_words;
    }
    if (cb.count == 0) return hipSuccess;
    const int64_t blocks = fill_build_batch(items, n_items, bb);
    hipLaunchKernelGGL(clear_batch_kernel, dim3((unsigned)clear_grid(clear_words)), dim3(256), 0, s, cb);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || bb.count == 0) return e;
    hipLaunchKernelGGL(build_batch_kernel, dim3((unsigned)blocks), dim3(256), 0, s, bb, status);
    return hipGetLastError();
}

hipError_t launch_ht_build_batch_fused(const crystal_ht_build_item *items, int n_items, const crystal_ht *const *clear,
                                       int n_clear, int64_t *zero, int64_t zero_n, int32_t *status, hipStream_t s) {
    ClearBatch cb = {};
    BuildBatch bb = {};
    int64_t clear_words = 0;
    for (int i = 0; i < n_clear; ++i) {
        ClearRange &c = cb.r[cb.count++];
        c = table_clear_range(*clear[i]);
        clear_words = c.n > clear_words ? c.n : clear_words;
    }
    if (zero_n > 0) {
        ClearRange &c = cb.r[cb.count++];
        c.p = (uint64_t *)zero;
        c.n = zero_n;
        c.value = 0;
        clear_words = c.n > clear_words ? c.n : clear_words;
    }
    const int64_t build_blocks = fill_build_batch(items, n_items, bb);
    const int64_t clear_blocks = cb.count ? clear_grid(clear_words) : 0;
    if (build_blocks + clear_blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(build_clear_kernel, dim3((unsigned)(build_blocks + clear_blocks)), dim3(256), 0, s, bb, cb,
                       build_blocks, status);
    return hipGetLastError();
}

hipError_t launch_ht_build(const crystal_ht &ht, const int32_t *keys, const int32_t *payload,
                           const int32_t *filter_col, int32_t flo, int32_t fhi, int64_t n,
                           int32_t *status, hipStream_t s) {
    hipError_t e = launch_ht_clear(ht, s);
    if (e != hipSuccess || n == 0) return e;
    const DevTable t = to_dev(ht);
    int64_t grid = (n + 255) / 256;
    const int64_t cap = (int64_t)device_cu_count() * 32;
    if (grid > cap) grid = cap;
    if (ht.kind == CRYSTAL_HT_DIRECT)
        hipLaunchKernelGGL(ht_build_kernel<CRYSTAL_HT_DIRECT>, dim3((unsigned)grid), dim3(256), 0, s,
                           t, keys, payload, filter_col, flo, fhi, n, status);
    else
        hipLaunchKernelGGL(ht_build_kernel<CRYSTAL_HT_LINEAR>, dim3((unsigned)grid), dim3(256), 0, s,
                           t, keys, payload, filter_col, flo, fhi, n, status);
    return hipGetLastError();
}

// A tile's probe keys (and probe payloads) in registers.
template <int IPT, bool PP>
struct ProbeRegs {
    int32_t key[IPT];
    int32_t pv[PP ? IPT : 1];
};

// --------------------------------------------------------------- probe ----
// Query Q4: BlockLoad a tile of probe keys (and probe payloads), probe every
// item, keep a per-thread sum and match count, BlockAggregate, and add the
// workgroup's totals with two 64-bit atomics.  MODE 0: linear probing in
// global memory; MODE 1: linear probing in a copy of the table staged in LDS
// once per workgroup; MODE 2: direct table.  PP: probe rows carry a payload
// (pp is not null), a separate instance so that the payload registers exist
// only when used.
template <int BLOCK, int IPT, int MODE, bool PP>
__global__ __launch_bounds__(BLOCK) void ht_probe_kernel(DevTable t, const int32_t *__restrict__ fk,
                                                         const int32_t *__restrict__ pp, int64_t n,
                                                         uint64_t *__restrict__ out_sum,
                                                         uint64_t *__restrict__ out_cnt,
                                                         int64_t n_tiles) {
    using T = TileShape<BLOCK, IPT>;
    extern __shared__ v4i lds_raw[];
    __shared__ uint64_t red[T::WAVES];
    const v2i *slots = t.slots;
    if constexpr (MODE == 1) {
        // stage the whole table: capacity * 8 bytes, 16 bytes per load
        const int64_t n16 = ((int64_t)t.mask + 1) / 2;
        const v4i *src = reinterpret_cast<const v4i *>(t.slots);
        for (int64_t i = threadIdx.x; i < n16; i += BLOCK) lds_raw[i] = src[i];
        __syncthreads();
        slots = reinterpret_cast<const v2i *>(lds_raw);
    }
    uint64_t sum = 0, cnt = 0;
    // one tile: the probes of its (already loaded) keys
    auto probe_tile = [&](int64_t tile, const ProbeRegs<IPT, PP> &r) {
        const int32_t(&key)[IPT] = r.key;
        const int64_t base = tile * T::ITEMS;
        const uint32_t valid = valid_mask<BLOCK, IPT>(base, n);
        uint32_t hit = 0;
        int32_t pay[IPT];
        if constexpr (MODE == 2) {
            // direct table: every item's presence word at once, then the payloads of the hits
            uint32_t word[IPT], ok = 0;
#pragma unroll
            for (int k = 0; k < IPT; ++k) {
                const uint32_t off = (uint32_t)key[k] - (uint32_t)t.key_min;
                const bool in = ((valid >> k) & 1u) && (int64_t)off < t.span;
                ok |= (uint32_t)in << k;
                word[k] = t.bitmap[in ? (off >> 5) : 0u];
            }
#pragma unroll
            for (int k = 0; k < IPT; ++k) {
                const uint32_t off = (uint32_t)key[k] - (uint32_t)t.key_min;
                hit |= (((word[k] >> (off & 31u)) & 1u) << k) & ok;
            }
#pragma unroll
            for (int k = 0; k < IPT; ++k) {
                const uint32_t off = (uint32_t)key[k] - (uint32_t)t.key_min;
                pay[k] = t.has_payload && ((hit >> k) & 1u) ? t.payload[off] : 0;
            }
        } else if constexpr (MODE == 0) {
            // table in global memory: one probe sequence per item (issuing every
            // item's slot at once measured slower when the table sits in the
            // last-level cache, and no faster from HBM)
#pragma unroll
            for (int k = 0; k < IPT; ++k) {
                pay[k] = 0;
                if (((valid >> k) & 1u) && key[k] != kEmptyKey && probe_linear(slots, t.mask, t.shift, key[k], pay[k]))
                    hit |= 1u << k;
            }
        } else {
            // table staged in LDS: every item's home slot is read at once and
            // compared without branches; only items whose home slot holds
            // another key continue, in rounds that read the next slot of every
            // item still searching at once (at fill rate 1/2 most items end in
            // the first round)
            uint32_t slot[IPT];
            uint32_t pending = 0;
            {
                v2i e[IPT];
#pragma unroll
                for (int k = 0; k < IPT; ++k) {
                    slot[k] = hash_slot(key[k], t.shift);
                    e[k] = slots[slot[k]];
                }
#pragma unroll
                for (int k = 0; k < IPT; ++k) {
                    const bool ok = ((valid >> k) & 1u) && key[k] != kEmptyKey;
                    const bool h = ok && e[k].x == key[k];
                    hit |= (uint32_t)h << k;
                    pay[k] = h ? e[k].y : 0;
                    pending |= (uint32_t)(ok && !h && e[k].x != kEmptyKey) << k;
                }
            }
            if (pending) {
#pragma unroll
                for (int k = 0; k < IPT; ++k) slot[k] = (slot[k] + 1u) & t.mask;
                for (uint32_t step = 1; pending && step <= t.mask; ++step) {
                    v2i e[IPT];
#pragma unroll
                    for (int k = 0; k < IPT; ++k)
                        if ((pending >> k) & 1u) e[k] = slots[slot[k]];
#pragma unroll
                    for (int k = 0; k < IPT; ++k) {
                        if (!((pending >> k) & 1u)) continue;
                        if (e[k].x == key[k]) {
                            hit |= 1u << k;
                            pay[k] = e[k].y;
                            pending &= ~(1u << k);
                        } else if (e[k].x == kEmptyKey) {
                            pending &= ~(1u << k);
                        } else {
                            slot[k] = (slot[k] + 1u) & t.mask;
                        }
                    }
                }
            }
        }
        if constexpr (MODE == 1) {
            // pay[k] is 0 for misses: the sum needs no per-item branch
#pragma unroll
            for (int k = 0; k < IPT; ++k) {
                sum += (uint64_t)(int64_t)pay[k];
                if constexpr (PP) sum += ((hit >> k) & 1u) ? (uint64_t)(int64_t)r.pv[k] : 0ull;
            }
            cnt += (uint64_t)__popc(hit);
            return;
        }
#pragma unroll
        for (int k = 0; k < IPT; ++k)
            if ((hit >> k) & 1u) {
                uint64_t add = (uint64_t)(int64_t)pay[k];
                if constexpr (PP) add += (uint64_t)(int64_t)r.pv[k];
                sum += add;
                cnt += 1;
            }
    };
    auto load = [&](int64_t tile, ProbeRegs<IPT, PP> &r) {
        block_load<BLOCK, IPT, true>(fk, tile * T::ITEMS, n, r.key);
        if constexpr (PP) block_load<BLOCK, IPT, true>(pp, tile * T::ITEMS, n, r.pv);
    };
    int64_t tile = blockIdx.x;
    if constexpr (PP) {
        // probe payloads too: one buffer (a second one would spill at 16 items per thread)
        ProbeRegs<IPT, PP> r;
        for (; tile < n_tiles; tile += gridDim.x) {
            load(tile, r);
            probe_tile(tile, r);
        }
    } else {
    // the next tile's keys are loaded while the current tile is probed, in
    // alternating register buffers so that a buffer receiving loads is never
    // copied
    ProbeRegs<IPT, PP> ra, rb;
    if (tile < n_tiles) load(tile, ra);
    while (tile < n_tiles) {
        int64_t nxt = tile + gridDim.x;
        if (nxt < n_tiles) load(nxt, rb);
        probe_tile(tile, ra);
        tile = nxt;
        if (tile >= n_tiles) break;
        nxt = tile + gridDim.x;
        if (nxt < n_tiles) load(nxt, ra);
        probe_tile(tile, rb);
        tile = nxt;
    }
    }
    const uint64_t bs = block_sum_u64<BLOCK>(sum, red);
    __syncthreads();
    const uint64_t bc = block_sum_u64<BLOCK>(cnt, red);
    if (threadIdx.x == 0) {
        if (bs) atomic_add_u64(out_sum, bs);
        if (bc) atomic_add_u64(out_cnt, bc);
    }
}

template <int BLOCK, int IPT, bool PP>
static hipError_t probe_launch(const crystal_ht &ht, const DevTable &t, bool stage, int64_t table_bytes,
                               int64_t grid, const int32_t *fk, const int32_t *pp, int64_t n, uint64_t *out,
                               uint64_t *cnt, int64_t n_tiles, hipStream_t s) {
    if (ht.kind == CRYSTAL_HT_DIRECT) {
        hipLaunchKernelGGL((ht_probe_kernel<BLOCK, IPT, 2, PP>), dim3((unsigned)grid), dim3(BLOCK), 0, s,
                           t, fk, pp, n, out, cnt, n_tiles);
    } else if (stage) {
        auto fn = ht_probe_kernel<BLOCK, IPT, 1, PP>;
        hipError_t e = hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)table_bytes);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(fn, dim3((unsigned)grid), dim3(BLOCK), (size_t)table_bytes, s, t, fk, pp, n,
                           out, cnt, n_tiles);
    } else {
        hipLaunchKernelGGL((ht_probe_kernel<BLOCK, IPT, 0, PP>), dim3((unsigned)grid), dim3(BLOCK), 0, s,
                           t, fk, pp, n, out, cnt, n_tiles);
    }
    return hipGetLastError();
}

template <int BLOCK, int IPT>
static hipError_t probe_t(const LaunchCfg &cfg_in, const crystal_ht &ht, const int32_t *fk,
                          const int32_t *pp, int64_t n, uint64_t *out, uint64_t *cnt, hipStream_t s) {
    using T = TileShape<BLOCK, IPT>;
    const int64_t n_tiles = (n + T::ITEMS - 1) / T::ITEMS;
    const DevTable t = to_dev(ht);
    LaunchCfg cfg = cfg_in;
    const int64_t table_bytes = ht.kind == CRYSTAL_HT_LINEAR ? ht.capacity * 8 : 0;
    const bool stage = ht.kind == CRYSTAL_HT_LINEAR && table_bytes <= device_lds_per_block() - 4096;
    if (stage && cfg.grid_per_cu <= 0) cfg.grid_per_cu = 1;  // stage once per resident workgroup
    const int64_t grid = grid_for(n_tiles, cfg);
    if (grid == 0) return hipSuccess;
    if (pp)
        return probe_launch<BLOCK, IPT, true>(ht, t, stage, table_bytes, grid, fk, pp, n, out, cnt, n_tiles, s);
    return probe_launch<BLOCK, IPT, false>(ht, t, stage, table_bytes, grid, fk, pp, n, out, cnt, n_tiles, s);
}

hipError_t launch_ht_probe(const LaunchCfg &cfg, const crystal_ht &ht, const int32_t *fk,
                           const int32_t *probe_payload, int64_t n, uint64_t *sum, uint64_t *count,
                           hipStream_t s) {
    hipError_t e = zero_pair(sum, count, s);
    if (e != hipSuccess || n == 0) return e;
    switch (CRYSTAL_VARIANT_KEY(cfg.block, cfg.ipt)) {
#define X(B, I) \
    case CRYSTAL_VARIANT_KEY(B, I): return probe_t<B, I>(cfg, ht, fk, probe_payload, n, sum, count, s);
        CRYSTAL_VARIANTS_VEC(X)
#undef X
    default: return hipErrorInvalidValue;
    }
}

// -------------------------------------------------------------- group-by ---
// LDS_PART: each workgroup accumulates into an LDS copy of the group array
// (ds_add_u64) over the tiles it strides through, then flushes the non-zero
// entries with global 64-bit atomics.  Otherwise every row adds directly.
template <int BLOCK, int IPT, bool LDS_PART>
__global__ __launch_bounds__(BLOCK) void groupby_kernel(const int32_t *__restrict__ g,
                                                        const int32_t *__restrict__ v, int64_t n,
                                                        int64_t n_groups,
                                                        uint64_t *__restrict__ sums,
                                                        int32_t *status, int64_t n_tiles) {
    using T = TileShape<BLOCK, IPT>;
    extern __shared__ uint64_t part[];
    if constexpr (LDS_PART) {
        for (int64_t i = threadIdx.x; i < n_groups; i += BLOCK) part[i] = 0;
        __syncthreads();
    }
    bool bad = false;
    for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const int64_t base = tile * T::ITEMS;
        int32_t gk[IPT], vk[IPT];
        block_load<BLOCK, IPT, true>(g, base, n, gk);
        block_load<BLOCK, IPT, true>(v, base, n, vk);
        const uint32_t valid = valid_mask<BLOCK, IPT>(base, n);
#pragma unroll
        for (int k = 0; k < IPT; ++k) {
            if (!((valid >> k) & 1u)) continue;
            if ((uint64_t)(int64_t)gk[k] >= (uint64_t)n_groups) {
                bad = true;
                continue;
            }
            const uint64_t add = (uint64_t)(int64_t)vk[k];
            if constexpr (LDS_PART)
                atomicAdd((unsigned long long *)&part[gk[k]], (unsigned long long)add);
            else
                atomic_add_u64(sums + gk[k], add);
        }
    }
    if (bad) set_status(status, CRYSTAL_ERANGE);
    if constexpr (LDS_PART) {
        __syncthreads();
        for (int64_t i = threadIdx.x; i < n_groups; i += BLOCK) {
            const uint64_t x = part[i];
            if (x) atomic_add_u64(sums + i, x);
        }
    }
}

template <int BLOCK, int IPT>
static hipError_t groupby_t(const LaunchCfg &cfg_in, const int32_t *g, const int32_t *v, int64_t n,
                            int64_t n_groups, uint64_t *sums, int32_t *status, hipStream_t s) {
    using T = TileShape<BLOCK, IPT>;
    const int64_t n_tiles = (n + T::ITEMS - 1) / T::ITEMS;
    LaunchCfg cfg = cfg_in;
    const int64_t lds = n_groups * 8;
    // LDS partials cost one flush of n_groups atomics per workgroup instead
    // of one atomic per row: worth it when rows outnumber those flushes
    LaunchCfg pcfg = cfg;
    if (pcfg.grid_per_cu <= 0) pcfg.grid_per_cu = 1;
    const bool part = lds <= device_lds_per_block() / 2 && n >= 4 * grid_for(n_tiles, pcfg) * n_groups;
    if (part) cfg = pcfg;
    const int64_t grid = grid_for(n_tiles, cfg);
    if (grid == 0) return hipSuccess;
    if (part) {
        auto fn = groupby_kernel<BLOCK, IPT, true>;
        hipError_t e = hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(fn, dim3((unsigned)grid), dim3(BLOCK), (size_t)lds, s, g, v, n, n_groups,
                           sums, status, n_tiles);
    } else {
        hipLaunchKernelGGL((groupby_kernel<BLOCK, IPT, false>), dim3((unsigned)grid), dim3(BLOCK), 0, s,
                           g, v, n, n_groups, sums, status, n_tiles);
    }
    return hipGetLastError();
}

hipError_t launch_groupby(const LaunchCfg &cfg, const int32_t *group, const int32_t *value,
                          int64_t n, int64_t n_groups, uint64_t *sums, int32_t *status,
                          hipStream_t s) {
    hipError_t e = fill_u64(sums, n_groups, 0ull, s);
    if (e != hipSuccess || n == 0) return e;
    switch (CRYSTAL_VARIANT_KEY(cfg.block, cfg.ipt)) {
#define X(B, I) \
    case CRYSTAL_VARIANT_KEY(B, I): return groupby_t<B, I>(cfg, group, value, n, n_groups, sums, status, s);
        CRYSTAL_VARIANTS_VEC(X)
#undef X
    default: return hipErrorInvalidValue;
    }
}

}  // namespace crystal
