// Selection (section 4.2, Q3; section 3.2, Q0) and projection (section 4.1,
// Q1 and Q2) kernels, plus the fill kernels used to clear outputs.
#include "block.hpp"
#include "internal.hpp"
#include "variants.hpp"

namespace crystal {

// ------------------------------------------------------------------ fills --
__global__ __launch_bounds__(256) void fill_u64_kernel(uint64_t *__restrict__ p, int64_t n,
                                                       uint64_t value) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        p[i] = value;
}

__global__ __launch_bounds__(256) void fill_u32_kernel(uint32_t *__restrict__ p, int64_t n,
                                                       uint32_t value) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        p[i] = value;
}

__global__ void zero_pair_kernel(uint64_t *a, uint64_t *b) {
    if (threadIdx.x == 0) *a = 0;
    if (threadIdx.x == 1) *b = 0;
}

hipError_t zero_pair(uint64_t *a, uint64_t *b, hipStream_t s) {
    hipLaunchKernelGGL(zero_pair_kernel, dim3(1), dim3(64), 0, s, a, b);
    return hipGetLastError();
}

static int64_t fill_grid(int64_t n) {
    int64_t g = (n + 255) / 256;
    int64_t cap = (int64_t)device_cu_count() * 16;
    return g < cap ? (g > 0 ? g : 1) : cap;
}

hipError_t fill_u64(uint64_t *p, int64_t n, uint64_t value, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_u64_kernel, dim3((unsigned)fill_grid(n)), dim3(256), 0, s, p, n, value);
    return hipGetLastError();
}

hipError_t fill_u32(uint32_t *p, int64_t n, uint32_t value, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)fill_grid(n)), dim3(256), 0, s, p, n, value);
    return hipGetLastError();
}

// Zero several equal-sized slots of one array in one launch: slot slots[i]
// covers base[slots[i] * len, (slots[i] + 1) * len).
struct SlotList {
    int32_t count;
    int32_t slot[kMaxSlots];
};

__global__ __launch_bounds__(256) void zero_slots_kernel(uint64_t *__restrict__ base, int64_t len, SlotList l) {
    const int64_t n = (int64_t)l.count * len;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const int64_t k = i / len;
        base[(int64_t)l.slot[k] * len + (i - k * len)] = 0ull;
    }
}

hipError_t zero_slots(uint64_t *base, int64_t len, const int32_t *slots, int count, hipStream_t s) {
    if (count <= 0 || len <= 0) return hipSuccess;
    if (count > kMaxSlots) return hipErrorInvalidValue;
    SlotList l = {};
    l.count = count;
    for (int i = 0; i < count; ++i) l.slot[i] = slots[i];
    hipLaunchKernelGGL(zero_slots_kernel, dim3((unsigned)fill_grid((int64_t)count * len)), dim3(256), 0, s, base, len,
                       l);
    return hipGetLastError();
}

// ------------------------------------------------------------- selection --
// Tile = BlockLoad -> BlockPred -> BlockScan of the match counts -> the tile's
// output offset -> BlockShuffle into LDS (matches in input order within the
// tile) -> BlockStore.
//
// Output offsets, two ways:
//  - unordered (the method of section 3.2): thread 0 reserves the tile's
//    output range with one 64-bit atomic on the global counter, skipped when
//    the tile has no match.  Same-address atomics from the eight XCDs
//    serialise at the memory-side atomic unit (about 12 ns each on MI355X),
//    so tiles are large (the tuned default is 1024 x 16 = 16 Ki items) to
//    keep the reservations well below the time the column takes to stream.
//  - stable: every tile publishes its match count in its own 64-bit status
//    word and finds its offset by decoupled look-back over its predecessors'
//    words (the single-pass scan of Merrill and Garland): each round the
//    workgroup reads BLOCK predecessors' words and stops at the nearest one
//    that holds an inclusive prefix.  Tiles then land in input order, so the
//    output is the qualifying values in input order on every run; the status
//    words live in memory that all XCDs see, so each round costs a memory
//    round trip.
//
// Status word: bits 63..62 = 0 (nothing yet), 1 (tile count), 2 (inclusive
// prefix); bits 61..0 = the count.  Words are read and written with
// agent-scope atomics (coherent across XCDs).  A tile only waits for lower-
// numbered tiles and there is one tile per workgroup, dispatched in order, so
// the lowest unfinished tile is always running; should a predecessor still
// never publish, the wait gives up after a bounded number of polls: that tile
// publishes the poison prefix 2^61, every later tile inherits it and writes
// nothing, and the last tile reports a count of -1.
static constexpr uint64_t kStAgg = 1ull << 62;
static constexpr uint64_t kStIncl = 2ull << 62;
static constexpr uint64_t kStValue = (1ull << 62) - 1;
static constexpr uint64_t kPoison = 1ull << 61;
static constexpr uint32_t kLookbackPolls = 1u << 15;

__device__ __forceinline__ uint64_t status_load(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void status_store(uint64_t *p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Called by every thread of the workgroup.  Publishes the tile's count and
// returns the number of matches in all earlier tiles (kPoison if unknown).
// Each round, thread i reads the status word of tile top - i, so a round
// covers BLOCK predecessors with one memory round trip; the waves' findings
// are combined through LDS (wave_incl / wave_ready / wave_sum).
template <int BLOCK>
__device__ __forceinline__ uint64_t block_lookback(uint64_t *st, int64_t tile, uint64_t count,
                                                   uint32_t *wave_flags, uint64_t *wave_sum) {
    constexpr int W = BLOCK / kWave;
    const uint32_t lane = lane_id();
    const int w = threadIdx.x / kWave;
    if (threadIdx.x == 0) status_store(st + tile, (tile == 0 ? kStIncl : kStAgg) | count);
    if (tile == 0) return 0;
    uint64_t running = 0;
    bool poisoned = false;
    int64_t top = tile - 1;
    uint32_t polls = 0;
    for (;;) {
        const int64_t idx = top - (int64_t)threadIdx.x;
        const uint64_t v = idx >= 0 ? status_load(st + idx) : kStIncl;  // before tile 0: prefix 0
        const uint32_t flag = (uint32_t)(v >> 62);
        const uint64_t incl = ballot(flag == 2u);
        const uint64_t none = ballot(flag == 0u);
        // lanes 0..stop, stop = this wave's nearest predecessor with an inclusive prefix
        const uint64_t upto = incl ? ((incl & (~incl + 1ull)) << 1) - 1ull : ~0ull;
        const bool mine = (upto >> lane) & 1ull;
        const bool poison = ballot(mine && (v & kStValue) >= kPoison) != 0;
        const uint64_t sum = wave_sum_u64(mine ? (v & kStValue) : 0ull);
        if (lane == 0) {
            wave_flags[w] = (incl ? 1u : 0u) | ((none & upto) ? 0u : 2u) | (poison ? 4u : 0u);
            wave_sum[w] = sum;
        }
        __syncthreads();
        // the nearest waves first: add ready waves until one holds an inclusive prefix
        bool ready = true, done = false;
        uint64_t add = 0;
        for (int ww = 0; ww < W; ++ww) {
            const uint32_t f = wave_flags[ww];
            if (!(f & 2u)) {
                ready = false;
                break;
            }
            if (f & 4u) poisoned = true;
            add += wave_sum[ww];
            if (f & 1u) {
                done = true;
                break;
            }
        }
        __syncthreads();
        if (poisoned) break;
        if (!ready) {
            if (++polls > kLookbackPolls) {
                poisoned = true;
                break;
            }
            __builtin_amdgcn_s_sleep(2);
            continue;
        }
        running += add;
        if (done) break;
        top -= BLOCK;
    }
    if (poisoned) running = kPoison;
    if (threadIdx.x == 0) status_store(st + tile, kStIncl | (poisoned ? kPoison : running + count));
    return running;
}

// Stable selection: one workgroup per tile, output offsets by decoupled look-back.
template <int BLOCK, int IPT>
__global__ __launch_bounds__(BLOCK) void select_kernel(const int32_t *__restrict__ in, int64_t n,
                                                       int32_t lo, int32_t hi,
                                                       int32_t *__restrict__ out,
                                                       uint64_t *__restrict__ st,
                                                       int64_t *__restrict__ count_out,
                                                       int64_t n_tiles) {
    using T = TileShape<BLOCK, IPT>;
    constexpr int C = T::CHUNKS, W = T::WAVES, V = T::VEC;
    constexpr int VBITS = V == 1 ? 1 : V == 2 ? 2 : 3;
    __shared__ int32_t buf[T::ITEMS];
    __shared__ uint32_t chunk_tot[C * W];
    __shared__ uint32_t wave_flags[W];
    __shared__ uint64_t wave_sum[W];
    const int w = threadIdx.x / kWave;
    const uint32_t lane = lane_id();
    {
        const int64_t tile = blockIdx.x;
        const int64_t base = tile * T::ITEMS;
        int32_t v[IPT];
        block_load<BLOCK, IPT, true>(in, base, n, v);
        const uint32_t flags = block_pred_range<IPT>(v, valid_mask<BLOCK, IPT>(base, n), lo, hi);
        // BlockScan in input order: item (c, t, e) precedes (c, t', e') when t < t',
        // and chunk c precedes chunk c + 1
        uint32_t pre[C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            uint32_t wt;
            pre[c] = wave_exclusive_scan_small<VBITS>((uint32_t)__popc((flags >> (c * V)) & T::VMASK), wt);
            if (lane == 0) chunk_tot[c * W + w] = wt;
        }
        __syncthreads();
        uint32_t cbase[C];
        uint32_t total = 0;
#pragma unroll
        for (int c = 0; c < C; ++c)
#pragma unroll
            for (int ww = 0; ww < W; ++ww) {
                const uint32_t t = chunk_tot[c * W + ww];
                if (ww == w) cbase[c] = total;
                total += t;
            }
        const uint64_t ob = block_lookback<BLOCK>(st, tile, total, wave_flags, wave_sum);
        // BlockShuffle: matches to their tile positions in LDS
#pragma unroll
        for (int c = 0; c < C; ++c) {
            uint32_t pos = cbase[c] + pre[c];
#pragma unroll
            for (int e = 0; e < V; ++e)
                if ((flags >> (c * V + e)) & 1u) buf[pos++] = v[c * V + e];
        }
        __syncthreads();
        if (ob < kPoison)
            for (uint32_t i = threadIdx.x; i < total; i += BLOCK) __builtin_nontemporal_store(buf[i], out + ob + i);
        if (tile == n_tiles - 1 && threadIdx.x == 0) *count_out = ob < kPoison ? (int64_t)(ob + total) : -1;
    }
}

// Unstable selection with buffered reservations.  Persistent workgroups
// stride over the tiles and compact each tile's matches into an LDS buffer of
// two tiles; output space is reserved with one atomic only when the buffer
// could not take another tile, then the whole buffer is written out with
// 16-byte stores.  Fewer reservations than one per tile (they serialise on
// one address), and the loads of the next two tiles are in flight while the
// current one is compacted.
//
// Compaction (BlockScan + BlockShuffle): for every item slot k, a ballot of
// the wave's flags gives each matching lane its rank among the wave's matches
// in that slot (mbcnt), so a wave's matches are laid out slot by slot, lane
// by lane, and each LDS store instruction writes consecutive words.  The
// waves' totals are exchanged once per tile.  Within a tile the order is
// therefore slot-major, not input order; the tile's matches stay contiguous.
// A non-matching item is stored to a per-thread spare word, so the scatter
// has no branches.
template <int BLOCK, int IPT>
__global__ __launch_bounds__(BLOCK) void select_buffered_kernel(const int32_t *__restrict__ in, int64_t n,
                                                                int32_t lo, int32_t hi,
                                                                int32_t *__restrict__ out,
                                                                int64_t *__restrict__ count_out,
                                                                int64_t n_tiles) {
    using T = TileShape<BLOCK, IPT>;
    constexpr int W = T::WAVES;
    constexpr uint32_t CAP = 2 * T::ITEMS;
    extern __shared__ int32_t buf[];  // CAP entries, then one spare word per thread
    __shared__ uint32_t wave_tot[W];
    __shared__ uint64_t flush_off;
    const int w = threadIdx.x / kWave;
    const uint32_t lane = lane_id();
    uint32_t fill = 0;  // entries in buf, equal in every thread

    auto flush = [&]() {
        if (threadIdx.x == 0) flush_off = atomic_add_u64((uint64_t *)count_out, fill);
        __syncthreads();
        int32_t *dst = out + flush_off;
        // scalar stores up to a 16-byte boundary, vectors, then the tail
        uint32_t head = (uint32_t)(((16u - ((uint32_t)(uintptr_t)dst & 15u)) & 15u) >> 2);
        if (head > fill) head = fill;
        if (threadIdx.x < head) __builtin_nontemporal_store(buf[threadIdx.x], dst + threadIdx.x);
        const uint32_t nvec = (fill - head) >> 2;
        for (uint32_t i = threadIdx.x; i < nvec; i += BLOCK) {
            const uint32_t b = head + 4 * i;
            const v4i x = {buf[b], buf[b + 1], buf[b + 2], buf[b + 3]};
            __builtin_nontemporal_store(x, reinterpret_cast<v4i *>(dst + b));
        }
        for (uint32_t i = head + 4 * nvec + threadIdx.x; i < fill; i += BLOCK) __builtin_nontemporal_store(buf[i], dst + i);
        __syncthreads();  // buf and flush_off are reused
        fill = 0;
    };
    // compact one tile's values (already loaded) into buf
    auto compact = [&](int64_t tile, const int32_t(&v)[IPT]) {
        const int64_t base = tile * T::ITEMS;
        const uint32_t flags = block_pred_range<IPT>(v, valid_mask<BLOCK, IPT>(base, n), lo, hi);
        uint32_t pos[IPT];
        uint32_t wt = 0;  // the wave's matches so far (uniform)
#pragma unroll
        for (int k = 0; k < IPT; ++k) {
            const uint64_t m = ballot((flags >> k) & 1u);
            pos[k] = wt + count_below(m);
            wt += (uint32_t)__popcll(m);
        }
        if (lane == 0) wave_tot[w] = wt;
        __syncthreads();
        uint32_t before = 0, total = 0;
#pragma unroll
        for (int i = 0; i < W; ++i) {
            const uint32_t t = wave_tot[i];
            before += i < w ? t : 0u;
            total += t;
        }
        const uint32_t b0 = fill + before;
        const uint32_t spare = CAP + threadIdx.x;
#pragma unroll
        for (int k = 0; k < IPT; ++k) buf[((flags >> k) & 1u) ? b0 + pos[k] : spare] = v[k];
        fill += total;
        __syncthreads();  // wave_tot is rewritten by the next tile; buf is complete
        if (fill + T::ITEMS > CAP) flush();
    };

    // three register buffers, rotated so that a buffer receiving loads is never copied
    int32_t va[IPT], vb[IPT], vc[IPT];
    int64_t tile = blockIdx.x;
    const int64_t g = gridDim.x;
    if (tile < n_tiles) block_load<BLOCK, IPT, true>(in, tile * T::ITEMS, n, va);
    if (tile + g < n_tiles) block_load<BLOCK, IPT, true>(in, (tile + g) * T::ITEMS, n, vb);
    while (tile < n_tiles) {
        if (tile + 2 * g < n_tiles) block_load<BLOCK, IPT, true>(in, (tile + 2 * g) * T::ITEMS, n, vc);
        compact(tile, va);
        tile += g;
        if (tile >= n_tiles) break;
        if (tile + 2 * g < n_tiles) block_load<BLOCK, IPT, true>(in, (tile + 2 * g) * T::ITEMS, n, va);
        compact(tile, vb);
        tile += g;
        if (tile >= n_tiles) break;
        if (tile + 2 * g < n_tiles) block_load<BLOCK, IPT, true>(in, (tile + 2 * g) * T::ITEMS, n, vb);
        compact(tile, vc);
        tile += g;
    }
    if (fill) flush();
}

template <int BLOCK, int IPT>
static hipError_t select_t(const LaunchCfg &cfg, const int32_t *in, int64_t n, int32_t lo, int32_t hi,
                           int32_t *out, int64_t *count, uint64_t *st, bool stable, hipStream_t s) {
    using T = TileShape<BLOCK, IPT>;
    const int64_t n_tiles = (n + T::ITEMS - 1) / T::ITEMS;
    // stable: one workgroup per tile, always: a stable tile only waits for
    // lower-numbered tiles, which in-order dispatch has already started;
    // workgroups striding over tiles could wait for a tile whose workgroup is
    // not resident
    hipError_t e;
    if (stable) {
        e = fill_u64(st, n_tiles, 0ull, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((select_kernel<BLOCK, IPT>), dim3((unsigned)n_tiles), dim3(BLOCK), 0, s, in, n,
                           lo, hi, out, st, count, n_tiles);
    } else {
        e = fill_u64((uint64_t *)count, 1, 0ull, s);
        if (e != hipSuccess) return e;
        // persistent: as many workgroups per CU as waves and the two-tile LDS buffer allow (or as tuned)
        const size_t lds = ((size_t)2 * T::ITEMS + BLOCK) * sizeof(int32_t);
        int64_t per_cu = cfg.grid_per_cu > 0 ? cfg.grid_per_cu : (2048 / BLOCK > 0 ? 2048 / BLOCK : 1);
        const int64_t lds_cap = device_lds_per_cu() / (int64_t)(lds + 1024);
        if (per_cu > lds_cap) per_cu = lds_cap > 0 ? lds_cap : 1;
        int64_t grid = per_cu * device_cu_count();
        if (grid > n_tiles) grid = n_tiles;
        if (lds > 65536) {
            e = hipFuncSetAttribute((const void *)select_buffered_kernel<BLOCK, IPT>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
        }
        hipLaunchKernelGGL((select_buffered_kernel<BLOCK, IPT>), dim3((unsigned)grid), dim3(BLOCK), lds, s, in, n,
                           lo, hi, out, count, n_tiles);
    }
    return hipGetLastError();
}

int64_t select_tile_items(const LaunchCfg &cfg) { return (int64_t)cfg.block * cfg.ipt; }

hipError_t launch_select(const LaunchCfg &cfg, const int32_t *in, int64_t n, int32_t lo, int32_t hi,
                         int32_t *out, int64_t *count, uint64_t *status_words, bool stable, hipStream_t s) {
    if (n == 0 || lo > hi) return fill_u64((uint64_t *)count, 1, 0ull, s);
    switch (CRYSTAL_VARIANT_KEY(cfg.block, cfg.ipt)) {
#define X(B, I) \
    case CRYSTAL_VARIANT_KEY(B, I): return select_t<B, I>(cfg, in, n, lo, hi, out, count, status_words, stable, s);
        CRYSTAL_VARIANTS_ALL(X)
#undef X
    default: return hipErrorInvalidValue;
    }
}

// ------------------------------------------------------------ projection --
__device__ __forceinline__ float linear2(float x1, float x2, float a, float b) {
#pragma clang fp contract(off)
    const float p = a * x1;
    const float q = b * x2;
    return p + q;
}

template <bool SIGMOID>
__device__ __forceinline__ float project_one(float x1, float x2, float a, float b) {
    const float t = linear2(x1, x2, a, b);
    if constexpr (SIGMOID) {
        return 1.0f / (1.0f + expf(-t));
    } else {
        return t;
    }
}

// Two BlockLoads, the arithmetic, one BlockStore (streaming, non-temporal).
template <int BLOCK, int IPT, bool SIGMOID>
__global__ __launch_bounds__(BLOCK) void project_kernel(const float *__restrict__ x1,
                                                        const float *__restrict__ x2, int64_t n,
                                                        float a, float b,
                                                        float *__restrict__ out,
                                                        int64_t n_tiles) {
    using T = TileShape<BLOCK, IPT>;
    for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const int64_t base = tile * T::ITEMS;
        if (base + T::ITEMS <= n) {
#pragma unroll
            for (int c = 0; c < T::CHUNKS; ++c) {
                const int64_t i = T::index(base, c, 0);
                if constexpr (T::VEC == 4) {
                    v4f p = __builtin_nontemporal_load(reinterpret_cast<const v4f *>(x1 + i));
                    v4f q = __builtin_nontemporal_load(reinterpret_cast<const v4f *>(x2 + i));
                    v4f r;
                    r.x = project_one<SIGMOID>(p.x, q.x, a, b);
                    r.y = project_one<SIGMOID>(p.y, q.y, a, b);
                    r.z = project_one<SIGMOID>(p.z, q.z, a, b);
                    r.w = project_one<SIGMOID>(p.w, q.w, a, b);
                    __builtin_nontemporal_store(r, reinterpret_cast<v4f *>(out + i));
                } else {
#pragma unroll
                    for (int e = 0; e < T::VEC; ++e)
                        __builtin_nontemporal_store(project_one<SIGMOID>(
                            __builtin_nontemporal_load(x1 + i + e),
                            __builtin_nontemporal_load(x2 + i + e), a, b), out + i + e);
                }
            }
        } else {
#pragma unroll
            for (int c = 0; c < T::CHUNKS; ++c)
#pragma unroll
                for (int e = 0; e < T::VEC; ++e) {
                    const int64_t i = T::index(base, c, e);
                    if (i < n) out[i] = project_one<SIGMOID>(x1[i], x2[i], a, b);
                }
        }
    }
}

template <int BLOCK, int IPT>
static hipError_t project_t(const LaunchCfg &cfg, const float *x1, const float *x2, int64_t n,
                            float a, float b, float *out, bool sigmoid, hipStream_t s) {
    using T = TileShape<BLOCK, IPT>;
    const int64_t n_tiles = (n + T::ITEMS - 1) / T::ITEMS;
    const int64_t grid = grid_for(n_tiles, cfg);
    if (grid == 0) return hipSuccess;
    if (sigmoid)
        hipLaunchKernelGGL((project_kernel<BLOCK, IPT, true>), dim3((unsigned)grid), dim3(BLOCK), 0,
                           s, x1, x2, n, a, b, out, n_tiles);
    else
        hipLaunchKernelGGL((project_kernel<BLOCK, IPT, false>), dim3((unsigned)grid), dim3(BLOCK),
                           0, s, x1, x2, n, a, b, out, n_tiles);
    return hipGetLastError();
}

hipError_t launch_project(const LaunchCfg &cfg, const float *x1, const float *x2, int64_t n,
                          float a, float b, float *out, bool sigmoid, hipStream_t s) {
    switch (CRYSTAL_VARIANT_KEY(cfg.block, cfg.ipt)) {
#define X(B, I) \
    case CRYSTAL_VARIANT_KEY(B, I): return project_t<B, I>(cfg, x1, x2, n, a, b, out, sigmoid, s);
        CRYSTAL_VARIANTS_VEC(X)
#undef X
    default: return hipErrorInvalidValue;
    }
}

// ------------------------------------------------------------ narrow columns --
// out[i] = in[i] - base as an unsigned E; values that do not fit are stored
// truncated and reported.
template <typename E>
__global__ __launch_bounds__(256) void pack_column_kernel(const int32_t *__restrict__ in, int64_t n, int32_t base,
                                                          E *__restrict__ out, int32_t *status) {
    constexpr uint32_t kMax = (uint32_t)(E)~(E)0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint32_t d = (uint32_t)in[i] - (uint32_t)base;
        bad |= in[i] < base || d > kMax;
        out[i] = (E)d;
    }
    if (bad) set_status(status, CRYSTAL_ERANGE);
}

// Bit-packed column: each thread assembles whole output words, so no word is
// written twice and no atomics are needed.  A row's range check is made by
// the word that holds its first bit; the padding words are written as zero.
__global__ __launch_bounds__(256) void pack_bits_kernel(const int32_t *__restrict__ in, int64_t n, int32_t base,
                                                        uint32_t bits, uint32_t *__restrict__ out, int64_t words,
                                                        int32_t *status) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const uint32_t mask = (1u << bits) - 1u;  // bits <= 16
    bool bad = false;
    for (int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; w < words; w += stride) {
        const int64_t b0 = w * 32;  // the stream bits of word w: [b0, b0 + 32)
        int64_t i0 = b0 / bits, i1 = (b0 + 32 + bits - 1) / bits;
        if (i1 > n) i1 = n;
        uint32_t word = 0;
        for (int64_t i = i0; i < i1; ++i) {
            const uint32_t d = (uint32_t)in[i] - (uint32_t)base;
            const int64_t sh = i * (int64_t)bits - b0;  // > -bits and < 32
            if (sh >= 0) {
                bad |= in[i] < base || d > mask;
                word |= (d & mask) << sh;
            } else {
                word |= (d & mask) >> (-sh);
            }
        }
        out[w] = word;
    }
    if (bad) set_status(status, CRYSTAL_ERANGE);
}

hipError_t launch_pack_column_bits(const int32_t *in, int64_t n, int32_t base, int32_t bits, uint32_t *out,
                                   int64_t words, int32_t *status, hipStream_t s) {
    int64_t grid = (words + 255) / 256;
    const int64_t cap = (int64_t)device_cu_count() * 16;
    if (grid > cap) grid = cap;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(pack_bits_kernel, dim3((unsigned)grid), dim3(256), 0, s, in, n, base, (uint32_t)bits, out,
                       words, status);
    return hipGetLastError();
}

hipError_t launch_pack_column(const int32_t *in, int64_t n, int32_t base, int32_t width, void *out,
                              int32_t *status, hipStream_t s) {
    int64_t grid = (n + 255) / 256;
    const int64_t cap = (int64_t)device_cu_count() * 16;
    if (grid > cap) grid = cap;
    if (width == 2)
        hipLaunchKernelGGL(pack_column_kernel<uint16_t>, dim3((unsigned)grid), dim3(256), 0, s, in, n, base,
                           (uint16_t *)out, status);
    else
        hipLaunchKernelGGL(pack_column_kernel<uint8_t>, dim3((unsigned)grid), dim3(256), 0, s, in, n, base,
                           (uint8_t *)out, status);
    return hipGetLastError();
}

}  // namespace crystal
