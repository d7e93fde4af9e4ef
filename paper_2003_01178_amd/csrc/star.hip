// Fused star-query kernel: the pipelined multi-join probe of the section 5.3
// case study, and the fact-side selection of SSB Q1.1 (section 3.1), in one
// launch with nothing materialised in device memory between operators.
//
// Workgroups are persistent and stride over tiles of BLOCK x IPT rows.
//
// Dense phase (the first one or two steps of the plan): the first step's
// column is read in full (BlockLoad), the second step's column only at the
// 128-bit vectors that still hold a live row (BlockLoadSel), so the bytes
// fetched per column fall with the selectivity before it (the r1 term of the
// section 5.3 model).  The two steps are software-pipelined across tiles:
// while tile k is finished, the second-step loads of tile k+1 and the
// first-step loads of tile k+2 are in flight.  Presence-only direct joins of
// the dense phase probe a copy of their bitmap staged in LDS.
//
// Sparse phase: rows alive after the dense phase are compacted into an LDS
// queue per wave (an exclusive scan of the per-lane counts with ballots, then
// each lane writes its rows at its offset: the BlockScan and BlockShuffle of
// section 3.2 at wave granularity, so no workgroup barrier is needed) and
// finished in batches of 64 rows, one row per lane, so the remaining steps'
// loads of a whole batch are in flight together instead of one dependent
// round trip per tile.
//
// Aggregation: grouped results are added with 64-bit atomics per surviving
// row (survivors are sparse); a scalar result is reduced per workgroup
// (BlockAggregate) into a partial in scratch memory and summed by a one-
// workgroup finalize kernel, which avoids same-address atomics from every
// workgroup.
#include <mutex>

#include "block.hpp"
#include "internal.hpp"
#include "variants.hpp"

namespace crystal {

__device__ __forceinline__ int step_col(const StarPlanDev &p, int s) {
    return s < p.n_preds ? p.pred_col[s] : p.joins[s - p.n_preds].fk_col;
}

// Column access for int32 and narrow (uint16 / uint8 offset) columns; the
// width is uniform, so the dispatch is a scalar branch.
__device__ __forceinline__ int32_t col_value(const StarPlanDev &p, int c, int64_t row) {
    const ColDev cd = p.col[c];  // a copy: keeps the plan in the kernel-argument segment
    if (cd.bits) return packed_value(reinterpret_cast<const uint32_t *>(cd.p), cd.base, (uint32_t)cd.bits, row);
    if (cd.width == 2) return cd.base + (int32_t)reinterpret_cast<const uint16_t *>(cd.p)[row];
    if (cd.width == 1) return cd.base + (int32_t)reinterpret_cast<const uint8_t *>(cd.p)[row];
    return cd.p[row];
}

// Tile loads of a dense-phase column.  The descriptor is passed by value (read
// once per kernel), which keeps the plan in the kernel-argument segment.
// NARROW 0: int32 columns; 2: both dense columns uint16 offsets; 3: both
// dense columns bit-packed (each its own width); 1: any formats, dispatched
// at run time.  Separate kernel instances, so that the common layouts carry
// no format dispatch in the pipelined loop.
template <int BLOCK, int IPT, int NARROW>
__device__ __forceinline__ void load_col_tile(const ColDev cd, int64_t n_rows, int64_t base, int32_t (&v)[IPT]) {
    if constexpr (NARROW == 0)
        block_load<BLOCK, IPT, true>(cd.p, base, n_rows, v);
    else if constexpr (NARROW == 2)
        block_load_narrow<BLOCK, IPT, uint16_t, true>(reinterpret_cast<const uint16_t *>(cd.p), cd.base, base,
                                                      n_rows, v);
    else if constexpr (NARROW == 3)
        block_load_packed<BLOCK, IPT, true>(reinterpret_cast<const uint32_t *>(cd.p), cd.base, (uint32_t)cd.bits,
                                            base, n_rows, v);
    else if (cd.bits)
        block_load_packed<BLOCK, IPT, true>(reinterpret_cast<const uint32_t *>(cd.p), cd.base, (uint32_t)cd.bits,
                                            base, n_rows, v);
    else if (cd.width == 2)
        block_load_narrow<BLOCK, IPT, uint16_t, true>(reinterpret_cast<const uint16_t *>(cd.p), cd.base, base,
                                                      n_rows, v);
    else if (cd.width == 1)
        block_load_narrow<BLOCK, IPT, uint8_t, true>(reinterpret_cast<const uint8_t *>(cd.p), cd.base, base,
                                                     n_rows, v);
    else
        block_load<BLOCK, IPT, true>(cd.p, base, n_rows, v);
}

template <int BLOCK, int IPT, int NARROW>
__device__ __forceinline__ void load_col_tile_sel(const ColDev cd, int64_t n_rows, int64_t base, uint32_t flags,
                                                  int32_t (&v)[IPT]) {
    if constexpr (NARROW == 0)
        block_load_sel<BLOCK, IPT, true>(cd.p, base, n_rows, flags, v);
    else if constexpr (NARROW == 2)
        block_load_sel_narrow<BLOCK, IPT, uint16_t, true>(reinterpret_cast<const uint16_t *>(cd.p), cd.base, base,
                                                          n_rows, flags, v);
    else if constexpr (NARROW == 3)
        block_load_sel_packed<BLOCK, IPT, true>(reinterpret_cast<const uint32_t *>(cd.p), cd.base,
                                                (uint32_t)cd.bits, base, n_rows, flags, v);
    else if (cd.bits)
        block_load_sel_packed<BLOCK, IPT, true>(reinterpret_cast<const uint32_t *>(cd.p), cd.base,
                                                (uint32_t)cd.bits, base, n_rows, flags, v);
    else if (cd.width == 2)
        block_load_sel_narrow<BLOCK, IPT, uint16_t, true>(reinterpret_cast<const uint16_t *>(cd.p), cd.base, base,
                                                          n_rows, flags, v);
    else if (cd.width == 1)
        block_load_sel_narrow<BLOCK, IPT, uint8_t, true>(reinterpret_cast<const uint8_t *>(cd.p), cd.base, base,
                                                         n_rows, flags, v);
    else
        block_load_sel<BLOCK, IPT, true>(cd.p, base, n_rows, flags, v);
}

// Dense-phase columns as loaded, carried across pipeline iterations and
// decoded where the step uses them.  Decoding a narrow or bit-packed column
// right after its loads are issued would make the wave wait for them there,
// so the next tiles' loads could not stay in flight while the current tile
// is processed.  NARROW 2: pairs of uint16 offsets per word; NARROW 3: the
// three stream words that hold each thread's 4-row vector.  The int32 and
// run-time dispatched instances (NARROW 0 and 1) keep values in registers.
template <int IPT, int NARROW>
struct RawTile {
    static_assert(NARROW == 2 || NARROW == 3, "raw tiles are narrow or bit-packed");
    uint32_t w[NARROW == 2 ? IPT / 2 : IPT / 4 * 3];  // stored words
};

template <int BLOCK, int IPT, int NARROW>
__device__ __forceinline__ void load_raw_tile(const ColDev cd, int64_t n_rows, int64_t base, bool sel, uint32_t flags,
                                              RawTile<IPT, NARROW> &r) {
    using T = TileShape<BLOCK, IPT>;
    if constexpr (NARROW == 2 || NARROW == 3) {
        static_assert(T::VEC == 4, "narrow tiles are read four rows at a time");
        const bool full = base + T::ITEMS <= n_rows;
#pragma unroll
        for (int c = 0; c < T::CHUNKS; ++c) {
            const uint32_t m = (flags >> (c * 4)) & 0xFu;
            if (sel && !m) continue;
            const int64_t r0 = T::index(base, c, 0);
            if constexpr (NARROW == 2) {
                const uint16_t *col = reinterpret_cast<const uint16_t *>(cd.p);
                if (full) {
                    typedef uint32_t u2 __attribute__((ext_vector_type(2)));
                    const u2 x = __builtin_nontemporal_load(reinterpret_cast<const u2 *>(col + r0));
                    r.w[c * 2] = x[0];
                    r.w[c * 2 + 1] = x[1];
                } else {
                    uint32_t lo = 0, hi = 0;
                    if (r0 < n_rows) lo |= col[r0];
                    if (r0 + 1 < n_rows) lo |= (uint32_t)col[r0 + 1] << 16;
                    if (r0 + 2 < n_rows) hi |= col[r0 + 2];
                    if (r0 + 3 < n_rows) hi |= (uint32_t)col[r0 + 3] << 16;
                    r.w[c * 2] = lo;
                    r.w[c * 2 + 1] = hi;
                }
            } else {
                // bit offset of the chunk's first row: a uniform part (the
                // tile's and the chunk's) plus the thread's, so the word index
                // is a scalar base plus a 32-bit per-thread offset; the
                // stream's padding makes the three words readable for any row < n
                const uint64_t u = (uint64_t)(base + (int64_t)c * BLOCK * T::VEC) * (uint32_t)cd.bits;
                const uint32_t off = ((uint32_t)u & 31u) + threadIdx.x * (uint32_t)(T::VEC * cd.bits);
                const uint32_t *q = reinterpret_cast<const uint32_t *>(cd.p) + (u >> 5) + (off >> 5);
                if (full || r0 < n_rows) {
                    r.w[c * 3] = __builtin_nontemporal_load(q);
                    r.w[c * 3 + 1] = __builtin_nontemporal_load(q + 1);
                    r.w[c * 3 + 2] = __builtin_nontemporal_load(q + 2);
                } else {
                    r.w[c * 3] = r.w[c * 3 + 1] = r.w[c * 3 + 2] = 0u;
                }
            }
        }
    }
}

// Values of a raw tile (rows past n_rows decode to arbitrary values; they are
// never alive).
template <int BLOCK, int IPT, int NARROW>
__device__ __forceinline__ void decode_tile(const ColDev cd, int64_t base, const RawTile<IPT, NARROW> &r,
                                            int32_t (&v)[IPT]) {
    using T = TileShape<BLOCK, IPT>;
    if constexpr (NARROW == 2) {
#pragma unroll
        for (int k = 0; k < IPT / 2; ++k) {
            v[2 * k] = cd.base + (int32_t)(r.w[k] & 0xFFFFu);
            v[2 * k + 1] = cd.base + (int32_t)(r.w[k] >> 16);
        }
    } else {
        static_assert(NARROW == 3, "raw tiles are narrow or bit-packed");
        const uint32_t bits = (uint32_t)cd.bits;
#pragma unroll
        for (int c = 0; c < T::CHUNKS; ++c) {
            // the low five bits of the chunk's bit offset, as in load_raw_tile
            const uint32_t s = (uint32_t)(base + (int64_t)c * BLOCK * T::VEC) * bits +
                               threadIdx.x * (uint32_t)T::VEC * bits;
            decode_packed_vec4(r.w[c * 3], r.w[c * 3 + 1], r.w[c * 3 + 2], s, bits, cd.base, &v[c * 4]);
        }
    }
}

__device__ __forceinline__ bool star_probe(const StarJoinDev &j, int32_t key, int32_t &payload) {
    if (j.kind == CRYSTAL_HT_DIRECT) {
        const uint32_t off = (uint32_t)key - (uint32_t)j.key_min;
        if ((int64_t)off >= j.span) return false;
        const bool hit = (j.bitmap[off >> 5] >> (off & 31u)) & 1u;
        if (hit && j.payload) payload = j.payload[off];
        return hit;
    }
    if (key == kEmptyKey) return false;
    return probe_linear((const v2i *)j.slots, j.mask, j.shift, key, payload);
}

// One step for one row (sparse phase).
__device__ __forceinline__ bool star_step_row(const StarPlanDev &p, int s, int32_t v) {
    if (s < p.n_preds) return in_range(v, p.pred_lo[s], p.pred_hi[s]);
    const StarJoinDev &j = p.joins[s - p.n_preds];
    int32_t pay = 0;
    bool hit = star_probe(j, v, pay);
    if (hit && j.f_bits > 0) hit = in_range(payload_field(pay, j.f_shift, j.f_mask, j.f_bits), j.f_lo, j.f_hi);
    return hit;
}

// BlockProbeHT of a direct table for a whole tile: presence bits for every
// item at once (dead items read entry 0), then the payload filter if any.
template <int IPT>
__device__ __forceinline__ uint32_t probe_direct_tile(const StarJoinDev &j, const uint32_t *bits,
                                                      const int32_t (&key)[IPT], uint32_t alive) {
    uint32_t word[IPT];
    uint32_t ok = 0;
    const uint32_t last = (uint32_t)(j.span - 1);  // span >= 1: off is in the table iff off <= last
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
        const uint32_t off = (uint32_t)key[k] - (uint32_t)j.key_min;
        const bool in = ((alive >> k) & 1u) && off <= last;
        ok |= (uint32_t)in << k;
        word[k] = bits[in ? (off >> 5) : 0u];
    }
    uint32_t hit = 0;
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
        const uint32_t off = (uint32_t)key[k] - (uint32_t)j.key_min;
        hit |= ((word[k] >> (off & 31u)) & 1u) << k;
    }
    hit &= ok;
    if (j.f_bits == 0) return hit;
    int32_t pay[IPT];
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
        const uint32_t off = (uint32_t)key[k] - (uint32_t)j.key_min;
        pay[k] = j.payload[((hit >> k) & 1u) ? off : 0u];
    }
    uint32_t pass = 0;
#pragma unroll
    for (int k = 0; k < IPT; ++k)
        pass |= (uint32_t)in_range(payload_field(pay[k], j.f_shift, j.f_mask, j.f_bits), j.f_lo, j.f_hi) << k;
    return hit & pass;
}

template <int IPT>
__device__ __forceinline__ uint32_t probe_linear_tile(const StarJoinDev &j, const int32_t (&key)[IPT],
                                                      uint32_t alive) {
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
        if (!((alive >> k) & 1u)) continue;
        int32_t pay = 0;
        bool hit = key[k] != kEmptyKey && probe_linear((const v2i *)j.slots, j.mask, j.shift, key[k], pay);
        if (hit && j.f_bits > 0) hit = in_range(payload_field(pay, j.f_shift, j.f_mask, j.f_bits), j.f_lo, j.f_hi);
        if (!hit) alive &= ~(1u << k);
    }
    return alive;
}

// Presence test of a whole tile against a bitmap staged in LDS.  `lds` is the
// workgroup's dynamic LDS, so every lookup is a ds_read (a pointer that might
// also point to global memory would compile to flat loads through the vector
// memory path).  The staged copy is followed by one zero word: a key's word
// index is clamped to it, so a key outside the table (or an item that is not
// alive) reads a valid LDS word and is masked afterwards, and the test needs
// no range compare.  The bit-field extract uses only the low five bits of its
// offset, so the bit is extracted at off with no masking of off.
__device__ __forceinline__ uint32_t staged_word_index(int32_t key, int32_t key_min, uint32_t words,
                                                      uint32_t &off) {
    off = (uint32_t)key - (uint32_t)key_min;
    const uint32_t w = off >> 5;
    return w < words ? w : words;
}

template <int IPT>
__device__ __forceinline__ uint32_t probe_staged_tile(const uint32_t *lds, int32_t stage_off, int32_t key_min,
                                                      uint32_t words, const int32_t (&key)[IPT], uint32_t alive) {
    uint32_t word[IPT], off[IPT];
#pragma unroll
    for (int k = 0; k < IPT; ++k) word[k] = lds[stage_off + staged_word_index(key[k], key_min, words, off[k])];
    uint32_t hit = 0;
#pragma unroll
    for (int k = 0; k < IPT; ++k) hit |= __builtin_amdgcn_ubfe(word[k], off[k], 1u) << k;  // bit off & 31
    return hit & alive;
}

// The LDS-staged presence test split in two, so that the registers holding
// the keys are free (and can receive the next tile's loads) while the
// ds_reads are in flight: begin() turns keys into word indices and bit
// positions and issues the reads; end() tests the bits.
template <int IPT>
struct StagedProbe {
    uint32_t word[IPT];
    uint32_t off[IPT];
    uint32_t alive;
    __device__ __forceinline__ void begin(const uint32_t *lds, int32_t stage_off, int32_t key_min, uint32_t words,
                                          const int32_t (&key)[IPT], uint32_t alive_in) {
        alive = alive_in;
#pragma unroll
        for (int k = 0; k < IPT; ++k) word[k] = lds[stage_off + staged_word_index(key[k], key_min, words, off[k])];
    }
    __device__ __forceinline__ uint32_t end() const {
        uint32_t hit = 0;
#pragma unroll
        for (int k = 0; k < IPT; ++k) hit |= __builtin_amdgcn_ubfe(word[k], off[k], 1u) << k;  // bit off & 31
        return hit & alive;
    }
};

// Words of a direct table's padded presence bitmap (the staged copy's zero
// word sits at this index).
__device__ __forceinline__ uint32_t bitmap_words_of(int64_t span) {
    return (uint32_t)(((span + 31) / 32 + 63) / 64 * 64);
}

// One dense step over a tile: a predicate, or a probe of the LDS-staged
// bitmap (stage_off >= 0), a direct table or a linear-probing table.
template <int IPT>
__device__ __forceinline__ uint32_t star_step_tile(const StarPlanDev &p, int s, const uint32_t *lds,
                                                   int32_t stage_off, const int32_t (&v)[IPT], uint32_t alive) {
    if (s < p.n_preds) return block_pred_range<IPT>(v, alive, p.pred_lo[s], p.pred_hi[s]);
    const StarJoinDev &j = p.joins[s - p.n_preds];
    if (stage_off >= 0) return probe_staged_tile<IPT>(lds, stage_off, j.key_min, bitmap_words_of(j.span), v, alive);
    if (j.kind == CRYSTAL_HT_DIRECT) return probe_direct_tile<IPT>(j, j.bitmap, v, alive);
    return probe_linear_tile<IPT>(j, v, alive);
}

// Group index and measure of one surviving row, added to the output (grouped)
// or to the thread's partial (scalar).
__device__ __forceinline__ void aggregate_row(const StarPlanDev &p, int64_t idx, uint64_t *__restrict__ out,
                                              uint64_t &scalar_acc, bool &bad_group) {
    int64_t g = 0;
    if (!p.scalar) {
        for (int jj = 0; jj < p.n_joins; ++jj) {
            const StarJoinDev &j = p.joins[jj];
            if (j.g_bits == 0) continue;
            int32_t pay = 0;
            star_probe(j, col_value(p, j.fk_col, idx), pay);
            g += ((int64_t)payload_field(pay, j.g_shift, j.g_mask, j.g_bits) - (int64_t)j.g_base) * j.g_stride;
        }
    }
    uint64_t val = 1;
    if (p.agg != CRYSTAL_AGG_COUNT) {
        const int64_t a = col_value(p, p.agg_col0, idx);
        if (p.agg == CRYSTAL_AGG_SUM) {
            val = (uint64_t)a;
        } else {
            const int64_t b = col_value(p, p.agg_col1, idx);
            val = p.agg == CRYSTAL_AGG_SUM_PRODUCT ? (uint64_t)(a * b) : (uint64_t)(a - b);
        }
    }
    if (p.scalar)
        scalar_acc += val;
    else if ((uint64_t)g < (uint64_t)p.n_groups)
        atomic_add_u64(out + g, val);
    else
        bad_group = true;
}

// Sparse phase for one queued row: the remaining steps, then the aggregate.
__device__ __forceinline__ void finish_row(const StarPlanDev &p, int dense, int64_t row,
                                           uint64_t *__restrict__ out, uint64_t &scalar_acc, bool &bad_group) {
    const int n_steps = p.n_preds + p.n_joins;
    for (int s = dense; s < n_steps; ++s)
        if (!star_step_row(p, s, col_value(p, step_col(p, s), row))) return;
    aggregate_row(p, row, out, scalar_acc, bad_group);
}

template <int BLOCK, int IPT, int NARROW>
__global__ __launch_bounds__(BLOCK) void star_kernel(const StarPlanDev p, uint64_t *__restrict__ out,
                                                     int32_t *status, int64_t n_tiles,
                                                     uint64_t *__restrict__ partials) {
    using T = TileShape<BLOCK, IPT>;
    static_assert(T::ITEMS <= 65536, "queue entries hold a 16-bit tile offset");
    __shared__ uint64_t red[T::WAVES];
    extern __shared__ v4i lds_dyn[];
    uint32_t *lds = reinterpret_cast<uint32_t *>(lds_dyn);

    const int n_steps = p.n_preds + p.n_joins;
    const int dense = n_steps < 2 ? n_steps : 2;
    // stage the dense steps' bitmaps (whole 64-word blocks, 16 bytes at a time)
    const int32_t so0 = dense >= 1 ? p.stage_off[0] : -1;
    const int32_t so1 = dense >= 2 ? p.stage_off[1] : -1;
    for (int d = 0; d < dense; ++d) {
        const int32_t so = d == 0 ? so0 : so1;
        if (so < 0) continue;
        const StarJoinDev &j = p.joins[d - p.n_preds];
        const int64_t n16 = bitmap_words_of(j.span) / 4;
        const v4i *src = reinterpret_cast<const v4i *>(j.bitmap);
        for (int64_t i = threadIdx.x; i < n16; i += BLOCK) lds_dyn[so / 4 + i] = src[i];
        if (threadIdx.x == 0) lds_dyn[so / 4 + n16] = v4i{0, 0, 0, 0};  // the zero word after the bitmap
    }
    // one survivor queue per wave: rows are compacted with ballots inside the
    // wave, so waves never wait for each other
    const uint32_t lane = lane_id();
    const uint32_t qmask = (uint32_t)p.queue_cap - 1u;
    uint32_t *queue = lds + p.queue_off + (threadIdx.x / kWave) * p.queue_cap;
    __syncthreads();

    uint64_t scalar_acc = 0;
    bool bad_group = false;
    uint32_t head = 0, tail = 0;  // queue cursors, equal in every lane of the wave
    const int64_t stride = gridDim.x;
    const ColDev cd0 = p.col[dense >= 1 ? step_col(p, 0) : 0];
    const ColDev cd1 = p.col[dense >= 2 ? step_col(p, 1) : 0];

    // Pipeline over this workgroup's tiles t_0, t_1, ...: an iteration runs
    // the first step of t_{k+1} and the second step of t_k, then issues the
    // second-step loads of t_{k+1} and the first-step loads of t_{k+2}, and
    // queues the rows of t_k still alive.  Each column has one register
    // buffer, reloaded once the step that reads it is done, so that more
    // waves fit on a SIMD.
    int64_t t_cur = blockIdx.x;
    uint32_t k_cur = 0;        // position of t_cur in this workgroup's tile sequence
    uint32_t alive_c = 0;

    // finish the queue 64 rows at a time
    auto drain = [&]() {
        __builtin_amdgcn_wave_barrier();
        while (tail - head >= (uint32_t)kWave) {
            const uint32_t e = queue[(head + lane) & qmask];
            const int64_t row = ((int64_t)blockIdx.x + (int64_t)(e >> 16) * stride) * T::ITEMS + (e & 0xffffu);
            finish_row(p, dense, row, out, scalar_acc, bad_group);
            head += kWave;
        }
        __builtin_amdgcn_wave_barrier();
    };
    // compact the wave's live rows of the current tile into its queue, half a
    // tile at a time, draining in between (so the queue holds fewer than 64
    // rows plus half a tile's share of the wave)
    auto enqueue = [&]() {
        constexpr int HALF = IPT >= 8 ? IPT / 2 : IPT;
#pragma unroll
        for (int h = 0; h < IPT; h += HALF) {
            const uint32_t part = alive_c & ((HALF == 32 ? 0xffffffffu : ((1u << HALF) - 1u)) << h);
            uint32_t total;
            const uint32_t off = wave_exclusive_scan_small<T::CBITS>((uint32_t)__popc(part), total);
            if (total) {
                uint32_t pos = tail + off;
                uint32_t m = part;
                while (m) {
                    const int k = __builtin_ctz(m);
                    m &= m - 1u;
                    const uint32_t local = (uint32_t)(((k / T::VEC) * BLOCK + threadIdx.x) * T::VEC + (k % T::VEC));
                    queue[pos & qmask] = (k_cur << 16) | local;
                    ++pos;
                }
                tail += total;
                drain();
            }
        }
    };

    if constexpr (NARROW == 2 || NARROW == 3) {
        // narrow and bit-packed columns: the buffers hold the loaded words,
        // decoded where a step uses them
        RawTile<IPT, NARROW> a, b;
        if (t_cur < n_tiles) {
            alive_c = valid_mask<BLOCK, IPT>(t_cur * T::ITEMS, p.n_rows);
            if (dense >= 1) {
                load_raw_tile<BLOCK, IPT, NARROW>(cd0, p.n_rows, t_cur * T::ITEMS, false, 0u, a);
                int32_t v[IPT];
                decode_tile<BLOCK, IPT, NARROW>(cd0, t_cur * T::ITEMS, a, v);
                alive_c = star_step_tile<IPT>(p, 0, lds, so0, v, alive_c);
            }
            if (dense >= 2) load_raw_tile<BLOCK, IPT, NARROW>(cd1, p.n_rows, t_cur * T::ITEMS, true, alive_c, b);
            if (dense >= 1 && t_cur + stride < n_tiles)
                load_raw_tile<BLOCK, IPT, NARROW>(cd0, p.n_rows, (t_cur + stride) * T::ITEMS, false, 0u, a);
        }
        if (t_cur < n_tiles) {
            for (;;) {
                const int64_t t_nxt = t_cur + stride;
                const bool has_nxt = t_nxt < n_tiles;
                uint32_t alive_n = 0;
                if (has_nxt) {
                    alive_n = valid_mask<BLOCK, IPT>(t_nxt * T::ITEMS, p.n_rows);
                    if (dense >= 1) {
                        int32_t v[IPT];
                        decode_tile<BLOCK, IPT, NARROW>(cd0, t_nxt * T::ITEMS, a, v);
                        if (t_nxt + stride < n_tiles)
                            load_raw_tile<BLOCK, IPT, NARROW>(cd0, p.n_rows, (t_nxt + stride) * T::ITEMS, false, 0u, a);
                        alive_n = star_step_tile<IPT>(p, 0, lds, so0, v, alive_n);
                    }
                }
                if (dense >= 2) {
                    int32_t v[IPT];
                    decode_tile<BLOCK, IPT, NARROW>(cd1, t_cur * T::ITEMS, b, v);
                    if (has_nxt) load_raw_tile<BLOCK, IPT, NARROW>(cd1, p.n_rows, t_nxt * T::ITEMS, true, alive_n, b);
                    alive_c = star_step_tile<IPT>(p, 1, lds, so1, v, alive_c);
                }
                enqueue();
                if (!has_nxt) break;
                t_cur = t_nxt;
                ++k_cur;
                alive_c = alive_n;
            }
        }
    } else {
        int32_t a[IPT];  // first-step column of the next tile
        int32_t b[IPT];  // second-step column of the current tile
        if (t_cur < n_tiles) {
            alive_c = valid_mask<BLOCK, IPT>(t_cur * T::ITEMS, p.n_rows);
            if (dense >= 1) {
                load_col_tile<BLOCK, IPT, NARROW>(cd0, p.n_rows, t_cur * T::ITEMS, a);
                alive_c = star_step_tile<IPT>(p, 0, lds, so0, a, alive_c);
            }
            if (dense >= 2) load_col_tile_sel<BLOCK, IPT, NARROW>(cd1, p.n_rows, t_cur * T::ITEMS, alive_c, b);
            if (dense >= 1 && t_cur + stride < n_tiles)
                load_col_tile<BLOCK, IPT, NARROW>(cd0, p.n_rows, (t_cur + stride) * T::ITEMS, a);
        }
        if (t_cur < n_tiles) {
            for (;;) {
                const int64_t t_nxt = t_cur + stride;
                const bool has_nxt = t_nxt < n_tiles;
                uint32_t alive_n = 0;
                if (has_nxt) {
                    alive_n = valid_mask<BLOCK, IPT>(t_nxt * T::ITEMS, p.n_rows);
                    if (dense >= 1) alive_n = star_step_tile<IPT>(p, 0, lds, so0, a, alive_n);
                }
                if (dense >= 2) alive_c = star_step_tile<IPT>(p, 1, lds, so1, b, alive_c);
                if (has_nxt) {
                    if (dense >= 2) load_col_tile_sel<BLOCK, IPT, NARROW>(cd1, p.n_rows, t_nxt * T::ITEMS, alive_n, b);
                    if (dense >= 1 && t_nxt + stride < n_tiles)
                        load_col_tile<BLOCK, IPT, NARROW>(cd0, p.n_rows, (t_nxt + stride) * T::ITEMS, a);
                }
                enqueue();
                if (!has_nxt) break;
                t_cur = t_nxt;
                ++k_cur;
                alive_c = alive_n;
            }
        }
    }
    if (lane < tail - head) {
        const uint32_t e = queue[(head + lane) & qmask];
        const int64_t row = ((int64_t)blockIdx.x + (int64_t)(e >> 16) * stride) * T::ITEMS + (e & 0xffffu);
        finish_row(p, dense, row, out, scalar_acc, bad_group);
    }
    if (bad_group) set_status(status, CRYSTAL_ERANGE);
    if (p.scalar) {
        const uint64_t t = block_sum_u64<BLOCK>(scalar_acc, red);
        if (threadIdx.x == 0) partials[blockIdx.x] = t;
    }
}

// Sum of the per-workgroup partials of a scalar query.
__global__ __launch_bounds__(256) void star_finalize_kernel(const uint64_t *__restrict__ partials, int64_t n,
                                                            uint64_t *__restrict__ out, int accumulate) {
    __shared__ uint64_t red[4];
    uint64_t s = 0;
    for (int64_t i = threadIdx.x; i < n; i += 256) s += partials[i];
    s = block_sum_u64<256>(s, red);
    if (threadIdx.x == 0) out[0] = accumulate ? out[0] + s : s;
}

// ------------------------------------------------------------------ host ---
static constexpr int64_t kStageBytesPerStep = 32768;

static int64_t bitmap_bytes(const StarJoinDev &j) { return ((j.span + 31) / 32 + 63) / 64 * 64 * 4; }

// Smallest tile is 64 x 4 rows; the grid also grows so that no workgroup
// handles more than 65535 tiles (queue entries hold a 16-bit tile index).
int64_t star_max_grid(int64_t n_rows) {
    const int64_t resident = (int64_t)kStarMaxGridPerCu * device_cu_count();
    const int64_t by_index = ((n_rows + 255) / 256 + 65534) / 65535;
    return resident > by_index ? resident : by_index;
}

template <int BLOCK, int IPT>
static hipError_t star_t(const LaunchCfg &cfg, StarPlanDev p, uint64_t *out, int32_t *status,
                         uint64_t *partials, bool accumulate, hipStream_t s) {
    using T = TileShape<BLOCK, IPT>;
    const int64_t n_tiles = (p.n_rows + T::ITEMS - 1) / T::ITEMS;
    // LDS: staged bitmaps of presence-only direct joins among the dense steps, then the queue
    const int n_steps = p.n_preds + p.n_joins;
    const int dense = n_steps < 2 ? n_steps : 2;
    int64_t words = 0;
    for (int d = 0; d < 2; ++d) {
        p.stage_off[d] = -1;
        if (d >= dense || d < p.n_preds) continue;
        const StarJoinDev &j = p.joins[d - p.n_preds];
        if (j.kind != CRYSTAL_HT_DIRECT || j.f_bits != 0 || bitmap_bytes(j) > kStageBytesPerStep) continue;
        p.stage_off[d] = (int32_t)words;
        words += bitmap_bytes(j) / 4 + 4;  // the bitmap, then one zero 16-byte chunk
    }
    // per-wave queue: half a tile's share of the wave (64 * IPT / 2 rows, or
    // the whole share below 8 items per thread) on top of fewer than 64 rows
    // left from earlier tiles
    int64_t qcap = 1;
    while (qcap < kWave + kWave * (IPT >= 8 ? IPT / 2 : IPT)) qcap <<= 1;
    p.queue_off = (int32_t)words;
    p.queue_cap = (int32_t)qcap;
    const int64_t lds_bytes = (words + qcap * T::WAVES) * 4;
    int n4 = 0, n2 = 0, nb = 0;
    for (int d = 0; d < dense; ++d) {
        const int c = d < p.n_preds ? p.pred_col[d] : p.joins[d - p.n_preds].fk_col;
        n4 += p.col[c].width == 4;
        n2 += p.col[c].width == 2;
        nb += p.col[c].bits > 0;
    }
    auto fn = n4 == dense   ? star_kernel<BLOCK, IPT, 0>
              : n2 == dense ? star_kernel<BLOCK, IPT, 2>
              : nb == dense ? star_kernel<BLOCK, IPT, 3>
                            : star_kernel<BLOCK, IPT, 1>;
    if (lds_bytes > 65536) {
        hipError_t e = hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)lds_bytes);
        if (e != hipSuccess) return e;
    }
    // workgroups: as many per CU as are resident at once (registers and LDS
    // permitting), or fewer if tuned; a persistent workgroup that is not
    // resident would start late and finish its tiles last
    int64_t per_cu = 0;
    hipError_t e = resident_per_cu((const void *)fn, BLOCK, lds_bytes, per_cu);
    if (e != hipSuccess) return e;
    if (cfg.grid_per_cu > 0 && cfg.grid_per_cu < per_cu) per_cu = cfg.grid_per_cu;
    if (per_cu > kStarMaxGridPerCu) per_cu = kStarMaxGridPerCu;
    if (per_cu < 1) per_cu = 1;
    int64_t grid = per_cu * device_cu_count();
    const int64_t min_grid = (n_tiles + 65534) / 65535;  // queue entries hold a 16-bit tile index
    if (grid < min_grid) grid = min_grid;
    if (grid > n_tiles) grid = n_tiles;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(fn, dim3((unsigned)grid), dim3(BLOCK), (size_t)lds_bytes, s, p, out, status, n_tiles,
                       partials);
    e = hipGetLastError();
    if (e != hipSuccess || !p.scalar) return e;
    hipLaunchKernelGGL(star_finalize_kernel, dim3(1), dim3(256), 0, s, partials, grid, out, accumulate ? 1 : 0);
    return hipGetLastError();
}

// Partials of scalar queries run without caller scratch
// (crystal_run_star_query_noalloc): one array per device, which the device
// holds until the process ends.  In host code `scratch` names a host-side
// stand-in, so kernels only ever receive the device address that
// hipGetSymbolAddress returned for the device current at the time.
static __device__ __align__(256) uint64_t scratch[kStarNoallocPartials];

hipError_t star_noalloc_partials(uint64_t **ptr) {
    static std::mutex mu;
    static uint64_t *addr[64];
    int d = -1;
    hipError_t e = hipGetDevice(&d);
    if (e != hipSuccess) return e;
    if (d < 0 || d >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[d]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[d] = (uint64_t *)p;
    }
    *ptr = addr[d];
    return hipSuccess;
}

hipError_t launch_star(const LaunchCfg &cfg, const StarPlanDev &plan, uint64_t *out, int32_t *status,
                       uint64_t *partials, bool accumulate, hipStream_t s) {
    if (!plan.scalar && !accumulate) {
        hipError_t e = fill_u64(out, plan.n_groups, 0ull, s);
        if (e != hipSuccess) return e;
    }
    if (plan.n_rows == 0) return plan.scalar && !accumulate ? fill_u64(out, 1, 0ull, s) : hipSuccess;
    switch (CRYSTAL_VARIANT_KEY(cfg.block, cfg.ipt)) {
#define X(B, I) \
    case CRYSTAL_VARIANT_KEY(B, I): return star_t<B, I>(cfg, plan, out, status, partials, accumulate, s);
        CRYSTAL_VARIANTS_VEC(X)
#undef X
    default: return hipErrorInvalidValue;
    }
}

}  // namespace crystal
