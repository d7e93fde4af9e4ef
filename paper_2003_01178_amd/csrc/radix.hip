// Radix partitioning and radix sort of 32-bit key / 32-bit value pairs
// (section 4.4).  A partition pass on radix r = bits and start bit a = shift
// places every pair into one of 2^r contiguous partitions by the digit
// (key >> a) & (2^r - 1).  It has the two phases of section 4.4:
//
//   histogram  each workgroup counts the digits of its contiguous chunk of
//              the input; one small kernel turns the digit x workgroup count
//              matrix into exclusive prefixes (digit-major), which are the
//              output offsets of every (digit, workgroup) run;
//   shuffle    each workgroup walks its chunk tile by tile and writes every
//              pair to its partition, advancing one running offset per digit.
//
// The shuffle is stable, also for 8-bit digits.  Within a tile each wave
// ranks its items per digit with ballots: the lanes whose digit equals the
// calling lane's are the AND over the digit's bits of ballot(bit) or its
// complement, so the rank of an item among equal digits is the number of
// such lanes below it plus a per-wave running count in LDS.  The tile is then
// sorted by digit in LDS and written out in that order, so consecutive lanes
// write consecutive addresses of one partition.  The section's GPU designs
// keep per-thread digit counters in registers, which limits a stable pass to
// 7 bits; the wave-level ranking needs no per-thread counters.
//
// Tile layout: a tile is BLOCK x IPT items; wave w owns the 64 * IPT
// consecutive items starting at w * 64 * IPT, and lane l's slot k is item
// k * 64 + l of that segment.  Processing slots in k order therefore visits
// a wave's items in input order, which is what makes the ranking stable.
// Every load instruction of a wave reads 256 consecutive bytes.
#include "block.hpp"
#include "internal.hpp"
#include "variants.hpp"

namespace crystal {
namespace {

constexpr int kBins = 256;  // digits of at most 8 bits

template <int BLOCK, int IPT>
struct RadixTile {
    static_assert(BLOCK >= kBins, "one thread per digit");
    static constexpr int W = BLOCK / kWave;
    static constexpr int ITEMS = BLOCK * IPT;
    __device__ static __forceinline__ int offset(int k) {
        return (int)(threadIdx.x / kWave) * (kWave * IPT) + k * kWave + (int)(threadIdx.x % kWave);
    }
};

__device__ __forceinline__ uint32_t digit_of(uint32_t key, int shift, uint32_t mask) {
    return (key >> shift) & mask;
}

// Inclusive prefix over the 64 lanes of a wave.
__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t x) {
    const int lane = (int)lane_id();
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        uint32_t y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    return x;
}

// Exclusive prefix of x over threads 0 .. BLOCK-1 in thread order; `tmp` holds
// one word per wave.  Every thread calls it.  With TRAIL it ends with a
// barrier, after which tmp may be reused; without, the caller must pass a
// barrier before tmp is written again.
template <int BLOCK, bool TRAIL = true>
__device__ __forceinline__ uint32_t block_exclusive_scan_u32(uint32_t x, uint32_t *tmp, uint32_t &total) {
    constexpr int W = BLOCK / kWave;
    const uint32_t inc = wave_inclusive_scan(x);
    const int w = threadIdx.x / kWave;
    if (lane_id() == kWave - 1) tmp[w] = inc;
    __syncthreads();
    uint32_t before = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < W; ++i) {
        uint32_t t = tmp[i];
        before += i < w ? t : 0u;
        tot += t;
    }
    total = tot;
    if (TRAIL) __syncthreads();
    return before + inc - x;
}

// Tiles [t0, t1) of the chunk that column `col` of the count matrix covers.
struct Chunk {
    int64_t t0, t1;
};

__device__ __forceinline__ Chunk chunk_of(int64_t col, int sub, int64_t tiles_per_block, int64_t n_tiles) {
    const int64_t b = col / sub, j = col % sub;
    const int64_t per_sub = (tiles_per_block + sub - 1) / sub;
    int64_t end = (b + 1) * tiles_per_block;
    if (end > n_tiles) end = n_tiles;
    int64_t t0 = b * tiles_per_block + j * per_sub;
    int64_t t1 = t0 + per_sub;
    if (t0 > end) t0 = end;
    if (t1 > end) t1 = end;
    return {t0, t1};
}

// ------------------------------------------------------------- histogram --
// Column c of the count matrix counts the digits of sub-chunk c (sub-chunks
// split each shuffle workgroup's chunk `sub` ways, in order; chunks are whole
// shuffle tiles of tile_items items).  MATRIX: write counts[d * cols + c];
// otherwise add into the global histogram counts[d].  The counting workgroup
// has its own shape: kHistBlock threads reading kHistIpt coalesced words each
// per step, with one LDS digit histogram per wave.
constexpr int kHistBlock = 256;
constexpr int kHistIpt = 16;

template <bool MATRIX>
__global__ __launch_bounds__(kHistBlock) void radix_hist_kernel(const uint32_t *__restrict__ keys, int64_t n,
                                                                int shift, uint32_t mask, int64_t tile_items,
                                                                int64_t n_tiles, int64_t tiles_per_block, int sub,
                                                                uint32_t *__restrict__ counts, int64_t cols) {
    constexpr int W = kHistBlock / kWave;
    constexpr int STEP = kHistBlock * kHistIpt;
    __shared__ uint32_t h[W][kBins];
    for (int i = threadIdx.x; i < W * kBins; i += kHistBlock) (&h[0][0])[i] = 0u;
    __syncthreads();
    const int w = threadIdx.x / kWave;
    const Chunk ch = chunk_of(blockIdx.x, sub, tiles_per_block, n_tiles);
    const int64_t i0 = ch.t0 * tile_items;
    int64_t i1 = ch.t1 * tile_items;
    if (i1 > n) i1 = n;
    // full batches of STEP keys, the next batch's loads in flight while the
    // current one is counted (two register buffers, so that the one receiving
    // loads is never copied); then the partial batch
    const int64_t nfull = i1 > i0 ? (i1 - i0) / STEP : 0;
    auto load = [&](int64_t bi, uint32_t(&v)[kHistIpt]) {
        const uint32_t *kb = keys + i0 + bi * STEP;
        asm volatile("" : "+s"(kb));
#pragma unroll
        for (int k = 0; k < kHistIpt; ++k) v[k] = __builtin_nontemporal_load(kb + k * kHistBlock + threadIdx.x);
    };
    auto count = [&](const uint32_t(&v)[kHistIpt]) {
#pragma unroll
        for (int k = 0; k < kHistIpt; ++k) atomicAdd(&h[w][digit_of(v[k], shift, mask)], 1u);
    };
    uint32_t va[kHistIpt], vb[kHistIpt];
    if (nfull > 0) load(0, va);
    for (int64_t bi = 0; bi < nfull;) {
        if (bi + 1 < nfull) load(bi + 1, vb);
        count(va);
        if (++bi >= nfull) break;
        if (bi + 1 < nfull) load(bi + 1, va);
        count(vb);
        ++bi;
    }
    const int64_t b = i0 + nfull * STEP;
    if (b < i1) {
        const uint32_t *kb = keys + b;
        const int64_t left = i1 - b;
#pragma unroll
        for (int k = 0; k < kHistIpt; ++k) {
            const int i = k * kHistBlock + (int)threadIdx.x;
            if (i < left) atomicAdd(&h[w][digit_of(kb[i], shift, mask)], 1u);
        }
    }
    __syncthreads();
    const int d = threadIdx.x;
    if (d < kBins && (uint32_t)d <= mask) {
        uint32_t s = 0;
#pragma unroll
        for (int i = 0; i < W; ++i) s += h[i][d];
        if (MATRIX)
            counts[(int64_t)d * cols + blockIdx.x] = s;
        else if (s)
            atomicAdd(&counts[d], s);
    }
}

// Row d of the count matrix becomes its exclusive prefix; totals[d] = row sum.
constexpr int kScanBlock = 1024;

__global__ __launch_bounds__(kScanBlock) void radix_scan_kernel(uint32_t *__restrict__ counts, int64_t cols,
                                                                uint32_t *__restrict__ totals) {
    __shared__ uint32_t tmp[kScanBlock / kWave];
    uint32_t *row = counts + (int64_t)blockIdx.x * cols;
    const int64_t per = (cols + kScanBlock - 1) / kScanBlock;
    const int64_t c0 = (int64_t)threadIdx.x * per;
    int64_t c1 = c0 + per;
    if (c1 > cols) c1 = cols;
    uint32_t s = 0;
    for (int64_t c = c0; c < c1; ++c) s += row[c];
    uint32_t total;
    uint32_t run = block_exclusive_scan_u32<kScanBlock>(s, tmp, total);
    for (int64_t c = c0; c < c1; ++c) {
        uint32_t v = row[c];
        row[c] = run;
        run += v;
    }
    if (threadIdx.x == 0) totals[blockIdx.x] = total;
}

// --------------------------------------------------------------- shuffle --
template <int BLOCK, int IPT, bool VALS>
struct ShuffleLds {
    static constexpr int W = BLOCK / kWave;
    static constexpr int ITEMS = BLOCK * IPT;
    // word offsets
    static constexpr int KEYS = 0;
    static constexpr int VALSO = KEYS + ITEMS;
    static constexpr int WC = VALSO + (VALS ? ITEMS : 0);  // [W][kBins]
    static constexpr int GBASE = WC + W * kBins;           // [kBins]
    static constexpr int RUN = GBASE + kBins;              // [kBins]
    static constexpr int TMP = RUN + kBins;                // [W]
    static constexpr int WORDS = TMP + W;
    static constexpr size_t BYTES = (size_t)WORDS * 4;
};

// The tile starting at `base`: slot k of this lane is item off0 + 64 k.  The
// tile's base pointers are made opaque to the compiler so that it addresses
// every item from one scalar base and one lane offset, instead of carrying a
// 64-bit address per item from tile to tile.
template <int BLOCK, int IPT, bool VALS>
__device__ __forceinline__ void load_tile(const uint32_t *__restrict__ keys, const uint32_t *__restrict__ vals,
                                          int64_t base, int rem, int off0, uint32_t (&key)[IPT],
                                          uint32_t (&val)[IPT]) {
    using RT = RadixTile<BLOCK, IPT>;
    // base is uniform; readfirstlane states it, so that the scalar constraint
    // below holds wherever the compiler places this call
    base = ((int64_t)__builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)base >> 32)) << 32) |
           (int64_t)(uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)base);
    const uint32_t *kb = keys + base;
    const uint32_t *vb = VALS ? vals + base : nullptr;
    asm volatile("" : "+s"(kb));
    if (VALS) asm volatile("" : "+s"(vb));
    if (rem >= RT::ITEMS) {
#pragma unroll
        for (int k = 0; k < IPT; ++k) {
            key[k] = __builtin_nontemporal_load(kb + off0 + k * kWave);
            if (VALS) val[k] = __builtin_nontemporal_load(vb + off0 + k * kWave);
        }
    } else {
#pragma unroll
        for (int k = 0; k < IPT; ++k) {
            const int i = off0 + k * kWave;
            key[k] = i < rem ? kb[i] : 0u;
            if (VALS) val[k] = i < rem ? vb[i] : 0u;
        }
    }
}

// One workgroup per chunk of tiles_per_block tiles (the chunks the count
// matrix's columns b * sub .. b * sub + sub - 1 counted).  STABLE: ballot
// ranking in input order; otherwise every item takes its rank from an LDS
// atomic on its wave's digit counter, which orders equal digits of one load
// arbitrarily (the unstable shuffle of section 4.4) for far fewer
// instructions per item.
template <int BLOCK, int IPT, bool VALS, bool STABLE>
__global__ __launch_bounds__(BLOCK) void radix_shuffle_kernel(
    const uint32_t *__restrict__ keys, const uint32_t *__restrict__ vals, int64_t n, int shift, uint32_t mask,
    int64_t n_tiles, int64_t tiles_per_block, int sub, const uint32_t *__restrict__ counts, int64_t cols,
    const uint32_t *__restrict__ totals, uint32_t *__restrict__ out_keys, uint32_t *__restrict__ out_vals,
    uint32_t *__restrict__ part_offsets) {
    using RT = RadixTile<BLOCK, IPT>;
    using L = ShuffleLds<BLOCK, IPT, VALS>;
    extern __shared__ uint32_t lds[];
    uint32_t *s_keys = lds + L::KEYS;
    uint32_t *s_vals = lds + L::VALSO;
    uint32_t *s_wc = lds + L::WC;
    uint32_t *s_gbase = lds + L::GBASE;
    uint32_t *s_run = lds + L::RUN;
    uint32_t *s_tmp = lds + L::TMP;

    const int tid = threadIdx.x;
    const int w = tid / kWave;
    uint32_t *my_wc = s_wc + w * kBins;

    // partition starts: exclusive prefix of the digit totals
    uint32_t unused;
    const uint32_t tot = (tid < kBins && (uint32_t)tid <= mask) ? totals[tid] : 0u;
    const uint32_t dstart = block_exclusive_scan_u32<BLOCK>(tot, s_tmp, unused);
    if (tid < kBins) {
        if ((uint32_t)tid <= mask) {
            s_run[tid] = dstart + counts[(int64_t)tid * cols + (int64_t)blockIdx.x * sub];
            if (blockIdx.x == 0 && part_offsets) part_offsets[tid] = dstart;
        }
    }
    if (blockIdx.x == 0 && part_offsets && tid == 0) part_offsets[mask + 1] = (uint32_t)n;
    __syncthreads();

    int64_t t0 = (int64_t)blockIdx.x * tiles_per_block;
    int64_t t1 = t0 + tiles_per_block;
    if (t1 > n_tiles) t1 = n_tiles;
    if (t0 >= t1) return;

    // slot k of this lane sits at tile offset off0 + 64 k
    const int off0 = RT::offset(0);
    auto items_from = [&](int64_t b) { return n - b >= RT::ITEMS ? RT::ITEMS : (int)(n - b); };
    uint32_t key[IPT], val[IPT];
    load_tile<BLOCK, IPT, VALS>(keys, vals, t0 * RT::ITEMS, items_from(t0 * RT::ITEMS), off0, key, val);
    for (int64_t t = t0; t < t1; ++t) {
        const int64_t base = t * RT::ITEMS;
        const int rem = items_from(base);  // items in this tile
        int tidv = tid;                    // opaque: keeps per-item offsets out of registers
        asm volatile("" : "+v"(tidv));
        // 1. rank every item among the wave's earlier items of its digit.  The
        //    wave clears its own counter row first: the previous tile last read
        //    it in this wave (step 3) and in the digit scan before that tile's
        //    scatter barrier, so no barrier is needed after the write-out, and a
        //    wave done writing ranks the next tile while others still write.
#pragma unroll
        for (int q = 0; q < kBins / kWave; ++q) my_wc[q * kWave + (int)lane_id()] = 0u;
        uint32_t rank[IPT];
        if constexpr (!STABLE) {
#pragma unroll
            for (int k = 0; k < IPT; ++k) {
                rank[k] = 0;
                if (off0 + k * kWave < rem) rank[k] = atomicAdd(&my_wc[digit_of(key[k], shift, mask)], 1u);
            }
        } else
#pragma unroll
        for (int k = 0; k < IPT; ++k) {
            const bool valid = off0 + k * kWave < rem;
            const uint32_t d = digit_of(key[k], shift, mask);
            // lanes whose digit differs from this lane's in some bit
            uint64_t diff = 0;
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                const bool bit = (d >> b) & 1u;
                const uint64_t m = ballot(bit);
                diff |= bit ? ~m : m;
            }
            const uint64_t peers = ballot(valid) & ~diff;
            const uint32_t below = count_below(peers);
            const uint32_t same = (uint32_t)__popcll(peers);
            rank[k] = 0;
            if (valid) {
                const uint32_t c = my_wc[d];
                rank[k] = c + below;
                if (below + 1 == same) my_wc[d] = c + same;
            }
            // one slot at a time: interleaving slots only raises register pressure,
            // since each slot waits for the previous slot's counter update anyway
            __builtin_amdgcn_sched_barrier(0);
        }
        __syncthreads();
        // 2. per digit: offsets of each wave's run inside the tile's run of
        //    that digit, the tile's digit starts, and the global base
        uint32_t cnt = 0;
        if (tid < kBins) {
#pragma unroll
            for (int i = 0; i < RT::W; ++i) {
                const uint32_t c = s_wc[i * kBins + tid];
                s_wc[i * kBins + tid] = cnt;
                cnt += c;
            }
        }
        // no trailing barrier: s_tmp is next written after this tile's later barriers
        const uint32_t tstart = block_exclusive_scan_u32<BLOCK, false>(cnt, s_tmp, unused);
        if (tid < kBins) {
#pragma unroll
            for (int i = 0; i < RT::W; ++i) s_wc[i * kBins + tid] += tstart;
            const uint32_t run = s_run[tid];
            s_gbase[tid] = run - tstart;
            s_run[tid] = run + cnt;
        }
        __syncthreads();
        // 3. the tile, sorted by digit (stable), into LDS
#pragma unroll
        for (int k = 0; k < IPT; ++k) {
            if (off0 + k * kWave < rem) {
                const uint32_t p = my_wc[digit_of(key[k], shift, mask)] + rank[k];
                s_keys[p] = key[k];
                if (VALS) s_vals[p] = val[k];
            }
        }
        __syncthreads();
        // 4. next tile's loads go out while this one is written
        if (t + 1 < t1)
            load_tile<BLOCK, IPT, VALS>(keys, vals, base + RT::ITEMS, items_from(base + RT::ITEMS), off0, key, val);
#pragma unroll
        for (int j = 0; j < IPT; ++j) {
            const int p = j * BLOCK + tidv;
            if (p < rem) {
                const uint32_t k = s_keys[p];
                const uint32_t g = s_gbase[digit_of(k, shift, mask)] + (uint32_t)p;  // < n < 2^32
                out_keys[g] = k;
                if (VALS) out_vals[g] = s_vals[p];
            }
            if (j % 4 == 3) __builtin_amdgcn_sched_barrier(0);
        }
        // no barrier: the next tile writes s_gbase, s_run, s_tmp and the LDS
        // tile only after its ranking barrier, which every wave reaches after
        // finishing this write-out
    }
}

// ---------------------------------------------------------------- launch --
struct RadixGeom {
    int64_t n_tiles, tiles_per_block, grid, cols;
    int sub;
};

template <int BLOCK, int IPT>
struct RadixKernels {
    template <bool VALS, bool STABLE>
    static hipError_t prepare_one() {
        static bool done = false;
        if (done) return hipSuccess;
        hipError_t e = hipFuncSetAttribute((const void *)radix_shuffle_kernel<BLOCK, IPT, VALS, STABLE>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)ShuffleLds<BLOCK, IPT, VALS>::BYTES);
        if (e == hipSuccess) done = true;
        return e;
    }

    static hipError_t histogram(const uint32_t *keys, int64_t n, int shift, uint32_t mask, const RadixGeom &g,
                                uint32_t *counts, bool matrix, hipStream_t s) {
        const dim3 grid((unsigned)(g.grid * g.sub)), block(kHistBlock);
        const int64_t items = (int64_t)BLOCK * IPT;
        if (matrix)
            hipLaunchKernelGGL((radix_hist_kernel<true>), grid, block, 0, s, keys, n, shift, mask, items,
                               g.n_tiles, g.tiles_per_block, g.sub, counts, g.cols);
        else
            hipLaunchKernelGGL((radix_hist_kernel<false>), grid, block, 0, s, keys, n, shift, mask, items,
                               g.n_tiles, g.tiles_per_block, g.sub, counts, g.cols);
        return hipGetLastError();
    }

    template <bool VALS, bool STABLE>
    static hipError_t shuffle_t(const uint32_t *keys, const uint32_t *vals, int64_t n, int shift, uint32_t mask,
                                const RadixGeom &g, const uint32_t *counts, const uint32_t *totals, uint32_t *ok,
                                uint32_t *ov, uint32_t *part_offsets, hipStream_t s) {
        hipError_t e = prepare_one<VALS, STABLE>();
        if (e != hipSuccess) return e;
        const size_t lds = ShuffleLds<BLOCK, IPT, VALS>::BYTES;
        hipLaunchKernelGGL((radix_shuffle_kernel<BLOCK, IPT, VALS, STABLE>), dim3((unsigned)g.grid), dim3(BLOCK),
                           lds, s, keys, vals, n, shift, mask, g.n_tiles, g.tiles_per_block, g.sub, counts, g.cols,
                           totals, ok, ov, part_offsets);
        return hipGetLastError();
    }

    static hipError_t shuffle(const uint32_t *keys, const uint32_t *vals, int64_t n, int shift, uint32_t mask,
                              const RadixGeom &g, const uint32_t *counts, const uint32_t *totals,
                              uint32_t *ok, uint32_t *ov, uint32_t *part_offsets, bool stable, hipStream_t s) {
        if (vals)
            return stable ? shuffle_t<true, true>(keys, vals, n, shift, mask, g, counts, totals, ok, ov, part_offsets, s)
                          : shuffle_t<true, false>(keys, vals, n, shift, mask, g, counts, totals, ok, ov,
                                                   part_offsets, s);
        return stable ? shuffle_t<false, true>(keys, vals, n, shift, mask, g, counts, totals, ok, ov, part_offsets, s)
                      : shuffle_t<false, false>(keys, vals, n, shift, mask, g, counts, totals, ok, ov, part_offsets, s);
    }
};

size_t shuffle_lds_bytes(int block, int ipt) {
    switch (CRYSTAL_VARIANT_KEY(block, ipt)) {
#define X(B, I) \
    case CRYSTAL_VARIANT_KEY(B, I): return ShuffleLds<B, I, true>::BYTES;
        CRYSTAL_VARIANTS_RADIX(X)
#undef X
    default: return 0;
    }
}

// Workgroups of the shuffle kernel per CU: the tuned value, else as many as
// the LDS allows (at most 8).
RadixGeom geometry(const LaunchCfg &cfg, int64_t n) {
    RadixGeom g{};
    const int64_t items = (int64_t)cfg.block * cfg.ipt;
    g.n_tiles = (n + items - 1) / items;
    int per_cu = cfg.grid_per_cu;
    if (per_cu <= 0) {
        const size_t lds = shuffle_lds_bytes(cfg.block, cfg.ipt);
        per_cu = lds ? (int)(device_lds_per_cu() / (int64_t)lds) : 1;
        if (per_cu < 1) per_cu = 1;
        if (per_cu > 8) per_cu = 8;
    }
    const int64_t cus = device_cu_count();
    int64_t grid = (int64_t)per_cu * cus;
    if (grid > g.n_tiles) grid = g.n_tiles;
    if (grid < 1) grid = 1;
    g.tiles_per_block = (g.n_tiles + grid - 1) / grid;
    g.grid = (g.n_tiles + g.tiles_per_block - 1) / g.tiles_per_block;
    if (g.grid < 1) g.grid = 1;
    // the histogram pass splits each chunk so that about 8 workgroups per CU count
    int64_t sub = (8 * cus + g.grid - 1) / g.grid;
    if (sub > g.tiles_per_block) sub = g.tiles_per_block;
    if (sub < 1) sub = 1;
    g.sub = (int)sub;
    g.cols = g.grid * g.sub;
    return g;
}

}  // namespace

// Scratch of one partition pass: the count matrix (kBins rows of cols words,
// 256-byte aligned) and the digit totals.
int64_t radix_pass_scratch_bytes(const LaunchCfg &cfg, int64_t n) {
    const RadixGeom g = geometry(cfg, n > 0 ? n : 1);
    return ((int64_t)kBins * g.cols * 4 + 255) / 256 * 256 + kBins * 4;
}

bool radix_variant_fits(int block, int ipt) {
    const size_t b = shuffle_lds_bytes(block, ipt);
    return b > 0 && (int64_t)b <= device_lds_per_block();
}

#define RADIX_DISPATCH(cfg, CALL)                                               \
    switch (CRYSTAL_VARIANT_KEY(cfg.block, cfg.ipt)) {                         \
        CRYSTAL_VARIANTS_RADIX(CALL)                                           \
    default: return hipErrorInvalidValue;                                      \
    }

hipError_t launch_radix_histogram(const LaunchCfg &cfg, const uint32_t *keys, int64_t n, int shift, int bits,
                                  uint32_t *hist, hipStream_t s) {
    const uint32_t mask = (1u << bits) - 1u;
    hipError_t e = fill_u32(hist, (int64_t)mask + 1, 0u, s);
    if (e != hipSuccess || n == 0) return e;
    const RadixGeom g = geometry(cfg, n);
#define X(B, I) \
    case CRYSTAL_VARIANT_KEY(B, I): return RadixKernels<B, I>::histogram(keys, n, shift, mask, g, hist, false, s);
    RADIX_DISPATCH(cfg, X)
#undef X
}

hipError_t launch_radix_partition(const LaunchCfg &cfg, const uint32_t *keys, const uint32_t *vals, int64_t n,
                                  int shift, int bits, uint32_t *out_keys, uint32_t *out_vals,
                                  uint32_t *part_offsets, void *scratch, bool stable, hipStream_t s) {
    const uint32_t mask = (1u << bits) - 1u;
    if (n == 0) return part_offsets ? fill_u32(part_offsets, (int64_t)mask + 2, 0u, s) : hipSuccess;
    const RadixGeom g = geometry(cfg, n);
    uint32_t *counts = (uint32_t *)scratch;
    uint32_t *totals = (uint32_t *)((char *)scratch + ((int64_t)kBins * g.cols * 4 + 255) / 256 * 256);
    hipError_t e;
#define X(B, I)                                                                                     \
    case CRYSTAL_VARIANT_KEY(B, I):                                                                 \
        e = RadixKernels<B, I>::histogram(keys, n, shift, mask, g, counts, true, s);                \
        break;
    RADIX_DISPATCH(cfg, X)
#undef X
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(radix_scan_kernel, dim3(mask + 1), dim3(kScanBlock), 0, s, counts, g.cols, totals);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
#define X(B, I)                                                                                              \
    case CRYSTAL_VARIANT_KEY(B, I):                                                                          \
        return RadixKernels<B, I>::shuffle(keys, vals, n, shift, mask, g, counts, totals, out_keys, out_vals, \
                                           part_offsets, stable, s);
    RADIX_DISPATCH(cfg, X)
#undef X
}

}  // namespace crystal
