// Block-wide functions of the tile-based execution model (section 3.3,
// Table "List of block-wide functions"), rebuilt for CDNA4 wave64.
//
// A tile is BLOCK threads x IPT items.  Items live in registers.  A thread
// holds CHUNKS = IPT / VEC vectors of VEC consecutive items (VEC = 4 when
// IPT >= 4, so every vector is one 128-bit load).  Item (c, e) of thread t
// sits at tile offset (c * BLOCK + t) * VEC + e: for a fixed chunk c the
// workgroup's loads cover BLOCK * VEC * 4 contiguous bytes, so each wave's
// load instruction reads 1 KiB of consecutive memory.
//
// Per-item flags are a bitmask in one register (bit c * VEC + e), which is
// what BlockPred produces and BlockLoadSel consumes.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace crystal {

constexpr int kWave = 64;
constexpr int32_t kEmptyKey = INT32_MIN;

typedef int32_t v2i __attribute__((ext_vector_type(2)));
typedef int32_t v4i __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

template <int N> struct VecOf;
template <> struct VecOf<1> { typedef int32_t type; };
template <> struct VecOf<2> { typedef v2i type; };
template <> struct VecOf<4> { typedef v4i type; };

template <int BLOCK, int IPT>
struct TileShape {
    static_assert(BLOCK % kWave == 0, "workgroups are whole waves");
    static_assert(IPT == 1 || IPT == 2 || IPT % 4 == 0, "IPT is 1, 2 or a multiple of 4");
    static_assert(IPT <= 32, "the per-item mask is one 32-bit register");
    static constexpr int VEC = IPT >= 4 ? 4 : IPT;
    static constexpr int CHUNKS = IPT / VEC;
    static constexpr int ITEMS = BLOCK * IPT;
    static constexpr int WAVES = BLOCK / kWave;
    static constexpr uint32_t VMASK = (1u << VEC) - 1u;
    static constexpr uint32_t ALL = IPT == 32 ? 0xffffffffu : ((1u << IPT) - 1u);
    // bits needed for a per-thread count 0..IPT
    static constexpr int CBITS = IPT < 2 ? 1 : IPT < 4 ? 2 : IPT < 8 ? 3 : IPT < 16 ? 4 : IPT < 32 ? 5 : 6;

    __device__ static __forceinline__ int64_t index(int64_t base, int c, int e) {
        return base + ((int64_t)c * BLOCK + (int64_t)threadIdx.x) * VEC + e;
    }
};

// ---------------------------------------------------------------- lanes ----
__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// number of set bits of m in lanes below the calling lane (v_mbcnt)
__device__ __forceinline__ uint32_t count_below(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ uint32_t lane_id() { return count_below(~0ull); }

// ---------------------------------------------------------- BlockLoad ------
// Valid-item mask of a tile that starts at `base` in a column of n items.
template <int BLOCK, int IPT>
__device__ __forceinline__ uint32_t valid_mask(int64_t base, int64_t n) {
    using T = TileShape<BLOCK, IPT>;
    if (base + T::ITEMS <= n) return T::ALL;
    uint32_t m = 0;
#pragma unroll
    for (int c = 0; c < T::CHUNKS; ++c)
#pragma unroll
        for (int e = 0; e < T::VEC; ++e)
            if (T::index(base, c, e) < n) m |= 1u << (c * T::VEC + e);
    return m;
}

template <int VEC, bool NT>
__device__ __forceinline__ void load_vec(const int32_t *__restrict__ p, int32_t *dst) {
    typedef typename VecOf<VEC>::type V;
    V v;
    if (NT)
        v = __builtin_nontemporal_load(reinterpret_cast<const V *>(p));
    else
        v = *reinterpret_cast<const V *>(p);
    if constexpr (VEC == 1) {
        dst[0] = v;
    } else {
#pragma unroll
        for (int e = 0; e < VEC; ++e) dst[e] = v[e];
    }
}

// BlockLoad: the whole tile (full tiles with vector loads, the tail item by item).
template <int BLOCK, int IPT, bool NT>
__device__ __forceinline__ void block_load(const int32_t *__restrict__ col, int64_t base,
                                           int64_t n, int32_t (&v)[IPT]) {
    using T = TileShape<BLOCK, IPT>;
    if (base + T::ITEMS <= n) {
#pragma unroll
        for (int c = 0; c < T::CHUNKS; ++c)
            load_vec<T::VEC, NT>(col + T::index(base, c, 0), &v[c * T::VEC]);
    } else {
#pragma unroll
        for (int c = 0; c < T::CHUNKS; ++c)
#pragma unroll
            for (int e = 0; e < T::VEC; ++e) {
                int64_t i = T::index(base, c, e);
                v[c * T::VEC + e] = i < n ? col[i] : 0;
            }
    }
}

// BlockLoadSel: only the vectors that hold at least one flagged item are read
// (a 128-bit load touches the same cache line as any single item in it).
template <int BLOCK, int IPT, bool NT>
__device__ __forceinline__ void block_load_sel(const int32_t *__restrict__ col, int64_t base,
                                               int64_t n, uint32_t flags, int32_t (&v)[IPT]) {
    using T = TileShape<BLOCK, IPT>;
    const bool full = base + T::ITEMS <= n;
#pragma unroll
    for (int c = 0; c < T::CHUNKS; ++c) {
        uint32_t m = (flags >> (c * T::VEC)) & T::VMASK;
        if (!m) continue;
        if (full) {
            load_vec<T::VEC, NT>(col + T::index(base, c, 0), &v[c * T::VEC]);
        } else {
#pragma unroll
            for (int e = 0; e < T::VEC; ++e)
                if (m & (1u << e)) v[c * T::VEC + e] = col[T::index(base, c, e)];
        }
    }
}

// Narrow (frame-of-reference) columns: stored values are unsigned E offsets
// from cbase.  A thread's VEC consecutive items are one VEC * sizeof(E)-byte
// load; values are widened to int32 in registers.
template <typename E, int VEC, bool NT>
__device__ __forceinline__ void load_narrow_vec(const E *__restrict__ p, int32_t cbase, int32_t *dst) {
    if constexpr (VEC == 1) {
        dst[0] = cbase + (int32_t)(NT ? __builtin_nontemporal_load(p) : *p);
    } else {
        typedef E V __attribute__((ext_vector_type(VEC)));
        const V x = NT ? __builtin_nontemporal_load(reinterpret_cast<const V *>(p)) : *reinterpret_cast<const V *>(p);
#pragma unroll
        for (int e = 0; e < VEC; ++e) dst[e] = cbase + (int32_t)x[e];
    }
}

template <int BLOCK, int IPT, typename E, bool NT>
__device__ __forceinline__ void block_load_narrow(const E *__restrict__ col, int32_t cbase, int64_t base,
                                                  int64_t n, int32_t (&v)[IPT]) {
    using T = TileShape<BLOCK, IPT>;
    if (base + T::ITEMS <= n) {
#pragma unroll
        for (int c = 0; c < T::CHUNKS; ++c)
            load_narrow_vec<E, T::VEC, NT>(col + T::index(base, c, 0), cbase, &v[c * T::VEC]);
    } else {
#pragma unroll
        for (int c = 0; c < T::CHUNKS; ++c)
#pragma unroll
            for (int e = 0; e < T::VEC; ++e) {
                int64_t i = T::index(base, c, e);
                v[c * T::VEC + e] = i < n ? cbase + (int32_t)col[i] : 0;
            }
    }
}

template <int BLOCK, int IPT, typename E, bool NT>
__device__ __forceinline__ void block_load_sel_narrow(const E *__restrict__ col, int32_t cbase, int64_t base,
                                                      int64_t n, uint32_t flags, int32_t (&v)[IPT]) {
    using T = TileShape<BLOCK, IPT>;
    const bool full = base + T::ITEMS <= n;
#pragma unroll
    for (int c = 0; c < T::CHUNKS; ++c) {
        uint32_t m = (flags >> (c * T::VEC)) & T::VMASK;
        if (!m) continue;
        if (full) {
            load_narrow_vec<E, T::VEC, NT>(col + T::index(base, c, 0), cbase, &v[c * T::VEC]);
        } else {
#pragma unroll
            for (int e = 0; e < T::VEC; ++e)
                if (m & (1u << e)) v[c * T::VEC + e] = cbase + (int32_t)col[T::index(base, c, e)];
        }
    }
}

// Bit-packed (frame-of-reference) columns: a stream of 32-bit words, least
// significant bit first; row i's field occupies stream bits
// [i * bits, (i + 1) * bits), bits <= 16.  The buffer carries four zero words
// after the last field, so a reader may load whole words past it.

// Field of one row: the two words that hold it, funnel-shifted.
__device__ __forceinline__ int32_t packed_value(const uint32_t *__restrict__ w, int32_t cbase, uint32_t bits,
                                                int64_t row) {
    const uint64_t o = (uint64_t)row * bits;
    const uint32_t *p = w + (o >> 5);
    const uint32_t f = __builtin_amdgcn_alignbit(p[1], p[0], (uint32_t)o & 31u);
    return cbase + (int32_t)(f & ((1u << bits) - 1u));
}

// Four consecutive fields whose first starts at bit s (< 32) of the window
// x2:x1:x0 (4 * bits <= 64, so three words hold them).  Two funnel shifts
// move the window to bit 0 (fields at 0, b, 2b, 3b of y1:y0); one 64-bit
// shift by 2b <= 32 brings fields 2 and 3 down to 0 and b of z.  Only the
// low five bits of s are used.
__device__ __forceinline__ void decode_packed_vec4(uint32_t x0, uint32_t x1, uint32_t x2, uint32_t s, uint32_t bits,
                                                   int32_t cbase, int32_t *dst) {
    const uint32_t y0 = __builtin_amdgcn_alignbit(x1, x0, s);
    const uint32_t y1 = __builtin_amdgcn_alignbit(x2, x1, s);
    const uint32_t z = (uint32_t)((((uint64_t)y1 << 32) | y0) >> (2u * bits));
    const uint32_t mask = (1u << bits) - 1u;
    dst[0] = cbase + (int32_t)(y0 & mask);
    dst[1] = cbase + (int32_t)((y0 >> bits) & mask);
    dst[2] = cbase + (int32_t)(z & mask);
    dst[3] = cbase + (int32_t)((z >> bits) & mask);
}

// VEC = 4 consecutive rows starting at r0.
template <bool NT>
__device__ __forceinline__ void load_packed_vec4(const uint32_t *__restrict__ w, int32_t cbase, uint32_t bits,
                                                 int64_t r0, int32_t *dst) {
    const uint64_t o = (uint64_t)r0 * bits;
    const uint32_t *p = w + (o >> 5);
    const uint32_t x0 = NT ? __builtin_nontemporal_load(p) : p[0];
    const uint32_t x1 = NT ? __builtin_nontemporal_load(p + 1) : p[1];
    const uint32_t x2 = NT ? __builtin_nontemporal_load(p + 2) : p[2];
    decode_packed_vec4(x0, x1, x2, (uint32_t)o, bits, cbase, dst);
}

// BlockLoad / BlockLoadSel of a bit-packed column (VEC = 4 tiles only).
template <int BLOCK, int IPT, bool NT>
__device__ __forceinline__ void block_load_packed(const uint32_t *__restrict__ w, int32_t cbase, uint32_t bits,
                                                  int64_t base, int64_t n, int32_t (&v)[IPT]) {
    using T = TileShape<BLOCK, IPT>;
    static_assert(T::VEC == 4, "bit-packed columns are read four rows at a time");
    if (base + T::ITEMS <= n) {
#pragma unroll
        for (int c = 0; c < T::CHUNKS; ++c) load_packed_vec4<NT>(w, cbase, bits, T::index(base, c, 0), &v[c * 4]);
    } else {
#pragma unroll
        for (int c = 0; c < T::CHUNKS; ++c)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t i = T::index(base, c, e);
                v[c * 4 + e] = i < n ? packed_value(w, cbase, bits, i) : 0;
            }
    }
}

template <int BLOCK, int IPT, bool NT>
__device__ __forceinline__ void block_load_sel_packed(const uint32_t *__restrict__ w, int32_t cbase, uint32_t bits,
                                                      int64_t base, int64_t n, uint32_t flags, int32_t (&v)[IPT]) {
    using T = TileShape<BLOCK, IPT>;
    static_assert(T::VEC == 4, "bit-packed columns are read four rows at a time");
    const bool full = base + T::ITEMS <= n;
#pragma unroll
    for (int c = 0; c < T::CHUNKS; ++c) {
        const uint32_t m = (flags >> (c * 4)) & 0xFu;
        if (!m) continue;
        if (full) {
            load_packed_vec4<NT>(w, cbase, bits, T::index(base, c, 0), &v[c * 4]);
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (m & (1u << e)) v[c * 4 + e] = packed_value(w, cbase, bits, T::index(base, c, e));
        }
    }
}

// ---------------------------------------------------------- BlockPred ------
__device__ __forceinline__ bool in_range(int32_t x, int32_t lo, int32_t hi) {
    return x >= lo && x <= hi;
}

template <int IPT>
__device__ __forceinline__ uint32_t block_pred_range(const int32_t (&v)[IPT], uint32_t flags,
                                                     int32_t lo, int32_t hi) {
    uint32_t m = 0;
#pragma unroll
    for (int k = 0; k < IPT; ++k) m |= (uint32_t)in_range(v[k], lo, hi) << k;
    return flags & m;
}

// ---------------------------------------------------------- BlockScan ------
// Exclusive prefix over the wave of small per-lane values x < 2^BITS: one
// ballot per bit, and the lanes below each lane counted with v_mbcnt.
template <int BITS>
__device__ __forceinline__ uint32_t wave_exclusive_scan_small(uint32_t x, uint32_t &wave_total) {
    uint32_t pre = 0, tot = 0;
#pragma unroll
    for (int b = 0; b < BITS; ++b) {
        uint64_t m = ballot((x >> b) & 1u);
        pre += count_below(m) << b;
        tot += (uint32_t)__popcll(m) << b;
    }
    wave_total = tot;
    return pre;
}

// Workgroup exclusive prefix of per-thread counts (all threads must call).
// lds_waves holds one word per wave; the caller syncs before reusing it.
template <int BLOCK, int BITS>
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t x, uint32_t *lds_waves,
                                                         uint32_t &block_total) {
    constexpr int W = BLOCK / kWave;
    uint32_t wave_total;
    uint32_t pre = wave_exclusive_scan_small<BITS>(x, wave_total);
    const int w = threadIdx.x / kWave;
    if (W == 1) {
        block_total = wave_total;
        return pre;
    }
    if (lane_id() == 0) lds_waves[w] = wave_total;
    __syncthreads();
    uint32_t before = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < W; ++i) {
        uint32_t t = lds_waves[i];
        before += i < w ? t : 0u;
        tot += t;
    }
    block_total = tot;
    return before + pre;
}

// ----------------------------------------------------- BlockAggregate ------
__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t x) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        uint32_t lo = __shfl_xor((uint32_t)x, o);
        uint32_t hi = __shfl_xor((uint32_t)(x >> 32), o);
        x += ((uint64_t)hi << 32) | lo;
    }
    return x;
}

// Hierarchical reduction; the result is valid in thread 0.
template <int BLOCK>
__device__ __forceinline__ uint64_t block_sum_u64(uint64_t x, uint64_t *lds_waves) {
    constexpr int W = BLOCK / kWave;
    x = wave_sum_u64(x);
    if (W == 1) return x;
    if (lane_id() == 0) lds_waves[threadIdx.x / kWave] = x;
    __syncthreads();
    uint64_t t = 0;
    if (threadIdx.x == 0)
#pragma unroll
        for (int i = 0; i < W; ++i) t += lds_waves[i];
    return t;
}

// ------------------------------------------------------------- atomics -----
__device__ __forceinline__ uint64_t atomic_add_u64(uint64_t *p, uint64_t v) {
    return atomicAdd(reinterpret_cast<unsigned long long *>(p), (unsigned long long)v);
}

__device__ __forceinline__ void set_status(int32_t *status, int32_t code) {
    if (status) atomicCAS(status, 0, code);
}

// --------------------------------------------------------- hash tables -----
struct DevTable {
    const uint32_t *bitmap;   // DIRECT presence bits
    const int32_t *payload;   // DIRECT payloads (or null)
    const v2i *slots;         // LINEAR {key, payload}
    int64_t span;             // DIRECT key span
    uint32_t mask;            // LINEAR capacity - 1
    int32_t key_min;          // DIRECT
    int32_t kind;             // 0 LINEAR, 1 DIRECT
    int32_t shift;            // LINEAR 32 - log2 capacity
    int32_t has_payload;
    int32_t pad;
};

__device__ __forceinline__ uint32_t hash_slot(int32_t k, int32_t shift) {
    return ((uint32_t)k * 2654435761u) >> shift;
}

// BlockProbeHT for one item: returns whether key k is present and its payload.
__device__ __forceinline__ bool probe_direct(const DevTable &t, int32_t k, int32_t &payload,
                                             bool want_payload) {
    uint32_t off = (uint32_t)k - (uint32_t)t.key_min;
    if ((int64_t)off >= t.span) return false;
    bool hit = (t.bitmap[off >> 5] >> (off & 31u)) & 1u;
    if (hit && want_payload) payload = t.payload[off];
    return hit;
}

__device__ __forceinline__ bool probe_linear(const v2i *__restrict__ slots, uint32_t mask,
                                             int32_t shift, int32_t k, int32_t &payload) {
    uint32_t s = hash_slot(k, shift);
    for (uint32_t step = 0; step <= mask; ++step) {
        v2i e = slots[s];
        if (e.x == k) {
            payload = e.y;
            return true;
        }
        if (e.x == kEmptyKey) return false;
        s = (s + 1u) & mask;
    }
    return false;
}

__device__ __forceinline__ bool probe_table(const DevTable &t, int32_t k, int32_t &payload,
                                            bool want_payload) {
    if (t.kind == 1) return probe_direct(t, k, payload, want_payload);
    if (k == kEmptyKey) return false;
    return probe_linear(t.slots, t.mask, t.shift, k, payload);
}

// Payload field extraction: bits == 32 takes the payload as a signed int32.
__device__ __forceinline__ int32_t payload_field(int32_t payload, int32_t shift, uint32_t mask,
                                                 int32_t bits) {
    return bits >= 32 ? payload : (int32_t)(((uint32_t)payload >> shift) & mask);
}

}  // namespace crystal
