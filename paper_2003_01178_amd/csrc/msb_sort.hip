// MSB radix sort of 32-bit key / 32-bit value pairs (section 4.4: the GPU
// sort partitions by the most significant 8-bit digit first, then within
// each partition by the next digit).
//
// Level 0 is the plain stable partition pass on the top byte (the whole
// input is one segment).  Level L >= 1 (shift 24 - 8L) partitions every
// "big" segment (more pairs than a workgroup sorts in LDS) by its digit at
// `shift`, stably:
//   chunks    each big segment is cut into chunks of at most kChunk pairs;
//   histogram one workgroup counts the digits of a chunk;
//   scan      one workgroup per segment turns its chunks' counts into output
//             offsets (digit-major within the segment) and classifies the
//             segment's 256 sub-segments: big ones go to the next level,
//             the others become local-sort tasks;
//   shuffle   one workgroup per chunk writes its pairs to their offsets, a
//             tile at a time, ranking equal digits stably with ballots (the
//             tile is sorted by digit in LDS, then written in that order).
// Two final launches sort every task in LDS by its remaining low bits
// (stable 8-bit passes from the low digit up), one workgroup per task, and
// write it to the output: tasks of at most kSmallMax pairs in a small shape
// (four workgroups per CU), the others in a large one.  Levels alternate
// between the output and a scratch copy; a task reads whichever holds its
// segment.  Uniform keys need two partition levels (256, then
// 65,536 segments of about 4,096 pairs) and the local pass; skewed keys
// simply keep more segments big for more levels.
//
// All work lists live in device memory and every kernel loops over its list
// (persistent workgroups), so the host never waits for the device.
#include <type_traits>

#include "block.hpp"
#include "internal.hpp"

namespace crystal {
namespace {

constexpr int kBinsM = 256;
constexpr uint32_t kLocalMax = 8192;  // pairs one local-sort workgroup holds (512 threads x 16)
constexpr uint32_t kSmallSeg = 1024;  // sub-segments shorter than this are grouped into one task
constexpr uint32_t kChunk = 65536;    // pairs per partition chunk (4 tiles)
constexpr int kPartBlock = 1024, kPartIpt = 16;
constexpr int kLocBlock = 512, kLocIpt = 16;  // tasks up to kLocalMax pairs
constexpr int kSmlBlock = 256, kSmlIpt = 17;  // tasks up to kSmallMax pairs, four workgroups per CU
constexpr uint32_t kSmallMax = kSmlBlock * kSmlIpt;
static_assert(kLocBlock * kLocIpt >= (int)kLocalMax, "the large shape holds every sorted task");
constexpr int kAuxBlock = 256;

struct Seg {
    uint32_t start, len, chunk_base, nchunks;
};
struct ChunkD {
    uint32_t seg, start, end, pad;
};
// src: where the segment lives (0 the input, 1 the output, 2 the scratch
// copy); bits: low key bits still to sort (0: copy only)
struct Task {
    uint32_t start, len, bits, src;
};
// two task lists: 0 for tasks of at most kSmallMax pairs, 1 for the others
struct Ctl {
    uint32_t n_big[2];
    uint32_t n_chunks;
    uint32_t n_tasks[2];
};

__device__ __forceinline__ int task_list(uint32_t len, uint32_t bits) { return bits && len <= kSmallMax ? 0 : 1; }

// Exclusive prefix over the block's threads in thread order; tmp: one word
// per wave.  Ends with a barrier, after which tmp may be reused.
template <int BLOCK>
__device__ __forceinline__ uint32_t block_scan_excl(uint32_t x, uint32_t *tmp, uint32_t &total) {
    constexpr int W = BLOCK / kWave;
    const int lane = (int)lane_id();
    uint32_t inc = x;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const uint32_t y = __shfl_up(inc, o);
        if (lane >= o) inc += y;
    }
    const int w = (int)threadIdx.x / kWave;
    if (lane == kWave - 1) tmp[w] = inc;
    __syncthreads();
    uint32_t before = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < W; ++i) {
        const uint32_t t = tmp[i];
        before += i < w ? t : 0u;
        tot += t;
    }
    total = tot;
    __syncthreads();
    return before + inc - x;
}

// Stable rank of item slot k among the wave's items of the same digit that
// come before it (earlier slots through the wave's LDS counter wc[d], earlier
// lanes of this slot through the ballots).  Invalid items are not counted.
__device__ __forceinline__ uint32_t stable_rank(uint32_t d, bool valid, uint32_t *wc) {
    uint64_t diff = 0;  // lanes whose digit differs from this lane's in some bit
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t m = ballot(bit);
        diff |= bit ? ~m : m;
    }
    const uint64_t peers = ballot(valid) & ~diff;
    const uint32_t below = count_below(peers);
    const uint32_t same = (uint32_t)__popcll(peers);
    uint32_t rank = 0;
    if (valid) {
        const uint32_t c = wc[d];
        rank = c + below;
        if (below + 1 == same) wc[d] = c + same;
    }
    return rank;
}

// ------------------------------------------------------------ work lists --
// An input of at most kLocalMax pairs: one task, the whole input, all 32 bits.
__global__ void msb_init_kernel(Ctl *ctl, Task *tasks, uint32_t list_stride, uint32_t n) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    ctl->n_big[0] = ctl->n_big[1] = 0;
    ctl->n_chunks = 0;
    const int l = task_list(n, 32u);
    ctl->n_tasks[0] = ctl->n_tasks[1] = 0;
    ctl->n_tasks[l] = 1;
    tasks[(int64_t)l * list_stride] = Task{0u, n, 32u, 0u};
}

// One workgroup: chunk counts of the level's big segments, their exclusive
// prefix (each segment's first chunk), the level's chunk total; clears the
// next level's big-segment count.
__global__ __launch_bounds__(1024) void msb_chunk_scan_kernel(Ctl *ctl, Seg *big, int cur) {
    __shared__ uint32_t tmp[1024 / kWave];
    const uint32_t nb = ctl->n_big[cur];
    const uint32_t per = (nb + 1023u) / 1024u;
    const uint32_t s0 = threadIdx.x * per;
    uint32_t s1 = s0 + per;
    if (s1 > nb) s1 = nb;
    uint32_t sum = 0;
    for (uint32_t i = s0; i < s1; ++i) sum += (big[i].len + kChunk - 1) / kChunk;
    uint32_t total;
    uint32_t run = block_scan_excl<1024>(sum, tmp, total);
    for (uint32_t i = s0; i < s1; ++i) {
        const uint32_t c = (big[i].len + kChunk - 1) / kChunk;
        big[i].chunk_base = run;
        big[i].nchunks = c;
        run += c;
    }
    if (threadIdx.x == 0) {
        ctl->n_chunks = total;
        ctl->n_big[cur ^ 1] = 0;
    }
}

// Chunk c of the level: its segment (binary search over the segments' first
// chunks) and its pair range.
__global__ __launch_bounds__(kAuxBlock) void msb_chunk_fill_kernel(const Ctl *ctl, const Seg *big, int cur,
                                                                   ChunkD *chunks) {
    const uint32_t nb = ctl->n_big[cur], nc = ctl->n_chunks;
    for (uint32_t c = blockIdx.x * kAuxBlock + threadIdx.x; c < nc; c += gridDim.x * kAuxBlock) {
        uint32_t lo = 0, hi = nb - 1;  // the last segment whose first chunk is <= c
        while (lo < hi) {
            const uint32_t mid = (lo + hi + 1) / 2;
            if (big[mid].chunk_base <= c)
                lo = mid;
            else
                hi = mid - 1;
        }
        const Seg s = big[lo];
        const uint32_t start = s.start + (c - s.chunk_base) * kChunk;
        const uint32_t seg_end = s.start + s.len;
        chunks[c] = ChunkD{lo, start, (seg_end - start > kChunk) ? start + kChunk : seg_end, 0u};
    }
}

// Digit counts of every chunk: hist[c * 256 + d].
__global__ __launch_bounds__(kAuxBlock) void msb_hist_kernel(const Ctl *ctl, const ChunkD *chunks,
                                                             const uint32_t *__restrict__ keys, int shift,
                                                             uint32_t *__restrict__ hist) {
    constexpr int W = kAuxBlock / kWave;
    __shared__ uint32_t h[W][kBinsM];
    const int w = threadIdx.x / kWave;
    const uint32_t nc = ctl->n_chunks;
    for (uint32_t c = blockIdx.x; c < nc; c += gridDim.x) {
        for (int i = threadIdx.x; i < W * kBinsM; i += kAuxBlock) (&h[0][0])[i] = 0u;
        __syncthreads();
        const ChunkD ch = chunks[c];
        // 16 keys per thread in flight at a time, then the tail
        constexpr int B = 16;
        uint32_t i = ch.start;
        for (; i + B * kAuxBlock <= ch.end; i += B * kAuxBlock) {
            uint32_t v[B];
#pragma unroll
            for (int k = 0; k < B; ++k) v[k] = __builtin_nontemporal_load(keys + i + k * kAuxBlock + threadIdx.x);
#pragma unroll
            for (int k = 0; k < B; ++k) atomicAdd(&h[w][(v[k] >> shift) & 0xFFu], 1u);
        }
        for (i += threadIdx.x; i < ch.end; i += kAuxBlock)
            atomicAdd(&h[w][(__builtin_nontemporal_load(keys + i) >> shift) & 0xFFu], 1u);
        __syncthreads();
        const int d = threadIdx.x;  // kAuxBlock == kBinsM
        uint32_t s = 0;
#pragma unroll
        for (int i = 0; i < W; ++i) s += h[i][d];
        hist[(int64_t)c * kBinsM + d] = s;
        __syncthreads();
    }
}

// The sub-segments of one big segment, after its partition at `shift`
// (starts st[], lengths tot[], per digit), become next-level big segments or
// local-sort tasks; run by one thread.  Sub-segments of kSmallSeg pairs or
// more are tasks of their own, sorted by the `shift` bits below their digit;
// shorter neighbours are grouped into tasks of at most kLocalMax pairs,
// sorted by their digit too.  At the last digit every sub-segment is final
// where the level wrote it: copy tasks of at most kChunk pairs when that is
// the scratch copy.  Two walks: count and reserve, then write.
__device__ void plan_subsegments(Ctl *ctl, int cur, const uint32_t *st, const uint32_t *tot, uint32_t seg_start,
                                 uint32_t seg_len, int shift, uint32_t dst, Seg *next, Task *tasks,
                                 uint32_t list_stride, uint32_t &base_big, uint32_t *base_task) {
    for (int write = 0; write < 2; ++write) {
        uint32_t nbig = 0, ntask[2] = {0u, 0u};
        auto emit_task = [&](uint32_t a, uint32_t len, uint32_t bits) {
            const int l = task_list(len, bits);
            if (write) tasks[(int64_t)l * list_stride + base_task[l] + ntask[l]] = Task{a, len, bits, dst};
            ++ntask[l];
        };
        if (shift == 0) {
            // copies in pieces of kChunk pairs, so that a long run of one key
            // is copied by many workgroups
            if (dst != 1u)
                for (uint64_t a = 0; a < seg_len; a += kChunk)
                    emit_task(seg_start + (uint32_t)a, seg_len - a < kChunk ? (uint32_t)(seg_len - a) : kChunk, 0u);
        } else {
            uint32_t g_start = 0, g_len = 0, g_digits = 0;
            auto flush = [&]() {
                if (g_len) emit_task(g_start, g_len, g_digits > 1 ? (uint32_t)shift + 8u : (uint32_t)shift);
                g_len = 0;
                g_digits = 0;
            };
            for (int e = 0; e < kBinsM; ++e) {
                const uint32_t len = tot[e];
                if (!len) continue;
                if (len > kLocalMax) {
                    flush();
                    if (write) next[base_big + nbig] = Seg{st[e], len, 0u, 0u};
                    ++nbig;
                } else if (len >= kSmallSeg) {
                    flush();
                    emit_task(st[e], len, (uint32_t)shift);
                } else {
                    if (g_len && g_len + len > kLocalMax) flush();
                    if (!g_len) g_start = st[e];
                    g_len += len;
                    ++g_digits;
                }
            }
            flush();
        }
        if (!write) {
            base_big = nbig ? atomicAdd(&ctl->n_big[cur ^ 1], nbig) : 0u;
            for (int l = 0; l < 2; ++l) base_task[l] = ntask[l] ? atomicAdd(&ctl->n_tasks[l], ntask[l]) : 0u;
        }
    }
}

// Level 0 done by the plain partition pass (the whole input is one segment):
// its partition offsets (part[d], part[256] = n) become the first level's
// sub-segments.  One workgroup of 256 threads; also resets the counters.
__global__ __launch_bounds__(kAuxBlock) void msb_level0_kernel(Ctl *ctl, const uint32_t *part, uint32_t n,
                                                               Seg *next, Task *tasks, uint32_t list_stride) {
    __shared__ uint32_t st[kBinsM], tot[kBinsM];
    __shared__ uint32_t base_big, base_task[2];
    const int d = threadIdx.x;
    st[d] = part[d];
    tot[d] = part[d + 1] - part[d];
    if (d == 0) {
        ctl->n_big[0] = 0;
        ctl->n_big[1] = 0;
        ctl->n_chunks = 0;
        ctl->n_tasks[0] = ctl->n_tasks[1] = 0;
    }
    __syncthreads();
    // big sub-segments go to list 1, which level 1 reads
    if (d == 0) plan_subsegments(ctl, 0, st, tot, 0u, n, 24, 1u, next, tasks, list_stride, base_big, base_task);
}

// One workgroup per big segment (thread d = digit d): the chunks' counts
// become global output offsets, in place; the segment's sub-segments become
// next-level big segments or tasks.  dst: where this level writes (1 the
// output, 2 the scratch copy).
__global__ __launch_bounds__(kAuxBlock) void msb_scan_kernel(Ctl *ctl, const Seg *big, int cur,
                                                             uint32_t *__restrict__ hist, Seg *next, Task *tasks,
                                                             uint32_t list_stride, int shift, uint32_t dst) {
    __shared__ uint32_t tmp[kAuxBlock / kWave];
    __shared__ uint32_t st[kBinsM], tot[kBinsM];
    __shared__ uint32_t base_big, base_task[2];
    const int d = threadIdx.x;
    const uint32_t nb = ctl->n_big[cur];
    for (uint32_t i = blockIdx.x; i < nb; i += gridDim.x) {
        const Seg s = big[i];
        uint32_t run = 0;
        for (uint32_t j = 0; j < s.nchunks; ++j) {
            uint32_t *p = hist + (int64_t)(s.chunk_base + j) * kBinsM + d;
            const uint32_t v = *p;
            *p = run;
            run += v;
        }
        uint32_t unused;
        const uint32_t dstart = block_scan_excl<kAuxBlock>(run, tmp, unused);
        const uint32_t at = s.start + dstart;
        for (uint32_t j = 0; j < s.nchunks; ++j) hist[(int64_t)(s.chunk_base + j) * kBinsM + d] += at;
        st[d] = at;
        tot[d] = run;
        __syncthreads();
        if (d == 0)
            plan_subsegments(ctl, cur, st, tot, s.start, s.len, shift, dst, next, tasks, list_stride, base_big,
                             base_task);
        __syncthreads();
    }
}

// ---------------------------------------------------------------- shuffle --
// Tile layout (as in the partition pass): wave w owns the 64 * IPT
// consecutive pairs from w * 64 * IPT, and lane l's slot k is pair k * 64 + l
// of them, so visiting slots in order visits a wave's pairs in input order.
template <bool VALS>
__global__ __launch_bounds__(kPartBlock) void msb_shuffle_kernel(const Ctl *ctl, const ChunkD *chunks,
                                                                 const uint32_t *__restrict__ hist,
                                                                 const uint32_t *__restrict__ ik,
                                                                 const uint32_t *__restrict__ iv,
                                                                 uint32_t *__restrict__ ok, uint32_t *__restrict__ ov,
                                                                 int shift) {
    constexpr int W = kPartBlock / kWave;
    constexpr int ITEMS = kPartBlock * kPartIpt;
    extern __shared__ uint32_t lds[];
    uint32_t *s_keys = lds;
    uint32_t *s_vals = lds + ITEMS;
    uint32_t *s_wc = lds + (VALS ? 2 : 1) * ITEMS;  // [W][256]
    uint32_t *s_gbase = s_wc + W * kBinsM;
    uint32_t *s_run = s_gbase + kBinsM;
    uint32_t *s_tmp = s_run + kBinsM;
    const int tid = threadIdx.x;
    const int w = tid / kWave;
    uint32_t *my_wc = s_wc + w * kBinsM;
    const int off0 = w * (kWave * kPartIpt) + (int)lane_id();
    const uint32_t nc = ctl->n_chunks;

    for (uint32_t c = blockIdx.x; c < nc; c += gridDim.x) {
        const ChunkD ch = chunks[c];
        if (tid < kBinsM) {
            s_run[tid] = hist[(int64_t)c * kBinsM + tid];
#pragma unroll
            for (int i = 0; i < W; ++i) s_wc[i * kBinsM + tid] = 0u;
        }
        __syncthreads();
        uint32_t key[kPartIpt], val[kPartIpt];
        auto load = [&](int64_t base) {
            const int rem = (int)((int64_t)ch.end - base < ITEMS ? (int64_t)ch.end - base : ITEMS);
            // the tile's base pointers are made opaque scalars, so every load
            // is one scalar base plus one lane offset (global address space:
            // a generic pointer would give flat loads)
            typedef const __attribute__((address_space(1))) uint32_t *gptr;
            // base is uniform; readfirstlane states it for the scalar constraint below
            base = ((int64_t)__builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)base >> 32)) << 32) |
                   (int64_t)(uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)base);
            gptr kb = (gptr)(ik + base);
            gptr vb = VALS ? (gptr)(iv + base) : nullptr;
            asm volatile("" : "+s"(kb));
            if (VALS) asm volatile("" : "+s"(vb));
            if (rem == ITEMS) {
#pragma unroll
                for (int k = 0; k < kPartIpt; ++k) {
                    key[k] = __builtin_nontemporal_load(&kb[off0 + k * kWave]);
                    if (VALS) val[k] = __builtin_nontemporal_load(&vb[off0 + k * kWave]);
                }
            } else {
#pragma unroll
                for (int k = 0; k < kPartIpt; ++k) {
                    const int i = off0 + k * kWave;
                    key[k] = i < rem ? kb[i] : 0u;
                    if (VALS) val[k] = i < rem ? vb[i] : 0u;
                }
            }
        };
        load(ch.start);
        for (int64_t base = ch.start; base < (int64_t)ch.end; base += ITEMS) {
            const int rem = (int)((int64_t)ch.end - base < ITEMS ? (int64_t)ch.end - base : ITEMS);
            // the wave clears its own counter row: the previous tile last read it
            // in this wave and in the digit scan before its scatter barrier, so
            // the write-out needs no barrier after it
#pragma unroll
            for (int q = 0; q < kBinsM / kWave; ++q) my_wc[q * kWave + (int)lane_id()] = 0u;
            uint32_t rank[kPartIpt];
#pragma unroll
            for (int k = 0; k < kPartIpt; ++k) {
                rank[k] = stable_rank((key[k] >> shift) & 0xFFu, off0 + k * kWave < rem, my_wc);
                __builtin_amdgcn_sched_barrier(0);
            }
            __syncthreads();
            // per digit: each wave's run inside the tile's run, the tile's
            // digit starts, and the global base of the digit for this tile
            uint32_t cnt = 0;
            if (tid < kBinsM) {
#pragma unroll
                for (int i = 0; i < W; ++i) {
                    const uint32_t v = s_wc[i * kBinsM + tid];
                    s_wc[i * kBinsM + tid] = cnt;
                    cnt += v;
                }
            }
            uint32_t unused;
            const uint32_t tstart = block_scan_excl<kPartBlock>(cnt, s_tmp, unused);
            if (tid < kBinsM) {
#pragma unroll
                for (int i = 0; i < W; ++i) s_wc[i * kBinsM + tid] += tstart;
                const uint32_t r = s_run[tid];
                s_gbase[tid] = r - tstart;
                s_run[tid] = r + cnt;
            }
            __syncthreads();
#pragma unroll
            for (int k = 0; k < kPartIpt; ++k) {
                if (off0 + k * kWave < rem) {
                    const uint32_t p = my_wc[(key[k] >> shift) & 0xFFu] + rank[k];
                    s_keys[p] = key[k];
                    if (VALS) s_vals[p] = val[k];
                }
            }
            __syncthreads();
            // the next tile's loads go out while this one is written
            if (base + ITEMS < (int64_t)ch.end) load(base + ITEMS);
            int tidv = tid;  // opaque: keeps the write-out's per-item offsets out of registers
            asm volatile("" : "+v"(tidv));
#pragma unroll
            for (int j = 0; j < kPartIpt; ++j) {
                const int p = j * kPartBlock + tidv;
                if (p < rem) {
                    const uint32_t k = s_keys[p];
                    const uint32_t g = s_gbase[(k >> shift) & 0xFFu] + (uint32_t)p;  // < n
                    ok[g] = k;
                    if (VALS) ov[g] = s_vals[p];
                }
                if (j % 4 == 3) __builtin_amdgcn_sched_barrier(0);
            }
            // no barrier: the next tile writes s_gbase, s_run, s_tmp and the LDS
            // tile only after its ranking barrier, and the next chunk's set-up
            // ends with one
        }
    }
}

// ------------------------------------------------------------ local sort --
// One task at a time per workgroup: its pairs in registers (the tile layout
// above), sorted by `bits` low key bits with stable 8-bit passes in LDS,
// then written out from LDS.  Two shapes: BLOCK x IPT holds the task list's
// largest task; the small shape fits four workgroups per CU.
template <bool VALS, int BLOCK, int IPT>
__global__ __launch_bounds__(BLOCK, 4) void msb_local_kernel(const Ctl *ctl, int list, const Task *tasks,
                                                          const uint32_t *__restrict__ in_k,
                                                          const uint32_t *__restrict__ in_v,
                                                          uint32_t *__restrict__ out_k, uint32_t *__restrict__ out_v,
                                                          const uint32_t *__restrict__ tmp_k,
                                                          const uint32_t *__restrict__ tmp_v) {
    constexpr int W = BLOCK / kWave;
    constexpr int ITEMS = BLOCK * IPT;
    extern __shared__ uint32_t lds[];
    uint32_t *s_keys = lds;
    uint32_t *s_vals = lds + ITEMS;
    uint32_t *s_wc = lds + (VALS ? 2 : 1) * ITEMS;  // [W][256]
    uint32_t *s_tmp = s_wc + W * kBinsM;
    const int tid = threadIdx.x;
    const int w = tid / kWave;
    uint32_t *my_wc = s_wc + w * kBinsM;
    const int wave0 = w * (kWave * IPT);
    const int off0 = wave0 + (int)lane_id();
    const uint32_t nt = ctl->n_tasks[list];
    auto src_k = [&](const Task &t) { return t.src == 0 ? in_k : t.src == 1 ? (const uint32_t *)out_k : tmp_k; };
    auto src_v = [&](const Task &t) { return t.src == 0 ? in_v : t.src == 1 ? (const uint32_t *)out_v : tmp_v; };
    uint32_t key[IPT], val[IPT];
    auto load = [&](const Task &t) {
        typedef const __attribute__((address_space(1))) uint32_t *gptr;
        gptr kb = (gptr)(src_k(t) + t.start);
        gptr vb = VALS ? (gptr)(src_v(t) + t.start) : nullptr;
        const int len = (int)t.len;
#pragma unroll
        for (int k = 0; k < IPT; ++k) {
            const int i = off0 + k * kWave;
            key[k] = i < len ? kb[i] : 0u;
            if (VALS) val[k] = i < len ? vb[i] : 0u;
        }
    };

    for (uint32_t t = blockIdx.x; t < nt; t += gridDim.x) {
        const Task task = tasks[t];
        const int len = (int)task.len;
        if (task.bits) load(task);
        if (task.bits == 0) {
            // already in order: copy unless it is in the output already
            if (task.src != 1) {
                const uint32_t *sk = src_k(task), *sv = src_v(task);
                for (uint32_t i = tid; i < task.len; i += BLOCK) {
                    out_k[task.start + i] = sk[task.start + i];
                    if (VALS) out_v[task.start + i] = sv[task.start + i];
                }
            }
        } else {
            for (uint32_t sh = 0; sh < task.bits; sh += 8) {
                const uint32_t left = task.bits - sh;
                const uint32_t mask = left >= 8 ? 0xFFu : (1u << left) - 1u;
                if (tid < kBinsM) {
#pragma unroll
                    for (int i = 0; i < W; ++i) s_wc[i * kBinsM + tid] = 0u;
                }
                __syncthreads();
                uint32_t rank[IPT];
                // slots whose 64 pairs all lie past the task's end are skipped
                // (the test is uniform across the wave)
#pragma unroll
                for (int k = 0; k < IPT; ++k) {
                    rank[k] = 0;
                    if (wave0 + k * kWave < len)
                        rank[k] = stable_rank((key[k] >> sh) & mask, off0 + k * kWave < len, my_wc);
                    __builtin_amdgcn_sched_barrier(0);
                }
                __syncthreads();
                uint32_t cnt = 0;
                if (tid < kBinsM) {
#pragma unroll
                    for (int i = 0; i < W; ++i) {
                        const uint32_t v = s_wc[i * kBinsM + tid];
                        s_wc[i * kBinsM + tid] = cnt;
                        cnt += v;
                    }
                }
                uint32_t unused;
                const uint32_t dstart = block_scan_excl<BLOCK>(cnt, s_tmp, unused);
                if (tid < kBinsM) {
#pragma unroll
                    for (int i = 0; i < W; ++i) s_wc[i * kBinsM + tid] += dstart;
                }
                __syncthreads();
#pragma unroll
                for (int k = 0; k < IPT; ++k) {
                    if (off0 + k * kWave < len) {
                        const uint32_t p = my_wc[(key[k] >> sh) & mask] + rank[k];
                        s_keys[p] = key[k];
                        if (VALS) s_vals[p] = val[k];
                    }
                }
                __syncthreads();
                if (sh + 8 < task.bits) {
#pragma unroll
                    for (int k = 0; k < IPT; ++k) {
                        const int i = off0 + k * kWave;
                        if (i < len) {
                            key[k] = s_keys[i];
                            if (VALS) val[k] = s_vals[i];
                        }
                    }
                    __syncthreads();
                }
            }
        }
        if (task.bits) {
            for (int i = tid; i < len; i += BLOCK) {
                out_k[task.start + i] = s_keys[i];
                if (VALS) out_v[task.start + i] = s_vals[i];
            }
            __syncthreads();  // the LDS is the next task's
        }
    }
}

constexpr size_t shuffle_lds(bool vals) {
    return ((size_t)(vals ? 2 : 1) * kPartBlock * kPartIpt + (kPartBlock / kWave) * kBinsM + 2 * kBinsM +
            kPartBlock / kWave) * 4;
}
constexpr size_t local_lds(bool vals, int block, int ipt) {
    return ((size_t)(vals ? 2 : 1) * block * ipt + (block / kWave) * kBinsM + block / kWave) * 4;
}

int64_t r256(int64_t b) { return (b + 255) / 256 * 256; }

struct MsbLayout {
    int64_t max_big, max_chunks, max_tasks;
    int64_t tmp_k, tmp_v, big0, big1, chunks, hist, tasks, ctl, part, pass, total;
};

MsbLayout msb_layout(int64_t n, bool vals) {
    MsbLayout L{};
    L.max_big = n / (kLocalMax + 1) > 1 ? n / (kLocalMax + 1) : 1;
    L.max_chunks = n / kChunk + L.max_big + 1;
    // tasks, per level with a digit left below it: one per sub-segment of
    // kSmallSeg pairs or more (at most n / kSmallSeg), and groups of shorter
    // ones; a group closes above kLocalMax - kSmallSeg pairs, before a longer
    // or a big sub-segment, or at its parent's end, so there are at most
    // n / (kLocalMax - kSmallSeg) + n / kSmallSeg + (big segments of this and
    // the next level) of them.  Then the last level's copies (pieces of at
    // most kChunk pairs of the big segments) and the single task of a short
    // input.
    L.max_tasks = 3 * (2 * (n / kSmallSeg) + n / (kLocalMax - kSmallSeg) + 2 * L.max_big + 2) + n / kChunk +
                  L.max_big + 8;
    int64_t at = 0;
    L.tmp_k = at;
    at += r256(n * 4);
    L.tmp_v = at;
    at += vals ? r256(n * 4) : 0;
    L.big0 = at;
    at += r256(L.max_big * (int64_t)sizeof(Seg));
    L.big1 = at;
    at += r256(L.max_big * (int64_t)sizeof(Seg));
    L.chunks = at;
    at += r256(L.max_chunks * (int64_t)sizeof(ChunkD));
    L.hist = at;
    at += r256(L.max_chunks * kBinsM * 4);
    L.tasks = at;  // two lists of max_tasks entries
    at += r256(2 * L.max_tasks * (int64_t)sizeof(Task));
    L.ctl = at;
    at += 256;
    L.part = at;
    at += r256((kBinsM + 1) * 4);
    L.pass = at;
    at += r256(radix_pass_scratch_bytes(tune_lookup(CRYSTAL_K_RADIX, n), n));
    L.total = at;
    return L;
}

template <bool VALS>
hipError_t msb_run(const uint32_t *keys, const uint32_t *vals, int64_t n, uint32_t *ok, uint32_t *ov, void *scratch,
                   hipStream_t s) {
    const MsbLayout L = msb_layout(n, VALS);
    char *base = (char *)scratch;
    uint32_t *tk = (uint32_t *)(base + L.tmp_k);
    uint32_t *tv = VALS ? (uint32_t *)(base + L.tmp_v) : nullptr;
    Seg *big[2] = {(Seg *)(base + L.big0), (Seg *)(base + L.big1)};
    ChunkD *chunks = (ChunkD *)(base + L.chunks);
    uint32_t *hist = (uint32_t *)(base + L.hist);
    Task *tasks = (Task *)(base + L.tasks);
    Ctl *ctl = (Ctl *)(base + L.ctl);

    const uint32_t stride = (uint32_t)L.max_tasks;
    auto large = msb_local_kernel<VALS, kLocBlock, kLocIpt>;
    auto small = msb_local_kernel<VALS, kSmlBlock, kSmlIpt>;
    const size_t large_lds = local_lds(VALS, kLocBlock, kLocIpt), small_lds = local_lds(VALS, kSmlBlock, kSmlIpt);
    static bool attrs = false;
    if (!attrs) {
        hipError_t e = hipFuncSetAttribute((const void *)msb_shuffle_kernel<VALS>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)shuffle_lds(VALS));
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void *)large, hipFuncAttributeMaxDynamicSharedMemorySize, (int)large_lds);
        if (e != hipSuccess) return e;
        attrs = true;
    }
    const int64_t cus = device_cu_count();
    int64_t part_per_cu = 0, large_per_cu = 0, small_per_cu = 0;
    hipError_t e = resident_per_cu((const void *)msb_shuffle_kernel<VALS>, kPartBlock, (int64_t)shuffle_lds(VALS),
                                   part_per_cu);
    if (e == hipSuccess) e = resident_per_cu((const void *)large, kLocBlock, (int64_t)large_lds, large_per_cu);
    if (e == hipSuccess) e = resident_per_cu((const void *)small, kSmlBlock, (int64_t)small_lds, small_per_cu);
    if (e != hipSuccess) return e;
    if (part_per_cu < 1) part_per_cu = 1;
    if (large_per_cu < 1) large_per_cu = 1;
    if (small_per_cu < 1) small_per_cu = 1;
    const dim3 aux_grid((unsigned)(cus * 8)), aux(kAuxBlock);
    auto local_sorts = [&](int64_t large_grid, int64_t small_grid) {
        hipLaunchKernelGGL(small, dim3((unsigned)small_grid), dim3(kSmlBlock), small_lds, s, ctl, 0, tasks, keys,
                           vals, ok, ov, tk, tv);
        hipLaunchKernelGGL(large, dim3((unsigned)large_grid), dim3(kLocBlock), large_lds, s, ctl, 1,
                           tasks + stride, keys, vals, ok, ov, tk, tv);
        return hipGetLastError();
    };

    if (n <= (int64_t)kLocalMax) {
        // one task: the whole input, sorted in LDS
        hipLaunchKernelGGL(msb_init_kernel, dim3(1), dim3(64), 0, s, ctl, tasks, stride, (uint32_t)n);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        return local_sorts(1, 1);
    }
    // level 0: the whole input is one segment, so the plain stable partition
    // pass on the top byte does it (input -> output), and its partition
    // offsets give the first level's sub-segments
    const LaunchCfg rcfg = tune_lookup(CRYSTAL_K_RADIX, n);
    e = launch_radix_partition(rcfg, keys, vals, n, 24, 8, ok, ov, (uint32_t *)(base + L.part), base + L.pass, true,
                               s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(msb_level0_kernel, dim3(1), dim3(kAuxBlock), 0, s, ctl, (const uint32_t *)(base + L.part),
                       (uint32_t)n, big[1], tasks, stride);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    for (int level = 1; level < 4; ++level) {
        const int shift = 24 - 8 * level, cur = level & 1;
        const uint32_t *sk = (level & 1) ? ok : tk;
        const uint32_t *sv = (level & 1) ? ov : tv;
        uint32_t *dk = (level & 1) ? tk : ok;
        uint32_t *dv = (level & 1) ? tv : ov;
        const uint32_t dst = (level & 1) ? 2u : 1u;
        hipLaunchKernelGGL(msb_chunk_scan_kernel, dim3(1), dim3(1024), 0, s, ctl, big[cur], cur);
        hipLaunchKernelGGL(msb_chunk_fill_kernel, aux_grid, aux, 0, s, ctl, big[cur], cur, chunks);
        hipLaunchKernelGGL(msb_hist_kernel, aux_grid, aux, 0, s, ctl, chunks, sk, shift, hist);
        hipLaunchKernelGGL(msb_scan_kernel, aux_grid, aux, 0, s, ctl, big[cur], cur, hist, big[cur ^ 1], tasks,
                           stride, shift, dst);
        hipLaunchKernelGGL(msb_shuffle_kernel<VALS>, dim3((unsigned)(cus * part_per_cu)), dim3(kPartBlock),
                           shuffle_lds(VALS), s, ctl, chunks, hist, sk, sv, dk, dv, shift);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return local_sorts(cus * large_per_cu, cus * small_per_cu);
}

}  // namespace

int64_t msb_sort_scratch_bytes(int64_t n, bool with_values) { return msb_layout(n, with_values).total; }

hipError_t launch_msb_sort(const uint32_t *keys, const uint32_t *vals, int64_t n, uint32_t *out_keys,
                           uint32_t *out_vals, void *scratch, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    return vals ? msb_run<true>(keys, vals, n, out_keys, out_vals, scratch, s)
                : msb_run<false>(keys, nullptr, n, out_keys, nullptr, scratch, s);
}

}  // namespace crystal
