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

// ------------------------------------------------------------- selection --
// Tile = BlockLoad -> BlockPred -> BlockScan of the per-thread match counts ->
// thread 0 reserves the tile's output range with one 64-bit atomic ->
// BlockShuffle the matches into LDS in thread order -> BlockStore.
template <int BLOCK, int IPT>
__global__ __launch_bounds__(BLOCK) void select_kernel(const int32_t *__restrict__ in, int64_t n,
                                                       int32_t lo, int32_t hi,
                                                       int32_t *__restrict__ out,
                                                       uint64_t *__restrict__ count,
                                                       int64_t n_tiles) {
    using T = TileShape<BLOCK, IPT>;
    __shared__ int32_t buf[T::ITEMS];
    __shared__ uint32_t wave_tot[T::WAVES];
    __shared__ uint64_t out_base;
    for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const int64_t base = tile * T::ITEMS;
        int32_t v[IPT];
        block_load<BLOCK, IPT, true>(in, base, n, v);
        const uint32_t flags = block_pred_range<IPT>(v, valid_mask<BLOCK, IPT>(base, n), lo, hi);
        uint32_t total;
        uint32_t off = block_exclusive_scan<BLOCK, T::CBITS>((uint32_t)__popc(flags), wave_tot, total);
        if (total != 0) {
            if (threadIdx.x == 0) out_base = atomic_add_u64(count, total);
#pragma unroll
            for (int k = 0; k < IPT; ++k)
                if ((flags >> k) & 1u) buf[off++] = v[k];
            __syncthreads();
            const uint64_t ob = out_base;
            for (uint32_t i = threadIdx.x; i < total; i += BLOCK)
                __builtin_nontemporal_store(buf[i], out + ob + i);
        }
        __syncthreads();
    }
}

template <int BLOCK, int IPT>
static hipError_t select_t(const LaunchCfg &cfg, const int32_t *in, int64_t n, int32_t lo,
                           int32_t hi, int32_t *out, uint64_t *count, hipStream_t s) {
    using T = TileShape<BLOCK, IPT>;
    const int64_t n_tiles = (n + T::ITEMS - 1) / T::ITEMS;
    const int64_t grid = grid_for(n_tiles, cfg);
    if (grid == 0) return hipSuccess;
    hipLaunchKernelGGL((select_kernel<BLOCK, IPT>), dim3((unsigned)grid), dim3(BLOCK), 0, s, in, n,
                       lo, hi, out, count, n_tiles);
    return hipGetLastError();
}

hipError_t launch_select(const LaunchCfg &cfg, const int32_t *in, int64_t n, int32_t lo,
                         int32_t hi, int32_t *out, uint64_t *count, hipStream_t s) {
    switch (CRYSTAL_VARIANT_KEY(cfg.block, cfg.ipt)) {
#define X(B, I) \
    case CRYSTAL_VARIANT_KEY(B, I): return select_t<B, I>(cfg, in, n, lo, hi, out, count, s);
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

}  // namespace crystal
