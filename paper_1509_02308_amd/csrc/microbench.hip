// microbench.hip -- the paper's microbenchmarks redesigned for one gfx950
// GPU.
//
// * microbench_pchase: the fine-grained P-chase (Section 4.2, Listing 3).
//   One lane initialises nothing itself; an init kernel writes the chase
//   array (Listing 1), then a single active lane walks it once untimed (the
//   preheat) and times k dependent loads one by one.  Each timed segment is
//   "read shader clock, load, wait for the load, read shader clock" in one
//   asm block, so the compiler cannot move work into or out of it; the
//   explicit wait for the load plays the role of the paper's dependent
//   s_index store.  Records stay in LDS until the walk ends, so recording
//   does not touch the caches under test.
// * microbench_hbm_stream: copy throughput over a grid x block x ILP sweep
//   (Section 5.1), throughput = 2 * size / time.
// * microbench_lds_bank: Listing 4 on one wave; lane t chases word t*stride
//   64 times, the average cycles per load show the bank-conflict degree
//   (Section 6.2).
#include <algorithm>
#include <vector>

#include "host_common.h"

namespace pc {

// ----------------------------------------------------------- P-chase ----
__global__ void pchase_init_kernel(int32_t* a, uint32_t ne, uint32_t se) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ne;
         i += (uint64_t)gridDim.x * blockDim.x) {
        uint64_t v = i + se;
        if (v >= ne) v -= ne;
        a[i] = (int32_t)v;
    }
}

template <int FLAVOR>
__device__ __forceinline__ void timed_load(const int32_t* addr, int32_t& j, uint64_t& t0, uint64_t& t1) {
    if constexpr (FLAVOR == PCHASE_LOAD_DEFAULT) {
        asm volatile(
            "s_memtime %0\n\t"
            "s_waitcnt lgkmcnt(0)\n\t"
            "global_load_dword %2, %3, off\n\t"
            "s_waitcnt vmcnt(0)\n\t"
            "s_memtime %1\n\t"
            "s_waitcnt lgkmcnt(0)"
            : "=&s"(t0), "=&s"(t1), "=&v"(j)
            : "v"(addr)
            : "memory");
    } else if constexpr (FLAVOR == PCHASE_LOAD_L2) {
        asm volatile(
            "s_memtime %0\n\t"
            "s_waitcnt lgkmcnt(0)\n\t"
            "global_load_dword %2, %3, off sc0\n\t"
            "s_waitcnt vmcnt(0)\n\t"
            "s_memtime %1\n\t"
            "s_waitcnt lgkmcnt(0)"
            : "=&s"(t0), "=&s"(t1), "=&v"(j)
            : "v"(addr)
            : "memory");
    } else if constexpr (FLAVOR == PCHASE_LOAD_SYSTEM) {
        asm volatile(
            "s_memtime %0\n\t"
            "s_waitcnt lgkmcnt(0)\n\t"
            "global_load_dword %2, %3, off sc0 sc1\n\t"
            "s_waitcnt vmcnt(0)\n\t"
            "s_memtime %1\n\t"
            "s_waitcnt lgkmcnt(0)"
            : "=&s"(t0), "=&s"(t1), "=&v"(j)
            : "v"(addr)
            : "memory");
    } else {
        asm volatile(
            "s_memtime %0\n\t"
            "s_waitcnt lgkmcnt(0)\n\t"
            "global_load_dword %2, %3, off nt\n\t"
            "s_waitcnt vmcnt(0)\n\t"
            "s_memtime %1\n\t"
            "s_waitcnt lgkmcnt(0)"
            : "=&s"(t0), "=&s"(t1), "=&v"(j)
            : "v"(addr)
            : "memory");
    }
}

// the same segment with the load replaced by a register move
__device__ __forceinline__ void timed_nothing(int32_t& j, uint64_t& t0, uint64_t& t1) {
    asm volatile(
        "s_memtime %0\n\t"
        "s_waitcnt lgkmcnt(0)\n\t"
        "v_mov_b32 %2, 0\n\t"
        "s_memtime %1\n\t"
        "s_waitcnt lgkmcnt(0)"
        : "=&s"(t0), "=&s"(t1), "=&v"(j)
        :
        : "memory");
}

// COMPACT: no index records, latencies as 16-bit values saturated at 65535
// cycles, so that four times as many accesses fit the LDS record store.
template <int FLAVOR, bool COMPACT>
__global__ void __launch_bounds__(64) pchase_walk_kernel(const int32_t* arr, uint32_t j0, uint64_t warm, uint64_t k,
                                                         uint32_t* lat_out, int32_t* idx_out, int32_t* ovh_out) {
    extern __shared__ uint32_t rec[];  // [k] latencies then [k] indices, or [k] 16-bit latencies
    uint16_t* rec16 = reinterpret_cast<uint16_t*>(rec);
    if (threadIdx.x != 0) return;
    int32_t j = (int32_t)j0;
    // preheat: one untimed walk over the cycle
    for (uint64_t i = 0; i < warm; ++i) {
        uint64_t t0, t1;
        int32_t nj;
        timed_load<FLAVOR>(arr + j, nj, t0, t1);
        j = nj;
    }
    j = (int32_t)j0;
    for (uint64_t i = 0; i < k; ++i) {
        uint64_t t0, t1;
        int32_t nj;
        timed_load<FLAVOR>(arr + j, nj, t0, t1);
        if constexpr (COMPACT) {
            const uint64_t d = t1 - t0;
            rec16[i] = (uint16_t)(d < 65535 ? d : 65535);
        } else {
            rec[i] = (uint32_t)(t1 - t0);
            rec[k + i] = (uint32_t)j;
        }
        j = nj;
    }
    // timer overhead: median of 63 empty segments
    uint32_t o[63];
    for (int r = 0; r < 63; ++r) {
        uint64_t t0, t1;
        int32_t z;
        timed_nothing(z, t0, t1);
        o[r] = (uint32_t)(t1 - t0) + (uint32_t)(z & 0);
    }
    for (int a = 1; a < 63; ++a)
        for (int b = a; b > 0 && o[b - 1] > o[b]; --b) {
            uint32_t t = o[b];
            o[b] = o[b - 1];
            o[b - 1] = t;
        }
    *ovh_out = (int32_t)o[31];
    for (uint64_t i = 0; i < k; ++i) {
        if constexpr (COMPACT) {
            lat_out[i] = rec16[i];
        } else {
            lat_out[i] = rec[i];
            idx_out[i] = (int32_t)rec[k + i];
        }
    }
}

using WalkFn = void (*)(const int32_t*, uint32_t, uint64_t, uint64_t, uint32_t*, int32_t*, int32_t*);
template <bool COMPACT>
static WalkFn walk_fn_t(uint32_t flavor) {
    switch (flavor) {
        case PCHASE_LOAD_DEFAULT: return pchase_walk_kernel<PCHASE_LOAD_DEFAULT, COMPACT>;
        case PCHASE_LOAD_L2: return pchase_walk_kernel<PCHASE_LOAD_L2, COMPACT>;
        case PCHASE_LOAD_SYSTEM: return pchase_walk_kernel<PCHASE_LOAD_SYSTEM, COMPACT>;
        default: return pchase_walk_kernel<PCHASE_LOAD_STREAM, COMPACT>;
    }
}
static WalkFn walk_fn(uint32_t flavor, bool compact) {
    return compact ? walk_fn_t<true>(flavor) : walk_fn_t<false>(flavor);
}

static uint64_t lds_record_bytes() {
    static uint64_t cached = 0;
    if (cached) return cached;
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return 64 * 1024;
    uint64_t lim = prop.maxSharedMemoryPerMultiProcessor ? prop.maxSharedMemoryPerMultiProcessor
                                                         : prop.sharedMemPerBlock;
    lim = std::min<uint64_t>(lim, 160 * 1024);
    cached = lim - 1024;  // leave room for static LDS
    return cached;
}

// --------------------------------------------------------- HBM stream ----
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <class V, int ILP>
__global__ void __launch_bounds__(1024) copy_kernel(const V* __restrict__ src, V* __restrict__ dst, uint64_t n) {
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t nthreads = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t base = tid; base < n; base += nthreads * ILP) {
        V v[ILP];
#pragma unroll
        for (int i = 0; i < ILP; ++i) {
            const uint64_t x = base + (uint64_t)i * nthreads;
            if (x < n) v[i] = __builtin_nontemporal_load(src + x);
        }
#pragma unroll
        for (int i = 0; i < ILP; ++i) {
            const uint64_t x = base + (uint64_t)i * nthreads;
            if (x < n) __builtin_nontemporal_store(v[i], dst + x);
        }
    }
}

template <class V>
static hipError_t launch_copy(const void* s, void* d, uint64_t n, uint32_t grid, uint32_t block, uint32_t ilp,
                              hipStream_t stream) {
    const V* src = static_cast<const V*>(s);
    V* dst = static_cast<V*>(d);
    switch (ilp) {
        case 1: hipLaunchKernelGGL((copy_kernel<V, 1>), dim3(grid), dim3(block), 0, stream, src, dst, n); break;
        case 2: hipLaunchKernelGGL((copy_kernel<V, 2>), dim3(grid), dim3(block), 0, stream, src, dst, n); break;
        case 4: hipLaunchKernelGGL((copy_kernel<V, 4>), dim3(grid), dim3(block), 0, stream, src, dst, n); break;
        default: hipLaunchKernelGGL((copy_kernel<V, 8>), dim3(grid), dim3(block), 0, stream, src, dst, n); break;
    }
    return hipGetLastError();
}

// ----------------------------------------------------------- LDS bank ----
// Lane t starts at word t*stride; the array holds its own word addresses
// (in bytes), so "data = sdata[data]" revisits the same word 64 times.
__global__ void __launch_bounds__(64) lds_bank_kernel(uint32_t stride, uint32_t reps, uint32_t* out) {
    __shared__ uint32_t sdata[64 * 64 + 64];
    const uint32_t lds_base = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) uint32_t*)sdata;
    for (uint32_t i = threadIdx.x; i < 64 * 64 + 64; i += 64) sdata[i] = lds_base + i * 4u;
    __syncthreads();
    uint32_t data = lds_base + threadIdx.x * stride * 4u;
    uint64_t best = ~0ull;
    for (uint32_t r = 0; r <= reps; ++r) {
        uint64_t t0, t1;
        uint32_t d = data;
        asm volatile(
            "s_memtime %0\n\t"
            "s_waitcnt lgkmcnt(0)\n\t"
            ".rept 64\n\t"
            "ds_read_b32 %2, %2\n\t"
            "s_waitcnt lgkmcnt(0)\n\t"
            ".endr\n\t"
            "s_memtime %1\n\t"
            "s_waitcnt lgkmcnt(0)"
            : "=&s"(t0), "=&s"(t1), "+v"(d)
            :
            : "memory");
        if (r > 0) best = min(best, t1 - t0);  // r == 0 warms the instruction cache
        data = d;
    }
    if (threadIdx.x == 0) *out = (uint32_t)((best * 100 + 32) / 64);
}

// LDS throughput (Section 6.1): every thread streams words of a 16 KB LDS
// source buffer, ILP independent reads in flight, consecutive lanes on
// consecutive words (no bank conflicts).  With COPY each value read is
// stored to the same place of a second 16 KB buffer (the paper's
// shared-to-shared copy); without it the xor of the values read is kept.
// Either way something observable depends on every access.
constexpr uint32_t kLdsStreamWords = 4096;

template <class V, int ILP, bool COPY>
__global__ void __launch_bounds__(1024) lds_stream_kernel(uint32_t reps, uint32_t* sink) {
    __shared__ __align__(16) uint32_t src[kLdsStreamWords];
    __shared__ __align__(16) uint32_t dst[COPY ? kLdsStreamWords : 4];
    for (uint32_t i = threadIdx.x; i < kLdsStreamWords; i += blockDim.x) src[i] = i * 2654435761u;
    __syncthreads();
    constexpr uint32_t per = sizeof(V) / 4;                 // words per access
    constexpr uint32_t n = kLdsStreamWords / per;           // accesses that fit a buffer
    const V* vs = reinterpret_cast<const V*>(src);
    V* vd = reinterpret_cast<V*>(dst);
    uint32_t acc[ILP];
#pragma unroll
    for (int j = 0; j < ILP; ++j) acc[j] = 0;
#pragma unroll 1   // reads in flight = ILP: each round waits for its own reads
    for (uint32_t r = 0; r < reps; ++r) {
        V v[ILP];
#pragma unroll
        for (int j = 0; j < ILP; ++j) v[j] = vs[(threadIdx.x + (r * ILP + j) * blockDim.x) & (n - 1)];
#pragma unroll
        for (int j = 0; j < ILP; ++j) {
            if constexpr (COPY) {
                vd[(threadIdx.x + (r * ILP + j) * blockDim.x) & (n - 1)] = v[j];
            } else if constexpr (sizeof(V) == 4) {
                acc[j] ^= (uint32_t)v[j];
            } else {
                acc[j] ^= v[j].x ^ v[j].y ^ v[j].z ^ v[j].w;
            }
        }
    }
    uint32_t x = 0;
    if constexpr (COPY) {
        __syncthreads();
        x = dst[threadIdx.x & (kLdsStreamWords - 1)];
    } else {
#pragma unroll
        for (int j = 0; j < ILP; ++j) x ^= acc[j];
    }
    if (x == 0x9E3779B9u) sink[blockIdx.x] = x;   // practically never: keeps the accesses alive
}

template <class V, bool COPY>
static hipError_t launch_lds_stream(uint32_t grid, uint32_t block, uint32_t ilp, uint32_t reps, uint32_t* sink,
                                    hipStream_t s) {
    switch (ilp) {
        case 1: hipLaunchKernelGGL((lds_stream_kernel<V, 1, COPY>), dim3(grid), dim3(block), 0, s, reps, sink); break;
        case 2: hipLaunchKernelGGL((lds_stream_kernel<V, 2, COPY>), dim3(grid), dim3(block), 0, s, reps, sink); break;
        case 4: hipLaunchKernelGGL((lds_stream_kernel<V, 4, COPY>), dim3(grid), dim3(block), 0, s, reps, sink); break;
        default: hipLaunchKernelGGL((lds_stream_kernel<V, 8, COPY>), dim3(grid), dim3(block), 0, s, reps, sink); break;
    }
    return hipGetLastError();
}

// VALU issue rate: every thread runs 8 independent chains of
// x = (x + c) ^ (x >> 1) (add, shift, xor: three full-rate 32-bit VALU
// instructions per chain and round, a nonlinear map the compiler cannot
// fold across rounds); the xor of the chains decides a store that keeps
// them alive.
constexpr int kValuChains = 8;
constexpr uint32_t kValuOpsPerChainRound = 3;

__global__ void __launch_bounds__(256) valu_kernel(uint32_t reps, uint32_t* sink) {
    uint32_t x[kValuChains];
#pragma unroll
    for (int j = 0; j < kValuChains; ++j) x[j] = threadIdx.x * 2654435761u + (uint32_t)j * 40503u + blockIdx.x;
    for (uint32_t r = 0; r < reps; ++r) {
#pragma unroll
        for (int j = 0; j < kValuChains; ++j) x[j] = (x[j] + 0x9E3779B9u + (uint32_t)j) ^ (x[j] >> 1);
    }
    uint32_t y = 0;
#pragma unroll
    for (int j = 0; j < kValuChains; ++j) y ^= x[j];
    if (y == 0x12345678u) sink[blockIdx.x] = y;   // practically never
}

}  // namespace pc

using namespace pc;

extern "C" int microbench_valu(uint32_t blocks_per_cu, uint32_t reps, double* lane_ops_per_s, hipStream_t stream) {
    if (!lane_ops_per_s) return set_error(PCHASE_EINVAL, "lane_ops_per_s is NULL");
    if (blocks_per_cu == 0 || blocks_per_cu > 32) return set_error(PCHASE_EINVAL, "blocks_per_cu must be 1..32");
    if (reps == 0) return set_error(PCHASE_EINVAL, "reps must be >= 1");
    Workspace* ws;
    std::unique_lock<std::mutex> lk;
    int rc = workspace(&ws, &lk);
    if (rc) return rc;
    const uint32_t grid = blocks_per_cu * (uint32_t)ws->cus;
    hipError_t e = ws->aux.ensure((size_t)grid * 4);
    if (e != hipSuccess) return set_error(PCHASE_ENOMEM, "aux: %s", hipGetErrorString(e));
    uint32_t* sink = ws->aux.as<uint32_t>();
    hipLaunchKernelGGL(valu_kernel, dim3(grid), dim3(256), 0, stream, reps, sink);   // warm-up
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "valu kernel");
    hipEvent_t a = nullptr, b = nullptr;
    float ms = 0;
    e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    if (e == hipSuccess) e = hipEventRecord(a, stream);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(valu_kernel, dim3(grid), dim3(256), 0, stream, reps, sink);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(b, stream);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (e != hipSuccess) return hip_fail(e, "valu kernel");
    const double ops = (double)grid * 256.0 * reps * kValuChains * kValuOpsPerChainRound;
    *lane_ops_per_s = ops / (ms * 1e-3);
    return PCHASE_OK;
}

extern "C" int microbench_lds_stream(uint32_t blocks_per_cu, uint32_t block, uint32_t ilp, uint32_t width_bytes,
                                     uint32_t copy, uint32_t reps, double* gbps, hipStream_t stream) {
    if (!gbps) return set_error(PCHASE_EINVAL, "gbps is NULL");
    if (blocks_per_cu == 0 || blocks_per_cu > 32) return set_error(PCHASE_EINVAL, "blocks_per_cu must be 1..32");
    if (block == 0 || block > 1024 || block % 64) return set_error(PCHASE_EINVAL, "block must be a multiple of 64 up to 1024");
    if (ilp != 1 && ilp != 2 && ilp != 4 && ilp != 8) return set_error(PCHASE_EINVAL, "ilp must be 1, 2, 4 or 8");
    if (width_bytes != 4 && width_bytes != 16) return set_error(PCHASE_EINVAL, "width_bytes must be 4 or 16");
    if (copy > 1) return set_error(PCHASE_EINVAL, "copy must be 0 or 1");
    if (reps == 0) return set_error(PCHASE_EINVAL, "reps must be >= 1");
    Workspace* ws;
    std::unique_lock<std::mutex> lk;
    int rc = workspace(&ws, &lk);
    if (rc) return rc;
    const uint32_t grid = blocks_per_cu * (uint32_t)ws->cus;
    hipError_t e = ws->aux.ensure((size_t)grid * 4);
    if (e != hipSuccess) return set_error(PCHASE_ENOMEM, "aux: %s", hipGetErrorString(e));
    uint32_t* sink = ws->aux.as<uint32_t>();
    auto run = [&]() -> hipError_t {
        if (copy)
            return width_bytes == 4 ? launch_lds_stream<uint32_t, true>(grid, block, ilp, reps, sink, stream)
                                    : launch_lds_stream<uint4, true>(grid, block, ilp, reps, sink, stream);
        return width_bytes == 4 ? launch_lds_stream<uint32_t, false>(grid, block, ilp, reps, sink, stream)
                                : launch_lds_stream<uint4, false>(grid, block, ilp, reps, sink, stream);
    };
    e = run();   // warm-up
    if (e != hipSuccess) return hip_fail(e, "lds stream kernel");
    hipEvent_t a = nullptr, b = nullptr;
    float ms = 0;
    e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    if (e == hipSuccess) e = hipEventRecord(a, stream);
    if (e == hipSuccess) e = run();
    if (e == hipSuccess) e = hipEventRecord(b, stream);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (e != hipSuccess) return hip_fail(e, "lds stream kernel");
    const double bytes = (double)grid * block * reps * ilp * width_bytes * (copy ? 2 : 1);
    *gbps = bytes / (ms * 1e-3) / 1e9;
    return PCHASE_OK;
}

extern "C" uint64_t pchase_microbench_max_k(void) { return lds_record_bytes() / 8; }

extern "C" int microbench_pchase(const pchase_probe* probe, uint32_t flavor, void* array_dev, uint64_t array_bytes,
                                 uint64_t k, uint32_t* lat_dev, int32_t* idx_dev, int32_t* overhead_cycles,
                                 hipStream_t stream) {
    if (!probe || !array_dev || !lat_dev || !overhead_cycles) return set_error(PCHASE_EINVAL, "NULL argument");
    const bool compact = idx_dev == nullptr;
    if (flavor > PCHASE_LOAD_STREAM) return set_error(PCHASE_EINVAL, "unknown load flavour %u", flavor);
    DevProbe dp;
    uint64_t len = 0;
    int rc = check_probe(*probe, &dp, &len, 0);
    if (rc) return rc;
    if (probe->base_offset + probe->n_bytes > array_bytes)
        return set_error(PCHASE_ERANGE, "array of %llu bytes is smaller than base_offset + N",
                         (unsigned long long)array_bytes);
    if ((uintptr_t)array_dev % 4) return set_error(PCHASE_EINVAL, "array_dev must be 4-byte aligned");
    const uint64_t maxk = compact ? lds_record_bytes() / 2 : pchase_microbench_max_k();
    if (k == 0 || k > maxk)
        return set_error(PCHASE_ERANGE, "k = %llu outside [1, %llu] (LDS record capacity)", (unsigned long long)k,
                         (unsigned long long)maxk);
    Workspace* ws;
    std::unique_lock<std::mutex> lk;
    rc = workspace(&ws, &lk);
    if (rc) return rc;
    int32_t* arr = reinterpret_cast<int32_t*>(static_cast<uint8_t*>(array_dev) + probe->base_offset);
    hipLaunchKernelGGL(pchase_init_kernel, dim3(1024), dim3(256), 0, stream, arr, dp.ne, dp.se);
    PC_HIP(hipGetLastError());
    const size_t lds = (size_t)k * (compact ? 2 : 8);
    WalkFn fn = walk_fn(flavor, compact);
    PC_HIP(hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_record_bytes()));
    hipError_t e = ws->aux.ensure(256);
    if (e != hipSuccess) return set_error(PCHASE_ENOMEM, "aux: %s", hipGetErrorString(e));
    int32_t* d_ovh = ws->aux.as<int32_t>();
    const uint64_t warm = dp.L < k ? (uint64_t)dp.L : k;
    hipLaunchKernelGGL(fn, dim3(1), dim3(64), lds, stream, arr, dp.j0, warm, k, lat_dev, idx_dev, d_ovh);
    PC_HIP(hipGetLastError());
    CopyFence fence(stream);
    PC_HIP(hipMemcpyAsync(overhead_cycles, d_ovh, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
    PC_HIP(hipStreamSynchronize(stream));
    fence.done();
    return PCHASE_OK;
}

extern "C" int microbench_hbm_stream(const void* src_dev, void* dst_dev, uint64_t bytes, uint32_t dtype,
                                     uint32_t grid, uint32_t block, uint32_t ilp, uint32_t reps, double* gbps,
                                     hipStream_t stream) {
    if (!src_dev || !dst_dev || !gbps) return set_error(PCHASE_EINVAL, "NULL argument");
    if (dtype > 1) return set_error(PCHASE_EINVAL, "dtype must be 0 (4-byte) or 1 (16-byte)");
    const uint64_t w = dtype ? 16 : 4;
    if (bytes == 0 || bytes % w) return set_error(PCHASE_EINVAL, "bytes must be a positive multiple of %llu",
                                                  (unsigned long long)w);
    if (grid == 0 || block == 0 || block > 1024 || block % 64) return set_error(PCHASE_EINVAL, "bad grid/block");
    if (ilp != 1 && ilp != 2 && ilp != 4 && ilp != 8) return set_error(PCHASE_EINVAL, "ilp must be 1, 2, 4 or 8");
    if (reps == 0) return set_error(PCHASE_EINVAL, "reps must be >= 1");
    const uint64_t n = bytes / w;
    // warm-up launch (first-touch, code load)
    hipError_t e = dtype ? launch_copy<f32x4>(src_dev, dst_dev, n, grid, block, ilp, stream)
                         : launch_copy<float>(src_dev, dst_dev, n, grid, block, ilp, stream);
    if (e != hipSuccess) return hip_fail(e, "copy kernel");
    hipEvent_t a = nullptr, b = nullptr;
    float ms = 0;
    e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    if (e == hipSuccess) e = hipEventRecord(a, stream);
    for (uint32_t r = 0; r < reps && e == hipSuccess; ++r)
        e = dtype ? launch_copy<f32x4>(src_dev, dst_dev, n, grid, block, ilp, stream)
                  : launch_copy<float>(src_dev, dst_dev, n, grid, block, ilp, stream);
    if (e == hipSuccess) e = hipEventRecord(b, stream);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (e != hipSuccess) return hip_fail(e, "copy kernel");
    *gbps = 2.0 * (double)bytes * reps / (ms * 1e-3) / 1e9;
    return PCHASE_OK;
}

extern "C" int microbench_lds_bank(uint32_t stride_lo, uint32_t stride_hi, uint32_t reps, uint32_t* cycles_dev,
                                   hipStream_t stream) {
    if (!cycles_dev) return set_error(PCHASE_EINVAL, "cycles_dev is NULL");
    if (stride_lo == 0 || stride_hi < stride_lo || stride_hi > 64)
        return set_error(PCHASE_EINVAL, "strides must satisfy 1 <= lo <= hi <= 64");
    if (reps == 0) return set_error(PCHASE_EINVAL, "reps must be >= 1");
    for (uint32_t s = stride_lo; s <= stride_hi; ++s) {
        hipLaunchKernelGGL(lds_bank_kernel, dim3(1), dim3(64), 0, stream, s, reps, cycles_dev + (s - stride_lo));
        PC_HIP(hipGetLastError());
    }
    PC_HIP(hipStreamSynchronize(stream));
    return PCHASE_OK;
}
