// misc_kernels.hip -- trace generation (Listing 1 + Listing 2), latency
// classification (Section 4.1, t = t0 + tm*r), exact argmin over candidate
// scores and small fill kernels.
#include "common.h"

namespace pc {

// ------------------------------------------------------ trace generation --
// Probe p's k-th access visits (j0 + k*se) mod ne; each thread writes a run
// of consecutive accesses, computing the first with one modulo and the rest
// by adding se with a conditional wrap.
constexpr int kTraceRun = 16;

__global__ void __launch_bounds__(256) trace_kernel(const DevProbe* probes, const uint64_t* off,
                                                    uint32_t n_probes, int32_t* idx) {
    const uint32_t p = blockIdx.x;
    if (p >= n_probes) return;
    const DevProbe pr = probes[p];
    const uint64_t len = off[p + 1] - off[p];
    int32_t* out = idx + off[p];
    const uint64_t step = (uint64_t)gridDim.y * blockDim.x * kTraceRun;
    for (uint64_t k = ((uint64_t)blockIdx.y * blockDim.x + threadIdx.x) * kTraceRun; k < len; k += step) {
        const uint64_t kc = k % pr.L;
        uint64_t j = (pr.j0 + kc * (uint64_t)pr.se) % pr.ne;
        uint64_t kk = kc;
#pragma unroll
        for (int i = 0; i < kTraceRun; ++i) {
            if (k + i < len) out[k + i] = (int32_t)j;
            ++kk;
            if (kk == pr.L) {
                kk = 0;
                j = pr.j0;
            } else {
                j += pr.se;
                if (j >= pr.ne) j -= pr.ne;
            }
        }
    }
}

hipError_t launch_trace(const DevProbe* probes, const uint64_t* off, uint32_t n_probes, uint64_t maxlen,
                        int32_t* idx, hipStream_t stream) {
    uint64_t per_block = 256ull * kTraceRun;
    uint64_t y = (maxlen + per_block - 1) / per_block;
    if (y < 1) y = 1;
    if (y > 65535) y = 65535;
    hipLaunchKernelGGL(trace_kernel, dim3(n_probes, (uint32_t)y), dim3(256), 0, stream, probes, off,
                       n_probes, idx);
    return hipGetLastError();
}

// ------------------------------------------------------------- fills ----
__global__ void fill_u32_kernel(uint32_t* p, uint64_t n, uint32_t v) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

hipError_t launch_fill_u32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    uint64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(fill_u32_kernel, dim3((uint32_t)blocks), dim3(256), 0, stream, p, n, v);
    return hipGetLastError();
}

// ------------------------------------------------------------- argmin ---
// best = argmin over candidates with n > 0 of m/n, compared exactly as
// m_i * n_j < m_j * n_i in 128 bits, ties to the lower index.


__device__ __forceinline__ bool better(uint64_t mi, uint64_t ni, uint32_t i, uint64_t mj, uint64_t nj,
                                       uint32_t j) {
    // lhs = mi*nj, rhs = mj*ni
    const uint64_t lh = __umul64hi(mi, nj), ll = mi * nj;
    const uint64_t rh = __umul64hi(mj, ni), rl = mj * ni;
    if (lh != rh) return lh < rh;
    if (ll != rl) return ll < rl;
    return i < j;
}

__global__ void __launch_bounds__(1024) argmin_kernel(const uint64_t* m, const uint64_t* n, uint32_t nc,
                                                      uint32_t* zero_bits, ArgminOut* out) {
    __shared__ uint64_t sm[1024], sn[1024];
    __shared__ uint32_t si[1024];
    __shared__ unsigned long long zeros;
    if (threadIdx.x == 0) zeros = 0;
    __syncthreads();
    uint64_t bm = 0, bn = 0;
    uint32_t bi = 0xFFFFFFFFu;
    uint64_t z = 0;
    for (uint32_t c = threadIdx.x; c < nc; c += blockDim.x) {
        const uint64_t mc = m[c], ncmp = n[c];
        if (ncmp == 0) continue;
        if (mc == 0) {
            ++z;
            if (zero_bits) atomicOr(zero_bits + (c >> 5), 1u << (c & 31));
        }
        if (bi == 0xFFFFFFFFu || better(mc, ncmp, c, bm, bn, bi)) {
            bm = mc;
            bn = ncmp;
            bi = c;
        }
    }
    atomicAdd(&zeros, (unsigned long long)z);
    sm[threadIdx.x] = bm;
    sn[threadIdx.x] = bn;
    si[threadIdx.x] = bi;
    __syncthreads();
    for (uint32_t s = blockDim.x / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            const uint32_t o = threadIdx.x + s;
            if (si[o] != 0xFFFFFFFFu &&
                (si[threadIdx.x] == 0xFFFFFFFFu ||
                 better(sm[o], sn[o], si[o], sm[threadIdx.x], sn[threadIdx.x], si[threadIdx.x]))) {
                sm[threadIdx.x] = sm[o];
                sn[threadIdx.x] = sn[o];
                si[threadIdx.x] = si[o];
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out->best = si[0] == 0xFFFFFFFFu ? -1 : (int64_t)si[0];
        out->m = sm[0];
        out->n = sn[0];
        out->n_zero = zeros;
    }
}

hipError_t launch_argmin(const uint64_t* m, const uint64_t* n, uint32_t nc, uint32_t* zero_bits,
                         ArgminOut* out, hipStream_t stream) {
    hipLaunchKernelGGL(argmin_kernel, dim3(1), dim3(1024), 0, stream, m, n, nc, zero_bits, out);
    return hipGetLastError();
}

// ------------------------------------------------ latency classification --
// Automatic threshold: the lower end of the widest gap between consecutive
// distinct latency values.  Values are marked in a presence bitmap over
// [lo, hi]; one block then scans the bitmap in 1024 contiguous slices and
// combines the slices in order (strictly wider gaps win, so the lowest of
// equally wide gaps is kept).
__global__ void minmax_kernel(const uint32_t* lat, uint64_t n, uint32_t* mm) {
    uint32_t lo = 0xFFFFFFFFu, hi = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        lo = min(lo, lat[i]);
        hi = max(hi, lat[i]);
    }
    atomicMin(mm, lo);
    atomicMax(mm + 1, hi);
}

__global__ void mark_kernel(const uint32_t* lat, uint64_t n, const uint32_t* mm, uint32_t* present,
                            uint64_t max_bits) {
    const uint32_t lo = mm[0];
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t v = lat[i] - lo;
        if (v < max_bits) atomicOr(present + (v >> 5), 1u << (v & 31));
    }
}

__global__ void __launch_bounds__(1024) gap_kernel(const uint32_t* mm, const uint32_t* present,
                                                   uint32_t* theta, uint64_t max_bits) {
    __shared__ uint32_t first[1024], last[1024], gap[1024], gap_lo[1024];
    const uint32_t lo = mm[0], hi = mm[1];
    const uint64_t range = (uint64_t)hi - lo + 1;
    if (range > max_bits) {  // the host reports the overflow
        if (threadIdx.x == 0) *theta = 0xFFFFFFFFu;
        return;
    }
    const uint64_t per = (range + blockDim.x - 1) / blockDim.x;
    const uint64_t b = per * threadIdx.x, e = min(range, b + per);
    uint32_t f = 0xFFFFFFFFu, l = 0xFFFFFFFFu, g = 0, glo = 0;
    for (uint64_t v = b; v < e; ++v) {
        if ((present[v >> 5] >> (v & 31)) & 1u) {
            if (f == 0xFFFFFFFFu) f = (uint32_t)v;
            else if ((uint32_t)v - l > g) {
                g = (uint32_t)v - l;
                glo = l;
            }
            l = (uint32_t)v;
        }
    }
    first[threadIdx.x] = f;
    last[threadIdx.x] = l;
    gap[threadIdx.x] = g;
    gap_lo[threadIdx.x] = glo;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t prev = 0xFFFFFFFFu, bg = 0, blo = hi - lo;
        for (uint32_t t = 0; t < blockDim.x; ++t) {
            if (first[t] == 0xFFFFFFFFu) continue;
            if (prev != 0xFFFFFFFFu && first[t] - prev > bg) {
                bg = first[t] - prev;
                blo = prev;
            }
            if (gap[t] > bg) {
                bg = gap[t];
                blo = gap_lo[t];
            }
            prev = last[t];
        }
        *theta = lo + blo;
    }
}

hipError_t launch_auto_threshold(const uint32_t* lat, uint64_t n, uint32_t* mm, uint32_t* present,
                                 uint64_t max_bits, uint32_t* theta, hipStream_t stream) {
    hipLaunchKernelGGL(minmax_kernel, dim3(256), dim3(256), 0, stream, lat, n, mm);
    hipLaunchKernelGGL(mark_kernel, dim3(256), dim3(256), 0, stream, lat, n, mm, present, max_bits);
    hipLaunchKernelGGL(gap_kernel, dim3(1), dim3(1024), 0, stream, mm, present, theta, max_bits);
    return hipGetLastError();
}


// hit bit of probe p's access k = (lat <= theta); one thread per output word
__global__ void classify_kernel(const uint32_t* lat, const uint64_t* lat_off, const uint64_t* bitoff,
                                uint32_t n_probes, const uint32_t* theta_p, uint32_t* bits) {
    const uint32_t p = blockIdx.x;
    if (p >= n_probes) return;
    const uint32_t theta = *theta_p;
    const uint64_t len = lat_off[p + 1] - lat_off[p];
    const uint64_t words = (len + 31) / 32;
    for (uint64_t w = (uint64_t)blockIdx.y * blockDim.x + threadIdx.x; w < words;
         w += (uint64_t)gridDim.y * blockDim.x) {
        uint32_t v = 0;
        for (uint32_t b = 0; b < 32; ++b) {
            const uint64_t k = w * 32 + b;
            if (k < len && lat[lat_off[p] + k] <= theta) v |= 1u << b;
        }
        bits[bitoff[p] + w] = v;
    }
}

hipError_t launch_classify(const uint32_t* lat, const uint64_t* lat_off, const uint64_t* bitoff,
                           uint32_t n_probes, uint64_t maxlen, const uint32_t* theta, uint32_t* bits,
                           hipStream_t stream) {
    uint64_t words = (maxlen + 31) / 32;
    uint64_t x = (words + 255) / 256;
    if (x < 1) x = 1;
    if (x > 1024) x = 1024;
    hipLaunchKernelGGL(classify_kernel, dim3(n_probes, (uint32_t)x), dim3(256), 0, stream, lat, lat_off,
                       bitoff, n_probes, theta, bits);
    return hipGetLastError();
}

// -------------------------------------------------------- range clear ---
// ranges[2i] = first word, ranges[2i+1] = word count; one block per range
__global__ void clear_ranges_kernel(uint32_t* bits, const uint64_t* ranges, uint32_t n) {
    for (uint32_t r = blockIdx.x; r < n; r += gridDim.x) {
        const uint64_t b = ranges[2 * (uint64_t)r], c = ranges[2 * (uint64_t)r + 1];
        for (uint64_t i = threadIdx.x; i < c; i += blockDim.x) bits[b + i] = 0;
    }
}

hipError_t launch_clear_ranges(uint32_t* bits, const uint64_t* ranges, uint32_t n, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    uint32_t blocks = n < 65536 ? n : 65536;
    hipLaunchKernelGGL(clear_ranges_kernel, dim3(blocks), dim3(256), 0, stream, bits, ranges, n);
    return hipGetLastError();
}

}  // namespace pc
