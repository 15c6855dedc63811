// misc_kernels.hip -- trace generation (Listing 1 + Listing 2), latency
// classification (Section 4.1, t = t0 + tm*r), exact argmin over candidate
// scores and small fill kernels.
#include "sweep_lane.h"

namespace pc {

// ------------------------------------------------------ trace generation --
// One block writes one chunk of 4096 consecutive accesses of one probe (the
// chunks of all probes form a flat 1-D grid; a table built on the device
// from the per-probe chunk offsets gives each block its probe and its chunk
// within the probe in one load).  Each thread computes a
// run of 16 consecutive accesses, the first from the closed form and the
// rest incrementally; the block then transposes the chunk through LDS so
// that consecutive threads store consecutive 16-byte groups of indices
// (coalesced writes; the up to 3 words before and after the chunk's
// 16-byte-aligned middle are stored one by one, whatever the alignment of
// the probe's offset).
constexpr int kTraceRun = 16;
constexpr uint32_t kTraceThreads = 256;
constexpr uint32_t kTraceChunk = kTraceThreads * kTraceRun;
static_assert(kTraceChunk == kTraceChunkAccesses, "chunk size shared with the host");
constexpr uint32_t kTraceLds = kTraceChunk + kTraceChunk / kTraceRun;   // one pad word per run

// v[r] is access 16 * threadIdx.x + r of the chunk starting at access k0.
__device__ inline void store_chunk(const int32_t (&v)[kTraceRun], int32_t* out, uint64_t k0, uint64_t len,
                                   int32_t* buf) {
    const uint32_t t = threadIdx.x;
#pragma unroll
    for (int r = 0; r < kTraceRun; ++r) buf[(kTraceRun + 1) * t + r] = v[r];   // word x at x + x/16
    __syncthreads();
    // 16-byte stores for the part of the chunk that is 16-byte aligned in
    // memory, single words for the up to 3 words before and after it
    int32_t* dst = out + k0;
    const uint32_t n = (uint32_t)((len - k0) < kTraceChunk ? (len - k0) : kTraceChunk);
    const uint32_t h = (uint32_t)((4u - (uint32_t)((reinterpret_cast<uintptr_t>(dst) >> 2) & 3u)) & 3u);
    auto word = [&](uint32_t x) { return buf[x + x / kTraceRun]; };
    if (t < h && t < n) dst[t] = word(t);
    const uint32_t nv = n > h ? (n - h) / 4u : 0u;
#pragma unroll
    for (int i = 0; i < kTraceRun / 4; ++i) {
        const uint32_t q = i * kTraceThreads + t;
        if (q < nv) {
            const uint32_t x = h + 4u * q;
            int4 w;
            w.x = word(x);
            w.y = word(x + 1);
            w.z = word(x + 2);
            w.w = word(x + 3);
            *reinterpret_cast<int4*>(dst + x) = w;
        }
    }
    const uint32_t t0 = h + 4u * nv;
    if (t < 4u && t0 + t < n) dst[t0 + t] = word(t0 + t);
}

// Uniform chase (Listing 1 + Listing 2): access k visits (j0 + (k mod L)*se)
// mod ne.
__global__ void __launch_bounds__(kTraceThreads) trace_kernel(const DevProbe* probes, const uint64_t* off,
                                                              const ChunkRef* chunks, int32_t* idx) {
    __shared__ int32_t buf[kTraceLds];
    const ChunkRef c = chunks[blockIdx.x];
    const uint32_t p = c.probe;
    const DevProbe pr = probes[p];
    const uint64_t len = off[p + 1] - off[p];
    const uint64_t k0 = (uint64_t)c.chunk * kTraceChunk;
    const uint64_t k = k0 + (uint64_t)threadIdx.x * kTraceRun;
    int32_t v[kTraceRun] = {};
    if (k < len) {                        // len < 2^32: 32-bit remainder
        uint64_t kk = (uint32_t)k % (uint32_t)pr.L;
        uint64_t j = (pr.j0 + kk * (uint64_t)pr.se) % pr.ne;
#pragma unroll
        for (int r = 0; r < kTraceRun; ++r) {
            v[r] = (int32_t)j;
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
    store_chunk(v, idx + off[p], k0, len, buf);
}

// Non-uniform-stride chase (Section 5.2 / Fig. 13(b)): access k of a pass
// lies in the segment with the last start <= k and visits
// (pos + se * (k - start)) mod ne; the run moves to the next segment at its
// start and back to the first segment at the end of a pass.
__global__ void __launch_bounds__(kTraceThreads) trace_nu_kernel(const DevNuProbe* probes, const DevNuSeg* segs,
                                                                 const uint64_t* off, const ChunkRef* chunks,
                                                                 int32_t* idx) {
    __shared__ int32_t buf[kTraceLds];
    const ChunkRef c = chunks[blockIdx.x];
    const uint32_t p = c.probe;
    const DevNuProbe pr = probes[p];
    const DevNuSeg* sg = segs + pr.first;
    const uint64_t len = off[p + 1] - off[p];
    const uint64_t k0 = (uint64_t)c.chunk * kTraceChunk;
    const uint64_t k = k0 + (uint64_t)threadIdx.x * kTraceRun;
    int32_t v[kTraceRun] = {};
    if (k < len) {                        // len < 2^32: 32-bit remainder
        const uint64_t kc = (uint32_t)k % (uint32_t)pr.pass_len;
        uint32_t lo = 0, hi = pr.nseg - 1;            // last segment with start <= kc
        while (lo < hi) {
            const uint32_t mid = (lo + hi + 1) / 2;
            if (sg[mid].start <= kc) lo = mid; else hi = mid - 1;
        }
        uint32_t i = lo;
        DevNuSeg cur = sg[i];
        uint64_t next = (i + 1 < pr.nseg) ? sg[i + 1].start : pr.pass_len;
        uint64_t j = (cur.pos + (uint64_t)cur.se * ((kc - cur.start) % pr.ne)) % pr.ne;
        uint64_t kk = kc;
#pragma unroll
        for (int r = 0; r < kTraceRun; ++r) {
            v[r] = (int32_t)j;
            ++kk;
            if (kk == pr.pass_len) {          // pass ends: back to the start
                kk = 0;
                i = 0;
                cur = sg[0];
                next = (pr.nseg > 1) ? sg[1].start : pr.pass_len;
                j = cur.pos;
            } else if (kk == next) {          // next segment
                ++i;
                cur = sg[i];
                next = (i + 1 < pr.nseg) ? sg[i + 1].start : pr.pass_len;
                j = cur.pos;
            } else {
                j += cur.se;
                if (j >= pr.ne) j -= pr.ne;
            }
        }
    }
    store_chunk(v, idx + off[p], k0, len, buf);
}

// Chunk table from the per-trace first chunks: block p writes the entries
// of trace p.
__global__ void __launch_bounds__(256) chunk_table_kernel(const uint64_t* chunk_off, ChunkRef* chunks) {
    const uint32_t p = blockIdx.x;
    const uint64_t c0 = chunk_off[p], n = chunk_off[p + 1] - c0;
    for (uint64_t k = threadIdx.x; k < n; k += blockDim.x) chunks[c0 + k] = ChunkRef{p, (uint32_t)k};
}

hipError_t launch_chunk_table(const uint64_t* chunk_off, uint32_t n_traces, ChunkRef* chunks, hipStream_t stream) {
    if (n_traces == 0) return hipSuccess;
    hipLaunchKernelGGL(chunk_table_kernel, dim3(n_traces), dim3(256), 0, stream, chunk_off, chunks);
    return hipGetLastError();
}

hipError_t launch_trace(const DevProbe* probes, const uint64_t* off, const ChunkRef* chunks, uint64_t n_chunks,
                        int32_t* idx, hipStream_t stream) {
    if (n_chunks == 0) return hipSuccess;
    hipLaunchKernelGGL(trace_kernel, dim3((uint32_t)n_chunks), dim3(kTraceThreads), 0, stream, probes, off, chunks,
                       idx);
    return hipGetLastError();
}

hipError_t launch_trace_nu(const DevNuProbe* probes, const DevNuSeg* segs, const uint64_t* off,
                           const ChunkRef* chunks, uint64_t n_chunks, int32_t* idx, hipStream_t stream) {
    if (n_chunks == 0) return hipSuccess;
    hipLaunchKernelGGL(trace_nu_kernel, dim3((uint32_t)n_chunks), dim3(kTraceThreads), 0, stream, probes, segs, off,
                       chunks, idx);
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

// Two ranges in one launch: p[0 .. n) and q[0 .. nq) set to v.
__global__ void fill2_u32_kernel(uint32_t* p, uint64_t n, uint32_t* q, uint64_t nq, uint32_t v) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n + nq;
         i += (uint64_t)gridDim.x * blockDim.x) {
        if (i < n) p[i] = v;
        else q[i - n] = v;
    }
}

hipError_t launch_fill2_u32(uint32_t* p, uint64_t n, uint32_t* q, uint64_t nq, uint32_t v, hipStream_t stream) {
    if (n + nq == 0) return hipSuccess;
    uint64_t blocks = (n + nq + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(fill2_u32_kernel, dim3((uint32_t)blocks), dim3(256), 0, stream, p, n, q, nq, v);
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

// One block; it clears the zero-class bitmap (nc bits) before setting it.
__global__ void __launch_bounds__(1024) argmin_kernel(const uint64_t* m, const uint64_t* n, uint32_t nc,
                                                      uint32_t* zero_bits, ArgminOut* out) {
    __shared__ uint64_t sm[1024], sn[1024];
    __shared__ uint32_t si[1024];
    __shared__ unsigned long long zeros;
    if (threadIdx.x == 0) zeros = 0;
    if (zero_bits)
        for (uint32_t w = threadIdx.x; w < (nc + 31) / 32; w += blockDim.x) zero_bits[w] = 0;
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

// ------------------------------------------ generalised-candidate scoring --
// Step (iv) of Section 4.2 over replayed hit bitmaps: one wave per (candidate,
// probe) pair, lanes over the pair's words, XOR with the observation,
// population count of the compared bits, one atomic per pair.
__global__ void __launch_bounds__(256) mismatch_kernel(const uint32_t* hits, uint64_t cand_words, const uint32_t* obs,
                                                       const uint64_t* hoff, const uint64_t* obits,
                                                       const uint64_t* cf, const uint64_t* len, uint32_t n_probes,
                                                       uint64_t n_pairs, unsigned long long* m) {
    const uint64_t pair = (uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const uint32_t lane = threadIdx.x & 63;
    if (pair >= n_pairs) return;
    const uint64_t c = pair / n_probes;
    const uint32_t p = (uint32_t)(pair % n_probes);
    const uint32_t* h = hits + c * cand_words + hoff[p];
    const uint32_t* o = obs + obits[p];
    const uint64_t a0 = cf[p], a1 = len[p];
    unsigned long long cnt = 0;
    if (a0 < a1) {
        const uint64_t w0 = a0 >> 5, w1 = (a1 + 31) >> 5;
        for (uint64_t w = w0 + lane; w < w1; w += 64) {
            uint32_t x = h[w] ^ o[w];
            if (w == w0) x &= ~0u << (a0 & 31);
            if (w == w1 - 1 && (a1 & 31)) x &= (1u << (a1 & 31)) - 1u;
            cnt += (unsigned long long)__popc(x);
        }
    }
    for (int s = 32; s > 0; s >>= 1) cnt += __shfl_xor(cnt, s);
    if (lane == 0 && cnt) atomicAdd(m + c, cnt);
}

hipError_t launch_mismatch(const uint32_t* hits, uint64_t cand_words, const uint32_t* obs, const uint64_t* hoff,
                           const uint64_t* obits, const uint64_t* cf, const uint64_t* len, uint32_t n_probes,
                           uint64_t n_pairs, uint64_t* m, hipStream_t stream) {
    if (n_pairs == 0) return hipSuccess;
    const uint64_t blocks = (n_pairs + 3) / 4;
    hipLaunchKernelGGL(mismatch_kernel, dim3((uint32_t)blocks), dim3(256), 0, stream, hits, cand_words, obs, hoff,
                       obits, cf, len, n_probes, n_pairs, reinterpret_cast<unsigned long long*>(m));
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

// Observed misses per probe, the constant term of the mismatch count (one
// wave per probe; lanes take words in turn).
__global__ void obs_zeros_kernel(const uint32_t* bits, const uint64_t* pinfo, uint32_t n, uint64_t* zeros) {
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t p = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (p >= n) return;
    const uint32_t* w = bits + pinfo[3 * (uint64_t)p];
    const uint64_t lo = pinfo[3 * (uint64_t)p + 1], hi = pinfo[3 * (uint64_t)p + 2];
    uint64_t z = 0;
    if (lo < hi) {
        const uint64_t w_lo = lo >> 5, w_hi = (hi - 1) >> 5;
        for (uint64_t i = w_lo + lane; i <= w_hi; i += kWave) {
            uint32_t mask = 0xFFFFFFFFu;
            if (i == w_lo) mask &= 0xFFFFFFFFu << (lo & 31);
            if (i == w_hi && (hi & 31)) mask &= (1u << (hi & 31)) - 1u;
            z += (uint64_t)__popc(~w[i] & mask);
        }
    }
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) z += __shfl_xor(z, off, kWave);
    if (lane == 0) zeros[p] = z;
}

__device__ __forceinline__ int64_t obs_weight(const uint32_t* ob, uint64_t k, uint64_t cf) {
    return k >= cf ? 2 * (int64_t)((ob[k >> 5] >> (k & 31)) & 1u) - 1 : 0;
}

// One wave per run table; lanes take 64 runs at a time and carry the prefix.
__global__ void run_table_kernel(const RunTable* tables, uint32_t n_tables, const DevProbe* probes,
                                 const uint64_t* ks, const uint64_t* pinfo, const uint32_t* bits, int32_t* prefix,
                                 int64_t* s1) {
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t w = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (w >= n_tables) return;
    const RunTable t = tables[w];
    const DevProbe p = probes[t.probe];
    const uint32_t* ob = bits + pinfo[3 * (uint64_t)t.probe];
    const uint64_t cf = pinfo[3 * (uint64_t)t.probe + 1];
    const uint64_t sb = (uint64_t)p.se << p.elem_shift;
    const uint64_t x0 = p.base + ((uint64_t)p.j0 << p.elem_shift);
    const uint64_t l0 = x0 >> t.line_shift;
    // runs are single accesses unless the stride is below the line
    const bool per_line = t.nsw == 0 && t.runs > 1 && sb < (1ull << t.line_shift);
    int32_t* out = prefix + t.off;
    int64_t carry = 0, first = 0;
    for (uint64_t i0 = 0; i0 < t.runs; i0 += kWave) {
        const uint64_t i = i0 + lane;
        int64_t w2 = 0;
        if (i < t.runs) {
            // first access of line l0 + i: ceil((line start - x0) / stride);
            // several sweeps: the (i / nsw)-th access of sweep i mod nsw
            uint64_t k;
            if (t.nsw) k = ks[t.koff + (uint32_t)i % t.nsw] + (uint32_t)i / t.nsw;
            else k = (per_line && i > 0) ? udiv64(((l0 + i) << t.line_shift) - x0 + sb - 1, sb) : i;
            first += obs_weight(ob, k, cf);
            uint64_t kk = k;
            for (uint32_t q = 1; q < p.passes; ++q) {
                kk += p.L;
                w2 += obs_weight(ob, kk, cf);
            }
        }
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            const int64_t o = __shfl_up(w2, d, kWave);
            if ((int)lane >= d) w2 += o;
        }
        if (i < t.runs) out[i + 1] = (int32_t)(carry + w2);
        carry += __shfl(w2, kWave - 1, kWave);
    }
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) first += __shfl_xor(first, d, kWave);
    if (lane == 0) {
        out[0] = 0;
        s1[w] = first;
    }
}

hipError_t launch_run_tables(const RunTable* tables, uint32_t n_tables, const DevProbe* probes,
                             const uint64_t* ks, const uint64_t* pinfo, const uint32_t* bits, int32_t* prefix,
                             int64_t* s1, hipStream_t stream) {
    if (n_tables == 0) return hipSuccess;
    const uint32_t wpb = 256 / kWave;
    hipLaunchKernelGGL(run_table_kernel, dim3((n_tables + wpb - 1) / wpb), dim3(256), 0, stream, tables, n_tables,
                       probes, ks, pinfo, bits, prefix, s1);
    return hipGetLastError();
}

// One lane per decided job (table order); the score goes to its slot.
__global__ void decided_kernel(const DecidedJob* dj, uint32_t n, const uint64_t* zeros, const RunTable* tables,
                               const int32_t* prefix, const int64_t* s1, const PlruPattern* pats,
                               const uint32_t* pat_bits, int64_t* vals) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const DecidedJob j = dj[i];
        int64_t v = (int64_t)zeros[j.probe];
        if (j.kind >= 1) v += s1[j.table];
        if (j.kind >= 2) {
            const RunTable t = tables[j.table];
            const int32_t* P = prefix + t.off;
            if (j.kind == 2) {
                v += (int64_t)P[t.runs];
            } else if (j.kind == 3) {
                for (uint64_t st = 0; st < t.runs; st += j.period) {
                    const uint64_t hi = st + j.rem < t.runs ? st + j.rem : t.runs;
                    v += (int64_t)P[hi] - (int64_t)P[st];
                }
            } else {
                // position i covers runs [i T', i T' + rem) of the big sets
                // (pattern pat_big) then [i T' + rem, (i + 1) T') of the
                // small ones (pat_small): in run order the missing ranges
                // are merged, and the prefix is read at their ends only
                const PlruPattern pb = pats[j.pat_big], ps = pats[j.pat_small];
                const uint32_t* wb = pat_bits + (pb.off >> 5);
                const uint32_t* wsm = pat_bits + (ps.off >> 5);
                const uint32_t nb = j.rem ? pb.lines : 0u, nsm = ps.lines;
                const uint32_t npos = nb > nsm ? nb : nsm;
                bool open = false;
                uint64_t from = 0;
                uint32_t bw = 0, sw = 0;
                for (uint32_t i = 0; i < npos; ++i) {
                    if ((i & 31) == 0) {
                        bw = i < nb ? wb[i >> 5] : 0u;
                        sw = i < nsm ? wsm[i >> 5] : 0u;
                    }
                    const uint64_t st = (uint64_t)i * j.period;
                    const uint64_t mid = st + j.rem < t.runs ? st + j.rem : t.runs;
                    const bool mb = i < nb && ((bw >> (i & 31)) & 1u);
                    const bool ms = i < nsm && ((sw >> (i & 31)) & 1u);
                    if (mb != open) {   // a range opens or closes at st
                        if (mb) from = st;
                        else v += (int64_t)P[st] - (int64_t)P[from];
                        open = mb;
                    }
                    if (ms != open) {   // ... or at mid
                        if (ms) from = mid;
                        else v += (int64_t)P[mid] - (int64_t)P[from];
                        open = ms;
                    }
                }
                if (open) {
                    const uint64_t end = (uint64_t)npos * j.period < t.runs ? (uint64_t)npos * j.period : t.runs;
                    v += (int64_t)P[end] - (int64_t)P[from];
                }
            }
        }
        vals[j.slot] = v;
    }
}

// One lane per slot (candidate order): a segmented wave sum over runs of one
// candidate, one atomic per run.
__global__ void decided_sum_kernel(const int64_t* vals, const uint32_t* cand, uint32_t n, uint64_t* m) {
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t key = 0xFFFFFFFFu;
    int64_t v = 0;
    if (q < n) {
        key = cand[q];
        v = vals[q];
    }
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const int64_t o = __shfl_down(v, off, kWave);
        const uint32_t ok = __shfl_down(key, off, kWave);
        if ((int)lane + off < kWave && ok == key) v += o;
    }
    const uint32_t up = __shfl_up(key, 1, kWave);
    if (key != 0xFFFFFFFFu && (lane == 0 || up != key) && v != 0)
        atomicAdd(reinterpret_cast<unsigned long long*>(m + key), (unsigned long long)v);
}

hipError_t launch_decided(const DecidedJob* dj, uint32_t n, const uint64_t* zeros, const RunTable* tables,
                          const int32_t* prefix, const int64_t* s1, const PlruPattern* pats,
                          const uint32_t* pat_bits, int64_t* vals, const uint32_t* cand, uint64_t* m,
                          hipStream_t stream) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(decided_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, dj, n, zeros, tables, prefix,
                       s1, pats, pat_bits, vals);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(decided_sum_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, vals, cand, n, m);
    return hipGetLastError();
}

// One lane per pattern: the set's way -> line and line -> way maps live in
// the lane's scratch words; the tree bits in registers.
__global__ void plru_pattern_kernel(const PlruPattern* pd, uint32_t n, uint32_t* bits, uint32_t* scratch) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const PlruPattern p = pd[t];
    uint32_t* way_line = scratch + p.scr;
    uint32_t* line_way = way_line + p.ways;
    uint32_t* out = bits + (p.off >> 5);
    for (uint32_t w = 0; w < p.ways; ++w) way_line[w] = kInvalidTag;
    for (uint32_t x = 0; x < p.lines; ++x) line_way[x] = kInvalidTag;
    for (uint32_t w = 0; w < (p.lines + 31) / 32; ++w) out[w] = 0;
    PlruBits tree;
    uint32_t nvalid = 0;
    for (uint32_t pass = 0; pass < 2; ++pass) {
        for (uint32_t x = 0; x < p.lines; ++x) {
            uint32_t w = line_way[x];
            const bool hit = w != kInvalidTag;
            if (!hit) {
                w = nvalid < p.ways ? nvalid++ : tree.victim(p.log2_ways, p.ways);
                const uint32_t old = way_line[w];
                if (old != kInvalidTag) line_way[old] = kInvalidTag;
                way_line[w] = x;
                line_way[x] = w;
                if (pass == 1) out[x >> 5] |= 1u << (x & 31);
            }
            tree.touch(w, p.log2_ways);
        }
    }
}

hipError_t launch_plru_patterns(const PlruPattern* pd, uint32_t n, uint32_t* bits, uint32_t* scratch,
                                hipStream_t stream) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(plru_pattern_kernel, dim3((n + 63) / 64), dim3(64), 0, stream, pd, n, bits, scratch);
    return hipGetLastError();
}

hipError_t launch_obs_zeros(const uint32_t* bits, const uint64_t* pinfo, uint32_t n, uint64_t* zeros,
                            hipStream_t stream) {
    if (n == 0) return hipSuccess;
    const uint32_t wpb = 256 / kWave;
    hipLaunchKernelGGL(obs_zeros_kernel, dim3((n + wpb - 1) / wpb), dim3(256), 0, stream, bits, pinfo, n, zeros);
    return hipGetLastError();
}

}  // namespace pc
