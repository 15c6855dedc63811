// planner.hip -- adaptive probe planning: the two-stage procedure of
// Sec. 4.2 (Fig. 6), where each next (N, s) is chosen from what the earlier
// runs showed, generalised to a greedy choice among a pool of probes.
//
// Every candidate is replayed once on every pool probe; on each probe the
// candidates fall into classes of identical steady-pass hit bits (accesses
// L .. len-1), each class named by its lowest candidate.  Given the
// surviving candidates, the next probe is the one whose largest class among
// them is smallest, then the one with more classes, then the lowest index.
// The class matrix is kept for the next call with the same candidates and
// pool, so the loop (choose, observe, keep the target's class) costs one
// scoring launch per step.
#include <cstring>

#include "host_common.h"
#include "plan.h"

namespace pc {

// Steady bit window of one (candidate, probe) bitmap: word i holds bits
// L + 32 i .. L + 32 i + 31 (zero past len).
__device__ __forceinline__ uint32_t steady_word(const uint32_t* bits, uint32_t L, uint32_t len, uint32_t i) {
    const uint32_t b0 = L + 32u * i;
    const uint32_t w = b0 >> 5, sh = b0 & 31u;
    uint64_t v = bits[w];
    if (sh && b0 + 32u - sh < len) v |= (uint64_t)bits[w + 1] << 32;
    uint32_t x = (uint32_t)(v >> sh);
    const uint32_t left = len - b0;
    if (left < 32u) x &= (1u << left) - 1u;
    return x;
}

struct PlanProbe {
    uint64_t bitbase;   // word offset of candidate 0's bitmap on this probe
    uint32_t words;     // words per candidate bitmap
    uint32_t L;         // steady bits start here
    uint32_t len;       // trace length
    uint32_t pad;
};

// h[p * nc + c]: 64-bit hash of candidate c's steady bits on probe p.
__global__ void __launch_bounds__(256) plan_hash_kernel(const PlanProbe* probes, const uint32_t* bits, uint32_t np,
                                                        uint32_t nc, uint64_t* h) {
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (uint64_t)np * nc) return;
    const uint32_t p = (uint32_t)(t / nc), c = (uint32_t)(t % nc);
    const PlanProbe pr = probes[p];
    const uint32_t* b = bits + pr.bitbase + (uint64_t)c * pr.words;
    const uint32_t n = (pr.len - pr.L + 31u) / 32u;
    uint64_t x = 0x243F6A8885A308D3ull ^ n;
    for (uint32_t i = 0; i < n; ++i) {
        x ^= steady_word(b, pr.L, pr.len, i);
        x *= 0xFF51AFD7ED558CCDull;
        x ^= x >> 33;
    }
    h[t] = x;
}

// cls[p * nc + c] = lowest c' <= c with the same steady bits on probe p
// (hash first, then word by word).
__global__ void __launch_bounds__(256) plan_class_kernel(const PlanProbe* probes, const uint32_t* bits,
                                                         const uint64_t* h, uint32_t np, uint32_t nc,
                                                         uint32_t* cls) {
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (uint64_t)np * nc) return;
    const uint32_t p = (uint32_t)(t / nc), c = (uint32_t)(t % nc);
    const PlanProbe pr = probes[p];
    const uint64_t* hp = h + (uint64_t)p * nc;
    const uint64_t mine = hp[c];
    const uint32_t* bc = bits + pr.bitbase + (uint64_t)c * pr.words;
    const uint32_t n = (pr.len - pr.L + 31u) / 32u;
    uint32_t out = c;
    for (uint32_t d = 0; d < c; ++d) {
        if (hp[d] != mine) continue;
        const uint32_t* bd = bits + pr.bitbase + (uint64_t)d * pr.words;
        bool same = true;
        for (uint32_t i = 0; i < n && same; ++i)
            same = steady_word(bc, pr.L, pr.len, i) == steady_word(bd, pr.L, pr.len, i);
        if (same) {
            out = d;
            break;
        }
    }
    cls[t] = out;
}

// One block per probe: class sizes of the alive candidates in LDS, then the
// key (largest class, nc - classes, probe) into an atomic minimum.
__global__ void __launch_bounds__(256) plan_score_kernel(const uint32_t* cls, const uint32_t* alive, uint32_t np,
                                                         uint32_t nc, unsigned long long* best) {
    extern __shared__ uint32_t hist[];
    const uint32_t p = blockIdx.x;
    if (p >= np) return;
    for (uint32_t c = threadIdx.x; c < nc; c += blockDim.x) hist[c] = 0;
    __syncthreads();
    const uint32_t* row = cls + (uint64_t)p * nc;
    for (uint32_t c = threadIdx.x; c < nc; c += blockDim.x)
        if ((alive[c >> 5] >> (c & 31)) & 1u) atomicAdd(&hist[row[c]], 1u);
    __syncthreads();
    uint32_t worst = 0, classes = 0;
    for (uint32_t c = threadIdx.x; c < nc; c += blockDim.x) {
        worst = max(worst, hist[c]);
        classes += hist[c] ? 1u : 0u;
    }
    __shared__ uint32_t rw[256], rc[256];
    rw[threadIdx.x] = worst;
    rc[threadIdx.x] = classes;
    __syncthreads();
    for (uint32_t s = blockDim.x / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            rw[threadIdx.x] = max(rw[threadIdx.x], rw[threadIdx.x + s]);
            rc[threadIdx.x] += rc[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const unsigned long long key = ((unsigned long long)rw[0] << 42) |
                                       ((unsigned long long)(nc - rc[0]) << 21) | (unsigned long long)p;
        atomicMin(best, key);
    }
}

constexpr uint32_t kPlanMaxCands = 1u << 13;   // LDS histogram of 32 KB
constexpr uint32_t kPlanMaxPool = 1u << 20;
constexpr uint64_t kPlanMaxBitBytes = 8ull << 30;

}  // namespace pc

using namespace pc;

extern "C" int pchase_plan_next_probe(const pchase_model* cands, uint32_t n_cands, const pchase_probe* pool,
                                      uint32_t n_pool, const uint32_t* alive_host, uint32_t* classes_dev,
                                      pchase_plan_choice* out, hipStream_t stream) {
    if (!out) return set_error(PCHASE_EINVAL, "out is NULL");
    if (n_cands == 0 || n_pool == 0) return set_error(PCHASE_EINVAL, "needs at least one candidate and one probe");
    if (n_cands > kPlanMaxCands) return set_error(PCHASE_ERANGE, "at most %u candidates", kPlanMaxCands);
    if (n_pool > kPlanMaxPool) return set_error(PCHASE_ERANGE, "at most %u pool probes", kPlanMaxPool);
    if (!alive_host) return set_error(PCHASE_EINVAL, "alive is NULL");
    std::vector<DevModel> dm(n_cands);
    std::vector<DevProbe> dp(n_pool);
    std::vector<uint64_t> len(n_pool);
    if (!cands || !pool) return set_error(PCHASE_EINVAL, "cands or pool is NULL");
    for (uint32_t i = 0; i < n_cands; ++i) {
        int rc = check_model(cands[i], &dm[i], i);
        if (rc) return rc;
    }
    for (uint32_t i = 0; i < n_pool; ++i) {
        int rc = check_probe(pool[i], &dp[i], &len[i], i);
        if (rc) return rc;
    }
    const uint32_t aw = (n_cands + 31) / 32;
    uint32_t n_alive = 0;
    for (uint32_t c = 0; c < n_cands; ++c) n_alive += (alive_host[c >> 5] >> (c & 31)) & 1u;

    Workspace* ws;
    std::unique_lock<std::mutex> lk;
    int rc = workspace(&ws, &lk);
    if (rc) return rc;
    const size_t cls_bytes = (size_t)n_pool * n_cands * sizeof(uint32_t);
    std::string key(reinterpret_cast<const char*>(cands), (size_t)n_cands * sizeof(pchase_model));
    key.append(reinterpret_cast<const char*>(pool), (size_t)n_pool * sizeof(pchase_probe));
    if (ws->planner_key != key) {
        ws->planner_key.clear();
        // every candidate on every probe, hit bits in one bank: probe p's
        // bitmaps start at bitbase[p], one per candidate
        std::vector<PlanProbe> pp(n_pool);
        uint64_t words = 0;
        for (uint32_t p = 0; p < n_pool; ++p) {
            const uint32_t w = (uint32_t)((len[p] + 31) / 32);
            pp[p] = PlanProbe{words, w, dp[p].L, (uint32_t)len[p], 0};
            words += (uint64_t)w * n_cands;
        }
        // jobs grouped by candidate (the sweep plan packs each model's jobs
        // into shared tasks)
        std::vector<SweepJob> jobs;
        jobs.reserve((size_t)n_pool * n_cands);
        for (uint32_t c = 0; c < n_cands; ++c) {
            for (uint32_t p = 0; p < n_pool; ++p) {
                SweepJob j{};
                j.model = c;
                j.probe = p;
                j.out = (uint32_t)jobs.size();
                j.trace_id = p;
                j.count_from = dp[p].L;
                j.bitoff = pp[p].bitbase + (uint64_t)c * pp[p].words;
                jobs.push_back(j);
            }
        }
        if (words * 4 > kPlanMaxBitBytes) return set_error(PCHASE_ERANGE, "pool x candidates needs %llu bytes of hit bits",
                                                           (unsigned long long)(words * 4));
        DevBuf bank;
        hipError_t e = bank.ensure(words * 4 + (size_t)n_pool * n_cands * 8 + n_pool * sizeof(PlanProbe) + 512);
        if (e != hipSuccess) {
            bank.release();
            return set_error(PCHASE_ENOMEM, "planner bank: %s", hipGetErrorString(e));
        }
        uint32_t* d_bits = bank.as<uint32_t>();
        uint64_t* d_h = reinterpret_cast<uint64_t*>(bank.as<uint8_t>() + (words * 4 + 255) / 256 * 256);
        PlanProbe* d_pp = reinterpret_cast<PlanProbe*>(reinterpret_cast<uint8_t*>(d_h) + (size_t)n_pool * n_cands * 8);
        rc = replay_jobs(ws, dm, dp, len, jobs, d_bits, words, stream);
        if (rc) {
            bank.release();
            return rc;
        }
        e = ws->planner.ensure(cls_bytes + aw * 4 + 256);
        if (e != hipSuccess) {
            bank.release();
            return set_error(PCHASE_ENOMEM, "planner classes: %s", hipGetErrorString(e));
        }
        CopyFence fence(stream);
        hipError_t he = hipMemcpyAsync(d_pp, pp.data(), pp.size() * sizeof(PlanProbe), hipMemcpyHostToDevice, stream);
        const uint64_t n = (uint64_t)n_pool * n_cands;
        const uint32_t blocks = (uint32_t)((n + 255) / 256);
        if (he == hipSuccess) {
            hipLaunchKernelGGL(plan_hash_kernel, dim3(blocks), dim3(256), 0, stream, d_pp, d_bits, n_pool, n_cands, d_h);
            he = hipGetLastError();
        }
        if (he == hipSuccess) {
            hipLaunchKernelGGL(plan_class_kernel, dim3(blocks), dim3(256), 0, stream, d_pp, d_bits, d_h, n_pool,
                               n_cands, ws->planner.as<uint32_t>());
            he = hipGetLastError();
        }
        if (he == hipSuccess)
            he = hipStreamSynchronize(stream);   // the bank is freed below
        else
            (void)hipStreamSynchronize(stream);  // nothing queued may outlive the bank or pp
        fence.done();
        bank.release();
        if (he != hipSuccess) return hip_fail(he, "planner classes");
        ws->planner_key = key;
    }
    uint32_t* d_cls = ws->planner.as<uint32_t>();
    uint32_t* d_alive = reinterpret_cast<uint32_t*>(ws->planner.as<uint8_t>() + cls_bytes);
    unsigned long long* d_best =
        reinterpret_cast<unsigned long long*>(ws->planner.as<uint8_t>() + (cls_bytes + aw * 4 + 7) / 8 * 8);
    const unsigned long long init = ~0ull;
    unsigned long long best = 0;
    CopyFence fence(stream);
    PC_HIP(hipMemcpyAsync(d_alive, alive_host, aw * 4, hipMemcpyHostToDevice, stream));
    PC_HIP(hipMemcpyAsync(d_best, &init, sizeof init, hipMemcpyHostToDevice, stream));
    hipLaunchKernelGGL(plan_score_kernel, dim3(n_pool), dim3(256), n_cands * sizeof(uint32_t), stream, d_cls, d_alive,
                       n_pool, n_cands, d_best);
    PC_HIP(hipGetLastError());
    if (classes_dev)
        PC_HIP(hipMemcpyAsync(classes_dev, d_cls, cls_bytes, hipMemcpyDeviceToDevice, stream));
    PC_HIP(hipMemcpyAsync(&best, d_best, sizeof best, hipMemcpyDeviceToHost, stream));
    PC_HIP(hipStreamSynchronize(stream));
    fence.done();
    const uint32_t worst = (uint32_t)(best >> 42), probe = (uint32_t)(best & ((1u << 21) - 1));
    const uint32_t classes = n_cands - (uint32_t)((best >> 21) & ((1u << 21) - 1));
    out->n_alive = n_alive;
    out->worst = n_alive ? worst : 0;
    out->n_classes = n_alive ? classes : 0;
    out->probe = (n_alive == 0 || worst >= n_alive) ? -1 : (int64_t)probe;
    out->reserved = 0;
    return PCHASE_OK;
}
