// sweep_kernels.hip -- replay of P-chase probes through set-associative
// cache models, one lane per (replay, cache set).
//
// Method (Mei & Chu, Section 4.1, Assumptions 1-3; Section 4.2): a probe's
// accesses are j_k = (j0 + k*s) mod N (Listing 1 + Listing 2); access k
// falls in set (address / unit) mod T and only touches that set's a ways,
// so the hit/miss decision of an access depends on the earlier accesses of
// its own set only.  Each lane therefore owns one set of one replay and
// walks that set's accesses in trace order, generating them from (N, s)
// instead of reading a materialised trace: within one increasing sweep of
// the chase the accesses of a set are the accesses that fall in the units
// t, t+T, t+2T, ... and the accesses inside one line are consecutive in the
// trace, so only the first of a run can miss and the others are hits that
// leave the policy state unchanged.
//
// Ways live in registers (a <= 16, loops unrolled to the class bound) or in
// an LDS column per lane (a <= 128).  Hit/miss counts are reduced per replay
// with a segmented wave reduction; per-access hit bits, when requested, are
// or-ed into a caller bitmap.  In scoring mode the lane compares its
// decisions with an observed bitmap instead and accumulates mismatches per
// candidate model.  Every access of a run after its first is a hit, so the
// mismatch count over [cf, len) is the observed misses there (a per-probe
// constant) plus, per modelled miss at k >= cf, +1 if the observation says
// hit and -1 if it says miss: scoring reads the observation only at the
// model's misses.
#include <type_traits>

#include "sweep_lane.h"

namespace pc {

// ------------------------------------------------------- bitmap helpers --
// Trace indices are below 2^32 (traces are shorter than 2^32 accesses).
__device__ __forceinline__ void or_bits(uint32_t* w, uint32_t lo, uint32_t hi) {
    // sets bits [lo, hi)
    while (lo < hi) {
        const uint32_t word = lo >> 5;
        const uint32_t b0 = lo & 31;
        const uint32_t n = (hi - lo < 32 - b0) ? hi - lo : 32 - b0;
        const uint32_t mask = (n == 32) ? 0xFFFFFFFFu : (((1u << n) - 1u) << b0);
        atomicOr(w + word, mask);
        lo += n;
    }
}

// ---------------------------------------------------------------- kernel --


// Per-run bookkeeping of one lane.  With an LDS bitmap (bm != nullptr) the
// run's hit bits are or-ed into it and compared or written out by the whole
// wave afterwards; otherwise they are compared with the observation or or-ed
// into the output bitmap in memory run by run.
// Sets bits [k0 + (hit ? 0 : 1), k0 + r) of an LDS bitmap: the run's hit
// bits.  Runs of up to 32 accesses touch at most two words.
__device__ __forceinline__ void or_run(uint32_t* w, uint32_t k0, uint32_t r, bool hit) {
    if (r <= 32) {
        uint64_t mask = (r == 32) ? 0xFFFFFFFFull : ((1ull << r) - 1ull);
        if (!hit) mask &= ~1ull;
        mask <<= (k0 & 31);
        const uint32_t word = k0 >> 5;
        atomicOr(w + word, (uint32_t)mask);   // or-ing 0 changes nothing: no branch
        if (mask >> 32) atomicOr(w + word + 1, (uint32_t)(mask >> 32));
    } else {
        or_bits(w, hit ? k0 : k0 + 1, k0 + r);
    }
}

template <class S, bool SCORE, bool BM>
struct Visitor {
    S* st;
    const DevModel* m;
    uint32_t trace_id;
    uint32_t cf;
    uint32_t* bits;   // memory bitmap of the job (observed or output), or null
    uint32_t* bm;     // LDS bitmap of the job (BM)
    uint32_t mt = 0;  // replay: misses
    uint32_t ms = 0;  // misses at k >= cf
    uint32_t mp = 0;  // score: misses at k >= cf that the observation calls hits
    __device__ __forceinline__ void operator()(uint32_t line, uint32_t q, uint32_t k0, uint32_t r) {
        const bool hit = st->access(line, q, *m, k0, trace_id);
        if constexpr (SCORE) {
            if (!hit && k0 >= cf) {
                ++ms;
                mp += (bits[k0 >> 5] >> (k0 & 31)) & 1u;
            }
        } else {
            if (!hit) {
                ++mt;
                ms += (k0 >= cf) ? 1u : 0u;
            }
            if constexpr (BM) or_run(bm, k0, r, hit);
            else if (bits != nullptr) or_bits(bits, hit ? k0 : k0 + 1, k0 + r);
        }
    }
};

// Scoring of an LRU or FIFO job whose every pass is one increasing sweep
// (Section 4.1's cyclic P-chase): each line of a set is visited by one run
// per pass, in the same order in every pass.  With n lines in the set and a
// ways, the first pass's run starts miss (cold), and when n > a so does
// every later run start: since a line's last use all n - 1 other lines of
// the set were used, which evicts it under LRU (its reuse distance is at
// least a), and under FIFO (every access so far missed and inserted, so the
// a lines held are the a used just before it).  When n <= a nothing is ever
// evicted.  Every other access hits.  The lane walks the first pass only and
// looks the observation up at every pass's copy of each run start.
struct CycVisitor {
    uint32_t cf, L, passes;
    const uint32_t* bits;
    uint32_t n = 0;               // runs (lines) of the set in a pass
    uint32_t ms1 = 0, mp1 = 0;    // first pass: counted misses, of which the observation calls hits
    uint32_t ms2 = 0, mp2 = 0;    // the later passes, if n > a
    __device__ __forceinline__ void operator()(uint32_t, uint32_t, uint32_t k0, uint32_t) {
        ++n;
        if (k0 >= cf) {
            ++ms1;
            mp1 += (bits[k0 >> 5] >> (k0 & 31)) & 1u;
        }
        uint32_t k = k0;
        for (uint32_t q = 1; q < passes; ++q) {
            k += L;
            if (k >= cf) {
                ++ms2;
                mp2 += (bits[k >> 5] >> (k & 31)) & 1u;
            }
        }
    }
};

__device__ __forceinline__ uint64_t seg_sum(uint64_t v, uint32_t key, int lane) {
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const uint64_t o = __shfl_down(v, off, kWave);
        const uint32_t ok = __shfl_down(key, off, kWave);
        if (lane + off < kWave && ok == key) v += o;
    }
    return v;
}

// Way classes of the kernel template: 1..16 are register classes.
constexpr int kClassMap = 1000;
constexpr int kClassScan = 2000;
constexpr int kClassCyc = 3000;   // closed form (CycVisitor), scoring only
constexpr uint32_t kMaxLdsRows = 240;  // with the bitmap, 64 KB per one-wave block at most

template <int POL, int A, bool SCORE>
__device__ __forceinline__ void run_task(const SweepArgs& args, const SweepTask& task, int lane, uint32_t* col,
                                         uint32_t* bm) {
    const DevModel m = args.models[task.model];
    const bool active = (uint32_t)lane < task.n;
    const bool use_bm = !SCORE && task.bm_words != 0 && args.bits != nullptr;
    const uint32_t T = m.sets;
    const uint32_t G = task.lanes;
    if (use_bm) {
        for (uint32_t w = (uint32_t)lane; w < task.bm_words; w += kWave) bm[w] = 0;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    uint32_t key = kInvalidTag;
    uint32_t mt = 0, ms = 0, mp = 0;   // per lane: below the trace length < 2^32
    uint64_t z = 0;                    // score: the job's observed misses, on its lane g = 0
    if (active) {
        // G lanes per replay (chosen by the plan); lane g of a replay owns
        // the sets g, g+G, g+2G, ... and replays them one after the other
        const uint32_t item = task.item0 + (uint32_t)lane;
        const uint32_t jrel = item / G;
        const uint32_t g = item - jrel * G;
        const SweepJob job = args.jobs[task.job + jrel];
        const DevProbe p = args.probes[job.probe];
        key = job.out;
        if (SCORE && g == 0) z = args.zeros[job.probe];
        uint32_t* bits = (args.bits == nullptr || use_bm) ? nullptr : args.bits + job.bitoff;
        uint32_t* jbm = use_bm ? bm + job.bm_off : nullptr;
        const uint32_t len = p.L * p.passes;
        const uint32_t cf = job.count_from < len ? (uint32_t)job.count_from : len;
        SweepCache sc;
        sweep_cache(sc, p, m);
        // the bitmap choice is uniform over the task: branch once, not per run
        auto sets = [&](auto bm_tag) {
            constexpr bool BM = decltype(bm_tag)::value;
            for (uint32_t set = g; set < T; set += G) {
                if constexpr (A == kClassCyc) {
                    CycVisitor v{cf, p.L, p.passes, bits};
                    if (sc.n <= kCachedSweeps) {
                        for (uint32_t i = 0; i < sc.n; ++i)
                            sweep_walk(pick_sweep(i != 0, sc.w1, sc.w0), 0, sc.sb, m, p, set, sc.qlo, v);
                    } else {
                        auto f = [&](const Sweep& w) { sweep_walk(w, 0, sc.sb, m, p, set, sc.qlo, v); };
                        pass_sweeps(p, m, f);
                    }
                    const bool thrash = v.n > m.ways;
                    ms += v.ms1 + (thrash ? v.ms2 : 0u);
                    mp += v.mp1 + (thrash ? v.mp2 : 0u);
                } else if constexpr (A == kClassMap) {
                    MapSet<POL> st;
                    st.init(col, args.map_rows, m.ways);
                    Visitor<MapSet<POL>, SCORE, BM> v{&st, &m, job.trace_id, cf, bits, jbm};
                    cached_runs(sc, p, m, set, v);
                    mt += v.mt; ms += v.ms; mp += v.mp;
                } else if constexpr (A == kClassScan) {
                    ScanSet<POL> st;
                    st.init(col, m.ways);
                    Visitor<ScanSet<POL>, SCORE, BM> v{&st, &m, job.trace_id, cf, bits, jbm};
                    cached_runs(sc, p, m, set, v);
                    mt += v.mt; ms += v.ms; mp += v.mp;
                } else {
                    RegSet<POL, A> st;
                    st.init();
                    Visitor<RegSet<POL, A>, SCORE, BM> v{&st, &m, job.trace_id, cf, bits, jbm};
                    cached_runs(sc, p, m, set, v);
                    mt += v.mt; ms += v.ms; mp += v.mp;
                }
            }
        };
        if (use_bm) sets(std::true_type{});
        else sets(std::false_type{});
    }
    if (use_bm) {
        // every lane's runs are in the LDS bitmap: store it, word by word,
        // coalesced
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const uint32_t jlo = task.item0 / G, jhi = (task.item0 + task.n - 1) / G;
        for (uint32_t jr = jlo; jr <= jhi; ++jr) {
            const SweepJob job = args.jobs[task.job + jr];
            const DevProbe p = args.probes[job.probe];
            const uint32_t words = (p.L * p.passes + 31) / 32;
            for (uint32_t w = (uint32_t)lane; w < words; w += kWave)
                args.bits[job.bitoff + w] = bm[job.bm_off + w];
        }
    }
    // every lane takes part in the shuffle (a shuffle from an inactive lane
    // is undefined, so it must not sit behind the lane == 0 test)
    const uint32_t key_up = __shfl_up(key, 1, kWave);
    const bool head = (lane == 0) || (key_up != key);
    if (SCORE) {
        // z + 2 mp - ms, summed modulo 2^64: a lane's part may be negative,
        // a candidate's total is not
        const uint64_t part = z + 2 * (uint64_t)mp - (uint64_t)ms;
        const uint64_t sm = seg_sum(part, key, lane);
        if (head && key != kInvalidTag && sm) atomicAdd((unsigned long long*)&args.counters[key], sm);
    } else {
        const uint64_t st = seg_sum(mt, key, lane);
        const uint64_t ss = seg_sum(ms, key, lane);
        if (head && key != kInvalidTag) {
            if (st) atomicAdd((unsigned long long*)&args.counters[2 * (uint64_t)key], st);
            if (ss) atomicAdd((unsigned long long*)&args.counters[2 * (uint64_t)key + 1], ss);
        }
    }
    if (use_bm) {
        // the next task reuses the bitmap: every lane must be done reading it
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

template <int POL, int A, bool SCORE>
// At least 4 waves per SIMD: the replay is bound by latency (LDS round
// trips, dependent compares, branches), not by issue, so occupancy wins even
// at the cost of a few spilled registers (measured: 3, 4, 5, 6, 8 waves per
// SIMD give 17.3, 15.8, 17.2, 20.3, 28.3 ms on the full inference sweep).
__global__ void __launch_bounds__(256, 4) sweep_kernel(SweepArgs args) {
    extern __shared__ uint32_t lds[];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    // per wave: the hit bitmap, then (LDS classes) one column per lane
    uint32_t* base = lds + (size_t)wave * (args.bm_words + (size_t)args.lds_rows * kWave);
    uint32_t* bm = base;
    uint32_t* col = base + args.bm_words + lane;
    if (!args.persistent) {
        const uint32_t t = blockIdx.x * (blockDim.x / kWave) + wave;
        if (t < args.n_tasks) run_task<POL, A, SCORE>(args, args.tasks[t], lane, col, bm);
        return;
    }
    for (uint32_t iter = 0;; ++iter) {
        uint32_t t = 0;
        if (lane == 0) {
            t = atomicAdd(args.queue, 1u);
            // abort: the host flag (a read across PCIe) on every 64th pull;
            // a flag already set when the call starts is seen by the host
            if ((iter & 63) == 63 && args.abort_flag != nullptr && *args.abort_flag != 0) {
                atomicOr(args.aborted, 1u);
                t = args.n_tasks;
            }
        }
        t = __shfl(t, 0, kWave);
        if (t >= args.n_tasks) break;
        run_task<POL, A, SCORE>(args, args.tasks[t], lane, col, bm);
    }
}

// ---------------------------------------------------------- launchers ---
using SweepFn = void (*)(SweepArgs);

template <bool SCORE>
static SweepFn pick(int pol, int cls) {
    if (cls == kACyc) {
        // one kernel for LRU and FIFO; replays that write bits never use it
        if constexpr (SCORE) return sweep_kernel<PCHASE_LRU, kClassCyc, true>;
        else return nullptr;
    }
#define PC_CASE(P)                                           \
    switch (cls) {                                           \
        case kA1: return sweep_kernel<P, 1, SCORE>;          \
        case kA2: return sweep_kernel<P, 2, SCORE>;          \
        case kA4: return sweep_kernel<P, 4, SCORE>;          \
        case kA8: return sweep_kernel<P, 8, SCORE>;          \
        case kA16: return sweep_kernel<P, 16, SCORE>;        \
        case kAMap: return sweep_kernel<P, kClassMap, SCORE>; \
        default: return sweep_kernel<P, kClassScan, SCORE>;  \
    }
    switch (pol) {
        case PCHASE_LRU: PC_CASE(PCHASE_LRU)
        case PCHASE_FIFO: PC_CASE(PCHASE_FIFO)
        case PCHASE_PLRU: PC_CASE(PCHASE_PLRU)
        default: PC_CASE(PCHASE_RANDOM)
    }
#undef PC_CASE
}

// Launch geometry of one (policy, class) sweep kernel: register classes run
// 4 waves per block without LDS; LDS classes run one wave per block with
// lds_rows dwords per lane.
void sweep_geometry(int cls, uint32_t lds_rows, uint32_t bm_words, uint32_t* threads, size_t* lds) {
    if (cls == kAMap || cls == kALds) {
        *threads = kWave;
        *lds = ((size_t)lds_rows * kWave + bm_words) * 4;
    } else {
        *threads = 256;
        *lds = (size_t)4 * bm_words * 4;
    }
}

hipError_t launch_sweep(bool score, int pol, int cls, const SweepArgs& args, uint32_t blocks,
                        hipStream_t stream) {
    uint32_t threads;
    size_t lds;
    sweep_geometry(cls, args.lds_rows, args.bm_words, &threads, &lds);
    SweepFn fn = score ? pick<true>(pol, cls) : pick<false>(pol, cls);
    if (fn == nullptr) return hipErrorInvalidDeviceFunction;
    hipLaunchKernelGGL(fn, dim3(blocks), dim3(threads), lds, stream, args);
    return hipGetLastError();
}

// Resident blocks per CU of a sweep kernel (for persistent grids).
hipError_t sweep_occupancy(bool score, int pol, int cls, uint32_t lds_rows, uint32_t bm_words, int* blocks_per_cu) {
    uint32_t threads;
    size_t lds;
    sweep_geometry(cls, lds_rows, bm_words, &threads, &lds);
    SweepFn fn = score ? pick<true>(pol, cls) : pick<false>(pol, cls);
    if (fn == nullptr) return hipErrorInvalidDeviceFunction;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, (const void*)fn, threads, lds);
}

hipError_t sweep_prepare_lds() {
    // LDS classes may ask for more than the default dynamic LDS limit
    for (int pol = 0; pol < 4; ++pol)
        for (int s = 0; s < 2; ++s)
            for (int cls : {(int)kAMap, (int)kALds}) {
                SweepFn fn = s ? pick<true>(pol, cls) : pick<false>(pol, cls);
                hipError_t e = hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                   (int)((kMaxLdsRows * kWave + kBmMaxWords) * 4));
                if (e != hipSuccess) return e;
            }
    return hipSuccess;
}

}  // namespace pc
