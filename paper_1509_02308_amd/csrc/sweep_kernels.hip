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
// candidate model.
#include "common.h"

namespace pc {

// ------------------------------------------------------------ PLRU tree --
// a-1 node bits in heap order (children of n: 2n+1 left, 2n+2 right; leaf of
// way w is a-1+w); a 0 bit sends the victim search left.
struct PlruBits {
    uint64_t lo = 0, hi = 0;
    __device__ __forceinline__ uint32_t get(uint32_t n) const {
        return n < 64 ? (uint32_t)(lo >> n) & 1u : (uint32_t)(hi >> (n - 64)) & 1u;
    }
    __device__ __forceinline__ void put(uint32_t n, uint32_t v) {
        if (n < 64) lo = (lo & ~(1ull << n)) | ((uint64_t)v << n);
        else hi = (hi & ~(1ull << (n - 64))) | ((uint64_t)v << (n - 64));
    }
    // a use of way x makes every node on its path point to the other child
    __device__ __forceinline__ void touch(uint32_t x, uint32_t depth) {
        uint32_t node = 0;
        for (uint32_t d = 0; d < depth; ++d) {
            uint32_t dir = (x >> (depth - 1 - d)) & 1u;
            put(node, dir ^ 1u);
            node = 2 * node + 1 + dir;
        }
    }
    __device__ __forceinline__ uint32_t victim(uint32_t depth, uint32_t a) const {
        uint32_t node = 0;
        for (uint32_t d = 0; d < depth; ++d) node = 2 * node + 1 + get(node);
        return node - (a - 1);
    }
};

// ----------------------------------------------- set state in registers --
template <int POL, int A>
struct RegSet {
    uint32_t tag[A];
    uint32_t age[A];  // LRU recency rank (0 = most recent); 0xFF = empty way
    uint32_t nvalid;  // ways fill in index order, so ways < nvalid are valid
    uint32_t ptr;     // FIFO: next way to replace
    PlruBits bits;

    __device__ __forceinline__ void init() {
#pragma unroll
        for (int w = 0; w < A; ++w) {
            tag[w] = kInvalidTag;
            age[w] = 0xFFu;
        }
        nvalid = 0;
        ptr = 0;
        bits = PlruBits();
    }

    __device__ __forceinline__ bool access(uint32_t line, const DevModel& m, uint64_t k,
                                           uint32_t trace_id) {
        const uint32_t a = m.ways;
        int hw = -1;
        uint32_t vic = 0;
#pragma unroll
        for (int w = 0; w < A; ++w) {
            if (w < (int)a) {
                if (tag[w] == line) hw = w;
                if constexpr (POL == PCHASE_LRU) if (age[w] == a - 1) vic = (uint32_t)w;
            }
        }
        const bool hit = hw >= 0;
        if constexpr (POL == PCHASE_LRU) {
            uint32_t x, ax = 0;
#pragma unroll
            for (int w = 0; w < A; ++w)
                if (w == hw) ax = age[w];
            if (hit) {
                x = (uint32_t)hw;
            } else if (nvalid < a) {
                x = nvalid;
                ax = nvalid;
                ++nvalid;
            } else {
                x = vic;
                ax = a - 1;
            }
#pragma unroll
            for (int w = 0; w < A; ++w) {
                if (w < (int)a) {
                    uint32_t g = age[w];
                    g += (g < ax) ? 1u : 0u;
                    if ((uint32_t)w == x) {
                        g = 0;
                        tag[w] = line;
                    }
                    age[w] = g;
                }
            }
        } else if constexpr (POL == PCHASE_FIFO) {
            if (!hit) {
                uint32_t x = ptr;
                ptr = (ptr + 1 == a) ? 0 : ptr + 1;
#pragma unroll
                for (int w = 0; w < A; ++w)
                    if ((uint32_t)w == x) tag[w] = line;
            }
        } else if constexpr (POL == PCHASE_PLRU) {
            uint32_t x;
            if (hit) x = (uint32_t)hw;
            else if (nvalid < a) x = nvalid++;
            else x = bits.victim(m.log2_ways, a);
            bits.touch(x, m.log2_ways);
            if (!hit) {
#pragma unroll
                for (int w = 0; w < A; ++w)
                    if ((uint32_t)w == x) tag[w] = line;
            }
        } else {  // RANDOM
            if (!hit) {
                uint32_t x;
                if (nvalid < a) x = nvalid++;
                else x = philox_x((uint32_t)k, (uint32_t)(k >> 32), trace_id, 0u, m.seed_lo,
                                  m.seed_hi) % a;
#pragma unroll
                for (int w = 0; w < A; ++w)
                    if ((uint32_t)w == x) tag[w] = line;
            }
        }
        return hit;
    }
};

// ------------------------------------------ set state in an LDS column --
// Way w of this lane's set sits at tag[w*64 + lane] (and age[w*64 + lane]):
// the lanes of a wave read one row together without bank conflicts.
template <int POL>
struct LdsSet {
    uint32_t* tag;
    uint8_t* age;
    uint32_t nvalid;
    uint32_t ptr;
    PlruBits bits;

    __device__ __forceinline__ void init(uint32_t* tag_col, uint8_t* age_col, uint32_t a) {
        tag = tag_col;
        age = age_col;
        nvalid = 0;
        ptr = 0;
        bits = PlruBits();
        for (uint32_t w = 0; w < a; ++w) {
            tag[w * kWave] = kInvalidTag;
            if (POL == PCHASE_LRU) age[w * kWave] = 0xFFu;
        }
    }

    __device__ __forceinline__ bool access(uint32_t line, const DevModel& m, uint64_t k,
                                           uint32_t trace_id) {
        const uint32_t a = m.ways;
        uint32_t hw = kInvalidTag;
        for (uint32_t w = 0; w < a; ++w)
            if (tag[w * kWave] == line) hw = w;
        const bool hit = hw != kInvalidTag;
        uint32_t x;
        if constexpr (POL == PCHASE_LRU) {
            uint32_t ax;
            if (hit) {
                x = hw;
                ax = age[hw * kWave];
            } else if (nvalid < a) {
                x = nvalid;
                ax = nvalid;
                ++nvalid;
            } else {
                ax = a - 1;
                x = 0;
                for (uint32_t w = 0; w < a; ++w)
                    if (age[w * kWave] == a - 1) x = w;
            }
            for (uint32_t w = 0; w < a; ++w) {
                uint32_t g = age[w * kWave];
                if (g < ax) age[w * kWave] = (uint8_t)(g + 1);
            }
            age[x * kWave] = 0;
            if (!hit) tag[x * kWave] = line;
        } else if constexpr (POL == PCHASE_FIFO) {
            if (!hit) {
                x = ptr;
                ptr = (ptr + 1 == a) ? 0 : ptr + 1;
                tag[x * kWave] = line;
            }
        } else if constexpr (POL == PCHASE_PLRU) {
            if (hit) x = hw;
            else if (nvalid < a) x = nvalid++;
            else x = bits.victim(m.log2_ways, a);
            bits.touch(x, m.log2_ways);
            if (!hit) tag[x * kWave] = line;
        } else {
            if (!hit) {
                if (nvalid < a) x = nvalid++;
                else x = philox_x((uint32_t)k, (uint32_t)(k >> 32), trace_id, 0u, m.seed_lo,
                                  m.seed_hi) % a;
                tag[x * kWave] = line;
            }
        }
        return hit;
    }
};

// ------------------------------------------------- access enumeration ----
// Calls visit(line, k0, r) for every run of r consecutive accesses
// k0 .. k0+r-1 of the probe that fall in one line of set `set`, in trace
// order.
template <class Visit>
__device__ __forceinline__ void sweep_runs(uint64_t xf, uint64_t sb, uint64_t cnt, uint64_t kstart,
                                           const DevModel& m, uint32_t set, Visit& visit) {
    const uint32_t T = m.sets;
    const uint32_t us = m.unit_shift, ls = m.line_shift;
    const uint64_t U = 1ull << us;
    if (sb < U * T) {
        // walk the units of this set inside the sweep's address range
        const uint64_t xl = xf + (cnt - 1) * sb;
        const uint64_t uf = xf >> us, ul = xl >> us;
        const uint64_t rem = umod64(uf, T);
        uint64_t u = uf + (set >= rem ? set - rem : set + T - rem);
        for (; u <= ul; u += T) {
            const uint64_t lo = u << us;
            const uint64_t ilo = lo <= xf ? 0 : udiv64(lo - xf + sb - 1, sb);
            uint64_t ihi = udiv64(lo + U - 1 - xf, sb);
            if (ihi > cnt - 1) ihi = cnt - 1;
            if (ilo > ihi) continue;
            if (us == ls) {
                visit(u, kstart + ilo, ihi - ilo + 1);
            } else {
                uint64_t i = ilo;
                while (i <= ihi) {
                    const uint64_t line = (xf + i * sb) >> ls;
                    const uint64_t lend = (line + 1) << ls;
                    uint64_t inext = udiv64(lend - xf + sb - 1, sb);
                    if (inext > ihi + 1) inext = ihi + 1;
                    visit(line, kstart + i, inext - i);
                    i = inext;
                }
            }
        }
    } else {
        // stride of at least T units: walk the accesses, tracking the set
        // incrementally (the unit advances by q or q+1 per access)
        uint64_t x = xf, u = xf >> us;
        uint32_t st = (uint32_t)umod64(u, T);
        const uint64_t q = sb >> us;
        const uint32_t qm = (uint32_t)umod64(q, T), qm1 = (uint32_t)umod64(q + 1, T);
        for (uint64_t i = 0; i < cnt; ++i) {
            if (st == set) visit(x >> ls, kstart + i, 1);
            const uint64_t xn = x + sb, un = xn >> us;
            st += (un - u == q) ? qm : qm1;
            if (st >= T) st -= T;
            x = xn;
            u = un;
        }
    }
}

template <class Visit>
__device__ __forceinline__ void probe_runs(const DevProbe& p, const DevModel& m, uint32_t set,
                                           Visit& visit) {
    const uint32_t es = p.elem_shift;
    const uint64_t sb = (uint64_t)p.se << es;
    for (uint32_t pass = 0; pass < p.passes; ++pass) {
        const uint64_t kpass = (uint64_t)pass * p.L;
        if (p.se == 0) {  // s is a multiple of N: the chase stays on j0
            const uint64_t x = p.base + ((uint64_t)p.j0 << es);
            if (umod64(x >> m.unit_shift, m.sets) == set) visit(x >> m.line_shift, kpass, 1);
            continue;
        }
        uint64_t r = p.j0, kpos = 0;
        while (kpos < p.L) {
            // one increasing sweep: r, r+se, ... < ne
            uint64_t cnt = (p.ne - r + p.se - 1) / p.se;
            if (cnt > p.L - kpos) cnt = p.L - kpos;
            sweep_runs(p.base + (r << es), sb, cnt, kpass + kpos, m, set, visit);
            kpos += cnt;
            r = r + cnt * p.se - p.ne;
        }
    }
}

// ------------------------------------------------------- bitmap helpers --
__device__ __forceinline__ void or_bits(uint32_t* w, uint64_t lo, uint64_t hi) {
    // sets bits [lo, hi)
    while (lo < hi) {
        const uint64_t word = lo >> 5;
        const uint32_t b0 = (uint32_t)(lo & 31);
        const uint64_t n = (hi - lo < 32 - b0) ? hi - lo : 32 - b0;
        const uint32_t mask = (n == 32) ? 0xFFFFFFFFu : (((1u << n) - 1u) << b0);
        atomicOr(w + word, mask);
        lo += n;
    }
}

__device__ __forceinline__ uint64_t ones_in(const uint32_t* w, uint64_t lo, uint64_t hi) {
    uint64_t c = 0;
    while (lo < hi) {
        const uint64_t word = lo >> 5;
        const uint32_t b0 = (uint32_t)(lo & 31);
        const uint64_t n = (hi - lo < 32 - b0) ? hi - lo : 32 - b0;
        const uint32_t mask = (n == 32) ? 0xFFFFFFFFu : (((1u << n) - 1u) << b0);
        c += __popc(w[word] & mask);
        lo += n;
    }
    return c;
}

// ---------------------------------------------------------------- kernel --


template <int POL, class S, bool SCORE>
struct Visitor {
    S* st;
    const DevModel* m;
    uint32_t trace_id;
    uint64_t cf;
    uint32_t* bits;
    uint64_t mt = 0, ms = 0, mm = 0;
    __device__ __forceinline__ void operator()(uint64_t line, uint64_t k0, uint64_t r) {
        const bool hit = st->access((uint32_t)line, *m, k0, trace_id);
        if (!hit) {
            ++mt;
            ms += (k0 >= cf) ? 1u : 0u;
        }
        if constexpr (SCORE) {
            if (k0 >= cf) {
                const uint32_t ob = (bits[k0 >> 5] >> (k0 & 31)) & 1u;
                mm += (ob != (hit ? 1u : 0u)) ? 1u : 0u;
            }
            const uint64_t lo = (k0 + 1 > cf) ? k0 + 1 : cf, hi = k0 + r;
            if (lo < hi) mm += (hi - lo) - ones_in(bits, lo, hi);
        } else if (bits != nullptr) {
            or_bits(bits, hit ? k0 : k0 + 1, k0 + r);
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

template <int POL, int A, bool SCORE>
__device__ __forceinline__ void run_task(const SweepArgs& args, const SweepTask& task, int lane,
                                         uint32_t* lds_tag, uint8_t* lds_age) {
    const DevModel m = args.models[task.model];
    const bool active = (uint32_t)lane < task.n;
    uint32_t key = kInvalidTag;
    uint64_t mt = 0, ms = 0, mm = 0;
    if (active) {
        // G = min(T, 64) lanes per replay; lane g of a replay owns the sets
        // g, g+G, g+2G, ... and replays them one after the other
        const uint32_t T = m.sets;
        const uint32_t G = T < (uint32_t)kWave ? T : (uint32_t)kWave;
        const uint32_t item = task.item0 + (uint32_t)lane;
        const uint32_t jrel = item / G;
        const uint32_t g = item - jrel * G;
        const SweepJob job = args.jobs[task.job + jrel];
        const DevProbe p = args.probes[job.probe];
        key = job.out;
        uint32_t* bits = args.bits == nullptr ? nullptr : args.bits + job.bitoff;
        for (uint32_t set = g; set < T; set += G) {
            if constexpr (A > 16) {
                LdsSet<POL> st;
                st.init(lds_tag, lds_age, m.ways);
                Visitor<POL, LdsSet<POL>, SCORE> v{&st, &m, job.trace_id, job.count_from, bits};
                probe_runs(p, m, set, v);
                mt += v.mt; ms += v.ms; mm += v.mm;
            } else {
                RegSet<POL, A> st;
                st.init();
                Visitor<POL, RegSet<POL, A>, SCORE> v{&st, &m, job.trace_id, job.count_from, bits};
                probe_runs(p, m, set, v);
                mt += v.mt; ms += v.ms; mm += v.mm;
            }
        }
    }
    // every lane takes part in the shuffle (a shuffle from an inactive lane
    // is undefined, so it must not sit behind the lane == 0 test)
    const uint32_t key_up = __shfl_up(key, 1, kWave);
    const bool head = (lane == 0) || (key_up != key);
    if (SCORE) {
        mm = seg_sum(mm, key, lane);
        if (head && key != kInvalidTag && mm) atomicAdd((unsigned long long*)&args.counters[key], mm);
    } else {
        mt = seg_sum(mt, key, lane);
        ms = seg_sum(ms, key, lane);
        if (head && key != kInvalidTag) {
            if (mt) atomicAdd((unsigned long long*)&args.counters[2 * (uint64_t)key], mt);
            if (ms) atomicAdd((unsigned long long*)&args.counters[2 * (uint64_t)key + 1], ms);
        }
    }
}

template <int POL, int A, bool SCORE>
__global__ void __launch_bounds__(256) sweep_kernel(SweepArgs args) {
    extern __shared__ uint32_t lds[];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    uint32_t* lds_tag = nullptr;
    uint8_t* lds_age = nullptr;
    if (A > 16) {
        // per wave: 128 x 64 tags, then 128 x 64 age bytes
        uint32_t* base = lds + (size_t)wave * (kMaxWays * kWave + kMaxWays * kWave / 4);
        lds_tag = base + lane;
        lds_age = reinterpret_cast<uint8_t*>(base + kMaxWays * kWave) + lane;
    }
    if (!args.persistent) {
        const uint32_t t = blockIdx.x * (blockDim.x / kWave) + wave;
        if (t < args.n_tasks) run_task<POL, A, SCORE>(args, args.tasks[t], lane, lds_tag, lds_age);
        return;
    }
    for (uint32_t iter = 0;; ++iter) {
        uint32_t t = 0;
        if (lane == 0) {
            t = atomicAdd(args.queue, 1u);
            if ((iter & 63) == 63 && args.abort_flag != nullptr && *args.abort_flag != 0) {
                atomicOr(args.aborted, 1u);
                t = args.n_tasks;
            }
        }
        t = __shfl(t, 0, kWave);
        if (t >= args.n_tasks) break;
        run_task<POL, A, SCORE>(args, args.tasks[t], lane, lds_tag, lds_age);
    }
}

// LDS bytes per wave of the large-associativity class
constexpr size_t kLdsPerWave = kMaxWays * kWave * 4 + kMaxWays * kWave;

// ---------------------------------------------------------- launchers ---
using SweepFn = void (*)(SweepArgs);

template <bool SCORE>
static SweepFn pick(int pol, int cls) {
#define PC_CASE(P)                                           \
    switch (cls) {                                           \
        case kA1: return sweep_kernel<P, 1, SCORE>;          \
        case kA2: return sweep_kernel<P, 2, SCORE>;          \
        case kA4: return sweep_kernel<P, 4, SCORE>;          \
        case kA8: return sweep_kernel<P, 8, SCORE>;          \
        case kA16: return sweep_kernel<P, 16, SCORE>;        \
        default: return sweep_kernel<P, 128, SCORE>;         \
    }
    switch (pol) {
        case PCHASE_LRU: PC_CASE(PCHASE_LRU)
        case PCHASE_FIFO: PC_CASE(PCHASE_FIFO)
        case PCHASE_PLRU: PC_CASE(PCHASE_PLRU)
        default: PC_CASE(PCHASE_RANDOM)
    }
#undef PC_CASE
}

// Launch geometry of one (policy, class) sweep kernel.
void sweep_geometry(int cls, uint32_t* threads, size_t* lds) {
    if (cls == kALds) {
        *threads = kWave;  // one wave per block: 40 KB of LDS each
        *lds = kLdsPerWave;
    } else {
        *threads = 256;
        *lds = 0;
    }
}

hipError_t launch_sweep(bool score, int pol, int cls, const SweepArgs& args, uint32_t blocks,
                        hipStream_t stream) {
    uint32_t threads;
    size_t lds;
    sweep_geometry(cls, &threads, &lds);
    SweepFn fn = score ? pick<true>(pol, cls) : pick<false>(pol, cls);
    hipLaunchKernelGGL(fn, dim3(blocks), dim3(threads), lds, stream, args);
    return hipGetLastError();
}

// Resident blocks per CU of a sweep kernel (for persistent grids).
hipError_t sweep_occupancy(bool score, int pol, int cls, int* blocks_per_cu) {
    uint32_t threads;
    size_t lds;
    sweep_geometry(cls, &threads, &lds);
    SweepFn fn = score ? pick<true>(pol, cls) : pick<false>(pol, cls);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, (const void*)fn, threads, lds);
}

hipError_t sweep_prepare_lds() {
    // the large-associativity class asks for more than the default dynamic
    // LDS limit on some runtimes; raise it once
    for (int pol = 0; pol < 4; ++pol)
        for (int s = 0; s < 2; ++s) {
            SweepFn fn = s ? pick<true>(pol, kALds) : pick<false>(pol, kALds);
            hipError_t e = hipFuncSetAttribute((const void*)fn,
                                               hipFuncAttributeMaxDynamicSharedMemorySize,
                                               (int)kLdsPerWave);
            if (e != hipSuccess) return e;
        }
    return hipSuccess;
}

}  // namespace pc
