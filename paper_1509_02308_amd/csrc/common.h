// common.h -- internal definitions shared by the HIP kernels and the host
// side of libpchase (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pchase.h"

namespace pc {

// ---------------------------------------------------------------- limits --
constexpr uint32_t kMaxWays = 128;
constexpr uint32_t kInvalidTag = 0xFFFFFFFFu;
constexpr int kWave = 64;

// Replay classes: ways held in registers (unrolled up to the class bound) or
// in an LDS column per lane for the large associativities.
// Large associativities use an LDS map (when the set's lines fit it) or an
// LDS scan.  kACyc (scoring only) holds no ways: LRU or FIFO jobs whose
// every pass is one increasing sweep, decided per set in closed form.
enum WayClass : int { kA1 = 0, kA2, kA4, kA8, kA16, kAMap, kALds, kACyc, kNumClasses };
constexpr uint32_t kMapMaxEntries = 448;   // map rows + ways <= 240 dwords per lane
__host__ __device__ inline int way_class(uint32_t a) {
    return a <= 1 ? kA1 : a <= 2 ? kA2 : a <= 4 ? kA4 : a <= 8 ? kA8 : a <= 16 ? kA16 : kALds;
}

// ------------------------------------------------------ device descriptors --
// A model as the kernels see it (derived on the host from pchase_model).
struct DevModel {
    uint32_t line_shift;  // log2(b)
    uint32_t unit_shift;  // log2 of the set-mapping unit (== line_shift by default)
    uint32_t sets;        // T
    uint32_t ways;        // a
    uint32_t policy;
    uint32_t log2_ways;   // PLRU tree depth
    uint32_t seed_lo, seed_hi;
};

// Exact floor(n / d) for 32-bit n through a multiply-high (Granlund &
// Montgomery, "Division by invariant integers using multiplication", 1994,
// Fig. 4.1): with l = ceil(log2 d) and m = floor(2^32 (2^l - d) / d) + 1,
// t = mulhi(m, n) and q = (t + ((n - t) >> min(l,1))) >> max(l-1, 0).
struct UDiv32 {
    uint32_t m, s1, s2;
    __host__ __device__ __forceinline__ uint32_t div(uint32_t n) const {
        const uint32_t t = (uint32_t)(((uint64_t)m * n) >> 32);
        return (t + ((n - t) >> s1)) >> s2;
    }
};

__host__ __device__ inline UDiv32 make_udiv32(uint32_t d) {
    uint32_t l = 0;
    while (l < 32 && (1ull << l) < d) ++l;
    UDiv32 u;
    u.m = (uint32_t)((((1ull << l) - d) << 32) / d + 1);
    u.s1 = l < 1 ? l : 1;
    u.s2 = l > 1 ? l - 1 : 0;
    return u;
}

// A probe as the kernels see it: element indices, one cycle = L accesses.
struct DevProbe {
    uint64_t base;        // byte address of element 0
    uint32_t ne;          // N / elem
    uint32_t se;          // (s / elem) mod ne
    uint32_t L;           // cycle length
    uint32_t j0;
    uint32_t passes;
    uint32_t elem_shift;  // log2(elem)
    UDiv32 sb_div;        // division by the stride in bytes, se << elem_shift
    uint32_t sb_fast;     // 1 if that stride fits 32 bits (sb_div valid)
};

// One replay job of the probe kernels: model x probe.
struct SweepJob {
    uint32_t model;
    uint32_t probe;
    uint32_t out;         // counter slot (pair index, or candidate index when scoring)
    uint32_t trace_id;    // RANDOM counter high word
    uint64_t count_from;
    uint64_t bitoff;      // word offset of the output / observed bitmap
    uint32_t bm_off;      // word offset of the job's bits in its task's LDS bitmap
    uint32_t cyc;         // scoring: 1 if the job is decided in closed form (kACyc)
};

// A wave's worth of (job, set) items: items item0 .. item0+n-1 of the run of
// jobs that starts at `job` (all with the same model; a task holds whole
// jobs only); item i is set group i % G of
// job job + i / T.
struct SweepTask {
    uint32_t job;
    uint32_t item0;
    uint32_t n;
    uint32_t model;
    uint32_t bm_words;    // LDS bitmap words of the task's jobs (0: bits go straight to memory)
    uint32_t lanes;       // G: lanes per job (lane g of a job owns sets g, g+G, ...)
};

// Materialised-trace pair.
struct StreamPair {
    uint64_t start;       // first index of the trace in idx
    uint64_t len;
    uint64_t base;        // byte address of element 0
    uint64_t count_from;
    uint64_t bitoff;
    uint32_t model;
    uint32_t trace_id;
    uint32_t out;
    uint32_t pad;
};


// ------------------------------------------------------- kernel arguments --
struct SweepArgs {
    const SweepTask* tasks;
    uint32_t n_tasks;
    uint32_t persistent;      // 1: waves pull tasks from *queue
    uint32_t* queue;
    const SweepJob* jobs;
    const DevModel* models;
    const DevProbe* probes;
    uint64_t* counters;       // replay: (total, steady) per out; score: m per out
    uint32_t* bits;           // replay: output bitmap or null; score: observed bitmap
    const uint64_t* zeros;    // score: per probe, 0 bits (observed misses) of its
                              // observed bitmap from count_from on; every job of
                              // a probe compares with that bitmap from that index
    const volatile uint32_t* abort_flag;
    uint32_t* aborted;
    uint32_t lds_rows;        // LDS classes: dwords per lane column
    uint32_t map_rows;        // map class: dwords of the map in a column
    uint32_t bm_words;        // dwords of the per-wave LDS hit bitmap
};

// Largest per-wave LDS hit bitmap (dwords); tasks needing more write their
// bits to memory directly.
constexpr uint32_t kBmMaxWords = 1024;

// Generalised model (per-set ways, set table, weighted random): offsets of
// its entries in the flat arrays of StreamArgs.
struct DevGeneral {
    uint32_t set_off;     // first (ways, entry base) pair of its sets in set_info
    uint32_t table_off;   // first entry of its set table
    uint32_t table_len;   // 0: set = unit mod sets
    uint32_t cum_off;     // first of its cumulative way weights
};

struct StreamArgs {
    const StreamPair* pairs;
    uint32_t n_pairs;
    uint32_t* queue;
    const DevModel* models;
    const int32_t* idx;
    uint64_t* misses;
    uint32_t* bits;
    uint8_t* slab;
    uint64_t slab_bytes;     // per group
    uint32_t epoch_base;
    uint32_t elem_shift;
    const volatile uint32_t* abort_flag;
    uint32_t* status;        // bit 0: aborted, bit 1: negative index seen
    // generalised models only
    const DevGeneral* gen;
    const uint2* set_info;   // per set: (ways, first entry of the set in the slab)
    const uint32_t* set_table;
    const uint32_t* cum_w;   // cumulative way weights
};

struct ArgminOut {
    int64_t best;
    uint64_t m, n;
    uint64_t n_zero;
};

// ------------------------------------------------------------ launchers --
hipError_t launch_sweep(bool score, int pol, int cls, const SweepArgs& args, uint32_t blocks,
                        hipStream_t stream);
hipError_t sweep_occupancy(bool score, int pol, int cls, uint32_t lds_rows, uint32_t bm_words, int* blocks_per_cu);
void sweep_geometry(int cls, uint32_t lds_rows, uint32_t bm_words, uint32_t* threads, size_t* lds);
hipError_t sweep_prepare_lds();
hipError_t launch_stream(int pol, int w, bool gen, const StreamArgs& args, uint32_t blocks, hipStream_t stream);
hipError_t stream_occupancy(int pol, int w, bool gen, int* blocks_per_cu);
// Trace generation: one block per chunk of kTraceChunkAccesses accesses;
// chunk table entry = (probe, chunk number within the probe).
constexpr uint64_t kTraceChunkAccesses = 4096;
struct ChunkRef {
    uint32_t probe;
    uint32_t chunk;
};
hipError_t launch_chunk_table(const uint64_t* chunk_off, uint32_t n_traces, ChunkRef* chunks, hipStream_t stream);
hipError_t launch_trace(const DevProbe* probes, const uint64_t* off, const ChunkRef* chunks, uint64_t n_chunks,
                        int32_t* idx, hipStream_t stream);
// Non-uniform-stride chase: a probe's pass is a list of segments; segment
// i of a probe starts at access `start` of the pass on element `pos` and
// steps by `se` (elements, reduced modulo ne) after each of its accesses.
struct DevNuSeg {
    uint64_t start;
    uint32_t pos;
    uint32_t se;
};
struct DevNuProbe {
    uint64_t pass_len;   // accesses per pass
    uint32_t first;      // its first segment in the DevNuSeg array
    uint32_t nseg;
    uint32_t ne;         // array size in elements
    uint32_t pad;
};
hipError_t launch_trace_nu(const DevNuProbe* probes, const DevNuSeg* segs, const uint64_t* off,
                           const ChunkRef* chunks, uint64_t n_chunks, int32_t* idx, hipStream_t stream);
hipError_t launch_fill_u32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t stream);
hipError_t launch_fill2_u32(uint32_t* p, uint64_t n, uint32_t* q, uint64_t nq, uint32_t v, hipStream_t stream);
hipError_t launch_argmin(const uint64_t* m, const uint64_t* n, uint32_t nc, uint32_t* zero_bits,
                         ArgminOut* out, hipStream_t stream);
hipError_t launch_auto_threshold(const uint32_t* lat, uint64_t n, uint32_t* mm, uint32_t* present,
                                 uint64_t max_bits, uint32_t* theta, hipStream_t stream);
hipError_t launch_classify(const uint32_t* lat, const uint64_t* lat_off, const uint64_t* bitoff,
                           uint32_t n_probes, uint64_t maxlen, const uint32_t* theta, uint32_t* bits,
                           hipStream_t stream);
hipError_t launch_clear_ranges(uint32_t* bits, const uint64_t* ranges, uint32_t n, hipStream_t stream);
// zeros[p] = number of 0 bits of bits + pinfo[3p] (a word offset) over bit
// indices [pinfo[3p+1], pinfo[3p+2]) (count_from, length), for p < n.
// Scoring without a replay.  A run table lists the runs (line visits) of one
// pass of a probe whose visited lines (line size 2^line_shift) form an
// arithmetic progression, each line visited once per pass, in the order of
// the lines: either one increasing sweep (nsw == 0; run i is the i-th line
// visited, first access per the stride) or nsw sweeps of stride nsw lines
// that together visit every line of a range once (run i is the range's
// i-th line, visited by the sweep starting at access ks[koff + i mod nsw],
// as its (i / nsw)-th access).  Per call, the prefix over runs of the later
// passes' signed weights w(k) = [k >= count_from] * (2 obs(k) - 1) at the
// run's start k goes to prefix[off .. off + runs] (32-bit: tables are built
// only when runs * (passes - 1) < 2^31) and the first pass's total to
// s1[table].
struct RunTable {
    uint32_t probe;
    uint32_t line_shift;
    uint64_t runs;
    uint64_t off;
    uint32_t nsw;
    uint32_t pad;
    uint64_t koff;
};
// A job decided without a replay, by kind:
//   0  no eviction, nothing of the first pass compared: the observed misses;
//   1  no eviction (first-pass run starts are the only misses): + s1;
//   2  LRU or FIFO, every visited set holds more lines than ways (every run
//      start misses): + s1 + all later-pass weights;
//   3  LRU or FIFO, the sets of runs i with i mod period < rem hold more
//      lines than ways and the others do not: + s1 + the later-pass weights
//      of those runs;
//   4  tree-PLRU, two passes, one sweep: the set of run i holds q0 + 1
//      lines if i mod period < rem, else q0, and run i is its set's
//      (i / period)-th line; + s1 + the second-pass weights of the runs
//      whose position misses in the second pass of a cyclic chase over
//      that many lines (pattern pat_big, pat_small).
struct DecidedJob {
    uint32_t probe;
    uint32_t table;
    uint32_t kind;
    uint32_t rem;
    uint64_t period;
    uint32_t cand;        // score slot
    uint32_t pat_big;     // kind 4: pattern of the sets with q0 + 1 lines
    uint32_t pat_small;   // kind 4: pattern of the sets with q0 lines
    uint32_t slot;        // position of the job in candidate order
};
// Second-pass miss pattern of a cyclic chase over n distinct lines through
// one a-way tree-PLRU set (ways filled in order, all node bits 0 at the
// start): bit i of bits[off ..] = the visit of the i-th line misses.
struct PlruPattern {
    uint32_t ways;
    uint32_t log2_ways;
    uint32_t lines;
    uint32_t scr;         // scratch offset (lines + ways words)
    uint64_t off;         // bit offset, a multiple of 32
};
hipError_t launch_plru_patterns(const PlruPattern* pd, uint32_t n, uint32_t* bits, uint32_t* scratch,
                                hipStream_t stream);
hipError_t launch_run_tables(const RunTable* tables, uint32_t n_tables, const DevProbe* probes,
                             const uint64_t* ks, const uint64_t* pinfo, const uint32_t* bits, int32_t* prefix,
                             int64_t* s1, hipStream_t stream);
// vals[dj[i].slot] = the score of decided job i, i < n (jobs in table order,
// so that lanes next to each other gather from the same run table); then
// m[cand[q]] += vals[q] (slots in candidate order, a candidate's contiguous).
hipError_t launch_decided(const DecidedJob* dj, uint32_t n, const uint64_t* zeros, const RunTable* tables,
                          const int32_t* prefix, const int64_t* s1, const PlruPattern* pats,
                          const uint32_t* pat_bits, int64_t* vals, const uint32_t* cand, uint64_t* m,
                          hipStream_t stream);
hipError_t launch_obs_zeros(const uint32_t* bits, const uint64_t* pinfo, uint32_t n, uint64_t* zeros,
                            hipStream_t stream);
// m[c] += accesses of pair (c, p) = (pair / n_probes, pair % n_probes), from
// cf[p] to len[p], whose hit bit in hits + c * cand_words + hoff[p] differs
// from the observation's in obs + obits[p] (word offsets).
hipError_t launch_mismatch(const uint32_t* hits, uint64_t cand_words, const uint32_t* obs, const uint64_t* hoff,
                           const uint64_t* obits, const uint64_t* cf, const uint64_t* len, uint32_t n_probes,
                           uint64_t n_pairs, uint64_t* m, hipStream_t stream);

// ------------------------------------------------------------ Philox ----
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32 multiplies; the high halves are xored into the other two words with
// the round key, which advances by the Weyl increments between rounds.
__device__ __forceinline__ uint32_t philox_x(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                             uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t m0 = 0xD2511F53u, m1 = 0xCD9E8D57u;
        uint32_t h0 = __umulhi(m0, c0), l0 = m0 * c0;
        uint32_t h1 = __umulhi(m1, c2), l1 = m1 * c2;
        uint32_t n0 = h1 ^ c1 ^ k0;
        uint32_t n2 = h0 ^ c3 ^ k1;
        c0 = n0;
        c1 = l1;
        c2 = n2;
        c3 = l0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c0;
}

// ------------------------------------------------------------- helpers ---
__device__ __forceinline__ uint64_t udiv64(uint64_t x, uint64_t d) {
    if ((x >> 32) == 0 && (d >> 32) == 0) return (uint32_t)x / (uint32_t)d;
    return x / d;
}
__device__ __forceinline__ uint64_t umod64(uint64_t x, uint64_t d) {
    if ((x >> 32) == 0 && (d >> 32) == 0) return (uint32_t)x % (uint32_t)d;
    return x % d;
}

}  // namespace pc

// ------------------------------------------------------ host-side errors --
namespace pc {
int set_error(int code, const char *fmt, ...);
int hip_fail(hipError_t e, const char *what);
}  // namespace pc

#define PC_HIP(call)                                          \
    do {                                                      \
        hipError_t e_ = (call);                               \
        if (e_ != hipSuccess) return pc::hip_fail(e_, #call); \
    } while (0)

static_assert(sizeof(pchase_model) == 40, "pchase_model layout");
static_assert(sizeof(pchase_probe) == 40, "pchase_probe layout");
static_assert(sizeof(pchase_segment) == 16, "pchase_segment layout");
static_assert(sizeof(pchase_nu_probe) == 40, "pchase_nu_probe layout");
static_assert(sizeof(pchase_general_model) == 56, "pchase_general_model layout");
static_assert(sizeof(pchase_plan_choice) == 24, "pchase_plan_choice layout");
static_assert(sizeof(pchase_result) == 56, "pchase_result layout");
