/*
 * pchase.h -- C ABI of the MI355X (gfx950) fine-grained P-chase cache-model
 * replay library, libpchase.so.
 *
 * The library replays pointer-chase access sequences through parameterised
 * set-associative cache models and searches candidate models for the one
 * that reproduces an observed hit/miss trace.  The method is the
 * fine-grained P-chase of Mei & Chu, "Dissecting GPU Memory Hierarchy
 * through Microbenchmarking" (IEEE TPDS 2017, arXiv:1509.02308):
 *   - the chase itself: Listing 1 (A[i] = (i + s) mod N) and Listing 2
 *     (j = A[j]), notation of Table 4 (C, b, a, T; N, s, k, r);
 *   - the cache model: Section 4.1, Assumptions 1-3 (T*a*b = C, set bits
 *     directly above the offset bits, LRU), with the non-LRU policies and
 *     non-bit-defined set mappings the paper finds in Sections 4.3-4.6;
 *   - per-access latency and index records: Section 4.2, Listing 3;
 *   - parameter search: Section 4.2, Fig. 6 two-stage procedure (here an
 *     exact exhaustive search over a candidate grid);
 *   - throughput / bank-conflict microbenchmarks: Section 5.1 (copy
 *     throughput = 2 * size / time), Section 6.2 (Listing 4 stride access).
 *
 * Conventions for every entry point:
 *   - return 0 (PCHASE_OK) or a negative PCHASE_E* code; the message of the
 *     last failure on the calling thread is pchase_last_error();
 *   - arguments are checked on the host before anything is launched; a
 *     failed check launches nothing and writes no output;
 *   - "_dev" pointers are device memory owned by the caller (the library
 *     never frees them); every other pointer is host memory, read during
 *     the call only;
 *   - work is enqueued on `stream` (0 = the null stream).  Functions that
 *     return values to host memory synchronise `stream` before returning;
 *     the others return as soon as the work is enqueued;
 *   - the library keeps per-device workspace (descriptor staging, replay
 *     state, work queues, cached inference schedules) that it allocates on
 *     first use and grows on demand; pchase_release() frees it (or a
 *     caller-owned pchase_plan takes its place, below).
 */
#ifndef PCHASE_H
#define PCHASE_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ errors --- */
#define PCHASE_OK        0
#define PCHASE_EINVAL   -1  /* malformed model, probe or argument          */
#define PCHASE_ERANGE   -2  /* a size exceeds a buffer or a kernel limit   */
#define PCHASE_ENOMEM   -3  /* device or host allocation failed            */
#define PCHASE_EHIP     -4  /* a HIP runtime call failed (message has it)  */
#define PCHASE_EABORTED -5  /* pchase_abort() stopped the work             */
#define PCHASE_ENODEV   -6  /* no usable gfx950 device                     */

/* Message of the last failure on this thread ("" if none).  The string is
 * owned by the library and valid until the next call on this thread. */
const char *pchase_last_error(void);

/* ------------------------------------------------------------- types --- */
/* Replacement policies.  LRU is Assumption 3 of Section 4.1; the paper
 * shows most GPU caches break it (Section 4.5: Fermi L1 is not LRU;
 * Section 4.6: L2 is not LRU).  FIFO and tree-PLRU are the usual hardware
 * alternatives; RANDOM evicts way Philox4x32-10(key = seed,
 * counter = (k_lo, k_hi, trace_lo, trace_hi)).x mod a, k = access index,
 * trace = trace id, so the draw depends on nothing but those values. */
enum {
    PCHASE_LRU = 0,
    PCHASE_FIFO = 1,
    PCHASE_PLRU = 2,
    PCHASE_RANDOM = 3,
    PCHASE_WRANDOM = 4   /* weighted random: generalised models only */
};

/* A cache model (Table 4 notation).  Valid iff sets*ways*line_bytes ==
 * capacity_bytes (Assumption 1), line_bytes is a power of two >= 4,
 * 1 <= ways <= 128, policy is one of the above, PLRU has a power-of-two
 * ways, and set_shift is 0 or >= log2(line_bytes).  The set of byte address
 * x is (x / line_bytes) mod sets when set_shift == 0 (Assumption 2), else
 * (x >> set_shift) mod sets (the texture-L1 style mapping of Section 4.3,
 * where bits above the line offset other than the next ones pick the set).
 * A cache starts empty; a miss fills the lowest-numbered empty way of its
 * set; only a full set asks the policy for a victim. */
typedef struct pchase_model {
    uint64_t capacity_bytes; /* C */
    uint32_t line_bytes;     /* b */
    uint32_t ways;           /* a */
    uint32_t sets;           /* T */
    uint32_t policy;         /* PCHASE_LRU .. PCHASE_RANDOM */
    uint32_t set_shift;      /* 0, or log2 of the set-mapping unit in bytes */
    uint32_t reserved;       /* must be 0 */
    uint64_t seed;           /* RANDOM key (ignored by other policies) */
} pchase_model;

/* A P-chase probe (Listing 1 + Listing 2).  Element i of the array sits at
 * byte base_offset + elem_bytes*i and holds (i + s/elem_bytes) mod
 * (n_bytes/elem_bytes).  The chase starts at element j0 and runs `passes`
 * full cycles; one cycle has L = Ne / gcd(Ne, Se mod Ne) accesses
 * (Ne = n_bytes/elem_bytes, Se = s_bytes/elem_bytes).  Valid iff elem_bytes
 * is 4, n_bytes and s_bytes are multiples of it, 1 <= Ne < 2^31,
 * j0 < Ne, passes >= 1 and base_offset/elem_bytes < 2^31.  s_bytes >= n_bytes
 * is legal (Fig. 4 sweeps s past N). */
typedef struct pchase_probe {
    uint64_t n_bytes;     /* N */
    uint64_t s_bytes;     /* s */
    uint64_t base_offset; /* byte address of element 0 */
    uint64_t j0;          /* first element visited */
    uint32_t elem_bytes;  /* 4 (int32 array) */
    uint32_t passes;      /* full cycles replayed */
} pchase_probe;

/* ------------------------------------------------------------ traces --- */
/* Length of one probe's trace: *len = passes * L, *cycle = L (either
 * pointer may be NULL).  Host only. */
int pchase_trace_len(const pchase_probe *probe, uint64_t *len, uint64_t *cycle);

/* Writes the visited element indices of n_probes probes back to back into
 * idx_dev (int32, capacity `cap` elements): probe p occupies
 * [off[p], off[p+1]).  off (host, n_probes+1 entries, may be NULL) receives
 * the offsets.  ERANGE if the total exceeds cap. */
int pchase_trace(const pchase_probe *probes, uint32_t n_probes, int32_t *idx_dev,
                 uint64_t *off, uint64_t cap, hipStream_t stream);

/* Non-uniform-stride chase (Section 5.2, Fig. 13(b)): the array is set up
 * so that the chase leaves each element by the stride of the segment it
 * belongs to, which lets one run mix access patterns (far strides that
 * miss every cache and TLB level, revisits of resident lines, steps inside
 * a line).  Segment i of a pass has `count` >= 1 accesses and each of them
 * is followed by a step of s_bytes (a multiple of elem_bytes; any size,
 * taken modulo n_bytes).  A pass visits segments first_segment ..
 * first_segment + n_segments - 1 of the segment array in order, starting
 * at element j0; each of the `passes` passes starts again at j0.  Element
 * i sits at byte base_offset + elem_bytes*i, as for pchase_probe.  Probes
 * may share segments.  Valid iff elem_bytes is 4, n_bytes is a multiple of
 * it with 1 <= Ne < 2^31, j0 < Ne, passes >= 1, n_segments >= 1, the
 * segment range lies inside the array, base_offset is a multiple of 4
 * below 2^33 and passes * (accesses per pass) < 2^32. */
typedef struct pchase_segment {
    uint64_t s_bytes;     /* step after each access of the segment */
    uint64_t count;       /* accesses in the segment, >= 1 */
} pchase_segment;

typedef struct pchase_nu_probe {
    uint64_t n_bytes;       /* N */
    uint64_t base_offset;   /* byte address of element 0 */
    uint64_t j0;            /* first element visited in every pass */
    uint32_t elem_bytes;    /* 4 */
    uint32_t passes;
    uint32_t first_segment; /* index into the segment array */
    uint32_t n_segments;
} pchase_nu_probe;

/* *len = passes * (accesses per pass), *pass_len = accesses per pass
 * (either may be NULL).  segs has n_segs entries.  Host only. */
int pchase_trace_nu_len(const pchase_nu_probe *probe, const pchase_segment *segs, uint32_t n_segs,
                        uint64_t *len, uint64_t *pass_len);

/* Writes the visited element indices of n_probes non-uniform probes back
 * to back into idx_dev (int32, device, capacity `cap` elements), laid out
 * and reported through `off` (host, n_probes+1 entries, may be NULL) as
 * for pchase_trace.  probes and segs are host arrays.  EINVAL for an
 * invalid probe, ERANGE if the total exceeds cap.  Synchronises. */
int pchase_trace_nu(const pchase_nu_probe *probes, uint32_t n_probes, const pchase_segment *segs,
                    uint32_t n_segs, int32_t *idx_dev, uint64_t *off, uint64_t cap, hipStream_t stream);

/* Generalised cache model: the organisations the paper finds that break
 * Assumptions 1-3.
 *   - set_ways: each set has its own associativity (the L2 TLB of
 *     Section 4.4 / Fig. 9: one set of 17 entries and six of 8);
 *   - set_table: the set of an address is set_table[unit mod table_len]
 *     (unit = address >> set_shift, or address / line_bytes when set_shift
 *     is 0), for mappings that are not a bit field (the read-only and
 *     texture caches of Section 4.3); table_len = 0 keeps unit mod n_sets;
 *   - PCHASE_WRANDOM: a miss in a full set of a ways draws
 *     u = Philox4x32-10(key = seed, counter = (k_lo, k_hi, trace_lo,
 *     trace_hi)).x and evicts the lowest way w with
 *     (u mod S) < way_weights[0] + ... + way_weights[w], S being the sum of
 *     the set's first a weights (the Fermi L1 of Section 4.5: weights
 *     1, 3, 1, 1 replace way 2 half of the time).
 * Valid iff line_bytes is a power of two >= 4, 1 <= n_sets, every set has
 * 1..128 ways (a power of two for PLRU), every table entry is below n_sets,
 * set_shift is 0 or >= log2(line_bytes), and for WRANDOM each set's weight
 * sum is in [1, 65536].  All arrays are host memory, read during the call. */
typedef struct pchase_general_model {
    uint32_t line_bytes;
    uint32_t n_sets;
    uint32_t policy;                /* PCHASE_LRU .. PCHASE_WRANDOM */
    uint32_t set_shift;
    const uint32_t *set_ways;       /* n_sets entries */
    const uint32_t *set_table;      /* table_len entries, or NULL */
    uint32_t table_len;
    uint32_t weights_len;           /* entries of way_weights (>= the widest set for WRANDOM) */
    const uint32_t *way_weights;    /* WRANDOM only, else NULL */
    uint64_t seed;                  /* RANDOM / WRANDOM key */
} pchase_general_model;

/* ------------------------------------------------------ probe planner --- */
/* Adaptive probing (Sec. 4.2, Fig. 6): the paper chooses each next (N, s)
 * from what the earlier runs showed.  Here the choice is made over a pool:
 * on each pool probe the candidates fall into classes of identical
 * steady-pass hit bits (accesses L .. len-1), a class named by its lowest
 * candidate index; among the surviving candidates (bitmap alive_host, bit c
 * of word c/32) the chosen probe has the smallest largest class, then the
 * most classes, then the lowest pool index.  probe = -1 when no pool probe
 * splits the survivors (they are indistinguishable on the pool) or none is
 * alive.  The caller observes the target on the chosen probe (e.g.
 * microbench_pchase + classification, or a replay) and keeps the survivors
 * whose prediction matches, e.g. through infer_cache_params's zero class.
 * classes_dev (nullable, device, n_pool x n_cands uint32, row = probe)
 * receives the class matrix.  The first call for a (cands, pool) pair
 * replays every candidate on every probe (at most 2^13 candidates, 2^20
 * probes and 8 GB of hit bits); later calls with the same pair only score.
 * Synchronises. */
typedef struct pchase_plan_choice {
    int64_t probe;        /* pool index, or -1 */
    uint32_t worst;       /* largest class among the survivors on that probe */
    uint32_t n_classes;   /* classes among the survivors on that probe */
    uint32_t n_alive;     /* survivors */
    uint32_t reserved;
} pchase_plan_choice;

int pchase_plan_next_probe(const pchase_model *cands, uint32_t n_cands, const pchase_probe *pool,
                           uint32_t n_pool, const uint32_t *alive_host, uint32_t *classes_dev,
                           pchase_plan_choice *out, hipStream_t stream);

/* ------------------------------------------------------------- plans --- */
/* A caller-owned plan: the device workspace of the replay and inference
 * calls that are given it (descriptor staging, observation bits, replay
 * schedules, slab state of generalised caches, cached inference schedules)
 * reserved once, as one allocation of device_bytes, when the plan is
 * created, together with the plan's own streams, events and pinned result
 * page.  A call given a plan allocates no device memory: it carves what it
 * needs from the plan's memory (returning PCHASE_ERANGE, before launching
 * anything that could write outputs, when that does not suffice).
 * The plan keeps the schedule of the last inference problem it served, so
 * repeating infer_cache_params on the same inputs rebuilds nothing; any
 * other call replaces what the plan held.  An inference schedule holds the
 * replay descriptors and, for the closed-form scoring (see
 * PCHASE_SCHED_FULL_REPLAY), 52 bytes per job scored without a replay and
 * 4 bytes per run of every run table (at most 2^26 entries): about 160 MB
 * for 438 candidates on their own N sweeps (1.08 million jobs, 24.7
 * million table entries).  A plan belongs to the device
 * that was current at creation (EINVAL on another device), and serves one
 * call at a time (calls are serialised on it).  A NULL plan selects the
 * library's own per-device workspace, which grows on demand. */
typedef struct pchase_plan pchase_plan;
int pchase_plan_create(uint64_t device_bytes, pchase_plan **plan);
/* Waits for the plan's device, then frees everything the plan holds.
 * NULL is a no-op. */
void pchase_plan_destroy(pchase_plan *plan);

/* ------------------------------------------------------------ replay --- */
/* Replay scheduling: BATCHED runs every pair in persistent kernels fed by
 * cost-ordered work queues, spread over parallel streams; PLAIN launches
 * ordinary kernels, one block per work item.  Results are identical. */
enum { PCHASE_BATCHED = 0, PCHASE_PLAIN = 1 };

/* Replays (model, trace) pairs over materialised index traces.
 *   models[n_models]                      host
 *   idx_dev                               element indices, int32, device
 *   trace_off[n_traces+1]                 host, trace t = idx[off[t], off[t+1])
 *   trace_base[n_traces]                  host, byte address of element 0
 *                                         (NULL = 0)
 *   elem_bytes                            bytes per element (4)
 *   pair_model[n_pairs], pair_trace[n_pairs]   host
 *   count_from[n_pairs]                   host, first access counted in
 *                                         misses_steady (NULL = 0)
 *   misses_dev[2*n_pairs]                 uint64 out: (total, steady) per pair
 *   hitbits_dev                           uint32 out or NULL: bit k%32 of word
 *                                         bitoff[i] + k/32 is pair i's access k
 *                                         (1 = hit); words the pairs touch are
 *                                         fully written
 *   bitoff[n_pairs]                       host, word offsets (needed iff hitbits)
 * The RANDOM policy's trace id is pair_trace[i].  Access k of a pair whose
 * trace holds a negative index is rejected (EINVAL, detected on device, the
 * outputs of that call are then unspecified). */
int cache_replay_batch(const pchase_model *models, uint32_t n_models,
                       const int32_t *idx_dev, const uint64_t *trace_off,
                       const uint64_t *trace_base, uint32_t elem_bytes, uint32_t n_traces,
                       const uint32_t *pair_model, const uint32_t *pair_trace,
                       const uint64_t *count_from, uint64_t n_pairs,
                       uint64_t *misses_dev, uint32_t *hitbits_dev, const uint64_t *bitoff,
                       uint32_t mode, pchase_plan *plan, hipStream_t stream);

/* For callers that cannot allocate device memory (code under stream
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * cache_replay_batch in the BATCHED schedule, for the same arguments and
 * with the same results, that allocates nothing.  Its device scratch (the
 * models, the per-(pair, part) work items, the status word and work-queue
 * counters) is a fixed array of 64 MiB in the library, one per GPU, set up
 * on the first call on that GPU and held until the process ends; a call
 * whose descriptors need more (about 56 bytes per pair or part of a split
 * pair) returns PCHASE_ERANGE before launching anything.  Every call on one
 * GPU uses that same array: calls that overlap on one GPU (other host
 * threads, or other streams before this call's synchronisation) race.
 * Everything launches on `stream`, one kernel after the other; the call
 * synchronises `stream` before it returns.  pchase_abort() does not stop
 * it.  Standard models only. */
int cache_replay_batch_static(const pchase_model *models, uint32_t n_models,
                              const int32_t *idx_dev, const uint64_t *trace_off,
                              const uint64_t *trace_base, uint32_t elem_bytes, uint32_t n_traces,
                              const uint32_t *pair_model, const uint32_t *pair_trace,
                              const uint64_t *count_from, uint64_t n_pairs,
                              uint64_t *misses_dev, uint32_t *hitbits_dev, const uint64_t *bitoff,
                              hipStream_t stream);

/* cache_replay_batch for generalised models (the declarations above):
 * same traces, pairs, outputs, ownership and errors.  A pair's state slab
 * holds n_sets 32-byte headers and 8 bytes per way; a long pair whose state
 * is at most 256 KB replays as up to 64 parts by set, each with its own copy
 * of that layout. */
int cache_replay_general(const pchase_general_model *models, uint32_t n_models, const int32_t *idx_dev,
                         const uint64_t *trace_off, const uint64_t *trace_base, uint32_t elem_bytes,
                         uint32_t n_traces, const uint32_t *pair_model, const uint32_t *pair_trace,
                         const uint64_t *count_from, uint64_t n_pairs, uint64_t *misses_dev,
                         uint32_t *hitbits_dev, const uint64_t *bitoff, uint32_t mode, pchase_plan *plan,
                         hipStream_t stream);

/* Same replay with traces given as probes instead of index arrays: pair i
 * replays probe pair_probe[i] through model pair_model[i]; the trace id of
 * the RANDOM policy is pair_probe[i]; count_from NULL means one cycle L of
 * the probe (one warm pass, the paper's "preheat").  Nothing is
 * materialised: each set's accesses are enumerated from (N, s) directly. */
int cache_replay_probes(const pchase_model *models, uint32_t n_models,
                        const pchase_probe *probes, uint32_t n_probes,
                        const uint32_t *pair_model, const uint32_t *pair_probe,
                        const uint64_t *count_from, uint64_t n_pairs,
                        uint64_t *misses_dev, uint32_t *hitbits_dev, const uint64_t *bitoff,
                        uint32_t mode, pchase_plan *plan, hipStream_t stream);

/* --------------------------------------------------------- inference --- */
enum { PCHASE_PROBES_ALL = 0, PCHASE_PROBES_OWN_SWEEP = 1 };
enum { PCHASE_EXHAUSTIVE = 0, PCHASE_LEARNED = 1 };
/* OR into infer_cache_params' mode to replay with the PLAIN schedule (one
 * launch per candidate) instead of the persistent batch. */
#define PCHASE_SCHED_PLAIN 0x100
/* The first call of a problem answers with the batched schedule's default
 * assignment of kernels to streams; the second call on the same inputs
 * times every assignment and keeps the fastest for the calls after it.  OR
 * this flag into infer_cache_params' mode to keep the default assignment
 * (for profiling runs, where the timing loop would be serialised by the
 * profiler). */
#define PCHASE_SCHED_UNTUNED 0x200
/* By default the scores of (candidate, probe) jobs whose outcome has a
 * closed form are computed without a replay through way state (results are
 * identical; pchase_result.closed_form_accesses counts their accesses):
 *  - no set of the candidate can hold more than a lines of the probe's array
 *    (Section 4.2 step 1: nothing is ever evicted, so only first touches
 *    miss);
 *  - LRU and FIFO (and one-way caches, and two-way tree-PLRU, which is LRU)
 *    on a chase whose every pass visits each line at most once (Section
 *    4.1: every pass visits a set's n lines in the same cyclic order, so
 *    after the first pass every run start misses when n > a and none does
 *    when n <= a);
 * single-sweep passes whose visited lines form an arithmetic progression
 * (one line per set-mapping unit) are scored from per-probe prefix sums of
 * the observation, the others by a walk over the first pass's runs.  OR
 * this flag into infer_cache_params' mode to replay every access through
 * the per-set state instead (to measure or check the replay engine). */
#define PCHASE_SCHED_FULL_REPLAY 0x400

/* Observed fine-grained P-chase runs (Listing 3 outputs): probe p's trace
 * is known from the probe; its hit bits are either given (bits_dev, layout
 * of cache_replay_batch with bitoff) or derived from latencies (lat_dev,
 * uint32 cycles back to back at lat_off[p]) as hit iff latency <= threshold;
 * threshold == UINT32_MAX asks for the lower end of the widest gap between
 * distinct latency values (the two populations of t = t0 + tm*r).  Accesses
 * before count_from[p] (NULL: one cycle L) are not compared. */
typedef struct pchase_observation {
    const pchase_probe *probes;
    uint32_t n_probes;
    uint32_t threshold;
    const uint32_t *bits_dev;   /* or NULL */
    const uint64_t *bitoff;     /* host, with bits_dev */
    const uint32_t *lat_dev;    /* or NULL */
    const uint64_t *lat_off;    /* host, with lat_dev */
    const uint64_t *count_from; /* host or NULL */
} pchase_observation;

/* Learned proposer (3-layer MLP, bf16 weights, fp32 accumulate) over the
 * fixed 768-probe feature grid; see pchase_mlp_* below. */
typedef struct pchase_mlp pchase_mlp;

typedef struct pchase_result {
    int64_t best;               /* candidate index, -1 if none compared */
    uint64_t best_m, best_n;    /* mismatches / compared accesses of best */
    uint64_t n_zero;            /* candidates with m == 0 (zero class) */
    uint64_t replayed_accesses; /* accesses whose hit or miss the call determined */
    uint64_t closed_form_accesses; /* of those, accesses of jobs scored in closed
                                      form, without a replay through way state */
    uint32_t fallback;          /* LEARNED: 1 no exact top-k match, 2 not the grid */
    uint32_t threshold_used;    /* latency threshold applied (UINT32_MAX: none) */
} pchase_result;

/* Scores every candidate against the observation and returns the exact
 * rational argmin of m/n (m = mismatched hit/miss decisions, n = compared
 * accesses), ties to the lowest candidate index, candidates with n == 0
 * skipped.  probe_select = ALL compares every probe with every candidate;
 * OWN_SWEEP compares candidate (C, b, ...) on the probes with
 * C/2 <= N <= 2C, N % b == 0 and s in {b/2, b, 2b} (the Section 4.2
 * overflow sweeps around a candidate capacity).
 * mode = LEARNED (observation = the 768 grid probes, see pchase_mlp_*)
 * computes the observation's features, ranks the candidates with `net`
 * (n_out == n_cands, class c = candidate c), replays only the top-k and
 * accepts the best of them when its m == 0; otherwise it runs the
 * exhaustive search (out->fallback = 1), and when the observation is not
 * the grid it runs the exhaustive search directly (out->fallback = 2).
 * mn_dev (uint64[2*n_cands], nullable) receives (m, n) per candidate;
 * zero_host (uint32[(n_cands+31)/32], nullable) the zero-class bitmap
 * (exhaustive results only; it passes through a 3840-byte pinned page, so
 * with zero_host at most 30,720 candidates, ERANGE above).  With a plan the
 * learned network's activations for one row must already exist (any
 * earlier forward or training call made them).  Synchronises `stream`. */
int infer_cache_params(const pchase_observation *obs, const pchase_model *cands,
                       uint32_t n_cands, int probe_select, int mode, uint32_t topk,
                       const pchase_mlp *net, pchase_result *out, uint64_t *mn_dev,
                       uint32_t *zero_host, pchase_plan *plan, hipStream_t stream);

/* Exhaustive inference over generalised candidates (Sections 4.3-4.5: per-
 * set associativity, set tables, shifted set mappings, weighted random
 * replacement; pchase_general_model above).  The observation is given as
 * for infer_cache_params (hit bits, or latencies with a threshold or the
 * widest-gap rule); every candidate replays every observed probe
 * (PCHASE_PROBES_ALL), the trace id of probe p being p.  m, n, best (exact
 * rational argmin of m/n, lowest index on ties), the zero class, mn_dev
 * (device, uint64 [2 * n_cands], (m, n) per candidate) and zero_host (at
 * most 30,720 candidates) are as for infer_cache_params; best_m/best_n
 * refer to best.  The probes' traces (4 bytes per access) and every
 * candidate's hit bits (one bit per access and probe) are held in device
 * memory during the call: ERANGE beyond 2^34 accesses or 32 GiB of hit
 * bits, or (with a plan) when they do not fit the plan's memory.  A
 * candidate's replay state is as for cache_replay_general.  Synchronises
 * `stream`. */
int infer_cache_params_general(const pchase_observation *obs, const pchase_general_model *cands,
                               uint32_t n_cands, pchase_result *out, uint64_t *mn_dev,
                               uint32_t *zero_host, pchase_plan *plan, hipStream_t stream);

/* ---------------------------------------------------- microbenchmarks --- */
/* Load flavours of the single-lane chase: the gfx950 cache-policy bits of
 * the load instruction.  What each does on MI355X was measured with this
 * chase (latency over sizes and strides): the default and the work-group
 * scope loads may hit the per-CU vector L1 (about 100 cycles); system
 * scope and non-temporal loads miss it and hit L2 (about 190 cycles);
 * beyond L2, default, work-group and system scope loads see about 490
 * cycles, non-temporal loads about 700 (they do not allocate in the
 * memory-side cache). */
enum {
    PCHASE_LOAD_DEFAULT = 0, /* no policy bits                                  */
    PCHASE_LOAD_L2 = 1,      /* sc0: work-group scope                           */
    PCHASE_LOAD_SYSTEM = 2,  /* sc0 sc1: system scope, misses the vector L1     */
    PCHASE_LOAD_STREAM = 3   /* nt: non-temporal, misses the vector L1          */
};

/* Fine-grained P-chase on the device (Listing 3 redesigned for one gfx950
 * lane): initialises the probe's array in array_dev (array_bytes >=
 * base_offset + n_bytes, 4-byte aligned), walks it once untimed (the
 * paper's preheat), then times k dependent loads one by one with the
 * shader clock, keeping the records in LDS until the walk ends.
 * lat_dev[i] = raw cycles of access i, idx_dev[i] = element index accessed
 * at step i (the paper's s_index holds the loaded value, one step later).
 * *overhead_cycles receives the median cost of the same timed sequence
 * with the load replaced by a register move (subtract it for net latency).
 * idx_dev may be NULL: then no indices are recorded and each latency is
 * kept as a 16-bit value saturated at 65535 cycles, so that up to
 * 4 * pchase_microbench_max_k() accesses fit (long single-pass walks over
 * caches of a few MB at line strides).
 * ERANGE if k exceeds the LDS record capacity (pchase_microbench_max_k, or
 * four times it without indices).  Synchronises `stream`. */
int microbench_pchase(const pchase_probe *probe, uint32_t flavor, void *array_dev,
                      uint64_t array_bytes, uint64_t k, uint32_t *lat_dev, int32_t *idx_dev,
                      int32_t *overhead_cycles, hipStream_t stream);
uint64_t pchase_microbench_max_k(void);

/* Copy throughput (Section 5.1): grid x block threads copy `bytes` from
 * src_dev to dst_dev, each thread moving `ilp` independent words per step
 * (dtype 0 = 4-byte words, 1 = 16-byte words), `reps` times; *gbps =
 * 2 * bytes * reps / elapsed (read + write), timed with HIP events.
 * Synchronises `stream`. */
int microbench_hbm_stream(const void *src_dev, void *dst_dev, uint64_t bytes, uint32_t dtype,
                          uint32_t grid, uint32_t block, uint32_t ilp, uint32_t reps,
                          double *gbps, hipStream_t stream);

/* LDS bank conflicts (Section 6.2, Listing 4): one wave, lane t chases
 * words t*stride, 64 dependent LDS loads per timed repetition; for every
 * stride in [stride_lo, stride_hi] writes the average cycles per load
 * (x100, rounded) to cycles_dev[stride - stride_lo].  stride_hi <= 64. */
int microbench_lds_bank(uint32_t stride_lo, uint32_t stride_hi, uint32_t reps,
                        uint32_t *cycles_dev, hipStream_t stream);

/* LDS throughput (Section 6.1): blocks_per_cu x (number of CUs) blocks of
 * `block` threads (a multiple of 64, at most 1024) each stream accesses of
 * width_bytes (4 or 16) over a 16 KB LDS buffer, ilp (1, 2, 4 or 8)
 * independent reads in flight per thread, reps rounds, consecutive lanes on
 * consecutive words (no bank conflicts).  copy = 1 stores every value read
 * into a second 16 KB buffer (the paper's shared-to-shared copy: read and
 * written bytes both count); copy = 0 only reads.  *gbps = LDS bytes moved
 * / elapsed time of one launch after a warm-up launch (HIP events).
 * Returns PCHASE_EINVAL for arguments outside those sets.  Synchronises. */
int microbench_lds_stream(uint32_t blocks_per_cu, uint32_t block, uint32_t ilp, uint32_t width_bytes,
                          uint32_t copy, uint32_t reps, double *gbps, hipStream_t stream);

/* VALU issue rate: not an experiment of the paper but the denominator of
 * the replay's roofline (the replay is integer VALU work).  blocks_per_cu x
 * (number of CUs) blocks of 256 threads each run reps rounds of 8
 * independent chains of three full-rate 32-bit VALU instructions (add,
 * shift, xor); *lane_ops_per_s = 32-bit lane operations / elapsed time of
 * one launch after a warm-up launch.  EINVAL for blocks_per_cu outside
 * 1..32 or reps = 0.  Synchronises. */
int microbench_valu(uint32_t blocks_per_cu, uint32_t reps, double *lane_ops_per_s, hipStream_t stream);

/* ------------------------------------------------------ learned model --- */
/* The learned proposer ranks candidates from a fixed set of fine-grained
 * runs (the Section 4.2 procedure of Fig. 6 frozen into one grid: array
 * sizes swept across the candidate capacities, strides around the line
 * sizes) with a 3-layer perceptron, so that only its top-k candidates are
 * replayed exactly.
 *
 * Feature grid: probe p = 256 * t + i has N = 4096 + 512 i bytes (i < 256),
 * s = {32, 64, 128}[t] bytes, 2 passes, j0 = 0, 4-byte elements.  Feature p
 * of a trace is its steady-pass miss ratio r (Section 4.1): misses over
 * accesses [L, 2L) divided by L, rounded once to float.
 * Network: h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), z = W3 h2 + b3 with
 * W1 [256][768], W2 [256][256], W3 [n_out][256] row-major; products run on
 * the bf16 matrix cores with fp32 accumulation: weights are bf16 copies
 * (nearest-even) of fp32 masters, the input features are rounded to bf16,
 * and the fp32 hidden activations and back-propagated errors enter each
 * product as a pair hi + lo of bf16 values (hi = bf16(v), lo = bf16(v - hi),
 * about 2^-17 relative); loss = mean softmax cross-entropy; Adam (beta1 0.9,
 * beta2 0.999, eps 1e-8, bias-corrected). */
#define PCHASE_MLP_IN 768
#define PCHASE_MLP_HIDDEN 256

/* Writes the 768 grid probes (host array) with the given base offset. */
int pchase_mlp_grid(pchase_probe *probes, uint64_t base_offset);

/* Creates a network for n_out (1..4096) classes on the current device:
 * weights uniform in [-1/sqrt(fan_in), 1/sqrt(fan_in)) from
 * Philox4x32-10(key = seed, counter = (element, tensor, 0, 0x494E4954)),
 * biases and Adam moments zero.  Device memory is owned by the network
 * and freed by pchase_mlp_destroy.  A network is used by one thread at a
 * time. */
int pchase_mlp_create(uint32_t n_out, uint64_t seed, pchase_mlp **net);
void pchase_mlp_destroy(pchase_mlp *net);

/* Clean features (fp32 [n][768], device) of n models at base offset 0,
 * by replaying the grid.  Synchronises `stream`. */
int pchase_mlp_features(const pchase_model *models, uint32_t n, float *x_dev, hipStream_t stream);

/* Canonical labels (host int32 [n]): labels[i] = the lowest j whose
 * steady-pass hit/miss bits on the whole grid (base 0) equal those of
 * model i -- the representative of i's zero class when every grid probe
 * is compared.  ERANGE above about 8,000 models.  Synchronises. */
int pchase_mlp_labels(const pchase_model *models, uint32_t n, int32_t *labels, hipStream_t stream);

/* Training samples first .. first+n-1 (x_dev fp32 [n][768], labels_dev
 * int32 [n]).  Sample i draws (x, y, z, w) = Philox4x32-10(key = seed,
 * counter = (i_lo, i_hi, 0, 0)): model = x mod n_models, base offset
 * = 4 (y mod (b / 4)), flip threshold t = z mod (rho_q16 + 1).  The grid is
 * replayed through that model at that base offset and steady bit k of probe
 * p is flipped when 16-bit word (k mod 8) -- bits 16 (w mod 2).. of output
 * word w div 2 -- of Philox4x32-10(key = seed, counter = (k div 8, p, i_lo,
 * 2^31 | i_hi)) is below t; the label is class_of_model[model] (host).
 * Lines must be at most 128 bytes.  Synchronises. */
int pchase_mlp_samples(const pchase_model *models, uint32_t n_models, const int32_t *class_of_model,
                       uint64_t first, uint32_t n, uint64_t seed, uint32_t rho_q16, float *x_dev,
                       int32_t *labels_dev, hipStream_t stream);

/* One Adam step at learning rate lr on a batch (1..65536 rows of x_dev
 * fp32 [batch][768] with labels_dev int32 [batch]).  *loss (nullable)
 * receives the batch's mean cross-entropy before the step (synchronises). */
int pchase_mlp_train_step(pchase_mlp *net, const float *x_dev, const int32_t *labels_dev,
                          uint32_t batch, float lr, float *loss, hipStream_t stream);
/* `epochs` passes of consecutive batches over n_samples rows (a trailing
 * partial batch is skipped); *last_loss (nullable) = loss of the last
 * batch.  The step is captured into a graph on the first call for given
 * (x_dev, labels_dev, batch, lr) and replayed once per batch; the result
 * equals that of pchase_mlp_train_step on each batch in turn.
 * Synchronises. */
int pchase_mlp_train(pchase_mlp *net, const float *x_dev, const int32_t *labels_dev, uint64_t n_samples,
                     uint32_t batch, uint32_t epochs, float lr, float *last_loss, hipStream_t stream);
/* Logits fp32 [batch][n_out] of x_dev (device). */
int pchase_mlp_forward(const pchase_mlp *net, const float *x_dev, uint32_t batch,
                       float *logits_dev, hipStream_t stream);
/* Indices of the k largest logits of each row, largest first, ties to the
 * lower index (idx_dev int32 [rows][k]; k <= 64, n_classes <= 4096). */
int pchase_mlp_topk(const float *logits_dev, uint32_t rows, uint32_t n_classes, uint32_t k,
                    int32_t *idx_dev, hipStream_t stream);
/* Parameter access for checkpoints and tests (host buffers, fp32):
 * which = 0..5 selects W1, b1, W2, b2, W3, b3; slot = 0 master parameter,
 * 1 Adam first moment, 2 second moment, 3 gradient of the last step
 * (read-only).  *bytes receives the size; data may be NULL to query it.
 * Writing a weight master refreshes its bf16 copy.  Synchronises. */
int pchase_mlp_param(const pchase_mlp *net, uint32_t which, uint32_t slot, void *data,
                     uint64_t *bytes, int write);
/* Adam step counter (for bias correction): read, or set when set != 0. */
int pchase_mlp_step_count(const pchase_mlp *net, uint64_t *steps, int set);

/* --------------------------------------------------------- lifecycle --- */
/* Sets a host flag that stops the BATCHED schedule's replays: a probe
 * replay or inference that starts while it is set returns PCHASE_EABORTED
 * before launching anything; running persistent replays poll it (every 8th
 * queue pull, the first included, for materialised traces; every 64th for
 * probe replays), drain, and the call that launched them returns
 * PCHASE_EABORTED, outputs unspecified.  pchase_abort(0) clears it; later
 * calls are unaffected. */
void pchase_abort(int on);
/* Frees the calling thread's current device workspace. */
int pchase_release(void);

#ifdef __cplusplus
}
#endif
#endif
