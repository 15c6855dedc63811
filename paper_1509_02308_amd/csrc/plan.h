// plan.h -- schedules of the probe-replay kernels: jobs (model x probe)
// split into wave tasks, grouped by (policy, way class), ordered longest
// first for the persistent batched launch, with the branch strategy the
// autotuner chose for them.
#pragma once

#include <functional>

#include "host_common.h"

namespace pc {

struct Bucket {
    int pol;
    int cls;
    uint32_t first;     // into the task array
    uint32_t count;
    uint32_t lds_rows;  // LDS classes: dwords per lane column
    uint32_t map_rows;  // map class: dwords of the map
    double cost;        // estimated lane work of the bucket
    uint32_t bm_words;  // per-wave LDS hit bitmap dwords
};

struct SweepPlan {
    uint32_t n_models = 0, n_probes = 0;
    uint64_t n_jobs = 0, n_tasks = 0;
    uint64_t accesses = 0;           // replayed accesses of one run
    std::vector<Bucket> batched;     // task ranges of the cost-ordered array
    std::vector<Bucket> plain;       // one range per model in the natural array
    std::vector<uint64_t> clear;     // (word, count) ranges of the output bitmap
    DevBuf dev;
    DevModel* d_models = nullptr;
    DevProbe* d_probes = nullptr;
    SweepJob* d_jobs = nullptr;
    SweepTask* d_lpt = nullptr;
    SweepTask* d_plain = nullptr;
    uint32_t* d_queues = nullptr;    // one per batched bucket, + status word
    uint64_t* d_clear = nullptr;
    const uint64_t* zeros = nullptr; // scoring: observed misses per probe (SweepArgs::zeros)
    int strategy = 0;                // branch strategy of the batched runs
    bool tuned = false;              // strategy chosen by timing
    SweepPlan() = default;
    SweepPlan(const SweepPlan&) = delete;
    SweepPlan& operator=(const SweepPlan&) = delete;
    ~SweepPlan();
};

// jobs must be grouped by model (each model's jobs contiguous).  With
// lds_bitmaps, tasks whose jobs' hit bits fit a wave's LDS bitmap gather
// them there and store them coalesced (replays that write hit bits);
// scoring plans need no bitmap.
int build_sweep_plan(SweepPlan* plan, const std::vector<DevModel>& models,
                     const std::vector<DevProbe>& probes, const std::vector<uint64_t>& probe_len,
                     const std::vector<SweepJob>& jobs, bool want_clear, bool lds_bitmaps = true);

// Runs the plan on `stream` (launches only; the caller synchronises):
// zeroes `counters` (n_counters words) and the bitmap ranges (when
// clear_bits), then replays every job; `tail` (may be empty) is enqueued
// after the replay.  With autotune (plans that are cached and run again),
// the first batched run that is not deferred times every branch strategy
// and keeps the fastest for the plan's later runs; defer_tuning leaves the
// tuning to a later run (a problem's first answer does not wait for it).
// `side` (may be empty) is work that needs the cleared counters but not the
// replay: it runs on a branch stream beside the replay (PLAIN: before it).
int run_sweep_plan(Workspace* ws, SweepPlan* plan, bool score, uint64_t* counters, uint64_t n_counters,
                   uint32_t* bits, bool clear_bits, uint32_t mode, hipStream_t stream,
                   const std::function<hipError_t(hipStream_t)>& tail, bool autotune = false,
                   bool defer_tuning = false, const std::function<hipError_t(hipStream_t)>& side = {});

// Cached schedule + score buffers of one inference problem.
struct InferPlan {
    std::string key;                // the exact inputs the plan was built for
    bool cached = false;            // kept for later calls (worth autotuning)
    SweepPlan sweep;
    std::vector<uint64_t> n_host;   // compared accesses per candidate
    uint32_t runs = 0;              // completed runs (the first one is not tuned)
    DevBuf dev;                     // m | n | zero bits | argmin out | probe info | observed misses |
                                    // decided jobs | run tables
    uint64_t* d_pinfo = nullptr;    // per probe: bitmap word offset, count_from, length
    uint64_t* d_zeros = nullptr;    // per probe: observed misses from count_from on
    uint32_t n_probes = 0;
    // jobs decided without a replay (grouped by candidate), scored from the
    // observed misses and the run tables
    DecidedJob* d_decided = nullptr;   // in table order
    int64_t* d_dec_vals = nullptr;     // per job score, candidate order
    uint32_t* d_dec_cand = nullptr;    // candidate of each slot
    RunTable* d_tables = nullptr;
    int64_t* d_s1 = nullptr;
    int32_t* d_prefix = nullptr;
    uint64_t* d_table_ks = nullptr;
    PlruPattern* d_patterns = nullptr;
    uint32_t* d_pat_bits = nullptr;
    uint32_t n_tables = 0;
    uint32_t n_decided = 0;
    uint64_t decided_accesses = 0;  // their accesses
    uint64_t cyc_accesses = 0;      // accesses of the plan's closed-form (kACyc) jobs
    uint64_t* d_m = nullptr;
    uint64_t* d_n = nullptr;
    uint32_t* d_zero = nullptr;
    ArgminOut* d_out = nullptr;
    uint32_t n_cands = 0;
    InferPlan() = default;
    InferPlan(const InferPlan&) = delete;
    InferPlan& operator=(const InferPlan&) = delete;
    ~InferPlan() { dev.release(); }
};

// Learned proposer: marks in *allow the top-k candidates of the network for
// the observation (defined with the MLP kernels); *on_grid is false (and
// nothing is marked) when the observation is not the feature grid.
int infer_learned(Workspace* ws, const pchase_observation* obs, const pchase_model* cands, uint32_t n_cands,
                  const std::vector<DevProbe>& dp, const std::vector<uint64_t>& len,
                  const std::vector<uint64_t>& cf, const std::vector<uint64_t>& bitoff, const uint32_t* bits,
                  uint32_t topk, const pchase_mlp* net, std::vector<uint8_t>* allow, bool* on_grid,
                  hipStream_t stream);

// Replays jobs (grouped by model) into a cleared hit bitmap of bits_words
// words (job bit offsets are word offsets) and waits.
int replay_jobs(Workspace* ws, const std::vector<DevModel>& dm, const std::vector<DevProbe>& dp,
                const std::vector<uint64_t>& len, const std::vector<SweepJob>& jobs, uint32_t* bits,
                uint64_t bits_words, hipStream_t stream);

// 128-bit FNV-style digest of byte ranges (plan cache keys).
struct Digest {
    uint64_t a = 1469598103934665603ull, b = 0x9E3779B97F4A7C15ull;
    void add(const void* p, size_t n);
    std::string str() const;
};

}  // namespace pc
