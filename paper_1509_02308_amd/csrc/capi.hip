// capi.hip -- C-ABI entry points: trace generation, replay of probes and of
// materialised traces, exhaustive and learned inference.
#include <sys/mman.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <map>
#include <new>

#include "plan.h"
#include "tile.h"

namespace pc {



// A workspace buffer could not grow: the plan's memory is used up (ERANGE),
// or a device allocation failed (ENOMEM).
static int buf_fail(const Workspace* ws, hipError_t e, const char* what) {
    if (ws->arena)
        return set_error(PCHASE_ERANGE, "%s does not fit the plan's %llu bytes of device memory", what,
                         (unsigned long long)ws->arena->cap);
    return set_error(PCHASE_ENOMEM, "%s: %s", what, hipGetErrorString(e));
}

static int validate_models(const pchase_model* models, uint32_t n, std::vector<DevModel>* out) {
    if (n && !models) return set_error(PCHASE_EINVAL, "models is NULL");
    out->resize(n);
    for (uint32_t i = 0; i < n; ++i) {
        int rc = check_model(models[i], &(*out)[i], i);
        if (rc) return rc;
    }
    return PCHASE_OK;
}

static int validate_probes(const pchase_probe* probes, uint32_t n, std::vector<DevProbe>* out,
                           std::vector<uint64_t>* len) {
    if (n && !probes) return set_error(PCHASE_EINVAL, "probes is NULL");
    out->resize(n);
    len->resize(n);
    for (uint32_t i = 0; i < n; ++i) {
        int rc = check_probe(probes[i], &(*out)[i], &(*len)[i], i);
        if (rc) return rc;
    }
    return PCHASE_OK;
}

// Every set of model m holds at most a lines of probe p's array: no access
// of the probe evicts (a bound: the set's units in the array's address range
// times the lines per unit).
static bool no_eviction(const DevModel& m, const DevProbe& p) {
    const uint64_t xlo = p.base, xhi = p.base + ((uint64_t)(p.ne - 1) << p.elem_shift);
    const uint64_t units = (xhi >> m.unit_shift) - (xlo >> m.unit_shift) + 1;
    const uint64_t per_set = ((units + m.sets - 1) / m.sets) << (m.unit_shift - m.line_shift);
    return per_set <= m.ways;
}

// Every pass of probe p is one increasing sweep of the array (the chase
// does not wrap around inside a pass): the first sweep from j0 holds all L
// accesses of the pass.
static bool one_sweep_per_pass(const DevProbe& p) {
    if (p.se == 0) return true;
    const uint64_t first = ((uint64_t)p.ne - p.j0 + p.se - 1) / p.se;
    return first >= p.L;
}

// Runs of one pass under line size 2^ls when the pass is one increasing
// sweep whose visited lines form an arithmetic progression (step d lines):
// every line of the swept range when the stride is at most a line, one line
// per access when the stride is a multiple of the line.  Returns 0 otherwise.
static uint64_t sweep_runs(const DevProbe& p, uint32_t ls, uint64_t* d) {
    if (!one_sweep_per_pass(p)) return 0;
    *d = 1;
    if (p.se == 0 || p.L == 1) return 1;
    const uint64_t sb = (uint64_t)p.se << p.elem_shift, b = 1ull << ls;
    const uint64_t x0 = p.base + ((uint64_t)p.j0 << p.elem_shift);
    if (sb <= b) return ((x0 + (uint64_t)(p.L - 1) * sb) >> ls) - (x0 >> ls) + 1;
    if (sb % b == 0) {
        *d = sb >> ls;
        return p.L;
    }
    return 0;
}

// Every line is visited by at most one run in a pass (so every pass visits
// each set's lines once, in the same order): one increasing sweep, or at most
// 64 sweeps whose stride is a multiple of the line (each sweep visits lines
// l, l + d, l + 2d, ..., d the stride in lines) and whose first lines differ
// modulo d.
static bool lines_once_per_pass(const DevProbe& p, uint32_t ls) {
    if (one_sweep_per_pass(p)) return true;
    const uint64_t sb = (uint64_t)p.se << p.elem_shift;
    if (sb & ((1ull << ls) - 1)) return false;
    const uint64_t d = sb >> ls;
    std::vector<uint64_t> first;
    uint64_t r = p.j0, kpos = 0;
    while (kpos < p.L) {
        if (first.size() == 64) return false;
        const uint64_t res = ((p.base + (r << p.elem_shift)) >> ls) % d;
        for (uint64_t f : first)
            if (f == res) return false;
        first.push_back(res);
        uint64_t cnt = ((uint64_t)p.ne - r + p.se - 1) / p.se;
        if (cnt > p.L - kpos) cnt = p.L - kpos;
        kpos += cnt;
        r = r + cnt * p.se - p.ne;
    }
    return true;
}

// Runs of one pass that visits every line of a range [lo, hi] exactly once
// with d sweeps of stride d lines (d <= 64): sweep o (after sorting) starts at
// line lo + o, at access (*ks)[o] of the pass.  Returns hi - lo + 1, or 0
// when the pass is not of that shape.
static uint64_t multi_sweep_runs(const DevProbe& p, uint32_t ls, std::vector<uint64_t>* ks) {
    if (p.se == 0 || one_sweep_per_pass(p)) return 0;
    const uint64_t sb = (uint64_t)p.se << p.elem_shift;
    if (sb & ((1ull << ls) - 1)) return 0;
    const uint64_t d = sb >> ls;
    if (d > 64) return 0;
    struct Sw {
        uint64_t first, last, k;
    };
    std::vector<Sw> sw;
    uint64_t r = p.j0, kpos = 0;
    while (kpos < p.L) {
        if (sw.size() == d) return 0;   // more sweeps than residues: some line repeats
        uint64_t cnt = ((uint64_t)p.ne - r + p.se - 1) / p.se;
        if (cnt > p.L - kpos) cnt = p.L - kpos;
        const uint64_t f = (p.base + (r << p.elem_shift)) >> ls;
        sw.push_back(Sw{f, f + (cnt - 1) * d, kpos});
        kpos += cnt;
        r = r + cnt * p.se - p.ne;
    }
    if (sw.size() != d) return 0;
    uint64_t lo = ~0ull, hi = 0;
    for (const Sw& x : sw) {
        lo = std::min(lo, x.first);
        hi = std::max(hi, x.last);
    }
    ks->assign(d, ~0ull);
    for (const Sw& x : sw) {
        const uint64_t o = x.first - lo;
        if (o >= d || hi - x.last >= d || (*ks)[o] != ~0ull) return 0;
        (*ks)[o] = x.k;
    }
    return hi - lo + 1;
}

static uint64_t gcd64(uint64_t x, uint64_t y) {
    while (y) {
        const uint64_t t = x % y;
        x = y;
        y = t;
    }
    return x;
}

// Largest run table (entries of 4 bytes) an inference plan builds.
constexpr uint64_t kMaxTableEntries = 1ull << 26;
// Largest set (lines) a tree-PLRU pattern is tabulated for.
constexpr uint64_t kMaxPatternLines = 4096;
// Associativities whose pattern ids a plan build keeps in a flat table.
constexpr uint64_t kPatternTableWays = 128;

static bool own_sweep(const pchase_model& c, const pchase_probe& p) {
    const uint64_t C = c.capacity_bytes, b = c.line_bytes, N = p.n_bytes, s = p.s_bytes;
    if (2 * N < C || N > 2 * C) return false;
    if (N % b) return false;
    return 2 * s == b || s == b || s == 2 * b;
}

// Pinned staging of a run's results (ws->host_res, 4 KB): the argmin at 0,
// a plan's status word at kHostStatus, the zero-class bitmap from 256.
constexpr size_t kHostStatus = 128;
static_assert(sizeof(ArgminOut) <= kHostStatus, "the argmin result overlaps the status word");

// Ends a plan's run: its status word (bit 0: aborted) comes back with the
// stream's last copy, then the stream is synchronised (one round trip).
static int finish_run(Workspace* ws, const SweepPlan& plan, hipStream_t stream) {
    uint32_t* hs = reinterpret_cast<uint32_t*>(static_cast<uint8_t*>(ws->host_res) + kHostStatus);
    PC_HIP(hipMemcpyAsync(hs, plan.d_queues + plan.batched.size(), sizeof(uint32_t), hipMemcpyDeviceToHost, stream));
    PC_HIP(hipStreamSynchronize(stream));
    if (*hs & 1u) return set_error(PCHASE_EABORTED, "replay aborted by pchase_abort");
    return PCHASE_OK;
}

// Replays `jobs` (grouped by model) with hit bits into `bits` (cleared
// first) and synchronises; the counters go to workspace scratch.
int replay_jobs(Workspace* ws, const std::vector<DevModel>& dm, const std::vector<DevProbe>& dp,
                const std::vector<uint64_t>& len, const std::vector<SweepJob>& jobs, uint32_t* bits,
                uint64_t bits_words, hipStream_t stream) {
    if (jobs.empty()) return PCHASE_OK;
    for (const SweepJob& j : jobs)
        if (j.model >= dm.size() || j.probe >= dp.size() || j.bitoff + (len[j.probe] + 31) / 32 > bits_words)
            return set_error(PCHASE_EINVAL, "internal replay job outside its model, probe or bitmap bounds");
    hipError_t e = ws->aux.ensure(jobs.size() * 16);
    if (e != hipSuccess) return buf_fail(ws, e, "replay counters");
    SweepPlan plan;
    plan.dev.arena = ws->arena;
    int rc = build_sweep_plan(&plan, dm, dp, len, jobs, true);
    if (rc) return rc;
    rc = run_sweep_plan(ws, &plan, false, ws->aux.as<uint64_t>(), 2 * jobs.size(), bits, true, PCHASE_BATCHED,
                        stream, {});
    if (rc) return rc;
    return finish_run(ws, plan, stream);
}

}  // namespace pc

using namespace pc;

// ------------------------------------------------------------- traces ---
// First chunk of every trace in the flat trace-generation grid (one block
// per chunk of kTraceChunkAccesses accesses), n + 1 entries.
static int chunk_offsets(const std::vector<uint64_t>& off, std::vector<uint64_t>* co) {
    co->assign(off.size(), 0);
    for (size_t i = 0; i + 1 < off.size(); ++i)
        (*co)[i + 1] = (*co)[i] + (off[i + 1] - off[i] + kTraceChunkAccesses - 1) / kTraceChunkAccesses;
    if (co->back() >= (1ull << 31)) return set_error(PCHASE_ERANGE, "trace too long for one launch");
    return PCHASE_OK;
}

static int materialise_traces(Workspace* ws, const std::vector<DevProbe>& dp, const std::vector<uint64_t>& o,
                              int32_t* idx_dev, hipStream_t stream);

extern "C" int pchase_trace(const pchase_probe* probes, uint32_t n_probes, int32_t* idx_dev, uint64_t* off,
                            uint64_t cap, hipStream_t stream) {
    std::vector<DevProbe> dp;
    std::vector<uint64_t> len;
    int rc = validate_probes(probes, n_probes, &dp, &len);
    if (rc) return rc;
    std::vector<uint64_t> o(n_probes + 1, 0);
    for (uint32_t i = 0; i < n_probes; ++i) o[i + 1] = o[i] + len[i];
    if (o[n_probes] > cap)
        return set_error(PCHASE_ERANGE, "trace needs %llu elements, capacity is %llu",
                         (unsigned long long)o[n_probes], (unsigned long long)cap);
    if (o[n_probes] && !idx_dev) return set_error(PCHASE_EINVAL, "idx_dev is NULL");
    if (off) std::memcpy(off, o.data(), o.size() * sizeof(uint64_t));
    if (n_probes == 0 || o[n_probes] == 0) return PCHASE_OK;
    Workspace* ws;
    std::unique_lock<std::mutex> lk;
    rc = workspace(&ws, &lk);
    if (rc) return rc;
    return materialise_traces(ws, dp, o, idx_dev, stream);
}

// Writes the probes' traces to idx_dev at offsets o (n + 1 entries) through
// the workspace's staging buffer; synchronises.
static int materialise_traces(Workspace* ws, const std::vector<DevProbe>& dp, const std::vector<uint64_t>& o,
                              int32_t* idx_dev, hipStream_t stream) {
    const uint32_t n_probes = (uint32_t)dp.size();
    if (n_probes == 0 || o[n_probes] == 0) return PCHASE_OK;
    std::vector<uint64_t> co;
    int rc = chunk_offsets(o, &co);
    if (rc) return rc;
    const size_t b_p = dp.size() * sizeof(DevProbe), b_o = o.size() * sizeof(uint64_t);
    const size_t b_c = co.back() * sizeof(ChunkRef);
    hipError_t e = ws->stage.ensure(b_p + 2 * b_o + b_c);
    if (e != hipSuccess) return set_error(PCHASE_ENOMEM, "staging: %s", hipGetErrorString(e));
    uint8_t* st = ws->stage.as<uint8_t>();
    DevProbe* d_p = reinterpret_cast<DevProbe*>(st);
    uint64_t* d_o = reinterpret_cast<uint64_t*>(st + b_p);
    uint64_t* d_co = reinterpret_cast<uint64_t*>(st + b_p + b_o);
    ChunkRef* d_c = reinterpret_cast<ChunkRef*>(st + b_p + 2 * b_o);
    CopyFence fence(stream);
    PC_HIP(hipMemcpyAsync(d_p, dp.data(), b_p, hipMemcpyHostToDevice, stream));
    PC_HIP(hipMemcpyAsync(d_o, o.data(), b_o, hipMemcpyHostToDevice, stream));
    PC_HIP(hipMemcpyAsync(d_co, co.data(), b_o, hipMemcpyHostToDevice, stream));
    PC_HIP(launch_chunk_table(d_co, n_probes, d_c, stream));
    PC_HIP(launch_trace(d_p, d_o, d_c, co.back(), idx_dev, stream));
    // the staging buffer is reused by the next call: finish before releasing it
    PC_HIP(hipStreamSynchronize(stream));
    fence.done();
    return PCHASE_OK;
}

// ------------------------------------------------- non-uniform traces ---
static int check_nu_probe(const pchase_nu_probe& p, const pchase_segment* segs, uint32_t n_segs, uint64_t i,
                          uint64_t* pass_len, uint64_t* len) {
    if (p.elem_bytes != 4) return set_error(PCHASE_EINVAL, "probe %llu: elem_bytes must be 4", (unsigned long long)i);
    if (p.n_bytes == 0 || p.n_bytes % 4)
        return set_error(PCHASE_EINVAL, "probe %llu: N must be a positive multiple of elem_bytes", (unsigned long long)i);
    const uint64_t ne = p.n_bytes / 4;
    if (ne >= (1ull << 31)) return set_error(PCHASE_EINVAL, "probe %llu: N/elem must be below 2^31", (unsigned long long)i);
    if (p.j0 >= ne) return set_error(PCHASE_EINVAL, "probe %llu: j0 outside the array", (unsigned long long)i);
    if (p.passes == 0) return set_error(PCHASE_EINVAL, "probe %llu: passes must be >= 1", (unsigned long long)i);
    if (p.base_offset >= (1ull << 33) || p.base_offset % 4)
        return set_error(PCHASE_EINVAL, "probe %llu: base_offset must be a multiple of 4 below 2^33", (unsigned long long)i);
    if (p.n_segments == 0) return set_error(PCHASE_EINVAL, "probe %llu: no segments", (unsigned long long)i);
    if ((uint64_t)p.first_segment + p.n_segments > n_segs || !segs)
        return set_error(PCHASE_EINVAL, "probe %llu: segment range outside the segment array", (unsigned long long)i);
    uint64_t k = 0;
    for (uint32_t t = 0; t < p.n_segments; ++t) {
        const pchase_segment& sg = segs[p.first_segment + t];
        if (sg.count == 0 || sg.s_bytes % 4)
            return set_error(PCHASE_EINVAL, "probe %llu: segment %u needs count >= 1 and a stride multiple of elem_bytes",
                             (unsigned long long)i, p.first_segment + t);
        if (sg.count >= (1ull << 32) || (k += sg.count) >= (1ull << 32))
            return set_error(PCHASE_ERANGE, "probe %llu: passes * accesses per pass must stay below 2^32", (unsigned long long)i);
    }
    if (k * (uint64_t)p.passes >= (1ull << 32))
        return set_error(PCHASE_ERANGE, "probe %llu: passes * accesses per pass must stay below 2^32", (unsigned long long)i);
    if (pass_len) *pass_len = k;
    if (len) *len = k * p.passes;
    return PCHASE_OK;
}

extern "C" int pchase_trace_nu_len(const pchase_nu_probe* probe, const pchase_segment* segs, uint32_t n_segs,
                                   uint64_t* len, uint64_t* pass_len) {
    if (!probe) return set_error(PCHASE_EINVAL, "probe is NULL");
    return check_nu_probe(*probe, segs, n_segs, 0, pass_len, len);
}

extern "C" int pchase_trace_nu(const pchase_nu_probe* probes, uint32_t n_probes, const pchase_segment* segs,
                               uint32_t n_segs, int32_t* idx_dev, uint64_t* off, uint64_t cap, hipStream_t stream) {
    if (n_probes && !probes) return set_error(PCHASE_EINVAL, "probes is NULL");
    std::vector<uint64_t> o(n_probes + 1, 0);
    std::vector<DevNuProbe> dp(n_probes);
    std::vector<DevNuSeg> ds;
    for (uint32_t i = 0; i < n_probes; ++i) {
        const pchase_nu_probe& p = probes[i];
        uint64_t K = 0, len = 0;
        int rc = check_nu_probe(p, segs, n_segs, i, &K, &len);
        if (rc) return rc;
        const uint64_t ne = p.n_bytes / 4;
        dp[i] = DevNuProbe{K, (uint32_t)ds.size(), p.n_segments, (uint32_t)ne, 0};
        // element of each segment's first access: j0 plus every step taken before it, modulo ne
        uint64_t pos = p.j0, start = 0;
        for (uint32_t t = 0; t < p.n_segments; ++t) {
            const pchase_segment& sg = segs[p.first_segment + t];
            const uint64_t se = (sg.s_bytes / 4) % ne;
            ds.push_back(DevNuSeg{start, (uint32_t)pos, (uint32_t)se});
            pos = (uint64_t)((pos + (unsigned __int128)se * (sg.count % ne)) % ne);
            start += sg.count;
        }
        o[i + 1] = o[i] + len;
    }
    if (o[n_probes] > cap)
        return set_error(PCHASE_ERANGE, "trace needs %llu elements, capacity is %llu",
                         (unsigned long long)o[n_probes], (unsigned long long)cap);
    if (o[n_probes] && !idx_dev) return set_error(PCHASE_EINVAL, "idx_dev is NULL");
    if (off) std::memcpy(off, o.data(), o.size() * sizeof(uint64_t));
    if (n_probes == 0 || o[n_probes] == 0) return PCHASE_OK;
    Workspace* ws;
    std::unique_lock<std::mutex> lk;
    int rc = workspace(&ws, &lk);
    if (rc) return rc;
    std::vector<uint64_t> co;
    rc = chunk_offsets(o, &co);
    if (rc) return rc;
    const size_t b_p = dp.size() * sizeof(DevNuProbe), b_s = ds.size() * sizeof(DevNuSeg);
    const size_t b_o = o.size() * sizeof(uint64_t), b_c = co.back() * sizeof(ChunkRef);
    hipError_t e = ws->stage.ensure(b_p + b_s + 2 * b_o + b_c);
    if (e != hipSuccess) return set_error(PCHASE_ENOMEM, "staging: %s", hipGetErrorString(e));
    uint8_t* st = ws->stage.as<uint8_t>();
    DevNuProbe* d_p = reinterpret_cast<DevNuProbe*>(st);
    DevNuSeg* d_s = reinterpret_cast<DevNuSeg*>(st + b_p);
    uint64_t* d_o = reinterpret_cast<uint64_t*>(st + b_p + b_s);
    uint64_t* d_co = reinterpret_cast<uint64_t*>(st + b_p + b_s + b_o);
    ChunkRef* d_c = reinterpret_cast<ChunkRef*>(st + b_p + b_s + 2 * b_o);
    CopyFence fence(stream);
    PC_HIP(hipMemcpyAsync(d_p, dp.data(), b_p, hipMemcpyHostToDevice, stream));
    PC_HIP(hipMemcpyAsync(d_s, ds.data(), b_s, hipMemcpyHostToDevice, stream));
    PC_HIP(hipMemcpyAsync(d_o, o.data(), b_o, hipMemcpyHostToDevice, stream));
    PC_HIP(hipMemcpyAsync(d_co, co.data(), b_o, hipMemcpyHostToDevice, stream));
    PC_HIP(launch_chunk_table(d_co, n_probes, d_c, stream));
    PC_HIP(launch_trace_nu(d_p, d_s, d_o, d_c, co.back(), idx_dev, stream));
    // the staging buffer is reused by the next call: finish before releasing it
    PC_HIP(hipStreamSynchronize(stream));
    fence.done();
    return PCHASE_OK;
}

// -------------------------------------------------------- probe replay ---
extern "C" int cache_replay_probes(const pchase_model* models, uint32_t n_models, const pchase_probe* probes,
                                   uint32_t n_probes, const uint32_t* pair_model, const uint32_t* pair_probe,
                                   const uint64_t* count_from, uint64_t n_pairs, uint64_t* misses_dev,
                                   uint32_t* hitbits_dev, const uint64_t* bitoff, uint32_t mode,
                                   pchase_plan* pplan, hipStream_t stream) {
    if (mode > PCHASE_PLAIN) return set_error(PCHASE_EINVAL, "unknown mode %u", mode);
    std::vector<DevModel> dm;
    std::vector<DevProbe> dp;
    std::vector<uint64_t> len;
    int rc = validate_models(models, n_models, &dm);
    if (rc) return rc;
    rc = validate_probes(probes, n_probes, &dp, &len);
    if (rc) return rc;
    if (n_pairs == 0) return PCHASE_OK;
    if (!pair_model || !pair_probe) return set_error(PCHASE_EINVAL, "pair arrays are NULL");
    if (!misses_dev) return set_error(PCHASE_EINVAL, "misses_dev is NULL");
    if (hitbits_dev && !bitoff) return set_error(PCHASE_EINVAL, "hitbits_dev needs bitoff");
    if (n_pairs >= (1ull << 32)) return set_error(PCHASE_ERANGE, "too many pairs");
    std::vector<uint32_t> order(n_pairs);
    for (uint64_t i = 0; i < n_pairs; ++i) {
        if (pair_model[i] >= n_models) return set_error(PCHASE_EINVAL, "pair %llu: model index out of range", (unsigned long long)i);
        if (pair_probe[i] >= n_probes) return set_error(PCHASE_EINVAL, "pair %llu: probe index out of range", (unsigned long long)i);
        order[i] = (uint32_t)i;
    }
    std::stable_sort(order.begin(), order.end(),
                     [&](uint32_t x, uint32_t y) { return pair_model[x] < pair_model[y]; });
    std::vector<SweepJob> jobs(n_pairs);
    for (uint64_t q = 0; q < n_pairs; ++q) {
        const uint32_t i = order[q];
        SweepJob& j = jobs[q];
        j.model = pair_model[i];
        j.probe = pair_probe[i];
        j.out = i;
        j.trace_id = pair_probe[i];
        j.count_from = count_from ? count_from[i] : dp[pair_probe[i]].L;
        j.bitoff = bitoff ? bitoff[i] : 0;
    }
    Workspace* ws;
    std::unique_lock<std::mutex> lk;
    rc = workspace_for(pplan, &ws, &lk);
    if (rc) return rc;
    ws->reset_arena();
    SweepPlan plan;
    plan.dev.arena = ws->arena;
    rc = build_sweep_plan(&plan, dm, dp, len, jobs, hitbits_dev != nullptr);
    if (rc) return rc;
    rc = run_sweep_plan(ws, &plan, false, misses_dev, 2 * n_pairs, hitbits_dev, hitbits_dev != nullptr, mode,
                        stream, {});
    if (rc) return rc;
    return finish_run(ws, plan, stream);
}

// -------------------------------------------------- trace-array replay ---
// Host-side descriptors of generalised models: per model its DevGeneral and
// the state bytes of one pair; flat per-set (ways, entry base), set tables
// and cumulative way weights.
struct GeneralDesc {
    std::vector<DevGeneral> gen;
    std::vector<uint64_t> state;
    std::vector<uint2> set_info;
    std::vector<uint32_t> table;
    std::vector<uint32_t> cum;
};

static int build_general(const pchase_general_model* models, uint32_t n, std::vector<DevModel>* dm,
                         GeneralDesc* gd) {
    if (n && !models) return set_error(PCHASE_EINVAL, "models is NULL");
    dm->assign(n, DevModel{});
    gd->gen.assign(n, DevGeneral{});
    gd->state.assign(n, 0);
    for (uint32_t i = 0; i < n; ++i) {
        const pchase_general_model& g = models[i];
        const uint32_t b = g.line_bytes;
        if (b < 4 || (b & (b - 1))) return set_error(PCHASE_EINVAL, "model %u: line_bytes must be a power of two >= 4", i);
        if (g.n_sets == 0 || !g.set_ways) return set_error(PCHASE_EINVAL, "model %u: needs n_sets >= 1 and set_ways", i);
        if (g.policy > PCHASE_WRANDOM) return set_error(PCHASE_EINVAL, "model %u: unknown policy %u", i, g.policy);
        const uint32_t lb = (uint32_t)__builtin_ctz(b);
        if (g.set_shift != 0 && (g.set_shift < lb || g.set_shift > 40))
            return set_error(PCHASE_EINVAL, "model %u: set_shift must be 0 or in [log2(line_bytes), 40]", i);
        if (g.table_len && !g.set_table) return set_error(PCHASE_EINVAL, "model %u: set_table is NULL", i);
        for (uint32_t t = 0; t < g.table_len; ++t)
            if (g.set_table[t] >= g.n_sets) return set_error(PCHASE_EINVAL, "model %u: set_table[%u] >= n_sets", i, t);
        if (gd->set_info.size() + g.n_sets >= (1ull << 31) || gd->table.size() + g.table_len >= (1ull << 31))
            return set_error(PCHASE_ERANGE, "generalised models: too many sets or table entries");
        uint32_t amax = 0;
        uint64_t entries = 0;
        DevGeneral& d = gd->gen[i];
        d.set_off = (uint32_t)gd->set_info.size();
        d.table_off = (uint32_t)gd->table.size();
        d.table_len = g.table_len;
        for (uint32_t t = 0; t < g.n_sets; ++t) {
            const uint32_t a = g.set_ways[t];
            if (a == 0 || a > 128) return set_error(PCHASE_EINVAL, "model %u: set %u needs 1..128 ways", i, t);
            if (g.policy == PCHASE_PLRU && (a & (a - 1)))
                return set_error(PCHASE_EINVAL, "model %u: PLRU needs a power-of-two number of ways", i);
            if (entries >= (1ull << 32)) return set_error(PCHASE_ERANGE, "model %u: too many ways", i);
            gd->set_info.push_back(make_uint2(a, (uint32_t)entries));
            entries += a;
            amax = std::max(amax, a);
        }
        for (uint32_t t = 0; t < g.table_len; ++t) gd->table.push_back(g.set_table[t]);
        d.cum_off = (uint32_t)gd->cum.size();
        if (g.policy == PCHASE_WRANDOM) {
            if (!g.way_weights || g.weights_len < amax)
                return set_error(PCHASE_EINVAL, "model %u: WRANDOM needs a weight for every way of its widest set", i);
            uint64_t c = 0;
            for (uint32_t w = 0; w < amax; ++w) {
                c += g.way_weights[w];
                if (c > 65536) c = 65537;   // flagged below for any set that reaches it
                gd->cum.push_back((uint32_t)c);
            }
            for (uint32_t t = 0; t < g.n_sets; ++t) {
                const uint32_t sum = gd->cum[d.cum_off + g.set_ways[t] - 1];
                if (sum == 0 || sum > 65536)
                    return set_error(PCHASE_EINVAL, "model %u: set %u's weights must sum to 1..65536", i, t);
            }
        }
        DevModel& m = (*dm)[i];
        m = DevModel{};
        m.line_shift = lb;
        m.unit_shift = g.set_shift ? g.set_shift : lb;
        m.sets = g.n_sets;
        m.ways = amax;
        m.policy = g.policy;
        m.log2_ways = 31u - (uint32_t)__builtin_clz(amax);
        m.seed_lo = (uint32_t)g.seed;
        m.seed_hi = (uint32_t)(g.seed >> 32);
        gd->state[i] = (uint64_t)g.n_sets * 32 + entries * 8;
    }
    return PCHASE_OK;
}

// held: a workspace the caller has locked and laid out already (its arena
// is not reset); NULL takes the plan's or the device's workspace.
static int replay_materialised(const std::vector<DevModel>& dm, const GeneralDesc* gd, uint32_t n_models,
                               const int32_t* idx_dev, const uint64_t* trace_off, const uint64_t* trace_base,
                               uint32_t n_traces, const uint32_t* pair_model, const uint32_t* pair_trace,
                               const uint64_t* count_from, uint64_t n_pairs, uint64_t* misses_dev,
                               uint32_t* hitbits_dev, const uint64_t* bitoff, uint32_t mode, pchase_plan* plan,
                               hipStream_t stream, Workspace* held = nullptr);

extern "C" int cache_replay_batch(const pchase_model* models, uint32_t n_models, const int32_t* idx_dev,
                                  const uint64_t* trace_off, const uint64_t* trace_base, uint32_t elem_bytes,
                                  uint32_t n_traces, const uint32_t* pair_model, const uint32_t* pair_trace,
                                  const uint64_t* count_from, uint64_t n_pairs, uint64_t* misses_dev,
                                  uint32_t* hitbits_dev, const uint64_t* bitoff, uint32_t mode,
                                  pchase_plan* plan, hipStream_t stream) {
    if (mode > PCHASE_PLAIN) return set_error(PCHASE_EINVAL, "unknown mode %u", mode);
    if (elem_bytes != 4) return set_error(PCHASE_EINVAL, "elem_bytes must be 4");
    std::vector<DevModel> dm;
    int rc = validate_models(models, n_models, &dm);
    if (rc) return rc;
    return replay_materialised(dm, nullptr, n_models, idx_dev, trace_off, trace_base, n_traces, pair_model,
                               pair_trace, count_from, n_pairs, misses_dev, hitbits_dev, bitoff, mode, plan, stream);
}

extern "C" int cache_replay_general(const pchase_general_model* models, uint32_t n_models, const int32_t* idx_dev,
                                    const uint64_t* trace_off, const uint64_t* trace_base, uint32_t elem_bytes,
                                    uint32_t n_traces, const uint32_t* pair_model, const uint32_t* pair_trace,
                                    const uint64_t* count_from, uint64_t n_pairs, uint64_t* misses_dev,
                                    uint32_t* hitbits_dev, const uint64_t* bitoff, uint32_t mode,
                                    pchase_plan* plan, hipStream_t stream) {
    if (mode > PCHASE_PLAIN) return set_error(PCHASE_EINVAL, "unknown mode %u", mode);
    if (elem_bytes != 4) return set_error(PCHASE_EINVAL, "elem_bytes must be 4");
    std::vector<DevModel> dm;
    GeneralDesc gd;
    int rc = build_general(models, n_models, &dm, &gd);
    if (rc) return rc;
    return replay_materialised(dm, &gd, n_models, idx_dev, trace_off, trace_base, n_traces, pair_model,
                               pair_trace, count_from, n_pairs, misses_dev, hitbits_dev, bitoff, mode, plan, stream);
}

// Host memory for the large arrays of a plan or schedule build (work
// items, decided jobs, descriptor images): from 4 MB on, 2 MB-aligned and
// advised as transparent huge pages, so that first touch costs a few dozen
// page faults instead of thousands; not initialised.
static void* huge_alloc(size_t bytes) {
    if (bytes < (4u << 20)) return std::malloc(bytes ? bytes : 1);
    const size_t al = 2u << 20, sz = (bytes + al - 1) / al * al;
    void* p = std::aligned_alloc(al, sz);
    if (p) (void)madvise(p, sz, MADV_HUGEPAGE);
    return p;
}
template <class T>
struct HugeAlloc {
    using value_type = T;
    HugeAlloc() = default;
    template <class U>
    HugeAlloc(const HugeAlloc<U>&) {}
    T* allocate(size_t n) {
        void* p = huge_alloc(n * sizeof(T));
        if (!p) throw std::bad_alloc();
        return static_cast<T*>(p);
    }
    void deallocate(T* p, size_t) { std::free(p); }
    template <class U>
    bool operator==(const HugeAlloc<U>&) const { return true; }
    template <class U>
    bool operator!=(const HugeAlloc<U>&) const { return false; }
};
struct HostImage {
    uint8_t* p = nullptr;
    explicit HostImage(size_t n) : p(static_cast<uint8_t*>(huge_alloc(n))) {}
    ~HostImage() { std::free(p); }
    HostImage(const HostImage&) = delete;
    HostImage& operator=(const HostImage&) = delete;
};

template <class T>
using HugeVec = std::vector<T, HugeAlloc<T>>;

// Standard models: the set-partitioned tile replay.  Every pair becomes
// one or more (pair, part) items: the fewest parts P (a power of two, at
// most T) for which one part's sets fit a wave's LDS state of at most
// row_cap dwords per lane.  Items are grouped by (policy, way class, row
// class: the state rows rounded up to a power of two, at least 16), each
// group one launch whose LDS fits its class, longest items first.
struct TileSchedule {
    HugeVec<TileItem> items;     // grouped, longest first in a group
    HugeVec<uint32_t> key;       // group key of each item
    HugeVec<float> cost;         // estimated cost of each item
    std::vector<uint64_t> zero_cnt;  // (word, count) ranges that split pairs merge into
    std::vector<uint64_t> zero_bits;
};

static int build_tile_schedule(const std::vector<DevModel>& dm, uint32_t n_models, const uint64_t* trace_off,
                               const uint64_t* trace_base, uint32_t n_traces, const uint32_t* pair_model,
                               const uint32_t* pair_trace, const uint64_t* count_from, uint64_t n_pairs,
                               bool want_bits, const uint64_t* bitoff, TileSchedule* ts) {
    const uint32_t row_cap = 256;
    HugeVec<TileItem> items;
    items.reserve(n_pairs);
    HugeVec<uint32_t> key;   // group key | cost bucket << 8 of each item
    HugeVec<float> cost;
    key.reserve(n_pairs);
    cost.reserve(n_pairs);
    ts->zero_cnt.clear();
    ts->zero_bits.clear();
    for (uint64_t i = 0; i < n_pairs; ++i) {
        if (pair_model[i] >= n_models) return set_error(PCHASE_EINVAL, "pair %llu: model index out of range", (unsigned long long)i);
        if (pair_trace[i] >= n_traces) return set_error(PCHASE_EINVAL, "pair %llu: trace index out of range", (unsigned long long)i);
        const DevModel& m = dm[pair_model[i]];
        // rows of the largest part's layout when split into 2^l parts (the
        // parts hold ceil(T / 2^l) or floor(T / 2^l) sets: parts 0 and last)
        auto rows_of = [&](uint32_t l) {
            const TileLayout l0 = tile_layout((int)m.policy, m.ways, m.sets, l, 0);
            const TileLayout l1 = tile_layout((int)m.policy, m.ways, m.sets, l, (1u << l) - 1);
            return std::max<uint64_t>((uint64_t)l0.slots * l0.rs, (uint64_t)l1.slots * l1.rs);
        };
        uint32_t lp = 0;
        while (rows_of(lp) > row_cap && (2ull << lp) <= m.sets) ++lp;
        if (rows_of(lp) > kTileMaxRows)
            return set_error(PCHASE_ERANGE, "pair %llu: a set of %u ways does not fit the replay state",
                             (unsigned long long)i, m.ways);
        const uint64_t len = trace_off[pair_trace[i] + 1] - trace_off[pair_trace[i]];
        const uint32_t P = 1u << lp;
        for (uint32_t p = 0; p < P; ++p) {
            const TileLayout ly = tile_layout((int)m.policy, m.ways, m.sets, lp, p);
            const uint64_t rows = (uint64_t)ly.slots * ly.rs;
            uint32_t rc = 16, cls = 0;
            while (rc < rows) {
                rc *= 2;
                ++cls;
            }
            TileItem t;
            t.start = trace_off[pair_trace[i]];
            t.len = len;
            t.base = trace_base ? trace_base[pair_trace[i]] : 0;
            t.count_from = count_from ? count_from[i] : 0;
            t.bitoff = bitoff ? bitoff[i] : 0;
            t.model = pair_model[i];
            t.trace_id = pair_trace[i];
            t.out = (uint32_t)i;
            t.part = p | (lp << 16);
            const uint32_t grp = m.policy * kTileWayClasses + (uint32_t)tile_way_class(ly.kw);
            const float c = (float)((double)len * (8.0 + (double)ly.kw * (1u << ly.lw) / P));
            // cost bucket: the float's exponent and top 4 mantissa bits, so
            // that larger costs come first at 1/16-octave resolution
            uint32_t cb;
            std::memcpy(&cb, &c, 4);
            key.push_back((grp * 8u + cls) | ((4095u - ((cb >> 19) & 4095u)) << 8));
            cost.push_back(c);
            items.push_back(t);
        }
        if (P > 1) {
            ts->zero_cnt.push_back(4 * i);   // the pair's two 64-bit counters, as 32-bit words
            ts->zero_cnt.push_back(4);
            if (want_bits) {
                ts->zero_bits.push_back(bitoff[i]);
                ts->zero_bits.push_back((len + 31) / 32);
            }
        }
    }
    if (items.size() >= (1ull << 32)) return set_error(PCHASE_ERANGE, "too many pairs");
    // counting sort by (group key, cost bucket), stable: groups contiguous,
    // longest items first within a group (to the bucket's resolution)
    const uint32_t n_keys = 4 * kTileWayClasses * 8;
    auto rank = [&](uint32_t k) { return (k & 0xFFu) * 4096u + (k >> 8); };
    std::vector<uint32_t> start((size_t)n_keys * 4096 + 1, 0);
    for (uint32_t k : key) ++start[rank(k) + 1];
    for (size_t b = 1; b < start.size(); ++b) start[b] += start[b - 1];
    const size_t n_items = items.size();
    ts->items.resize(n_items);
    ts->key.resize(n_items);
    ts->cost.resize(n_items);
    for (size_t q = 0; q < n_items; ++q) {
        const uint32_t pos = start[rank(key[q])]++;
        ts->items[pos] = items[q];
        ts->key[pos] = key[q] & 0xFFu;
        ts->cost[pos] = cost[q];
    }
    return PCHASE_OK;
}

// Device bytes a schedule's descriptors take in scratch.
struct TileScratch {
    size_t o_models, o_items, o_status, o_zero, total;
};
static TileScratch tile_scratch_layout(size_t n_models, const TileSchedule& ts) {
    TileScratch L;
    L.o_models = 0;
    L.o_items = (n_models * sizeof(DevModel) + 255) / 256 * 256;
    L.o_status = L.o_items + (ts.items.size() * sizeof(TileItem) + 255) / 256 * 256;
    L.o_zero = L.o_status + 512;
    L.total = L.o_zero + (ts.zero_cnt.size() + ts.zero_bits.size()) * sizeof(uint64_t) + 256;
    return L;
}

// Enqueues a schedule whose descriptors go to device scratch `sb` (at least
// tile_scratch_layout(...).total bytes), waits and reads the status.  With
// a workspace the groups run concurrently on its replay streams; without
// one (ws = NULL) every launch goes to `stream`, one after the other.
// BATCHED runs each group as a persistent grid pulling items from an atomic
// queue; PLAIN launches one block per item.  occ caches resident blocks per
// (group, row class) (0 = unknown).
static int run_tile_schedule(const std::vector<DevModel>& dm, const TileSchedule& ts, uint8_t* sb, Workspace* ws,
                             int (*occ)[8], int cus, const volatile uint32_t* abort_flag, const int32_t* idx_dev,
                             uint64_t* misses_dev, uint32_t* hitbits_dev, uint32_t mode, hipStream_t stream) {
    const TileScratch SL = tile_scratch_layout(dm.size(), ts);
    DevModel* d_models = reinterpret_cast<DevModel*>(sb + SL.o_models);
    TileItem* d_items = reinterpret_cast<TileItem*>(sb + SL.o_items);
    uint32_t* d_status = reinterpret_cast<uint32_t*>(sb + SL.o_status);
    CopyFence fence(stream);
    PC_HIP(hipMemcpyAsync(d_models, dm.data(), dm.size() * sizeof(DevModel), hipMemcpyHostToDevice, stream));
    PC_HIP(hipMemcpyAsync(d_items, ts.items.data(), ts.items.size() * sizeof(TileItem), hipMemcpyHostToDevice,
                          stream));
    PC_HIP(launch_fill_u32(d_status, 128, 0, stream));
    if (!ts.zero_cnt.empty()) {
        // split pairs merge into their outputs: zero those first
        uint64_t* d_zc = reinterpret_cast<uint64_t*>(sb + SL.o_zero);
        uint64_t* d_zb = d_zc + ts.zero_cnt.size();
        PC_HIP(hipMemcpyAsync(d_zc, ts.zero_cnt.data(), ts.zero_cnt.size() * 8, hipMemcpyHostToDevice, stream));
        PC_HIP(launch_clear_ranges(reinterpret_cast<uint32_t*>(misses_dev), d_zc,
                                   (uint32_t)(ts.zero_cnt.size() / 2), stream));
        if (!ts.zero_bits.empty()) {
            PC_HIP(hipMemcpyAsync(d_zb, ts.zero_bits.data(), ts.zero_bits.size() * 8, hipMemcpyHostToDevice, stream));
            PC_HIP(launch_clear_ranges(hitbits_dev, d_zb, (uint32_t)(ts.zero_bits.size() / 2), stream));
        }
    }
    // one launch per group
    struct Launch {
        int pol, wcls;
        uint32_t rows;
        uint64_t q, e2, blocks;
        double cost;
    };
    std::vector<Launch> launches;
    for (uint64_t q = 0; q < ts.items.size();) {
        const uint32_t key = ts.key[q];
        uint64_t e2 = q;
        double work = 0;
        while (e2 < ts.items.size() && ts.key[e2] == key) work += ts.cost[e2++];
        Launch L;
        L.pol = (int)(key / 8 / kTileWayClasses);
        L.wcls = (int)(key / 8 % kTileWayClasses);
        L.rows = 16u << (key % 8);
        L.q = q;
        L.e2 = e2;
        int& oc = occ[key / 8][key % 8];
        if (oc == 0) {
            PC_HIP(tile_occupancy(L.pol, L.wcls, L.rows, &oc));
            if (oc < 1) oc = 1;
        }
        L.blocks = mode == PCHASE_PLAIN ? e2 - q : std::min<uint64_t>((uint64_t)oc * cus, e2 - q);
        L.cost = std::max((double)ts.cost[q], work / (double)L.blocks);
        launches.push_back(L);
        q = e2;
    }
    if (launches.size() > 120) return set_error(PCHASE_ERANGE, "too many replay groups");
    std::vector<size_t> order(launches.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = i;
    std::sort(order.begin(), order.end(), [&](size_t x, size_t y) { return launches[x].cost > launches[y].cost; });
    const int ns = (mode == PCHASE_PLAIN || !ws) ? 0 : (int)std::min<size_t>(kBranches, launches.size());
    double load[kBranches] = {};
    if (ns > 1) PC_HIP(fork_branches(ws, stream, ns));
    for (size_t oi = 0; oi < order.size(); ++oi) {
        const Launch& L = launches[order[oi]];
        hipStream_t st = stream;
        if (ns > 1) {
            int b = 0;
            for (int c = 1; c < ns; ++c)
                if (load[c] < load[b]) b = c;
            load[b] += L.cost;
            st = branch_stream(ws, stream, b);
        }
        TileArgs a;
        a.items = d_items + L.q;
        a.n_items = (uint32_t)(L.e2 - L.q);
        a.persistent = mode == PCHASE_PLAIN ? 0u : 1u;
        a.queue = d_status + 2 + order[oi];
        a.models = d_models;
        a.idx = idx_dev;
        a.misses = misses_dev;
        a.bits = hitbits_dev;
        a.rows = L.rows;
        a.abort_flag = mode == PCHASE_PLAIN ? nullptr : abort_flag;
        a.status = d_status;
        PC_HIP(launch_tile(L.pol, L.wcls, a, (uint32_t)L.blocks, st));
    }
    if (ns > 1) PC_HIP(join_branches(ws, stream, ns));
    PC_HIP(hipStreamSynchronize(stream));
    fence.done();
    uint32_t status = 0;
    PC_HIP(hipMemcpy(&status, d_status, sizeof status, hipMemcpyDeviceToHost));
    if (status & 1u) return set_error(PCHASE_EABORTED, "replay aborted by pchase_abort");
    if (status & 2u) return set_error(PCHASE_EINVAL, "a trace holds a negative element index");
    return PCHASE_OK;
}

static int replay_tiles(const std::vector<DevModel>& dm, uint32_t n_models, const int32_t* idx_dev,
                        const uint64_t* trace_off, const uint64_t* trace_base, uint32_t n_traces,
                        const uint32_t* pair_model, const uint32_t* pair_trace, const uint64_t* count_from,
                        uint64_t n_pairs, uint64_t* misses_dev, uint32_t* hitbits_dev, const uint64_t* bitoff,
                        uint32_t mode, pchase_plan* plan, hipStream_t stream) {
    TileSchedule ts;
    int rc = build_tile_schedule(dm, n_models, trace_off, trace_base, n_traces, pair_model, pair_trace, count_from,
                                 n_pairs, hitbits_dev != nullptr, bitoff, &ts);
    if (rc) return rc;
    Workspace* ws;
    std::unique_lock<std::mutex> lk;
    rc = workspace_for(plan, &ws, &lk);
    if (rc) return rc;
    ws->reset_arena();
    const TileScratch SL = tile_scratch_layout(dm.size(), ts);
    hipError_t e = ws->stage.ensure(SL.total);
    if (e != hipSuccess) return buf_fail(ws, e, "the replay's descriptors");
    if (!ws->tile_ready) {
        PC_HIP(tile_prepare_lds());
        ws->tile_ready = true;
    }
    return run_tile_schedule(dm, ts, ws->stage.as<uint8_t>(), ws, ws->occ_tile, ws->cus, abort_flag_dev(), idx_dev,
                             misses_dev, hitbits_dev, mode, stream);
}

// ------------------------------------------- replay without allocation ---
// Descriptor scratch of cache_replay_batch_static: a file-scope device array
// (each GPU the library runs on holds its own copy until the process ends).
// Host code reaches it only through the address hipGetSymbolAddress gives
// on each device.
constexpr size_t kStaticScratchBytes = 64ull << 20;
static __device__ __align__(256) uint8_t scratch[kStaticScratchBytes];

struct StaticDev {
    uint8_t* ptr = nullptr;   // device address of `scratch` on this device
    int cus = 0;
    int occ[4 * kTileWayClasses][8] = {};
};
static std::mutex g_static_mu;
static std::map<int, StaticDev> g_static;

// Set-up on the current device, once: the scratch address, the CU count and
// the replay kernels' LDS limit.
static int static_device(StaticDev** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return set_error(PCHASE_ENODEV, "no HIP device: %s", hipGetErrorString(e));
    std::lock_guard<std::mutex> g(g_static_mu);
    StaticDev& sd = g_static[dev];
    if (!sd.ptr) {
        hipDeviceProp_t prop;
        e = hipGetDeviceProperties(&prop, dev);
        if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
        if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
            return set_error(PCHASE_ENODEV, "device %d is %s, the library is built for gfx950", dev, prop.gcnArchName);
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        PC_HIP(tile_prepare_lds());
        sd.cus = prop.multiProcessorCount;
        sd.ptr = static_cast<uint8_t*>(p);
    }
    *out = &sd;
    return PCHASE_OK;
}

extern "C" int cache_replay_batch_static(const pchase_model* models, uint32_t n_models, const int32_t* idx_dev,
                                         const uint64_t* trace_off, const uint64_t* trace_base, uint32_t elem_bytes,
                                         uint32_t n_traces, const uint32_t* pair_model, const uint32_t* pair_trace,
                                         const uint64_t* count_from, uint64_t n_pairs, uint64_t* misses_dev,
                                         uint32_t* hitbits_dev, const uint64_t* bitoff, hipStream_t stream) {
    if (elem_bytes != 4) return set_error(PCHASE_EINVAL, "elem_bytes must be 4");
    std::vector<DevModel> dm;
    int rc = validate_models(models, n_models, &dm);
    if (rc) return rc;
    if (n_pairs == 0) return PCHASE_OK;
    if (!trace_off || !pair_model || !pair_trace) return set_error(PCHASE_EINVAL, "trace or pair arrays are NULL");
    if (!misses_dev) return set_error(PCHASE_EINVAL, "misses_dev is NULL");
    if (hitbits_dev && !bitoff) return set_error(PCHASE_EINVAL, "hitbits_dev needs bitoff");
    if (n_pairs >= (1ull << 32)) return set_error(PCHASE_ERANGE, "too many pairs");
    for (uint32_t t = 0; t < n_traces; ++t) {
        if (trace_off[t + 1] < trace_off[t]) return set_error(PCHASE_EINVAL, "trace_off is not monotone at %u", t);
        if (trace_base && (trace_base[t] >= (1ull << 33) || trace_base[t] % 4))
            return set_error(PCHASE_EINVAL, "trace %u: base must be a multiple of 4 below 2^33", t);
    }
    if (trace_off[n_traces] && !idx_dev) return set_error(PCHASE_EINVAL, "idx_dev is NULL");
    TileSchedule ts;
    rc = build_tile_schedule(dm, n_models, trace_off, trace_base, n_traces, pair_model, pair_trace, count_from,
                             n_pairs, hitbits_dev != nullptr, bitoff, &ts);
    if (rc) return rc;
    const TileScratch SL = tile_scratch_layout(dm.size(), ts);
    if (SL.total > kStaticScratchBytes)
        return set_error(PCHASE_ERANGE, "the call's descriptors take %zu bytes, the fixed scratch holds %zu",
                         SL.total, kStaticScratchBytes);
    StaticDev* sd;
    rc = static_device(&sd);
    if (rc) return rc;
    // (no abort flag: the mapped page behind it would be an allocation)
    return run_tile_schedule(dm, ts, sd->ptr, nullptr, sd->occ, sd->cus, nullptr, idx_dev, misses_dev, hitbits_dev,
                             PCHASE_BATCHED, stream);
}

static int replay_materialised(const std::vector<DevModel>& dm, const GeneralDesc* gd, uint32_t n_models,
                               const int32_t* idx_dev, const uint64_t* trace_off, const uint64_t* trace_base,
                               uint32_t n_traces, const uint32_t* pair_model, const uint32_t* pair_trace,
                               const uint64_t* count_from, uint64_t n_pairs, uint64_t* misses_dev,
                               uint32_t* hitbits_dev, const uint64_t* bitoff, uint32_t mode, pchase_plan* plan,
                               hipStream_t stream, Workspace* held) {
    int rc = PCHASE_OK;
    if (n_pairs == 0) return PCHASE_OK;
    if (!trace_off || !pair_model || !pair_trace) return set_error(PCHASE_EINVAL, "trace or pair arrays are NULL");
    if (!misses_dev) return set_error(PCHASE_EINVAL, "misses_dev is NULL");
    if (hitbits_dev && !bitoff) return set_error(PCHASE_EINVAL, "hitbits_dev needs bitoff");
    if (n_pairs >= (1ull << 32)) return set_error(PCHASE_ERANGE, "too many pairs");
    for (uint32_t t = 0; t < n_traces; ++t) {
        if (trace_off[t + 1] < trace_off[t]) return set_error(PCHASE_EINVAL, "trace_off is not monotone at %u", t);
        if (trace_base && (trace_base[t] >= (1ull << 33) || trace_base[t] % 4))
            return set_error(PCHASE_EINVAL, "trace %u: base must be a multiple of 4 below 2^33", t);
    }
    if (trace_off[n_traces] && !idx_dev) return set_error(PCHASE_EINVAL, "idx_dev is NULL");
    if (!gd) {
        if (held) return set_error(PCHASE_EINVAL, "internal: standard replay in a held workspace");
        return replay_tiles(dm, n_models, idx_dev, trace_off, trace_base, n_traces, pair_model, pair_trace, count_from,
                            n_pairs, misses_dev, hitbits_dev, bitoff, mode, plan, stream);
    }

    // generalised models: bucket pairs by (policy, group width), longest first inside a bucket;
    // a pair that is long, or whose state is large, is split by set into
    // parts that run side by side: each part's serial chain of state updates
    // and its state slab shrink by the number of parts
    // Every part scans the whole trace, so a length split trades scanning
    // work for a shorter chain; it pays only while pairs alone do not fill
    // the chip.  Measured: 1e6 pairs of 1e3..1e5 accesses take 7.9 s with a
    // split above 8192 accesses, 5.5 s above 32768 and 5.2 s above 131072;
    // 4096 pairs of up to 1.1e6 accesses take 0.80 s above 8192 and 0.91 s
    // above 131072.
    const uint64_t kSplitLen = n_pairs >= 65536 ? 131072 : 8192;
    constexpr uint64_t kPartState = 256 << 10;
    struct Item {
        int key;
        uint64_t len;
        uint32_t i;
        uint32_t parts, part;
    };
    std::vector<Item> items;
    items.reserve(n_pairs);
    std::map<int, uint64_t> bucket_state;   // largest model state of each (policy, width) bucket
    std::vector<uint64_t> zero_cnt, zero_bits;   // (word, count) ranges merged into by split pairs
    for (uint64_t i = 0; i < n_pairs; ++i) {
        if (pair_model[i] >= n_models) return set_error(PCHASE_EINVAL, "pair %llu: model index out of range", (unsigned long long)i);
        if (pair_trace[i] >= n_traces) return set_error(PCHASE_EINVAL, "pair %llu: trace index out of range", (unsigned long long)i);
        const DevModel& m = dm[pair_model[i]];
        uint32_t w = 1;
        while (w < m.ways && w < 64) w *= 2;
        int wl = 0;
        while ((1u << wl) < w) ++wl;
        const uint64_t len = trace_off[pair_trace[i] + 1] - trace_off[pair_trace[i]];
        const int key = (gd ? 64 : 0) + (int)m.policy * 8 + wl;
        // parts: a power of two (at most 64 and at most T) until each part's
        // chain is at most kSplitLen accesses and its state at most
        // kPartState.  A generalised model's sets differ in size, so each of
        // its parts keeps the whole state layout: it splits only for length
        // and only while that state is small.
        const uint64_t per_set = 32 + (uint64_t)m.ways * 8;
        uint32_t parts = 1;
        if (!gd) {
            while (parts < 64 && 2 * parts <= m.sets &&
                   ((uint64_t)parts * kSplitLen < len || ((m.sets + parts - 1) / parts) * per_set > kPartState))
                parts *= 2;
        } else if (gd->state[pair_model[i]] <= kPartState) {
            while (parts < 64 && 2 * parts <= m.sets && (uint64_t)parts * kSplitLen < len) parts *= 2;
        }
        uint64_t& bs = bucket_state[key];
        bs = std::max<uint64_t>(bs, gd ? gd->state[pair_model[i]] : (uint64_t)((m.sets + parts - 1) / parts) * per_set);
        for (uint32_t p = 0; p < parts; ++p) items.push_back(Item{key, len, (uint32_t)i, parts, p});
        if (parts > 1) {
            zero_cnt.push_back(4 * i);   // the pair's two 64-bit counters, as 32-bit words
            zero_cnt.push_back(4);
            if (hitbits_dev) {
                zero_bits.push_back(bitoff[i]);
                zero_bits.push_back((len + 31) / 32);
            }
        }
    }
    if (items.size() >= (1ull << 32)) return set_error(PCHASE_ERANGE, "too many pairs");
    std::sort(items.begin(), items.end(), [](const Item& x, const Item& y) {
        if (x.key != y.key) return x.key < y.key;
        if (x.len != y.len) return x.len > y.len;
        if (x.i != y.i) return x.i < y.i;
        return x.part < y.part;
    });
    const uint64_t n_items = items.size();
    std::vector<StreamPair> pairs(n_items);
    for (uint64_t q = 0; q < n_items; ++q) {
        const uint32_t i = items[q].i;
        StreamPair& p = pairs[q];
        p.start = trace_off[pair_trace[i]];
        p.len = items[q].len;
        p.base = trace_base ? trace_base[pair_trace[i]] : 0;
        p.count_from = count_from ? count_from[i] : 0;
        p.bitoff = bitoff ? bitoff[i] : 0;
        p.model = pair_model[i];
        p.trace_id = pair_trace[i];
        p.out = i;
        p.pad = items[q].parts > 1 ? (items[q].parts << 16) | items[q].part : 0;
    }

    Workspace* ws = held;
    std::unique_lock<std::mutex> lk;
    if (!ws) {
        rc = workspace_for(plan, &ws, &lk);
        if (rc) return rc;
        ws->reset_arena();
    }
    // descriptors
    const size_t o_models = 0;
    const size_t o_pairs = (dm.size() * sizeof(DevModel) + 255) / 256 * 256;
    const size_t o_status = o_pairs + (pairs.size() * sizeof(StreamPair) + 255) / 256 * 256;
    const size_t o_zero = o_status + 512;
    const size_t o_gen = (o_zero + (zero_cnt.size() + zero_bits.size()) * sizeof(uint64_t) + 255) / 256 * 256;
    size_t o_info = o_gen, o_table = o_gen, o_cum = o_gen, total = o_gen + 256;
    if (gd) {
        o_info = o_gen + (gd->gen.size() * sizeof(DevGeneral) + 255) / 256 * 256;
        o_table = o_info + (gd->set_info.size() * sizeof(uint2) + 255) / 256 * 256;
        o_cum = o_table + (gd->table.size() * sizeof(uint32_t) + 255) / 256 * 256;
        total = o_cum + (gd->cum.size() * sizeof(uint32_t) + 255) / 256 * 256 + 256;
    }
    hipError_t e = ws->stage.ensure(total);
    if (e != hipSuccess) return buf_fail(ws, e, "the replay's descriptors");
    uint8_t* sb = ws->stage.as<uint8_t>();
    DevModel* d_models = reinterpret_cast<DevModel*>(sb + o_models);
    StreamPair* d_pairs = reinterpret_cast<StreamPair*>(sb + o_pairs);
    uint32_t* d_status = reinterpret_cast<uint32_t*>(sb + o_status);
    const DevGeneral* d_gen = nullptr;
    const uint2* d_info = nullptr;
    const uint32_t *d_table = nullptr, *d_cum = nullptr;
    if (gd) {
        d_gen = reinterpret_cast<const DevGeneral*>(sb + o_gen);
        d_info = reinterpret_cast<const uint2*>(sb + o_info);
        d_table = reinterpret_cast<const uint32_t*>(sb + o_table);
        d_cum = reinterpret_cast<const uint32_t*>(sb + o_cum);
    }

    // state slabs: one per resident group, sized per bucket; the pool may
    // take half of the free device memory (at least 4 GiB, at most 64 GiB)
    // (with a plan: what the plan's memory has left)
    size_t mem_free = 0, mem_total = 0;
    uint64_t pool_cap;
    if (ws->arena) {
        const size_t at = (ws->arena->used + 255) / 256 * 256;
        pool_cap = at < ws->arena->cap ? ws->arena->cap - at : 0;
    } else {
        PC_HIP(hipMemGetInfo(&mem_free, &mem_total));
        pool_cap = std::max<uint64_t>(4ull << 30, std::min<uint64_t>((mem_free + ws->slab.cap) / 2, 64ull << 30));
    }
    for (const auto& kv : bucket_state)
        if ((kv.second + 255) / 256 * 256 > pool_cap)
            return set_error(PCHASE_ERANGE, "model state of %llu bytes exceeds the slab pool",
                             (unsigned long long)kv.second);

    // epochs are unique per pair across calls; on wrap the pool is cleared
    if ((uint64_t)ws->epoch + n_items + 1 >= 0xFFFFFFFFull) {
        ws->epoch = 0;
        ws->slab_clean = 0;
    }
    // one launch per (policy, width) bucket; buckets run concurrently on
    // the workspace's replay streams, each on its own region of the slab
    // pool, so that one bucket's longest pair does not wait for another's
    struct Launch {
        bool gen;
        int pol, W;
        uint64_t q, e2, blocks, gpb, slab_bytes, region;
        double cost;
    };
    std::vector<Launch> launches;
    for (uint64_t q = 0; q < n_items;) {
        const int key = items[q].key;
        uint64_t e2 = q;
        double work = 0;
        while (e2 < n_items && items[e2].key == key) {
            work += (double)items[e2].len / items[e2].parts;
            ++e2;
        }
        const bool gen = key >= 64;
        const int pol = (key % 64) / 8, wl = key % 8, W = 1 << wl;
        int occ = ws->occ_stream[gen][pol][wl];
        if (occ == 0) {
            hipError_t eo = stream_occupancy(pol, W, gen, &occ);
            if (eo != hipSuccess) return hip_fail(eo, "hipOccupancyMaxActiveBlocksPerMultiprocessor");
            if (occ < 1) occ = 1;
            ws->occ_stream[gen][pol][wl] = occ;
        }
        Launch L;
        L.gen = gen;
        L.pol = pol;
        L.W = W;
        L.q = q;
        L.e2 = e2;
        L.gpb = 4ull * (64 / W);  // groups per 256-thread block
        L.slab_bytes = (bucket_state[key] + 255) / 256 * 256;
        const uint64_t need = (e2 - q + L.gpb - 1) / L.gpb;
        L.blocks = mode == PCHASE_PLAIN ? need : std::min<uint64_t>((uint64_t)occ * ws->cus, need);
        // the longest pair (first, pairs are longest first) or the bucket's share
        L.cost = std::max((double)items[q].len / items[q].parts, work / (double)(L.blocks * L.gpb));
        launches.push_back(L);
        q = e2;
    }
    // concurrent when every bucket's claim fits the pool at once; otherwise
    // one bucket after the other, each with the whole pool (a large batch
    // is bound by resident groups, a small one by its longest pairs)
    uint64_t claims = 0, largest = 0;
    for (const Launch& L : launches) {
        const uint64_t c = (L.blocks * L.gpb * L.slab_bytes + 255) / 256 * 256;
        claims += c;
        largest = std::max(largest, c);
    }
    const bool concurrent = claims <= pool_cap;
    uint64_t pool = 0;
    for (Launch& L : launches) {
        if (!concurrent) {
            L.blocks = std::max<uint64_t>(1, std::min<uint64_t>(L.blocks, pool_cap / (L.gpb * L.slab_bytes)));
            L.region = 0;
            pool = std::max<uint64_t>(pool, L.blocks * L.gpb * L.slab_bytes);
        } else {
            L.region = pool;
            pool += (L.blocks * L.gpb * L.slab_bytes + 255) / 256 * 256;
        }
    }
    if (pool > ws->slab.cap) {
        e = ws->slab.ensure(pool);
        if (e != hipSuccess) return buf_fail(ws, e, "the replay state slabs");
        ws->slab_clean = 0;
    }
    if (ws->slab_clean < ws->slab.cap) {
        PC_HIP(launch_fill_u32(ws->slab.as<uint32_t>(), ws->slab.cap / 4, 0, stream));
        ws->slab_clean = ws->slab.cap;
    }
    // descriptors up, and (split pairs merge into their outputs) those zeroed
    CopyFence fence(stream);
    PC_HIP(hipMemcpyAsync(d_models, dm.data(), dm.size() * sizeof(DevModel), hipMemcpyHostToDevice, stream));
    PC_HIP(hipMemcpyAsync(d_pairs, pairs.data(), pairs.size() * sizeof(StreamPair), hipMemcpyHostToDevice, stream));
    PC_HIP(launch_fill_u32(d_status, 128, 0, stream));
    if (gd) {
        PC_HIP(hipMemcpyAsync(sb + o_gen, gd->gen.data(), gd->gen.size() * sizeof(DevGeneral), hipMemcpyHostToDevice,
                              stream));
        PC_HIP(hipMemcpyAsync(sb + o_info, gd->set_info.data(), gd->set_info.size() * sizeof(uint2),
                              hipMemcpyHostToDevice, stream));
        if (!gd->table.empty())
            PC_HIP(hipMemcpyAsync(sb + o_table, gd->table.data(), gd->table.size() * sizeof(uint32_t),
                                  hipMemcpyHostToDevice, stream));
        if (!gd->cum.empty())
            PC_HIP(hipMemcpyAsync(sb + o_cum, gd->cum.data(), gd->cum.size() * sizeof(uint32_t), hipMemcpyHostToDevice,
                                  stream));
    }
    if (!zero_cnt.empty()) {
        uint64_t* d_zc = reinterpret_cast<uint64_t*>(sb + o_zero);
        uint64_t* d_zb = d_zc + zero_cnt.size();
        PC_HIP(hipMemcpyAsync(d_zc, zero_cnt.data(), zero_cnt.size() * 8, hipMemcpyHostToDevice, stream));
        PC_HIP(launch_clear_ranges(reinterpret_cast<uint32_t*>(misses_dev), d_zc, (uint32_t)(zero_cnt.size() / 2),
                                   stream));
        if (!zero_bits.empty()) {
            PC_HIP(hipMemcpyAsync(d_zb, zero_bits.data(), zero_bits.size() * 8, hipMemcpyHostToDevice, stream));
            PC_HIP(launch_clear_ranges(hitbits_dev, d_zb, (uint32_t)(zero_bits.size() / 2), stream));
        }
    }
    // longest buckets first; concurrently onto the least-loaded stream
    std::vector<size_t> order(launches.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = i;
    std::sort(order.begin(), order.end(), [&](size_t x, size_t y) { return launches[x].cost > launches[y].cost; });
    const int ns = concurrent ? (int)std::min<size_t>(kBranches, launches.size()) : 0;
    double load[kBranches] = {};
    if (ns > 1) PC_HIP(fork_branches(ws, stream, ns));
    for (size_t oi = 0; oi < order.size(); ++oi) {
        const Launch& L = launches[order[oi]];
        hipStream_t st = stream;
        if (ns > 1) {
            int b = 0;
            for (int c = 1; c < ns; ++c)
                if (load[c] < load[b]) b = c;
            load[b] += L.cost;
            st = branch_stream(ws, stream, b);
        }
        StreamArgs a;
        a.pairs = d_pairs + L.q;
        a.n_pairs = (uint32_t)(L.e2 - L.q);
        a.queue = d_status + 2 + order[oi];
        a.models = d_models;
        a.idx = idx_dev;
        a.misses = misses_dev;
        a.bits = hitbits_dev;
        a.slab = ws->slab.as<uint8_t>() + L.region;
        a.slab_bytes = L.slab_bytes;
        a.epoch_base = ws->epoch + (uint32_t)L.q;
        a.elem_shift = 2;
        a.abort_flag = abort_flag_dev();
        a.status = d_status;
        a.gen = d_gen;
        a.set_info = d_info;
        a.set_table = d_table;
        a.cum_w = d_cum;
        PC_HIP(launch_stream(L.pol, L.W, L.gen, a, (uint32_t)L.blocks, st));
    }
    if (ns > 1) PC_HIP(join_branches(ws, stream, ns));
    ws->epoch += (uint32_t)n_items + 1;
    PC_HIP(hipStreamSynchronize(stream));
    fence.done();
    uint32_t status = 0;
    PC_HIP(hipMemcpy(&status, d_status, sizeof status, hipMemcpyDeviceToHost));
    if (status & 1u) return set_error(PCHASE_EABORTED, "replay aborted by pchase_abort");
    if (status & 2u) return set_error(PCHASE_EINVAL, "a trace holds a negative element index");
    return PCHASE_OK;
}


// ----------------------------------------------------------- inference ---
static int build_infer_plan(Workspace* ws, const pchase_observation* obs, const pchase_model* cands,
                            uint32_t n_cands, const std::vector<DevModel>& dm, const std::vector<DevProbe>& dp,
                            const std::vector<uint64_t>& len, const std::vector<uint64_t>& cf,
                            const std::vector<uint64_t>& bitoff, int probe_select,
                            const std::vector<uint8_t>* allow, bool closed, std::unique_ptr<InferPlan>* out,
                            InferPlan* reuse = nullptr) {
    std::unique_ptr<InferPlan> np(new InferPlan());
    np->dev.arena = ws->arena;
    np->sweep.dev.arena = ws->arena;
    if (reuse && !ws->arena) {
        // take over the device buffers of a plan that is no longer needed
        std::swap(np->dev.p, reuse->dev.p);
        std::swap(np->dev.cap, reuse->dev.cap);
        std::swap(np->sweep.dev.p, reuse->sweep.dev.p);
        std::swap(np->sweep.dev.cap, reuse->sweep.dev.cap);
    }
    np->n_cands = n_cands;
    np->n_host.assign(n_cands, 0);
    std::vector<SweepJob> jobs;
    HugeVec<DecidedJob> decided;
    std::vector<RunTable> tables;
    std::vector<uint64_t> table_ks;   // first access of each sweep of the multi-sweep tables
    uint64_t entries = 0;
    std::vector<PlruPattern> patterns;
    std::map<std::pair<uint32_t, uint32_t>, uint32_t> pattern_of;   // (ways, lines) -> pattern, > 128 ways
    std::vector<int32_t> pattern_flat;                               // the same, up to 128 ways
    uint64_t pat_bits = 0, pat_scratch = 0;
    // own sweeps: probes indexed by stride, sorted by array size
    std::map<uint64_t, std::vector<std::pair<uint64_t, uint32_t>>> by_stride;
    if (probe_select == PCHASE_PROBES_OWN_SWEEP) {
        for (uint32_t p = 0; p < obs->n_probes; ++p)
            by_stride[obs->probes[p].s_bytes].push_back({obs->probes[p].n_bytes, p});
        for (auto& kv : by_stride) std::sort(kv.second.begin(), kv.second.end());
    }
    // sweep geometry per (probe, line shift), computed once
    struct Geo {
        uint64_t U = 0, d = 1;
        uint32_t ks_off = 0, nsw = 0;
        int32_t table = -1;   // its run table, once one is built
        bool done = false;
    };
    // indexed by (probe, the candidates' distinct line shifts)
    std::vector<int32_t> ls_slot(64, -1);
    uint32_t n_ls = 0;
    for (uint32_t c = 0; c < n_cands; ++c)
        if (ls_slot[dm[c].line_shift] < 0) ls_slot[dm[c].line_shift] = (int32_t)n_ls++;
    std::vector<Geo> geo;
    std::vector<uint64_t> geo_ks;
    // the (candidate, probe) pairs first, so that the job arrays are sized once
    std::vector<uint64_t> pair_off(n_cands + 1, 0);
    std::vector<uint32_t> pairs;
    for (uint32_t c = 0; c < n_cands; ++c) {
        pair_off[c] = pairs.size();
        if (allow && !(*allow)[c]) continue;
        if (probe_select == PCHASE_PROBES_OWN_SWEEP) {
            const size_t first = pairs.size();
            const uint64_t C = cands[c].capacity_bytes, b = cands[c].line_bytes;
            const uint64_t strides[3] = {b / 2, b, 2 * b};
            for (int si = 0; si < 3; ++si) {
                if (si == 0 && (b & 1)) continue;   // no half-line stride
                auto it = by_stride.find(strides[si]);
                if (it == by_stride.end()) continue;
                const auto& v = it->second;
                auto lo = std::lower_bound(v.begin(), v.end(), std::make_pair((C + 1) / 2, 0u));
                for (; lo != v.end() && lo->first <= 2 * C; ++lo)
                    if (own_sweep(cands[c], obs->probes[lo->second])) pairs.push_back(lo->second);
            }
            std::sort(pairs.begin() + first, pairs.end());
        } else {
            for (uint32_t p = 0; p < obs->n_probes; ++p) pairs.push_back(p);
        }
    }
    pair_off[n_cands] = pairs.size();
    if (closed) decided.reserve(pairs.size());
    else jobs.reserve(pairs.size());
    for (uint32_t c = 0; c < n_cands; ++c) {
        const DevModel& md = dm[c];
        // the closed forms hold for LRU and FIFO; with one way every policy
        // replaces as LRU does, and two-way tree-PLRU is LRU
        const bool lru_fifo = md.policy == PCHASE_LRU || md.policy == PCHASE_FIFO || md.ways == 1 ||
                              (md.ways == 2 && md.policy == PCHASE_PLRU);
        for (uint64_t pi = pair_off[c]; pi < pair_off[c + 1]; ++pi) {
            const uint32_t p = pairs[pi];
            if (len[p] > cf[p]) np->n_host[c] += len[p] - cf[p];
            // no access evicts and nothing before the second pass is
            // compared: the only misses are first touches, all in the first
            // pass, so the score is the observed misses alone
            if (closed && cf[p] >= dp[p].L && no_eviction(md, dp[p])) {
                decided.push_back(DecidedJob{p, 0, 0, 0, 1, c, 0, 0, 0});   // slot set below
                np->decided_accesses += len[p];
                continue;
            }
            // single-sweep passes over an arithmetic progression of lines
            // (one line per set-mapping unit): run i of a pass lies in set
            // (l0 + i d) mod T, so runs i and i + T' (T' = T / gcd(d, T))
            // share a set and the runs of one period are in distinct sets;
            // a visited set holds q0 or q0 + 1 lines (the latter for
            // i mod T' < r, with U runs = q0 T' + r)
            // (several sweeps that visit every line of a range once: the
            // runs in line order, d = 1)
            uint64_t d = 1, U = 0;
            uint32_t nsw = 0, ks_off = 0;
            if (closed && md.unit_shift == md.line_shift) {
                if (geo.empty()) geo.resize((size_t)obs->n_probes * n_ls);
                Geo& gg = geo[(size_t)p * n_ls + (uint32_t)ls_slot[md.line_shift]];
                if (!gg.done) {
                    gg.done = true;
                    gg.U = sweep_runs(dp[p], md.line_shift, &gg.d);
                    if (!gg.U) {
                        std::vector<uint64_t> ks;
                        gg.U = multi_sweep_runs(dp[p], md.line_shift, &ks);
                        if (gg.U) {
                            gg.ks_off = (uint32_t)geo_ks.size();
                            gg.nsw = (uint32_t)ks.size();
                            geo_ks.insert(geo_ks.end(), ks.begin(), ks.end());
                        }
                    }
                }
                U = gg.U;
                d = gg.d;
                nsw = gg.nsw;
                ks_off = gg.ks_off;
            }
            if (U) {
                const uint64_t Tp = md.sets / gcd64(d % md.sets, md.sets);
                const uint64_t q0 = U / Tp, r = U % Tp;
                const bool none = q0 + (r ? 1 : 0) <= md.ways;   // no eviction
                // tree-PLRU: per-(a, n) second-pass patterns, for two-pass
                // chases that visit each set's lines in line order (one
                // sweep; or sweeps of stride nsw lines with nsw dividing T,
                // so that a set's lines all lie in one sweep)
                const bool plru_pat = md.policy == PCHASE_PLRU && dp[p].passes == 2 &&
                                      (nsw == 0 || md.sets % nsw == 0) && q0 + 1 <= kMaxPatternLines;
                const int kind = none ? (cf[p] >= dp[p].L ? 0 : 1)
                                 : lru_fifo ? (q0 > md.ways ? 2 : 3) : plru_pat ? 4 : -1;
                uint32_t tid = 0, pb = 0, ps = 0;
                if (kind == 4) {
                    auto pattern = [&](uint32_t n) -> uint32_t {
                        // ids of (ways, n) in a flat table for up to 128 ways
                        int32_t* slot = nullptr;
                        if (md.ways <= kPatternTableWays) {
                            if (pattern_flat.empty())
                                pattern_flat.assign((kPatternTableWays + 1) * (kMaxPatternLines + 2), -1);
                            slot = &pattern_flat[(size_t)md.ways * (kMaxPatternLines + 2) + n];
                            if (*slot >= 0) return (uint32_t)*slot;
                        } else {
                            auto it = pattern_of.find(std::make_pair(md.ways, n));
                            if (it != pattern_of.end()) return it->second;
                        }
                        const uint32_t id = (uint32_t)patterns.size();
                        patterns.push_back(PlruPattern{md.ways, md.log2_ways, n, (uint32_t)pat_scratch, pat_bits});
                        pat_scratch += n + md.ways;
                        pat_bits += (n + 31) / 32 * 32;
                        if (slot) *slot = (int32_t)id;
                        else pattern_of.emplace(std::make_pair(md.ways, n), id);
                        return id;
                    };
                    ps = pattern((uint32_t)q0);
                    pb = r ? pattern((uint32_t)q0 + 1) : ps;
                }
                bool ok = kind >= 0;
                if (kind >= 1) {
                    Geo& gg = geo[(size_t)p * n_ls + (uint32_t)ls_slot[md.line_shift]];
                    if (gg.table >= 0) {
                        tid = (uint32_t)gg.table;
                    } else if (entries + U + 1 <= kMaxTableEntries &&
                               U * (uint64_t)(dp[p].passes - 1) < (1ull << 31)) {
                        tid = (uint32_t)tables.size();
                        tables.push_back(RunTable{p, md.line_shift, U, entries, nsw, 0, (uint64_t)table_ks.size()});
                        table_ks.insert(table_ks.end(), geo_ks.begin() + ks_off, geo_ks.begin() + ks_off + nsw);
                        gg.table = (int32_t)tid;
                        entries += U + 1;
                    } else {
                        ok = false;
                    }
                }
                if (ok) {
                    decided.push_back(DecidedJob{p, tid, (uint32_t)kind, (uint32_t)r, Tp, c, pb, ps, 0});
                    np->decided_accesses += len[p];
                    continue;
                }
            }
            SweepJob j;
            j.model = c;
            j.probe = p;
            j.out = c;
            j.trace_id = p;
            j.count_from = cf[p];
            j.bitoff = bitoff[p];
            j.bm_off = 0;
            j.cyc = closed && lru_fifo && lines_once_per_pass(dp[p], md.line_shift) ? 1u : 0u;
            if (j.cyc) np->cyc_accesses += len[p];
            jobs.push_back(j);
        }
    }
    int rc = build_sweep_plan(&np->sweep, dm, dp, len, jobs, false, false);
    if (rc) return rc;
    const size_t zw = (n_cands + 31) / 32;
    const uint32_t n_probes = (uint32_t)obs->n_probes;
    auto up256 = [](size_t x) { return (x + 255) / 256 * 256; };
    // what the host writes first, as one image uploaded in one copy; then
    // what the kernels write
    const size_t o_n = 0;
    const size_t o_pinfo = up256(o_n + n_cands * sizeof(uint64_t));
    const size_t o_dec = up256(o_pinfo + 3 * (size_t)n_probes * sizeof(uint64_t));
    const size_t o_dcand = up256(o_dec + decided.size() * sizeof(DecidedJob));
    const size_t o_tab = up256(o_dcand + decided.size() * sizeof(uint32_t));
    const size_t o_ks = up256(o_tab + tables.size() * sizeof(RunTable));
    const size_t o_pat = up256(o_ks + table_ks.size() * sizeof(uint64_t));
    const size_t o_img = o_pat + patterns.size() * sizeof(PlruPattern);
    const size_t o_m = up256(o_img);
    const size_t o_zero = o_m + n_cands * sizeof(uint64_t);
    const size_t o_out = up256(o_zero + zw * 4);
    const size_t o_zeros = up256(o_out + sizeof(ArgminOut));
    const size_t o_dval = up256(o_zeros + (size_t)n_probes * sizeof(uint64_t));
    const size_t o_s1 = up256(o_dval + decided.size() * sizeof(int64_t));
    const size_t o_pbits = up256(o_s1 + tables.size() * sizeof(int64_t));
    const size_t o_pscr = up256(o_pbits + pat_bits / 8);
    const size_t o_pre = up256(o_pscr + pat_scratch * sizeof(uint32_t));
    const size_t bytes = o_pre + entries * sizeof(int32_t);
    HostImage img(o_img);
    if (o_img && !img.p) return set_error(PCHASE_ENOMEM, "host image of %zu bytes", o_img);
    auto put = [&](size_t at, const void* src, size_t n) {
        if (n) std::memcpy(img.p + at, src, n);
    };
    // the alignment gaps between the regions (the regions are all written)
    const size_t region[8][2] = {{o_n, n_cands * sizeof(uint64_t)},
                                 {o_pinfo, 3 * (size_t)n_probes * sizeof(uint64_t)},
                                 {o_dec, decided.size() * sizeof(DecidedJob)},
                                 {o_dcand, decided.size() * sizeof(uint32_t)},
                                 {o_tab, tables.size() * sizeof(RunTable)},
                                 {o_ks, table_ks.size() * sizeof(uint64_t)},
                                 {o_pat, patterns.size() * sizeof(PlruPattern)},
                                 {o_img, 0}};
    for (int r = 0; r < 7; ++r) {
        const size_t end = region[r][0] + region[r][1];
        if (region[r + 1][0] > end) std::memset(img.p + end, 0, region[r + 1][0] - end);
    }
    put(o_n, np->n_host.data(), n_cands * sizeof(uint64_t));
    for (uint32_t p = 0; p < n_probes; ++p) {
        const uint64_t row[3] = {bitoff[p], std::min(cf[p], len[p]), len[p]};
        put(o_pinfo + 3 * (size_t)p * sizeof(uint64_t), row, sizeof row);
    }
    // jobs in table order for the gathers (a stable counting sort), slots in
    // candidate order for the sums
    {
        std::vector<uint32_t> cnt(tables.size() + 2, 0);
        for (const DecidedJob& x : decided) ++cnt[x.table + 1];
        for (size_t t = 1; t < cnt.size(); ++t) cnt[t] += cnt[t - 1];
        for (size_t q = 0; q < decided.size(); ++q) {
            DecidedJob x = decided[q];
            x.slot = (uint32_t)q;
            put(o_dcand + q * sizeof(uint32_t), &x.cand, sizeof(uint32_t));
            put(o_dec + (size_t)cnt[x.table]++ * sizeof(DecidedJob), &x, sizeof x);
        }
    }
    put(o_tab, tables.data(), tables.size() * sizeof(RunTable));
    put(o_ks, table_ks.data(), table_ks.size() * sizeof(uint64_t));
    put(o_pat, patterns.data(), patterns.size() * sizeof(PlruPattern));
    hipError_t e = np->dev.ensure(bytes);
    if (e != hipSuccess) return buf_fail(ws, e, "the inference scores");
    uint8_t* b = np->dev.as<uint8_t>();
    np->d_m = reinterpret_cast<uint64_t*>(b + o_m);
    np->d_n = reinterpret_cast<uint64_t*>(b + o_n);
    np->d_zero = reinterpret_cast<uint32_t*>(b + o_zero);
    np->d_out = reinterpret_cast<ArgminOut*>(b + o_out);
    np->d_pinfo = reinterpret_cast<uint64_t*>(b + o_pinfo);
    np->d_zeros = reinterpret_cast<uint64_t*>(b + o_zeros);
    np->n_probes = n_probes;
    np->sweep.zeros = np->d_zeros;
    np->d_decided = reinterpret_cast<DecidedJob*>(b + o_dec);
    np->d_dec_vals = reinterpret_cast<int64_t*>(b + o_dval);
    np->d_dec_cand = reinterpret_cast<uint32_t*>(b + o_dcand);
    np->d_tables = reinterpret_cast<RunTable*>(b + o_tab);
    np->d_s1 = reinterpret_cast<int64_t*>(b + o_s1);
    np->d_prefix = reinterpret_cast<int32_t*>(b + o_pre);
    np->d_table_ks = reinterpret_cast<uint64_t*>(b + o_ks);
    np->d_patterns = reinterpret_cast<PlruPattern*>(b + o_pat);
    np->d_pat_bits = reinterpret_cast<uint32_t*>(b + o_pbits);
    np->n_tables = (uint32_t)tables.size();
    np->n_decided = (uint32_t)decided.size();
    if (o_img) PC_HIP(hipMemcpy(b, img.p, o_img, hipMemcpyHostToDevice));
    if (!patterns.empty()) {
        // the patterns depend on the plan only: computed once, here
        PC_HIP(launch_plru_patterns(np->d_patterns, (uint32_t)patterns.size(), np->d_pat_bits,
                                    reinterpret_cast<uint32_t*>(b + o_pscr), nullptr));
        PC_HIP(hipStreamSynchronize(nullptr));
    }
    *out = std::move(np);
    return PCHASE_OK;
}

// The exact inputs that shape an inference plan, as bytes: a cached plan is
// used only when its stored inputs equal these (the digest only finds it).
static std::string infer_key(const pchase_observation* obs, const pchase_model* cands, uint32_t n_cands,
                             int probe_select, const uint64_t* bitoff, const std::vector<uint8_t>* allow,
                             bool closed) {
    std::string k;
    auto put = [&](const void* p, size_t n) { k.append(static_cast<const char*>(p), n); };
    k.push_back(closed ? 'c' : 'r');
    put(&n_cands, sizeof n_cands);
    put(&obs->n_probes, sizeof obs->n_probes);
    put(&probe_select, sizeof probe_select);
    const uint8_t has_cf = obs->count_from != nullptr, has_allow = allow != nullptr;
    put(&has_cf, 1);
    put(&has_allow, 1);
    put(cands, n_cands * sizeof(pchase_model));
    put(obs->probes, obs->n_probes * sizeof(pchase_probe));
    if (has_cf) put(obs->count_from, obs->n_probes * sizeof(uint64_t));
    put(bitoff, obs->n_probes * sizeof(uint64_t));
    if (has_allow) put(allow->data(), allow->size());
    return k;
}

// Whether `k` (an infer_key) holds exactly these inputs, compared in place
// (no key is built: the repeated call's lookup reads the inputs once).
static bool infer_key_equals(const std::string& k, const pchase_observation* obs, const pchase_model* cands,
                             uint32_t n_cands, int probe_select, const uint64_t* bitoff, bool closed) {
    size_t at = 0;
    auto eq = [&](const void* p, size_t n) {
        if (at + n > k.size() || std::memcmp(k.data() + at, p, n) != 0) return false;
        at += n;
        return true;
    };
    const char tag = closed ? 'c' : 'r';
    const uint8_t has_cf = obs->count_from != nullptr, has_allow = 0;
    const size_t np = obs->n_probes;
    return eq(&tag, 1) && eq(&n_cands, sizeof n_cands) && eq(&obs->n_probes, sizeof obs->n_probes) &&
           eq(&probe_select, sizeof probe_select) && eq(&has_cf, 1) && eq(&has_allow, 1) &&
           eq(cands, n_cands * sizeof(pchase_model)) && eq(obs->probes, np * sizeof(pchase_probe)) &&
           (!has_cf || eq(obs->count_from, np * sizeof(uint64_t))) && eq(bitoff, np * sizeof(uint64_t)) &&
           at == k.size();
}

static std::string digest_of(const std::string& blob) {
    Digest dg;
    dg.add(blob.data(), blob.size());
    return dg.str();
}

// Runs a built plan and reads its result back (synchronises).
static int run_infer_plan(Workspace* ws, InferPlan* ip, const uint32_t* bits, pchase_result* out, uint64_t* mn_dev,
                          uint32_t* zero_host, hipStream_t stream, uint64_t* replayed, uint32_t sched,
                          bool tune = true);

// cache = false builds a one-off plan (the learned path's top-k subsets)
static int infer_exhaustive(Workspace* ws, const pchase_observation* obs, const pchase_model* cands,
                            uint32_t n_cands, const std::vector<DevModel>& dm, const std::vector<DevProbe>& dp,
                            const std::vector<uint64_t>& len, const std::vector<uint64_t>& cf,
                            const std::vector<uint64_t>& bitoff, const uint32_t* bits, int probe_select,
                            const std::vector<uint8_t>* allow, pchase_result* out, uint64_t* mn_dev,
                            uint32_t* zero_host, hipStream_t stream, uint64_t* replayed, uint32_t sched,
                            bool closed, bool cache = true, bool tune = true) {
    InferPlan* ip;
    if (!cache) {
        std::unique_ptr<InferPlan> once, prev = std::move(ws->oneoff);
        int rc = build_infer_plan(ws, obs, cands, n_cands, dm, dp, len, cf, bitoff, probe_select, allow, closed,
                                  &once, prev.get());
        if (rc) return rc;
        prev.reset();
        ws->oneoff = std::move(once);
        ip = ws->oneoff.get();
    } else {
        std::string blob = infer_key(obs, cands, n_cands, probe_select, bitoff.data(), allow, closed);
        const std::string key = digest_of(blob);
        auto it = ws->plans.find(key);
        if (it == ws->plans.end() || it->second->key != blob) {
            std::unique_ptr<InferPlan> np;
            int rc = build_infer_plan(ws, obs, cands, n_cands, dm, dp, len, cf, bitoff, probe_select, allow, closed,
                                      &np);
            if (rc) return rc;
            np->key = std::move(blob);
            np->cached = true;
            if (ws->plans.size() > 16) ws->plans.clear();
            ip = np.get();
            ws->plans[key] = std::move(np);
        } else {
            ip = it->second.get();
        }
    }
    return run_infer_plan(ws, ip, bits, out, mn_dev, zero_host, stream, replayed, sched, tune);
}

static int run_infer_plan(Workspace* ws, InferPlan* ip, const uint32_t* bits, pchase_result* out, uint64_t* mn_dev,
                          uint32_t* zero_host, hipStream_t stream, uint64_t* replayed, uint32_t sched, bool tune) {
    const uint32_t n_cands = ip->n_cands;
    const size_t zw = (n_cands + 31) / 32;
    InferPlan* pp = ip;
    auto tail = [pp](hipStream_t s) -> hipError_t {
        return launch_argmin(pp->d_m, pp->d_n, pp->n_cands, pp->d_zero, pp->d_out, s);
    };
    // the jobs decided without a replay, beside the replay: their run
    // tables, then their scores into the cleared counters
    auto side = [pp, bits](hipStream_t s) -> hipError_t {
        hipError_t e = launch_run_tables(pp->d_tables, pp->n_tables, pp->sweep.d_probes, pp->d_table_ks, pp->d_pinfo,
                                         bits, pp->d_prefix, pp->d_s1, s);
        if (e != hipSuccess) return e;
        return launch_decided(pp->d_decided, pp->n_decided, pp->d_zeros, pp->d_tables, pp->d_prefix, pp->d_s1,
                              pp->d_patterns, pp->d_pat_bits, pp->d_dec_vals, pp->d_dec_cand, pp->d_m, s);
    };
    const bool has_side = ip->n_decided != 0;
    // the observed misses of each probe, the constant part of every score
    PC_HIP(launch_obs_zeros(bits, ip->d_pinfo, ip->n_probes, ip->d_zeros, stream));
    // the first run of a cached plan answers at once with the default branch
    // strategy; the next run times the strategies and keeps the fastest
    int rc = run_sweep_plan(ws, &ip->sweep, true, ip->d_m, n_cands, const_cast<uint32_t*>(bits), false,
                            sched, stream, tail, ip->cached && tune, ip->runs == 0,
                            has_side ? std::function<hipError_t(hipStream_t)>(side)
                                     : std::function<hipError_t(hipStream_t)>());
    if (rc) return rc;
    ArgminOut* hr = static_cast<ArgminOut*>(ws->host_res);
    PC_HIP(hipMemcpyAsync(hr, ip->d_out, sizeof(ArgminOut), hipMemcpyDeviceToHost, stream));
    if (zero_host) PC_HIP(hipMemcpyAsync(static_cast<uint8_t*>(ws->host_res) + 256, ip->d_zero, zw * 4,
                                         hipMemcpyDeviceToHost, stream));
    if (mn_dev) {
        PC_HIP(hipMemcpy2DAsync(mn_dev, 16, ip->d_m, 8, 8, n_cands, hipMemcpyDeviceToDevice, stream));
        PC_HIP(hipMemcpy2DAsync(mn_dev + 1, 16, ip->d_n, 8, 8, n_cands, hipMemcpyDeviceToDevice, stream));
    }
    uint32_t* hs = reinterpret_cast<uint32_t*>(static_cast<uint8_t*>(ws->host_res) + kHostStatus);
    PC_HIP(hipMemcpyAsync(hs, ip->sweep.d_queues + ip->sweep.batched.size(), sizeof(uint32_t), hipMemcpyDeviceToHost,
                          stream));
    PC_HIP(hipStreamSynchronize(stream));
    if (*hs & 1u) return set_error(PCHASE_EABORTED, "inference aborted by pchase_abort");
    out->best = hr->best;
    out->best_m = hr->m;
    out->best_n = hr->n;
    out->n_zero = hr->n_zero;
    if (zero_host && zw * 4 <= 4096 - 256) std::memcpy(zero_host, static_cast<uint8_t*>(ws->host_res) + 256, zw * 4);
    *replayed = ip->sweep.accesses + ip->decided_accesses;
    out->closed_form_accesses += ip->decided_accesses + ip->cyc_accesses;
    ++ip->runs;
    return PCHASE_OK;
}


// Layout of an observation's hit bits (Section 4.2, steps 3-4): probe p's
// bits at word bitoff[p] of bits_dev as given, or, for latencies, packed
// back to back (words in total) in the bitmap observation_bits writes;
// cf[p] = the first access compared (one cycle L unless given).
static int observation_layout(const pchase_observation* obs, const std::vector<DevProbe>& dp,
                              const std::vector<uint64_t>& len, std::vector<uint64_t>* cf_out,
                              std::vector<uint64_t>* bitoff_out, uint64_t* words_out, uint64_t* maxlen_out) {
    const bool have_bits = obs->bits_dev != nullptr, have_lat = obs->lat_dev != nullptr;
    if (have_bits == have_lat) return set_error(PCHASE_EINVAL, "give exactly one of bits_dev and lat_dev");
    if (have_bits && !obs->bitoff) return set_error(PCHASE_EINVAL, "bits_dev needs bitoff");
    if (have_lat && !obs->lat_off) return set_error(PCHASE_EINVAL, "lat_dev needs lat_off");
    std::vector<uint64_t>& cf = *cf_out;
    std::vector<uint64_t>& bitoff = *bitoff_out;
    cf.assign(obs->n_probes, 0);
    bitoff.assign(obs->n_probes, 0);
    uint64_t words = 0, maxlen = 0;
    for (uint32_t p = 0; p < obs->n_probes; ++p) {
        cf[p] = obs->count_from ? obs->count_from[p] : dp[p].L;
        maxlen = std::max(maxlen, len[p]);
        if (have_bits) {
            bitoff[p] = obs->bitoff[p];
        } else {
            if (obs->lat_off[p + 1] - obs->lat_off[p] != len[p])
                return set_error(PCHASE_EINVAL, "probe %u: %llu latencies for a trace of %llu accesses", p,
                                 (unsigned long long)(obs->lat_off[p + 1] - obs->lat_off[p]),
                                 (unsigned long long)len[p]);
            bitoff[p] = words;
            words += (len[p] + 31) / 32;
        }
    }
    *words_out = words;
    *maxlen_out = maxlen;
    return PCHASE_OK;
}

// The observation's hit bits on the device: bits_dev as given, or the
// latencies classified (the given threshold, or the widest gap) into
// ws->obs.  *threshold_used = the threshold applied (0xFFFFFFFF for bits).
static int observation_bits(Workspace* ws, const pchase_observation* obs, const std::vector<uint64_t>& bitoff,
                            uint64_t words, uint64_t maxlen, const uint32_t** bits_out, uint32_t* threshold_used,
                            hipStream_t stream) {
    const uint32_t* bits = obs->bits_dev;
    *threshold_used = 0xFFFFFFFFu;
    if (!obs->bits_dev) {
        // latency -> hit bits on the device
        const uint64_t n_lat = obs->lat_off[obs->n_probes] - obs->lat_off[0];
        const size_t o_bits = 0;
        const size_t o_off = (words * 4 + 255) / 256 * 256;
        const size_t o_mm = o_off + ((2 * (size_t)obs->n_probes + 1) * 8 + 255) / 256 * 256;
        const size_t o_present = o_mm + 256;
        const uint64_t present_words = (1ull << 26) / 32;
        size_t total = o_present + (obs->threshold == 0xFFFFFFFFu ? present_words * 4 : 0);
        hipError_t e = ws->obs.ensure(total);
        if (e != hipSuccess) return buf_fail(ws, e, "the observed bits");
        uint8_t* b = ws->obs.as<uint8_t>();
        uint32_t* d_bits = reinterpret_cast<uint32_t*>(b + o_bits);
        uint64_t* d_latoff = reinterpret_cast<uint64_t*>(b + o_off);
        uint64_t* d_bitoff = d_latoff + obs->n_probes + 1;
        uint32_t* d_mm = reinterpret_cast<uint32_t*>(b + o_mm);
        uint32_t mm_init[4] = {0xFFFFFFFFu, 0u, obs->threshold, 0u};
        uint32_t mmh[3] = {}, th = 0;   // copy targets live as long as the fence
        CopyFence fence(stream);
        PC_HIP(hipMemcpyAsync(d_latoff, obs->lat_off, (obs->n_probes + 1) * 8, hipMemcpyHostToDevice, stream));
        PC_HIP(hipMemcpyAsync(d_bitoff, bitoff.data(), obs->n_probes * 8, hipMemcpyHostToDevice, stream));
        PC_HIP(hipMemcpyAsync(d_mm, mm_init, sizeof mm_init, hipMemcpyHostToDevice, stream));
        if (obs->threshold == 0xFFFFFFFFu) {
            PC_HIP(launch_fill_u32(reinterpret_cast<uint32_t*>(b + o_present), present_words, 0, stream));
            // the presence bitmap covers 2^26 distinct values above the minimum
            PC_HIP(launch_auto_threshold(obs->lat_dev + obs->lat_off[0], n_lat, d_mm,
                                         reinterpret_cast<uint32_t*>(b + o_present), present_words * 32,
                                         d_mm + 2, stream));
            PC_HIP(hipMemcpyAsync(mmh, d_mm, sizeof mmh, hipMemcpyDeviceToHost, stream));
            PC_HIP(hipStreamSynchronize(stream));
            if ((uint64_t)mmh[1] - mmh[0] >= present_words * 32 || mmh[2] == 0xFFFFFFFFu)
                return set_error(PCHASE_ERANGE, "latency range %u..%u too wide for the automatic threshold", mmh[0], mmh[1]);
        }
        PC_HIP(launch_classify(obs->lat_dev, d_latoff, d_bitoff, obs->n_probes, maxlen, d_mm + 2, d_bits, stream));
        PC_HIP(hipMemcpyAsync(&th, d_mm + 2, 4, hipMemcpyDeviceToHost, stream));
        PC_HIP(hipStreamSynchronize(stream));
        fence.done();
        *threshold_used = th;
        bits = d_bits;
    }
    *bits_out = bits;
    return PCHASE_OK;
}

extern "C" int infer_cache_params(const pchase_observation* obs, const pchase_model* cands, uint32_t n_cands,
                                  int probe_select, int mode, uint32_t topk, const pchase_mlp* net,
                                  pchase_result* out, uint64_t* mn_dev, uint32_t* zero_host, pchase_plan* plan,
                                  hipStream_t stream) {
    if (!obs || !out) return set_error(PCHASE_EINVAL, "obs and out must not be NULL");
    if (probe_select != PCHASE_PROBES_ALL && probe_select != PCHASE_PROBES_OWN_SWEEP)
        return set_error(PCHASE_EINVAL, "unknown probe_select %d", probe_select);
    const uint32_t sched = (mode & PCHASE_SCHED_PLAIN) ? PCHASE_PLAIN : PCHASE_BATCHED;
    const bool tune = !(mode & PCHASE_SCHED_UNTUNED);
    const bool closed = !(mode & PCHASE_SCHED_FULL_REPLAY);
    mode &= ~(PCHASE_SCHED_PLAIN | PCHASE_SCHED_UNTUNED | PCHASE_SCHED_FULL_REPLAY);
    if (mode != PCHASE_EXHAUSTIVE && mode != PCHASE_LEARNED) return set_error(PCHASE_EINVAL, "unknown mode %d", mode);
    if (mode == PCHASE_LEARNED && (!net || topk == 0)) return set_error(PCHASE_EINVAL, "LEARNED needs a network and topk >= 1");
    if (n_cands == 0) return set_error(PCHASE_EINVAL, "no candidates");
    if (zero_host && (n_cands + 31) / 32 * 4 > 4096 - 256) return set_error(PCHASE_ERANGE, "zero-class bitmap too large");
    out->closed_form_accesses = 0;
    if (mode == PCHASE_EXHAUSTIVE && obs->bits_dev && !obs->lat_dev && obs->bitoff && obs->probes && obs->n_probes) {
        // repeated inference on the same inputs: the cached plan (built, and
        // so validated, for exactly these inputs) runs without re-validation
        Workspace* ws;
        std::unique_lock<std::mutex> lk;
        int rc = workspace_for(plan, &ws, &lk);
        if (rc) return rc;
        for (auto& kv : ws->plans) {
            if (!infer_key_equals(kv.second->key, obs, cands, n_cands, probe_select, obs->bitoff, closed)) continue;
            out->threshold_used = 0xFFFFFFFFu;
            out->fallback = 0;
            uint64_t replayed = 0;
            rc = run_infer_plan(ws, kv.second.get(), obs->bits_dev, out, mn_dev, zero_host, stream, &replayed, sched,
                                tune);
            out->replayed_accesses = replayed;
            return rc;
        }
    }
    std::vector<DevModel> dm;
    std::vector<DevProbe> dp;
    std::vector<uint64_t> len;
    int rc = validate_models(cands, n_cands, &dm);
    if (rc) return rc;
    rc = validate_probes(obs->probes, obs->n_probes, &dp, &len);
    if (rc) return rc;
    if (obs->n_probes == 0) return set_error(PCHASE_EINVAL, "no observed probes");
    std::vector<uint64_t> cf, bitoff;
    uint64_t words = 0, maxlen = 0;
    rc = observation_layout(obs, dp, len, &cf, &bitoff, &words, &maxlen);
    if (rc) return rc;
    Workspace* ws;
    std::unique_lock<std::mutex> lk;
    rc = workspace_for(plan, &ws, &lk);
    if (rc) return rc;
    ws->reset_arena();   // a plan serves one inference problem at a time
    const uint32_t* bits = nullptr;
    rc = observation_bits(ws, obs, bitoff, words, maxlen, &bits, &out->threshold_used, stream);
    if (rc) return rc;

    out->fallback = 0;
    uint64_t replayed = 0;
    if (mode == PCHASE_LEARNED) {
        std::vector<uint8_t> allow;
        bool on_grid = false;
        rc = infer_learned(ws, obs, cands, n_cands, dp, len, cf, bitoff, bits, topk, net, &allow, &on_grid, stream);
        if (rc) return rc;
        if (on_grid) {
            // confirm the proposals exactly: one-off plan, eager launches
            rc = infer_exhaustive(ws, obs, cands, n_cands, dm, dp, len, cf, bitoff, bits, probe_select, &allow, out,
                                  nullptr, nullptr, stream, &replayed, PCHASE_PLAIN, closed, false);
            if (rc) return rc;
            out->replayed_accesses = replayed;
            if (out->best >= 0 && out->best_m == 0) return PCHASE_OK;
            out->fallback = 1;
        } else {
            out->fallback = 2;
        }
    }
    rc = infer_exhaustive(ws, obs, cands, n_cands, dm, dp, len, cf, bitoff, bits, probe_select, nullptr, out, mn_dev,
                          zero_host, stream, &replayed, sched, closed, true, tune);
    if (rc) return rc;
    out->replayed_accesses += replayed;
    if (mode == PCHASE_EXHAUSTIVE) out->replayed_accesses = replayed;
    return PCHASE_OK;
}

// ------------------------------------------- generalised-candidate search --
// Sections 4.3-4.5 widen the candidates beyond (C, b, a, policy): per-set
// associativity, set tables, shifted set mappings, weighted replacement.
// Such a candidate has no closed-form trace per set, so each observed probe
// is materialised once and every (candidate, probe) pair replayed through
// the generalised engine into a hit bitmap, which one wave per pair then
// compares with the observation (step (iv) of Section 4.2).
extern "C" int infer_cache_params_general(const pchase_observation* obs, const pchase_general_model* cands,
                                          uint32_t n_cands, pchase_result* out, uint64_t* mn_dev,
                                          uint32_t* zero_host, pchase_plan* plan, hipStream_t stream) {
    if (!obs || !out) return set_error(PCHASE_EINVAL, "obs and out must not be NULL");
    if (n_cands == 0) return set_error(PCHASE_EINVAL, "no candidates");
    if (zero_host && (n_cands + 31) / 32 * 4 > 4096 - 256) return set_error(PCHASE_ERANGE, "zero-class bitmap too large");
    std::vector<DevModel> dm;
    GeneralDesc gd;
    int rc = build_general(cands, n_cands, &dm, &gd);
    if (rc) return rc;
    std::vector<DevProbe> dp;
    std::vector<uint64_t> len;
    rc = validate_probes(obs->probes, obs->n_probes, &dp, &len);
    if (rc) return rc;
    if (obs->n_probes == 0) return set_error(PCHASE_EINVAL, "no observed probes");
    std::vector<uint64_t> cf, obits;
    uint64_t words = 0, maxlen = 0;
    rc = observation_layout(obs, dp, len, &cf, &obits, &words, &maxlen);
    if (rc) return rc;
    const uint32_t np = obs->n_probes;
    const uint64_t n_pairs = (uint64_t)n_cands * np;
    if (n_pairs >= (1ull << 32)) return set_error(PCHASE_ERANGE, "too many (candidate, probe) pairs");
    // traces back to back; hit words of one candidate: every probe's, word aligned
    std::vector<uint64_t> toff(np + 1, 0), hoff(np), base(np), n_cmp(n_cands, 0);
    uint64_t cand_words = 0, compared = 0;
    for (uint32_t p = 0; p < np; ++p) {
        toff[p + 1] = toff[p] + len[p];
        hoff[p] = cand_words;
        cand_words += (len[p] + 31) / 32;
        base[p] = obs->probes[p].base_offset;
        compared += len[p] > cf[p] ? len[p] - cf[p] : 0;
    }
    for (uint32_t c = 0; c < n_cands; ++c) n_cmp[c] = compared;
    const uint64_t hit_bytes = (uint64_t)n_cands * cand_words * 4;
    if (toff[np] >= (1ull << 34) || hit_bytes >= (32ull << 30))
        return set_error(PCHASE_ERANGE, "the search needs %llu accesses and %llu bytes of hit bits",
                         (unsigned long long)toff[np], (unsigned long long)hit_bytes);
    std::vector<uint32_t> pm(n_pairs), pt(n_pairs);
    std::vector<uint64_t> pcf(n_pairs), pbit(n_pairs);
    for (uint64_t i = 0; i < n_pairs; ++i) {
        const uint32_t c = (uint32_t)(i / np), p = (uint32_t)(i % np);
        pm[i] = c;
        pt[i] = p;
        pcf[i] = cf[p];
        pbit[i] = (uint64_t)c * cand_words + hoff[p];
    }

    Workspace* ws;
    std::unique_lock<std::mutex> lk;
    rc = workspace_for(plan, &ws, &lk);
    if (rc) return rc;
    ws->reset_arena();
    const uint32_t* bits = nullptr;
    rc = observation_bits(ws, obs, obits, words, maxlen, &bits, &out->threshold_used, stream);
    if (rc) return rc;
    // idx | hits | misses | m | n | zero | argmin | hoff | obits | cf | len
    auto up = [](uint64_t b) { return (b + 255) / 256 * 256; };
    const size_t zw = (n_cands + 31) / 32;
    const size_t o_hits = up(toff[np] * 4);
    const size_t o_miss = o_hits + up(hit_bytes);
    const size_t o_m = o_miss + up(n_pairs * 16);
    const size_t o_n = o_m + up((uint64_t)n_cands * 8);
    const size_t o_zero = o_n + up((uint64_t)n_cands * 8);
    const size_t o_out = o_zero + up(zw * 4);
    const size_t o_tab = o_out + up(sizeof(ArgminOut));
    const size_t total = o_tab + 4 * up((uint64_t)np * 8);
    hipError_t e = ws->gsearch.ensure(total);
    if (e != hipSuccess) return buf_fail(ws, e, "the generalised search's buffers");
    uint8_t* g = ws->gsearch.as<uint8_t>();
    int32_t* d_idx = reinterpret_cast<int32_t*>(g);
    uint32_t* d_hits = reinterpret_cast<uint32_t*>(g + o_hits);
    uint64_t* d_miss = reinterpret_cast<uint64_t*>(g + o_miss);
    uint64_t* d_m = reinterpret_cast<uint64_t*>(g + o_m);
    uint64_t* d_n = reinterpret_cast<uint64_t*>(g + o_n);
    uint32_t* d_zero = reinterpret_cast<uint32_t*>(g + o_zero);
    ArgminOut* d_out = reinterpret_cast<ArgminOut*>(g + o_out);
    uint64_t* d_hoff = reinterpret_cast<uint64_t*>(g + o_tab);
    uint64_t* d_obits = reinterpret_cast<uint64_t*>(g + o_tab + up((uint64_t)np * 8));
    uint64_t* d_cf = reinterpret_cast<uint64_t*>(g + o_tab + 2 * up((uint64_t)np * 8));
    uint64_t* d_len = reinterpret_cast<uint64_t*>(g + o_tab + 3 * up((uint64_t)np * 8));

    rc = materialise_traces(ws, dp, toff, d_idx, stream);
    if (rc) return rc;
    rc = replay_materialised(dm, &gd, n_cands, d_idx, toff.data(), base.data(), np, pm.data(), pt.data(), pcf.data(),
                             n_pairs, d_miss, d_hits, pbit.data(), PCHASE_BATCHED, plan, stream, ws);
    if (rc) return rc;
    ArgminOut* hr = static_cast<ArgminOut*>(ws->host_res);
    CopyFence fence(stream);
    PC_HIP(hipMemcpyAsync(d_hoff, hoff.data(), np * 8, hipMemcpyHostToDevice, stream));
    PC_HIP(hipMemcpyAsync(d_obits, obits.data(), np * 8, hipMemcpyHostToDevice, stream));
    PC_HIP(hipMemcpyAsync(d_cf, cf.data(), np * 8, hipMemcpyHostToDevice, stream));
    PC_HIP(hipMemcpyAsync(d_len, len.data(), np * 8, hipMemcpyHostToDevice, stream));
    PC_HIP(hipMemcpyAsync(d_n, n_cmp.data(), (size_t)n_cands * 8, hipMemcpyHostToDevice, stream));
    PC_HIP(launch_fill_u32(reinterpret_cast<uint32_t*>(d_m), 2 * (uint64_t)n_cands, 0, stream));
    PC_HIP(launch_mismatch(d_hits, cand_words, bits, d_hoff, d_obits, d_cf, d_len, np, n_pairs, d_m, stream));
    PC_HIP(launch_argmin(d_m, d_n, n_cands, d_zero, d_out, stream));
    PC_HIP(hipMemcpyAsync(hr, d_out, sizeof(ArgminOut), hipMemcpyDeviceToHost, stream));
    if (zero_host)
        PC_HIP(hipMemcpyAsync(static_cast<uint8_t*>(ws->host_res) + 256, d_zero, zw * 4, hipMemcpyDeviceToHost,
                              stream));
    if (mn_dev) {
        PC_HIP(hipMemcpy2DAsync(mn_dev, 16, d_m, 8, 8, n_cands, hipMemcpyDeviceToDevice, stream));
        PC_HIP(hipMemcpy2DAsync(mn_dev + 1, 16, d_n, 8, 8, n_cands, hipMemcpyDeviceToDevice, stream));
    }
    PC_HIP(hipStreamSynchronize(stream));
    fence.done();
    out->best = hr->best;
    out->best_m = hr->m;
    out->best_n = hr->n;
    out->n_zero = hr->n_zero;
    out->fallback = 0;
    out->replayed_accesses = (uint64_t)n_cands * toff[np];
    out->closed_form_accesses = 0;
    if (zero_host) std::memcpy(zero_host, static_cast<uint8_t*>(ws->host_res) + 256, zw * 4);
    return PCHASE_OK;
}
